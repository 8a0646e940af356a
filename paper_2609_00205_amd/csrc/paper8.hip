// The paper's own In-cache Block form (Sec. IV-A, IV-C): disjoint 8^3
// blocks, each decomposed as one MGARD level (Sec. II-B) with natural ends
// on its own 8 nodes per axis (coarse nodes 0 2 4 6 7, spacings 2 2 2 1);
// the 5^3 coarse outputs of a level's blocks, side by side in block order,
// form the next level's grid, zero-filled to a multiple of 8 (Sec. IV-D's
// zero fill).
//
// Mapping to gfx950: a workgroup takes four x-neighbouring blocks, one lane
// per z-column (256 lanes; a wavefront covers two rows of 32 consecutive
// values, one 128 B line each).  The column stays in registers; the
// interpolant reads the coarse-z planes of the block from LDS; the z pass
// (restriction by P^T M and the 5x5 coarse mass-matrix solve) runs in
// registers, the y and x passes on short LDS lines: the block's working
// set is the paper's 8^3 + 5x8x8 + 5x5x8 + 5^3 values.  Every operator
// entry is a compile-time constant.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <vector>

#include "block.h"
#include "internal.h"

namespace bm {
namespace p8 {

constexpr int B = 8, MC = 5, NBX = 4, NT = 256;
// coarse node j of an axis: 0 2 4 6 7
__device__ inline int cz(int j) { return j < MC - 1 ? 2 * j : B - 1; }

__device__ inline bool coarse(int i) { return (i & 1) == 0 || i == B - 1; }
// neighbours that interpolate node i (equal for a coarse node)
__device__ inline int lo_of(int i) { return coarse(i) ? i : i - 1; }
__device__ inline int hi_of(int i) { return coarse(i) ? i : i + 1; }
// slot of coarse node i in 0..4
__device__ inline int slot(int i) { return i == B - 1 ? MC - 1 : i >> 1; }

// Thomas elimination of the coarse mass matrix on nodes 0 2 4 6 7 (unit
// fine spacing): diagonal {2/3, 4/3, 4/3, 1, 1/3}, off-diagonal {1/3, 1/3,
// 1/3, 1/6}.  inv[k] = 1 / (pivot k), up[k] = off[k] / pivot k.
struct McSolve {
  double inv[MC], up[MC - 1], lo[MC - 1];
  constexpr McSolve() : inv(), up(), lo() {
    const double d[MC] = {2.0 / 3, 4.0 / 3, 4.0 / 3, 1.0, 1.0 / 3};
    const double e[MC - 1] = {1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 6};
    double piv = d[0];
    for (int k = 0; k < MC; ++k) {
      if (k > 0) piv = d[k] - e[k - 1] * up[k - 1];
      inv[k] = 1.0 / piv;
      if (k < MC - 1) up[k] = e[k] / piv;
      if (k > 0) lo[k - 1] = e[k - 1];
    }
  }
};

// z = Mc^{-1} P^T M w for a line of 8 values (natural end rows).
template <typename T>
__device__ inline void restrict_solve8(const T (&w)[B], T (&z)[MC]) {
  constexpr McSolve S{};
  const T a = T(1.0 / 12), h = T(0.5), c = T(5.0 / 6);
  T r[MC];
  r[0] = T(5.0 / 12) * w[0] + h * w[1] + a * w[2];
  r[1] = a * (w[0] + w[4]) + h * (w[1] + w[3]) + c * w[2];
  r[2] = a * (w[2] + w[6]) + h * (w[3] + w[5]) + c * w[4];
  r[3] = a * w[4] + h * w[5] + T(0.75) * w[6] + T(1.0 / 6) * w[7];
  r[4] = T(1.0 / 6) * w[6] + T(1.0 / 3) * w[7];
  T y[MC];
  y[0] = r[0] * T(S.inv[0]);
#pragma unroll
  for (int k = 1; k < MC; ++k) y[k] = (r[k] - T(S.lo[k - 1]) * y[k - 1]) * T(S.inv[k]);
  z[MC - 1] = y[MC - 1];
#pragma unroll
  for (int k = MC - 2; k >= 0; --k) z[k] = y[k] - T(S.up[k]) * z[k + 1];
}

template <typename T>
struct Args {
  const T* src;        // level input (decompose) or coefficients (recompose)
  int64_t sn[3];       // extent readable from src (zero fill beyond: decompose)
  int64_t ss[3];       // strides of src
  T* coeff;            // level array (decompose output), dims n
  int64_t cs[3];
  T* cdst;             // coarse values: next grid (decompose output) or its source (recompose)
  int64_t ds[3];
  T* out;              // recompose output grid
  int64_t on[3], os[3];
  int64_t nb[3], ngx;  // blocks per axis; workgroups along x (blocks of 4)
  int64_t nwg, per;
  // fused quantization (Sec. IV-D): codes instead of coefficients
  int32_t* q;          // level codes (same layout as coeff / src)
  int32_t* qc;         // coarsest codes (last level), layout of cdst
  const double* tau;   // this level's block taus
  double k, kc;        // Delta per unit tau: details, coarsest values
  int last;            // last level: the coarse values are the coarsest codes
  int64_t* flag;       // set when a code does not fit in int32
};

// q = rint(c * (1/Delta)) in FP64; a code outside int32 raises the flag
template <typename T>
__device__ inline int32_t quant8(T c, double inv, unsigned& bad) {
  const double v = rint(mul_rn(double(c), inv));
  const bool ok = fabs(v) <= 2147483647.0;
  if (!ok) bad |= code_flag(double(c));
  return ok ? int32_t(v) : 0;
}

// lane -> (block of the workgroup, y, x)
__device__ inline void lane_map(int t, int& bl, int& y, int& x) {
  y = t >> 5;
  const int xx = t & 31;
  bl = xx >> 3;
  x = xx & 7;
}

__device__ inline void wg_blocks(const int64_t g, const int64_t nb[3], int64_t ngx, int64_t& bz, int64_t& by,
                                 int64_t& bx0) {
  const int64_t gx = g % ngx, t = g / ngx;
  by = t % nb[1];
  bz = t / nb[1];
  bx0 = gx * NBX;
}

// LDS per block: UE[5][64] coarse-z planes, T1[5][64] z-pass result,
// T2[5][5][8] y-pass result, Z[5][5][5] the correction at the coarse nodes
constexpr int LDS_BLOCK = MC * 64 + MC * 64 + MC * MC * B + MC * MC * MC;

template <typename T>
__device__ inline void yx_passes(T* T1, T* T2, T* Z, int t) {
  if (t < MC * B) {   // y pass: line (Jz, x) over y
    const int J = t / B, x = t - (t / B) * B;
    T w[B], z[MC];
#pragma unroll
    for (int y = 0; y < B; ++y) w[y] = T1[J * 64 + y * B + x];
    restrict_solve8(w, z);
#pragma unroll
    for (int I = 0; I < MC; ++I) T2[(J * MC + I) * B + x] = z[I];
  }
  __syncthreads();
  if (t < MC * MC) {  // x pass: line (Jz, Jy) over x
    T w[B], z[MC];
#pragma unroll
    for (int x = 0; x < B; ++x) w[x] = T2[t * B + x];
    restrict_solve8(w, z);
#pragma unroll
    for (int K = 0; K < MC; ++K) Z[t * MC + K] = z[K];
  }
  __syncthreads();
}

// interpolant of the block's coarse values along y, x at (y, x) for each
// coarse z plane; then along z
template <typename T>
__device__ inline void interp_column(const T* UE, int y, int x, T (&I)[B]) {
  const int ya = lo_of(y), yb = hi_of(y), xa = lo_of(x), xb = hi_of(x);
  T I2[MC];
#pragma unroll
  for (int j = 0; j < MC; ++j) {
    const T* p = UE + j * 64;
    I2[j] = T(0.25) * ((p[ya * B + xa] + p[ya * B + xb]) + (p[yb * B + xa] + p[yb * B + xb]));
  }
#pragma unroll
  for (int z = 0; z < B; ++z) I[z] = (z & 1) && z != B - 1 ? T(0.5) * (I2[z >> 1] + I2[(z >> 1) + 1]) : I2[slot(z)];
}

template <typename T, bool Q>
__global__ __launch_bounds__(NT) void k_p8_decompose(Args<T> a) {
  __shared__ T lds[NBX * LDS_BLOCK];
  const int64_t g = xcd_group(blockIdx.x, a.per);
  if (g >= a.nwg) return;
  const int t = threadIdx.x;
  int bl, y, x;
  lane_map(t, bl, y, x);
  int64_t bz, by, bx0;
  wg_blocks(g, a.nb, a.ngx, bz, by, bx0);
  const int64_t bx = bx0 + bl;
  const bool act = bx < a.nb[2];
  T* UE = lds + bl * LDS_BLOCK;
  T* T1 = UE + MC * 64;
  T* T2 = T1 + MC * 64;
  T* Z = T2 + MC * MC * B;
  const int64_t gz = bz * B, gy = by * B + y, gx = bx * B + x;
  T v[B];
  if (act) {
    const bool yx_in = gy < a.sn[1] && gx < a.sn[2];
    const T* col = a.src + gy * a.ss[1] + gx * a.ss[2];
#pragma unroll
    for (int z = 0; z < B; ++z) v[z] = (yx_in && gz + z < a.sn[0]) ? col[(gz + z) * a.ss[0]] : T(0);
#pragma unroll
    for (int j = 0; j < MC; ++j) UE[j * 64 + y * B + x] = v[cz(j)];
  }
  __syncthreads();
  const bool ccol = coarse(y) && coarse(x);
  T w[B];
  if (act) {
    T I[B];
    interp_column(UE, y, x, I);
#pragma unroll
    for (int z = 0; z < B; ++z) w[z] = (ccol && coarse(z)) ? T(0) : v[z] - I[z];
    const int64_t o = gz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2];
    if (Q) {
      // the block's Delta of this level's details
      const double inv = 1.0 / (a.tau[(bz * a.nb[1] + by) * a.nb[2] + bx] * a.k);
      unsigned bad = 0;
#pragma unroll
      for (int z = 0; z < B; ++z) a.q[o + z * a.cs[0]] = quant8(w[z], inv, bad);
      if (bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), (unsigned long long)bad);
    } else {
#pragma unroll
      for (int z = 0; z < B; ++z) a.coeff[o + z * a.cs[0]] = w[z];
    }
    T zc[MC];
    restrict_solve8(w, zc);
#pragma unroll
    for (int J = 0; J < MC; ++J) T1[J * 64 + y * B + x] = zc[J];
  }
  __syncthreads();
  yx_passes(T1, T2, Z, act ? y * B + x : NT);   // each block's 64 lanes run its passes
  if (act && ccol) {
    // coarse values u_C + z, to the next grid at 5 b + slot
    const int sy = slot(y), sx = slot(x);
    const int64_t o = (bz * MC) * a.ds[0] + (by * MC + sy) * a.ds[1] + (bx * MC + sx) * a.ds[2];
    if (Q && a.last) {
      // the coarsest values: codes with the block's Delta
      const double inv = 1.0 / (a.tau[(bz * a.nb[1] + by) * a.nb[2] + bx] * a.kc);
      unsigned bad = 0;
#pragma unroll
      for (int j = 0; j < MC; ++j) a.qc[o + j * a.ds[0]] = quant8(v[cz(j)] + Z[(j * MC + sy) * MC + sx], inv, bad);
      if (bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), (unsigned long long)bad);
    } else {
#pragma unroll
      for (int j = 0; j < MC; ++j) a.cdst[o + j * a.ds[0]] = v[cz(j)] + Z[(j * MC + sy) * MC + sx];
    }
  }
}

template <typename T, bool Q>
__global__ __launch_bounds__(NT) void k_p8_recompose(Args<T> a) {
  __shared__ T lds[NBX * LDS_BLOCK];
  const int64_t g = xcd_group(blockIdx.x, a.per);
  if (g >= a.nwg) return;
  const int t = threadIdx.x;
  int bl, y, x;
  lane_map(t, bl, y, x);
  int64_t bz, by, bx0;
  wg_blocks(g, a.nb, a.ngx, bz, by, bx0);
  const int64_t bx = bx0 + bl;
  const bool act = bx < a.nb[2];
  T* UE = lds + bl * LDS_BLOCK;
  T* T1 = UE + MC * 64;
  T* T2 = T1 + MC * 64;
  T* Z = T2 + MC * MC * B;
  const int64_t gz = bz * B, gy = by * B + y, gx = bx * B + x;
  const bool ccol = coarse(y) && coarse(x);
  const int sy = slot(y), sx = slot(x);
  T w[B], c[MC];
  if (act) {
    const int64_t o = gz * a.ss[0] + gy * a.ss[1] + gx * a.ss[2];
    if (Q) {
      // fused dequantization: c_hat = (T)(q * Delta)
      const double del = a.tau[(bz * a.nb[1] + by) * a.nb[2] + bx] * a.k;
#pragma unroll
      for (int z = 0; z < B; ++z) w[z] = T(mul_rn(double(a.q[o + z * a.ss[0]]), del));
    } else {
#pragma unroll
      for (int z = 0; z < B; ++z) w[z] = a.src[o + z * a.ss[0]];
    }
    if (ccol) {
      const int64_t oc = (bz * MC) * a.ds[0] + (by * MC + sy) * a.ds[1] + (bx * MC + sx) * a.ds[2];
      if (Q && a.last) {
        const double del = a.tau[(bz * a.nb[1] + by) * a.nb[2] + bx] * a.kc;
#pragma unroll
        for (int j = 0; j < MC; ++j) c[j] = T(mul_rn(double(a.qc[oc + j * a.ds[0]]), del));
      } else {
#pragma unroll
        for (int j = 0; j < MC; ++j) c[j] = a.cdst[oc + j * a.ds[0]];
      }
#pragma unroll
      for (int z = 0; z < B; ++z)
        if (coarse(z)) w[z] = T(0);
    }
    T zc[MC];
    restrict_solve8(w, zc);
#pragma unroll
    for (int J = 0; J < MC; ++J) T1[J * 64 + y * B + x] = zc[J];
  }
  __syncthreads();
  yx_passes(T1, T2, Z, act ? y * B + x : NT);
  if (act && ccol) {
    // u_C = c - z on this column's coarse nodes
#pragma unroll
    for (int j = 0; j < MC; ++j) UE[j * 64 + y * B + x] = c[j] - Z[(j * MC + sy) * MC + sx];
  }
  __syncthreads();
  if (act) {
    T I[B];
    interp_column(UE, y, x, I);
    if (gy < a.on[1] && gx < a.on[2]) {
      T* dst = a.out + gz * a.os[0] + gy * a.os[1] + gx * a.os[2];
#pragma unroll
      for (int z = 0; z < B; ++z)
        if (gz + z < a.on[0]) dst[z * a.os[0]] = I[z] + w[z];
    }
  }
}

// ---- ROI quantization of this form (Sec. IV-C, IV-D) ----

// level-1 block map: the smallest voxel tolerance over a block's real nodes
__global__ __launch_bounds__(256) void k_p8_block_tol(const double* vt, int64_t n0, int64_t n1, int64_t n2,
                                                      int64_t nb0, int64_t nb1, int64_t nb2, double* out) {
  const int64_t tot = nb0 * nb1 * nb2;
  for (int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x; b < tot; b += int64_t(gridDim.x) * 256) {
    const int64_t bx = b % nb2, t = b / nb2, by = t % nb1, bz = t / nb1;
    double m = INFINITY;
    for (int64_t z = bz * B; z < bz * B + B && z < n0; ++z)
      for (int64_t y = by * B; y < by * B + B && y < n1; ++y)
        for (int64_t x = bx * B; x < bx * B + B && x < n2; ++x) m = fmin(m, vt[(z * n1 + y) * n2 + x]);
    out[b] = m;
  }
}

// Eq. 2 on the assembled grid (Fig. 6): next-level block I takes the smallest
// tau over the blocks J whose outputs 5J..5J+4 meet 8I..8I+7
__global__ __launch_bounds__(256) void k_p8_propagate(const double* tau, int64_t s0, int64_t s1, int64_t s2,
                                                      double* out, int64_t m0, int64_t m1, int64_t m2) {
  const int64_t tot = m0 * m1 * m2;
  for (int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x; b < tot; b += int64_t(gridDim.x) * 256) {
    const int64_t I2 = b % m2, t = b / m2, I1 = t % m1, I0 = t / m1;
    auto lo = [](int64_t I) { return B * I / MC; };
    auto hi = [](int64_t I, int64_t n) { return i64min((B * I + B - 1) / MC, n - 1); };
    double m = INFINITY;
    for (int64_t z = lo(I0); z <= hi(I0, s0); ++z)
      for (int64_t y = lo(I1); y <= hi(I1, s1); ++y)
        for (int64_t x = lo(I2); x <= hi(I2, s2); ++x) m = fmin(m, tau[(z * s1 + y) * s2 + x]);
    out[b] = m;
  }
}

constexpr int kMaxL = 8;

struct QArgs8 {
  int L;
  uint32_t off[kMaxL + 2];       // flat offset of level s (s = 0..L-1), coarsest at L, end at L+1
  Unflat32 uf[kMaxL + 1];        // level grid (s < L) or coarsest dims (s = L)
  uint32_t nb1[kMaxL], nb2[kMaxL];   // blocks along y, x of level s
  const double* tau[kMaxL];      // block taus of level s
  double k[kMaxL + 1];           // Delta per unit tau: level s, coarsest at L
  int64_t* flag;                 // set when a code does not fit in int32
};

// Delta of flat coefficient i
__device__ inline double delta_of(const QArgs8& a, uint32_t i) {
  int s = 0;
  while (s < a.L && i >= a.off[s + 1]) ++s;
  uint32_t z, y, x;
  a.uf[s](i - a.off[s], z, y, x);
  if (s < a.L) return a.tau[s][(size_t(z >> 3) * a.nb1[s] + (y >> 3)) * a.nb2[s] + (x >> 3)] * a.k[s];
  // a coarsest value: the tau of the last level's block it came from
  const int l = a.L - 1;
  return a.tau[l][(size_t(z / MC) * a.nb1[l] + y / MC) * a.nb2[l] + x / MC] * a.k[a.L];
}

template <typename T>
__global__ __launch_bounds__(256) void k_p8_quantize(const T* c, uint32_t n, QArgs8 a, int32_t* q) {
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
    const double inv = 1.0 / delta_of(a, i);
    const double v = rint(mul_rn(double(c[i]), inv));
    const bool ok = fabs(v) <= 2147483647.0;
    if (!ok) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), (unsigned long long)code_flag(double(c[i])));
    q[i] = ok ? int32_t(v) : 0;
  }
}

// The smallest of n taus: tau_global of the hybrid, written to out[0].  The
// workgroups meet in one 64-bit integer atomicMin on out[1], which holds the
// running minimum as an order-preserving key of the double's bits (a sign
// flip of the magnitude bits of negatives makes signed-integer order equal
// double order); k_p8_min_init sets it to the key of +inf and k_p8_min_done
// turns it back into a double.  NaN taus are ignored, as fmin ignores them.
__device__ inline long long min_key(double v) {
  const long long b = __double_as_longlong(v);
  return b >= 0 ? b : b ^ 0x7FFFFFFFFFFFFFFFll;
}

__global__ void k_p8_min_init(double* out) {
  if (threadIdx.x == 0) reinterpret_cast<long long*>(out)[1] = min_key(INFINITY);
}

__global__ __launch_bounds__(256) void k_p8_min(const double* t, int64_t n, double* out) {
  __shared__ double m[256];
  double v = INFINITY;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) v = fmin(v, t[i]);
  m[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) m[threadIdx.x] = fmin(m[threadIdx.x], m[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMin(reinterpret_cast<long long*>(out) + 1, min_key(m[0]));
}

__global__ void k_p8_min_done(double* out) {
  if (threadIdx.x == 0) out[0] = __longlong_as_double(min_key(__longlong_as_double(reinterpret_cast<long long*>(out)[1])));
}

template <typename T>
__global__ __launch_bounds__(256) void k_p8_dequantize(const int32_t* q, uint32_t n, QArgs8 a, T* c) {
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u)
    c[i] = T(mul_rn(double(q[i]), delta_of(a, i)));
}

}  // namespace p8
}  // namespace bm

// ------------------------------------------------------------------ host

struct bm_p8_s {
  int device = 0;
  int dtype = BM_F32;
  size_t esize = 4;
  int L = 0;
  int64_t dims[3] = {1, 1, 1};
  std::vector<std::array<int64_t, 3>> n;   // level grid dims (multiples of 8)
  int64_t last[3] = {0, 0, 0};             // coarsest dims
  std::vector<int64_t> off;                // level array offsets in the coefficients (elements); off[L] = coarsest
  std::vector<void*> grid;                 // grid[s] (s = 1..L-1): assembled coarse values, zero fill kept
  std::vector<double*> tau;                // tau[s] (s = 1..L-1): propagated block tolerances
  int64_t* flag = nullptr;                 // quantizer overflow flag
  int32_t* codes = nullptr;                // codes of the compress path (allocated on first use)
  // the hybrid (M > 0): global levels on the assembled coarsest grid
  int M = 0;
  bm_plan_s* glob = nullptr;               // global-only plan over the coarsest grid (dims last)
  void* gin = nullptr;                     // the coarsest grid between the block and global levels (the
                                           // global plan's padded level-1 grid, owned by that plan)
  double* tg = nullptr;                    // tau_global (the smallest last-level block tau), then its reduction key
};

bm_plan_s* bm_plan_build(const bm_config* c);
void bm_plan_free(bm_plan_s* p);

namespace bm {

namespace {

inline int64_t up8(int64_t v) { return (v + 7) / 8 * 8; }

template <typename T>
p8::Args<T> p8_args(const bm_p8_s& p, int s) {
  p8::Args<T> a{};
  const auto& n = p.n[s];
  for (int k = 0; k < 3; ++k) a.nb[k] = n[k] / 8;
  a.ngx = (a.nb[2] + p8::NBX - 1) / p8::NBX;
  a.nwg = a.nb[0] * a.nb[1] * a.ngx;
  a.per = (a.nwg + 7) / 8;
  a.cs[0] = n[1] * n[2];
  a.cs[1] = n[2];
  a.cs[2] = 1;
  // the coarse values' array: the next level's grid, the global levels'
  // padded level-1 grid (the hybrid), or the coarsest values
  int64_t d1 = p.last[1], d2 = p.last[2];
  if (s + 1 < p.L) {
    d1 = p.n[s + 1][1];
    d2 = p.n[s + 1][2];
  } else if (p.M) {
    d1 = p.glob->pdims[1];
    d2 = p.glob->pdims[2];
  }
  a.ds[0] = d1 * d2;
  a.ds[1] = d2;
  a.ds[2] = 1;
  return a;
}

// quantization context of a fused call: the levels' taus and Delta factors
struct P8Quant {
  const double* tau[p8::kMaxL];
  double k[p8::kMaxL + 1];
};

template <typename T, bool Q>
void p8_decompose_t(const bm_p8_s& p, const void* x, void* coeff, int32_t* codes, const P8Quant* qz,
                    hipStream_t st) {
  T* c = static_cast<T*>(coeff);
  for (int s = 0; s < p.L; ++s) {
    p8::Args<T> a = p8_args<T>(p, s);
    const auto& n = p.n[s];
    if (s == 0) {
      a.src = static_cast<const T*>(x);
      for (int k = 0; k < 3; ++k) a.sn[k] = p.dims[k];
      a.ss[0] = p.dims[1] * p.dims[2];
      a.ss[1] = p.dims[2];
      a.ss[2] = 1;
    } else {
      a.src = static_cast<const T*>(p.grid[s]);
      for (int k = 0; k < 3; ++k) a.sn[k] = n[k];
      a.ss[0] = n[1] * n[2];
      a.ss[1] = n[2];
      a.ss[2] = 1;
    }
    if (Q) {
      a.q = codes + p.off[s];
      a.qc = codes + p.off[p.L];
      a.tau = qz->tau[s];
      a.k = qz->k[s];
      a.kc = qz->k[p.L];
      a.last = s == p.L - 1;
      a.flag = p.flag;
      a.cdst = s + 1 < p.L ? static_cast<T*>(p.grid[s + 1]) : nullptr;
    } else {
      a.coeff = c + p.off[s];
      a.cdst = s + 1 < p.L ? static_cast<T*>(p.grid[s + 1]) : (p.M ? static_cast<T*>(p.gin) : c + p.off[p.L]);
    }
    if (Q && p.M && s == p.L - 1) {   // hybrid: the coarsest values go to the global levels
      a.last = 0;
      a.cdst = static_cast<T*>(p.gin);
    }
    hipLaunchKernelGGL((p8::k_p8_decompose<T, Q>), dim3(unsigned(8 * a.per)), dim3(p8::NT), 0, st, a);
    BM_HIP(hipGetLastError());
  }
}

template <typename T, bool Q>
void p8_recompose_t(const bm_p8_s& p, const void* coeff, void* x, const int32_t* codes, const P8Quant* qz,
                    hipStream_t st) {
  const T* c = static_cast<const T*>(coeff);
  for (int s = p.L - 1; s >= 0; --s) {
    p8::Args<T> a = p8_args<T>(p, s);
    const auto& n = p.n[s];
    for (int k = 0; k < 3; ++k) a.sn[k] = n[k];
    a.ss[0] = n[1] * n[2];
    a.ss[1] = n[2];
    a.ss[2] = 1;
    if (Q) {
      a.q = const_cast<int32_t*>(codes) + p.off[s];
      a.qc = const_cast<int32_t*>(codes) + p.off[p.L];
      a.tau = qz->tau[s];
      a.k = qz->k[s];
      a.kc = qz->k[p.L];
      a.last = s == p.L - 1;
      a.cdst = s + 1 < p.L ? static_cast<T*>(p.grid[s + 1]) : nullptr;
    } else {
      a.src = c + p.off[s];
      a.cdst = s + 1 < p.L ? static_cast<T*>(p.grid[s + 1])
                           : (p.M ? static_cast<T*>(p.gin) : const_cast<T*>(c) + p.off[p.L]);
    }
    if (Q && p.M && s == p.L - 1) {   // hybrid: the coarsest values come from the global levels
      a.last = 0;
      a.cdst = static_cast<T*>(p.gin);
    }
    if (s == 0) {
      a.out = static_cast<T*>(x);
      for (int k = 0; k < 3; ++k) a.on[k] = p.dims[k];
      a.os[0] = p.dims[1] * p.dims[2];
      a.os[1] = p.dims[2];
    } else {
      // only the assembled values: the zero fill beyond them stays zero
      a.out = static_cast<T*>(p.grid[s]);
      for (int k = 0; k < 3; ++k) a.on[k] = 5 * (p.n[s - 1][k] / 8);
      a.os[0] = n[1] * n[2];
      a.os[1] = n[2];
    }
    a.os[2] = 1;
    hipLaunchKernelGGL((p8::k_p8_recompose<T, Q>), dim3(unsigned(8 * a.per)), dim3(p8::NT), 0, st, a);
    BM_HIP(hipGetLastError());
  }
}

}  // namespace

bm_p8_s* p8_create(const int64_t dims[3], int dtype, int L, int M) {
  if (dtype != BM_F32 && dtype != BM_F64) fail(BM_EINVAL, "dtype must be BM_F32 or BM_F64");
  if (L < 1 || L > 8) fail(BM_EINVAL, "L must lie in [1, 8]");
  if (M < 0 || M > 16) fail(BM_EINVAL, "M must lie in [0, 16]");
  for (int k = 0; k < 3; ++k)
    if (dims[k] < 1 || dims[k] > (int64_t(1) << 31)) fail(BM_EINVAL, "dims must lie in [1, 2^31]");
  if (up8(dims[1]) * up8(dims[2]) > (int64_t(1) << 40) / up8(dims[0]))
    fail(BM_EINVAL, "grid of more than 2^40 nodes");
  auto* p = new bm_p8_s();
  try {
    BM_HIP(hipGetDevice(&p->device));
    p->dtype = dtype;
    p->esize = dtype == BM_F32 ? 4 : 8;
    p->L = L;
    std::array<int64_t, 3> n{up8(dims[0]), up8(dims[1]), up8(dims[2])};
    for (int k = 0; k < 3; ++k) p->dims[k] = dims[k];
    int64_t o = 0;
    for (int s = 0; s < L; ++s) {
      p->n.push_back(n);
      p->off.push_back(o);
      o += n[0] * n[1] * n[2];
      std::array<int64_t, 3> m{5 * (n[0] / 8), 5 * (n[1] / 8), 5 * (n[2] / 8)};
      if (s + 1 < L) {
        n = {up8(m[0]), up8(m[1]), up8(m[2])};
      } else {
        for (int k = 0; k < 3; ++k) p->last[k] = m[k];
      }
    }
    p->off.push_back(o);
    p->grid.assign(L, nullptr);
    p->tau.assign(L, nullptr);
    for (int s = 1; s < L; ++s) {
      const size_t bytes = size_t(p->n[s][0] * p->n[s][1] * p->n[s][2]) * p->esize;
      BM_HIP(hipMalloc(&p->grid[s], bytes));
      BM_HIP(hipMemset(p->grid[s], 0, bytes));   // the zero fill beyond the assembled values
      BM_HIP(hipMalloc(&p->tau[s], size_t(p->n[s][0] / 8) * (p->n[s][1] / 8) * (p->n[s][2] / 8) * sizeof(double)));
    }
    BM_HIP(hipMalloc(&p->flag, sizeof(int64_t)));
    if (M > 0) {
      // the global levels: a plan of their own over the coarsest grid (clamp
      // extension to the lengths they halve, natural ends)
      bm_config c{};
      c.ndim = 3;
      for (int k = 0; k < 3; ++k) c.dims[k] = p->last[k];
      c.dtype = dtype;
      c.block = 0;
      c.L = 0;
      c.M = M;
      c.pad_mode = 0;
      c.eta = 0.0;
      c.nested = 0;
      p->glob = bm_plan_build(&c);
      p->M = M;
      // the last block level writes its assembled values straight into the
      // global plan's padded level-1 grid, and reads them back from there
      p->gin = level1_grid(*p->glob);
      BM_HIP(hipMalloc(&p->tg, 2 * sizeof(double)));
    }
  } catch (...) {
    for (void* g : p->grid)
      if (g) (void)hipFree(g);
    for (double* t : p->tau)
      if (t) (void)hipFree(t);
    if (p->flag) (void)hipFree(p->flag);
    if (p->glob) bm_plan_free(p->glob);
    delete p;
    throw;
  }
  return p;
}

int p8_global_levels(const bm_p8_s& p) { return p.M; }

void p8_free(bm_p8_s* p) {
  if (!p) return;
  for (void* g : p->grid)
    if (g) (void)hipFree(g);
  for (double* t : p->tau)
    if (t) (void)hipFree(t);
  if (p->flag) (void)hipFree(p->flag);
  if (p->codes) (void)hipFree(p->codes);
  if (p->glob) bm_plan_free(p->glob);
  if (p->tg) (void)hipFree(p->tg);
  delete p;
}

int32_t* p8_codes(bm_p8_s& p) {
  if (!p.codes) BM_HIP(hipMalloc(&p.codes, size_t(p8_coeff_size(p)) * sizeof(int32_t)));
  return p.codes;
}

void p8_info(const bm_p8_s& p, int64_t dims[3], int* dtype, int* L, size_t* esize) {
  for (int k = 0; k < 3; ++k) dims[k] = p.dims[k];
  *dtype = p.dtype;
  *L = p.L;
  *esize = p.esize;
}

void p8_block_grid(const bm_p8_s& p, int64_t nb[3]) {
  for (int k = 0; k < 3; ++k) nb[k] = p.n[0][k] / 8;
}

void p8_tolmap_from_voxels(const bm_p8_s& p, const double* vt, double* block_tol, hipStream_t st) {
  int64_t nb[3];
  p8_block_grid(p, nb);
  const int64_t tot = nb[0] * nb[1] * nb[2];
  const unsigned g = unsigned(std::min<int64_t>(65536, (tot + 255) / 256));
  hipLaunchKernelGGL(p8::k_p8_block_tol, dim3(g), dim3(256), 0, st, vt, p.dims[0], p.dims[1], p.dims[2], nb[0],
                     nb[1], nb[2], block_tol);
  BM_HIP(hipGetLastError());
}

// L-inf gain of the details of one natural 8-node level in its
// reconstruction: max over nodes x of the sum over detail nodes y of
// |delta_xy - prod_d a(x_d, y_d)|, a = P K on the 8-node axis (K = Mc^{-1}
// P^T M with the coarse nodes 0 2 4 6 7), from the 1D row profiles (sum of
// |a| over all and over coarse columns, diagonal, coarse flag); rounded up
// to 4 decimals with a 1e-6 slack in units of the last decimal.
static double p8_gain() {
  constexpr int n = 8, m = 5;
  const int cn[m] = {0, 2, 4, 6, 7};
  double P[n][m] = {};
  for (int j = 0; j < m; ++j) P[cn[j]][j] = 1.0;
  for (int i : {1, 3, 5}) P[i][i / 2] = P[i][i / 2 + 1] = 0.5;
  double M[n][n] = {};
  for (int i = 0; i < n; ++i) {
    M[i][i] = (i == 0 || i == n - 1) ? 1.0 / 3 : 2.0 / 3;
    if (i + 1 < n) M[i][i + 1] = M[i + 1][i] = 1.0 / 6;
  }
  const double d[m] = {2.0 / 3, 4.0 / 3, 4.0 / 3, 1.0, 1.0 / 3};
  const double e[m - 1] = {1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 6};
  double K[m][n];
  for (int c = 0; c < n; ++c) {
    double r[m];
    for (int j = 0; j < m; ++j) {
      r[j] = 0;
      for (int i = 0; i < n; ++i) r[j] += P[i][j] * M[i][c];
    }
    // Thomas on Mc
    double cp[m], dp[m];
    cp[0] = e[0] / d[0];
    dp[0] = r[0] / d[0];
    for (int j = 1; j < m; ++j) {
      const double den = d[j] - e[j - 1] * cp[j - 1];
      cp[j] = j < m - 1 ? e[j] / den : 0.0;
      dp[j] = (r[j] - e[j - 1] * dp[j - 1]) / den;
    }
    K[m - 1][c] = dp[m - 1];
    for (int j = m - 2; j >= 0; --j) K[j][c] = dp[j] - cp[j] * K[j + 1][c];
  }
  double sall[n], sc[n], dg[n];
  bool cf[n];
  for (int i = 0; i < n; ++i) {
    sall[i] = sc[i] = 0;
    cf[i] = (i & 1) == 0 || i == n - 1;
    for (int j = 0; j < n; ++j) {
      double a = 0;
      for (int k = 0; k < m; ++k) a += P[i][k] * K[k][j];
      sall[i] += std::fabs(a);
      if ((j & 1) == 0 || j == n - 1) sc[i] += std::fabs(a);
      if (j == i) dg[i] = a;
    }
  }
  double best = 0;
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        double v = sall[z] * sall[y] * sall[x] - sc[z] * sc[y] * sc[x];
        if (!(cf[z] && cf[y] && cf[x])) v += std::fabs(1.0 - dg[z] * dg[y] * dg[x]) - std::fabs(dg[z] * dg[y] * dg[x]);
        best = std::max(best, v);
      }
  return std::ceil(best * 10000.0 - 1e-6) / 10000.0;
}

// Budget shares of the levels' details and of the coarsest values:
// proportional to their counts, floored at 1/(64 (L+1)), renormalised
// (summed in order).
// The hybrid: L block levels, then the M global levels (their details split
// equally) and the coarsest values of the global plan, floored at
// 1/(64 (L+M+1)).
static std::vector<double> p8_weights(const bm_p8_s& p) {
  int64_t tot = 0;
  for (int s = 0; s < p.L; ++s) tot += p.n[s][0] * p.n[s][1] * p.n[s][2];
  const int64_t nlast = p.last[0] * p.last[1] * p.last[2];
  std::vector<double> w;
  if (p.M == 0) {
    tot += nlast;
    const double N = double(tot);
    for (int s = 0; s < p.L; ++s) w.push_back(double(p.n[s][0] * p.n[s][1] * p.n[s][2]) * (512 - 125) / 512 / N);
    w.push_back(double(nlast) / N);
  } else {
    const bm_plan_s& g = *p.glob;
    const int64_t gsize = g.pdims[0] * g.pdims[1] * g.pdims[2];
    const Level& lc = g.lv[g.nlev - 1];
    const int64_t ncoarse = lc.m[0] * lc.m[1] * lc.m[2];
    const double N = double(tot + gsize);
    for (int s = 0; s < p.L; ++s) w.push_back(double(p.n[s][0] * p.n[s][1] * p.n[s][2]) * (512 - 125) / 512 / N);
    for (int s = 0; s < p.M; ++s) w.push_back((double(gsize - ncoarse) / N) / double(p.M));
    w.push_back(double(ncoarse) / N);
  }
  const double floor = 1.0 / (64.0 * double(p.L + p.M + 1));
  double sum = 0.0;
  for (double& v : w) {
    v = v > floor ? v : floor;
    sum += v;
  }
  for (double& v : w) v /= sum;
  return w;
}

static p8::QArgs8 p8_qargs(const bm_p8_s& p, const double* block_tol, double eta, hipStream_t st) {
  if (!(eta >= 0.0 && eta < 0.5)) fail(BM_EINVAL, "eta must lie in [0, 0.5)");
  if (p8_coeff_size(p) >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "2^32 coefficients or more");
  // propagated taus of levels 2..L
  std::vector<const double*> tau(p.L);
  tau[0] = block_tol;
  for (int s = 1; s < p.L; ++s) {
    const auto& a = p.n[s - 1];
    const auto& b = p.n[s];
    const int64_t tot = (b[0] / 8) * (b[1] / 8) * (b[2] / 8);
    const unsigned g = unsigned(std::min<int64_t>(65536, (tot + 255) / 256));
    hipLaunchKernelGGL(p8::k_p8_propagate, dim3(g), dim3(256), 0, st, tau[s - 1], a[0] / 8, a[1] / 8, a[2] / 8,
                       p.tau[s], b[0] / 8, b[1] / 8, b[2] / 8);
    BM_HIP(hipGetLastError());
    tau[s] = p.tau[s];
  }
  const double A = p8_gain();
  const std::vector<double> w = p8_weights(p);
  p8::QArgs8 q{};
  q.L = p.L;
  for (int s = 0; s <= p.L; ++s) q.off[s] = uint32_t(p.off[s]);
  q.off[p.L + 1] = uint32_t(p8_coeff_size(p));
  for (int s = 0; s < p.L; ++s) {
    q.uf[s] = Unflat32(p.n[s][1], p.n[s][2]);
    q.nb1[s] = uint32_t(p.n[s][1] / 8);
    q.nb2[s] = uint32_t(p.n[s][2] / 8);
    q.tau[s] = tau[s];
    q.k[s] = (2.0 * (1.0 - eta)) * w[s] / A;
  }
  q.uf[p.L] = Unflat32(p.last[1], p.last[2]);
  q.k[p.L] = (2.0 * (1.0 - eta)) * w[p.L];
  q.flag = p.flag;
  if (p.M) {
    // the global levels quantize at tau_global (the smallest last-level
    // block tau, Sec. IV-C) with this budget's shares of them
    const auto& nl = p.n[p.L - 1];
    const int64_t nbl = (nl[0] / 8) * (nl[1] / 8) * (nl[2] / 8);
    hipLaunchKernelGGL(p8::k_p8_min_init, dim3(1), dim3(64), 0, st, p.tg);
    hipLaunchKernelGGL(p8::k_p8_min, dim3(unsigned(std::max<int64_t>(1, std::min<int64_t>(1024, (nbl + 255) / 256)))),
                       dim3(256), 0, st, tau[p.L - 1], nbl, p.tg);
    hipLaunchKernelGGL(p8::k_p8_min_done, dim3(1), dim3(64), 0, st, p.tg);
    BM_HIP(hipGetLastError());
    p.glob->cfg.eta = eta;
    p.glob->w_override.assign(w.begin() + p.L, w.end());
  }
  return q;
}

// coefficient offset (bytes) of the global levels' array of the hybrid
static size_t p8_goff(const bm_p8_s& p) { return size_t(p.off[p.L]) * p.esize; }

void p8_quantize(const bm_p8_s& p, const void* coeff, const double* block_tol, double eta, int32_t* codes,
                 hipStream_t st) {
  const p8::QArgs8 q = p8_qargs(p, block_tol, eta, st);
  BM_HIP(hipMemsetAsync(p.flag, 0, sizeof(int64_t), st));
  const uint32_t n = uint32_t(p.M ? p.off[p.L] : p8_coeff_size(p));
  const unsigned g = unsigned(std::min<int64_t>(65536, (int64_t(n) + 255) / 256));
  if (p.dtype == BM_F32)
    hipLaunchKernelGGL(p8::k_p8_quantize<float>, dim3(g), dim3(256), 0, st, static_cast<const float*>(coeff), n, q,
                       codes);
  else
    hipLaunchKernelGGL(p8::k_p8_quantize<double>, dim3(g), dim3(256), 0, st, static_cast<const double*>(coeff), n,
                       q, codes);
  BM_HIP(hipGetLastError());
  int64_t f = 0;
  BM_HIP(hipMemcpyAsync(&f, p.flag, sizeof(f), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  check_code_flag(f, "tolerance too small for the data");
  if (p.M) {
    bm_qstats qs;
    quantize(*p.glob, static_cast<const uint8_t*>(coeff) + p8_goff(p), p.tg, codes + p.off[p.L], &qs, st);
  }
}

void p8_dequantize(const bm_p8_s& p, const int32_t* codes, const double* block_tol, double eta, void* coeff,
                   hipStream_t st) {
  const p8::QArgs8 q = p8_qargs(p, block_tol, eta, st);
  const uint32_t n = uint32_t(p.M ? p.off[p.L] : p8_coeff_size(p));
  const unsigned g = unsigned(std::min<int64_t>(65536, (int64_t(n) + 255) / 256));
  if (p.dtype == BM_F32)
    hipLaunchKernelGGL(p8::k_p8_dequantize<float>, dim3(g), dim3(256), 0, st, codes, n, q, static_cast<float*>(coeff));
  else
    hipLaunchKernelGGL(p8::k_p8_dequantize<double>, dim3(g), dim3(256), 0, st, codes, n, q,
                       static_cast<double*>(coeff));
  BM_HIP(hipGetLastError());
  if (p.M) dequantize(*p.glob, codes + p.off[p.L], p.tg, static_cast<uint8_t*>(coeff) + p8_goff(p), st);
}

int64_t p8_coeff_size(const bm_p8_s& p) {
  if (p.M) return p.off[p.L] + p.glob->pdims[0] * p.glob->pdims[1] * p.glob->pdims[2];
  return p.off[p.L] + p.last[0] * p.last[1] * p.last[2];
}

int p8_device(const bm_p8_s& p) { return p.device; }

void p8_decompose(const bm_p8_s& p, const void* x, void* coeff, hipStream_t st) {
  if (p.dtype == BM_F32)
    p8_decompose_t<float, false>(p, x, coeff, nullptr, nullptr, st);
  else
    p8_decompose_t<double, false>(p, x, coeff, nullptr, nullptr, st);
  if (p.M) decompose(*p.glob, p.gin, static_cast<uint8_t*>(coeff) + p8_goff(p), st);
}

void p8_recompose(const bm_p8_s& p, const void* coeff, void* x, hipStream_t st) {
  if (p.M) recompose(*p.glob, static_cast<const uint8_t*>(coeff) + p8_goff(p), p.gin, st);
  if (p.dtype == BM_F32)
    p8_recompose_t<float, false>(p, coeff, x, nullptr, nullptr, st);
  else
    p8_recompose_t<double, false>(p, coeff, x, nullptr, nullptr, st);
}

// Fused pipeline of this form (the paper's Sec. IV-D): the block kernel
// writes the codes of each level's details (and, at the last level, of the
// coarsest values); the recomposition dequantizes on load.  Codes and
// values equal bm_p8_quantize after bm_p8_decompose, and bm_p8_recompose
// after bm_p8_dequantize, bit for bit.
static P8Quant p8_quant(const p8::QArgs8& q) {
  P8Quant z{};
  for (int s = 0; s < q.L; ++s) z.tau[s] = q.tau[s];
  for (int s = 0; s <= q.L; ++s) z.k[s] = q.k[s];
  return z;
}

void p8_decompose_quantize(const bm_p8_s& p, const void* x, const double* block_tol, double eta, int32_t* codes,
                           hipStream_t st) {
  const P8Quant z = p8_quant(p8_qargs(p, block_tol, eta, st));
  BM_HIP(hipMemsetAsync(p.flag, 0, sizeof(int64_t), st));
  if (p.dtype == BM_F32)
    p8_decompose_t<float, true>(p, x, nullptr, codes, &z, st);
  else
    p8_decompose_t<double, true>(p, x, nullptr, codes, &z, st);
  int64_t f = 0;
  BM_HIP(hipMemcpyAsync(&f, p.flag, sizeof(f), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  check_code_flag(f, "tolerance too small for the data");
  if (p.M) {
    bm_qstats qs;
    decompose_quantize(*p.glob, p.gin, p.tg, codes + p.off[p.L], &qs, st);
  }
}

void p8_dequantize_recompose(const bm_p8_s& p, const int32_t* codes, const double* block_tol, double eta, void* x,
                             hipStream_t st) {
  const P8Quant z = p8_quant(p8_qargs(p, block_tol, eta, st));
  if (p.M) dequantize_recompose(*p.glob, codes + p.off[p.L], p.tg, p.gin, st);
  if (p.dtype == BM_F32)
    p8_recompose_t<float, true>(p, nullptr, x, codes, &z, st);
  else
    p8_recompose_t<double, true>(p, nullptr, x, codes, &z, st);
}

}  // namespace bm
