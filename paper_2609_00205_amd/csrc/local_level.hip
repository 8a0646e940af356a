// In-cache Block levels (Sec. IV-A): every b^3 block is decomposed on chip,
// between one coalesced load and one store.
//
// Block geometry: b = 2^k+1 nodes per side; neighbouring blocks share one
// face.  Inside a block the level is the MGARD step of Sec. II-B with the
// correction of the block's surface coarse nodes held at zero
// ("face-fixed"): details d = u - multilinear interpolant of the coarse
// nodes; correction z = (Mc^{-1} P^T M)_x (Mc^{-1} P^T M)_y
// (Mc^{-1} P^T M)_z w over the interior coarse rows; c = u_C + z.  Face values
// depend on face data only, so every node is written once, by its owner.
//
// Mapping to gfx950: one thread owns one z-column (y, x) of a block and keeps
// it in registers.  The multilinear interpolant needs the even-z planes of
// the four neighbouring columns (LDS); the z pass (restriction by P^T M and
// the tridiagonal solve) runs in registers; the y and x passes read short
// LDS lines, one thread per line.  The weights are compile-time constants
// (Sec. IV-A, compile-time index resolution): interior rows of P^T M on a
// unit grid are {1/12, 1/2, 5/6, 1/2, 1/12}; 3 Mc restricted to the interior
// coarse nodes is tridiag(1, 4, 1).  Small blocks are packed several to a
// workgroup so wavefronts stay full.

#include "block.h"
#include "internal.h"

namespace bm {
namespace {

// Restriction by the interior rows of P^T M (centre 2J+2) followed by the
// interior tridiagonal solve, on a line of B values: out[J], J < MI.
template <typename T, int B>
__device__ inline void restrict_solve(const T (&w)[B], T (&out)[Geo<B>::MI]) {
  constexpr int MI = Geo<B>::MI;
  constexpr Pivots<MI> P{};
  const T C0 = T(5.0 / 6.0), C1 = T(0.5), C2 = T(1.0 / 12.0);
  T d[MI];
#pragma unroll
  for (int J = 0; J < MI; ++J) {
    const int c = 2 * J + 2;
    const T r = C2 * (w[c - 2] + w[c + 2]) + C1 * (w[c - 1] + w[c + 1]) + C0 * w[c];
    d[J] = J == 0 ? T(3) * r * T(P.v[0]) : (T(3) * r - d[J - 1]) * T(P.v[J]);
  }
  out[MI - 1] = d[MI - 1];
#pragma unroll
  for (int J = MI - 2; J >= 0; --J) out[J] = d[J] - T(P.v[J]) * out[J + 1];
}

// y and x passes of the correction: T1[MI][B][B] -> T2[MI][MI][B] -> Z[MI][MI][MI]
template <typename T, int B>
__device__ inline void pass_y(const T* T1, T* T2, int tb) {
  constexpr int MI = Geo<B>::MI, BB = Geo<B>::BB;
  if (tb < MI * B) {
    const int J = tb / B, x = tb - (tb / B) * B;
    T line[B], o[MI];
#pragma unroll
    for (int y = 0; y < B; ++y) line[y] = T1[J * BB + y * B + x];
    restrict_solve<T, B>(line, o);
#pragma unroll
    for (int I = 0; I < MI; ++I) T2[(J * MI + I) * B + x] = o[I];
  }
}

template <typename T, int B>
__device__ inline void pass_x(const T* T2, T* Z, int tb) {
  constexpr int MI = Geo<B>::MI;
  if (tb < MI * MI) {
    T line[B], o[MI];
#pragma unroll
    for (int x = 0; x < B; ++x) line[x] = T2[tb * B + x];
    restrict_solve<T, B>(line, o);
#pragma unroll
    for (int K = 0; K < MI; ++K) Z[tb * MI + K] = o[K];
  }
}

template <typename T>
struct DecArgs {
  const T* src;
  int64_t sn[3], ss[3];   // source grid dims and strides (level 1: logical dims)
  int first, zero_pad;    // level 1 reads the unpadded input with clamp / zero fill
  T* coeff;
  int64_t cs[3];          // coefficient strides of this level's grid
  T* cout;                // compact coarse grid G^s
  int64_t cn[3];
  int64_t nb[3], nblocks, nwg, per;
  // fused quantization (codes written instead of coefficients)
  int32_t* codes;         // same layout as coeff
  QTab tab;               // this level's block tables
  QTab ctab;              // coarsest-value tables (last block level when M == 0)
  int coarsest_here;
  int64_t* flag;          // set when a code does not fit in int32
};

template <typename T>
struct RecArgs {
  const T* coeff;
  int64_t cs[3];
  const T* cin;           // compact coarse grid G^s
  int64_t cn[3];
  T* out;                 // output grid view (cropped to on)
  int64_t on[3], os[3];
  int64_t nb[3], nblocks, nwg, per;
  const int32_t* codes;   // fused dequantization: codes instead of coefficients
  QTab tab, ctab;
  int coarsest_here;
};

// Delta and 1/Delta of the nodes of one z-column: a node takes the smallest
// Delta (largest 1/Delta) of the blocks that contain it.  A node on a block
// face (local coordinate 0 or B-1) also lies in the neighbour across it.
// Results for z = 0, for 0 < z < B-1 and for z = B-1.
// INV: read 1/Delta and keep the largest, else read Delta and keep the smallest.
template <int B, bool INV>
__device__ inline void column_tables(const QTab& t, int64_t bz, int64_t by, int64_t bx, int y, int x, double out[3]) {
  // candidate blocks per axis: own block, plus the neighbour across a face
  const int64_t y2 = (y == 0 && by > 0) ? by - 1 : ((y == B - 1 && by + 1 < t.nb[1]) ? by + 1 : by);
  const int64_t x2 = (x == 0 && bx > 0) ? bx - 1 : ((x == B - 1 && bx + 1 < t.nb[2]) ? bx + 1 : bx);
  const int64_t zc[3] = {bz > 0 ? bz - 1 : bz, bz, bz + 1 < t.nb[0] ? bz + 1 : bz};
  const double* tab = INV ? t.inv : t.del;
  auto pick = [](double a, double b) { return INV ? fmax(a, b) : fmin(a, b); };
  double l[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t r0 = zc[c] * t.nb[1];
    double v = tab[(r0 + by) * t.nb[2] + bx];
    if (x2 != bx) v = pick(v, tab[(r0 + by) * t.nb[2] + x2]);
    if (y2 != by) {
      v = pick(v, tab[(r0 + y2) * t.nb[2] + bx]);
      if (x2 != bx) v = pick(v, tab[(r0 + y2) * t.nb[2] + x2]);
    }
    l[c] = v;
  }
  out[0] = pick(l[0], l[1]);
  out[1] = l[1];
  out[2] = pick(l[1], l[2]);
}

// Register budget of the block decomposition: FP32 fits 64 VGPRs (8 waves per
// SIMD), so more blocks are in flight to cover HBM latency; FP64 columns need
// twice the space.
template <typename T>
constexpr int kWavesPerEU = sizeof(T) == 4 ? 8 : 4;

template <int B>
__device__ inline int zcase(int z) { return z == 0 ? 0 : (z == B - 1 ? 2 : 1); }

// q = rint(c * (1/Delta)) in FP64; a code outside int32 raises the flag
template <typename T>
__device__ inline int32_t quant(T c, double inv, bool& bad) {
  const double v = rint(mul_rn(double(c), inv));
  const bool ok = fabs(v) <= 2147483647.0;
  bad |= !ok;
  return ok ? int32_t(v) : 0;
}

template <typename T, int B, bool Q>
__global__ __launch_bounds__(Geo<B>::NT) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<T>))) void k_local_decompose(DecArgs<T> a) {
  using G = Geo<B>;
  constexpr int BB = G::BB, MC = G::MC, MI = G::MI, NB = G::NB;
  __shared__ T lds[NB * G::DEC_LDS];
  const int64_t g = xcd_group(blockIdx.x, a.per);
  if (g >= a.nwg) return;
  const int tid = threadIdx.x;
  const int bl = tid / BB;                           // block within the workgroup
  const int tb = tid - bl * BB;                      // column within the block
  const int64_t blk = g * NB + bl;
  const bool act = bl < NB && blk < a.nblocks;
  T* UE = lds + (bl < NB ? bl : 0) * G::DEC_LDS;     // even-z planes [MC][B][B]
  T* T1 = UE + MC * BB;                              // [MI][B][B]
  T* T2 = UE;                                        // [MI][MI][B], after UE is dead
  T* Z = T1;                                         // [MI][MI][MI], after T1 is dead
  const int y = tb / B, x = tb - (tb / B) * B;
  const bool ecol = ((y | x) & 1) == 0;
  int64_t bz = 0, by = 0, bx = 0;
  if (act) {
    bx = blk % a.nb[2];
    const int64_t t = blk / a.nb[2];
    by = t % a.nb[1];
    bz = t / a.nb[1];
  }
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  // a node on a shared face is written by the block that starts on it
  const bool owned = (y < B - 1 || by == a.nb[1] - 1) && (x < B - 1 || bx == a.nb[2] - 1);
  const bool lastz = bz == a.nb[0] - 1;
  // fused quantization: this column's 1/Delta, loaded early so the latency hides
  double iv[3];
  if (Q && act) column_tables<B, true>(a.tab, bz, by, bx, y, x, iv);
  T v[B];
  if (act) {
    // one column: clamp or zero-fill outside the logical input on level 1
    bool yx_in = true;
    int64_t ry = gy, rx = gx;
    if (a.first) {
      yx_in = gy < a.sn[1] && gx < a.sn[2];
      ry = gy < a.sn[1] ? gy : a.sn[1] - 1;
      rx = gx < a.sn[2] ? gx : a.sn[2] - 1;
    }
    const T* col = a.src + ry * a.ss[1] + rx * a.ss[2];
#pragma unroll
    for (int z = 0; z < B; ++z) {
      int64_t gz = oz + z;
      bool in = yx_in;
      if (a.first) {
        in = in && gz < a.sn[0];
        gz = gz < a.sn[0] ? gz : a.sn[0] - 1;
      }
      v[z] = (a.zero_pad && !in) ? T(0) : col[gz * a.ss[0]];
    }
#pragma unroll
    for (int j = 0; j < MC; ++j) UE[j * BB + tb] = v[2 * j];
  }
  __syncthreads();
  if (act) {
    // details: u minus the multilinear interpolant of the coarse nodes.  They
    // are final, so they are stored at once; v keeps u_C on the coarse nodes.
    const int y0 = y & ~1, y1 = y0 + (y & 1) * 2, x0 = x & ~1, x1 = x0 + (x & 1) * 2;
    T I2[MC];
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      const T* pl = UE + j * BB;
      I2[j] = T(0.25) * ((pl[y0 * B + x0] + pl[y0 * B + x1]) + (pl[y1 * B + x0] + pl[y1 * B + x1]));
    }
#pragma unroll
    for (int z = 0; z < B; ++z) {
      if (z & 1)
        v[z] = v[z] - T(0.5) * (I2[z >> 1] + I2[(z >> 1) + 1]);
      else if (!ecol)
        v[z] = v[z] - I2[z >> 1];
    }
    if (owned) {
      if (!Q) {
        T* dst = a.coeff + gy * a.cs[1] + gx * a.cs[2];
#pragma unroll
        for (int z = 0; z < B; ++z)
          if (((z & 1) || !ecol) && (z < B - 1 || lastz)) dst[(oz + z) * a.cs[0]] = v[z];
      } else {
        int32_t* dst = a.codes + gy * a.cs[1] + gx * a.cs[2];
        bool bad = false;
#pragma unroll
        for (int z = 0; z < B; ++z)
          if (((z & 1) || !ecol) && (z < B - 1 || lastz)) dst[(oz + z) * a.cs[0]] = quant(v[z], iv[zcase<B>(z)], bad);
        if (bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), 1ull);
      }
    }
    // correction, z pass: w is zero on the coarse nodes
    T w[B], o[MI];
#pragma unroll
    for (int z = 0; z < B; ++z) w[z] = ((z & 1) || !ecol) ? v[z] : T(0);
    restrict_solve<T, B>(w, o);
#pragma unroll
    for (int J = 0; J < MI; ++J) T1[J * BB + tb] = o[J];
  }
  __syncthreads();
  if (act) pass_y<T, B>(T1, T2, tb);
  __syncthreads();
  if (act) pass_x<T, B>(T2, Z, tb);
  __syncthreads();
  if (act && ecol && owned) {
    // coarse values c = u_C + z (z = 0 on the block surface).  The coefficient
    // array gets them from a later level (or from the coarsest copy); the
    // compact coarse grid feeds the next level.
    T c[MC];
#pragma unroll
    for (int j = 0; j < MC; ++j) c[j] = v[2 * j];
    if (y >= 2 && y <= B - 3 && x >= 2 && x <= B - 3) {
      const int I = (y - 2) >> 1, K = (x - 2) >> 1;
#pragma unroll
      for (int J = 0; J < MI; ++J) c[J + 1] += Z[(J * MI + I) * MI + K];
    }
    if (Q && a.coarsest_here) {
      // last level of the hierarchy: codes for the coarsest values
      double ci[3];
      column_tables<B, true>(a.ctab, bz, by, bx, y, x, ci);
      int32_t* dst = a.codes + gy * a.cs[1] + gx * a.cs[2];
      bool bad = false;
#pragma unroll
      for (int j = 0; j < MC; ++j)
        if (j < MC - 1 || lastz) dst[(oz + 2 * j) * a.cs[0]] = quant(c[j], ci[zcase<B>(2 * j)], bad);
      if (bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), 1ull);
    } else {
      T* cdst = a.cout + (gy >> 1) * a.cn[2] + (gx >> 1);
#pragma unroll
      for (int j = 0; j < MC; ++j)
        if (j < MC - 1 || lastz) cdst[((oz >> 1) + j) * a.cn[1] * a.cn[2]] = c[j];
    }
  }
}

template <typename T, int B, bool Q>
__global__ __launch_bounds__(Geo<B>::NT) void k_local_recompose(RecArgs<T> a) {
  using G = Geo<B>;
  constexpr int BB = G::BB, MC = G::MC, MI = G::MI, NB = G::NB;
  __shared__ T lds[NB * G::REC_LDS];
  const int64_t g = xcd_group(blockIdx.x, a.per);
  if (g >= a.nwg) return;
  const int tid = threadIdx.x;
  const int bl = tid / BB;
  const int tb = tid - bl * BB;
  const int64_t blk = g * NB + bl;
  const bool act = bl < NB && blk < a.nblocks;
  T* UC = lds + (bl < NB ? bl : 0) * G::REC_LDS;     // coarse values u_C [MC][MC][MC]
  T* T1 = UC + MC * MC * MC;                         // [MI][B][B]
  T* T2 = T1 + MI * BB;                              // [MI][MI][B]
  T* Z = T1;                                         // [MI][MI][MI], after T1 is dead
  const int y = tb / B, x = tb - (tb / B) * B;
  const bool ecol = ((y | x) & 1) == 0;
  int64_t bz = 0, by = 0, bx = 0;
  if (act) {
    bx = blk % a.nb[2];
    const int64_t t = blk / a.nb[2];
    by = t % a.nb[1];
    bz = t / a.nb[1];
  }
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  T w[B], ce[MC];
  if (act) {
    if (!Q) {
      const T* col = a.coeff + gy * a.cs[1] + gx * a.cs[2];
#pragma unroll
      for (int z = 0; z < B; ++z)
        if ((z & 1) || !ecol) w[z] = col[(oz + z) * a.cs[0]];
    } else {
      // fused dequantization: c_hat = (T)(q * Delta); codes and tables load together
      const int32_t* col = a.codes + gy * a.cs[1] + gx * a.cs[2];
      int32_t qv[B];
#pragma unroll
      for (int z = 0; z < B; ++z) qv[z] = ((z & 1) || !ecol) ? col[(oz + z) * a.cs[0]] : 0;
      double dd[3];
      column_tables<B, false>(a.tab, bz, by, bx, y, x, dd);
#pragma unroll
      for (int z = 0; z < B; ++z)
        if ((z & 1) || !ecol) w[z] = T(mul_rn(double(qv[z]), dd[zcase<B>(z)]));
    }
    if (ecol) {
      if (Q && a.coarsest_here) {
        const int32_t* col = a.codes + gy * a.cs[1] + gx * a.cs[2];
        int32_t qc[MC];
#pragma unroll
        for (int j = 0; j < MC; ++j) qc[j] = col[(oz + 2 * j) * a.cs[0]];
        double cd[3];
        column_tables<B, false>(a.ctab, bz, by, bx, y, x, cd);
#pragma unroll
        for (int j = 0; j < MC; ++j) ce[j] = T(mul_rn(double(qc[j]), cd[zcase<B>(2 * j)]));
      } else {
        const T* ccol = a.cin + (gy >> 1) * a.cn[2] + (gx >> 1);
#pragma unroll
        for (int j = 0; j < MC; ++j) ce[j] = ccol[((oz >> 1) + j) * a.cn[1] * a.cn[2]];
      }
#pragma unroll
      for (int j = 0; j < MC; ++j) w[2 * j] = T(0);
    }
    T o[MI];
    restrict_solve<T, B>(w, o);
#pragma unroll
    for (int J = 0; J < MI; ++J) T1[J * BB + tb] = o[J];
  }
  __syncthreads();
  if (act) pass_y<T, B>(T1, T2, tb);
  __syncthreads();
  if (act) pass_x<T, B>(T2, Z, tb);
  __syncthreads();
  if (act && ecol) {
    // u_C = c - z on this column's coarse nodes
    const bool icol = y >= 2 && y <= B - 3 && x >= 2 && x <= B - 3;
    const int I = (y - 2) >> 1, K = (x - 2) >> 1;
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      T u = ce[j];
      if (icol && j >= 1 && j <= MC - 2) u -= Z[((j - 1) * MI + I) * MI + K];
      UC[(j * MC + (y >> 1)) * MC + (x >> 1)] = u;
    }
  }
  __syncthreads();
  if (act) {
    // u = interpolant(u_C) + w
    const int cy0 = y >> 1, cy1 = (y + 1) >> 1, cx0 = x >> 1, cx1 = (x + 1) >> 1;
    T I2[MC];
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      const T* pl = UC + j * MC * MC;
      I2[j] = T(0.25) * ((pl[cy0 * MC + cx0] + pl[cy0 * MC + cx1]) + (pl[cy1 * MC + cx0] + pl[cy1 * MC + cx1]));
    }
    const bool owny = (y < B - 1 || by == a.nb[1] - 1) && gy < a.on[1];
    const bool ownx = (x < B - 1 || bx == a.nb[2] - 1) && gx < a.on[2];
    const bool lastz = bz == a.nb[0] - 1;
    if (owny && ownx) {
      T* dst = a.out + gy * a.os[1] + gx * a.os[2];
#pragma unroll
      for (int z = 0; z < B; ++z) {
        const T u = (z & 1) ? T(0.5) * (I2[z >> 1] + I2[(z >> 1) + 1]) + w[z]
                            : (ecol ? I2[z >> 1] : I2[z >> 1] + w[z]);
        if ((z < B - 1 || lastz) && oz + z < a.on[0]) dst[(oz + z) * a.os[0]] = u;
      }
    }
  }
}

template <typename T, int B>
void launch_dec(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout, int32_t* codes,
                const QPrep* q, hipStream_t st) {
  using G = Geo<B>;
  const Level& L = p.lv[s - 1];
  DecArgs<T> a{};
  a.src = static_cast<const T*>(src.ptr);
  for (int k = 0; k < 3; ++k) {
    a.sn[k] = src.n[k];
    a.ss[k] = src.s[k];
    a.cn[k] = L.m[k];
    a.nb[k] = L.nb[k];
  }
  a.first = first;
  a.zero_pad = p.cfg.pad_mode == 1;
  a.coeff = static_cast<T*>(coeff);
  const View3 cv = level_view(p, s, q ? static_cast<void*>(codes) : coeff);
  for (int k = 0; k < 3; ++k) a.cs[k] = cv.s[k];
  a.cout = static_cast<T*>(cout);
  a.nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  a.nwg = (a.nblocks + G::NB - 1) / G::NB;
  a.per = (a.nwg + 7) / 8;
  if (q) {
    a.codes = codes;
    a.tab = q->lv[s - 1];
    a.coarsest_here = (p.M == 0 && s == p.L) ? 1 : 0;
    if (a.coarsest_here) a.ctab = q->lv[kCoarseSlotHost];
    a.flag = q->flag;
    hipLaunchKernelGGL((k_local_decompose<T, B, true>), dim3(unsigned(8 * a.per)), dim3(G::NT), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_local_decompose<T, B, false>), dim3(unsigned(8 * a.per)), dim3(G::NT), 0, st, a);
  }
  BM_HIP(hipGetLastError());
}

template <typename T, int B>
void launch_rec(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* out, bool last,
                const int32_t* codes, const QPrep* q, hipStream_t st) {
  using G = Geo<B>;
  const Level& L = p.lv[s - 1];
  RecArgs<T> a{};
  a.coeff = static_cast<const T*>(coeff);
  const View3 cv = level_view(p, s, q ? const_cast<int32_t*>(codes) : const_cast<void*>(coeff));
  for (int k = 0; k < 3; ++k) {
    a.cs[k] = cv.s[k];
    a.cn[k] = L.m[k];
    a.nb[k] = L.nb[k];
  }
  a.cin = static_cast<const T*>(cin);
  a.out = static_cast<T*>(out);
  // last: writing the caller's output with the logical (unpadded) dims
  const int64_t* on = last ? p.dims : L.n;
  for (int k = 0; k < 3; ++k) a.on[k] = on[k];
  a.os[0] = on[1] * on[2];
  a.os[1] = on[2];
  a.os[2] = 1;
  a.nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  a.nwg = (a.nblocks + G::NB - 1) / G::NB;
  a.per = (a.nwg + 7) / 8;
  if (q) {
    a.codes = codes;
    a.tab = q->lv[s - 1];
    a.coarsest_here = (p.M == 0 && s == p.L) ? 1 : 0;
    if (a.coarsest_here) a.ctab = q->lv[kCoarseSlotHost];
    hipLaunchKernelGGL((k_local_recompose<T, B, true>), dim3(unsigned(8 * a.per)), dim3(G::NT), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_local_recompose<T, B, false>), dim3(unsigned(8 * a.per)), dim3(G::NT), 0, st, a);
  }
  BM_HIP(hipGetLastError());
}

template <int B>
void dispatch_dec(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout, int32_t* codes,
                  const QPrep* q, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    launch_dec<float, B>(p, s, src, first, coeff, cout, codes, q, st);
  else
    launch_dec<double, B>(p, s, src, first, coeff, cout, codes, q, st);
}

template <int B>
void dispatch_rec(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* out, bool last,
                  const int32_t* codes, const QPrep* q, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    launch_rec<float, B>(p, s, coeff, cin, out, last, codes, q, st);
  else
    launch_rec<double, B>(p, s, coeff, cin, out, last, codes, q, st);
}

}  // namespace

void local_decompose(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* coarse_out,
                     hipStream_t st) {
  if (p.cfg.block == 9)
    dispatch_dec<9>(p, s, src, first, coeff, coarse_out, nullptr, nullptr, st);
  else
    dispatch_dec<17>(p, s, src, first, coeff, coarse_out, nullptr, nullptr, st);
}

void local_recompose(const bm_plan_s& p, int s, const void* coeff, const void* coarse_in, void* out, bool last,
                     hipStream_t st) {
  if (p.cfg.block == 9)
    dispatch_rec<9>(p, s, coeff, coarse_in, out, last, nullptr, nullptr, st);
  else
    dispatch_rec<17>(p, s, coeff, coarse_in, out, last, nullptr, nullptr, st);
}

void local_decompose_q(const bm_plan_s& p, int s, const View3& src, bool first, int32_t* codes, void* coarse_out,
                       const QPrep& q, hipStream_t st) {
  if (p.cfg.block == 9)
    dispatch_dec<9>(p, s, src, first, nullptr, coarse_out, codes, &q, st);
  else
    dispatch_dec<17>(p, s, src, first, nullptr, coarse_out, codes, &q, st);
}

void local_recompose_q(const bm_plan_s& p, int s, const int32_t* codes, const void* coarse_in, void* out, bool last,
                       const QPrep& q, hipStream_t st) {
  if (p.cfg.block == 9)
    dispatch_rec<9>(p, s, nullptr, coarse_in, out, last, codes, &q, st);
  else
    dispatch_rec<17>(p, s, nullptr, coarse_in, out, last, codes, &q, st);
}

}  // namespace bm
