// In-cache Block levels (Sec. IV-A): one workgroup per b^3 block, the whole
// level computed in LDS between one coalesced load and one store.
//
// Block geometry: b = 2^k+1 nodes per side; neighbouring blocks share one
// face.  Inside a block the level is the MGARD step of Sec. II-B with the
// correction of the block's surface coarse nodes held at zero
// ("face-fixed"): details d = u - multilinear interpolant of the coarse
// nodes; load vector f = (P^T M)_x (P^T M)_y (P^T M)_z w over the interior
// coarse rows (three shrinking passes b^3 -> mi b^2 -> mi^2 b -> mi^3 with
// mi = (b+1)/2 - 2); tridiagonal solves with the coarse mass matrix along
// x, y, z; coarse value c = u_C + z.  Face values depend on face data only,
// so every node is written once, by the block that owns it.
//
// The weights are compile-time constants (Sec. IV-A, compile-time index
// resolution): interior rows of P^T M on a unit grid are
// {1/12, 1/2, 5/6, 1/2, 1/12}; 3 Mc restricted to interior coarse nodes is
// tridiag(1, 4, 1).

#include "internal.h"

namespace bm {
namespace {

constexpr int NT = 256;

template <int B>
struct Geo {
  static constexpr int N = B * B * B;
  static constexpr int BB = B * B;
  static constexpr int MI = (B + 1) / 2 - 2;   // interior coarse nodes per axis
  static constexpr int SCR = MI * BB + MI * MI * B;
};

// Reciprocal pivots of Thomas elimination for tridiag(1, 4, 1) of size MI.
template <int MI>
struct Pivots {
  double v[MI];
  constexpr Pivots() : v() {
    double c = 0.0;
    for (int i = 0; i < MI; ++i) {
      v[i] = 1.0 / (4.0 - c);
      c = v[i];
    }
  }
};

// XCD-aware block order: consecutive hardware workgroup ids go round-robin
// over the 8 XCDs; this map gives each XCD a contiguous run of blocks so
// shared faces are re-read from the same L2.
__device__ inline int64_t xcd_block(int64_t wg, int64_t per) { return (wg & 7) * per + (wg >> 3); }

template <typename T>
struct DecArgs {
  const T* src;
  int64_t sn[3], ss[3];   // source grid dims and strides (level 1: logical dims)
  int first, zero_pad;    // level 1 reads the unpadded input with clamp / zero fill
  T* coeff;
  int64_t cs[3];          // coefficient strides of this level's grid
  T* cout;                // compact coarse grid G^s
  int64_t cn[3];
  int64_t nb[3], nblocks, per;
};

template <typename T>
struct RecArgs {
  const T* coeff;
  int64_t cs[3];
  const T* cin;           // compact coarse grid G^s
  int64_t cn[3];
  T* out;                 // output grid view (cropped to on)
  int64_t on[3], os[3];
  int64_t nb[3], nblocks, per;
};

template <int B>
__device__ inline int lidx(int z, int y, int x) {
  return (z * B + y) * B + x;
}

// Multilinear interpolant of the block's coarse nodes at node (z, y, x):
// the mean of the 8 corners of the coarse cell, where an even coordinate
// uses the node itself twice (weights 1/2 per odd axis).
template <typename T, int B>
__device__ inline T interp(const T* U, int z, int y, int x) {
  const int z0 = z & ~1, z1 = z0 + (z & 1) * 2;
  const int y0 = y & ~1, y1 = y0 + (y & 1) * 2;
  const int x0 = x & ~1, x1 = x0 + (x & 1) * 2;
  const T s = ((U[lidx<B>(z0, y0, x0)] + U[lidx<B>(z0, y0, x1)]) + (U[lidx<B>(z0, y1, x0)] + U[lidx<B>(z0, y1, x1)])) +
              ((U[lidx<B>(z1, y0, x0)] + U[lidx<B>(z1, y0, x1)]) + (U[lidx<B>(z1, y1, x0)] + U[lidx<B>(z1, y1, x1)]));
  return s * T(0.125);
}

// Thomas elimination for tridiag(1,4,1) x = 3 f on MI values at stride S.
template <typename T, int MI, int S>
__device__ inline void solve_interior(T* x) {
  constexpr Pivots<MI> P{};
  T d[MI];
  d[0] = T(3) * x[0] * T(P.v[0]);
#pragma unroll
  for (int i = 1; i < MI; ++i) d[i] = (T(3) * x[i * S] - d[i - 1]) * T(P.v[i]);
  x[(MI - 1) * S] = d[MI - 1];
#pragma unroll
  for (int i = MI - 2; i >= 0; --i) {
    d[i] = d[i] - T(P.v[i]) * d[i + 1];
    x[i * S] = d[i];
  }
}

// Correction of the interior coarse nodes from the fine-only values held in
// U (coarse entries of U are read as zero).  Leaves z[J][I][K] in S[0, MI^3).
template <typename T, int B>
__device__ void correction(const T* U, T* S, int tid) {
  using G = Geo<B>;
  constexpr int MI = G::MI, BB = G::BB;
  const T C0 = T(5.0 / 6.0), C1 = T(0.5), C2 = T(1.0 / 12.0);
  T* RZ = S;                 // [MI][B][B]
  T* RY = S + MI * BB;       // [MI][MI][B]
  T* RX = S;                 // [MI][MI][MI], overwrites RZ after the y pass
  for (int i = tid; i < MI * BB; i += NT) {
    const int J = i / BB, r = i - J * BB, y = r / B, x = r - y * B;
    const int zc = 2 * J + 2;
    const bool xyeven = ((x | y) & 1) == 0;
    const int base = y * B + x;
    const T w0 = xyeven ? T(0) : U[zc * BB + base];
    const T wm2 = xyeven ? T(0) : U[(zc - 2) * BB + base];
    const T wp2 = xyeven ? T(0) : U[(zc + 2) * BB + base];
    const T wm1 = U[(zc - 1) * BB + base];
    const T wp1 = U[(zc + 1) * BB + base];
    RZ[i] = C2 * (wm2 + wp2) + C1 * (wm1 + wp1) + C0 * w0;
  }
  __syncthreads();
  for (int i = tid; i < MI * MI * B; i += NT) {
    const int J = i / (MI * B), r = i - J * (MI * B), I = r / B, x = r - I * B;
    const int yc = 2 * I + 2;
    const T* p = RZ + J * BB + x;
    RY[i] = C2 * (p[(yc - 2) * B] + p[(yc + 2) * B]) + C1 * (p[(yc - 1) * B] + p[(yc + 1) * B]) + C0 * p[yc * B];
  }
  __syncthreads();
  // RZ is dead once the y pass has finished, so RX may take its space
  for (int i = tid; i < MI * MI * MI; i += NT) {
    const int J = i / (MI * MI), r = i - J * (MI * MI), I = r / MI, K = r - I * MI;
    const int xc = 2 * K + 2;
    const T* p = RY + (J * MI + I) * B;
    RX[i] = C2 * (p[xc - 2] + p[xc + 2]) + C1 * (p[xc - 1] + p[xc + 1]) + C0 * p[xc];
  }
  __syncthreads();
  static_assert(MI * MI <= NT, "one thread per interior line");
  if (tid < MI * MI) solve_interior<T, MI, 1>(RX + tid * MI);                       // x lines
  __syncthreads();
  if (tid < MI * MI) {
    const int J = tid / MI, K = tid - J * MI;
    solve_interior<T, MI, MI>(RX + J * MI * MI + K);                                 // y lines
  }
  __syncthreads();
  if (tid < MI * MI) solve_interior<T, MI, MI * MI>(RX + tid);                       // z lines
  __syncthreads();
}

template <typename T, int B>
__global__ __launch_bounds__(NT) void k_local_decompose(DecArgs<T> a) {
  using G = Geo<B>;
  constexpr int N = G::N, BB = G::BB, MI = G::MI;
  __shared__ T U[N];
  __shared__ T S[G::SCR];
  const int64_t blk = xcd_block(blockIdx.x, a.per);
  if (blk >= a.nblocks) return;
  const int64_t bx = blk % a.nb[2], t = blk / a.nb[2], by = t % a.nb[1], bz = t / a.nb[1];
  const int64_t oz = bz * (B - 1), oy = by * (B - 1), ox = bx * (B - 1);
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) {
    const int lz = i / BB, r = i - lz * BB, ly = r / B, lx = r - ly * B;
    int64_t gz = oz + lz, gy = oy + ly, gx = ox + lx;
    T v;
    if (a.first && (gz >= a.sn[0] || gy >= a.sn[1] || gx >= a.sn[2])) {
      if (a.zero_pad) {
        v = T(0);
      } else {
        gz = gz < a.sn[0] ? gz : a.sn[0] - 1;
        gy = gy < a.sn[1] ? gy : a.sn[1] - 1;
        gx = gx < a.sn[2] ? gx : a.sn[2] - 1;
        v = a.src[gz * a.ss[0] + gy * a.ss[1] + gx * a.ss[2]];
      }
    } else {
      v = a.src[gz * a.ss[0] + gy * a.ss[1] + gx * a.ss[2]];
    }
    U[i] = v;
  }
  __syncthreads();
  for (int i = tid; i < N; i += NT) {
    const int lz = i / BB, r = i - lz * BB, ly = r / B, lx = r - ly * B;
    if (((lz | ly | lx) & 1) == 0) continue;
    U[i] -= interp<T, B>(U, lz, ly, lx);
  }
  __syncthreads();
  correction<T, B>(U, S, tid);
  for (int i = tid; i < MI * MI * MI; i += NT) {
    const int J = i / (MI * MI), r = i - J * (MI * MI), I = r / MI, K = r - I * MI;
    U[lidx<B>(2 * J + 2, 2 * I + 2, 2 * K + 2)] += S[i];
  }
  __syncthreads();
  const bool lastz = bz == a.nb[0] - 1, lasty = by == a.nb[1] - 1, lastx = bx == a.nb[2] - 1;
  for (int i = tid; i < N; i += NT) {
    const int lz = i / BB, r = i - lz * BB, ly = r / B, lx = r - ly * B;
    if ((lz == B - 1 && !lastz) || (ly == B - 1 && !lasty) || (lx == B - 1 && !lastx)) continue;
    const int64_t gz = oz + lz, gy = oy + ly, gx = ox + lx;
    const T v = U[i];
    a.coeff[gz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2]] = v;
    if (((lz | ly | lx) & 1) == 0) a.cout[((gz >> 1) * a.cn[1] + (gy >> 1)) * a.cn[2] + (gx >> 1)] = v;
  }
}

template <typename T, int B>
__global__ __launch_bounds__(NT) void k_local_recompose(RecArgs<T> a) {
  using G = Geo<B>;
  constexpr int N = G::N, BB = G::BB, MI = G::MI;
  __shared__ T U[N];
  __shared__ T S[G::SCR];
  const int64_t blk = xcd_block(blockIdx.x, a.per);
  if (blk >= a.nblocks) return;
  const int64_t bx = blk % a.nb[2], t = blk / a.nb[2], by = t % a.nb[1], bz = t / a.nb[1];
  const int64_t oz = bz * (B - 1), oy = by * (B - 1), ox = bx * (B - 1);
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) {
    const int lz = i / BB, r = i - lz * BB, ly = r / B, lx = r - ly * B;
    const int64_t gz = oz + lz, gy = oy + ly, gx = ox + lx;
    T v;
    if (((lz | ly | lx) & 1) == 0)
      v = a.cin[((gz >> 1) * a.cn[1] + (gy >> 1)) * a.cn[2] + (gx >> 1)];
    else
      v = a.coeff[gz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2]];
    U[i] = v;
  }
  __syncthreads();
  correction<T, B>(U, S, tid);
  for (int i = tid; i < MI * MI * MI; i += NT) {
    const int J = i / (MI * MI), r = i - J * (MI * MI), I = r / MI, K = r - I * MI;
    U[lidx<B>(2 * J + 2, 2 * I + 2, 2 * K + 2)] -= S[i];
  }
  __syncthreads();
  for (int i = tid; i < N; i += NT) {
    const int lz = i / BB, r = i - lz * BB, ly = r / B, lx = r - ly * B;
    if (((lz | ly | lx) & 1) == 0) continue;
    U[i] += interp<T, B>(U, lz, ly, lx);
  }
  __syncthreads();
  const bool lastz = bz == a.nb[0] - 1, lasty = by == a.nb[1] - 1, lastx = bx == a.nb[2] - 1;
  for (int i = tid; i < N; i += NT) {
    const int lz = i / BB, r = i - lz * BB, ly = r / B, lx = r - ly * B;
    if ((lz == B - 1 && !lastz) || (ly == B - 1 && !lasty) || (lx == B - 1 && !lastx)) continue;
    const int64_t gz = oz + lz, gy = oy + ly, gx = ox + lx;
    if (gz >= a.on[0] || gy >= a.on[1] || gx >= a.on[2]) continue;
    a.out[gz * a.os[0] + gy * a.os[1] + gx * a.os[2]] = U[i];
  }
}

template <typename T, int B>
void launch_dec(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout,
                hipStream_t st) {
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
  const View3 cv = level_view(p, s, coeff);
  for (int k = 0; k < 3; ++k) a.cs[k] = cv.s[k];
  a.cout = static_cast<T*>(cout);
  a.nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  a.per = (a.nblocks + 7) / 8;
  hipLaunchKernelGGL((k_local_decompose<T, B>), dim3(unsigned(8 * a.per)), dim3(NT), 0, st, a);
  BM_HIP(hipGetLastError());
}

template <typename T, int B>
void launch_rec(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* out, bool last,
                hipStream_t st) {
  const Level& L = p.lv[s - 1];
  RecArgs<T> a{};
  a.coeff = static_cast<const T*>(coeff);
  const View3 cv = level_view(p, s, const_cast<void*>(coeff));
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
  a.per = (a.nblocks + 7) / 8;
  hipLaunchKernelGGL((k_local_recompose<T, B>), dim3(unsigned(8 * a.per)), dim3(NT), 0, st, a);
  BM_HIP(hipGetLastError());
}

}  // namespace

void local_decompose(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* coarse_out,
                     hipStream_t st) {
  const int b = p.cfg.block;
  if (p.cfg.dtype == BM_F32) {
    if (b == 9) launch_dec<float, 9>(p, s, src, first, coeff, coarse_out, st);
    else launch_dec<float, 17>(p, s, src, first, coeff, coarse_out, st);
  } else {
    if (b == 9) launch_dec<double, 9>(p, s, src, first, coeff, coarse_out, st);
    else launch_dec<double, 17>(p, s, src, first, coeff, coarse_out, st);
  }
}

void local_recompose(const bm_plan_s& p, int s, const void* coeff, const void* coarse_in, void* out, bool last,
                     hipStream_t st) {
  const int b = p.cfg.block;
  if (p.cfg.dtype == BM_F32) {
    if (b == 9) launch_rec<float, 9>(p, s, coeff, coarse_in, out, last, st);
    else launch_rec<float, 17>(p, s, coeff, coarse_in, out, last, st);
  } else {
    if (b == 9) launch_rec<double, 9>(p, s, coeff, coarse_in, out, last, st);
    else launch_rec<double, 17>(p, s, coeff, coarse_in, out, last, st);
  }
}

}  // namespace bm
