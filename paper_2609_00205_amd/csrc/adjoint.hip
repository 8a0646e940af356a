// Transposes of the multilevel transform: D^T (decompose) and R^T
// (recompose), level by level in the reverse order of the forward map.  They
// give gradients through the transform and the coefficient sensitivities of
// a quantity of interest.
//
// One decomposition level (Sec. II-B) on a grid F with coarse nodes C maps u
// to  w = (I - P3 S) u on the fine-only nodes and  c = S u + K3 w on C,
// with S the selection of C, P3 the multilinear interpolation and
// K3 = (Mc^{-1} P^T M) per axis.  Its transpose takes (g on F\C, cbar on C) to
//   fine-only nodes:  v = g + K3^T cbar        (K^T = M P Mc^{-1} per axis)
//   coarse nodes:     cbar - P3^T v0           (v0 = v with zeros on C).
// One recomposition level u = P3 (c - K3 w) + w has the transpose
//   coarse nodes:     r = P3^T g,
//   fine-only nodes:  g - K3^T r.
// K^T along one axis is a solve with Mc followed by the transposed rows of
// P^T M (a spread from m to n nodes); P3^T is a gather over the 3^3
// neighbourhood of each coarse node with weights 1, 1/2, 1/4, 1/8.
//
// Block levels (Sec. IV-A, face-fixed): every block applies the transpose of
// its own level to the values of the nodes it owns and adds the result into
// every node it covers, shared faces included.  Blocks run in 8 passes by
// the parity of their block coordinates: two blocks of one parity class never
// share a node, so a pass needs no atomics, and the order in which shared
// nodes are summed is fixed (the first class that covers a node writes it,
// later classes add).  The transpose of the clamp padding adds the gradient
// of every padded node into the node it copied.

#include "block.h"
#include "internal.h"
#include "line_solve.h"

namespace bm {
namespace {

constexpr int NT = 256;

inline unsigned grid_for(int64_t tot) {
  int64_t g = (tot + NT - 1) / NT;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return unsigned(g);
}

// --------------------------------------------------------------- block levels

// K_D^T on one line of a face-fixed block: s = Mc_I^{-1} y on the MI interior
// coarse nodes (3 Mc_I = tridiag(1, 4, 1)), then the transposed interior rows
// of P^T M ({1/12, 1/2, 5/6, 1/2, 1/12} around node 2J+2) spread s over the B
// nodes of the line.
template <typename T, int B>
__device__ inline void solve_spread(const T (&yv)[Geo<B>::MI], T (&out)[B]) {
  constexpr int MI = Geo<B>::MI;
  constexpr Pivots<MI> P{};
  T d[MI], s[MI];
#pragma unroll
  for (int J = 0; J < MI; ++J) d[J] = J == 0 ? T(3) * yv[0] * T(P.v[0]) : (T(3) * yv[J] - d[J - 1]) * T(P.v[J]);
  s[MI - 1] = d[MI - 1];
#pragma unroll
  for (int J = MI - 2; J >= 0; --J) s[J] = d[J] - T(P.v[J]) * s[J + 1];
  const T C0 = T(5.0 / 6.0), C1 = T(0.5), C2 = T(1.0 / 12.0);
#pragma unroll
  for (int i = 0; i < B; ++i) out[i] = T(0);
#pragma unroll
  for (int J = 0; J < MI; ++J) {
    const int c = 2 * J + 2;
    out[c - 2] += C2 * s[J];
    out[c - 1] += C1 * s[J];
    out[c] += C0 * s[J];
    out[c + 1] += C1 * s[J];
    out[c + 2] += C2 * s[J];
  }
}

// Blocks of one parity class: block coordinates b_k = 2 i_k + bit_k.
struct ColorSet {
  int64_t nb[3];          // blocks per axis
  int bit[3];             // parity of this pass
  int64_t nbc[3];         // blocks of this parity per axis
  int64_t nblocks, nwg, per;
};

__device__ inline void color_block(const ColorSet& c, int64_t k, int64_t& bz, int64_t& by, int64_t& bx) {
  const int64_t kx = k % c.nbc[2];
  const int64_t t = k / c.nbc[2];
  bx = 2 * kx + c.bit[2];
  by = 2 * (t % c.nbc[1]) + c.bit[1];
  bz = 2 * (t / c.nbc[1]) + c.bit[0];
}

// Is this block the first (lowest parity class) of the blocks covering a
// node at local coordinate loc along one axis?  The only other candidate is
// the neighbour across a face, whose parity differs.
template <int B>
__device__ inline bool first_on_axis(int loc, int64_t bk, int64_t nbk) {
  const bool other = (loc == 0 && bk > 0) || (loc == B - 1 && bk + 1 < nbk);
  return !other || (bk & 1) == 0;
}

template <typename T>
__device__ inline void put(T* dst, T v, bool first) {
  *dst = first ? v : *dst + v;
}

// Transposed passes x, y (LDS lines) and z (registers) of K_D^T:
// Z[J][I][K] -> T2[J][I][x] -> T1[J][y][x] -> t[z] of column tb.
template <typename T, int B>
__device__ inline void kd_transpose_xy(const T* Z, T* T2, T* T1, int tb, bool act) {
  constexpr int MI = Geo<B>::MI, BB = Geo<B>::BB;
  if (act && tb < MI * MI) {
    T l[MI], o[B];
#pragma unroll
    for (int K = 0; K < MI; ++K) l[K] = Z[tb * MI + K];
    solve_spread<T, B>(l, o);
#pragma unroll
    for (int x = 0; x < B; ++x) T2[tb * B + x] = o[x];
  }
  __syncthreads();
  if (act && tb < MI * B) {
    const int J = tb / B, x = tb - (tb / B) * B;
    T l[MI], o[B];
#pragma unroll
    for (int I = 0; I < MI; ++I) l[I] = T2[(J * MI + I) * B + x];
    solve_spread<T, B>(l, o);
#pragma unroll
    for (int y = 0; y < B; ++y) T1[J * BB + y * B + x] = o[y];
  }
  __syncthreads();
}

// z part of P3^T at the even planes of one column: R[j] = v[2j] + (v[2j-1] + v[2j+1]) / 2
template <typename T, int B>
__device__ inline void restrict_z(const T (&v)[B], T* R, int tb) {
  constexpr int MC = Geo<B>::MC, BB = Geo<B>::BB;
#pragma unroll
  for (int j = 0; j < MC; ++j) {
    T r = v[2 * j];
    if (j > 0 && j < MC - 1)
      r += T(0.5) * (v[2 * j - 1] + v[2 * j + 1]);
    else if (j > 0)
      r += T(0.5) * v[2 * j - 1];
    else
      r += T(0.5) * v[2 * j + 1];
    R[j * BB + tb] = r;
  }
}

// y and x parts of P3^T at the coarse nodes of an even column (y, x)
template <typename T, int B>
__device__ inline T gather_yx(const T* R, int j, int y, int x) {
  constexpr int BB = Geo<B>::BB;
  const T* pl = R + j * BB;
  T acc = pl[y * B + x];
  T side = T(0), corner = T(0);
  if (y > 0) side += pl[(y - 1) * B + x];
  if (y < B - 1) side += pl[(y + 1) * B + x];
  if (x > 0) side += pl[y * B + x - 1];
  if (x < B - 1) side += pl[y * B + x + 1];
  if (y > 0 && x > 0) corner += pl[(y - 1) * B + x - 1];
  if (y > 0 && x < B - 1) corner += pl[(y - 1) * B + x + 1];
  if (y < B - 1 && x > 0) corner += pl[(y + 1) * B + x - 1];
  if (y < B - 1 && x < B - 1) corner += pl[(y + 1) * B + x + 1];
  return acc + T(0.5) * side + T(0.25) * corner;
}

template <typename T>
struct DecTArgs {
  const T* gc;            // gradient of the coefficients, this level's view (strides cs)
  int64_t cs[3];
  const T* gcur;          // gradient of the coarse grid G^s (compact, dims cn)
  int64_t cn[3];
  T* out;                 // gradient of G^{s-1} (dense, dims on)
  int64_t on[3];
  ColorSet c;
};

template <typename T, int B>
__global__ __launch_bounds__((Geo<B, sizeof(T)>::NT)) void k_local_decompose_T(DecTArgs<T> a) {
  using G = Geo<B, sizeof(T)>;
  constexpr int BB = G::BB, MC = G::MC, MI = G::MI, NB = G::NB;
  __shared__ T lds[NB * G::ADJ_LDS];
  const int64_t g = xcd_group(blockIdx.x, a.c.per);
  if (g >= a.c.nwg) return;
  const int tid = threadIdx.x;
  const int bl = tid / BB;
  const int tb = tid - bl * BB;
  const int64_t blk = g * NB + bl;
  const bool act = bl < NB && blk < a.c.nblocks;
  T* T1 = lds + (bl < NB ? bl : 0) * G::ADJ_LDS;     // [MI][B][B]
  T* T2 = T1 + MI * BB;                              // [MI][MI][B]
  T* Z = T2 + MI * MI * B;                           // [MI][MI][MI]
  T* R = T1;                                         // [MC][B][B], once T1 and T2 are dead
  const int y = tb / B, x = tb - (tb / B) * B;
  const bool ecol = ((y | x) & 1) == 0;
  int64_t bz = 0, by = 0, bx = 0;
  if (act) color_block(a.c, blk, bz, by, bx);
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  // the gradient on the nodes this block owns (zero elsewhere)
  T gv[B];
  if (act) {
    const bool own_yx = (y < B - 1 || by == a.c.nb[1] - 1) && (x < B - 1 || bx == a.c.nb[2] - 1);
    const bool lastz = bz == a.c.nb[0] - 1;
    const T* col = a.gc + gy * a.cs[1] + gx * a.cs[2];
    const T* ccol = a.gcur + (gy >> 1) * a.cn[2] + (gx >> 1);
    const int64_t cpl = a.cn[1] * a.cn[2];
#pragma unroll
    for (int z = 0; z < B; ++z) {
      T v = T(0);
      if (own_yx && (z < B - 1 || lastz))
        v = (ecol && !(z & 1)) ? ccol[((oz >> 1) + (z >> 1)) * cpl] : col[(oz + z) * a.cs[0]];
      gv[z] = v;
    }
    if (ecol && y >= 2 && y <= B - 3 && x >= 2 && x <= B - 3) {
      const int I = (y - 2) >> 1, K = (x - 2) >> 1;
#pragma unroll
      for (int J = 0; J < MI; ++J) Z[(J * MI + I) * MI + K] = gv[2 * J + 2];
    }
  }
  __syncthreads();
  kd_transpose_xy<T, B>(Z, T2, T1, tb, act);
  T v[B];
  if (act) {
    T l[MI], t[B];
#pragma unroll
    for (int J = 0; J < MI; ++J) l[J] = T1[J * BB + tb];
    solve_spread<T, B>(l, t);
#pragma unroll
    for (int z = 0; z < B; ++z) v[z] = (ecol && !(z & 1)) ? T(0) : gv[z] + t[z];
    // R aliases T1 (this column only, read above) and the dead T2 / Z
    restrict_z<T, B>(v, R, tb);
  }
  __syncthreads();
  if (act) {
    if (ecol) {
#pragma unroll
      for (int j = 0; j < MC; ++j) v[2 * j] = gv[2 * j] - gather_yx<T, B>(R, j, y, x);
    }
    const bool fy = first_on_axis<B>(y, by, a.c.nb[1]), fx = first_on_axis<B>(x, bx, a.c.nb[2]);
    T* dst = a.out + gy * a.on[2] + gx;
    const int64_t pl = a.on[1] * a.on[2];
#pragma unroll
    for (int z = 0; z < B; ++z) put(dst + (oz + z) * pl, v[z], fy && fx && first_on_axis<B>(z, bz, a.c.nb[0]));
  }
}

template <typename T>
struct RecTArgs {
  const T* gin;           // gradient of G^{s-1} (dense, dims in); zero at or beyond lim
  int64_t in[3], lim[3];
  T* gc;                  // gradient of the coefficients, this level's view (strides cs)
  int64_t cs[3];
  T* gcur;                // gradient of the coarse grid G^s (compact, dims cn)
  int64_t cn[3];
  ColorSet c;
};

template <typename T, int B>
__global__ __launch_bounds__((Geo<B, sizeof(T)>::NT)) void k_local_recompose_T(RecTArgs<T> a) {
  using G = Geo<B, sizeof(T)>;
  constexpr int BB = G::BB, MC = G::MC, MI = G::MI, NB = G::NB;
  __shared__ T lds[NB * G::ADJ_LDS];
  const int64_t g = xcd_group(blockIdx.x, a.c.per);
  if (g >= a.c.nwg) return;
  const int tid = threadIdx.x;
  const int bl = tid / BB;
  const int tb = tid - bl * BB;
  const int64_t blk = g * NB + bl;
  const bool act = bl < NB && blk < a.c.nblocks;
  T* T1 = lds + (bl < NB ? bl : 0) * G::ADJ_LDS;
  T* T2 = T1 + MI * BB;
  T* Z = T2 + MI * MI * B;
  T* R = T1;
  const int y = tb / B, x = tb - (tb / B) * B;
  const bool ecol = ((y | x) & 1) == 0;
  int64_t bz = 0, by = 0, bx = 0;
  if (act) color_block(a.c, blk, bz, by, bx);
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  T gv[B];
  if (act) {
    const bool own_yx = (y < B - 1 || by == a.c.nb[1] - 1) && (x < B - 1 || bx == a.c.nb[2] - 1) &&
                        gy < a.lim[1] && gx < a.lim[2];
    const bool lastz = bz == a.c.nb[0] - 1;
    const T* col = a.gin + gy * a.in[2] + gx;
    const int64_t pl = a.in[1] * a.in[2];
#pragma unroll
    for (int z = 0; z < B; ++z)
      gv[z] = (own_yx && (z < B - 1 || lastz) && oz + z < a.lim[0]) ? col[(oz + z) * pl] : T(0);
    restrict_z<T, B>(gv, R, tb);
  }
  __syncthreads();
  T rc[MC];
  if (act && ecol) {
#pragma unroll
    for (int j = 0; j < MC; ++j) rc[j] = gather_yx<T, B>(R, j, y, x);
  }
  __syncthreads();
  if (act && ecol && y >= 2 && y <= B - 3 && x >= 2 && x <= B - 3) {
    const int I = (y - 2) >> 1, K = (x - 2) >> 1;
#pragma unroll
    for (int J = 0; J < MI; ++J) Z[(J * MI + I) * MI + K] = rc[J + 1];
  }
  __syncthreads();
  kd_transpose_xy<T, B>(Z, T2, T1, tb, act);
  if (act) {
    T l[MI], t[B];
#pragma unroll
    for (int J = 0; J < MI; ++J) l[J] = T1[J * BB + tb];
    solve_spread<T, B>(l, t);
    const bool fy = first_on_axis<B>(y, by, a.c.nb[1]), fx = first_on_axis<B>(x, bx, a.c.nb[2]);
    T* dst = a.gc + gy * a.cs[1] + gx * a.cs[2];
    T* cdst = a.gcur + (gy >> 1) * a.cn[2] + (gx >> 1);
    const int64_t cpl = a.cn[1] * a.cn[2];
#pragma unroll
    for (int z = 0; z < B; ++z) {
      const bool first = fy && fx && first_on_axis<B>(z, bz, a.c.nb[0]);
      if (ecol && !(z & 1))
        put(cdst + ((oz >> 1) + (z >> 1)) * cpl, rc[z >> 1], first);
      else
        put(dst + (oz + z) * a.cs[0], gv[z] - t[z], first);
    }
  }
}

ColorSet color_set(const Level& L, int color, int nb_per_wg) {
  ColorSet c{};
  c.nblocks = 1;
  for (int k = 0; k < 3; ++k) {
    c.nb[k] = L.nb[k];
    c.bit[k] = (color >> (2 - k)) & 1;
    c.nbc[k] = (L.nb[k] - c.bit[k] + 1) / 2;
    c.nblocks *= c.nbc[k];
  }
  c.nwg = (c.nblocks + nb_per_wg - 1) / nb_per_wg;
  c.per = (c.nwg + 7) / 8;
  return c;
}

template <typename T, int B>
void launch_local_dec_T(const bm_plan_s& p, int s, const void* gcoeff, void* out, hipStream_t st) {
  using G = Geo<B, sizeof(T)>;
  const Level& L = p.lv[s - 1];
  DecTArgs<T> a{};
  const View3 cv = level_view(p, s, const_cast<void*>(gcoeff));
  a.gc = static_cast<const T*>(cv.ptr);
  a.gcur = static_cast<const T*>(p.ws.grid[s]);
  a.out = static_cast<T*>(out);
  for (int k = 0; k < 3; ++k) {
    a.cs[k] = cv.s[k];
    a.cn[k] = L.m[k];
    a.on[k] = L.n[k];
  }
  for (int color = 0; color < 8; ++color) {
    a.c = color_set(L, color, G::NB);
    if (a.c.nblocks == 0) continue;
    hipLaunchKernelGGL((k_local_decompose_T<T, B>), dim3(unsigned(8 * a.c.per)), dim3(G::NT), 0, st, a);
    BM_HIP(hipGetLastError());
  }
}

template <typename T, int B>
void launch_local_rec_T(const bm_plan_s& p, int s, const void* gin, const int64_t in[3], const int64_t lim[3],
                        void* gcoeff, hipStream_t st) {
  using G = Geo<B, sizeof(T)>;
  const Level& L = p.lv[s - 1];
  RecTArgs<T> a{};
  const View3 cv = level_view(p, s, gcoeff);
  a.gin = static_cast<const T*>(gin);
  a.gc = static_cast<T*>(cv.ptr);
  a.gcur = static_cast<T*>(p.ws.grid[s]);
  for (int k = 0; k < 3; ++k) {
    a.in[k] = in[k];
    a.lim[k] = lim[k];
    a.cs[k] = cv.s[k];
    a.cn[k] = L.m[k];
  }
  for (int color = 0; color < 8; ++color) {
    a.c = color_set(L, color, G::NB);
    if (a.c.nblocks == 0) continue;
    hipLaunchKernelGGL((k_local_recompose_T<T, B>), dim3(unsigned(8 * a.c.per)), dim3(G::NT), 0, st, a);
    BM_HIP(hipGetLastError());
  }
}

// ------------------------------------------------------- 33^3 block levels
// Transposes of the 33^3 block level, split like the forward kernels: a
// block is cut along x into halves, here overlapping by two columns (x in
// [0, 17] and [15, 32]) so that the transposed interpolation at the coarse
// columns next to the cut (16 and 18) has both neighbours; the first half
// stores x <= 16, the second x >= 17.  The transposed correction runs as an
// x spread per block into a scratch array (the plan's line-pass buffer),
// then the y and z spreads per half.  Halves of one colour class write
// disjoint nodes, so the colour passes keep the summation order fixed.
namespace w33 {
constexpr int B = 33, MC = 17, MI = 15, HW = 18, NCOL = B * HW, NT = 640, T2B = MI * MI * B, ZB = MI * MI * MI;
__device__ inline int x0(int h) { return h ? 15 : 0; }
__device__ inline bool stores(int h, int x) { return h ? x >= 17 : x <= 16; }
}  // namespace w33

template <typename T>
struct W33Args {
  const T* gc;            // decompose: gradient of the coefficients (level view); recompose: output
  int64_t cs[3];
  const T* gcur;          // gradient of the coarse grid G^s (compact, dims cn); recompose: output
  int64_t cn[3];
  T* out;                 // decompose: gradient of G^{s-1} (dense, dims on)
  int64_t on[3];
  const T* gin;           // recompose: gradient of G^{s-1} (dense, dims in, zero at or beyond lim)
  int64_t in[3], lim[3];
  T* zs;                  // recompose: interior coarse gradients per block [ZB]
  T* t2;                  // x-spread result per block [MI][MI][B]
  int64_t nb[3];
  ColorSet c;
};

// z part of P3^T at the even planes of a column of 33 values
template <typename T>
__device__ inline T restrict_z33(const T (&v)[w33::B], int j) {
  using namespace w33;
  T r = v[2 * j];
  if (j > 0 && j < MC - 1)
    r += T(0.5) * (v[2 * j - 1] + v[2 * j + 1]);
  else if (j > 0)
    r += T(0.5) * v[2 * j - 1];
  else
    r += T(0.5) * v[2 * j + 1];
  return r;
}

// y and x parts of P3^T at coarse node (j, y, x) from R[MC][B][HW] of half h
template <typename T>
__device__ inline T gather33(const T* R, int j, int y, int xl, int x) {
  using namespace w33;
  const T* pl = R + j * B * HW;
  auto at = [&](int yy, int dx) { return pl[yy * HW + xl + dx]; };
  T acc = at(y, 0);
  T side = T(0), corner = T(0);
  if (y > 0) side += at(y - 1, 0);
  if (y < B - 1) side += at(y + 1, 0);
  if (x > 0) side += at(y, -1);
  if (x < B - 1) side += at(y, 1);
  if (y > 0 && x > 0) corner += at(y - 1, -1);
  if (y > 0 && x < B - 1) corner += at(y - 1, 1);
  if (y < B - 1 && x > 0) corner += at(y + 1, -1);
  if (y < B - 1 && x < B - 1) corner += at(y + 1, 1);
  return acc + T(0.5) * side + T(0.25) * corner;
}

// x spread of the transposed correction, one workgroup per block: Z[MI]^3
// (from the coarse grid's interior nodes, or from zs) -> t2[MI][MI][B]
template <typename T>
__global__ __launch_bounds__(256) void k_w33_spread_x(W33Args<T> a, int from_zs) {
  using namespace w33;
  __shared__ T Z[ZB];
  const int64_t blk = blockIdx.x;
  const int64_t bx = blk % a.nb[2], t = blk / a.nb[2], by = t % a.nb[1], bz = t / a.nb[1];
  const int64_t c0 = bz * (MC - 1), c1 = by * (MC - 1), c2 = bx * (MC - 1), cpl = a.cn[1] * a.cn[2];
  for (int i = threadIdx.x; i < ZB; i += 256) {
    const int J = i / (MI * MI), r = i - J * MI * MI, I = r / MI, K = r - I * MI;
    Z[i] = from_zs ? a.zs[blk * ZB + i] : a.gcur[(c0 + J + 1) * cpl + (c1 + I + 1) * a.cn[2] + (c2 + K + 1)];
  }
  __syncthreads();
  if (threadIdx.x < MI * MI) {
    T l[MI], o[B];
#pragma unroll
    for (int K = 0; K < MI; ++K) l[K] = Z[threadIdx.x * MI + K];
    solve_spread<T, B>(l, o);
    T* dst = a.t2 + blk * T2B + threadIdx.x * B;
#pragma unroll
    for (int x = 0; x < B; ++x) dst[x] = o[x];
  }
}

// y spread of one half's columns: t2 -> T1[MI][B][HW]
template <typename T>
__device__ inline void w33_spread_y(const W33Args<T>& a, int64_t blk, int h, T* T1) {
  using namespace w33;
  const int tid = threadIdx.x;
  if (tid < MI * HW) {
    const int J = tid / HW, c = tid - (tid / HW) * HW;
    T l[MI], o[B];
    const T* src = a.t2 + blk * T2B + J * MI * B + x0(h) + c;
#pragma unroll
    for (int I = 0; I < MI; ++I) l[I] = src[I * B];
    solve_spread<T, B>(l, o);
#pragma unroll
    for (int y = 0; y < B; ++y) T1[(J * B + y) * HW + c] = o[y];
  }
}

// Transpose of a decomposition level, per half: v = g + K^T cbar on the
// fine nodes, then cbar - P3^T v on the coarse nodes, added into G^{s-1}.
template <typename T>
__global__ __launch_bounds__(w33::NT) void k_w33_dec_T(W33Args<T> a) {
  using namespace w33;
  __shared__ T lds[MC * B * HW];       // T1 [MI][B][HW], then R [MC][B][HW]
  const int64_t g = blockIdx.x;
  if (g >= 2 * a.c.nblocks) return;
  const int h = int(g & 1);
  int64_t bz, by, bx;
  color_block(a.c, g >> 1, bz, by, bx);
  const int64_t blk = (bz * a.nb[1] + by) * a.nb[2] + bx;
  w33_spread_y(a, blk, h, lds);
  __syncthreads();
  const int tid = threadIdx.x;
  const bool act = tid < NCOL;
  const int y = act ? tid / HW : 0, xl = act ? tid - (tid / HW) * HW : 0, x = x0(h) + xl;
  const bool ecol = ((y | x) & 1) == 0;
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  T gv[B], v[B];
  if (act) {
    const bool own_yx = (y < B - 1 || by == a.nb[1] - 1) && (x < B - 1 || bx == a.nb[2] - 1);
    const bool lastz = bz == a.nb[0] - 1;
    const T* col = a.gc + gy * a.cs[1] + gx * a.cs[2];
    const T* ccol = a.gcur + (gy >> 1) * a.cn[2] + (gx >> 1);
    const int64_t cpl = a.cn[1] * a.cn[2];
#pragma unroll
    for (int z = 0; z < B; ++z) {
      T w = T(0);
      if (own_yx && (z < B - 1 || lastz))
        w = (ecol && !(z & 1)) ? ccol[((oz >> 1) + (z >> 1)) * cpl] : col[(oz + z) * a.cs[0]];
      gv[z] = w;
    }
    T l[MI], t[B];
#pragma unroll
    for (int J = 0; J < MI; ++J) l[J] = lds[(J * B + y) * HW + xl];
    solve_spread<T, B>(l, t);
#pragma unroll
    for (int z = 0; z < B; ++z) v[z] = (ecol && !(z & 1)) ? T(0) : gv[z] + t[z];
  }
  __syncthreads();                     // T1 is dead: R takes its place
  if (act) {
#pragma unroll
    for (int j = 0; j < MC; ++j) lds[(j * B + y) * HW + xl] = restrict_z33<T>(v, j);
  }
  __syncthreads();
  if (act && stores(h, x)) {
    if (ecol) {
#pragma unroll
      for (int j = 0; j < MC; ++j) v[2 * j] = gv[2 * j] - gather33<T>(lds, j, y, xl, x);
    }
    const bool fy = first_on_axis<B>(y, by, a.c.nb[1]), fx = first_on_axis<B>(x, bx, a.c.nb[2]);
    T* dst = a.out + gy * a.on[2] + gx;
    const int64_t pl = a.on[1] * a.on[2];
#pragma unroll
    for (int z = 0; z < B; ++z) put(dst + (oz + z) * pl, v[z], fy && fx && first_on_axis<B>(z, bz, a.c.nb[0]));
  }
}

// gradient of G^{s-1} on the nodes a block owns (zero elsewhere), one column
template <typename T>
__device__ inline void w33_owned_column(const W33Args<T>& a, int64_t bz, int64_t by, int64_t bx, int y, int x,
                                        T (&gv)[w33::B]) {
  using namespace w33;
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  const bool own_yx = (y < B - 1 || by == a.nb[1] - 1) && (x < B - 1 || bx == a.nb[2] - 1) && gy < a.lim[1] &&
                      gx < a.lim[2];
  const bool lastz = bz == a.nb[0] - 1;
  const T* col = a.gin + gy * a.in[2] + gx;
  const int64_t pl = a.in[1] * a.in[2];
#pragma unroll
  for (int z = 0; z < B; ++z)
    gv[z] = (own_yx && (z < B - 1 || lastz) && oz + z < a.lim[0]) ? col[(oz + z) * pl] : T(0);
}

// Transpose of a recomposition level, first part per half: r = P3^T g at
// the coarse nodes, added into the coarse grid's gradient; the interior ones
// also go to zs for the transposed correction.
template <typename T>
__global__ __launch_bounds__(w33::NT) void k_w33_rec_T_coarse(W33Args<T> a) {
  using namespace w33;
  __shared__ T R[MC * B * HW];
  const int64_t g = blockIdx.x;
  if (g >= 2 * a.c.nblocks) return;
  const int h = int(g & 1);
  int64_t bz, by, bx;
  color_block(a.c, g >> 1, bz, by, bx);
  const int64_t blk = (bz * a.nb[1] + by) * a.nb[2] + bx;
  const int tid = threadIdx.x;
  const bool act = tid < NCOL;
  const int y = act ? tid / HW : 0, xl = act ? tid - (tid / HW) * HW : 0, x = x0(h) + xl;
  const bool ecol = ((y | x) & 1) == 0;
  if (act) {
    T gv[B];
    w33_owned_column(a, bz, by, bx, y, x, gv);
#pragma unroll
    for (int j = 0; j < MC; ++j) R[(j * B + y) * HW + xl] = restrict_z33<T>(gv, j);
  }
  __syncthreads();
  if (act && ecol && stores(h, x)) {
    const bool fy = first_on_axis<B>(y, by, a.c.nb[1]), fx = first_on_axis<B>(x, bx, a.c.nb[2]);
    const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
    T* cdst = const_cast<T*>(a.gcur) + (gy >> 1) * a.cn[2] + (gx >> 1);
    const int64_t cpl = a.cn[1] * a.cn[2];
    const bool icol = y >= 2 && y <= B - 3 && x >= 2 && x <= B - 3;
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      const T rc = gather33<T>(R, j, y, xl, x);
      put(cdst + ((oz >> 1) + j) * cpl, rc, fy && fx && first_on_axis<B>(2 * j, bz, a.c.nb[0]));
      if (icol && j >= 1 && j <= MC - 2) a.zs[blk * ZB + ((j - 1) * MI + ((y - 2) >> 1)) * MI + ((x - 2) >> 1)] = rc;
    }
  }
}

// Transpose of a recomposition level, last part per half: g - K^T r on the
// fine nodes, added into the coefficients' gradient.
template <typename T>
__global__ __launch_bounds__(w33::NT) void k_w33_rec_T_fine(W33Args<T> a) {
  using namespace w33;
  __shared__ T T1[MI * B * HW];
  const int64_t g = blockIdx.x;
  if (g >= 2 * a.c.nblocks) return;
  const int h = int(g & 1);
  int64_t bz, by, bx;
  color_block(a.c, g >> 1, bz, by, bx);
  const int64_t blk = (bz * a.nb[1] + by) * a.nb[2] + bx;
  w33_spread_y(a, blk, h, T1);
  __syncthreads();
  const int tid = threadIdx.x;
  const bool act = tid < NCOL;
  const int y = act ? tid / HW : 0, xl = act ? tid - (tid / HW) * HW : 0, x = x0(h) + xl;
  if (!(act && stores(h, x))) return;
  const bool ecol = ((y | x) & 1) == 0;
  T gv[B], l[MI], t[B];
  w33_owned_column(a, bz, by, bx, y, x, gv);
#pragma unroll
  for (int J = 0; J < MI; ++J) l[J] = T1[(J * B + y) * HW + xl];
  solve_spread<T, B>(l, t);
  const bool fy = first_on_axis<B>(y, by, a.c.nb[1]), fx = first_on_axis<B>(x, bx, a.c.nb[2]);
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  T* dst = const_cast<T*>(a.gc) + gy * a.cs[1] + gx * a.cs[2];
#pragma unroll
  for (int z = 0; z < B; ++z) {
    if (ecol && !(z & 1)) continue;    // coarse nodes: the coarse part above
    put(dst + (oz + z) * a.cs[0], gv[z] - t[z], fy && fx && first_on_axis<B>(z, bz, a.c.nb[0]));
  }
}

template <typename T>
W33Args<T> w33_args(const bm_plan_s& p, int s) {
  const Level& L = p.lv[s - 1];
  W33Args<T> a{};
  for (int k = 0; k < 3; ++k) {
    a.cn[k] = L.m[k];
    a.nb[k] = L.nb[k];
  }
  const int64_t nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  if (size_t(nblocks) * w33::T2B > p.ws.t_elems) fail(BM_EINVAL, "plan workspace too small for 33^3 blocks");
  a.t2 = static_cast<T*>(p.ws.t1);
  a.zs = static_cast<T*>(p.ws.t2);
  return a;
}

template <typename T>
void launch_w33_dec_T(const bm_plan_s& p, int s, const void* gcoeff, void* out, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  W33Args<T> a = w33_args<T>(p, s);
  const View3 cv = level_view(p, s, const_cast<void*>(gcoeff));
  a.gc = static_cast<const T*>(cv.ptr);
  a.gcur = static_cast<const T*>(p.ws.grid[s]);
  a.out = static_cast<T*>(out);
  for (int k = 0; k < 3; ++k) {
    a.cs[k] = cv.s[k];
    a.on[k] = L.n[k];
  }
  const int64_t nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  hipLaunchKernelGGL(k_w33_spread_x<T>, dim3(unsigned(nblocks)), dim3(256), 0, st, a, 0);
  BM_HIP(hipGetLastError());
  for (int color = 0; color < 8; ++color) {
    a.c = color_set(L, color, 1);
    if (a.c.nblocks == 0) continue;
    hipLaunchKernelGGL(k_w33_dec_T<T>, dim3(unsigned(2 * a.c.nblocks)), dim3(w33::NT), 0, st, a);
    BM_HIP(hipGetLastError());
  }
}

template <typename T>
void launch_w33_rec_T(const bm_plan_s& p, int s, const void* gin, const int64_t in[3], const int64_t lim[3],
                      void* gcoeff, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  W33Args<T> a = w33_args<T>(p, s);
  const View3 cv = level_view(p, s, gcoeff);
  a.gc = static_cast<const T*>(cv.ptr);
  a.gcur = static_cast<const T*>(p.ws.grid[s]);
  a.gin = static_cast<const T*>(gin);
  for (int k = 0; k < 3; ++k) {
    a.cs[k] = cv.s[k];
    a.in[k] = in[k];
    a.lim[k] = lim[k];
  }
  const int64_t nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  for (int color = 0; color < 8; ++color) {
    a.c = color_set(L, color, 1);
    if (a.c.nblocks == 0) continue;
    hipLaunchKernelGGL(k_w33_rec_T_coarse<T>, dim3(unsigned(2 * a.c.nblocks)), dim3(w33::NT), 0, st, a);
    BM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_w33_spread_x<T>, dim3(unsigned(nblocks)), dim3(256), 0, st, a, 1);
  BM_HIP(hipGetLastError());
  for (int color = 0; color < 8; ++color) {
    a.c = color_set(L, color, 1);
    if (a.c.nblocks == 0) continue;
    hipLaunchKernelGGL(k_w33_rec_T_fine<T>, dim3(unsigned(2 * a.c.nblocks)), dim3(w33::NT), 0, st, a);
    BM_HIP(hipGetLastError());
  }
}

template <typename T>
void local_dec_T(const bm_plan_s& p, int s, const void* gcoeff, void* out, hipStream_t st) {
  if (p.lv[s - 1].b == 33)
    launch_w33_dec_T<T>(p, s, gcoeff, out, st);
  else if (p.lv[s - 1].b == 9)
    launch_local_dec_T<T, 9>(p, s, gcoeff, out, st);
  else
    launch_local_dec_T<T, 17>(p, s, gcoeff, out, st);
}

template <typename T>
void local_rec_T(const bm_plan_s& p, int s, const void* gin, const int64_t in[3], const int64_t lim[3], void* gcoeff,
                 hipStream_t st) {
  if (p.lv[s - 1].b == 33)
    launch_w33_rec_T<T>(p, s, gin, in, lim, gcoeff, st);
  else if (p.lv[s - 1].b == 9)
    launch_local_rec_T<T, 9>(p, s, gin, in, lim, gcoeff, st);
  else
    launch_local_rec_T<T, 17>(p, s, gin, in, lim, gcoeff, st);
}

// --------------------------------------------------------------- global levels

// K^T along one axis: lines of m coarse values in, lines of nl values out.
template <typename T>
struct PassTArgs {
  const T* in;
  int64_t is[3];          // input strides (dims: n with m along axis)
  int axis;
  T* out;
  int64_t os[3];          // output strides (dims n)
  const T* base;          // optional: out = base + sgn * result
  int64_t bs[3];
  T sgn;
  int mask;               // write zero at the level's coarse nodes
  int cm[3];
  const double* inv;      // reciprocal Thomas pivots of 3 Mc (natural ends), length m
  int64_t nl, m;
  int W, lw;              // lines per tile (a power of two) and its log2
  int64_t nq, ntq;        // extent of the fastest other axis, tiles along it
  int pa, qa;             // the two other axes (q fastest)
};

template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_line_pass_T(PassTArgs<T> a) {
  extern __shared__ unsigned char smem[];
  T* tin = reinterpret_cast<T*>(smem);               // [m][W+1]
  const int WP = a.W + 1;
  T* piv = tin + int(a.m) * WP;                      // [m] reciprocal pivots
  const uint32_t tile = blockIdx.x;
  const uint32_t p = tile / uint32_t(a.ntq);
  const int64_t q0 = int64_t(tile - p * uint32_t(a.ntq)) * a.W;
  const int wv = int(i64min(a.W, a.nq - q0));
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m = int(a.m), nl = int(a.nl);
  const int64_t ibase = int64_t(p) * a.is[a.pa] + q0 * a.is[a.qa];
  for (int J = tid; J < m; J += NT) piv[J] = T(a.inv[J]);
  auto load = [&](int J, int w) { tin[J * WP + w] = a.in[ibase + w * a.is[a.qa] + J * a.is[a.axis]]; };
  if (a.axis == 2) {
    for (int w = wave; w < wv; w += NT / 64)
      for (int J = lane; J < m; J += 64) load(J, w);
  } else {
    const int w = tid & (a.W - 1);
    if (w < wv)
      for (int J = tid >> a.lw; J < m; J += NT >> a.lw) load(J, w);
  }
  __syncthreads();
  // in place: each lane reads, and later overwrites, only its own rows
  solve_lines<T, NT, Q>(m, piv, wv, tid, [&](int w, int J) { return T(3) * tin[J * WP + w]; },
                     [&](int w, int J, T x) { tin[J * WP + w] = x; });
  __syncthreads();
  const bool pe = !(a.cm[a.pa] && (p & 1));
  const int cmA = a.cm[a.axis], cmQ = a.cm[a.qa];
  auto store = [&](int i, int w) {
    // transposed rows of P^T M: row J has 5/6 (5/12 at the two ends) at
    // node 2J, 1/2 at 2J +- 1 and 1/12 at 2J +- 2
    const T* col = tin + w;
    const int h = i >> 1;
    T v;
    if (i & 1) {
      v = T(0.5) * (col[h * WP] + col[(h + 1) * WP]);
    } else {
      v = ((h == 0 || h == m - 1) ? T(5.0 / 12.0) : T(5.0 / 6.0)) * col[h * WP];
      T e = T(0);
      if (h > 0) e += col[(h - 1) * WP];
      if (h + 1 < m) e += col[(h + 1) * WP];
      v += T(1.0 / 12.0) * e;
    }
    int64_t c[3];
    c[a.axis] = i;
    c[a.pa] = p;
    c[a.qa] = q0 + w;
    if (a.mask && pe && !(cmA && (i & 1)) && !(cmQ && ((q0 + w) & 1))) v = T(0);
    else if (a.base) v = a.base[c[0] * a.bs[0] + c[1] * a.bs[1] + c[2] * a.bs[2]] + a.sgn * v;
    a.out[c[0] * a.os[0] + c[1] * a.os[1] + c[2] * a.os[2]] = v;
  };
  if (a.axis == 2) {
    for (int w = wave; w < wv; w += NT / 64)
      for (int i = lane; i < nl; i += 64) store(i, w);
  } else {
    const int w = tid & (a.W - 1);
    if (w < wv)
      for (int i = tid >> a.lw; i < nl; i += NT >> a.lw) store(i, w);
  }
}

template <typename T>
void launch_pass_T(const bm_plan_s& p, int s, int axis, const View3& in, const View3& out, const View3* base,
                   T sgn, bool mask, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  PassTArgs<T> a{};
  a.in = static_cast<const T*>(in.ptr);
  a.out = static_cast<T*>(out.ptr);
  a.base = base ? static_cast<const T*>(base->ptr) : nullptr;
  for (int k = 0; k < 3; ++k) {
    a.is[k] = in.s[k];
    a.os[k] = out.s[k];
    a.bs[k] = base ? base->s[k] : 0;
    a.cm[k] = L.coarsen[k] ? 1 : 0;
  }
  a.sgn = sgn;
  a.mask = mask;
  a.axis = axis;
  a.nl = out.n[axis];
  a.m = in.n[axis];
  if (a.nl < 3 || a.m != (a.nl + 1) / 2 || a.m > 64 * kLineQ) fail(BM_EUNSUPPORTED, "line length not supported");
  a.inv = L.d_inv[axis];
  a.pa = axis == 0 ? 1 : 0;
  a.qa = axis == 2 ? 1 : 2;
  a.nq = out.n[a.qa];
  const int64_t np = out.n[a.pa];
  a.W = tile_width(a.m + 1, sizeof(T), np, a.nq);
  a.lw = 0;
  while ((1 << a.lw) < a.W) ++a.lw;
  a.ntq = (a.nq + a.W - 1) / a.W;
  const int64_t tiles = np * a.ntq;
  if (tiles >= (int64_t(1) << 31)) fail(BM_EUNSUPPORTED, "too many lines");
  const size_t shm = (size_t(a.m) * (a.W + 1) + size_t(a.m)) * sizeof(T);
  switch (row_q_for(a.m)) {
    case 3: hipLaunchKernelGGL((k_line_pass_T<T, 3>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    case 5: hipLaunchKernelGGL((k_line_pass_T<T, 5>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    case 9: hipLaunchKernelGGL((k_line_pass_T<T, 9>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    case 11: hipLaunchKernelGGL((k_line_pass_T<T, 11>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    case kRowQ: hipLaunchKernelGGL((k_line_pass_T<T, kRowQ>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    default: hipLaunchKernelGGL((k_line_pass_T<T, 0>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
  }
  BM_HIP(hipGetLastError());
}

// P3^T at the coarse nodes (dims m) of a dense fine grid (dims n): the
// weighted sum over the 3^3 neighbourhood (an axis that does not coarsen
// contributes the node's own plane only).  self = 0 leaves out the node
// itself; with cbar the result is cbar - sum.  Written through a strided
// view; in place is safe when self = 0, since only coarse nodes are written
// and only fine-only nodes are read.
template <typename T>
struct RestrArgs {
  const T* src;
  int64_t n[3];
  int cm[3];
  int self;
  const T* cbar;          // optional, compact dims m
  T* out;
  int64_t os[3];
  int64_t m[3];
  Unflat32 uf;            // over dims m
};

template <typename T>
__global__ __launch_bounds__(NT) void k_restrict_T(RestrArgs<T> a) {
  const int64_t tot = a.m[0] * a.m[1] * a.m[2];
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < tot; i += int64_t(gridDim.x) * NT) {
    uint32_t uz, uy, ux;
    a.uf(uint32_t(i), uz, uy, ux);
    const int64_t cz = uz, cy = uy, cx = ux;
    const int64_t fz = a.cm[0] ? 2 * cz : cz, fy = a.cm[1] ? 2 * cy : cy, fx = a.cm[2] ? 2 * cx : cx;
    T acc = T(0);
    for (int dz = -a.cm[0]; dz <= a.cm[0]; ++dz) {
      const int64_t zz = fz + dz;
      if (zz < 0 || zz >= a.n[0]) continue;
      for (int dy = -a.cm[1]; dy <= a.cm[1]; ++dy) {
        const int64_t yy = fy + dy;
        if (yy < 0 || yy >= a.n[1]) continue;
        for (int dx = -a.cm[2]; dx <= a.cm[2]; ++dx) {
          const int64_t xx = fx + dx;
          if (xx < 0 || xx >= a.n[2]) continue;
          if (!a.self && dz == 0 && dy == 0 && dx == 0) continue;
          const T w = T((dz ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dx ? 0.5 : 1.0));
          acc += w * a.src[(zz * a.n[1] + yy) * a.n[2] + xx];
        }
      }
    }
    a.out[cz * a.os[0] + cy * a.os[1] + cx * a.os[2]] = a.cbar ? a.cbar[i] - acc : acc;
  }
}

template <typename T>
void launch_restrict_T(const Level& L, const void* src, bool self, const void* cbar, const View3& out,
                       hipStream_t st) {
  RestrArgs<T> a{};
  a.src = static_cast<const T*>(src);
  a.self = self;
  a.cbar = static_cast<const T*>(cbar);
  a.out = static_cast<T*>(out.ptr);
  for (int k = 0; k < 3; ++k) {
    a.n[k] = L.n[k];
    a.cm[k] = L.coarsen[k] ? 1 : 0;
    a.os[k] = out.s[k];
    a.m[k] = L.m[k];
  }
  if (a.m[0] * a.m[1] * a.m[2] >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "coarse grid too large");
  a.uf = Unflat32(a.m[1], a.m[2]);
  hipLaunchKernelGGL(k_restrict_T<T>, dim3(grid_for(a.m[0] * a.m[1] * a.m[2])), dim3(NT), 0, st, a);
  BM_HIP(hipGetLastError());
}

// K3^T applied to the compact coarse grid G^s in the plan's grid buffer, one
// axis at a time (z, y, x, over the axes that coarsen); the last pass writes
// out (dims n) as base + sgn * result, or masked.
template <typename T>
void apply_K3_T(bm_plan_s& p, int s, const View3& out, const View3* base, T sgn, bool mask, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  int axes[3], na = 0;
  for (int a : {0, 1, 2})
    if (L.coarsen[a]) axes[na++] = a;
  void* tmp[2] = {p.ws.t1, p.ws.t2};
  View3 cur = dense_view(p.ws.grid[s], L.m);
  for (int k = 0; k < na; ++k) {
    const int ax = axes[k];
    int64_t on[3] = {cur.n[0], cur.n[1], cur.n[2]};
    on[ax] = L.n[ax];
    if (k == na - 1) {
      launch_pass_T<T>(p, s, ax, cur, out, base, sgn, mask, st);
    } else {
      const View3 dst = dense_view(tmp[k & 1], on);
      launch_pass_T<T>(p, s, ax, cur, dst, nullptr, T(1), false, st);
      cur = dst;
    }
  }
}

// global decomposition level transposed: grid[s] holds cbar; out (dense, dims
// n) receives the gradient of G^{s-1}
template <typename T>
void global_dec_T(bm_plan_s& p, int s, const void* gcoeff, void* out, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  const View3 ov = dense_view(out, L.n);
  const View3 gv = level_view(p, s, const_cast<void*>(gcoeff));
  apply_K3_T<T>(p, s, ov, &gv, T(1), true, st);
  View3 cview = ov;
  for (int k = 0; k < 3; ++k) {
    cview.n[k] = L.m[k];
    cview.s[k] = L.coarsen[k] ? 2 * ov.s[k] : ov.s[k];
  }
  launch_restrict_T<T>(L, out, false, p.ws.grid[s], cview, st);
}

// global recomposition level transposed: gin (dense, dims n) is the gradient
// of G^{s-1}; grid[s] receives r = P3^T gin, the coefficient view gin - K3^T r
template <typename T>
void global_rec_T(bm_plan_s& p, int s, const void* gin, void* gcoeff, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  launch_restrict_T<T>(L, gin, true, nullptr, dense_view(p.ws.grid[s], L.m), st);
  const View3 base = dense_view(const_cast<void*>(gin), L.n);
  apply_K3_T<T>(p, s, level_view(p, s, gcoeff), &base, T(-1), false, st);
}

// transpose of the padding: gx = sum of the padded gradient over the padded
// nodes that read each logical node (clamp), or the crop (zero fill)
template <typename T>
__global__ __launch_bounds__(NT) void k_unpad_T(const T* gp, int64_t p0, int64_t p1, int64_t p2, T* gx, int64_t n0,
                                                int64_t n1, int64_t n2, Unflat32 uf, int zero) {
  const int64_t tot = n0 * n1 * n2;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < tot; i += int64_t(gridDim.x) * NT) {
    uint32_t uz, uy, ux;
    uf(uint32_t(i), uz, uy, ux);
    const int64_t z = uz, y = uy, x = ux;
    const int64_t ze = (!zero && z == n0 - 1) ? p0 : z + 1;
    const int64_t ye = (!zero && y == n1 - 1) ? p1 : y + 1;
    const int64_t xe = (!zero && x == n2 - 1) ? p2 : x + 1;
    T acc = T(0);
    for (int64_t zz = z; zz < ze; ++zz)
      for (int64_t yy = y; yy < ye; ++yy)
        for (int64_t xx = x; xx < xe; ++xx) acc += gp[(zz * p1 + yy) * p2 + xx];
    gx[i] = acc;
  }
}

template <typename T>
void decompose_adjoint_t(bm_plan_s& p, const void* gcoeff, void* gx, hipStream_t st) {
  const Level& last = p.lv[p.nlev - 1];
  strided_copy(p.esize, coarsest_view(p, const_cast<void*>(gcoeff)), dense_view(p.ws.grid[p.nlev], last.m), st);
  const bool padded = p.dims[0] != p.pdims[0] || p.dims[1] != p.pdims[1] || p.dims[2] != p.pdims[2];
  void* top = gx;
  if (padded) {
    if (p.L == 0) {
      top = p.ws.grid[0];
    } else {
      if (!p.ws.gpad) plan_alloc(p, &p.ws.gpad, size_t(p.pdims[0] * p.pdims[1] * p.pdims[2]) * p.esize);
      top = p.ws.gpad;
    }
  }
  for (int s = p.nlev; s >= 1; --s) {
    const Level& L = p.lv[s - 1];
    void* out = s > 1 ? p.ws.grid[s - 1] : top;
    if (L.local)
      local_dec_T<T>(p, s, gcoeff, out, st);
    else
      global_dec_T<T>(p, s, gcoeff, out, st);
  }
  if (padded) {
    const int64_t tot = p.dims[0] * p.dims[1] * p.dims[2];
    if (tot >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "grid too large for the pad transpose");
    hipLaunchKernelGGL(k_unpad_T<T>, dim3(grid_for(tot)), dim3(NT), 0, st, static_cast<const T*>(top), p.pdims[0],
                       p.pdims[1], p.pdims[2], static_cast<T*>(gx), p.dims[0], p.dims[1], p.dims[2],
                       Unflat32(p.dims[1], p.dims[2]), p.cfg.pad_mode == 1 ? 1 : 0);
    BM_HIP(hipGetLastError());
  }
}

template <typename T>
void recompose_adjoint_t(bm_plan_s& p, const void* gx, void* gcoeff, hipStream_t st) {
  const bool padded = p.dims[0] != p.pdims[0] || p.dims[1] != p.pdims[1] || p.dims[2] != p.pdims[2];
  for (int s = 1; s <= p.nlev; ++s) {
    const Level& L = p.lv[s - 1];
    if (L.local) {
      // level 1 reads the logical gradient; the crop's transpose is zero beyond it
      const void* gin = s == 1 ? gx : p.ws.grid[s - 1];
      const int64_t* dims = s == 1 ? p.dims : L.n;
      local_rec_T<T>(p, s, gin, dims, dims, gcoeff, st);
    } else {
      const void* gin = p.ws.grid[s - 1];
      if (s == 1) {
        if (padded)
          pad_input(p, gx, p.ws.grid[0], true, st);
        else
          gin = gx;
      }
      global_rec_T<T>(p, s, gin, gcoeff, st);
    }
  }
  const Level& last = p.lv[p.nlev - 1];
  strided_copy(p.esize, dense_view(p.ws.grid[p.nlev], last.m), coarsest_view(p, gcoeff), st);
}

}  // namespace

void decompose_adjoint(bm_plan_s& p, const void* gcoeff, void* gx, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    decompose_adjoint_t<float>(p, gcoeff, gx, st);
  else
    decompose_adjoint_t<double>(p, gcoeff, gx, st);
}

void recompose_adjoint(bm_plan_s& p, const void* gx, void* gcoeff, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    recompose_adjoint_t<float>(p, gx, gcoeff, st);
  else
    recompose_adjoint_t<double>(p, gx, gcoeff, st);
}

}  // namespace bm
