// Global MGARD levels (Sec. II-B; run on the block-coarse grid in the hybrid
// hierarchy of Sec. IV-B) and the decompose / recompose drivers.
//
// A global level on grid G (dims n) with coarse grid C (dims m):
//   details  d = u - multilinear interpolant of u_C, on the fine-only nodes;
//   coarse   c = K_z K_y K_x u with K = Mc^{-1} P^T M per axis (natural
//            ends).  Because K P = I this equals u_C + K w of the
//            step-by-step definition (w = u - P u_C), i.e. the L2 projection.
// Recomposition: z = K_z K_y K_x w (w = details, zero on coarse nodes),
// u_C = c - z, u = interpolant(u_C) + w.
//
// Each K along one axis is a "line pass": restriction by P^T M (5-point
// rows {1/12, 1/2, 5/6, 1/2, 1/12}; end rows {5/12, 1/2, 1/12}) and a solve
// with 3 Mc = tridiag(1, 4, 1) (end diagonals 2).  A workgroup stages a tile
// of lines in LDS (coalesced loads); one wavefront solves a line with its
// lanes: both Thomas sweeps are first-order affine recurrences, evaluated
// by a lane-local pass and a 64-lane scan of affine maps with wave shuffles.

#include <type_traits>
#include <utility>

#include "internal.h"
#include "line_solve.h"

namespace bm {
namespace {

constexpr int NT = 256;

// ------------------------------------------------------------- elementwise

// Grid dims plus a 32-bit multiply-high unflattening of node indices (a
// 64-bit division per element would dominate these memory-bound kernels).
struct Idx3 {
  int64_t n0 = 0, n1 = 0, n2 = 0;
  Unflat32 uf;
  Idx3() = default;
  Idx3(int64_t a, int64_t b, int64_t c) : n0(a), n1(b), n2(c), uf(b, c) {
    if (a * b * c >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "a global level grid must have fewer than 2^32 nodes");
  }
};

__device__ inline void unflat(int64_t i, const Idx3& d, int64_t& z, int64_t& y, int64_t& x) {
  uint32_t zz, yy, xx;
  d.uf(uint32_t(i), zz, yy, xx);
  z = zz;
  y = yy;
  x = xx;
}

template <typename T>
struct DetArgs {
  const T* u;            // compact G^{s-1}
  Idx3 n;
  Idx3 m;                // dims of G^s: one thread per coarse cell
  int cm0, cm1, cm2;     // 1 if the axis coarsens at this level
  T* coeff;
  int64_t cs[3];
  int32_t* codes;        // fused quantization: write codes instead (same strides)
  const double* qinv;    // 1/Delta of this level (device scalar)
  int64_t* flag;         // set when a code does not fit in int32
};

// q = rint(c * (1/Delta)) in FP64; a code outside int32 raises the flag
template <typename T>
__device__ inline int32_t quant_g(T c, double inv, int64_t* flag) {
  const double v = rint(mul_rn(double(c), inv));
  if (!(fabs(v) <= 2147483647.0)) {
    atomicOr(reinterpret_cast<unsigned long long*>(flag), (unsigned long long)code_flag(double(c)));
    return 0;
  }
  return int32_t(v);
}

// The fine-only nodes of a global level are handled per coarse cell: the
// thread of coarse node (cz, cy, cx) takes the nodes 2c + d, d in {0,1}^3
// (d = 1 only along axes that coarsen and stay inside the grid), so the 8
// cell corners are read once for its 7 nodes.  The interpolant at 2c + d is
// the mean of the corners c + {0, d} per axis, summed in the order z-plane,
// y-row, x-pair.
template <typename T>
struct Cell {
  T c[2][2][2];   // corners c + (0|1, 0|1, 0|1); index 1 only where the offset exists
  int oz, oy, ox; // offset 1 exists along the axis
  __device__ inline T interp(int dz, int dy, int dx) const {
    return cell_mean<T>(dz, dy, dx, [&](int az, int ay, int ax) { return c[az][ay][ax]; });
  }
};

// corners from a reader of coarse-grid values at coarse coordinates
template <typename T, typename F>
__device__ inline void load_corners(Cell<T>& k, int64_t cz, int64_t cy, int64_t cx, F rd) {
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx)
        k.c[dz][dy][dx] = (dz <= k.oz && dy <= k.oy && dx <= k.ox) ? rd(cz + dz, cy + dy, cx + dx) : T(0);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_details(DetArgs<T> a) {
  const int64_t tot = a.m.n0 * a.m.n1 * a.m.n2;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < tot; i += int64_t(gridDim.x) * NT) {
    int64_t cz, cy, cx;
    unflat(i, a.m, cz, cy, cx);
    const int64_t z = a.cm0 ? 2 * cz : cz, y = a.cm1 ? 2 * cy : cy, x = a.cm2 ? 2 * cx : cx;
    Cell<T> k;
    k.oz = a.cm0 && z + 1 < a.n.n0;
    k.oy = a.cm1 && y + 1 < a.n.n1;
    k.ox = a.cm2 && x + 1 < a.n.n2;
    auto U = [&](int64_t zz, int64_t yy, int64_t xx) { return a.u[(zz * a.n.n1 + yy) * a.n.n2 + xx]; };
    load_corners(k, cz, cy, cx, [&](int64_t zz, int64_t yy, int64_t xx) {
      return U(a.cm0 ? 2 * zz : zz, a.cm1 ? 2 * yy : yy, a.cm2 ? 2 * xx : xx);
    });
    const double inv = a.codes ? *a.qinv : 0.0;
    // the cell's fine values are all fetched before the first store
    T f[8];
#pragma unroll
    for (int t = 1; t < 8; ++t) {
      const int dz = t >> 2, dy = (t >> 1) & 1, dx = t & 1;
      f[t] = (dz > k.oz || dy > k.oy || dx > k.ox) ? T(0) : U(z + dz, y + dy, x + dx);
    }
#pragma unroll
    for (int t = 1; t < 8; ++t) {
      const int dz = t >> 2, dy = (t >> 1) & 1, dx = t & 1;
      if (dz > k.oz || dy > k.oy || dx > k.ox) continue;
      const T d = f[t] - k.interp(dz, dy, dx);
      const int64_t o = (z + dz) * a.cs[0] + (y + dy) * a.cs[1] + (x + dx) * a.cs[2];
      if (a.codes)
        a.codes[o] = quant_g(d, inv, a.flag);
      else
        a.coeff[o] = d;
    }
  }
}

template <typename T>
struct IntArgs {
  const T* coeff;
  int64_t cs[3];
  const T* uc;           // compact G^s (coarse values u_C)
  Idx3 m;
  Idx3 n;                // dims of G^{s-1}
  int cm0, cm1, cm2;
  T* out;                // dense G^{s-1}
  const int32_t* codes;  // fused dequantization: details from codes (same strides)
  const double* qdel;    // Delta of this level (device scalar)
};

template <typename T>
__global__ __launch_bounds__(NT) void k_interp_add(IntArgs<T> a) {
  const int64_t tot = a.m.n0 * a.m.n1 * a.m.n2;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < tot; i += int64_t(gridDim.x) * NT) {
    int64_t cz, cy, cx;
    unflat(i, a.m, cz, cy, cx);
    const int64_t z = a.cm0 ? 2 * cz : cz, y = a.cm1 ? 2 * cy : cy, x = a.cm2 ? 2 * cx : cx;
    Cell<T> k;
    k.oz = a.cm0 && z + 1 < a.n.n0;
    k.oy = a.cm1 && y + 1 < a.n.n1;
    k.ox = a.cm2 && x + 1 < a.n.n2;
    load_corners(k, cz, cy, cx,
                 [&](int64_t zz, int64_t yy, int64_t xx) { return a.uc[(zz * a.m.n1 + yy) * a.m.n2 + xx]; });
    const double del = a.codes ? *a.qdel : 0.0;
    // the cell's details are all fetched before the first store
    T w[8];
    int32_t qc[8];
    auto co = [&](int t) {
      return (z + (t >> 2)) * a.cs[0] + (y + ((t >> 1) & 1)) * a.cs[1] + (x + (t & 1)) * a.cs[2];
    };
    auto in = [&](int t) { return !((t >> 2) > k.oz || ((t >> 1) & 1) > k.oy || (t & 1) > k.ox); };
    if (a.codes) {
#pragma unroll
      for (int t = 1; t < 8; ++t) qc[t] = in(t) ? a.codes[co(t)] : 0;
    } else {
#pragma unroll
      for (int t = 1; t < 8; ++t) w[t] = in(t) ? a.coeff[co(t)] : T(0);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int dz = t >> 2, dy = (t >> 1) & 1, dx = t & 1;
      if (dz > k.oz || dy > k.oy || dx > k.ox) continue;
      const int64_t o = ((z + dz) * a.n.n1 + (y + dy)) * a.n.n2 + (x + dx);
      if (t == 0) {
        a.out[o] = k.c[0][0][0];
        continue;
      }
      const T wt = a.codes ? T(mul_rn(double(qc[t]), del)) : w[t];
      a.out[o] = wt + k.interp(dz, dy, dx);
    }
  }
}

template <typename T>
struct CopyArgs {
  const T* src;
  int64_t ss[3];
  T* dst;
  int64_t ds[3];
  Idx3 n;
};

template <typename T>
__global__ __launch_bounds__(NT) void k_copy(CopyArgs<T> a) {
  const int64_t tot = a.n.n0 * a.n.n1 * a.n.n2;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < tot; i += int64_t(gridDim.x) * NT) {
    int64_t z, y, x;
    unflat(i, a.n, z, y, x);
    a.dst[z * a.ds[0] + y * a.ds[1] + x * a.ds[2]] = a.src[z * a.ss[0] + y * a.ss[1] + x * a.ss[2]];
  }
}

// Pad the logical input to the padded grid (clamp or zero fill).
template <typename T>
struct PadArgs {
  const T* src;
  Idx3 sn;
  T* dst;
  Idx3 dn;
  int zero;
};

template <typename T>
__global__ __launch_bounds__(NT) void k_pad(PadArgs<T> a) {
  const int64_t tot = a.dn.n0 * a.dn.n1 * a.dn.n2;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < tot; i += int64_t(gridDim.x) * NT) {
    int64_t z, y, x;
    unflat(i, a.dn, z, y, x);
    const bool in = z < a.sn.n0 && y < a.sn.n1 && x < a.sn.n2;
    T v;
    if (!in && a.zero) {
      v = T(0);
    } else {
      z = z < a.sn.n0 ? z : a.sn.n0 - 1;
      y = y < a.sn.n1 ? y : a.sn.n1 - 1;
      x = x < a.sn.n2 ? x : a.sn.n2 - 1;
      v = a.src[(z * a.sn.n1 + y) * a.sn.n2 + x];
    }
    a.dst[i] = v;
  }
}

// The extension of a padded grid whose logical region already sits at its
// place in it (the padded strides): nodes past the logical extent take the
// value of the nearest logical node, or zero.  The extension is walked as
// three slabs (z past the end; then y past the end; then x past the end), so
// only nodes outside the logical region are written and only nodes inside
// it are read.
template <typename T>
struct PadExtArgs {
  T* g;
  int64_t sn[3], dn[3];   // logical and padded dims
  Idx3 ez, ey, ex;        // the three slabs
  int zero;
};

template <typename T>
__global__ __launch_bounds__(NT) void k_pad_extend(PadExtArgs<T> a) {
  const int64_t nz = a.ez.n0 * a.ez.n1 * a.ez.n2, ny = a.ey.n0 * a.ey.n1 * a.ey.n2;
  const int64_t tot = nz + ny + a.ex.n0 * a.ex.n1 * a.ex.n2;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < tot; i += int64_t(gridDim.x) * NT) {
    int64_t z, y, x;
    if (i < nz) {
      unflat(i, a.ez, z, y, x);
      z += a.sn[0];
    } else if (i < nz + ny) {
      unflat(i - nz, a.ey, z, y, x);
      y += a.sn[1];
    } else {
      unflat(i - nz - ny, a.ex, z, y, x);
      x += a.sn[2];
    }
    T v = T(0);
    if (!a.zero) {
      const int64_t cz = z < a.sn[0] ? z : a.sn[0] - 1, cy = y < a.sn[1] ? y : a.sn[1] - 1;
      const int64_t cx = x < a.sn[2] ? x : a.sn[2] - 1;
      v = a.g[(cz * a.dn[1] + cy) * a.dn[2] + cx];
    }
    a.g[(z * a.dn[1] + y) * a.dn[2] + x] = v;
  }
}

inline unsigned grid_for(int64_t tot) {
  int64_t g = (tot + NT - 1) / NT;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return unsigned(g);
}

// ------------------------------------------------------------- line pass

template <typename T>
struct PassArgs {
  const T* in;
  int64_t is[3];         // input strides
  int64_t n[3];          // input dims
  int axis;              // axis of the lines
  int mask;              // zero the level's coarse nodes on load
  int cm[3];             // coarsening flags (coarse node: every coarsening coordinate even)
  T* out;                // dense, dims on
  int64_t on[3];
  const T* base;         // optional: out = base - result (dense, dims on)
  const int32_t* qin;    // optional: read codes (same strides as in) and dequantize with *qdel
  const double* qdel;
  const double* inv;     // Thomas reciprocal pivots, length m
  int64_t nl, m;         // line length, coarse length
  int W, lw;             // lines per tile (a power of two) and its log2
  int64_t nq;            // extent of the fastest other axis
  int64_t nlines;        // lines in all: tile t takes lines t*W .. t*W+W-1 of (p, q) in row order
  FastDiv fq;            // line index -> (p, q)
  int pa, qa;            // the two other axes (q fastest)
  int solve_only;        // lines of m values that already hold 3 P^T M u: solve only
  float* out_f32;        // optional: the result narrowed to FP32 here instead of out
  // the coarsest values of the hierarchy in the code array (last pass of the
  // last level only): the result quantized into cout instead of out, or the
  // base values dequantized from cbase instead of read from base
  int32_t* cout;
  const int32_t* cbase;
  int64_t cst[3];        // strides of those codes per axis
  const double* cq;      // 1/Delta for cout, Delta for cbase (device scalar)
  int64_t* flag;         // set when a code does not fit in int32
};

// The coarsest values' codes for the last line pass of the hierarchy.
struct CoarseIO {
  int32_t* cout = nullptr;
  const int32_t* cbase = nullptr;
  int64_t s[3] = {0, 0, 0};
  const double* q = nullptr;
  int64_t* flag = nullptr;
};

constexpr int kU = 8;   // requests in flight per lane in the line passes

template <typename T, int Q>
__global__ __launch_bounds__(NT) void k_line_pass(PassArgs<T> a) {
  extern __shared__ unsigned char smem[];
  const int WP = a.W + 1;
  const int nl = int(a.nl), m = int(a.m);
  T* piv = reinterpret_cast<T*>(smem);                 // [m] reciprocal pivots
  T* tin = piv + m;                                    // [nl][W+1]
  // the solution overwrites the first m rows of its own line: a line is
  // solved by one wavefront, which reads all of its right-hand side first
  T* tout = tin;                                       // [m][W+1]
  const int64_t L0 = int64_t(blockIdx.x) * a.W;
  const int wv = int(i64min(a.W, a.nlines - L0));   // valid lines in this tile
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t sA = a.is[a.axis], sQ = a.is[a.qa], sP = a.is[a.pa];
  const int cmA = a.cm[a.axis], cmQ = a.cm[a.qa], cmP = a.cm[a.pa];
  // line w of the tile: its coordinates (p, q) on the two other axes
  auto line = [&](int w, uint32_t& p, uint32_t& q) {
    const uint32_t l = uint32_t(L0 + w);
    p = a.fq.div(l);
    q = l - p * uint32_t(a.nq);
  };
  // Loads are issued kU at a time before any of them is written to LDS, so a
  // lane keeps kU requests in flight instead of waiting on each element.
  // (codes are dequantized after the batch has arrived)
  const double qd = a.qin ? *a.qdel : 0.0;
  auto value = [&](auto r) -> T {
    if constexpr (std::is_same_v<decltype(r), int32_t>)
      return T(mul_rn(double(r), qd));
    else
      return r;
  };
  // coarse-node test of line (p, q) at position i: every coarsening coordinate even
  auto masked = [&](uint32_t p, uint32_t q, int i) {
    return a.mask && !(cmP && (p & 1)) && !(cmQ && (q & 1)) && !(cmA && (i & 1));
  };
  auto load = [&](const auto* src) {
    using R = std::remove_const_t<std::remove_pointer_t<decltype(src)>>;
    if (a.axis == 2) {
      // a wavefront per line (rows are contiguous): the wave's lines
      // wave, wave + NW, ... in 64-wide slots, spl slots per line
      constexpr int NW = NT / 64;
      const int spl = (nl + 63) >> 6;
      const int tot = wave < wv ? ((wv - wave + NW - 1) / NW) * spl : 0;
      int lw = 0, sl = 0;
      for (int g0 = 0; g0 < tot; g0 += kU) {
        R v[kU];
        int dst[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int i = sl * 64 + lane, w = wave + lw * NW;
          dst[u] = -1;
          if (g0 + u < tot && i < nl) {
            uint32_t p, q;
            line(w, p, q);
            dst[u] = masked(p, q, i) ? -2 - (i * WP + w) : i * WP + w;
            v[u] = src[int64_t(p) * sP + int64_t(q) * sQ + int64_t(i) * sA];
          }
          if (++sl == spl) {
            sl = 0;
            ++lw;
          }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (dst[u] >= 0)
            tin[dst[u]] = value(v[u]);
          else if (dst[u] < -1)
            tin[-2 - dst[u]] = T(0);
        }
      }
    } else {
      // the W lines of the tile side by side (W a power of two)
      const int w = tid & (a.W - 1);
      if (w >= wv) return;
      uint32_t p, q;
      line(w, p, q);
      const R* lp = src + int64_t(p) * sP + int64_t(q) * sQ;
      const int di = NT >> a.lw;
      const int64_t step = int64_t(di) * sA;
      for (int ib = tid >> a.lw; ib < nl; ib += kU * di) {
        const R* bp = lp + int64_t(ib) * sA;
        R v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (ib + u * di < nl) v[u] = bp[u * step];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int i = ib + u * di;
          if (i < nl) tin[i * WP + w] = masked(p, q, i) ? T(0) : value(v[u]);
        }
      }
    }
  };
  // the pivots (m <= 3 NT) are fetched with the first batch
  static_assert(64 * kLineQ <= 3 * NT, "pivots: three per thread");
  double pv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) pv[k] = tid + k * NT < m ? a.inv[tid + k * NT] : 0.0;
  if (a.qin)
    load(a.qin);
  else
    load(a.in);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (tid + k * NT < m) piv[tid + k * NT] = T(pv[k]);
  __syncthreads();
  // right-hand side 3 (P^T M u)_J: 5-point interior rows, 3-point end rows
  auto rhs = [&](int w, int J) {
    const T* col = tin + w;
    if (a.solve_only) return col[J * WP];
    const int c = 2 * J;
    T r;
    if (J == 0) {
      r = T(5.0 / 12.0) * col[0] + T(0.5) * col[WP] + T(1.0 / 12.0) * col[2 * WP];
    } else if (J == m - 1) {
      r = T(1.0 / 12.0) * col[(nl - 3) * WP] + T(0.5) * col[(nl - 2) * WP] + T(5.0 / 12.0) * col[(nl - 1) * WP];
    } else {
      r = T(1.0 / 12.0) * (col[(c - 2) * WP] + col[(c + 2) * WP]) + T(0.5) * (col[(c - 1) * WP] + col[(c + 1) * WP]) +
          T(5.0 / 6.0) * col[c * WP];
    }
    return T(3) * r;
  };
  solve_lines<T, NT, Q>(m, piv, wv, tid, rhs, [&](int w, int J, T x) { tout[J * WP + w] = x; });
  __syncthreads();
  const int64_t os[3] = {a.on[1] * a.on[2], a.on[2], 1};
  const int64_t oA = os[a.axis], oQ = os[a.qa], oP = os[a.pa];
  const int64_t cA = a.cst[a.axis], cQ = a.cst[a.qa], cP = a.cst[a.pa];
  // stores kU at a time as well; one loop per kind of store (narrowed to
  // FP32, subtracted from base values, plain, quantized into the coarsest
  // codes, subtracted from the dequantized coarsest codes), so each keeps
  // its loads and stores in flight
  auto store = [&](auto kind) {
    constexpr int K = decltype(kind)::value;
    auto put = [&](const int64_t (&o)[kU], const int64_t (&oc)[kU], const T (&v)[kU]) {
      if constexpr (K == 0) {
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (o[u] >= 0) a.out_f32[o[u]] = float(v[u]);
      } else if constexpr (K == 1) {
        // (every lane loads, from element 0 where it has no value, so that
        // all loads are issued before the first store)
        T r[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) r[u] = a.base[o[u] >= 0 ? o[u] : 0];
#pragma unroll
        for (int u = 0; u < kU; ++u) r[u] -= v[u];
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (o[u] >= 0) a.out[o[u]] = r[u];
      } else if constexpr (K == 4) {
        const double inv = *a.cq;
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (o[u] >= 0) a.cout[oc[u]] = quant_g(v[u], inv, a.flag);
      } else if constexpr (K == 5) {
        const double del = *a.cq;
        int32_t c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) c[u] = a.cbase[o[u] >= 0 ? oc[u] : 0];
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (o[u] >= 0) a.out[o[u]] = T(mul_rn(double(c[u]), del)) - v[u];
      } else {
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (o[u] >= 0) a.out[o[u]] = v[u];
      }
    };
    if (a.axis == 2) {
      constexpr int NW = NT / 64;
      const int spl = (m + 63) >> 6;
      const int tot = wave < wv ? ((wv - wave + NW - 1) / NW) * spl : 0;
      int lw = 0, sl = 0;
      for (int g0 = 0; g0 < tot; g0 += kU) {
        T v[kU];
        int64_t o[kU], oc[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int J = sl * 64 + lane, w = wave + lw * NW;
          o[u] = -1;
          oc[u] = 0;
          v[u] = T(0);
          if (g0 + u < tot && J < m) {
            uint32_t p, q;
            line(w, p, q);
            o[u] = int64_t(p) * oP + int64_t(q) * oQ + int64_t(J) * oA;
            if constexpr (K >= 4) oc[u] = int64_t(p) * cP + int64_t(q) * cQ + int64_t(J) * cA;
            v[u] = tout[J * WP + w];
          }
          if (++sl == spl) {
            sl = 0;
            ++lw;
          }
        }
        put(o, oc, v);
      }
    } else {
      const int w = tid & (a.W - 1);
      if (w >= wv) return;
      uint32_t p, q;
      line(w, p, q);
      const int64_t ob = int64_t(p) * oP + int64_t(q) * oQ;
      const int64_t cb = int64_t(p) * cP + int64_t(q) * cQ;
      const int dJ = NT >> a.lw;
      for (int Jb = tid >> a.lw; Jb < m; Jb += kU * dJ) {
        T v[kU];
        int64_t o[kU], oc[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int J = Jb + u * dJ;
          o[u] = -1;
          oc[u] = 0;
          v[u] = T(0);
          if (J < m) {
            o[u] = ob + int64_t(J) * oA;
            if constexpr (K >= 4) oc[u] = cb + int64_t(J) * cA;
            v[u] = tout[J * WP + w];
          }
        }
        put(o, oc, v);
      }
    }
  };
  if (a.cout)
    store(std::integral_constant<int, 4>{});
  else if (a.cbase)
    store(std::integral_constant<int, 5>{});
  else if (a.out_f32)
    store(std::integral_constant<int, 0>{});
  else if (a.base)
    store(std::integral_constant<int, 1>{});
  else
    store(std::integral_constant<int, 2>{});
}

template <typename T>
void launch_pass(const bm_plan_s& p, int s, int axis, const View3& in, const int64_t cmask[3], void* out,
                 const void* base, const int32_t* qin, const double* qdel, hipStream_t st, bool solve_only = false,
                 float* out_f32 = nullptr, const CoarseIO* cio = nullptr) {
  const Level& L = p.lv[s - 1];
  PassArgs<T> a{};
  a.in = static_cast<const T*>(in.ptr);
  a.qin = qin;
  a.qdel = qdel;
  for (int k = 0; k < 3; ++k) {
    a.is[k] = in.s[k];
    a.n[k] = in.n[k];
    a.on[k] = in.n[k];
    a.cm[k] = L.coarsen[k] ? 1 : 0;
  }
  a.axis = axis;
  a.mask = cmask != nullptr;
  a.nl = in.n[axis];
  a.m = L.m[axis];
  a.on[axis] = a.m;
  a.solve_only = solve_only ? 1 : 0;
  a.out_f32 = out_f32;
  if (cio) {
    if (out_f32 || base) fail(BM_EINVAL, "line pass: coarsest codes with another output kind");
    a.cout = cio->cout;
    a.cbase = cio->cbase;
    for (int k = 0; k < 3; ++k) a.cst[k] = cio->s[k];
    a.cq = cio->q;
    a.flag = cio->flag;
  }
  if (solve_only) {
    if (a.nl != a.m || a.m < 2 || a.m > 64 * kLineQ) fail(BM_EUNSUPPORTED, "line length not supported");
  } else if (a.nl < 3 || a.m != (a.nl + 1) / 2 || a.m > 64 * kLineQ) {
    fail(BM_EUNSUPPORTED, "line length not supported");
  }
  a.out = static_cast<T*>(out);
  a.base = static_cast<const T*>(base);
  a.inv = L.d_inv[axis];
  a.pa = axis == 0 ? 1 : 0;
  a.qa = axis == 2 ? 1 : 2;
  a.nq = in.n[a.qa];
  const int64_t np = in.n[a.pa];
  a.W = tile_width(a.nl + 1, sizeof(T), np, a.nq);
  // rows (x lines) load a wavefront per line, so wider tiles do not coalesce
  // better there; 16 lines keep more workgroups in flight (measured faster)
  if (axis == 2 && a.W > 16) a.W = 16;
  a.lw = 0;
  while ((1 << a.lw) < a.W) ++a.lw;
  a.nlines = np * a.nq;
  if (a.nlines >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "too many lines");
  a.fq = FastDiv(uint32_t(a.nq));
  const int64_t tiles = (a.nlines + a.W - 1) / a.W;
  const size_t shm = (size_t(a.nl) * (a.W + 1) + size_t(a.m)) * sizeof(T);
  switch (row_q_for(a.m)) {
    case 3: hipLaunchKernelGGL((k_line_pass<T, 3>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    case 5: hipLaunchKernelGGL((k_line_pass<T, 5>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    case 9: hipLaunchKernelGGL((k_line_pass<T, 9>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    case 11: hipLaunchKernelGGL((k_line_pass<T, 11>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    case kRowQ: hipLaunchKernelGGL((k_line_pass<T, kRowQ>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
    default: hipLaunchKernelGGL((k_line_pass<T, 0>), dim3(unsigned(tiles)), dim3(NT), shm, st, a); break;
  }
  BM_HIP(hipGetLastError());
}

// ------------------------------------------------------------- plane pass

// K along x, then along y, for every z-plane of a level grid in one launch.
// A workgroup stages its plane in LDS (dequantized, coarse nodes zeroed on
// request), restricts and solves its rows along x into a second LDS plane
// (in place when the lines hold the restriction already), then restricts
// and solves that plane's columns along y in place, and stores the m1 x m2
// result.  The arithmetic is the line passes' own (same restriction rows,
// same 16-lane solves), so the result equals theirs bit for bit; the plane
// pass only saves the launch and the round trip of the x pass's result.
// It is used where both planes fit a workgroup's LDS and both axes take the
// same row layout Q.
constexpr int kPlaneNT = 1024;
constexpr int kPlaneLds = 152 * 1024;

template <typename T>
struct PlaneArgs {
  const T* in;
  const int32_t* qin;    // optional: codes (same strides), times *qdel
  const double* qdel;
  int64_t is[3];         // input strides
  int n1, n2;            // plane dims (y, x)
  int m1, m2;            // result dims
  FastDiv fn2;           // plane index -> (y, x)
  int mask;              // zero the level's coarse nodes on load
  int cm[3];             // coarsening flags
  int solve_only;        // lines already hold 3 P^T M u: solve only (n = m)
  int sr, sp;            // LDS row strides of the staged plane and of the x result
  const double* inv_x;   // reciprocal pivots along x (m2) and y (m1)
  const double* inv_y;
  T* out;                // dense [planes][m1][m2]
};

// 3 (P^T M v)_J of a line of nl values read by v(i): interior rows
// {1/12, 1/2, 5/6, 1/2, 1/12}, the natural end rows {5/12, 1/2, 1/12}
template <typename T, typename V>
__device__ inline T restrict_row(int J, int nl, int m, V v) {
  const int c = 2 * J;
  T r;
  if (J == 0)
    r = T(5.0 / 12.0) * v(0) + T(0.5) * v(1) + T(1.0 / 12.0) * v(2);
  else if (J == m - 1)
    r = T(1.0 / 12.0) * v(nl - 3) + T(0.5) * v(nl - 2) + T(5.0 / 12.0) * v(nl - 1);
  else
    r = T(1.0 / 12.0) * (v(c - 2) + v(c + 2)) + T(0.5) * (v(c - 1) + v(c + 1)) + T(5.0 / 6.0) * v(c);
  return T(3) * r;
}

template <typename T, int Q>
__global__ __launch_bounds__(kPlaneNT) void k_plane_pass(PlaneArgs<T> a) {
  __shared__ __align__(16) unsigned char smem[kPlaneLds];
  const int n1 = a.n1, n2 = a.n2, m1 = a.m1, m2 = a.m2, sr = a.sr, sp = a.sp;
  T* px = reinterpret_cast<T*>(smem);                 // [m2] pivots along x
  T* py = px + m2;                                    // [m1] pivots along y
  T* R = py + m1;                                     // [n1][sr] the staged plane
  T* P = a.solve_only ? R : R + int64_t(n1) * sr;     // [n1][sp] its rows solved along x
  const int tid = threadIdx.x;
  const int64_t zb = int64_t(blockIdx.x) * a.is[0];
  const bool zc = !(a.cm[0] && (blockIdx.x & 1));     // even z along a coarsening z axis
  const double qd = a.qin ? *a.qdel : 0.0;
  auto stage = [&](const auto* src) {
    using Rt = std::remove_const_t<std::remove_pointer_t<decltype(src)>>;
    const int tot = n1 * n2;
    for (int i0 = tid; i0 < tot; i0 += kU * kPlaneNT) {
      Rt v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = i0 + u * kPlaneNT;
        if (i < tot) {
          const int y = int(a.fn2.div(uint32_t(i))), x = i - y * n2;
          v[u] = src[zb + int64_t(y) * a.is[1] + int64_t(x) * a.is[2]];
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = i0 + u * kPlaneNT;
        if (i < tot) {
          const int y = int(a.fn2.div(uint32_t(i))), x = i - y * n2;
          const bool coarse = a.mask && zc && !(a.cm[1] && (y & 1)) && !(a.cm[2] && (x & 1));
          T w;
          if constexpr (std::is_same_v<Rt, int32_t>)
            w = T(mul_rn(double(v[u]), qd));
          else
            w = v[u];
          R[y * sr + x] = coarse ? T(0) : w;
        }
      }
    }
  };
  for (int k = tid; k < m2; k += kPlaneNT) px[k] = T(a.inv_x[k]);
  for (int k = tid; k < m1; k += kPlaneNT) py[k] = T(a.inv_y[k]);
  if (a.qin)
    stage(a.qin);
  else
    stage(a.in);
  __syncthreads();
  // rows along x: R -> P (in place when solving only)
  solve_lines<T, kPlaneNT, Q>(
      m2, px, n1, tid,
      [&](int w, int J) {
        const T* row = R + w * sr;
        if (a.solve_only) return row[J];
        return restrict_row<T>(J, n2, m2, [&](int i) { return row[i]; });
      },
      [&](int w, int J, T v) { P[w * sp + J] = v; });
  __syncthreads();
  // columns along y, in place in P (a column is read whole before it is written)
  solve_lines<T, kPlaneNT, Q>(
      m1, py, m2, tid,
      [&](int w, int J) {
        const T* col = P + w;
        if (a.solve_only) return col[J * sp];
        return restrict_row<T>(J, n1, m1, [&](int i) { return col[i * sp]; });
      },
      [&](int w, int J, T v) { P[J * sp + w] = v; });
  __syncthreads();
  T* dst = a.out + int64_t(blockIdx.x) * m1 * m2;
  for (int i = tid; i < m1 * m2; i += kPlaneNT) {
    const int J1 = i / m2, J2 = i - J1 * m2;
    dst[i] = P[J1 * sp + J2];
  }
}

// K_y K_x of every z-plane of `in` into the dense array out (dims n0, m1,
// m2) with one plane pass; false (nothing launched) where the planes do not
// fit a workgroup's LDS or the two axes take different row layouts.
template <typename T>
bool launch_plane(const bm_plan_s& p, int s, const View3& in, bool mask, void* out, const int32_t* qin,
                  const double* qdel, hipStream_t st, bool solve_only = false) {
  const Level& L = p.lv[s - 1];
  if (!p.plane_pass || !L.coarsen[1] || !L.coarsen[2]) return false;
  const int64_t n1 = in.n[1], n2 = in.n[2], m1 = L.m[1], m2 = L.m[2];
  if (solve_only ? (n1 != m1 || n2 != m2) : (m1 != (n1 + 1) / 2 || m2 != (n2 + 1) / 2 || n1 < 3 || n2 < 3))
    return false;
  const int q = row_q_for(m2);
  if (q != row_q_for(m1) || (q != 3 && q != 5 && q != 9 && q != 11)) return false;
  const int64_t sr = n2 | 1, sp = solve_only ? sr : (m2 | 1);
  const int64_t elems = m1 + m2 + n1 * sr + (solve_only ? 0 : n1 * sp);
  if (elems * int64_t(sizeof(T)) > kPlaneLds) return false;
  if (in.n[0] >= (int64_t(1) << 31)) return false;
  PlaneArgs<T> a{};
  a.in = static_cast<const T*>(in.ptr);
  a.qin = qin;
  a.qdel = qdel;
  for (int k = 0; k < 3; ++k) {
    a.is[k] = in.s[k];
    a.cm[k] = L.coarsen[k] ? 1 : 0;
  }
  a.n1 = int(n1);
  a.n2 = int(n2);
  a.m1 = int(m1);
  a.m2 = int(m2);
  a.fn2 = FastDiv(uint32_t(n2));
  a.mask = mask ? 1 : 0;
  a.solve_only = solve_only ? 1 : 0;
  a.sr = int(sr);
  a.sp = int(sp);
  a.inv_x = L.d_inv[2];
  a.inv_y = L.d_inv[1];
  a.out = static_cast<T*>(out);
  const dim3 g{unsigned(in.n[0])}, b{unsigned(kPlaneNT)};
  switch (q) {
    case 3: hipLaunchKernelGGL((k_plane_pass<T, 3>), g, b, 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_plane_pass<T, 5>), g, b, 0, st, a); break;
    case 9: hipLaunchKernelGGL((k_plane_pass<T, 9>), g, b, 0, st, a); break;
    default: hipLaunchKernelGGL((k_plane_pass<T, 11>), g, b, 0, st, a); break;
  }
  BM_HIP(hipGetLastError());
  return true;
}

// The first global level's load vector when the last block level is fused
// with it: every block left partial sums, over its own coarse nodes, at the
// H^3 coarse nodes of the next level inside it; node c along an axis lies in
// block c / (H-1), and a node on a shared face also in the block before.
// The partials are added in a fixed order (lower blocks first).
template <typename T>
struct GatherArgs {
  const double* part;     // [block][H][H][H]
  uint32_t nb[3];
  Idx3 m;                 // dims of the level's coarse grid
  T* out;                 // dense, dims m
};

template <typename T, int H>
__global__ __launch_bounds__(NT) void k_gather_part(GatherArgs<T> a) {
  const uint32_t tot = uint32_t(a.m.n0 * a.m.n1 * a.m.n2);
  for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < tot; i += gridDim.x * NT) {
    uint32_t c[3];
    a.m.uf(i, c[0], c[1], c[2]);
    uint32_t b0[3], b1[3];
    int k0[3], k1[3];
    bool two[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const uint32_t bb = c[d] / (H - 1);
      const int kk = int(c[d] - bb * (H - 1));
      two[d] = kk == 0 && bb > 0 && bb < a.nb[d];   // a shared face: the block before, then this one
      b1[d] = bb;
      k1[d] = 0;
      if (bb == a.nb[d] || two[d]) {                // (or the far end node)
        b0[d] = bb - 1;
        k0[d] = H - 1;
      } else {
        b0[d] = bb;
        k0[d] = kk;
      }
    }
    // all (up to 8) partials are fetched before the sum; an absent one adds
    // +0, which leaves the sum unchanged (it starts at +0)
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int iz = t >> 2, iy = (t >> 1) & 1, ix = t & 1;
      v[t] = 0.0;
      if ((iz && !two[0]) || (iy && !two[1]) || (ix && !two[2])) continue;
      const uint64_t blk = (uint64_t(iz ? b1[0] : b0[0]) * a.nb[1] + (iy ? b1[1] : b0[1])) * a.nb[2] +
                           (ix ? b1[2] : b0[2]);
      v[t] = a.part[blk * (H * H * H) + ((iz ? k1[0] : k0[0]) * H + (iy ? k1[1] : k0[1])) * H + (ix ? k1[2] : k0[2])];
    }
    double sum = 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t) sum += v[t];
    a.out[i] = T(sum);
  }
}

// ------------------------------------------------------------- launchers

template <typename T>
void launch_details(const bm_plan_s& p, int s, const void* u, void* coeff, int32_t* codes, const double* qinv,
                    int64_t* flag, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  const View3 cv = level_view(p, s, codes ? static_cast<void*>(codes) : coeff);
  DetArgs<T> a{static_cast<const T*>(u), {L.n[0], L.n[1], L.n[2]}, {L.m[0], L.m[1], L.m[2]}, L.coarsen[0],
               L.coarsen[1], L.coarsen[2], static_cast<T*>(coeff), {cv.s[0], cv.s[1], cv.s[2]}, codes, qinv, flag};
  hipLaunchKernelGGL(k_details<T>, dim3(grid_for(L.m[0] * L.m[1] * L.m[2])), dim3(NT), 0, st, a);
  BM_HIP(hipGetLastError());
}

template <typename T>
void launch_interp(const bm_plan_s& p, int s, const void* coeff, const int32_t* codes, const double* qdel,
                   const void* uc, void* out, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  const View3 cv = level_view(p, s, codes ? const_cast<int32_t*>(codes) : const_cast<void*>(coeff));
  IntArgs<T> a{static_cast<const T*>(coeff), {cv.s[0], cv.s[1], cv.s[2]}, static_cast<const T*>(uc),
               {L.m[0], L.m[1], L.m[2]}, {L.n[0], L.n[1], L.n[2]}, L.coarsen[0], L.coarsen[1], L.coarsen[2],
               static_cast<T*>(out), codes, qdel};
  hipLaunchKernelGGL(k_interp_add<T>, dim3(grid_for(L.m[0] * L.m[1] * L.m[2])), dim3(NT), 0, st, a);
  BM_HIP(hipGetLastError());
}

// quantize (to_codes) or dequantize a strided view; *scale is 1/Delta or Delta
template <typename T>
__global__ __launch_bounds__(NT) void k_qcopy(const T* src, int64_t ss0, int64_t ss1, int64_t ss2, const int32_t* csrc,
                                              T* dst, int32_t* cdst, int64_t ds0, int64_t ds1, int64_t ds2, Idx3 n,
                                              const double* scale, int64_t* flag) {
  const int64_t tot = n.n0 * n.n1 * n.n2;
  const double sc = *scale;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < tot; i += int64_t(gridDim.x) * NT) {
    int64_t z, y, x;
    unflat(i, n, z, y, x);
    const int64_t so = z * ss0 + y * ss1 + x * ss2, dO = z * ds0 + y * ds1 + x * ds2;
    if (cdst)
      cdst[dO] = quant_g(src[so], sc, flag);
    else
      dst[dO] = T(mul_rn(double(csrc[so]), sc));
  }
}

}  // namespace

void global_details(const bm_plan_s& p, int s, const void* u, void* coeff, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    launch_details<float>(p, s, u, coeff, nullptr, nullptr, nullptr, st);
  else
    launch_details<double>(p, s, u, coeff, nullptr, nullptr, nullptr, st);
}

void global_interp_add(const bm_plan_s& p, int s, const void* coeff, const void* uc, void* out, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    launch_interp<float>(p, s, coeff, nullptr, nullptr, uc, out, st);
  else
    launch_interp<double>(p, s, coeff, nullptr, nullptr, uc, out, st);
}

void line_pass(const bm_plan_s& p, int s, int axis, const View3& in, const int64_t cmask[3], void* out,
               const void* base, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    launch_pass<float>(p, s, axis, in, cmask, out, base, nullptr, nullptr, st);
  else
    launch_pass<double>(p, s, axis, in, cmask, out, base, nullptr, nullptr, st);
}

namespace {

void line_pass_q(const bm_plan_s& p, int s, int axis, const View3& in, const int64_t cmask[3], void* out,
                 const void* base, const int32_t* qin, const double* qdel, hipStream_t st,
                 const CoarseIO* cio = nullptr) {
  if (p.cfg.dtype == BM_F32)
    launch_pass<float>(p, s, axis, in, cmask, out, base, qin, qdel, st, false, nullptr, cio);
  else
    launch_pass<double>(p, s, axis, in, cmask, out, base, qin, qdel, st, false, nullptr, cio);
}

void qcopy(const bm_plan_s& p, const View3& src, const int32_t* csrc, const View3& dst, int32_t* cdst,
           const double* scale, int64_t* flag, hipStream_t st) {
  const int64_t tot = src.n[0] * src.n[1] * src.n[2];
  const Idx3 n{src.n[0], src.n[1], src.n[2]};
  if (p.cfg.dtype == BM_F32)
    hipLaunchKernelGGL(k_qcopy<float>, dim3(grid_for(tot)), dim3(NT), 0, st, static_cast<const float*>(src.ptr),
                       src.s[0], src.s[1], src.s[2], csrc, static_cast<float*>(dst.ptr), cdst, dst.s[0], dst.s[1],
                       dst.s[2], n, scale, flag);
  else
    hipLaunchKernelGGL(k_qcopy<double>, dim3(grid_for(tot)), dim3(NT), 0, st, static_cast<const double*>(src.ptr),
                       src.s[0], src.s[1], src.s[2], csrc, static_cast<double*>(dst.ptr), cdst, dst.s[0], dst.s[1],
                       dst.s[2], n, scale, flag);
  BM_HIP(hipGetLastError());
}

}  // namespace

void strided_copy(size_t esize, const View3& src, const View3& dst, hipStream_t st) {
  const int64_t tot = src.n[0] * src.n[1] * src.n[2];
  if (esize == 4) {
    CopyArgs<float> a{static_cast<const float*>(src.ptr), {src.s[0], src.s[1], src.s[2]},
                      static_cast<float*>(dst.ptr), {dst.s[0], dst.s[1], dst.s[2]}, {src.n[0], src.n[1], src.n[2]}};
    hipLaunchKernelGGL(k_copy<float>, dim3(grid_for(tot)), dim3(NT), 0, st, a);
  } else {
    CopyArgs<double> a{static_cast<const double*>(src.ptr), {src.s[0], src.s[1], src.s[2]},
                       static_cast<double*>(dst.ptr), {dst.s[0], dst.s[1], dst.s[2]}, {src.n[0], src.n[1], src.n[2]}};
    hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(tot)), dim3(NT), 0, st, a);
  }
  BM_HIP(hipGetLastError());
}

template <typename T>
void launch_pad_extend(const bm_plan_s& p, void* g, bool zero, hipStream_t st) {
  const int64_t* d = p.dims;
  const int64_t* n = p.pdims;
  // an axis that is not extended leaves its slab empty (no divisor of 0 on the host)
  auto slab = [](int64_t a, int64_t b, int64_t c) { return a > 0 && b > 0 && c > 0 ? Idx3(a, b, c) : Idx3(0, 1, 1); };
  PadExtArgs<T> a{static_cast<T*>(g), {d[0], d[1], d[2]}, {n[0], n[1], n[2]}, slab(n[0] - d[0], n[1], n[2]),
                  slab(d[0], n[1] - d[1], n[2]), slab(d[0], d[1], n[2] - d[2]), zero ? 1 : 0};
  const int64_t tot = n[0] * n[1] * n[2] - d[0] * d[1] * d[2];
  if (tot == 0) return;
  hipLaunchKernelGGL(k_pad_extend<T>, dim3(grid_for(tot)), dim3(NT), 0, st, a);
  BM_HIP(hipGetLastError());
}

// The level-1 grid of a plan without block levels: the input padded into
// the plan's grid, or, when the input is that grid already (its logical
// region at the padded strides, as a caller inside the library leaves it),
// only its extension filled in place.
static void level1_input(const bm_plan_s& p, const void* x, hipStream_t st) {
  const bool zero = p.cfg.pad_mode == 1;
  if (x != p.ws.grid[0]) {
    pad_input(p, x, p.ws.grid[0], zero, st);
  } else if (p.cfg.dtype == BM_F32) {
    launch_pad_extend<float>(p, p.ws.grid[0], zero, st);
  } else {
    launch_pad_extend<double>(p, p.ws.grid[0], zero, st);
  }
}

void* level1_grid(const bm_plan_s& p) { return p.cfg.L == 0 ? p.ws.grid[0] : nullptr; }

void pad_input(const bm_plan_s& p, const void* x, void* dst, bool zero, hipStream_t st) {
  const int64_t tot = p.pdims[0] * p.pdims[1] * p.pdims[2];
  if (p.cfg.dtype == BM_F32) {
    PadArgs<float> a{static_cast<const float*>(x), {p.dims[0], p.dims[1], p.dims[2]}, static_cast<float*>(dst),
                     {p.pdims[0], p.pdims[1], p.pdims[2]}, zero};
    hipLaunchKernelGGL(k_pad<float>, dim3(grid_for(tot)), dim3(NT), 0, st, a);
  } else {
    PadArgs<double> a{static_cast<const double*>(x), {p.dims[0], p.dims[1], p.dims[2]}, static_cast<double*>(dst),
                      {p.pdims[0], p.pdims[1], p.pdims[2]}, zero};
    hipLaunchKernelGGL(k_pad<double>, dim3(grid_for(tot)), dim3(NT), 0, st, a);
  }
  BM_HIP(hipGetLastError());
}

// ------------------------------------------------------------- drivers

static bool plane_pass(const bm_plan_s& p, int s, const View3& in, bool mask, void* out, const int32_t* qin,
                       const double* qdel, hipStream_t st) {
  if (p.cfg.dtype == BM_F32) return launch_plane<float>(p, s, in, mask, out, qin, qdel, st);
  return launch_plane<double>(p, s, in, mask, out, qin, qdel, st);
}

// coarse = K_z K_y K_x (in), applied as line passes over the axes that
// coarsen; intermediate results go through the plan's temporaries.
static void apply_K3(bm_plan_s& p, int s, View3 in, bool mask, void* out, const void* base, hipStream_t st,
                     const int32_t* qin = nullptr, const double* qdel = nullptr, const CoarseIO* cio = nullptr) {
  const Level& L = p.lv[s - 1];
  // x and y in one plane pass where the planes fit, then z
  if (L.coarsen[0] && plane_pass(p, s, in, mask, p.ws.t1, qin, qdel, st)) {
    const int64_t on[3] = {in.n[0], L.m[1], L.m[2]};
    line_pass_q(p, s, 0, dense_view(p.ws.t1, on), nullptr, out, base, nullptr, qdel, st, cio);
    return;
  }
  int axes[3], na = 0;
  for (int a : {2, 1, 0})
    if (L.coarsen[a]) axes[na++] = a;
  const int64_t cm[3] = {1, 1, 1};
  void* tmp[2] = {p.ws.t1, p.ws.t2};
  View3 cur = in;
  for (int k = 0; k < na; ++k) {
    const int ax = axes[k];
    const bool last = k == na - 1;
    void* dst = last ? out : tmp[k & 1];
    line_pass_q(p, s, ax, cur, (k == 0 && mask) ? cm : nullptr, dst, last ? base : nullptr, k == 0 ? qin : nullptr,
                qdel, st, last ? cio : nullptr);
    int64_t on[3] = {cur.n[0], cur.n[1], cur.n[2]};
    on[ax] = L.m[ax];
    cur = dense_view(dst, on);
  }
}

// Coarse values of the first global level (s = L+1) when the last block level
// is fused with it: the gathered load vector 27 (P^T M)^3 u, then the three
// tridiagonal solves along x, y and z.  Gather and solves run in FP64 (the
// values are rounded once, to the plan's type, at the end): a level-wide
// restriction followed by three solves would otherwise round more often
// than the interleaved restriction + solve passes it replaces.
static void global_from_parts(bm_plan_s& p, int s, hipStream_t st) {
  const Level& L = p.lv[s - 1];
  const Level& B = p.lv[s - 2];
  const int64_t* m = L.m;
  const int64_t tot = m[0] * m[1] * m[2];
  if (size_t(tot) * sizeof(double) > p.ws.t_elems * p.esize) fail(BM_EINVAL, "plan workspace too small");
  double* t1 = static_cast<double*>(p.ws.t1);
  double* t2 = static_cast<double*>(p.ws.t2);
  GatherArgs<double> a{static_cast<const double*>(p.ws.part),
                       {uint32_t(B.nb[0]), uint32_t(B.nb[1]), uint32_t(B.nb[2])}, {m[0], m[1], m[2]}, t1};
  if (B.b == 9)
    hipLaunchKernelGGL((k_gather_part<double, 3>), dim3(grid_for(tot)), dim3(NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_gather_part<double, 5>), dim3(grid_for(tot)), dim3(NT), 0, st, a);
  BM_HIP(hipGetLastError());
  // x and y: t1 -> t2 (one plane pass where the planes fit), z: t2 -> the
  // coarse grid (narrowed to FP32 on the store for an FP32 plan)
  const bool f64 = p.cfg.dtype == BM_F64;
  if (!launch_plane<double>(p, s, dense_view(t1, m), false, t2, nullptr, nullptr, st, true)) {
    launch_pass<double>(p, s, 2, dense_view(t1, m), nullptr, t2, nullptr, nullptr, nullptr, st, true);
    launch_pass<double>(p, s, 1, dense_view(t2, m), nullptr, t1, nullptr, nullptr, nullptr, st, true);
    std::swap(t1, t2);
  }
  launch_pass<double>(p, s, 0, dense_view(t2, m), nullptr, f64 ? p.ws.grid[s] : t1, nullptr, nullptr, nullptr, st,
                      true, f64 ? nullptr : static_cast<float*>(p.ws.grid[s]));
}

void decompose(bm_plan_s& p, const void* x, void* coeff, hipStream_t st) {
  const View3 xv = dense_view(const_cast<void*>(x), p.dims);
  for (int s = 1; s <= p.nlev; ++s) {
    const Level& L = p.lv[s - 1];
    TimedScope ts(p, 2 * (s - 1), st);
    if (L.local) {
      const View3 src = s == 1 ? xv : dense_view(p.ws.grid[s - 1], L.n);
      if (nest_pair(p, s)) {
        local_decompose_nest(p, s, src, s == 1, coeff, nullptr, nullptr, st);
        ++s;   // block level s+1 ran in the same launch
        continue;
      }
      local_decompose(p, s, src, s == 1, coeff, p.ws.grid[s], st);
    } else {
      const void* u;
      if (s == 1) {
        level1_input(p, x, st);
        u = p.ws.grid[0];
      } else {
        u = p.ws.grid[s - 1];
      }
      // (the first global level's details and load vector come from the
      // last block level when fused)
      if (p.fuse_next && s == p.L + 1) {
        global_from_parts(p, s, st);
        continue;
      }
      global_details(p, s, u, coeff, st);
      apply_K3(p, s, dense_view(const_cast<void*>(u), L.n), false, p.ws.grid[s], nullptr, st);
    }
  }
  const Level& last = p.lv[p.nlev - 1];
  strided_copy(p.esize, dense_view(p.ws.grid[p.nlev], last.m), coarsest_view(p, coeff), st);
}

void recompose(bm_plan_s& p, const void* coeff, void* x, hipStream_t st) {
  const Level& last = p.lv[p.nlev - 1];
  strided_copy(p.esize, coarsest_view(p, const_cast<void*>(coeff)), dense_view(p.ws.grid[p.nlev], last.m), st);
  for (int s = p.nlev; s >= 1; --s) {
    const Level& L = p.lv[s - 1];
    TimedScope ts(p, 2 * (s - 1) + 1, st);
    if (L.local) {
      if (s > 1 && nest_pair(p, s - 1)) {
        // block levels s and s-1 in one launch
        void* out = s == 2 ? x : p.ws.grid[s - 2];
        local_recompose_nest(p, s - 1, coeff, p.ws.grid[s], out, s == 2, nullptr, nullptr, st);
        --s;
        continue;
      }
      void* out = s == 1 ? x : p.ws.grid[s - 1];
      local_recompose(p, s, coeff, p.ws.grid[s], out, s == 1, st);
    } else {
      // u_C = c - K3 w in place in grid[s], then u = interpolant + w (which
      // the last block level does itself when fused)
      apply_K3(p, s, level_view(p, s, const_cast<void*>(coeff)), true, p.ws.grid[s], p.ws.grid[s], st);
      if (p.fuse_next && s == p.L + 1) continue;
      void* out = p.ws.grid[s - 1];
      global_interp_add(p, s, coeff, p.ws.grid[s], out, st);
      if (s == 1 && x != out) {   // (a caller that passed the plan's grid reads it in place)
        View3 src = dense_view(out, p.pdims);
        src.n[0] = p.dims[0];
        src.n[1] = p.dims[1];
        src.n[2] = p.dims[2];
        strided_copy(p.esize, src, dense_view(x, p.dims), st);
      }
    }
  }
}

// Fused pipeline (the paper's BMF form, Sec. IV-D): the block levels write
// quantization codes directly, global levels quantize their details as the
// detail stencil produces them, and the coarsest values last.  The codes are
// identical to bm_decompose followed by bm_quantize_roi.
void decompose_quantize_global(bm_plan_s& p, const void* x, int32_t* codes, const QPrep& q, hipStream_t st) {
  bool coarsest_done = false;
  for (int s = p.L + 1; s <= p.nlev; ++s) {
    const Level& L = p.lv[s - 1];
    TimedScope ts(p, 2 * (s - 1), st);
    const void* u;
    if (s == 1) {
      level1_input(p, x, st);
      u = p.ws.grid[0];
    } else {
      u = p.ws.grid[s - 1];
    }
    if (p.fuse_next && s == p.L + 1) {
      // details (codes) and load vector from the last block level
      global_from_parts(p, s, st);
      continue;
    }
    if (p.cfg.dtype == BM_F32)
      launch_details<float>(p, s, u, nullptr, codes, q.q + 2 * (s - 1) + 1, q.flag, st);
    else
      launch_details<double>(p, s, u, nullptr, codes, q.q + 2 * (s - 1) + 1, q.flag, st);
    // the last level's last pass quantizes the coarsest values into the codes
    CoarseIO cio;
    if (s == p.nlev) {
      const View3 cv = coarsest_view(p, codes);
      cio.cout = codes;
      for (int k = 0; k < 3; ++k) cio.s[k] = cv.s[k];
      cio.q = q.q + 2 * p.nlev + 1;
      cio.flag = q.flag;
      coarsest_done = true;
    }
    apply_K3(p, s, dense_view(const_cast<void*>(u), L.n), false, p.ws.grid[s], nullptr, st, nullptr, nullptr,
             s == p.nlev ? &cio : nullptr);
  }
  if ((p.M > 0 || p.L == 0) && !coarsest_done) {
    const Level& last = p.lv[p.nlev - 1];
    const View3 cv = coarsest_view(p, codes);
    qcopy(p, dense_view(p.ws.grid[p.nlev], last.m), nullptr, cv, codes, q.q + 2 * p.nlev + 1, q.flag, st);
  }
}

void decompose_quantize(bm_plan_s& p, const void* x, const double* block_tol, int32_t* codes, bm_qstats* stats,
                        hipStream_t st) {
  const QPrep q = quant_prepare(p, block_tol, st);   // also clears the overflow flag
  const View3 xv = dense_view(const_cast<void*>(x), p.dims);
  for (int s = 1; s <= p.L; ++s) {
    const Level& L = p.lv[s - 1];
    TimedScope ts(p, 2 * (s - 1), st);
    const View3 src = s == 1 ? xv : dense_view(p.ws.grid[s - 1], L.n);
    if (nest_pair(p, s)) {
      local_decompose_nest(p, s, src, s == 1, nullptr, codes, &q, st);
      ++s;   // block level s+1 ran in the same launch
      continue;
    }
    local_decompose_q(p, s, src, s == 1, codes, p.ws.grid[s], q, st);
  }
  decompose_quantize_global(p, x, codes, q, st);
  if (stats) {
    int64_t f = 0;
    BM_HIP(hipMemcpyAsync(&f, q.flag, sizeof(f), hipMemcpyDeviceToHost, st));
    BM_HIP(hipStreamSynchronize(st));
    stats->n_codes = p.pdims[0] * p.pdims[1] * p.pdims[2];
    stats->n_outliers = -1;
    stats->max_abs_code = -1;
    check_code_flag(f, "tolerance too small for the data");
  }
}

void dequantize_recompose_global(bm_plan_s& p, const int32_t* codes, const QPrep& q, void* x, hipStream_t st) {
  // (the coarsest values, a global level's, are dequantized by the last pass
  // of that level, where they are the base of u_C = c - K3 w)
  for (int s = p.nlev; s > p.L; --s) {
    const Level& L = p.lv[s - 1];
    TimedScope ts(p, 2 * (s - 1) + 1, st);
    const double* qdel = q.q + 2 * (s - 1);
    const View3 lvw = level_view(p, s, const_cast<int32_t*>(codes));
    if (s == p.nlev) {
      CoarseIO cio;
      const View3 cv = coarsest_view(p, const_cast<int32_t*>(codes));
      cio.cbase = codes;
      for (int k = 0; k < 3; ++k) cio.s[k] = cv.s[k];
      cio.q = q.q + 2 * p.nlev;
      apply_K3(p, s, lvw, true, p.ws.grid[s], nullptr, st, codes, qdel, &cio);
    } else {
      apply_K3(p, s, lvw, true, p.ws.grid[s], p.ws.grid[s], st, codes, qdel);
    }
    if (p.fuse_next && s == p.L + 1) continue;   // the last block level interpolates
    void* out = p.ws.grid[s - 1];
    if (p.cfg.dtype == BM_F32)
      launch_interp<float>(p, s, nullptr, codes, qdel, p.ws.grid[s], out, st);
    else
      launch_interp<double>(p, s, nullptr, codes, qdel, p.ws.grid[s], out, st);
    if (s == 1 && x != out) {   // (a caller that passed the plan's grid reads it in place)
      View3 src = dense_view(out, p.pdims);
      src.n[0] = p.dims[0];
      src.n[1] = p.dims[1];
      src.n[2] = p.dims[2];
      strided_copy(p.esize, src, dense_view(x, p.dims), st);
    }
  }
}

// Inverse of decompose_quantize: dequantize on load, then recompose.  Equal
// to bm_dequantize followed by bm_recompose.
void dequantize_recompose(bm_plan_s& p, const int32_t* codes, const double* block_tol, void* x, hipStream_t st) {
  const QPrep q = quant_prepare(p, block_tol, st, false);
  dequantize_recompose_global(p, codes, q, x, st);
  for (int s = p.L; s >= 1; --s) {
    TimedScope ts(p, 2 * (s - 1) + 1, st);
    if (s > 1 && nest_pair(p, s - 1)) {
      // block levels s and s-1 in one launch
      void* out = s == 2 ? x : p.ws.grid[s - 2];
      local_recompose_nest(p, s - 1, nullptr, p.ws.grid[s], out, s == 2, codes, &q, st);
      --s;
      continue;
    }
    void* out = s == 1 ? x : p.ws.grid[s - 1];
    local_recompose_q(p, s, codes, p.ws.grid[s], out, s == 1, q, st);
  }
}

}  // namespace bm
