// ROI tolerance maps and the reciprocal quantizer (Sec. IV-C, IV-D).
//
// Block-wise tolerance assignment: a level-1 block takes the minimum voxel
// tolerance over its closed node range (a partly covered block is strict;
// padded nodes count as the node they copy).  Conservative propagation
// (Eq. 2): a block of local level s+1 takes the minimum over the level-s
// blocks that share a node with it.  Global levels use tau_global, the
// minimum over the last local level.
//
// Budget (the L-infinity bound of Sec. II-B): level s gets the share w_s of
// every tolerance (proportional to its coefficient count, equal among the
// global levels, floored at 1/(64 T) and renormalised; see level_weights);
// a detail of level s on a node with tolerance tau gets bin width
// Delta = tau * kappa_s, kappa_s = 2 (1 - eta) w_s / A_s, where A_s is the
// level's L-infinity gain; the coarsest values get kappa = 2 (1 - eta) w_c.
// q = rint(c * (1/Delta)) in FP64 (the per-block reciprocal quantizer of
// Sec. IV-D), c_hat = q * Delta.  A node inside several blocks of its level
// uses the smallest Delta (largest reciprocal) of those blocks; because
// rounding is monotone this equals computing Delta from the smallest tau.

#include <algorithm>
#include <cmath>

#include <cstring>

#include "internal.h"

namespace bm {
namespace {

constexpr int NT = 256;

inline unsigned grid_for(int64_t tot) {
  int64_t g = (tot + NT - 1) / NT;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return unsigned(g);
}

// tolerances are positive doubles: their bit patterns order like the values
__device__ inline void atomic_min_pos(double* p, double v) {
  atomicMin(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(__double_as_longlong(v)));
}

__global__ void k_fill_u64(unsigned long long* p) {
  if (threadIdx.x == 0) *p = 0;
}

__global__ void k_fill(double* p, int64_t n, double v) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) p[i] = v;
}

struct BoxArgs {
  const double* boxes;   // nbox x 7
  int nbox;
  double background;
  int64_t n[3];          // logical dims
  int64_t nb[3];
  int64_t w;             // block width in nodes (b-1); 0 when L == 0 (one block)
  double* out;
};

__global__ void k_tol_boxes(BoxArgs a) {
  const int64_t nbt = a.nb[0] * a.nb[1] * a.nb[2];
  for (int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x; k < nbt; k += int64_t(gridDim.x) * NT) {
    const int64_t bx = k % a.nb[2], t = k / a.nb[2], by = t % a.nb[1], bz = t / a.nb[1];
    const int64_t bi[3] = {bz, by, bx};
    int64_t lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      if (a.w == 0) {
        lo[d] = 0;
        hi[d] = a.n[d] - 1;
      } else {
        lo[d] = i64min(bi[d] * a.w, a.n[d] - 1);
        hi[d] = i64min((bi[d] + 1) * a.w, a.n[d] - 1);
      }
    }
    double v = a.background;
    for (int j = 0; j < a.nbox; ++j) {
      const double* r = a.boxes + 7 * j;
      bool hit = true;
      for (int d = 0; d < 3; ++d) {
        const int64_t b0 = int64_t(r[d]), b1 = int64_t(r[d + 3]);
        hit = hit && b0 < b1 && b0 <= hi[d] && b1 > lo[d];
      }
      if (hit && r[6] < v) v = r[6];
    }
    a.out[k] = v;
  }
}

struct VoxArgs {
  const double* vt;
  int64_t n[3];
  int64_t nb[3];
  int64_t w;
  double* out;
};

// one workgroup per block: min over the block's closed node range
__global__ __launch_bounds__(NT) void k_tol_voxels(VoxArgs a) {
  __shared__ double red[NT];
  const int64_t k = blockIdx.x;
  const int64_t bx = k % a.nb[2], t = k / a.nb[2], by = t % a.nb[1], bz = t / a.nb[1];
  const int64_t bi[3] = {bz, by, bx};
  int64_t lo[3], ext[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = i64min(bi[d] * a.w, a.n[d] - 1);
    ext[d] = i64min((bi[d] + 1) * a.w, a.n[d] - 1) - lo[d] + 1;
  }
  double v = INFINITY;
  const int64_t cnt = ext[0] * ext[1] * ext[2];
  for (int64_t i = threadIdx.x; i < cnt; i += NT) {
    const int64_t x = i % ext[2], r = i / ext[2], y = r % ext[1], z = r / ext[1];
    const double tv = a.vt[((lo[0] + z) * a.n[1] + lo[1] + y) * a.n[2] + lo[2] + x];
    v = tv < v ? tv : v;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.out[k] = red[0];
}

// min over everything (L == 0): grid-stride + atomic min into out[0] (pre-filled with +inf)
__global__ __launch_bounds__(NT) void k_min_all(const double* v, int64_t n, double* out) {
  __shared__ double red[NT];
  double m = INFINITY;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) m = fmin(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomic_min_pos(out, red[0]);
}



struct QArgs {
  uint32_t tot;               // padded node count (< 2^32)
  Unflat32 uf;                // flat index -> (z, y, x) of the padded grid
  int L, M;
  int D[3];                   // levels each axis coarsens
  int lw;                     // log2(b - 1), b of the first block level
  int nested;                 // nested block schedule: every level's blocks span b - 1 padded cells
  // per-block Delta and 1/Delta: slot s-1 for the details of local level s;
  // slot kCoarseSlot for the coarsest values when M == 0 (level-L blocks)
  const double* bdelta[9];
  const double* binv[9];
  uint32_t nb[9][3];
  const double* q;            // scalar Delta / inverse per level (index s-1), coarsest at L+M
  int64_t* counters;          // [0] outliers, [1] max |q|, [2] out of range
  const double* pdel;         // optional per-node Delta (padded grid); 1/Delta is its IEEE reciprocal
};

__device__ inline int ctz32(uint32_t v) { return v == 0 ? 32 : __builtin_ctz(v); }

// level of a node: 1..L+M for a detail of that level, L+M+1 for a coarsest value
__device__ inline int node_level(const QArgs& a, uint32_t g0, uint32_t g1, uint32_t g2) {
  int lev = a.L + a.M + 1;
  const uint32_t g[3] = {g0, g1, g2};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t = ctz32(g[d]);
    if (t < a.D[d] && t + 1 < lev) lev = t + 1;
  }
  return lev;
}

constexpr int kCoarseSlot = 8;

// Delta and 1/Delta of a node whose tolerance comes from the blocks of local
// level s (grid coordinates q = g >> (s-1)), from table slot `slot`.  Block i
// spans nodes [i w, (i+1) w]: a node on a shared face lies in two blocks per
// axis.  In the nested schedule the blocks of every level span the same
// padded-grid regions, so the padded coordinates g index them directly.
__device__ inline void block_delta(const QArgs& a, int s, int slot, uint32_t g0, uint32_t g1, uint32_t g2,
                                   double& del, double& inv) {
  const int sh = a.nested ? 0 : s - 1;
  const uint32_t q[3] = {g0 >> sh, g1 >> sh, g2 >> sh};
  const uint32_t wm = (1u << a.lw) - 1;
  uint32_t lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const uint32_t nb = a.nb[slot][d];
    const uint32_t f = q[d] >> a.lw;
    lo[d] = ((q[d] & wm) == 0 && q[d] > 0) ? f - 1 : f;
    hi[d] = f < nb - 1 ? f : nb - 1;
    if (lo[d] > hi[d]) lo[d] = hi[d];
  }
  const double* bd = a.bdelta[slot];
  const double* bi = a.binv[slot];
  const uint32_t n1 = a.nb[slot][1], n2 = a.nb[slot][2];
  uint32_t k = (lo[0] * n1 + lo[1]) * n2 + lo[2];
  del = bd[k];
  inv = bi[k];
  if (lo[0] != hi[0] || lo[1] != hi[1] || lo[2] != hi[2]) {
    for (uint32_t z = lo[0]; z <= hi[0]; ++z)
      for (uint32_t y = lo[1]; y <= hi[1]; ++y)
        for (uint32_t x = lo[2]; x <= hi[2]; ++x) {
          k = (z * n1 + y) * n2 + x;
          del = fmin(del, bd[k]);
          inv = fmax(inv, bi[k]);
        }
  }
}

__device__ inline void node_delta(const QArgs& a, uint32_t z, uint32_t y, uint32_t x, double& del, double& inv) {
  const int lev = node_level(a, z, y, x);
  if (lev <= a.L) {
    block_delta(a, lev, lev - 1, z, y, x, del, inv);
  } else if (lev == a.L + a.M + 1 && a.M == 0) {
    block_delta(a, a.L, kCoarseSlot, z, y, x, del, inv);
  } else {
    del = a.q[2 * (lev - 1)];
    inv = a.q[2 * (lev - 1) + 1];
  }
}

// Each thread handles QU nodes of a tile of NT*QU consecutive nodes per
// iteration, so the independent loads of those nodes overlap.
constexpr int QU = 4;
constexpr int kMaxQGroups = 8192;

inline unsigned qgroups(uint32_t tot) {
  const int64_t tiles = (int64_t(tot) + NT * QU - 1) / (NT * QU);
  return unsigned(tiles < kMaxQGroups ? (tiles > 0 ? tiles : 1) : kMaxQGroups);
}

// Per-workgroup statistics go to partials[3 * group]: outliers, max |q|,
// out-of-range flag; k_reduce_stats folds them into counters[0..2].
template <typename T>
__global__ __launch_bounds__(NT) void k_quantize(QArgs a, const T* c, int32_t* codes, int64_t* partials) {
  int64_t nout = 0, mx = 0, bad = 0;
  const uint32_t ntiles = (a.tot + NT * QU - 1) / (NT * QU);
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t base = tile * (NT * QU) + threadIdx.x;
    double cv[QU], inv[QU];
#pragma unroll
    for (int k = 0; k < QU; ++k) {
      const uint32_t i = base + k * NT;
      cv[k] = 0.0;
      inv[k] = 0.0;
      if (i < a.tot) {
        uint32_t z, y, x;
        a.uf(i, z, y, x);
        double del;
        if (a.pdel) {
          inv[k] = 1.0 / a.pdel[i];
        } else {
          node_delta(a, z, y, x, del, inv[k]);
        }
        cv[k] = double(c[i]);
      }
    }
#pragma unroll
    for (int k = 0; k < QU; ++k) {
      const uint32_t i = base + k * NT;
      if (i >= a.tot) continue;
      const double v = rint(mul_rn(cv[k], inv[k]));
      int32_t qv;
      if (!(fabs(v) <= 2147483647.0)) {
        bad |= int64_t(code_flag(double(cv[k])));
        qv = 0;
      } else {
        qv = int32_t(v);
      }
      codes[i] = qv;
      const int64_t aq = qv < 0 ? -int64_t(qv) : int64_t(qv);
      nout += aq >= 32768;
      mx = aq > mx ? aq : mx;
    }
  }
  __shared__ int64_t red[3][NT / 64];
  for (int off = 32; off > 0; off >>= 1) {
    nout += __shfl_down(nout, off, 64);
    const int64_t o = __shfl_down(mx, off, 64);
    mx = o > mx ? o : mx;
    bad |= __shfl_down(bad, off, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = nout;
    red[1][wv] = mx;
    red[2][wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s0 = 0, s1 = 0, s2 = 0;
    for (int k = 0; k < NT / 64; ++k) {
      s0 += red[0][k];
      s1 = red[1][k] > s1 ? red[1][k] : s1;
      s2 |= red[2][k];
    }
    partials[3 * blockIdx.x] = s0;
    partials[3 * blockIdx.x + 1] = s1;
    partials[3 * blockIdx.x + 2] = s2;
  }
}

__global__ __launch_bounds__(NT) void k_reduce_stats(const int64_t* partials, int n, int64_t* counters) {
  __shared__ int64_t r[3][NT];
  int64_t s0 = 0, s1 = 0, s2 = 0;
  for (int k = threadIdx.x; k < n; k += NT) {
    s0 += partials[3 * k];
    s1 = partials[3 * k + 1] > s1 ? partials[3 * k + 1] : s1;
    s2 |= partials[3 * k + 2];
  }
  r[0][threadIdx.x] = s0;
  r[1][threadIdx.x] = s1;
  r[2][threadIdx.x] = s2;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      r[0][threadIdx.x] += r[0][threadIdx.x + s];
      r[1][threadIdx.x] = r[1][threadIdx.x + s] > r[1][threadIdx.x] ? r[1][threadIdx.x + s] : r[1][threadIdx.x];
      r[2][threadIdx.x] |= r[2][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counters[0] = r[0][0];
    counters[1] = r[1][0];
    counters[2] = r[2][0];
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_dequantize(QArgs a, const int32_t* codes, T* c) {
  const uint32_t ntiles = (a.tot + NT * QU - 1) / (NT * QU);
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t base = tile * (NT * QU) + threadIdx.x;
    double q[QU], del[QU];
#pragma unroll
    for (int k = 0; k < QU; ++k) {
      const uint32_t i = base + k * NT;
      q[k] = 0.0;
      del[k] = 0.0;
      if (i < a.tot) {
        uint32_t z, y, x;
        a.uf(i, z, y, x);
        double inv;
        if (a.pdel)
          del[k] = a.pdel[i];
        else
          node_delta(a, z, y, x, del[k], inv);
        q[k] = double(codes[i]);
      }
    }
#pragma unroll
    for (int k = 0; k < QU; ++k) {
      const uint32_t i = base + k * NT;
      if (i < a.tot) c[i] = T(mul_rn(q[k], del[k]));
    }
  }
}

int64_t prod3(const int64_t n[3]) { return n[0] * n[1] * n[2]; }

}  // namespace

// Adjoint-guided widths for a linear quantity of interest Q = <g, x>: with
// s = R^T g, quantization moves Q by at most sum |s_i| Delta_i / 2.  Each
// coefficient's share |s_i| Delta_i / 2 is one level lambda, except where the
// node's L-inf width cap_i is smaller: share = min(a_i, lambda) with
// a_i = |s_i| cap_i / 2, and lambda the root of sum_i min(a_i, lambda) =
// (1 - eta) tol_q.  Sums are reduced per workgroup in a fixed order, then by
// one workgroup (deterministic).
constexpr int kQoiK = 15;           // candidate levels per pass
constexpr int kQoiGroups = 1024;    // workgroups of a pass (partials: kQoiK per group)

struct Cand {
  double v[kQoiK];
};

__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// a_i = |s_i| cap_i / 2 into share[i]; partials[2 g] = sum, [2 g + 1] = max
template <typename T>
__global__ __launch_bounds__(NT) void k_qoi_shares(QArgs a, const T* s, double* share, double* partials) {
  __shared__ double red[NT];
  double sum = 0.0, mx = 0.0;
  for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < a.tot; i += gridDim.x * NT) {
    uint32_t z, y, x;
    a.uf(i, z, y, x);
    double del, inv;
    node_delta(a, z, y, x, del, inv);
    const double v = fabs(double(s[i])) * del * 0.5;
    share[i] = v;
    sum += v;
    mx = fmax(mx, v);
  }
  sum = block_sum(sum, red);
  mx = block_max(mx, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sum;
    partials[2 * blockIdx.x + 1] = mx;
  }
}

// f(c_j) = sum_i min(a_i, c_j) for the kQoiK candidates: partials[g kQoiK + j]
__global__ __launch_bounds__(NT) void k_qoi_eval(const double* share, uint32_t n, Cand c, double* partials) {
  __shared__ double red[NT];
  double acc[kQoiK];
#pragma unroll
  for (int j = 0; j < kQoiK; ++j) acc[j] = 0.0;
  for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
    const double v = share[i];
#pragma unroll
    for (int j = 0; j < kQoiK; ++j) acc[j] += fmin(v, c.v[j]);
  }
  for (int j = 0; j < kQoiK; ++j) {
    const double r = block_sum(acc[j], red);
    if (threadIdx.x == 0) partials[blockIdx.x * kQoiK + j] = r;
  }
}

// out[j] = sum (or max, for odd j when max_odd) over ng groups of partials[g k + j]
__global__ __launch_bounds__(NT) void k_qoi_fold(const double* partials, int ng, int k, int max_odd, double* out) {
  __shared__ double red[NT];
  for (int j = 0; j < k; ++j) {
    const bool mx = max_odd && (j & 1);
    double v = 0.0;
    for (int g = threadIdx.x; g < ng; g += NT) v = mx ? fmax(v, partials[g * k + j]) : v + partials[g * k + j];
    v = mx ? block_max(v, red) : block_sum(v, red);
    if (threadIdx.x == 0) out[j] = v;
  }
}

// Delta_i = 2 lambda / |s_i| where a_i > lambda (the quantity sets the
// width), else the node's L-inf width; counts the former
template <typename T>
__global__ __launch_bounds__(NT) void k_qoi_final(QArgs a, const T* s, double lambda, double* delta,
                                                  unsigned long long* count) {
  __shared__ double red[NT];
  double c = 0.0;
  for (uint32_t i = blockIdx.x * NT + threadIdx.x; i < a.tot; i += gridDim.x * NT) {
    const double ai = delta[i];
    uint32_t z, y, x;
    a.uf(i, z, y, x);
    double del, inv;
    node_delta(a, z, y, x, del, inv);
    if (ai > lambda) {
      delta[i] = 2.0 * lambda / fabs(double(s[i]));
      c += 1.0;
    } else {
      delta[i] = del;
    }
  }
  c = block_sum(c, red);
  if (threadIdx.x == 0 && c > 0.0) atomicAdd(count, (unsigned long long)c);
}

QPrep qprep_layout(bm_plan_s& p, const double* block_tol) {
  (void)block_tol;
  if (p.L > 8) fail(BM_EUNSUPPORTED, "more than 8 local levels");
  QPrep a{};
  a.flag = p.ws.counters + 2;
  const int64_t tot = p.ws.tol_off[p.L + 1];
  double* bdel = p.ws.tolbuf + tot;
  double* binv = p.ws.tolbuf + 2 * tot;
  double* tg = p.ws.tolbuf + 3 * tot;     // tau_global
  const int64_t nlastb = p.L > 0 ? prod3(p.lv[p.L - 1].nb) : 0;
  double* cls = tg + 8 + 2 * nlastb + 8;  // 27-class tables: level s at 54 tol_off[s], coarsest at 54 tot
  for (int s = 1; s <= p.L; ++s) {
    const int64_t nbs = prod3(p.lv[s - 1].nb);
    const int64_t off = p.ws.tol_off[s];
    QTab& t = a.lv[s - 1];
    t.del = bdel + off;
    t.inv = binv + off;
    t.cdel = cls + 54 * off;
    t.cinv = cls + 54 * off + 27 * nbs;
    for (int d = 0; d < 3; ++d) t.nb[d] = p.lv[s - 1].nb[d];
  }
  if (p.L > 0 && p.M == 0) {
    // coarsest values (no gain), over the level-L blocks
    QTab& t = a.lv[kCoarseSlotHost];
    t.del = tg + 8;
    t.inv = tg + 8 + nlastb;
    t.cdel = cls + 54 * tot;
    t.cinv = cls + 54 * tot + 27 * nlastb;
    for (int d = 0; d < 3; ++d) t.nb[d] = p.lv[p.L - 1].nb[d];
  }
  a.q = p.ws.qparam;
  return a;
}

// One plan's tables are built by the many-field kernels with one field: one
// launch per propagation step, one per table level, one for tau_global and
// the scalar Deltas (which also clears the overflow flag).  The field record
// is uploaded only when it changes (a new tolerance map pointer).
namespace {
__global__ void k_clear_flag(int64_t* flag) {
  if (threadIdx.x == 0) *flag = 0;
}
}  // namespace

QPrep quant_prepare(bm_plan_s& p, const double* block_tol, hipStream_t st, bool clear_flag) {
  const QPrep a = qprep_layout(p, block_tol);
  if (block_tol && block_tol == p.ws.kept_tol) {   // the kept tables are this map's
    if (clear_flag) {
      hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, a.flag);
      BM_HIP(hipGetLastError());
    }
    return a;
  }
  p.ws.kept_tol = nullptr;   // the tables built here replace the kept ones
  const PrepField f = prep_field(p, block_tol, a);
  constexpr size_t kFirst = 2048;                   // offset of the task prefix arrays
  static_assert(sizeof(PrepField) <= kFirst, "field record too large");
  int64_t cnt_prop[9] = {}, cnt_tab[9] = {};
  for (int s = 1; s < 9; ++s) cnt_prop[s] = p.L > s ? prod3(p.lv[s].nb) : 0;
  for (int s = 1; s < 9; ++s) cnt_tab[s] = p.L >= s ? 27 * prod3(p.lv[s - 1].nb) : 0;
  cnt_tab[0] = (p.L > 0 && p.M == 0) ? 27 * prod3(p.lv[p.L - 1].nb) : 0;
  if (!p.ws.prep_dev) {
    std::vector<int64_t> first(4 * 9);
    for (int s = 0; s < 9; ++s) {
      first[2 * s] = 0;
      first[2 * s + 1] = cnt_prop[s];
      first[18 + 2 * s] = 0;
      first[18 + 2 * s + 1] = cnt_tab[s];
    }
    plan_alloc(p, &p.ws.prep_dev, kFirst + first.size() * sizeof(int64_t));
    BM_HIP(hipMemcpy(static_cast<uint8_t*>(p.ws.prep_dev) + kFirst, first.data(), first.size() * sizeof(int64_t),
                     hipMemcpyHostToDevice));
  }
  const uint8_t* fb = reinterpret_cast<const uint8_t*>(&f);
  if (p.ws.prep_key.size() != sizeof(f) || std::memcmp(p.ws.prep_key.data(), fb, sizeof(f)) != 0) {
    BM_HIP(hipMemcpyAsync(p.ws.prep_dev, fb, sizeof(f), hipMemcpyHostToDevice, st));
    BM_HIP(hipStreamSynchronize(st));
    p.ws.prep_key.assign(fb, fb + sizeof(f));
  }
  PrepStages g;
  const int64_t* first = reinterpret_cast<const int64_t*>(static_cast<uint8_t*>(p.ws.prep_dev) + kFirst);
  for (int s = 0; s < 9; ++s) {
    g.prop_first[s] = first + 2 * s;
    g.prop_n[s] = cnt_prop[s];
    g.tab_first[s] = first + 18 + 2 * s;
    g.tab_n[s] = cnt_tab[s];
  }
  launch_prep_batch(g, static_cast<const PrepField*>(p.ws.prep_dev), 1, st);
  return a;
}

void quant_keep(bm_plan_s& p, const double* block_tol, hipStream_t st) {
  p.ws.kept_tol = nullptr;
  if (!block_tol) return;
  quant_prepare(p, block_tol, st);
  p.ws.kept_tol = block_tol;
}

// ---- many fields per launch -------------------------------------------------

namespace {

// Eq. 2 from level s to level s+1 (s 1-based) for every field that has it
__global__ void k_batch_propagate(const PrepField* F, const int64_t* first, int nf, int64_t ntot, int s) {
  for (int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x; k < ntot; k += int64_t(gridDim.x) * NT) {
    const int f = task_field(first, nf, k);
    const PrepField& P = F[f];
    const int64_t i = k - first[f];
    const int64_t* nb = P.nb[s - 1];
    const int64_t* nn = P.nb[s];
    const int64_t X = i % nn[2], t = i / nn[2], Y = t % nn[1], Z = t / nn[1];
    // next-level block (Z, Y, X) spans blocks 2Z, 2Z+1 of this level and
    // touches 2Z-1, 2Z+2; nested, it is block Z itself, touching Z-1, Z+1
    const int64_t c0 = P.nested ? Z : 2 * Z, c1 = P.nested ? Y : 2 * Y, c2 = P.nested ? X : 2 * X;
    const int64_t e = P.nested ? 1 : 2;
    double v = INFINITY;
    for (int64_t z = i64max(0, c0 - 1); z <= i64min(nb[0] - 1, c0 + e); ++z)
      for (int64_t y = i64max(0, c1 - 1); y <= i64min(nb[1] - 1, c1 + e); ++y)
        for (int64_t x = i64max(0, c2 - 1); x <= i64min(nb[2] - 1, c2 + e); ++x)
          v = fmin(v, P.tau[s - 1][(z * nb[1] + y) * nb[2] + x]);
    const_cast<double*>(P.tau[s])[i] = v;
  }
}

// Per-block Delta, 1/Delta and 27-class tables of local level s (s = 0: the
// coarsest values of a field with M == 0) straight from the taus: rounding
// of tau * kappa is monotone, so the smallest Delta over a set of blocks is
// the smallest tau times kappa, and its reciprocal is the largest 1/Delta.
// Task = (block, class), consecutive tasks write consecutive entries; class
// 13 (interior) also writes the block's own entry.  Along an axis, class 0
// (first face) takes the block and the one before, 1 the block alone, 2
// (last face) the block and the one after.  32-bit index arithmetic (a
// level has fewer than 2^32 / 27 blocks).
// one task of k_batch_tables: task i of field P
__device__ inline void table_task(const PrepField& P, int s, uint32_t i) {
  const int li = s > 0 ? s - 1 : P.L - 1;
  const QTab& T = s > 0 ? P.tab[li] : P.tab[kCoarseSlotHost];
  const double kap = s > 0 ? P.kap[li] : P.kapc;
  const double* tau = P.tau[li];
  const uint32_t blk = i / 27u;
  const int c = int(i - blk * 27u);
  const int cls[3] = {c / 9, (c / 3) % 3, c % 3};
  const uint32_t n0 = uint32_t(P.nb[li][0]), n1 = uint32_t(P.nb[li][1]), n2 = uint32_t(P.nb[li][2]);
  const uint32_t t = blk / n2;
  const uint32_t b[3] = {t / n1, t - (t / n1) * n1, blk - t * n2};
  const uint32_t nb[3] = {n0, n1, n2};
  uint32_t lo[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = (cls[d] == 0 && b[d] > 0) ? b[d] - 1 : b[d];
    hi[d] = (cls[d] == 2 && b[d] + 1 < nb[d]) ? b[d] + 1 : b[d];
  }
  // each axis spans at most two blocks: the eight corners of the box
  // (repeated where lo == hi) are loaded together, then reduced
  double tv[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    tv[j] = tau[(((j & 4) ? hi[0] : lo[0]) * n1 + ((j & 2) ? hi[1] : lo[1])) * n2 + ((j & 1) ? hi[2] : lo[2])];
  const double m = fmin(fmin(fmin(tv[0], tv[1]), fmin(tv[2], tv[3])), fmin(fmin(tv[4], tv[5]), fmin(tv[6], tv[7])));
  const double d = m * kap, iv = 1.0 / d;
  const_cast<double*>(T.cdel)[i] = d;
  const_cast<double*>(T.cinv)[i] = iv;
  if (c == 13) {
    const_cast<double*>(T.del)[blk] = d;
    const_cast<double*>(T.inv)[blk] = iv;
  }
}

__global__ void k_batch_tables(const PrepField* F, const int64_t* first, int nf, int64_t ntot, int s) {
  if (nf == 1) {
    // one field: its record is the same for every lane (scalar loads)
    for (int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x; k < ntot; k += int64_t(gridDim.x) * NT)
      table_task(F[0], s, uint32_t(k - first[0]));
    return;
  }
  for (int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x; k < ntot; k += int64_t(gridDim.x) * NT) {
    const int f = task_field(first, nf, k);
    table_task(F[f], s, uint32_t(k - first[f]));
  }
}

// tau_global (minimum over the last block level, or the single map value
// when there is none) and the scalar Deltas; one workgroup per field, which
// also clears the field's overflow flag.
constexpr int kScalarNT = 1024;

__global__ __launch_bounds__(kScalarNT) void k_batch_scalar(const PrepField* F) {
  __shared__ double red[kScalarNT];
  const PrepField& P = F[blockIdx.x];
  double m = INFINITY;
  if (P.L > 0) {
    const int64_t* nb = P.nb[P.L - 1];
    const int64_t n = nb[0] * nb[1] * nb[2];
    const double* tau = P.tau[P.L - 1];
    // eight independent loads in flight per lane
    double mm[8] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
    int64_t i = threadIdx.x;
    for (; i + 7 * kScalarNT < n; i += 8 * kScalarNT)
#pragma unroll
      for (int u = 0; u < 8; ++u) mm[u] = fmin(mm[u], tau[i + u * kScalarNT]);
    for (; i < n; i += kScalarNT) mm[0] = fmin(mm[0], tau[i]);
#pragma unroll
    for (int u = 0; u < 8; ++u) m = fmin(m, mm[u]);
  } else if (threadIdx.x == 0) {
    m = P.tau[0][0];
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kScalarNT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *P.tg = red[0];
    *P.flag = 0;
  }
  if (threadIdx.x <= P.nlev) {
    const double d = red[0] * P.kq[threadIdx.x];
    P.q[2 * threadIdx.x] = d;
    P.q[2 * threadIdx.x + 1] = 1.0 / d;
  }
}

}  // namespace

PrepField prep_field(bm_plan_s& p, const double* block_tol, const QPrep& q) {
  PrepField f{};
  const double eta = p.cfg.eta;
  const std::vector<double> w = level_weights(p);
  f.L = p.L;
  f.M = p.M;
  f.nlev = p.nlev;
  f.nested = p.cfg.nested;
  if (p.nlev + 1 > 26) fail(BM_EUNSUPPORTED, "too many levels");
  for (int s = 1; s <= p.L; ++s) {
    f.tau[s - 1] = s == 1 ? block_tol : p.ws.tolbuf + p.ws.tol_off[s];
    for (int d = 0; d < 3; ++d) f.nb[s - 1][d] = p.lv[s - 1].nb[d];
    f.kap[s - 1] = (2.0 * (1.0 - eta)) * w[s - 1] / p.lv[s - 1].gain;
    f.tab[s - 1] = q.lv[s - 1];
  }
  if (p.L == 0) f.tau[0] = block_tol;
  f.kapc = (2.0 * (1.0 - eta)) * w[p.nlev];
  f.tab[kCoarseSlotHost] = q.lv[kCoarseSlotHost];
  f.tg = p.ws.tolbuf + 3 * p.ws.tol_off[p.L + 1];
  f.q = p.ws.qparam;
  for (int s = 1; s <= p.nlev; ++s) f.kq[s - 1] = (2.0 * (1.0 - eta)) * w[s - 1] / p.lv[s - 1].gain;
  f.kq[p.nlev] = (2.0 * (1.0 - eta)) * w[p.nlev];
  f.flag = q.flag;
  return f;
}

void launch_prep_batch(const PrepStages& g, const PrepField* F, int nf, hipStream_t st) {
  for (int s = 1; s < 9; ++s)
    if (g.prop_n[s] > 0)
      hipLaunchKernelGGL(k_batch_propagate, dim3(grid_for(g.prop_n[s])), dim3(NT), 0, st, F, g.prop_first[s], nf,
                         g.prop_n[s], s);
  for (int s = 0; s < 9; ++s)
    if (g.tab_n[s] > 0)
      hipLaunchKernelGGL(k_batch_tables, dim3(grid_for(g.tab_n[s])), dim3(NT), 0, st, F, g.tab_first[s], nf,
                         g.tab_n[s], s);
  hipLaunchKernelGGL(k_batch_scalar, dim3(unsigned(nf)), dim3(kScalarNT), 0, st, F);
  BM_HIP(hipGetLastError());
}

namespace {

QArgs prepare(bm_plan_s& p, const double* block_tol, hipStream_t st, bool tables = true, bool clear_flag = true) {
  const QPrep qp = tables ? quant_prepare(p, block_tol, st, clear_flag) : qprep_layout(p, block_tol);
  QArgs a{};
  const int64_t npad = prod3(p.pdims);
  if (npad >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "quantizer: padded grid of 2^32 nodes or more");
  a.tot = uint32_t(npad);
  a.uf = Unflat32(p.pdims[1], p.pdims[2]);
  for (int d = 0; d < 3; ++d) {
    int D = 0;
    for (auto& L : p.lv) D += L.coarsen[d] ? 1 : 0;
    a.D[d] = D;
  }
  a.L = p.L;
  a.M = p.M;
  a.lw = 0;
  if (p.L > 0)
    while ((1 << a.lw) < p.cfg.block - 1) ++a.lw;
  a.nested = p.cfg.nested;
  a.counters = p.ws.counters;
  for (int k = 0; k < 9; ++k) {
    a.bdelta[k] = qp.lv[k].del;
    a.binv[k] = qp.lv[k].inv;
    for (int d = 0; d < 3; ++d) a.nb[k][d] = uint32_t(qp.lv[k].nb[d]);
  }
  a.q = qp.q;
  return a;
}

}  // namespace

void tolmap_from_boxes(bm_plan_s& p, const double* boxes, int nbox, double background, double* block_tol,
                       hipStream_t st) {
  if (nbox < 0 || (nbox > 0 && !boxes)) fail(BM_EINVAL, "bad box list");
  if (!(background > 0) || !std::isfinite(background)) fail(BM_ENONFINITE, "background tolerance must be positive and finite");
  for (int j = 0; j < nbox; ++j)
    if (!(boxes[7 * j + 6] > 0) || !std::isfinite(boxes[7 * j + 6])) fail(BM_ENONFINITE, "box tolerance must be positive and finite");
  if (nbox > kMaxBoxes) fail(BM_EINVAL, "at most 4096 boxes");
  double* dbox = nullptr;
  if (nbox) {
    // the caller's list goes through pinned staging; the call then waits for
    // the copy so the staging buffer can be reused
    std::copy(boxes, boxes + 7 * nbox, p.ws.boxhost);
    BM_HIP(hipMemcpyAsync(p.ws.boxbuf, p.ws.boxhost, size_t(nbox) * 7 * sizeof(double), hipMemcpyHostToDevice, st));
    dbox = p.ws.boxbuf;
  }
  BoxArgs a{dbox, nbox, background, {p.dims[0], p.dims[1], p.dims[2]}, {p.nb1[0], p.nb1[1], p.nb1[2]},
            p.L > 0 ? p.cfg.block - 1 : 0, block_tol};
  hipLaunchKernelGGL(k_tol_boxes, dim3(grid_for(prod3(p.nb1))), dim3(NT), 0, st, a);
  BM_HIP(hipGetLastError());
  if (dbox) BM_HIP(hipStreamSynchronize(st));
}

void tolmap_from_voxels(bm_plan_s& p, const double* voxel_tol, double* block_tol, hipStream_t st) {
  if (p.L > 0) {
    VoxArgs a{voxel_tol, {p.dims[0], p.dims[1], p.dims[2]}, {p.nb1[0], p.nb1[1], p.nb1[2]}, p.cfg.block - 1, block_tol};
    hipLaunchKernelGGL(k_tol_voxels, dim3(unsigned(prod3(p.nb1))), dim3(NT), 0, st, a);
  } else {
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(NT), 0, st, block_tol, int64_t(1), double(INFINITY));
    hipLaunchKernelGGL(k_min_all, dim3(grid_for(prod3(p.dims))), dim3(NT), 0, st, voxel_tol, prod3(p.dims), block_tol);
  }
  BM_HIP(hipGetLastError());
}

void quantize(bm_plan_s& p, const void* coeff, const double* block_tol, int32_t* codes, bm_qstats* stats,
              hipStream_t st) {
  const int64_t tot = prod3(p.pdims);
  {
    TimedScope ts(p, 2 * p.nlev, st);
    QArgs a = prepare(p, block_tol, st);
    const unsigned g = qgroups(a.tot);
    int64_t* partials = p.ws.counters + 16;
    if (p.cfg.dtype == BM_F32)
      hipLaunchKernelGGL(k_quantize<float>, dim3(g), dim3(NT), 0, st, a, static_cast<const float*>(coeff), codes,
                         partials);
    else
      hipLaunchKernelGGL(k_quantize<double>, dim3(g), dim3(NT), 0, st, a, static_cast<const double*>(coeff), codes,
                         partials);
    hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(NT), 0, st, partials, int(g), p.ws.counters);
    BM_HIP(hipGetLastError());
  }
  if (stats) {
    int64_t h[4];
    BM_HIP(hipMemcpyAsync(h, p.ws.counters, sizeof(h), hipMemcpyDeviceToHost, st));
    BM_HIP(hipStreamSynchronize(st));
    stats->n_codes = tot;
    stats->n_outliers = h[0];
    stats->max_abs_code = h[1];
    check_code_flag(h[2], "tolerance too small for the data");
  }
}

void dequantize(bm_plan_s& p, const int32_t* codes, const double* block_tol, void* coeff, hipStream_t st) {
  TimedScope ts(p, 2 * p.nlev + 1, st);
  QArgs a = prepare(p, block_tol, st, true, false);
  const int64_t tot = prod3(p.pdims);
  (void)tot;
  const unsigned g = qgroups(a.tot);
  if (p.cfg.dtype == BM_F32)
    hipLaunchKernelGGL(k_dequantize<float>, dim3(g), dim3(NT), 0, st, a, codes, static_cast<float*>(coeff));
  else
    hipLaunchKernelGGL(k_dequantize<double>, dim3(g), dim3(NT), 0, st, a, codes, static_cast<double*>(coeff));
  BM_HIP(hipGetLastError());
}

int64_t qoi_deltas(bm_plan_s& p, const void* g, double tol_q, const double* block_tol, double* delta,
                   hipStream_t st) {
  if (!(tol_q > 0) || !std::isfinite(tol_q)) fail(BM_ENONFINITE, "tol_q must be positive and finite");
  const size_t npad = size_t(prod3(p.pdims));
  if (!p.ws.coeff) plan_alloc(p, &p.ws.coeff, npad * p.esize);
  // sensitivities s = R^T g of the quantity to the coefficients
  recompose_adjoint(p, g, p.ws.coeff, st);
  QArgs a = prepare(p, block_tol, st);
  const bool f32 = p.cfg.dtype == BM_F32;
  // partial sums live in the plan's statistics scratch (3 x 8192 slots after
  // the 16 counters): up to kQoiGroups x kQoiK partials, then 16 folded values
  double* part = reinterpret_cast<double*>(p.ws.counters + 16);
  double* fold = part + kQoiGroups * kQoiK;
  static_assert(kQoiGroups * kQoiK + 16 <= 3 * 8192, "QoI partials exceed the statistics scratch");
  const unsigned gs = std::min<unsigned>(grid_for(int64_t(a.tot)), unsigned(kQoiGroups));
  // a_i = |s_i| cap_i / 2 (held in delta until the last pass), their sum and max
  if (f32)
    hipLaunchKernelGGL(k_qoi_shares<float>, dim3(gs), dim3(NT), 0, st, a, static_cast<const float*>(p.ws.coeff),
                       delta, part);
  else
    hipLaunchKernelGGL(k_qoi_shares<double>, dim3(gs), dim3(NT), 0, st, a, static_cast<const double*>(p.ws.coeff),
                       delta, part);
  hipLaunchKernelGGL(k_qoi_fold, dim3(1), dim3(NT), 0, st, part, int(gs), 2, 1, fold);
  BM_HIP(hipGetLastError());
  double sm[2];
  BM_HIP(hipMemcpyAsync(sm, fold, sizeof(sm), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  const double target = (1.0 - p.cfg.eta) * tol_q;
  double lambda = INFINITY;   // every cap fits: no width is set by the quantity
  if (sm[0] > target) {
    // f(lambda) = sum min(a_i, lambda) rises from f(lo) <= tot lo = target to
    // f(max a) = sum a > target; kQoiK candidates per pass narrow [lo, hi]
    // (geometric steps while hi > 2 lo, then even steps) until no double lies
    // between; lambda = lo keeps f(lambda) <= target, so the quantity's bound holds
    double lo = target / double(a.tot), hi = sm[1];
    for (int pass = 0; pass < 80 && hi > lo; ++pass) {
      Cand c;
      for (int j = 0; j < kQoiK; ++j) {
        const double t = double(j + 1) / double(kQoiK + 1);
        c.v[j] = hi > 2.0 * lo ? lo * std::pow(hi / lo, t) : lo + (hi - lo) * t;
      }
      hipLaunchKernelGGL(k_qoi_eval, dim3(unsigned(kQoiGroups)), dim3(NT), 0, st, static_cast<const double*>(delta),
                         a.tot, c, part);
      hipLaunchKernelGGL(k_qoi_fold, dim3(1), dim3(NT), 0, st, part, kQoiGroups, kQoiK, 0, fold);
      BM_HIP(hipGetLastError());
      double f[kQoiK];
      BM_HIP(hipMemcpyAsync(f, fold, sizeof(f), hipMemcpyDeviceToHost, st));
      BM_HIP(hipStreamSynchronize(st));
      double nlo = lo, nhi = hi;
      for (int j = 0; j < kQoiK; ++j) {
        if (!(c.v[j] > lo && c.v[j] < hi)) continue;
        if (f[j] <= target)
          nlo = std::max(nlo, c.v[j]);
        else
          nhi = std::min(nhi, c.v[j]);
      }
      if (nlo == lo && nhi == hi) break;   // no candidate strictly inside: converged
      if (nlo >= nhi) {                    // sums not monotone at rounding level
        lo = nlo;
        break;
      }
      lo = nlo;
      hi = nhi;
    }
    lambda = lo;
  }
  auto* cnt = reinterpret_cast<unsigned long long*>(p.ws.counters + 3);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, cnt);
  const unsigned gq = grid_for(int64_t(a.tot));
  if (f32)
    hipLaunchKernelGGL(k_qoi_final<float>, dim3(gq), dim3(NT), 0, st, a, static_cast<const float*>(p.ws.coeff),
                       lambda, delta, cnt);
  else
    hipLaunchKernelGGL(k_qoi_final<double>, dim3(gq), dim3(NT), 0, st, a, static_cast<const double*>(p.ws.coeff),
                       lambda, delta, cnt);
  BM_HIP(hipGetLastError());
  unsigned long long nset = 0;
  BM_HIP(hipMemcpyAsync(&nset, cnt, sizeof(nset), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  return int64_t(nset);
}

void quantize_delta(bm_plan_s& p, const void* coeff, const double* delta, int32_t* codes, bm_qstats* stats,
                    hipStream_t st) {
  QArgs a = prepare(p, nullptr, st, false);
  a.pdel = delta;
  const unsigned g = qgroups(a.tot);
  int64_t* partials = p.ws.counters + 16;
  if (p.cfg.dtype == BM_F32)
    hipLaunchKernelGGL(k_quantize<float>, dim3(g), dim3(NT), 0, st, a, static_cast<const float*>(coeff), codes, partials);
  else
    hipLaunchKernelGGL(k_quantize<double>, dim3(g), dim3(NT), 0, st, a, static_cast<const double*>(coeff), codes,
                       partials);
  hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(NT), 0, st, partials, int(g), p.ws.counters);
  BM_HIP(hipGetLastError());
  if (stats) {
    int64_t h[4];
    BM_HIP(hipMemcpyAsync(h, p.ws.counters, sizeof(h), hipMemcpyDeviceToHost, st));
    BM_HIP(hipStreamSynchronize(st));
    stats->n_codes = int64_t(a.tot);
    stats->n_outliers = h[0];
    stats->max_abs_code = h[1];
    check_code_flag(h[2], "Delta too small for the data");
  }
}

void dequantize_delta(bm_plan_s& p, const int32_t* codes, const double* delta, void* coeff, hipStream_t st) {
  QArgs a = prepare(p, nullptr, st, false);
  a.pdel = delta;
  const unsigned g = qgroups(a.tot);
  if (p.cfg.dtype == BM_F32)
    hipLaunchKernelGGL(k_dequantize<float>, dim3(g), dim3(NT), 0, st, a, codes, static_cast<float*>(coeff));
  else
    hipLaunchKernelGGL(k_dequantize<double>, dim3(g), dim3(NT), 0, st, a, codes, static_cast<double*>(coeff));
  BM_HIP(hipGetLastError());
}

}  // namespace bm
