// Time model of the pipeline and the choice of (L, M) by Algorithm 1
// (Sec. IV-B).
//
// Eq. 1: N concurrent blocks run at TP(N) = N / (1/Slope + N/TP_peak), so a
// block level of N blocks takes N / TP(N) = 1/Slope + N/TP_peak.  Global
// levels are fitted by a line in their node count; quantization by
// max(slope N, T_lat); the lossless stage by one line per Huffman stage.
// Algorithm 1 predicts decomposition + quantization + lossless time of every
// valid (L, M) and keeps, among those within the time budget, the one with
// the most global levels, then the fewest block levels.
//
// The fits are measured here on the device (bm_model_calibrate): each stage
// is run on synthetic inputs of growing size and timed with HIP events (the
// per-level events of the fused pipeline, the Huffman stages one by one), and
// a least-squares line is taken through (N, t).  The pipeline as built has
// two kinds of block level and of global level: a block level followed by a
// global level forms that level's details and partial load vectors itself
// (the "fused" block level), and the global level after it only gathers and
// solves (the "fused" global level); both get their own fit.

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

bm_plan_s* bm_plan_build(const bm_config* c);
void bm_plan_free(bm_plan_s* p);

namespace bm {
namespace {

__device__ inline uint32_t mix32(uint32_t v) {
  v ^= v >> 16;
  v *= 0x7feb352du;
  v ^= v >> 15;
  v *= 0x846ca68bu;
  v ^= v >> 16;
  return v;
}

// calibration field: three smooth modes plus small hashed noise
template <typename T>
__global__ void k_synth(T* x, int64_t n0, int64_t n1, int64_t n2, uint32_t seed) {
  const int64_t tot = n0 * n1 * n2;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < tot; i += int64_t(gridDim.x) * 256) {
    const int64_t z = i / (n1 * n2), r = i - z * n1 * n2, y = r / n2, xx = r - y * n2;
    const double u = double(z) / double(n0), v = double(y) / double(n1), w = double(xx) / double(n2);
    const double noise = double(mix32(uint32_t(i) ^ seed) >> 8) / 16777216.0 - 0.5;
    x[i] = T(sin(6.3 * u + 1.0) * cos(9.1 * v) + 0.5 * sin(12.7 * w + 2.0 * u) + 1e-3 * noise);
  }
}

// calibration codes: two-sided geometric (discrete Laplace, scale 4) from a hash
__global__ void k_synth_codes(int32_t* q, int64_t n, uint32_t seed) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const uint32_t h = mix32(uint32_t(i) * 2654435761u ^ seed);
    const double u = (double(h >> 9) + 0.5) / 8388608.0;
    const int32_t m = int32_t(-4.0 * log(u));
    q[i] = (h & 1u) ? m : -m;
  }
}

struct Line {
  double a = 0, b = 0;   // t = a + b N
};

Line fit_line(const std::vector<double>& N, const std::vector<double>& t) {
  const double k = double(N.size());
  double sn = 0, st = 0, snn = 0, snt = 0;
  for (size_t i = 0; i < N.size(); ++i) {
    sn += N[i];
    st += t[i];
    snn += N[i] * N[i];
    snt += N[i] * t[i];
  }
  Line l;
  const double den = k * snn - sn * sn;
  l.b = den != 0 ? (k * snt - sn * st) / den : 0.0;
  l.a = (st - l.b * sn) / k;
  if (l.b < 0) {   // flat data: latency only
    l.b = 0;
    l.a = st / k;
  }
  if (l.a < 0) l.a = 0;
  return l;
}

struct Run {
  std::vector<double> level_ms;   // per level s = 1..L+M, mean per call
  double call_ms = 0;             // whole fused decompose + quantize call, mean
  int64_t nodes = 0;              // padded nodes
};

// the fused decompose + quantize of a synthetic cube of side n with (b, L, M)
Run time_plan(int dtype, int b, int L, int M, int64_t n, int reps, hipStream_t st) {
  bm_config c{};
  c.ndim = 3;
  c.dims[0] = c.dims[1] = c.dims[2] = n;
  c.dtype = dtype;
  c.block = b;
  c.L = L;
  c.M = M;
  c.eta = dtype == BM_F32 ? 0.1 : 1e-6;
  struct G {
    bm_plan_s* p = nullptr;
    void *x = nullptr, *codes = nullptr, *tol = nullptr;
    ~G() {
      for (void* q : {x, codes, tol})
        if (q) (void)hipFree(q);
      if (p) bm_plan_free(p);
    }
  } g;
  g.p = bm_plan_build(&c);
  bm_plan_s& p = *g.p;
  const size_t es = dtype == BM_F32 ? 4 : 8;
  const int64_t nlog = n * n * n, npad = p.pdims[0] * p.pdims[1] * p.pdims[2];
  const int64_t ntol = p.nb1[0] * p.nb1[1] * p.nb1[2];
  BM_HIP(hipMalloc(&g.x, size_t(nlog) * es));
  BM_HIP(hipMalloc(&g.codes, size_t(npad) * 4));
  BM_HIP(hipMalloc(&g.tol, size_t(ntol) * 8));
  const unsigned grid = unsigned(std::min<int64_t>(4096, (nlog + 255) / 256));
  if (dtype == BM_F32)
    hipLaunchKernelGGL(k_synth<float>, dim3(grid), dim3(256), 0, st, static_cast<float*>(g.x), n, n, n, 12345u);
  else
    hipLaunchKernelGGL(k_synth<double>, dim3(grid), dim3(256), 0, st, static_cast<double*>(g.x), n, n, n, 12345u);
  BM_HIP(hipGetLastError());
  tolmap_from_boxes(p, nullptr, 0, 1e-3, static_cast<double*>(g.tol), st);
  int32_t* codes = static_cast<int32_t*>(g.codes);
  const double* tol = static_cast<const double*>(g.tol);
  for (int r = 0; r < 2; ++r) decompose_quantize(p, g.x, tol, codes, nullptr, st);
  BM_HIP(hipStreamSynchronize(st));
  drain_timing(p);
  p.timing.ms.assign(2 * p.nlev + 2, 0.0);
  p.timing.calls.assign(2 * p.nlev + 2, 0);
  p.timing.on = true;
  hipEvent_t a, e;
  BM_HIP(hipEventCreate(&a));
  BM_HIP(hipEventCreate(&e));
  BM_HIP(hipEventRecord(a, st));
  for (int r = 0; r < reps; ++r) decompose_quantize(p, g.x, tol, codes, nullptr, st);
  BM_HIP(hipEventRecord(e, st));
  BM_HIP(hipEventSynchronize(e));
  float tot = 0.f;
  BM_HIP(hipEventElapsedTime(&tot, a, e));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(e);
  drain_timing(p);
  p.timing.on = false;
  Run out;
  out.call_ms = double(tot) / reps;
  out.nodes = npad;
  for (int s = 1; s <= p.nlev; ++s) out.level_ms.push_back(p.timing.ms[2 * (s - 1)] / reps);
  return out;
}

}  // namespace

void model_calibrate(int dtype, int b, bm_model& m, hipStream_t st) {
  if (dtype != BM_F32 && dtype != BM_F64) fail(BM_EINVAL, "dtype must be BM_F32 or BM_F64");
  if (b != 9 && b != 17 && b != 33) fail(BM_EINVAL, "block must be 9, 17 or 33");
  m = bm_model{};
  m.dtype = dtype;
  m.block = b;
  const int reps = 5;
  const int64_t w = b - 1;
  // block levels: cubes of k blocks per side, (L, M) = (1, 0) (plain) and (1, 1)
  // (fused block level + fused global level); the quantizer preparation is the
  // call time outside the level events
  std::vector<double> nb, tp, tf, nf, tg2, nq, tq, ngq, tgq;
  for (int k : {1, 2, 4, 8, 16, 32}) {
    const int64_t n = w * k + 1;
    if (n > 1025 || (b == 33 && k > 16)) continue;
    const Run r0 = time_plan(dtype, b, 1, 0, n, reps, st);
    nb.push_back(double(k) * k * k);
    tp.push_back(r0.level_ms[0]);
    nq.push_back(double(r0.nodes));
    tq.push_back(std::max(0.0, r0.call_ms - r0.level_ms[0]));
    if (b != 33) {
      const Run r1 = time_plan(dtype, b, 1, 1, n, reps, st);
      tf.push_back(r1.level_ms[0]);
      const int64_t m2 = (n + 1) / 2;   // nodes per axis of the global level's grid
      nf.push_back(double(m2) * m2 * m2);
      tg2.push_back(r1.level_ms[1]);
    }
  }
  const Line lb = fit_line(nb, tp);
  m.blk_lat_ms = lb.a;
  m.blk_tp = lb.b > 0 ? 1.0 / lb.b : 0.0;
  if (!tf.empty()) {
    const Line lf = fit_line(nb, tf);
    m.fblk_lat_ms = lf.a;
    m.fblk_tp = lf.b > 0 ? 1.0 / lf.b : 0.0;
    const Line lg = fit_line(nf, tg2);
    m.fglob_a_ms = lg.a;
    m.fglob_b_ms = lg.b;
  } else {   // 33^3 blocks take no fused global level: the plain fits serve
    m.fblk_lat_ms = m.blk_lat_ms;
    m.fblk_tp = m.blk_tp;
  }
  // global levels: pure global (L, M) = (0, 1) on cubes 2^j + 1
  std::vector<double> ng, tgl;
  for (int j = 4; j <= 9; ++j) {
    const int64_t n = (int64_t(1) << j) + 1;
    const Run r = time_plan(dtype, b, 0, 1, n, reps, st);
    ng.push_back(double(n) * n * n);
    tgl.push_back(r.level_ms[0]);
    ngq.push_back(double(r.nodes));
    tgq.push_back(std::max(0.0, r.call_ms - r.level_ms[0]));
  }
  const Line lg = fit_line(ng, tgl);
  m.glob_a_ms = lg.a;
  m.glob_b_ms = lg.b;
  if (tf.empty()) {
    m.fglob_a_ms = m.glob_a_ms;
    m.fglob_b_ms = m.glob_b_ms;
  }
  // quantization: max(slope N, T_lat), fitted apart for the local quantizer
  // (block plans: per-block tables) and the global one (all-global plans);
  // T_lat the smallest inputs' mean, slope from the largest
  auto quant_fit = [](const std::vector<double>& N, const std::vector<double>& t, double& slope, double& lat) {
    std::vector<size_t> idx(N.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return N[x] < N[y]; });
    double s = 0;
    const size_t k0 = std::min<size_t>(3, idx.size());
    for (size_t i = 0; i < k0; ++i) s += t[idx[i]];
    lat = k0 ? s / double(k0) : 0.0;
    const size_t il = idx.empty() ? 0 : idx.back();
    slope = (!idx.empty() && N[il] > 0) ? t[il] / N[il] : 0.0;
  };
  quant_fit(nq, tq, m.q_slope_ms, m.q_lat_ms);
  quant_fit(ngq, tgq, m.gq_slope_ms, m.gq_lat_ms);
  // lossless: one line per Huffman stage, on code arrays of 2^16 .. 2^26
  int32_t* q = nullptr;
  const int64_t qmax = int64_t(1) << 26;
  BM_HIP(hipMalloc(&q, size_t(qmax) * 4));
  struct QG {
    int32_t* q;
    ~QG() { (void)hipFree(q); }
  } qg{q};
  hipLaunchKernelGGL(k_synth_codes, dim3(4096), dim3(256), 0, st, q, qmax, 777u);
  BM_HIP(hipGetLastError());
  std::vector<double> nh;
  std::vector<double> th[4];
  for (int e = 16; e <= 26; e += 2) {
    const int64_t n = int64_t(1) << e;
    double ms[4] = {0, 0, 0, 0}, acc[4] = {0, 0, 0, 0};
    huffman_stage_times(q, n, st, ms);   // warm-up
    for (int r = 0; r < 3; ++r) {
      huffman_stage_times(q, n, st, ms);
      for (int k = 0; k < 4; ++k) acc[k] += ms[k] / 3.0;
    }
    nh.push_back(double(n));
    for (int k = 0; k < 4; ++k) th[k].push_back(acc[k]);
  }
  for (int k = 0; k < 4; ++k) {
    const Line l = fit_line(nh, th[k]);
    m.huf_a_ms[k] = l.a;
    m.huf_b_ms[k] = l.b;
  }
}

// Predicted decomposition, quantization and lossless times of cfg (with the
// model's block size).
void model_predict(const bm_model& m, const bm_config& cfg, double out[4]) {
  bm_config c = cfg;
  c.block = m.block;
  c.dtype = m.dtype;
  int64_t d[3] = {1, 1, 1};
  if (c.ndim < 1 || c.ndim > 3) fail(BM_EINVAL, "ndim must be 1, 2 or 3");
  for (int a = 0; a < c.ndim; ++a) d[3 - c.ndim + a] = c.dims[a];
  int64_t n[3];
  for (int a = 0; a < 3; ++a) n[a] = padded_length(d[a], c.L > 0 ? c.block : 0, c.L, c.M, c.nested != 0);
  const double nodes = double(n[0]) * double(n[1]) * double(n[2]);
  const bool fused = c.L > 0 && c.M > 0 && c.block != 33;
  double td = 0, tq = 0;
  for (int s = 1; s <= c.L + c.M; ++s) {
    if (s <= c.L) {
      double blocks = 1;
      for (int a = 0; a < 3; ++a) blocks *= double((n[a] - 1) / (c.block - 1));
      const bool fb = fused && s == c.L;
      const double lat = fb ? m.fblk_lat_ms : m.blk_lat_ms, tp = fb ? m.fblk_tp : m.blk_tp;
      td += lat + (tp > 0 ? blocks / tp : 0.0);
      // the local quantizer builds its tables per block level
      tq += std::max(m.q_slope_ms * double(n[0]) * double(n[1]) * double(n[2]), m.q_lat_ms);
    } else {
      const double g = double(n[0]) * double(n[1]) * double(n[2]);
      const bool fg = fused && s == c.L + 1;
      td += fg ? m.fglob_a_ms + m.fglob_b_ms * g : m.glob_a_ms + m.glob_b_ms * g;
    }
    for (int a = 0; a < 3; ++a)
      if (n[a] > 2) n[a] = (n[a] + 1) / 2;
  }
  // an all-global hierarchy: the global quantizer alone
  if (c.L == 0) tq = std::max(m.gq_slope_ms * nodes, m.gq_lat_ms);
  double tl = 0;
  for (int k = 0; k < 4; ++k) tl += m.huf_a_ms[k] + m.huf_b_ms[k] * nodes;
  out[0] = td;
  out[1] = tq;
  out[2] = tl;
  out[3] = td + tq + tl;
}

// Algorithm 1 over the model's block size: every (L, M) the dims admit
// (L = 0..4, M = 0..6, L + M >= 1, padding at most 1/8 of the volume);
// among the candidates whose predicted total fits the budget, the most
// global levels, then the fewest block levels.  Returns false (and the
// fastest predicted candidate) when none fits.
bool select_levels(const bm_config& in, const bm_model& m, double budget_ms, bm_config& out,
                   std::vector<bm_candidate>& cands) {
  if (!(budget_ms > 0) || !std::isfinite(budget_ms)) fail(BM_EINVAL, "budget must be positive and finite");
  int64_t d[3] = {1, 1, 1};
  for (int a = 0; a < in.ndim; ++a) d[3 - in.ndim + a] = in.dims[a];
  const double nlog = double(d[0]) * double(d[1]) * double(d[2]);
  cands.clear();
  for (int L = 0; L <= 4; ++L)
    for (int M = 0; M <= 6; ++M) {
      if (L + M < 1) continue;
      bm_config c = in;
      c.block = m.block;
      c.dtype = m.dtype;
      c.L = L;
      c.M = M;
      c.nested = 0;
      int64_t pd[3];
      bool ok = true;
      try {
        for (int a = 0; a < 3; ++a) pd[a] = padded_length(d[a], L > 0 ? c.block : 0, L, M, false);
        // every level must coarsen some axis, and global levels take axes of at most 1151 nodes
        int64_t n[3] = {pd[0], pd[1], pd[2]};
        for (int s = 1; s <= L + M && ok; ++s) {
          bool any = false;
          for (int a = 0; a < 3; ++a) {
            if (n[a] <= 2) continue;
            any = true;
            if (s > L && (n[a] + 1) / 2 > 576) ok = false;
            n[a] = (n[a] + 1) / 2;
          }
          ok = ok && any;
        }
      } catch (const Error&) {
        ok = false;
      }
      if (!ok) continue;
      if (double(pd[0]) * double(pd[1]) * double(pd[2]) > 1.125 * nlog) continue;
      double t[4];
      model_predict(m, c, t);
      bm_candidate k{};
      k.block = L > 0 ? m.block : 0;
      k.L = L;
      k.M = M;
      k.status = BM_OK;
      k.ms = t[3];
      k.ratio = 0.0;
      cands.push_back(k);
    }
  if (cands.empty()) fail(BM_EINVAL, "no admissible (L, M) for these dims");
  const bm_candidate* win = nullptr;
  for (auto& k : cands) {
    if (k.ms > budget_ms) continue;
    if (!win || k.M > win->M || (k.M == win->M && k.L < win->L)) win = &k;
  }
  const bool fits = win != nullptr;
  if (!win)
    for (auto& k : cands)
      if (!win || k.ms < win->ms) win = &k;
  out = in;
  out.block = m.block;
  out.dtype = m.dtype;
  out.L = win->L;
  out.M = win->M;
  out.nested = 0;
  return fits;
}

}  // namespace bm
