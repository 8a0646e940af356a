// Choice of block size and level split (b, L, M) by measurement.
//
// The hybrid hierarchy trades block levels (on chip, one sweep each) against
// global levels (whole-grid line solves); the paper picks (L, M) from a
// fitted throughput model under a time budget (Sec. IV-B, Algorithm 1).  Here
// every admissible candidate is run on the caller's field and tolerance:
// the fused decompose + quantize is timed with HIP events (median over
// repetitions), the coded size is the exact Huffman stream size of its
// codes, and the Huffman encode of those codes is timed on the host.  Two
// rules pick from the measured table: the fastest candidate (decompose +
// quantize) whose compression ratio is within a slack of the best ratio, or
// the rule of Algorithm 1 under a time budget on the whole pipeline
// (transform, quantization, lossless encode): of the candidates that fit it,
// the most global levels M, then the fewest block levels L (the paper's
// order), then the best ratio.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "internal.h"

bm_plan_s* bm_plan_build(const bm_config* c);
void bm_plan_free(bm_plan_s* p);

namespace bm {

namespace {

struct PlanGuard {
  bm_plan_s* p = nullptr;
  double* tol = nullptr;
  ~PlanGuard() {
    if (tol) (void)hipFree(tol);
    if (p) bm_plan_free(p);
  }
};

// pinned host memory for the candidates' Huffman streams, kept across the
// candidates of one autotune call (grown when a stream needs more)
struct PinnedStream {
  uint8_t* p = nullptr;
  size_t cap = 0;
  uint8_t* get(size_t n) {
    if (n > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      BM_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), n, hipHostMallocDefault));
      cap = n;
    }
    return p;
  }
  ~PinnedStream() {
    if (p) (void)hipHostFree(p);
  }
};

// one candidate: time (ms) and ratio; status BM_OK, or BM_ERANGE when codes
// overflow (the container would store the raw data: ratio 1)
void measure(const bm_config& cfg, const void* x, const double* voxel_tol, int reps, bm_candidate& c,
             PinnedStream& pin, hipStream_t st) {
  PlanGuard g;
  g.p = bm_plan_build(&cfg);
  bm_plan_s& p = *g.p;
  const int64_t npad = p.pdims[0] * p.pdims[1] * p.pdims[2];
  const int64_t nlog = p.dims[0] * p.dims[1] * p.dims[2];
  const int64_t ntol = p.nb1[0] * p.nb1[1] * p.nb1[2];
  BM_HIP(hipMalloc(&g.tol, size_t(ntol) * sizeof(double)));
  plan_alloc(p, &p.ws.codes, size_t(npad) * sizeof(int32_t));
  int32_t* codes = static_cast<int32_t*>(p.ws.codes);
  tolmap_from_voxels(p, voxel_tol, g.tol, st);
  bm_qstats qs;
  c.status = BM_OK;
  try {
    decompose_quantize(p, x, g.tol, codes, &qs, st);   // warm-up, and the overflow check
  } catch (const Error& e) {
    if (e.code != BM_ERANGE) throw;
    c.status = BM_ERANGE;
  }
  std::vector<float> ms;
  hipEvent_t a, b;
  BM_HIP(hipEventCreate(&a));
  BM_HIP(hipEventCreate(&b));
  for (int r = 0; r < std::max(1, reps); ++r) {
    BM_HIP(hipEventRecord(a, st));
    decompose_quantize(p, x, g.tol, codes, nullptr, st);
    BM_HIP(hipEventRecord(b, st));
    BM_HIP(hipEventSynchronize(b));
    float t = 0;
    BM_HIP(hipEventElapsedTime(&t, a, b));
    ms.push_back(t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::sort(ms.begin(), ms.end());
  c.ms = ms[ms.size() / 2];
  const double raw = double(nlog) * double(p.esize);
  double coded = raw;
  c.lossless_ms = 0.0;
  if (c.status == BM_OK) {
    // one encode into pinned host memory gives the coded size and the
    // lossless stage's time (histogram, code table, chunk sizes, encode, copy
    // out; its work buffers are allocated per encode, as in compress)
    const auto t0 = std::chrono::steady_clock::now();
    HuffmanEncoder enc(codes, npad, st);
    const size_t bytes = enc.bytes();
    enc.write(pin.get(bytes), bytes);
    c.lossless_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    coded = double(bytes) + 8.0 * double(ntol) + 128.0;
  }
  c.ratio = raw / std::min(coded, raw);
}

}  // namespace

std::vector<bm_candidate> autotune(const bm_config& in, const void* x, const double* voxel_tol, double slack, int reps,
                                   bm_config& out, hipStream_t st, double budget_ms, bool* fits) {
  const bool budget = budget_ms > 0.0;
  if (!budget && !(slack >= 0.0 && slack < 1.0)) fail(BM_EINVAL, "slack must lie in [0, 1)");
  if (budget_ms < 0.0 || !std::isfinite(budget_ms)) fail(BM_EINVAL, "budget must be positive and finite");
  std::vector<bm_candidate> cands;
  PinnedStream pin;
  int64_t nlog = 1;
  for (int a = 0; a < in.ndim; ++a) nlog *= in.dims[a];
  auto consider = [&](int block, int L, int M, int nested) {
    bm_config c = in;
    c.block = block;
    c.L = L;
    c.M = M;
    c.nested = nested;
    // admissible: the plan exists and pads the volume by at most 1/8
    bm_plan_s* probe = nullptr;
    try {
      probe = bm_plan_build(&c);
    } catch (const Error&) {
      return;
    }
    const int64_t npad = probe->pdims[0] * probe->pdims[1] * probe->pdims[2];
    bm_plan_free(probe);
    if (double(npad) > 1.125 * double(nlog)) return;
    bm_candidate k{};
    k.block = block;
    k.L = L;
    k.M = M;
    k.nested = nested;
    measure(c, x, voxel_tol, reps, k, pin, st);
    cands.push_back(k);
  };
  for (int M = 1; M <= 6; ++M) consider(0, 0, M, 0);
  for (int block : {9, 17, 33})
    for (int L = 1; L <= 4; ++L)
      for (int M = 0; M <= 4; ++M) {
        consider(block, L, M, 0);
        if (L >= 2) consider(block, L, M, 1);   // (a plan the schedule does not admit is skipped)
      }
  if (cands.empty()) fail(BM_EINVAL, "no admissible (block, L, M) for these dims");
  const bm_candidate* win = nullptr;
  if (budget) {
    // Algorithm 1: argmax (M, -L) over the candidates whose pipeline
    // (transform + quantization + lossless encode) fits the budget; ties
    // (block sizes) by the better ratio.  None fits: the fastest pipeline.
    for (auto& k : cands) {
      if (k.ms + k.lossless_ms > budget_ms) continue;
      if (!win || k.M > win->M || (k.M == win->M && (k.L < win->L || (k.L == win->L && k.ratio > win->ratio))))
        win = &k;
    }
    if (fits) *fits = win != nullptr;
    if (!win)
      for (auto& k : cands)
        if (!win || k.ms + k.lossless_ms < win->ms + win->lossless_ms) win = &k;
  } else {
    double best = 0;
    for (auto& k : cands) best = std::max(best, k.ratio);
    for (auto& k : cands)
      if (k.ratio >= (1.0 - slack) * best && (!win || k.ms < win->ms)) win = &k;
  }
  out = in;
  out.block = win->block == 0 ? in.block : win->block;
  out.L = win->L;
  out.M = win->M;
  out.nested = win->nested;
  return cands;
}

}  // namespace bm
