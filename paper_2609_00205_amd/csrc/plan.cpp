// Plan construction: padding, level schedule, per-level gains, Thomas pivots,
// device workspace.  Host code.
//
// Sec. II-B: an axis of n nodes coarsens to floor(n/2)+1; levels are applied
// down to the coarsest representation.  Sec. IV-B: the hybrid hierarchy runs
// L In-cache Block levels, then M global levels on the block-coarse grid.

#include <cstdlib>
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"
#include "line_solve.h"

namespace bm {

[[noreturn]] void fail(bm_status code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(BM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void check_code_flag(int64_t f, const char* what) {
  if (f & kFlagNonFinite) fail(BM_ENONFINITE, "NaN or Inf in the data (a coefficient is not finite)");
  if (f) fail(BM_ERANGE, std::string("a quantization code does not fit in 32 bits (") + what + ")");
}

// ------------------------------------------------------------------ padding
// Smallest n' >= n on which L levels of b-node shared-face blocks tile
// exactly ((n'-1) divisible by (b-1) 2^(L-1), at least b nodes at every
// local level) and each of the M global levels halves an odd length (a
// length <= 2 is left as it is).  Nested schedule: level s has
// (b-1)/2^(s-1)+1-node blocks over the level-1 block regions, so the
// first level's tiling ((n'-1) divisible by b-1) is all that is needed.
static bool global_chain_ok(int64_t n, int M) {
  for (int j = 0; j < M; ++j) {
    if (n <= 2) continue;
    if ((n & 1) == 0) return false;
    n = (n + 1) / 2;
  }
  return true;
}

int64_t padded_length(int64_t n, int b, int L, int M, bool nested) {
  if (n < 1) fail(BM_EINVAL, "empty axis");
  const int64_t q = L > 0 ? (nested ? int64_t(b - 1) : int64_t(b - 1) << (L - 1)) : 1;
  int64_t c = std::max<int64_t>(n, L > 0 ? b : 1);
  // first candidate of the form k*q + 1
  c = ((c - 1 + q - 1) / q) * q + 1;
  for (int iter = 0; iter < (1 << 22); ++iter, c += q) {
    bool ok = true;
    for (int s = 1; s <= L && ok; ++s) ok = ((c - 1) >> (s - 1)) >= (nested ? (b - 1) >> (s - 1) : b - 1);
    const int64_t nl = L > 0 ? ((c - 1) >> L) + 1 : c;
    if (ok && global_chain_ok(nl, M)) return c;
  }
  fail(BM_EINVAL, "no padded length satisfies the level schedule");
}

// ------------------------------------------------------------------ gains
// Per-axis row profile of a = P K (P: linear interpolation from the coarse
// nodes, K: correction operator of the level).  For every row i:
// sum_j |a_ij|, sum over coarse j of |a_ij|, a_ii, and whether i is coarse.
struct RowProf {
  double sall, sc, dg;
  int coarse;
};

// Solve T x = r in place for the tridiagonal T with constant off-diagonals
// `off` and diagonal `diag` (length k).
static void tridiag_solve(std::vector<double>& r, const std::vector<double>& diag, double off) {
  const size_t k = r.size();
  std::vector<double> cp(k);
  double den = diag[0];
  cp[0] = off / den;
  r[0] /= den;
  for (size_t i = 1; i < k; ++i) {
    den = diag[i] - off * cp[i - 1];
    cp[i] = off / den;
    r[i] = (r[i] - off * r[i - 1]) / den;
  }
  for (size_t i = k - 1; i-- > 0;) r[i] -= cp[i] * r[i + 1];
}

static std::vector<RowProf> axis_profile(int64_t n, bool face_fixed) {
  std::vector<RowProf> prof;
  if (n <= 2) {
    for (int64_t i = 0; i < n; ++i) prof.push_back({1.0, 1.0, 1.0, 1});
    return prof;
  }
  const int64_t m = (n + 1) / 2;
  // load-vector operator P^T M on a unit-spaced fine grid: interior coarse
  // row J weighs nodes 2J-2..2J+2 by 1/12, 1/2, 5/6, 1/2, 1/12; the end
  // rows keep the half of the stencil inside the grid (5/12 at the end node).
  auto rt = [&](int64_t J, int64_t i) -> double {
    const int64_t d = i - 2 * J;
    if (d < -2 || d > 2) return 0.0;
    static const double w[5] = {1.0 / 12, 0.5, 5.0 / 6, 0.5, 1.0 / 12};
    double v = w[d + 2];
    if ((J == 0 && d == 0) || (J == m - 1 && d == 0)) v = 5.0 / 12;
    return v;
  };
  // rows solved for and their coarse mass matrix (coarse spacing 2):
  // off-diagonal 1/3, diagonal 4/3 inside and 2/3 at a natural end.
  const int64_t r0 = face_fixed ? 1 : 0, r1 = face_fixed ? m - 1 : m;
  const int64_t k = r1 - r0;
  std::vector<double> diag(k);
  for (int64_t t = 0; t < k; ++t) {
    const int64_t J = r0 + t;
    diag[t] = (!face_fixed && (J == 0 || J == m - 1)) ? 2.0 / 3 : 4.0 / 3;
  }
  std::vector<double> K(size_t(m) * n, 0.0);  // K[J*n + i]
  std::vector<double> col(k);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t t = 0; t < k; ++t) col[t] = rt(r0 + t, i);
    tridiag_solve(col, diag, 1.0 / 3);
    for (int64_t t = 0; t < k; ++t) K[size_t(r0 + t) * n + i] = col[t];
  }
  prof.resize(n);
  std::vector<double> a(n);
  for (int64_t i = 0; i < n; ++i) {
    if ((i & 1) == 0) {
      for (int64_t j = 0; j < n; ++j) a[j] = K[size_t(i / 2) * n + j];
    } else {
      for (int64_t j = 0; j < n; ++j) a[j] = 0.5 * (K[size_t(i / 2) * n + j] + K[size_t(i / 2 + 1) * n + j]);
    }
    double sall = 0, sc = 0;
    for (int64_t j = 0; j < n; ++j) {
      sall += std::fabs(a[j]);
      if ((j & 1) == 0) sc += std::fabs(a[j]);
    }
    prof[i] = {sall, sc, a[i], (i & 1) == 0};
  }
  return prof;
}

static std::vector<RowProf> unique_profiles(std::vector<RowProf> p) {
  auto key = [](const RowProf& r) {
    auto q = [](double v) { return std::llround(v * 1e13); };
    return std::make_tuple(q(r.sall), q(r.sc), q(r.dg), r.coarse);
  };
  std::map<decltype(key(p[0])), RowProf> m;
  for (auto& r : p) m.emplace(key(r), r);
  std::vector<RowProf> out;
  for (auto& kv : m) out.push_back(kv.second);
  return out;
}

// Max over nodes x of sum over detail columns y of |delta_xy - prod a_d(x_d, y_d)|.
static double gain_from_profiles(const std::vector<RowProf> p[3]) {
  double best = 0;
  for (const auto& z : p[0])
    for (const auto& y : p[1])
      for (const auto& x : p[2]) {
        const double sall = z.sall * y.sall * x.sall;
        const double sc = z.sc * y.sc * x.sc;
        const double dg = z.dg * y.dg * x.dg;
        double v = sall - sc;
        if (!(z.coarse && y.coarse && x.coarse)) v += std::fabs(1.0 - dg) - std::fabs(dg);
        best = std::max(best, v);
      }
  return best;
}

// Round up to 4 decimals; the 1e-6 slack (in units of the last decimal)
// keeps exact 4-decimal gains from being pushed up by summation noise.
static double round_up4(double a) { return std::ceil(a * 10000.0 - 1e-6) / 10000.0; }

double level_gain_local(int b) {
  static std::mutex mu;
  static std::map<int, double> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(b);
  if (it != cache.end()) return it->second;
  std::vector<RowProf> p[3];
  p[0] = p[1] = p[2] = unique_profiles(axis_profile(b, true));
  const double v = round_up4(gain_from_profiles(p));
  cache[b] = v;
  return v;
}

double level_gain_global(const int64_t n[3]) {
  static std::mutex mu;
  static std::map<std::tuple<int64_t, int64_t, int64_t>, double> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_tuple(n[0], n[1], n[2]);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  std::vector<RowProf> p[3];
  for (int a = 0; a < 3; ++a) p[a] = unique_profiles(axis_profile(n[a], false));
  const double v = round_up4(gain_from_profiles(p));
  cache[key] = v;
  return v;
}

// Reciprocal pivots of Thomas elimination for 3*Mc with natural ends:
// tridiag(1, 4, 1) with end diagonals 2.  inv[J] = 1 / (diag_J - inv[J-1]).
void thomas_pivots_natural(int64_t m, std::vector<double>& inv) {
  inv.resize(m);
  for (int64_t J = 0; J < m; ++J) {
    const double diag = (J == 0 || J == m - 1) ? 2.0 : 4.0;
    inv[J] = 1.0 / (diag - (J ? inv[J - 1] : 0.0));
  }
}

// Share of the L-infinity budget per level (index s-1) and for the coarsest
// values (index L+M).  Sec. II-B: the share tightens as levels coarsen; here
// it is proportional to the number of coefficients a level holds (the split
// that minimises the total code length).  Sec. IV-C: the M global levels
// share their part equally.  The shares sum to 1.
std::vector<double> level_weights(const bm_plan_s& p) {
  if (p.w_override.size() == size_t(p.nlev + 1)) return p.w_override;
  auto prod = [](const int64_t* n) { return n[0] * n[1] * n[2]; };
  const double N = double(prod(p.pdims));
  std::vector<double> w(p.nlev + 1, 0.0);
  int64_t nglob = 0;
  for (int s = 1; s <= p.nlev; ++s) {
    const Level& L = p.lv[s - 1];
    const int64_t ns = prod(L.n) - prod(L.m);
    if (L.local)
      w[s - 1] = double(ns) / N;
    else
      nglob += ns;
  }
  for (int s = p.L + 1; s <= p.nlev; ++s) w[s - 1] = (double(nglob) / N) / double(p.M);
  w[p.nlev] = double(prod(p.lv[p.nlev - 1].m)) / N;
  // no share below 1/(64 T), T = L+M+1, so small deep levels keep codes in
  // 32 bits; then renormalise so the shares sum to 1
  const double floor_w = 1.0 / (64.0 * double(p.nlev + 1));
  double total = 0.0;
  for (auto& v : w) {
    v = v > floor_w ? v : floor_w;
    total += v;
  }
  for (auto& v : w) v = v / total;
  return w;
}

TimedScope::TimedScope(bm_plan_s& p_, int slot_, hipStream_t st_) : p(p_), slot(slot_), st(st_) {
  if (!p.timing.on) return;
  BM_HIP(hipEventCreate(&a));
  BM_HIP(hipEventCreate(&b));
  BM_HIP(hipEventRecord(a, st));
}

TimedScope::~TimedScope() {
  if (!a) return;
  (void)hipEventRecord(b, st);
  p.timing.pending.push_back({slot, a, b});
}

View3 level_view(const bm_plan_s& p, int s, void* coeff) {
  const Level& L = p.lv[s - 1];
  const int64_t P1 = p.pdims[1], P2 = p.pdims[2];
  return View3{coeff, {L.n[0], L.n[1], L.n[2]}, {L.ps[0] * P1 * P2, L.ps[1] * P2, L.ps[2]}};
}

View3 coarsest_view(const bm_plan_s& p, void* coeff) {
  const Level& L = p.lv[p.nlev - 1];
  int64_t ps[3];
  for (int a = 0; a < 3; ++a) ps[a] = L.coarsen[a] ? 2 * L.ps[a] : L.ps[a];
  const int64_t P1 = p.pdims[1], P2 = p.pdims[2];
  return View3{coeff, {L.m[0], L.m[1], L.m[2]}, {ps[0] * P1 * P2, ps[1] * P2, ps[2]}};
}

}  // namespace bm

using namespace bm;

static int64_t prod3(const int64_t n[3]) { return n[0] * n[1] * n[2]; }

bm_plan_s* bm_plan_build(const bm_config* c) {
  if (!c) fail(BM_EINVAL, "null config");
  if (c->ndim < 1 || c->ndim > 3) fail(BM_EINVAL, "ndim must be 1, 2 or 3");
  if (c->dtype != BM_F32 && c->dtype != BM_F64) fail(BM_EINVAL, "dtype must be BM_F32 or BM_F64");
  if (c->L < 0 || c->M < 0 || c->L + c->M < 1 || c->L + c->M > 24) fail(BM_EINVAL, "need 1 <= L+M <= 24");
  if (c->L > 0 && c->block != 9 && c->block != 17 && c->block != 33) fail(BM_EINVAL, "block must be 9, 17 or 33");
  if (c->pad_mode != 0 && c->pad_mode != 1) fail(BM_EINVAL, "pad_mode must be 0 (clamp) or 1 (zero)");
  if (!(c->eta >= 0.0 && c->eta < 0.5)) fail(BM_EINVAL, "eta must lie in [0, 0.5)");
  if (c->nested != 0 && c->nested != 1) fail(BM_EINVAL, "nested must be 0 or 1");
  // nested schedule: every block level keeps at least 9 nodes per side
  if (c->nested && c->L > 0 && ((c->block - 1) >> (c->L - 1)) < 8)
    fail(BM_EINVAL, "nested schedule: block level L would have fewer than 9 nodes per side");
  // ndim < 3: dims[0..ndim-1] become the trailing axes
  int64_t d[3] = {1, 1, 1};
  for (int a = 0; a < c->ndim; ++a) d[3 - c->ndim + a] = c->dims[a];
  for (int a = 0; a < 3; ++a)
    if (d[a] < 1 || d[a] > (int64_t(1) << 31)) fail(BM_EINVAL, "dims must lie in [1, 2^31]");
  {
    // element counts stay far from int64 overflow (each padded length is at
    // most about 2^31, so the product of two fits)
    int64_t pd[3];
    for (int a = 0; a < 3; ++a) pd[a] = padded_length(d[a], c->L > 0 ? c->block : 0, c->L, c->M, c->nested != 0);
    if (pd[1] * pd[2] > (int64_t(1) << 40) / pd[0]) fail(BM_EINVAL, "padded grid of more than 2^40 nodes");
    // the line solves of a global level take at most 64 kLineQ coarse nodes
    // per line, i.e. axes of at most 2 (64 kLineQ) - 1 = 1151 nodes
    for (int a = 0; a < 3; ++a) {
      int64_t n = pd[a];
      for (int s = 1; s <= c->L + c->M; ++s) {
        if (n <= 2) break;
        const int64_t m = (n + 1) / 2;
        if (s > c->L && m > 64 * kLineQ)
          fail(BM_EUNSUPPORTED, "global level " + std::to_string(s) + " has an axis of " + std::to_string(n) +
                                    " nodes; global levels take axes of at most " +
                                    std::to_string(2 * 64 * kLineQ - 1) + " nodes (add a block level)");
        n = m;
      }
    }
  }
  int dev = 0;
  BM_HIP(hipGetDevice(&dev));
  auto p = new bm_plan_s();
  p->cfg = *c;
  p->device = dev;
  p->esize = c->dtype == BM_F32 ? 4 : 8;
  for (int a = 0; a < 3; ++a) p->dims[a] = d[a];
  p->L = c->L;
  p->M = c->M;
  p->nlev = c->L + c->M;
  const int b = c->L > 0 ? c->block : 0;
  try {
    const bool nested = c->nested != 0;
    for (int a = 0; a < 3; ++a) p->pdims[a] = padded_length(d[a], b, c->L, c->M, nested);
    int64_t n[3] = {p->pdims[0], p->pdims[1], p->pdims[2]};
    int64_t ps[3] = {1, 1, 1};
    for (int s = 1; s <= p->nlev; ++s) {
      Level L{};
      L.local = s <= c->L;
      bool any = false;
      for (int a = 0; a < 3; ++a) {
        L.n[a] = n[a];
        L.ps[a] = ps[a];
        L.coarsen[a] = n[a] > 2;
        L.m[a] = n[a] > 2 ? (n[a] + 1) / 2 : n[a];
        any |= L.coarsen[a];
        if (L.local) {
          L.b = nested ? ((b - 1) >> (s - 1)) + 1 : b;
          L.nb[a] = (n[a] - 1) / (L.b - 1);
        }
      }
      if (!any) fail(BM_EINVAL, "level " + std::to_string(s) + " has no axis left to coarsen; lower M");
      if (L.local) {
        L.gain = level_gain_local(L.b);
      } else {
        L.gain = level_gain_global(L.n);
        for (int a = 0; a < 3; ++a) {
          L.d_inv[a] = nullptr;
          if (!L.coarsen[a]) continue;
          std::vector<double> inv;
          thomas_pivots_natural(L.m[a], inv);
          plan_alloc(*p, &L.d_inv[a], inv.size() * sizeof(double));
          BM_HIP(hipMemcpy(L.d_inv[a], inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice));
        }
      }
      p->lv.push_back(L);
      for (int a = 0; a < 3; ++a) {
        if (L.coarsen[a]) ps[a] *= 2;
        n[a] = L.m[a];
      }
    }
    for (int a = 0; a < 3; ++a) p->nb1[a] = c->L > 0 ? p->lv[0].nb[a] : 1;
    const int bL = c->L > 0 ? p->lv[c->L - 1].b : 0;   // block size of the last block level
    p->fuse_next = c->L > 0 && c->M > 0 && bL != 33;
    {
      const char* e = std::getenv("BM_PLANE_PASS");
      p->plane_pass = !(e && e[0] == '0' && e[1] == '\0');
    }
    if (p->fuse_next) {
      // per-block partial load vectors of the first global level (FP64): H^3 per block, H = (b+3)/4
      const int64_t h = (bL + 3) / 4;
      plan_alloc(*p, &p->ws.part, size_t(prod3(p->lv[c->L - 1].nb)) * h * h * h * sizeof(double));
    }
    // workspace
    p->ws.grid.assign(p->nlev + 1, nullptr);
    if (c->L == 0) plan_alloc(*p, &p->ws.grid[0], size_t(prod3(p->pdims)) * p->esize);
    for (int s = 1; s <= p->nlev; ++s)
      plan_alloc(*p, &p->ws.grid[s], size_t(prod3(p->lv[s - 1].m)) * p->esize);
    size_t t = 0;
    for (auto& L : p->lv) {
      if (L.local) {
        if (L.b == 33) t = std::max(t, wide_scratch_elems(L.nb));   // y-pass result of the 33^3 blocks
        continue;
      }
      t = std::max<size_t>(t, size_t(L.n[0]) * L.n[1] * L.m[2]);
      t = std::max<size_t>(t, size_t(L.n[0]) * L.m[1] * L.m[2]);
    }
    p->ws.t_elems = t;
    if (t) {
      plan_alloc(*p, &p->ws.t1, t * p->esize);
      plan_alloc(*p, &p->ws.t2, t * p->esize);
    }
    int64_t tot = 0;
    p->ws.tol_off.assign(p->nlev + 2, 0);
    for (int s = 1; s <= c->L; ++s) {
      p->ws.tol_off[s] = tot;
      tot += prod3(p->lv[s - 1].nb);
    }
    p->ws.tol_off[c->L + 1] = tot;
    const int64_t nlastb = c->L > 0 ? prod3(p->lv[c->L - 1].nb) : 0;
    // propagated taus, Delta, 1/Delta per block; tau_global; coarsest-value
    // Delta and 1/Delta; then the 27-class Delta and 1/Delta tables
    plan_alloc(*p, &p->ws.tolbuf, size_t(3 * tot + 8 + 2 * nlastb + 8 + 54 * (tot + nlastb)) * sizeof(double));
    plan_alloc(*p, &p->ws.boxbuf, size_t(kMaxBoxes) * 7 * sizeof(double));
    BM_HIP(hipHostMalloc(&p->ws.boxhost, size_t(kMaxBoxes) * 7 * sizeof(double), hipHostMallocDefault));
    plan_alloc(*p, &p->ws.qparam, size_t(4 * (p->nlev + 2)) * sizeof(double));
    // 16 counters, then per-workgroup partial statistics of the quantizer (3 x 8192)
    plan_alloc(*p, &p->ws.counters, (16 + 3 * 8192) * sizeof(int64_t));
  } catch (...) {
    // release what was allocated, then rethrow
    for (auto& L : p->lv)
      for (int a = 0; a < 3; ++a)
        if (!L.local && L.d_inv[a]) (void)hipFree(L.d_inv[a]);
    for (void* g : p->ws.grid)
      if (g) (void)hipFree(g);
    if (p->ws.t1) (void)hipFree(p->ws.t1);
    if (p->ws.t2) (void)hipFree(p->ws.t2);
    if (p->ws.tolbuf) (void)hipFree(p->ws.tolbuf);
    if (p->ws.qparam) (void)hipFree(p->ws.qparam);
    if (p->ws.counters) (void)hipFree(p->ws.counters);
    if (p->ws.boxbuf) (void)hipFree(p->ws.boxbuf);
    if (p->ws.boxhost) (void)hipHostFree(p->ws.boxhost);
    if (p->ws.part) (void)hipFree(p->ws.part);
    delete p;
    throw;
  }
  return p;
}

void bm_plan_free(bm_plan_s* p) {
  if (!p) return;
  for (auto& e : p->timing.pending) {
    (void)hipEventSynchronize(e.b);
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto& L : p->lv)
    for (int a = 0; a < 3; ++a)
      if (!L.local && L.d_inv[a]) (void)hipFree(L.d_inv[a]);
  for (void* g : p->ws.grid)
    if (g) (void)hipFree(g);
  for (void* q : {p->ws.t1, p->ws.t2, p->ws.codes, p->ws.coeff, (void*)p->ws.tolbuf, (void*)p->ws.qparam,
                  (void*)p->ws.counters, (void*)p->ws.boxbuf, p->ws.gpad, p->ws.prep_dev, p->ws.part})
    if (q) (void)hipFree(q);
  if (p->ws.boxhost) (void)hipHostFree(p->ws.boxhost);
  delete p;
}
