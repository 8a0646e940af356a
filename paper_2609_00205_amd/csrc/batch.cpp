// Many independent fields of one dtype and block size, in few launches.
//
// The fused pipeline of every field (decompose + ROI quantize, or dequantize
// + recompose) is issued as: one launch per stage of the quantizer-table
// preparation for all fields, one persistent launch per block level
// covering the blocks of every field that has that level (a 33-node level:
// one per step of the split block, over halves or blocks; the nested
// schedule: one for the 17/9 pairs), and the (small) global levels of each
// field.  The whole sequence can be captured once in
// a HIP graph and replayed while the bound buffers stay the same.
//
// Per-field kernel arguments and task lists are built on the host and
// uploaded into a device arena when the binding (the set of buffer
// pointers) changes; capture and replay never copy from the host.

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

bm_plan_s* bm_plan_build(const bm_config* c);
void bm_plan_free(bm_plan_s* p);

namespace bm {
namespace {

constexpr int kMaxLev = 9;

// one bound direction (decompose+quantize or dequantize+recompose)
struct Bound {
  std::vector<const void*> key;   // bound pointers, in order
  std::vector<QPrep> q;
  PrepStages stages;
  const PrepField* fields = nullptr;
  const void* args[kMaxLev] = {};  // per block level: packed kernel arguments
  const int64_t* first[kMaxLev] = {};
  int nf[kMaxLev] = {};
  int64_t ntasks[kMaxLev] = {};
  int blk[kMaxLev] = {};           // block size of the level's launch
  // 33-node levels: tasks are block halves (first[]) and blocks (firstb[])
  const int64_t* firstb[kMaxLev] = {};
  int64_t nblk[kMaxLev] = {};
  // nested schedule: the fields whose levels 1 and 2 run as one pair
  const void* nargs1 = nullptr;
  const void* nargs2 = nullptr;
  const int64_t* nfirst = nullptr;
  int nnf = 0;
  int64_t nntasks = 0;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  hipGraphExec_t graph = nullptr;
  std::vector<const void*> x, tol, codes;   // as bound
};

void free_bound(Bound& b) {
  if (b.graph) (void)hipGraphExecDestroy(b.graph);
  if (b.arena) (void)hipFree(b.arena);
  b = Bound{};
}

// host image of the arena, assembled with 16-byte alignment
struct Image {
  std::vector<uint8_t> bytes;
  size_t put(const void* p, size_t n) {
    const size_t off = (bytes.size() + 15) & ~size_t(15);
    bytes.resize(off + n);
    if (n) std::memcpy(bytes.data() + off, p, n);
    return off;
  }
};

}  // namespace
}  // namespace bm

struct bm_batch_s {
  std::vector<bm_plan_s*> plans;
  int block = 0, dtype = 0, Lmax = 0, device = 0, nested = 0;
  bm::Bound dq, rq;
};

namespace bm {
namespace {

int64_t prod(const int64_t n[3]) { return n[0] * n[1] * n[2]; }

// Builds (or reuses) the binding of one direction: quantizer layout per
// field, prep task lists, per-level kernel arguments, uploaded to the arena.
void bind(bm_batch_s& b, Bound& B, bool dec, const void* const* x, const double* const* tol, int32_t* const* codes,
          hipStream_t st) {
  const int nf = int(b.plans.size());
  std::vector<const void*> key;
  key.reserve(3 * nf);
  for (int f = 0; f < nf; ++f) {
    key.push_back(x[f]);
    key.push_back(tol[f]);
    key.push_back(codes[f]);
  }
  if (key == B.key && B.arena) return;
  free_bound(B);
  B.key = key;
  Image im;
  // quantizer tables
  B.q.resize(nf);
  std::vector<PrepField> pf(nf);
  for (int f = 0; f < nf; ++f) {
    B.q[f] = qprep_layout(*b.plans[f], tol[f]);
    pf[f] = prep_field(*b.plans[f], tol[f], B.q[f]);
  }
  const size_t off_fields = im.put(pf.data(), pf.size() * sizeof(PrepField));
  size_t off_prop[kMaxLev] = {}, off_tab[kMaxLev] = {};
  for (int s = 0; s < kMaxLev; ++s) {
    std::vector<int64_t> fp(nf + 1, 0), ft(nf + 1, 0);
    for (int f = 0; f < nf; ++f) {
      const bm_plan_s& p = *b.plans[f];
      const int64_t np = (s >= 1 && p.L > s) ? prod(p.lv[s].nb) : 0;                        // into level s+1
      const int64_t nt = s >= 1 ? (p.L >= s ? 27 * prod(p.lv[s - 1].nb) : 0)
                                : ((p.L > 0 && p.M == 0) ? 27 * prod(p.lv[p.L - 1].nb) : 0);  // coarsest values
      fp[f + 1] = fp[f] + np;
      ft[f + 1] = ft[f] + nt;
    }
    B.stages.prop_n[s] = fp[nf];
    B.stages.tab_n[s] = ft[nf];
    off_prop[s] = im.put(fp.data(), fp.size() * sizeof(int64_t));
    off_tab[s] = im.put(ft.data(), ft.size() * sizeof(int64_t));
  }
  // block levels: arguments of the fields that have level s, in field order
  // (a field whose levels 1 and 2 form a nested pair is in neither list: it
  // takes the pair launch below)
  size_t off_args[kMaxLev] = {}, off_first[kMaxLev] = {}, off_firstb[kMaxLev] = {};
  for (int s = 1; s <= b.Lmax; ++s) {
    std::vector<uint8_t> args;
    std::vector<int64_t> first(1, 0), firstb(1, 0);
    B.blk[s] = 0;
    for (int f = 0; f < nf; ++f) {
      bm_plan_s& p = *b.plans[f];
      if (p.L < s) continue;
      if (s <= 2 && nest_pair(p, 1)) continue;
      if (!B.blk[s]) B.blk[s] = p.lv[s - 1].b;
      if (p.lv[s - 1].b != B.blk[s]) fail(BM_EUNSUPPORTED, "fields of one batched level use one block size");
      if (B.blk[s] == 33) {
        // a 33-node level: column and coarse steps (and interpolation) over halves and blocks
        const size_t sz = wide_args_size(p);
        args.resize(args.size() + sz);
        uint8_t* dst = args.data() + args.size() - sz;
        const View3 src =
            dec ? (s == 1 ? dense_view(const_cast<void*>(x[f]), p.dims) : dense_view(p.ws.grid[s - 1], p.lv[s - 1].n))
                : View3{};
        void* out = s == 1 ? const_cast<void*>(x[f]) : p.ws.grid[s - 1];
        wide_batch_args(p, s, dec, src, s == 1, out, codes[f], &B.q[f], dst);
        const int64_t nb = p.lv[s - 1].nb[0] * p.lv[s - 1].nb[1] * p.lv[s - 1].nb[2];
        first.push_back(first.back() + 2 * nb);
        firstb.push_back(firstb.back() + nb);
        continue;
      }
      const size_t sz = block_args_size(p, dec);
      args.resize(args.size() + sz);
      uint8_t* dst = args.data() + args.size() - sz;
      if (dec) {
        const View3 src = s == 1 ? dense_view(const_cast<void*>(x[f]), p.dims) : dense_view(p.ws.grid[s - 1], p.lv[s - 1].n);
        block_dec_args(p, s, src, s == 1, nullptr, p.ws.grid[s], codes[f], &B.q[f], dst);
      } else {
        void* out = s == 1 ? const_cast<void*>(x[f]) : p.ws.grid[s - 1];
        block_rec_args(p, s, nullptr, p.ws.grid[s], out, s == 1, codes[f], &B.q[f], dst);
      }
      first.push_back(first.back() + block_groups(p, s, dec));
    }
    B.nf[s] = int(first.size()) - 1;
    B.ntasks[s] = first.back();
    B.nblk[s] = firstb.back();
    off_args[s] = im.put(args.data(), args.size());
    off_first[s] = im.put(first.data(), first.size() * sizeof(int64_t));
    off_firstb[s] = im.put(firstb.data(), firstb.size() * sizeof(int64_t));
  }
  // nested pairs: level 1's and level 2's arguments side by side
  size_t off_n1 = 0, off_n2 = 0, off_nfirst = 0;
  {
    std::vector<uint8_t> a1, a2;
    std::vector<int64_t> first(1, 0);
    for (int f = 0; f < nf; ++f) {
      bm_plan_s& p = *b.plans[f];
      if (!nest_pair(p, 1)) continue;
      const size_t sz = block_args_size(p, dec);
      a1.resize(a1.size() + sz);
      a2.resize(a2.size() + sz);
      const View3 src = dense_view(const_cast<void*>(x[f]), p.dims);
      block_nest_args(p, dec, src, const_cast<void*>(x[f]), codes[f], &B.q[f], a1.data() + a1.size() - sz,
                      a2.data() + a2.size() - sz);
      first.push_back(first.back() + block_groups(p, 1, dec));
    }
    B.nnf = int(first.size()) - 1;
    B.nntasks = first.back();
    off_n1 = im.put(a1.data(), a1.size());
    off_n2 = im.put(a2.data(), a2.size());
    off_nfirst = im.put(first.data(), first.size() * sizeof(int64_t));
  }
  B.arena_bytes = im.bytes.size();
  BM_HIP(hipMalloc(&B.arena, B.arena_bytes));
  BM_HIP(hipMemcpyAsync(B.arena, im.bytes.data(), B.arena_bytes, hipMemcpyHostToDevice, st));
  BM_HIP(hipStreamSynchronize(st));
  auto at = [&](size_t off) { return static_cast<const void*>(static_cast<const uint8_t*>(B.arena) + off); };
  B.fields = static_cast<const PrepField*>(at(off_fields));
  for (int s = 0; s < kMaxLev; ++s) {
    B.stages.prop_first[s] = static_cast<const int64_t*>(at(off_prop[s]));
    B.stages.tab_first[s] = static_cast<const int64_t*>(at(off_tab[s]));
  }
  for (int s = 1; s <= b.Lmax; ++s) {
    B.args[s] = at(off_args[s]);
    B.first[s] = static_cast<const int64_t*>(at(off_first[s]));
    B.firstb[s] = static_cast<const int64_t*>(at(off_firstb[s]));
  }
  B.nargs1 = at(off_n1);
  B.nargs2 = at(off_n2);
  B.nfirst = static_cast<const int64_t*>(at(off_nfirst));
  B.x.assign(x, x + nf);
  B.tol.assign(tol, tol + nf);
  B.codes.assign(codes, codes + nf);
}

void level_launch(const bm_batch_s& b, const Bound& B, int s, bool dec, hipStream_t st) {
  if (B.ntasks[s] <= 0) return;
  if (B.blk[s] == 33)
    launch_wide_batch(b.dtype, dec, B.args[s], B.first[s], B.firstb[s], B.nf[s], B.ntasks[s], B.nblk[s], st);
  else
    launch_block_batch(B.blk[s], b.dtype, dec, true, B.args[s], B.first[s], B.nf[s], B.ntasks[s], st);
}

void enqueue(bm_batch_s& b, Bound& B, bool dec, hipStream_t st) {
  const int nf = int(b.plans.size());
  launch_prep_batch(B.stages, B.fields, nf, st);
  if (dec) {
    for (int s = 1; s <= b.Lmax; ++s) {
      if (s == 1) launch_block_batch_nest(b.dtype, true, B.nargs1, B.nargs2, B.nfirst, B.nnf, B.nntasks, st);
      level_launch(b, B, s, true, st);
    }
    for (int f = 0; f < nf; ++f)
      decompose_quantize_global(*b.plans[f], B.x[f], static_cast<int32_t*>(const_cast<void*>(B.codes[f])), B.q[f], st);
  } else {
    for (int f = 0; f < nf; ++f)
      dequantize_recompose_global(*b.plans[f], static_cast<const int32_t*>(B.codes[f]), B.q[f],
                                  const_cast<void*>(B.x[f]), st);
    for (int s = b.Lmax; s >= 1; --s) {
      level_launch(b, B, s, false, st);
      if (s == 1) launch_block_batch_nest(b.dtype, false, B.nargs1, B.nargs2, B.nfirst, B.nnf, B.nntasks, st);
    }
  }
}

void run(bm_batch_s& b, Bound& B, bool dec, bool graph, hipStream_t st) {
  if (graph && st == nullptr) fail(BM_EINVAL, "graph capture needs a stream other than the null stream");
  if (!graph) {
    enqueue(b, B, dec, st);
    return;
  }
  if (!B.graph) {
    hipGraph_t g = nullptr;
    BM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    try {
      enqueue(b, B, dec, st);
    } catch (...) {
      (void)hipStreamEndCapture(st, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    BM_HIP(hipStreamEndCapture(st, &g));
    const hipError_t e = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    BM_HIP(e);
  }
  BM_HIP(hipGraphLaunch(B.graph, st));
}

}  // namespace

bm_batch_s* batch_build(int nfields, const bm_config* cfgs) {
  if (nfields <= 0 || !cfgs) fail(BM_EINVAL, "empty batch");
  auto* b = new bm_batch_s();
  try {
    BM_HIP(hipGetDevice(&b->device));
    for (int f = 0; f < nfields; ++f) {
      if (f > 0 && (cfgs[f].dtype != cfgs[0].dtype || cfgs[f].block != cfgs[0].block))
        fail(BM_EINVAL, "all fields of a batch share dtype and block size");
      if (f > 0 && cfgs[f].nested != cfgs[0].nested) fail(BM_EINVAL, "all fields of a batch share the block schedule");
      bm_config c = cfgs[f];
      if (c.nested && c.block != 17)
        fail(BM_EUNSUPPORTED, "batched nested schedule: b = 17 (17- then 9-node blocks)");
      if (c.L == -1 && c.nested) {
        // nested: level 2 tiles wherever level 1 does (9-node blocks inside the
        // 17-node regions); both levels when the dims tile without padding
        int64_t d[3] = {1, 1, 1};
        if (c.ndim < 1 || c.ndim > 3) fail(BM_EINVAL, "ndim must be 1, 2 or 3");
        for (int a = 0; a < c.ndim; ++a) d[3 - c.ndim + a] = c.dims[a];
        bool tiles = true;
        for (int a = 0; a < 3; ++a) tiles = tiles && d[a] >= 17 && (d[a] - 1) % 16 == 0;
        c.L = tiles ? 2 : 1;
      } else if (c.L == -1) {
        // the most block levels the logical dims tile without padding (at least 1)
        if (c.block != 9 && c.block != 17 && c.block != 33) fail(BM_EINVAL, "L = -1 needs block 9, 17 or 33");
        int64_t d[3] = {1, 1, 1};
        if (c.ndim < 1 || c.ndim > 3) fail(BM_EINVAL, "ndim must be 1, 2 or 3");
        for (int a = 0; a < c.ndim; ++a) d[3 - c.ndim + a] = c.dims[a];
        const int64_t q = c.block - 1;
        c.L = 1;
        auto tiles = [&](int L) {
          for (int a = 0; a < 3; ++a)
            if (((d[a] - 1) >> L) < q || (d[a] - 1) % (q << L) != 0) return false;
          return true;
        };
        while (c.L < 24 && tiles(c.L)) ++c.L;
      }
      b->plans.push_back(bm_plan_build(&c));
      b->Lmax = std::max(b->Lmax, b->plans.back()->L);
    }
    b->block = cfgs[0].block;
    b->dtype = cfgs[0].dtype;
    b->nested = cfgs[0].nested;
    if (b->Lmax >= kMaxLev) fail(BM_EUNSUPPORTED, "too many block levels");
  } catch (...) {
    for (auto* p : b->plans) bm_plan_free(p);
    delete b;
    throw;
  }
  return b;
}

void batch_free(bm_batch_s* b) {
  if (!b) return;
  free_bound(b->dq);
  free_bound(b->rq);
  for (auto* p : b->plans) bm_plan_free(p);
  delete b;
}

int batch_size(const bm_batch_s& b) { return int(b.plans.size()); }

bm_plan_s* batch_plan(bm_batch_s& b, int field) { return b.plans[field]; }

void batch_decompose_quantize(bm_batch_s& b, const void* const* x, const double* const* tol, int32_t* const* codes,
                              bool graph, hipStream_t st) {
  bind(b, b.dq, true, x, tol, codes, st);
  run(b, b.dq, true, graph, st);
}

void batch_dequantize_recompose(bm_batch_s& b, const int32_t* const* codes, const double* const* tol, void* const* x,
                                bool graph, hipStream_t st) {
  std::vector<const void*> xs(x, x + b.plans.size());
  bind(b, b.rq, false, xs.data(), tol, const_cast<int32_t* const*>(codes), st);
  run(b, b.rq, false, graph, st);
}

int batch_overflows(bm_batch_s& b, std::vector<int>& bad, hipStream_t st) {
  const int nf = int(b.plans.size());
  std::vector<int64_t> flags(nf, 0);
  for (int f = 0; f < nf; ++f)
    BM_HIP(hipMemcpyAsync(&flags[f], b.plans[f]->ws.counters + 2, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  bad.assign(nf, 0);
  int n = 0;
  for (int f = 0; f < nf; ++f)
    if (flags[f] & kFlagNonFinite) fail(BM_ENONFINITE, "field " + std::to_string(f) + ": NaN or Inf in the data");
  for (int f = 0; f < nf; ++f)
    if (flags[f]) {
      bad[f] = 1;
      ++n;
    }
  return n;
}

}  // namespace bm
