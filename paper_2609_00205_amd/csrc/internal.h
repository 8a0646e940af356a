// Internal declarations of the BlockMGARD library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "blockmgard.h"

namespace bm {

constexpr int kMaxBoxes = 4096;

// ---------------------------------------------------------------- errors
struct Error {
  bm_status code;
  std::string msg;
};

[[noreturn]] void fail(bm_status code, const std::string& msg);
void check_hip(hipError_t e, const char* what);

#define BM_HIP(call) ::bm::check_hip((call), #call)

// Unsigned 32-bit division by a run-time constant d >= 1 with a multiply-high
// and a shift (Granlund-Montgomery round-up method): valid for all n < 2^32.
struct FastDiv {
  uint32_t d = 1, m = 0, s = 0;
  FastDiv() = default;
  explicit FastDiv(uint32_t dv) : d(dv) {
    s = 0;
    while ((uint64_t(1) << s) < d) ++s;
    m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1);
  }
  __device__ inline uint32_t div(uint32_t n) const {
    const uint32_t t = __umulhi(n, m);
    return uint32_t((uint64_t(t) + n) >> s);
  }
};

// (z, y, x) of a flat index into dims (n0, n1, n2) with fewer than 2^32 entries.
struct Unflat32 {
  FastDiv d2, d1;
  uint32_t n1 = 1, n2 = 1;
  Unflat32() = default;
  Unflat32(int64_t n1_, int64_t n2_) : d2(uint32_t(n2_)), d1(uint32_t(n1_)), n1(uint32_t(n1_)), n2(uint32_t(n2_)) {}
  __device__ inline void operator()(uint32_t i, uint32_t& z, uint32_t& y, uint32_t& x) const {
    const uint32_t t = d2.div(i);
    x = i - t * n2;
    z = d1.div(t);
    y = t - z * n1;
  }
};

// Product rounded on its own (never contracted into a neighbouring add), so
// a dequantized value q * Delta is the same number whether it is stored to
// memory or consumed in registers.
__device__ inline double mul_rn(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}

// Multilinear interpolant at offset (dz, dy, dx) in {0,1}^3 of a cell of a
// level's coarse grid: rd(az, ay, ax) reads corner (az, ay, ax), and only
// az <= dz, ay <= dy, ax <= dx are read.  The 8-term sum in this fixed order
// (pairs along x, then y, then z) is used wherever a level's details or its
// inverse are formed, so every kernel produces the same bits.
template <typename T, typename F>
__device__ inline T cell_mean(int dz, int dy, int dx, F rd) {
  const T s = ((rd(0, 0, 0) + rd(0, 0, dx)) + (rd(0, dy, 0) + rd(0, dy, dx))) +
              ((rd(dz, 0, 0) + rd(dz, 0, dx)) + (rd(dz, dy, 0) + rd(dz, dy, dx)));
  return s * T(0.125);
}

// Bits of a quantizer's error flag: a code beyond int32 (tolerance too small
// for the data), and a NaN or infinite coefficient (non-finite data: a NaN or
// Inf input reaches the coefficient of its own node at some level).
constexpr unsigned kFlagRange = 1u, kFlagNonFinite = 2u;
__device__ inline unsigned code_flag(double c) { return isfinite(c) ? kFlagRange : kFlagNonFinite; }

// Persistent launches over many fields: task k belongs to field f with
// first[f] <= k < first[f+1] (first[] ascending, first[nf] = total).
__device__ inline int task_field(const int64_t* first, int nf, int64_t k) {
  int lo = 0, hi = nf;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= k)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}
// Host side: BM_ENONFINITE or BM_ERANGE for a non-zero flag word.
void check_code_flag(int64_t f, const char* what);

__host__ __device__ inline int64_t i64min(int64_t a, int64_t b) { return a < b ? a : b; }
__host__ __device__ inline int64_t i64max(int64_t a, int64_t b) { return a > b ? a : b; }

// ---------------------------------------------------------------- views
// A 3D strided view of device memory: element (z, y, x) lives at
// ptr + z*s[0] + y*s[1] + x*s[2] (strides in elements).
struct View3 {
  void* ptr;
  int64_t n[3];
  int64_t s[3];
};

inline View3 dense_view(void* p, const int64_t n[3]) {
  return View3{p, {n[0], n[1], n[2]}, {n[1] * n[2], n[2], 1}};
}

// ---------------------------------------------------------------- levels
// Level s (1-based) maps the grid G^{s-1} (dims n) to details on its
// fine-only nodes plus the coarse grid G^s (dims m).
struct Level {
  bool local;          // In-cache Block level (face-fixed blocks) or global
  int64_t n[3];        // dims of G^{s-1}
  int64_t m[3];        // dims of G^s
  int64_t nb[3];       // blocks per axis (local levels)
  int b;               // nodes per block side (local levels)
  int64_t ps[3];       // spacing of G^{s-1} nodes in the padded grid, per axis
  bool coarsen[3];     // axis is halved at this level (false: length <= 2 stays)
  double gain;         // rounded-up L-inf gain of this level's details
  double* d_inv[3];    // device: Thomas reciprocal pivots of the coarse mass matrix (global levels)
};

// Device workspace sizes and buffers owned by a plan.
struct Workspace {
  std::vector<void*> grid;       // grid[s] = compact G^s, s = 1..L+M (grid[0] unused)
  void* t1 = nullptr;            // global-level pass temporaries
  void* t2 = nullptr;
  size_t t_elems = 0;
  void* codes = nullptr;         // int32, padded grid (compress path)
  void* coeff = nullptr;         // dtype, padded grid (bm_qoi_deltas: the adjoint of the quantity)
  double* tolbuf = nullptr;      // propagated block tolerances, all local levels
  double* qparam = nullptr;      // per-level quantizer parameters (device)
  std::vector<int64_t> tol_off;  // offset of level-s block map in tolbuf
  int64_t* counters = nullptr;   // device scratch counters (stats)
  double* boxbuf = nullptr;      // device copy of an ROI box list (kMaxBoxes x 7)
  double* boxhost = nullptr;     // pinned staging for the box list
  void* gpad = nullptr;          // dtype, padded grid: level-1 gradient before the pad transpose
  void* prep_dev = nullptr;      // quantizer preparation of this plan: field record + task prefixes (device)
  void* part = nullptr;          // double: per-block partial load vectors of the first global level (fused)
  std::vector<uint8_t> prep_key; // field record last uploaded
  const double* kept_tol = nullptr;  // map whose tables are kept (bm_quant_prepare); null: none
};

}  // namespace bm

namespace bm {
// Optional per-level event timing (bm_timing): pending event pairs per slot.
struct Timing {
  bool on = false;
  struct Pending {
    int slot;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<double> ms;
  std::vector<int64_t> calls;
};
// a compress call planned but not written (bm_compress_plan)
struct PendingContainer;

}  // namespace bm

struct bm_plan_s {
  bm::Timing timing;
  bm_config cfg;
  int device;
  size_t esize;                  // bytes per element of dtype
  int64_t dims[3];               // logical
  int64_t pdims[3];              // padded
  int L, M, nlev;
  std::vector<bm::Level> lv;     // lv[0] is level 1
  bm::Workspace ws;
  int64_t nb1[3];                // level-1 block grid (1,1,1 when L == 0)
  // the last block level also forms the details of the first global level
  // (decomposition) and its interpolation (recomposition): a global cell of
  // that level never crosses a block face (b = 9, 17 with M >= 1)
  bool fuse_next = false;
  // global levels may run K along x and y as one plane pass (cleared by
  // BM_PLANE_PASS=0 at plan creation: line passes only, same results)
  bool plane_pass = true;
  std::shared_ptr<bm::PendingContainer> pending;   // dropped by every compress call on the plan
  // budget shares (levels 1..L+M, coarsest) set by an owner that spreads one
  // budget over more levels than the plan's (the 8^3 form's hybrid); empty:
  // the plan's own rule
  std::vector<double> w_override;
  size_t dev_bytes = 0;          // device memory the plan holds (bm_workspace_size)
};

namespace bm {

// Device memory owned by a plan, counted for bm_workspace_size.
template <typename P>
void plan_alloc(bm_plan_s& p, P** ptr, size_t bytes) {
  BM_HIP(hipMalloc(reinterpret_cast<void**>(ptr), bytes));
  p.dev_bytes += bytes;
}

// Workgroups of a persistent launch over ntasks tasks: as many as stay
// resident on the device (at least 1, at most ntasks).
template <typename K>
unsigned resident_grid(K kernel, int nt, int64_t ntasks) {
  int dev = 0, per_cu = 0, cus = 0;
  BM_HIP(hipGetDevice(&dev));
  BM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0));
  BM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t g = per_cu * int64_t(cus) > 1 ? per_cu * int64_t(cus) : 1;
  return unsigned(g < ntasks ? g : ntasks);
}

int64_t padded_length(int64_t n, int b, int L, int M, bool nested = false);
double level_gain_local(int b);
double level_gain_global(const int64_t n[3]);
void thomas_pivots_natural(int64_t m, std::vector<double>& inv);
std::vector<double> level_weights(const bm_plan_s& p);

// ---- kernels (launchers, stream-ordered) ----
void local_decompose(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff,
                     void* coarse_out, hipStream_t st);
void local_recompose(const bm_plan_s& p, int s, const void* coeff, const void* coarse_in, void* out,
                     bool last, hipStream_t st);

// block levels with b = 33 (local_decompose / local_recompose and their
// quantized forms dispatch here): scratch values the plan keeps in ws.t1 for
// a level of nb blocks; the recomposition turns the compact coarse grid cin
// into u_C in place
struct QPrep;
size_t wide_scratch_elems(const int64_t nb[3]);
void wide_decompose(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout, int32_t* codes,
                    const QPrep* q, hipStream_t st);
void wide_recompose(const bm_plan_s& p, int s, const void* coeff, void* cin, void* out, bool last,
                    const int32_t* codes, const QPrep* q, hipStream_t st);

// global level pieces
void global_details(const bm_plan_s& p, int s, const void* u, void* coeff, hipStream_t st);
void global_interp_add(const bm_plan_s& p, int s, const void* coeff, const void* uc, void* out,
                       hipStream_t st);
// restriction + tridiagonal solve along one axis (0=z,1=y,2=x) of a view;
// mask: zero the coarse nodes of the level on load; base != null: out = base - result
void line_pass(const bm_plan_s& p, int s, int axis, const View3& in, const int64_t cmask[3], void* out,
               const void* base, hipStream_t st);
void strided_copy(size_t esize, const View3& src, const View3& dst, hipStream_t st);
// logical input -> padded grid (clamp, or zero fill when zero is set)
void pad_input(const bm_plan_s& p, const void* x, void* dst, bool zero, hipStream_t st);
// The level-1 grid of a plan without block levels (padded dims, C order), or
// null.  Passed as the input of decompose / decompose_quantize, its logical
// region is taken in place (only the extension is filled); passed as the
// output of recompose / dequantize_recompose, the result is left there at the
// padded strides (no cropping copy).
void* level1_grid(const bm_plan_s& p);

// decompose / recompose drivers
void decompose(bm_plan_s& p, const void* x, void* coeff, hipStream_t st);
void recompose(bm_plan_s& p, const void* coeff, void* x, hipStream_t st);
// transposes: gx = D^T gcoeff, gcoeff = R^T gx
void decompose_adjoint(bm_plan_s& p, const void* gcoeff, void* gx, hipStream_t st);
void recompose_adjoint(bm_plan_s& p, const void* gx, void* gcoeff, hipStream_t st);

// quantization tables on the device, built from a level-1 block map:
// per local level s (slot s-1) the per-block Delta and 1/Delta; slot 8 for
// the coarsest values when M == 0 (level-L blocks); scalar Delta / 1/Delta
// per global level (q[2(s-1)], q[2(s-1)+1]) and for the coarsest values
// (q[2(L+M)], q[2(L+M)+1]).
struct QTab {
  const double* del = nullptr;
  const double* inv = nullptr;
  // per block, per class of node position (first face / interior / last face
  // along z, y, x: 27 classes, index 9 cz + 3 cy + cx) the smallest Delta and
  // the largest 1/Delta over the blocks that contain such a node
  const double* cdel = nullptr;
  const double* cinv = nullptr;
  int64_t nb[3] = {1, 1, 1};
};
struct QPrep {
  QTab lv[9];
  const double* q = nullptr;
  int64_t* flag = nullptr;      // set to 1 when a code does not fit in int32
};
constexpr int kCoarseSlotHost = 8;
// where a plan's quantizer tables live (host arithmetic, no launches)
QPrep qprep_layout(bm_plan_s& p, const double* block_tol);
// builds the tables on the device (stream-ordered) and returns their layout;
// with the kept map (quant_keep) only the overflow flag is cleared, and not
// even that for the dequantizing callers (clear_flag false: they set no flag)
QPrep quant_prepare(bm_plan_s& p, const double* block_tol, hipStream_t st, bool clear_flag = true);
// builds the tables of block_tol and keeps them (null: drops the kept ones)
void quant_keep(bm_plan_s& p, const double* block_tol, hipStream_t st);

// The same preparation for many fields at once: one field's inputs...
struct PrepField {
  const double* tau[9];       // block taus of local level s at [s-1] (level 1: the caller's map)
  int64_t nb[9][3];           // blocks per axis of local level s at [s-1]
  double kap[9];              // kappa of local level s at [s-1]
  double kapc;                // kappa of the coarsest values (M == 0)
  QTab tab[9];                // output tables (layout of qprep_layout); [8]: coarsest values
  double* tg;                 // tau_global
  double* q;                  // scalar Delta, 1/Delta per level and for the coarsest values
  double kq[26];              // kappa per level and for the coarsest values
  int L, M, nlev;
  int nested;                 // nested block schedule (propagation within the 3x3x3 block neighbourhood)
  int64_t* flag;              // overflow flag, cleared here
};
PrepField prep_field(bm_plan_s& p, const double* block_tol, const QPrep& q);
// ...and the task lists of its launches: propagation into level s+1 (index
// s), tables of level s (index s; index 0: coarsest values), each a device
// prefix array over the fields (first[nf] = total tasks)
struct PrepStages {
  const int64_t* prop_first[9] = {};
  int64_t prop_n[9] = {};
  const int64_t* tab_first[9] = {};
  int64_t tab_n[9] = {};
};
void launch_prep_batch(const PrepStages& g, const PrepField* F, int nf, hipStream_t st);

// fused decompose + quantize and dequantize + recompose (codes in place)
void decompose_quantize(bm_plan_s& p, const void* x, const double* block_tol, int32_t* codes, bm_qstats* stats,
                        hipStream_t st);
void dequantize_recompose(bm_plan_s& p, const int32_t* codes, const double* block_tol, void* x, hipStream_t st);
// the global levels (s > L) and the coarsest values of the fused pipeline
void decompose_quantize_global(bm_plan_s& p, const void* x, int32_t* codes, const QPrep& q, hipStream_t st);
void dequantize_recompose_global(bm_plan_s& p, const int32_t* codes, const QPrep& q, void* x, hipStream_t st);
void local_decompose_q(const bm_plan_s& p, int s, const View3& src, bool first, int32_t* codes, void* coarse_out,
                       const QPrep& q, hipStream_t st);
void local_recompose_q(const bm_plan_s& p, int s, const int32_t* codes, const void* coarse_in, void* out, bool last,
                       const QPrep& q, hipStream_t st);
// nested schedule: block levels s (17-node blocks) and s+1 (9-node blocks
// over the same regions) in one launch.  Decomposition writes level s's and
// s+1's coefficients (codes when q) and G^{s+1}; recomposition reads G^{s+1}
// (cin) and writes level s's output.
bool nest_pair(const bm_plan_s& p, int s);
void local_decompose_nest(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, int32_t* codes,
                          const QPrep* q, hipStream_t st);
void local_recompose_nest(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* out, bool last,
                          const int32_t* codes, const QPrep* q, hipStream_t st);

// many fields per launch (block levels): per-field kernel arguments are
// built on the host (block_*_args writes block_args_size bytes), uploaded,
// and one persistent launch covers block_groups(p_f, s) groups of every field
int64_t block_groups(const bm_plan_s& p, int s, bool dec);
size_t block_args_size(const bm_plan_s& p, bool dec);
void block_dec_args(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout, int32_t* codes,
                    const QPrep* q, void* out);
void block_rec_args(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* outp, bool last,
                    const int32_t* codes, const QPrep* q, void* out);
void launch_block_batch(int block, int dtype, bool dec, bool quant, const void* args, const int64_t* first, int nf,
                        int64_t ntasks, hipStream_t st);
// the nested pair (levels 1 and 2) of many fields per launch: level 1's and
// level 2's arguments of each field (block_args_size bytes each; x is the
// recomposition's output), block_groups(p_f, 1) groups per field
void block_nest_args(const bm_plan_s& p, bool dec, const View3& src, void* x, int32_t* codes, const QPrep* q,
                     void* out1, void* out2);
void launch_block_batch_nest(int dtype, bool dec, const void* a1, const void* a2, const int64_t* first, int nf,
                             int64_t ntasks, hipStream_t st);
// 33-node block levels of many fields: each field's arguments
// (wide_args_size bytes; src / first as for the decomposition, out / first =
// the caller's output for the recomposition), then the column, coarse (and,
// recomposing, interpolation) steps as persistent launches over all fields'
// block halves (first_half: 2 x blocks per field) and blocks (first_block)
size_t wide_args_size(const bm_plan_s& p);
void wide_batch_args(const bm_plan_s& p, int s, bool dec, const View3& src, bool first, void* out, int32_t* codes,
                     const QPrep* q, void* dst);
void launch_wide_batch(int dtype, bool dec, const void* args, const int64_t* first_half, const int64_t* first_block,
                       int nf, int64_t nhalf, int64_t nblock, hipStream_t st);

// quantization
void tolmap_from_boxes(bm_plan_s& p, const double* boxes, int nbox, double background, double* block_tol,
                       hipStream_t st);
void tolmap_from_voxels(bm_plan_s& p, const double* voxel_tol, double* block_tol, hipStream_t st);
void quantize(bm_plan_s& p, const void* coeff, const double* block_tol, int32_t* codes, bm_qstats* stats,
              hipStream_t st);
void dequantize(bm_plan_s& p, const int32_t* codes, const double* block_tol, void* coeff, hipStream_t st);
// per-node Delta for a linear quantity of interest <g, x> (returns the number
// of coefficients it depends on; synchronizes), and quantization with an
// explicit per-node Delta
int64_t qoi_deltas(bm_plan_s& p, const void* g, double tol_q, const double* block_tol, double* delta, hipStream_t st);
void quantize_delta(bm_plan_s& p, const void* coeff, const double* delta, int32_t* codes, bm_qstats* stats,
                    hipStream_t st);
void dequantize_delta(bm_plan_s& p, const int32_t* codes, const double* delta, void* coeff, hipStream_t st);

// compress path: lazily allocated code / coefficient buffers of a plan, the
// tolerance-map check, and the container writer (false: capacity too small,
// *needed holds the size)
void ensure_code_buffer(bm_plan_s& p);
void check_block_tol(bm_plan_s& p, const double* block_tol, hipStream_t st);
bool write_container(bm_plan_s& p, const void* x, const double* block_tol, bool too_fine, void* out, size_t capacity,
                     size_t* needed, hipStream_t st);
// the same in two steps: plan (sizes, Huffman plan; synchronizes), then write
std::shared_ptr<PendingContainer> plan_container(bm_plan_s& p, const void* x, const double* block_tol, bool too_fine,
                                                 hipStream_t st);
size_t pending_bytes(const PendingContainer& c);
void write_pending(PendingContainer& c, void* out);

// batches of fields (one dtype and block size): build / free, the fused
// pipeline both ways (graph: capture once per binding, then replay), and the
// fields whose codes overflowed int32 (synchronizes)
// the paper's own 8^3 block form (paper8.hip)
// M > 0: the paper's hybrid, M global levels on the assembled coarsest grid
bm_p8_s* p8_create(const int64_t dims[3], int dtype, int L, int M = 0);
int p8_global_levels(const bm_p8_s& p);
void p8_free(bm_p8_s* p);
int64_t p8_coeff_size(const bm_p8_s& p);
void p8_decompose(const bm_p8_s& p, const void* x, void* coeff, hipStream_t st);
void p8_recompose(const bm_p8_s& p, const void* coeff, void* x, hipStream_t st);
int p8_device(const bm_p8_s& p);
void p8_block_grid(const bm_p8_s& p, int64_t nb[3]);
void p8_tolmap_from_voxels(const bm_p8_s& p, const double* vt, double* block_tol, hipStream_t st);
void p8_quantize(const bm_p8_s& p, const void* coeff, const double* block_tol, double eta, int32_t* codes,
                 hipStream_t st);
void p8_dequantize(const bm_p8_s& p, const int32_t* codes, const double* block_tol, double eta, void* coeff,
                   hipStream_t st);
void p8_decompose_quantize(const bm_p8_s& p, const void* x, const double* block_tol, double eta, int32_t* codes,
                           hipStream_t st);
int32_t* p8_codes(bm_p8_s& p);
void p8_info(const bm_p8_s& p, int64_t dims[3], int* dtype, int* L, size_t* esize);
void p8_dequantize_recompose(const bm_p8_s& p, const int32_t* codes, const double* block_tol, double eta, void* x,
                             hipStream_t st);

bm_batch_s* batch_build(int nfields, const bm_config* cfgs);
void batch_free(bm_batch_s* b);
int batch_size(const bm_batch_s& b);
bm_plan_s* batch_plan(bm_batch_s& b, int field);
void batch_decompose_quantize(bm_batch_s& b, const void* const* x, const double* const* tol, int32_t* const* codes,
                              bool graph, hipStream_t st);
void batch_dequantize_recompose(bm_batch_s& b, const int32_t* const* codes, const double* const* tol, void* const* x,
                                bool graph, hipStream_t st);
int batch_overflows(bm_batch_s& b, std::vector<int>& bad, hipStream_t st);

// measured choice of (b, L, M); returns every measured candidate
// (budget_ms > 0: Algorithm 1's rule under that budget; *fits tells whether
// a candidate fit it, else the fastest is returned)
std::vector<bm_candidate> autotune(const bm_config& in, const void* x, const double* voxel_tol, double slack, int reps,
                                   bm_config& out, hipStream_t st, double budget_ms = 0.0, bool* fits = nullptr);

// huffman (host buffers).  An encoder plans its stream once on creation
// (histogram and chunk sizes on the device, code table on the host;
// synchronizes): bytes() is the exact stream size, write() encodes into a
// host buffer of at least that size.  Stage times of the calling thread's
// last encode and decode are kept for lossless_times().
// A part of a byte stream that is also on the device, with the CRC-32 of
// each of its whole kCrcBlock-byte blocks formed there.
struct CrcSpan {
  size_t offset = 0, bytes = 0;
  std::vector<uint32_t> block_crc;
};
constexpr size_t kCrcBlock = 16384;
// CRC-32 (zlib's) of buf[0, n), continuing from crc: the spans' block CRCs
// folded on the host, every other byte read there.
uint32_t crc_with_spans(const uint8_t* buf, size_t n, uint32_t crc, const CrcSpan* spans, int nspans);

class HuffmanEncoder {
 public:
  HuffmanEncoder(const int32_t* codes, int64_t n, hipStream_t st);
  ~HuffmanEncoder();
  HuffmanEncoder(const HuffmanEncoder&) = delete;
  HuffmanEncoder& operator=(const HuffmanEncoder&) = delete;
  size_t bytes() const;
  void write(uint8_t* dst, size_t capacity);
  // after write: the stream's parts that came from the device (the code
  // words, the outlier values), where they lie in it, and the CRC-32 of each
  // whole kCrcBlock of them, formed on the device before they were copied
  const CrcSpan (&device_spans() const)[2];

 private:
  struct Impl;
  std::unique_ptr<Impl> d_;
};
// The 32 columns of the GF(2) map that moves a CRC-32 register over `bytes`
// zero bytes (crc(A B) = shift(crc(A), |B|) ^ crc(B)).
void crc32_shift_matrix(uint64_t bytes, uint32_t out[32]);
// CRC-32 of a stream an encoder wrote (after its write), continuing from
// crc: the device's block CRCs of its code words, the rest on the host.
uint32_t stream_crc(const HuffmanEncoder& e, const uint8_t* stream, size_t n, uint32_t crc);
size_t huffman_encode(const int32_t* codes, int64_t n, std::vector<uint8_t>& out, hipStream_t st);
// exact size of the stream an encoder of these codes writes (synchronizes)
size_t huffman_size(const int32_t* codes, int64_t n, hipStream_t st);
void huffman_decode(const uint8_t* in, size_t in_bytes, int32_t* codes, int64_t n, hipStream_t st);
// The same in steps: the constructor checks the stream, builds the decode
// tables and uploads the stream (stream-ordered); crc() gives the CRC-32 of
// the stream's bytes continuing from crc, the code words and outlier values
// CRC'd on the device (synchronizes); decode() writes the n codes
// (synchronizes; BM_ECORRUPT if the stream does not decode).
class HuffmanDecoder {
 public:
  HuffmanDecoder(const uint8_t* in, size_t in_bytes, hipStream_t st);
  ~HuffmanDecoder();
  HuffmanDecoder(const HuffmanDecoder&) = delete;
  HuffmanDecoder& operator=(const HuffmanDecoder&) = delete;
  uint32_t crc(uint32_t crc);
  void decode(int32_t* codes, int64_t n);

 private:
  struct Impl;
  std::unique_ptr<Impl> d_;
};
bm_lossless_times lossless_times();
void huffman_code_lengths(const uint64_t* hist, uint8_t* len);
void set_lossless_crc_ms(double ms);
// Stage times of the Huffman encoder for n codes (ms): histogram (device),
// code table (host), chunk sizes and encode (device, with the host's offsets),
// copy of the stream to the host and its CRC-32.
void huffman_stage_times(const int32_t* codes, int64_t n, hipStream_t st, double ms[4]);
// time model of the pipeline and Algorithm 1 (model.hip)
void model_calibrate(int dtype, int b, bm_model& m, hipStream_t st);
void model_predict(const bm_model& m, const bm_config& cfg, double out[4]);
bool select_levels(const bm_config& in, const bm_model& m, double budget_ms, bm_config& out,
                   std::vector<bm_candidate>& cands);
// waits for a plan's recorded timing events and adds them to its totals
void drain_timing(bm_plan_s& p);
// CRC-32 of the container (zlib's polynomial), on host threads
uint32_t container_crc(const uint8_t* p, size_t n);
// the encoder that allocates nothing: stream written to device memory, work
// arrays of fixed size (at most kNoAllocMaxCodes codes)
constexpr int64_t kNoAllocMaxCodes = int64_t(1) << 28;
size_t huffman_encode_noalloc(const int32_t* codes, int64_t n, void* out, size_t capacity, size_t* out_bytes,
                              hipStream_t st);

// RAII event pair around the work of one timing slot (no-op unless timing is on)
struct TimedScope {
  bm_plan_s& p;
  int slot;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  TimedScope(bm_plan_s& p_, int slot_, hipStream_t st_);
  ~TimedScope();
};

// plan view of a coefficient array for level s (nodes of G^{s-1} inside the padded grid)
View3 level_view(const bm_plan_s& p, int s, void* coeff);
View3 coarsest_view(const bm_plan_s& p, void* coeff);

}  // namespace bm
