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

#include <algorithm>
#include <cstring>

#include "block.h"
#include "internal.h"

namespace bm {
namespace {

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
  uint32_t ss0;           // z stride of the source, 32-bit (within one column)
  int first, zero_pad;    // level 1 reads the unpadded input with clamp / zero fill
  T* coeff;
  int64_t cs[3];          // coefficient strides of this level's grid
  uint32_t cs0;           // z stride of the coefficients, 32-bit
  T* cout;                // compact coarse grid G^s
  int64_t cn[3];
  uint32_t cpl;           // plane size of the coarse grid
  int64_t nb[3], nblocks, nwg, per;
  FastDiv fnb2, fnb1;     // block index -> (bz, by, bx)
  // fused quantization (codes written instead of coefficients)
  int32_t* codes;         // same layout as coeff
  QTab tab;               // this level's block tables
  QTab ctab;              // coarsest-value tables (last block level when M == 0)
  int coarsest_here;
  int64_t* flag;          // set when a code does not fit in int32
  // last block level followed by a global level: its details are formed
  // here from the block's coarse values (codes with that level's 1/Delta)
  int fuse;
  const double* nqinv;
  double* part;           // per block: the next level's partial load vector [H][H][H] (FP64)
  // nested schedule, next block level in the same launch: the block's coarse
  // values stay in LDS (CC) for it, and nothing is written at them here
  int nest;
};

template <typename T>
struct RecArgs {
  const T* coeff;
  int64_t cs[3];
  uint32_t cs0;
  const T* cin;           // compact coarse grid G^s
  int64_t cn[3];
  uint32_t cpl;
  T* out;                 // output grid view (cropped to on)
  int64_t on[3], os[3];
  uint32_t os0;
  int64_t nb[3], nblocks, nwg, per;
  FastDiv fnb2, fnb1;
  const int32_t* codes;   // fused dequantization: codes instead of coefficients
  QTab tab, ctab;
  int coarsest_here;
  // last block level under a global level: the coarse values of G^s are
  // interpolated here from the next level's coarse grid G^{s+1} plus its
  // details (dequantized with that level's Delta), instead of read from cin
  int fuse;
  const T* cin2;
  int64_t cn2[3];
  const double* nqdel;
};

// Register budget of the block decomposition: FP32 fits 64 VGPRs (8 waves per
// SIMD), so more blocks are in flight to cover HBM latency; FP64 columns need
// more: 5 waves per SIMD (at most 102 VGPRs) fits them without spills and
// leaves four 17^3 workgroups per CU instead of three (512^3 FP64 level 1:
// 0.678 -> 0.574 ms; the recomposition spills at that budget and has none).
template <typename T>
constexpr int kWavesPerEU = sizeof(T) == 4 ? 8 : 5;

// Nested schedule, two block levels in one launch: the finer level (blocks
// of 2B-1 nodes) leaves each block's B^3 coarse values at the start of the
// block's LDS region; the coarser level (B-node blocks over the same
// regions) works in the same region after them, 16-byte aligned.
template <typename T, int B>
constexpr int nest_offset() {
  return int(((size_t(B) * B * B * sizeof(T) + 15) / 16) * 16 / sizeof(T));
}

// One workgroup's block group g (NBG blocks) of a decomposition level.
// SRC_LDS: the level's input is the coarse values a (2B-1)-node block level
// left in LDS for this group (nested schedule), not the source grid.
template <typename T, int B, bool Q, int NBG = Geo<B, sizeof(T)>::NB, bool SRC_LDS = false>
__device__ __attribute__((always_inline)) inline void decompose_group(const DecArgs<T>& a, int64_t g, T* lds) {
  using G = Geo<B, sizeof(T)>;
  constexpr int BB = G::BB, MC = G::MC, MI = G::MI, NB = NBG;
  constexpr int PREG = SRC_LDS ? Geo<2 * B - 1>::DEC_LDS : G::DEC_LDS;   // LDS elements per block
  constexpr int POFF = SRC_LDS ? nest_offset<T, B>() : 0;
  static_assert(!SRC_LDS || POFF + G::DEC_LDS <= PREG, "nested level must fit in its parent's LDS region");
  const int tid = threadIdx.x;
  // lanes run along the rows of the group's x-neighbouring blocks (NB
  // columns x of row y side by side), so a wavefront reads and writes
  // contiguous runs of NB * B values
  const int row = tid / (NB * B), rr = tid - row * (NB * B);
  const int bl = row < B ? rr / B : NB;              // block within the workgroup
  const int tb = row < B ? row * B + (rr - (rr / B) * B) : 0;   // column within the block
  const int64_t blk = g * NB + bl;
  const bool act = bl < NB && blk < a.nblocks;
  T* UE = lds + (bl < NB ? bl : 0) * PREG + POFF;   // even-z planes [MC][B][B]
  T* T1 = UE + MC * BB;                              // [MI][B][B]
  T* T2 = UE;                                        // [MI][MI][B], after UE is dead
  T* Z = T1;                                         // [MI][MI][MI], after T1 is dead
  const int y = tb / B, x = tb - (tb / B) * B;
  const bool ecol = ((y | x) & 1) == 0;
  int64_t bz = 0, by = 0, bx = 0;
  if (act) block_coords(uint32_t(blk), a.fnb2, a.fnb1, a.nb, bz, by, bx);
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  // a node on a shared face is written by the block that starts on it
  const bool owned = (y < B - 1 || by == a.nb[1] - 1) && (x < B - 1 || bx == a.nb[2] - 1);
  const bool lastz = bz == a.nb[0] - 1;
  // fused quantization: this column's 1/Delta, loaded early so the latency hides
  double iv[3];
  if (Q && act) column_class<B>(a.tab.cinv, blk, y, x, iv);
  T v[B];
  if (act && SRC_LDS) {
    const T* cc = lds + bl * PREG;                   // [B][B][B] coarse values of the finer level
#pragma unroll
    for (int z = 0; z < B; ++z) v[z] = cc[(z * B + y) * B + x];
#pragma unroll
    for (int j = 0; j < MC; ++j) UE[j * BB + tb] = v[2 * j];
  } else if (act) {
    if (!a.first || (oz + B <= a.sn[0] && gy < a.sn[1] && gx < a.sn[2])) {
      const T* col = a.src + oz * a.ss[0] + gy * a.ss[1] + gx * a.ss[2];
#pragma unroll
      for (int z = 0; z < B; ++z) v[z] = col[z * a.ss0];
    } else {
      // level 1 at the far faces: clamp or zero-fill outside the logical input
      const bool yx_in = gy < a.sn[1] && gx < a.sn[2];
      const int64_t ry = gy < a.sn[1] ? gy : a.sn[1] - 1;
      const int64_t rx = gx < a.sn[2] ? gx : a.sn[2] - 1;
      const T* col = a.src + ry * a.ss[1] + rx * a.ss[2];
#pragma unroll
      for (int z = 0; z < B; ++z) {
        const int64_t gz = oz + z;
        const bool in = yx_in && gz < a.sn[0];
        v[z] = (a.zero_pad && !in) ? T(0) : col[(gz < a.sn[0] ? gz : a.sn[0] - 1) * a.ss[0]];
      }
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
      // The coarse nodes of an even column get a placeholder (u_C, or code
      // 0): a later level (or the coarsest copy) overwrites them.  The plane
      // z = B-1 belongs to the next block unless this is the last one.
      // (fused with the next level: the coarse nodes are written at the end)
      const bool later = (a.fuse || a.nest) && ecol;
      if (!Q) {
        T* dst = a.coeff + oz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2];
#pragma unroll
        for (int z = 1; z < B - 1; z += 2) dst[z * a.cs0] = v[z];
        if (!later) {
#pragma unroll
          for (int z = 0; z < B - 1; z += 2) dst[z * a.cs0] = v[z];
          if (lastz) dst[(B - 1) * a.cs0] = v[B - 1];
        }
      } else {
        int32_t* dst = a.codes + oz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2];
        unsigned bad = 0;
#pragma unroll
        for (int z = 1; z < B - 1; z += 2) dst[z * a.cs0] = quant(v[z], iv[zcase<B>(z)], false, bad);
        if (!later) {   // even planes in one branch
#pragma unroll
          for (int z = 0; z < B - 1; z += 2) dst[z * a.cs0] = quant(v[z], iv[zcase<B>(z)], ecol, bad);
          if (lastz) dst[(B - 1) * a.cs0] = quant(v[B - 1], iv[2], ecol, bad);
        }
        if (bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), (unsigned long long)bad);
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
  // coarse values c = u_C + z (z = 0 on the block surface); the compact
  // coarse grid feeds the next level
  T c[MC];
  T* CC = UE;                                        // [MC][MC][MC] when fused (T2 is dead)
  // fused: the next level's load vector, in FP64 (see below): z pass in
  // registers, then y and x passes in LDS after CC
  constexpr int H = (MC + 1) / 2;
  double* Z1 = reinterpret_cast<double*>(CC + ((MC * MC * MC * sizeof(T) + 7) / 8) * (8 / sizeof(T)));   // [H][MC][MC]
  double* Y1 = Z1 + H * MC * MC;                     // [H][H][MC]
  if (act && ecol) {
#pragma unroll
    for (int j = 0; j < MC; ++j) c[j] = v[2 * j];
    if (y >= 2 && y <= B - 3 && x >= 2 && x <= B - 3) {
      const int I = (y - 2) >> 1, K = (x - 2) >> 1;
#pragma unroll
      for (int J = 0; J < MI; ++J) c[J + 1] += Z[(J * MI + I) * MI + K];
    }
    if (a.fuse || a.nest) {
#pragma unroll
      for (int j = 0; j < MC; ++j) CC[(j * MC + (y >> 1)) * MC + (x >> 1)] = c[j];
    }
    if (a.fuse) {
#pragma unroll
      for (int k = 0; k < H; ++k)
        Z1[(k * MC + (y >> 1)) * MC + (x >> 1)] = restrict_half<double, MC>(k, [&](int t) { return double(c[t]); });
    }
  }
  if (act && ecol && owned) {
    if (Q && a.coarsest_here) {
      // last level of the hierarchy: codes for the coarsest values
      double ci[3];
      column_class<B>(a.ctab.cinv, blk, y, x, ci);
      int32_t* dst = a.codes + oz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2];
      unsigned bad = 0;
#pragma unroll
      for (int j = 0; j < MC - 1; ++j) dst[2 * j * a.cs0] = quant(c[j], ci[zcase<B>(2 * j)], false, bad);
      if (lastz) dst[(B - 1) * a.cs0] = quant(c[MC - 1], ci[2], false, bad);
      if (bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), (unsigned long long)bad);
    } else if (!a.fuse && !a.nest) {
      T* cdst = a.cout + (oz >> 1) * int64_t(a.cpl) + (gy >> 1) * a.cn[2] + (gx >> 1);
#pragma unroll
      for (int j = 0; j < MC - 1; ++j) cdst[j * a.cpl] = c[j];
      if (lastz) cdst[(MC - 1) * a.cpl] = c[MC - 1];
    }
  }
  if (a.fuse) {
    // details of the next (global) level at this column's coarse nodes: c
    // minus the interpolant over the cell of the next coarse grid (every
    // such cell lies inside the block); its coarse nodes get a placeholder
    // (c, or code 0) that a later level or the coarsest values overwrite
    __syncthreads();
    if (act && ecol && owned) {
      const int p = y >> 1, q = x >> 1, op = p & 1, oq = q & 1;
      const double inv = Q ? *a.nqinv : 0.0;
      T in[MC];
      column_interp<T, MC>(p, q, [&](int J, int P, int K) { return CC[((2 * J) * MC + 2 * P) * MC + 2 * K]; }, in);
      unsigned bad = 0;
#pragma unroll
      for (int j = 0; j < MC; ++j) {
        if (j == MC - 1 && !lastz) continue;
        const bool cn = ((j & 1) | op | oq) == 0;
        const T d = cn ? c[j] : c[j] - in[j];
        const int64_t o = oz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2] + int64_t(2 * j) * a.cs0;
        if (Q)
          a.codes[o] = quant(d, inv, cn, bad);
        else
          a.coeff[o] = d;
      }
      if (Q && bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), (unsigned long long)bad);
    }
    // The next level's load vector 3 P^T M (per axis) at its coarse nodes in
    // this block, from the block's own coarse values only: rows on the block
    // faces take the half of the stencil on this side ({5/12, 1/2, 1/12}, the
    // natural end row), the neighbour adds the other half.  Shrinking passes
    // z (in registers, above), y and x (LDS), in FP64 so that the sum of 125
    // terms and the gather of up to 8 partials round once; the partial sums
    // go to a per-block array that a gather completes, so the global level
    // needs no pass over G^s.
    if (act) {
      for (int i = tb; i < H * H * MC; i += BB) {
        const int k0 = i / (H * MC), r = i - k0 * (H * MC), k1 = r / MC, q = r - k1 * MC;
        Y1[i] = restrict_half<double, MC>(k1, [&](int t) { return Z1[(k0 * MC + t) * MC + q]; });
      }
    }
    __syncthreads();
    if (act) {
      double* dst = a.part + blk * (H * H * H);
      for (int i = tb; i < H * H * H; i += BB) {
        const int r = i / H, k2 = i - r * H;
        dst[i] = restrict_half<double, MC>(k2, [&](int t) { return Y1[r * MC + t]; });
      }
    }
  }
}

// One workgroup's block group g (NBG blocks) of a recomposition level.
// Nested schedule, two block levels in one launch: MODE 1 is the coarser
// level (B-node blocks), which writes all B^3 values of each block to the
// start of the block's LDS region of the finer (2B-1)-node level and works
// after them; MODE 2 is that finer level, which reads its coarse values
// there instead of from the coarse grid.
template <typename T, int B, bool Q, int NBG = Geo<B, sizeof(T), false>::NB, int MODE = 0>
__device__ __attribute__((always_inline)) inline void recompose_group(const RecArgs<T>& a, int64_t g, T* lds) {
  using G = Geo<B, sizeof(T), false>;
  constexpr int BB = G::BB, MC = G::MC, MI = G::MI, NB = NBG;
  constexpr int PREG = MODE == 1 ? Geo<2 * B - 1>::REC_LDS : G::REC_LDS;   // LDS elements per block
  constexpr int POFF = MODE == 1 ? nest_offset<T, B>() : 0;
  static_assert(MODE != 1 || POFF + G::REC_LDS <= PREG, "nested level must fit in its parent's LDS region");
  const int tid = threadIdx.x;
  const int row = tid / (NB * B), rr = tid - row * (NB * B);   // as in decompose_group
  const int bl = row < B ? rr / B : NB;
  const int tb = row < B ? row * B + (rr - (rr / B) * B) : 0;
  const int64_t blk = g * NB + bl;
  const bool act = bl < NB && blk < a.nblocks;
  T* UC = lds + (bl < NB ? bl : 0) * PREG + POFF;   // coarse values u_C [MC][MC][MC]
  T* T1 = UC + MC * MC * MC;                         // [MI][B][B]
  T* T2 = T1 + MI * BB;                              // [MI][MI][B]
  T* Z = T1;                                         // [MI][MI][MI], after T1 is dead
  const int y = tb / B, x = tb - (tb / B) * B;
  const bool ecol = ((y | x) & 1) == 0;
  int64_t bz = 0, by = 0, bx = 0;
  if (act) block_coords(uint32_t(blk), a.fnb2, a.fnb1, a.nb, bz, by, bx);
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  // fused with the next (global) level: its coarse values over this block,
  // UC2[H][H][H] (in T2, which is first written by the y pass)
  constexpr int H = (MC + 1) / 2;
  T* UC2 = T2;
  if (a.fuse) {
    if (act) {
      const int64_t h0 = (MC - 1) / 2, pl2 = a.cn2[1] * a.cn2[2];
      const T* src = a.cin2 + bz * h0 * pl2 + by * h0 * a.cn2[2] + bx * h0;
      for (int i = tb; i < H * H * H; i += BB) {
        const int k0 = i / (H * H), r = i - k0 * H * H, k1 = r / H, k2 = r - k1 * H;
        UC2[i] = src[k0 * pl2 + k1 * a.cn2[2] + k2];
      }
    }
    __syncthreads();
  }
  T w[B], ce[MC];
  if (act) {
    // the whole column is read (coarse nodes too, then zeroed): one load per node
    const int64_t off = oz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2];
    if (!Q) {
      const T* col = a.coeff + off;
#pragma unroll
      for (int z = 0; z < B; ++z) w[z] = col[z * a.cs0];
    } else {
      // fused dequantization: c_hat = (T)(q * Delta)
      const int32_t* col = a.codes + off;
      int32_t qv[B];
#pragma unroll
      for (int z = 0; z < B; ++z) qv[z] = col[z * a.cs0];
      double dd[3];
      column_class<B>(a.tab.cdel, blk, y, x, dd);
#pragma unroll
      for (int z = 0; z < B; ++z) w[z] = T(mul_rn(double(qv[z]), dd[zcase<B>(z)]));
    }
    if (ecol) {
      if (Q && a.coarsest_here) {
        const int32_t* col = a.codes + off;
        int32_t qc[MC];
#pragma unroll
        for (int j = 0; j < MC; ++j) qc[j] = col[2 * j * a.cs0];
        double cd[3];
        column_class<B>(a.ctab.cdel, blk, y, x, cd);
#pragma unroll
        for (int j = 0; j < MC; ++j) ce[j] = T(mul_rn(double(qc[j]), cd[zcase<B>(2 * j)]));
      } else if (a.fuse) {
        // u at this column's coarse nodes = next level's detail + interpolant
        // of its coarse values (exactly the next level's recomposition)
        const int p = y >> 1, q = x >> 1, op = p & 1, oq = q & 1;
        const double del2 = Q ? *a.nqdel : 0.0;
        const int32_t* qcol = a.codes + off;
        T in[MC];
        column_interp<T, MC>(p, q, [&](int J, int P, int K) { return UC2[(J * H + P) * H + K]; }, in);
#pragma unroll
        for (int j = 0; j < MC; ++j) {
          if (((j & 1) | op | oq) == 0) {
            ce[j] = in[j];   // the next level's coarse value itself (exact)
          } else {
            const T w2 = Q ? T(mul_rn(double(qcol[2 * j * a.cs0]), del2)) : w[2 * j];
            ce[j] = w2 + in[j];
          }
        }
      } else if (MODE == 2) {
        // left here by the coarser level of the same launch
#pragma unroll
        for (int j = 0; j < MC; ++j) ce[j] = UC[(j * MC + (y >> 1)) * MC + (x >> 1)];
      } else {
        const T* ccol = a.cin + (oz >> 1) * int64_t(a.cpl) + (gy >> 1) * a.cn[2] + (gx >> 1);
#pragma unroll
        for (int j = 0; j < MC; ++j) ce[j] = ccol[j * a.cpl];
      }
      // c waits in UC through the correction passes (which do not touch UC)
      // instead of in registers; a nested finer level finds it there already
      if (MODE != 2) {
#pragma unroll
        for (int j = 0; j < MC; ++j) UC[(j * MC + (y >> 1)) * MC + (x >> 1)] = ce[j];
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
  if (act && ecol && y >= 2 && y <= B - 3 && x >= 2 && x <= B - 3) {
    // u_C = c - z on this column's interior coarse nodes (z = 0 on the block
    // surface, where u_C = c already)
    const int I = (y - 2) >> 1, K = (x - 2) >> 1;
#pragma unroll
    for (int j = 1; j <= MC - 2; ++j) {
      T& u = UC[(j * MC + (y >> 1)) * MC + (x >> 1)];
      u = u - Z[((j - 1) * MI + I) * MI + K];
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
    auto val = [&](int z) {
      return (z & 1) ? T(0.5) * (I2[z >> 1] + I2[(z >> 1) + 1]) + w[z] : (ecol ? I2[z >> 1] : I2[z >> 1] + w[z]);
    };
    if (MODE == 1) {
      // every node of the block, faces included: the finer level's coarse values
      T* dst = lds + bl * PREG;
#pragma unroll
      for (int z = 0; z < B; ++z) dst[(z * B + y) * B + x] = val(z);
      return;
    }
    const bool owny = (y < B - 1 || by == a.nb[1] - 1) && gy < a.on[1];
    const bool ownx = (x < B - 1 || bx == a.nb[2] - 1) && gx < a.on[2];
    const bool lastz = bz == a.nb[0] - 1;
    if (owny && ownx) {
      T* dst = a.out + oz * a.os[0] + gy * a.os[1] + gx * a.os[2];
      if (oz + B <= a.on[0]) {
#pragma unroll
        for (int z = 0; z < B - 1; ++z) dst[z * a.os0] = val(z);
        if (lastz) dst[(B - 1) * a.os0] = val(B - 1);
      } else {
        // the block reaches past the (cropped) output
#pragma unroll
        for (int z = 0; z < B; ++z)
          if ((z < B - 1 || lastz) && oz + z < a.on[0]) dst[z * a.os0] = val(z);
      }
    }
  }
}

template <typename T, int B, bool Q>
__global__ __launch_bounds__((Geo<B, sizeof(T)>::NT)) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<T>))) void k_local_decompose(DecArgs<T> a) {
  __shared__ __attribute__((aligned(16))) T lds[Geo<B, sizeof(T)>::NB * Geo<B>::DEC_LDS];   // FP64 scratch inside
  const int64_t g = xcd_group(blockIdx.x, a.per);
  if (g >= a.nwg) return;
  decompose_group<T, B, Q>(a, g, lds);
}

template <typename T, int B, bool Q>
__global__ __launch_bounds__((Geo<B, sizeof(T), false>::NT)) void k_local_recompose(RecArgs<T> a) {
  __shared__ T lds[Geo<B, sizeof(T), false>::NB * Geo<B>::REC_LDS];
  const int64_t g = xcd_group(blockIdx.x, a.per);
  if (g >= a.nwg) return;
  recompose_group<T, B, Q>(a, g, lds);
}

// Nested schedule: block levels of 17- and 9-node blocks over the same
// regions in one launch.  Decomposition: the 17-node level keeps each
// block's 9^3 coarse values in LDS and the 9-node level decomposes them
// there (the level-2 grid never goes through HBM).  Recomposition: the
// 9-node level recomposes each block's 9^3 values into LDS, and the
// 17-node level takes them as its coarse values.
template <typename T, bool Q>
__global__ __launch_bounds__((Geo<17, sizeof(T)>::NT)) __attribute__((amdgpu_waves_per_eu(kWavesPerEU<T>))) void k_local_decompose_nest(DecArgs<T> a1, DecArgs<T> a2) {
  constexpr int NB = Geo<17, sizeof(T)>::NB;
  __shared__ __attribute__((aligned(16))) T lds[NB * Geo<17>::DEC_LDS];   // FP64 scratch inside
  const int64_t g = xcd_group(blockIdx.x, a1.per);
  if (g >= a1.nwg) return;
  decompose_group<T, 17, Q>(a1, g, lds);
  __syncthreads();
  decompose_group<T, 9, Q, NB, true>(a2, g, lds);
}

template <typename T, bool Q>
__global__ __launch_bounds__((Geo<17, sizeof(T), false>::NT)) void k_local_recompose_nest(RecArgs<T> a2, RecArgs<T> a1) {
  constexpr int NB = Geo<17, sizeof(T), false>::NB;
  __shared__ __attribute__((aligned(16))) T lds[NB * Geo<17>::REC_LDS];
  const int64_t g = xcd_group(blockIdx.x, a1.per);
  if (g >= a1.nwg) return;
  recompose_group<T, 9, Q, NB, 1>(a2, g, lds);
  __syncthreads();
  recompose_group<T, 17, Q, NB, 2>(a1, g, lds);
}

// Many fields in one persistent launch: task k is block group k - first[f]
// of field f (first[] ascending, first[nf] = total, task_field); workgroups
// stride over the tasks.

// (no wave target here: the per-field arguments come from memory and the
// extra registers are cheaper than spills.  The field index is the same for
// every lane of the workgroup; said so with readfirstlane, and with the
// argument array read-only and unaliased, the record is read by scalar
// loads instead of vector loads kept in vector registers: the FP32
// decomposition went from 113 to 102 VGPRs, and a batched step of 256
// fields from 5.61 to 5.14 ms)
template <typename T, int B, bool Q>
__global__ __launch_bounds__((Geo<B, sizeof(T)>::NT)) void k_batch_decompose(
    const DecArgs<T>* __restrict__ fa, const int64_t* __restrict__ first, int nf, int64_t ntasks) {
  __shared__ __attribute__((aligned(16))) T lds[Geo<B, sizeof(T)>::NB * Geo<B>::DEC_LDS];   // FP64 scratch inside
  for (int64_t k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const int f = __builtin_amdgcn_readfirstlane(task_field(first, nf, k));
    decompose_group<T, B, Q>(fa[f], k - first[f], lds);
    __syncthreads();
  }
}

template <typename T, int B, bool Q>
__global__ __launch_bounds__((Geo<B, sizeof(T), false>::NT)) void k_batch_recompose(const RecArgs<T>* __restrict__ fa,
                                                                              const int64_t* __restrict__ first, int nf,
                                                                              int64_t ntasks) {
  __shared__ T lds[Geo<B, sizeof(T), false>::NB * Geo<B>::REC_LDS];
  for (int64_t k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const int f = __builtin_amdgcn_readfirstlane(task_field(first, nf, k));
    recompose_group<T, B, Q>(fa[f], k - first[f], lds);
    __syncthreads();
  }
}

// The nested schedule of every field in one persistent launch: task k is
// block group k - first[f] of field f at its 17-node level (arguments f1[f]),
// then the same group of its 9-node level (f2[f]) on the coarse values the
// first left in LDS, as k_local_decompose_nest / k_local_recompose_nest do
// for one field.
template <typename T, bool Q>
__global__ __launch_bounds__((Geo<17, sizeof(T)>::NT)) void k_batch_decompose_nest(
    const DecArgs<T>* __restrict__ f1, const DecArgs<T>* __restrict__ f2, const int64_t* __restrict__ first, int nf,
    int64_t ntasks) {
  constexpr int NB = Geo<17, sizeof(T)>::NB;
  __shared__ __attribute__((aligned(16))) T lds[NB * Geo<17>::DEC_LDS];   // FP64 scratch inside
  for (int64_t k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const int f = __builtin_amdgcn_readfirstlane(task_field(first, nf, k));
    const int64_t g = k - first[f];
    decompose_group<T, 17, Q>(f1[f], g, lds);
    __syncthreads();
    decompose_group<T, 9, Q, NB, true>(f2[f], g, lds);
    __syncthreads();
  }
}

template <typename T, bool Q>
__global__ __launch_bounds__((Geo<17, sizeof(T), false>::NT)) void k_batch_recompose_nest(
    const RecArgs<T>* __restrict__ f1, const RecArgs<T>* __restrict__ f2, const int64_t* __restrict__ first, int nf,
    int64_t ntasks) {
  constexpr int NB = Geo<17, sizeof(T), false>::NB;
  __shared__ T lds[NB * Geo<17>::REC_LDS];
  for (int64_t k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const int f = __builtin_amdgcn_readfirstlane(task_field(first, nf, k));
    const int64_t g = k - first[f];
    recompose_group<T, 9, Q, NB, 1>(f2[f], g, lds);
    __syncthreads();
    recompose_group<T, 17, Q, NB, 2>(f1[f], g, lds);
    __syncthreads();
  }
}

// 32-bit z stride within one block column
inline uint32_t column_stride(int64_t s, int B) {
  if (s * (B - 1) >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "grid planes too large for 32-bit column offsets");
  return uint32_t(s);
}

template <typename T, int B>
DecArgs<T> dec_args(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout, int32_t* codes,
                    const QPrep* q) {
  using G = Geo<B, sizeof(T)>;
  const Level& L = p.lv[s - 1];
  DecArgs<T> a{};
  a.src = static_cast<const T*>(src.ptr);
  for (int k = 0; k < 3; ++k) {
    a.sn[k] = src.n[k];
    a.ss[k] = src.s[k];
    a.cn[k] = L.m[k];
    a.nb[k] = L.nb[k];
  }
  a.ss0 = column_stride(src.s[0], B);
  a.first = first;
  a.zero_pad = p.cfg.pad_mode == 1;
  a.coeff = static_cast<T*>(coeff);
  const View3 cv = level_view(p, s, q ? static_cast<void*>(codes) : coeff);
  for (int k = 0; k < 3; ++k) a.cs[k] = cv.s[k];
  a.cs0 = column_stride(cv.s[0], B);
  a.cout = static_cast<T*>(cout);
  a.cpl = column_stride(L.m[1] * L.m[2], B);
  a.nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  if (a.nblocks >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "too many blocks");
  a.fnb2 = FastDiv(uint32_t(L.nb[2]));
  a.fnb1 = FastDiv(uint32_t(L.nb[1]));
  a.nwg = (a.nblocks + G::NB - 1) / G::NB;
  a.per = (a.nwg + 7) / 8;
  if (q) {
    a.codes = codes;
    a.tab = q->lv[s - 1];
    a.coarsest_here = (p.M == 0 && s == p.L) ? 1 : 0;
    if (a.coarsest_here) a.ctab = q->lv[kCoarseSlotHost];
    a.flag = q->flag;
  }
  a.fuse = (p.fuse_next && s == p.L) ? 1 : 0;
  if (a.fuse && q) a.nqinv = q->q + 2 * s + 1;   // 1/Delta of level s+1
  if (a.fuse) a.part = static_cast<double*>(p.ws.part);
  return a;
}

template <typename T, int B>
void launch_dec(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout, int32_t* codes,
                const QPrep* q, hipStream_t st) {
  using G = Geo<B, sizeof(T)>;
  const DecArgs<T> a = dec_args<T, B>(p, s, src, first, coeff, cout, codes, q);
  if (q)
    hipLaunchKernelGGL((k_local_decompose<T, B, true>), dim3(unsigned(8 * a.per)), dim3(G::NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_local_decompose<T, B, false>), dim3(unsigned(8 * a.per)), dim3(G::NT), 0, st, a);
  BM_HIP(hipGetLastError());
}

template <typename T, int B>
RecArgs<T> rec_args(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* out, bool last,
                    const int32_t* codes, const QPrep* q) {
  using G = Geo<B, sizeof(T), false>;
  const Level& L = p.lv[s - 1];
  RecArgs<T> a{};
  a.coeff = static_cast<const T*>(coeff);
  const View3 cv = level_view(p, s, q ? const_cast<int32_t*>(codes) : const_cast<void*>(coeff));
  for (int k = 0; k < 3; ++k) {
    a.cs[k] = cv.s[k];
    a.cn[k] = L.m[k];
    a.nb[k] = L.nb[k];
  }
  a.cs0 = column_stride(cv.s[0], B);
  a.cpl = column_stride(L.m[1] * L.m[2], B);
  a.cin = static_cast<const T*>(cin);
  a.out = static_cast<T*>(out);
  // last: writing the caller's output with the logical (unpadded) dims
  const int64_t* on = last ? p.dims : L.n;
  for (int k = 0; k < 3; ++k) a.on[k] = on[k];
  a.os[0] = on[1] * on[2];
  a.os[1] = on[2];
  a.os[2] = 1;
  a.os0 = column_stride(a.os[0], B);
  a.nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  if (a.nblocks >= (int64_t(1) << 32)) fail(BM_EUNSUPPORTED, "too many blocks");
  a.fnb2 = FastDiv(uint32_t(L.nb[2]));
  a.fnb1 = FastDiv(uint32_t(L.nb[1]));
  a.nwg = (a.nblocks + G::NB - 1) / G::NB;
  a.per = (a.nwg + 7) / 8;
  if (q) {
    a.codes = codes;
    a.tab = q->lv[s - 1];
    a.coarsest_here = (p.M == 0 && s == p.L) ? 1 : 0;
    if (a.coarsest_here) a.ctab = q->lv[kCoarseSlotHost];
  }
  a.fuse = (p.fuse_next && s == p.L) ? 1 : 0;
  if (a.fuse) {
    a.cin2 = static_cast<const T*>(p.ws.grid[s + 1]);
    for (int k = 0; k < 3; ++k) a.cn2[k] = p.lv[s].m[k];
    if (q) a.nqdel = q->q + 2 * s;                // Delta of level s+1
  }
  return a;
}

template <typename T, int B>
void launch_rec(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* out, bool last,
                const int32_t* codes, const QPrep* q, hipStream_t st) {
  using G = Geo<B, sizeof(T), false>;
  const RecArgs<T> a = rec_args<T, B>(p, s, coeff, cin, out, last, codes, q);
  if (q)
    hipLaunchKernelGGL((k_local_recompose<T, B, true>), dim3(unsigned(8 * a.per)), dim3(G::NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_local_recompose<T, B, false>), dim3(unsigned(8 * a.per)), dim3(G::NT), 0, st, a);
  BM_HIP(hipGetLastError());
}


template <typename T, int B>
void launch_batch(bool dec, bool quant, const void* args, const int64_t* first, int nf, int64_t ntasks,
                  hipStream_t st) {
  using G = Geo<B, sizeof(T)>;
  if (ntasks <= 0) return;
  if (dec) {
    const auto* fa = static_cast<const DecArgs<T>*>(args);
    if (quant) {
      auto k = k_batch_decompose<T, B, true>;
      hipLaunchKernelGGL(k, dim3(resident_grid(k, G::NT, ntasks)), dim3(G::NT), 0, st, fa, first, nf, ntasks);
    } else {
      auto k = k_batch_decompose<T, B, false>;
      hipLaunchKernelGGL(k, dim3(resident_grid(k, G::NT, ntasks)), dim3(G::NT), 0, st, fa, first, nf, ntasks);
    }
  } else {
    using R = Geo<B, sizeof(T), false>;
    const auto* fa = static_cast<const RecArgs<T>*>(args);
    if (quant) {
      auto k = k_batch_recompose<T, B, true>;
      hipLaunchKernelGGL(k, dim3(resident_grid(k, R::NT, ntasks)), dim3(R::NT), 0, st, fa, first, nf, ntasks);
    } else {
      auto k = k_batch_recompose<T, B, false>;
      hipLaunchKernelGGL(k, dim3(resident_grid(k, R::NT, ntasks)), dim3(R::NT), 0, st, fa, first, nf, ntasks);
    }
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

template <typename T>
void launch_dec_nest(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, int32_t* codes,
                     const QPrep* q, hipStream_t st) {
  using G = Geo<17, sizeof(T)>;
  DecArgs<T> a1 = dec_args<T, 17>(p, s, src, first, coeff, nullptr, codes, q);
  a1.nest = 1;
  const DecArgs<T> a2 = dec_args<T, 9>(p, s + 1, dense_view(p.ws.grid[s], p.lv[s].n), false, coeff,
                                       p.ws.grid[s + 1], codes, q);
  if (a1.fuse || a1.coarsest_here || a2.nblocks != a1.nblocks) fail(BM_EINVAL, "nested pair: inconsistent levels");
  if (q)
    hipLaunchKernelGGL((k_local_decompose_nest<T, true>), dim3(unsigned(8 * a1.per)), dim3(G::NT), 0, st, a1, a2);
  else
    hipLaunchKernelGGL((k_local_decompose_nest<T, false>), dim3(unsigned(8 * a1.per)), dim3(G::NT), 0, st, a1, a2);
  BM_HIP(hipGetLastError());
}

template <typename T>
void launch_rec_nest(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* out, bool last,
                     const int32_t* codes, const QPrep* q, hipStream_t st) {
  using G = Geo<17, sizeof(T), false>;
  const RecArgs<T> a1 = rec_args<T, 17>(p, s, coeff, nullptr, out, last, codes, q);
  const RecArgs<T> a2 = rec_args<T, 9>(p, s + 1, coeff, cin, nullptr, false, codes, q);
  if (a1.fuse || a1.coarsest_here || a2.nblocks != a1.nblocks) fail(BM_EINVAL, "nested pair: inconsistent levels");
  if (q)
    hipLaunchKernelGGL((k_local_recompose_nest<T, true>), dim3(unsigned(8 * a1.per)), dim3(G::NT), 0, st, a2, a1);
  else
    hipLaunchKernelGGL((k_local_recompose_nest<T, false>), dim3(unsigned(8 * a1.per)), dim3(G::NT), 0, st, a2, a1);
  BM_HIP(hipGetLastError());
}

}  // namespace

bool nest_pair(const bm_plan_s& p, int s) {
  return p.cfg.nested && s >= 1 && s < p.L && p.lv[s - 1].b == 17 && p.lv[s].b == 9;
}

void local_decompose_nest(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, int32_t* codes,
                          const QPrep* q, hipStream_t st) {
  if (!nest_pair(p, s)) fail(BM_EINVAL, "block levels s, s+1 are not a nested 17/9 pair");
  if (p.cfg.dtype == BM_F32)
    launch_dec_nest<float>(p, s, src, first, coeff, codes, q, st);
  else
    launch_dec_nest<double>(p, s, src, first, coeff, codes, q, st);
}

void local_recompose_nest(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* out, bool last,
                          const int32_t* codes, const QPrep* q, hipStream_t st) {
  if (!nest_pair(p, s)) fail(BM_EINVAL, "block levels s, s+1 are not a nested 17/9 pair");
  if (p.cfg.dtype == BM_F32)
    launch_rec_nest<float>(p, s, coeff, cin, out, last, codes, q, st);
  else
    launch_rec_nest<double>(p, s, coeff, cin, out, last, codes, q, st);
}

void local_decompose(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* coarse_out,
                     hipStream_t st) {
  if (p.lv[s - 1].b == 33)
    wide_decompose(p, s, src, first, coeff, coarse_out, nullptr, nullptr, st);
  else if (p.lv[s - 1].b == 9)
    dispatch_dec<9>(p, s, src, first, coeff, coarse_out, nullptr, nullptr, st);
  else
    dispatch_dec<17>(p, s, src, first, coeff, coarse_out, nullptr, nullptr, st);
}

void local_recompose(const bm_plan_s& p, int s, const void* coeff, const void* coarse_in, void* out, bool last,
                     hipStream_t st) {
  if (p.lv[s - 1].b == 33)
    wide_recompose(p, s, coeff, const_cast<void*>(coarse_in), out, last, nullptr, nullptr, st);
  else if (p.lv[s - 1].b == 9)
    dispatch_rec<9>(p, s, coeff, coarse_in, out, last, nullptr, nullptr, st);
  else
    dispatch_rec<17>(p, s, coeff, coarse_in, out, last, nullptr, nullptr, st);
}

void local_decompose_q(const bm_plan_s& p, int s, const View3& src, bool first, int32_t* codes, void* coarse_out,
                       const QPrep& q, hipStream_t st) {
  if (p.lv[s - 1].b == 33)
    wide_decompose(p, s, src, first, nullptr, coarse_out, codes, &q, st);
  else if (p.lv[s - 1].b == 9)
    dispatch_dec<9>(p, s, src, first, nullptr, coarse_out, codes, &q, st);
  else
    dispatch_dec<17>(p, s, src, first, nullptr, coarse_out, codes, &q, st);
}

void local_recompose_q(const bm_plan_s& p, int s, const int32_t* codes, const void* coarse_in, void* out, bool last,
                       const QPrep& q, hipStream_t st) {
  if (p.lv[s - 1].b == 33)
    wide_recompose(p, s, nullptr, const_cast<void*>(coarse_in), out, last, codes, &q, st);
  else if (p.lv[s - 1].b == 9)
    dispatch_rec<9>(p, s, nullptr, coarse_in, out, last, codes, &q, st);
  else
    dispatch_rec<17>(p, s, nullptr, coarse_in, out, last, codes, &q, st);
}

int64_t block_groups(const bm_plan_s& p, int s, bool dec) {
  const int nbw = p.lv[s - 1].b <= 9 ? Geo<9>::NB
                                   : (p.esize == 4 ? (dec ? Geo<17, 4, true>::NB : Geo<17, 4, false>::NB) : Geo<17, 8>::NB);
  const int64_t* nb = p.lv[s - 1].nb;
  return (nb[0] * nb[1] * nb[2] + nbw - 1) / nbw;
}

size_t block_args_size(const bm_plan_s& p, bool dec) {
  if (p.cfg.dtype == BM_F32) return dec ? sizeof(DecArgs<float>) : sizeof(RecArgs<float>);
  return dec ? sizeof(DecArgs<double>) : sizeof(RecArgs<double>);
}

void block_dec_args(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout, int32_t* codes,
                    const QPrep* q, void* out) {
  if (p.cfg.dtype == BM_F32) {
    const auto a = p.lv[s - 1].b == 9 ? dec_args<float, 9>(p, s, src, first, coeff, cout, codes, q)
                                    : dec_args<float, 17>(p, s, src, first, coeff, cout, codes, q);
    std::memcpy(out, &a, sizeof(a));
  } else {
    const auto a = p.lv[s - 1].b == 9 ? dec_args<double, 9>(p, s, src, first, coeff, cout, codes, q)
                                    : dec_args<double, 17>(p, s, src, first, coeff, cout, codes, q);
    std::memcpy(out, &a, sizeof(a));
  }
}

void block_rec_args(const bm_plan_s& p, int s, const void* coeff, const void* cin, void* outp, bool last,
                    const int32_t* codes, const QPrep* q, void* out) {
  if (p.cfg.dtype == BM_F32) {
    const auto a = p.lv[s - 1].b == 9 ? rec_args<float, 9>(p, s, coeff, cin, outp, last, codes, q)
                                    : rec_args<float, 17>(p, s, coeff, cin, outp, last, codes, q);
    std::memcpy(out, &a, sizeof(a));
  } else {
    const auto a = p.lv[s - 1].b == 9 ? rec_args<double, 9>(p, s, coeff, cin, outp, last, codes, q)
                                    : rec_args<double, 17>(p, s, coeff, cin, outp, last, codes, q);
    std::memcpy(out, &a, sizeof(a));
  }
}

void launch_block_batch(int block, int dtype, bool dec, bool quant, const void* args, const int64_t* first, int nf,
                        int64_t ntasks, hipStream_t st) {
  if (dtype == BM_F32) {
    if (block == 9)
      launch_batch<float, 9>(dec, quant, args, first, nf, ntasks, st);
    else
      launch_batch<float, 17>(dec, quant, args, first, nf, ntasks, st);
  } else {
    if (block == 9)
      launch_batch<double, 9>(dec, quant, args, first, nf, ntasks, st);
    else
      launch_batch<double, 17>(dec, quant, args, first, nf, ntasks, st);
  }
}

namespace {

template <typename T>
void nest_dec_pair(const bm_plan_s& p, const View3& src, int32_t* codes, const QPrep* q, void* out1, void* out2) {
  DecArgs<T> a1 = dec_args<T, 17>(p, 1, src, true, nullptr, nullptr, codes, q);
  a1.nest = 1;
  const DecArgs<T> a2 = dec_args<T, 9>(p, 2, dense_view(p.ws.grid[1], p.lv[1].n), false, nullptr, p.ws.grid[2], codes, q);
  if (a1.fuse || a1.coarsest_here || a2.nblocks != a1.nblocks) fail(BM_EINVAL, "nested pair: inconsistent levels");
  std::memcpy(out1, &a1, sizeof(a1));
  std::memcpy(out2, &a2, sizeof(a2));
}

template <typename T>
void nest_rec_pair(const bm_plan_s& p, void* x, const int32_t* codes, const QPrep* q, void* out1, void* out2) {
  const RecArgs<T> a1 = rec_args<T, 17>(p, 1, nullptr, nullptr, x, true, codes, q);
  const RecArgs<T> a2 = rec_args<T, 9>(p, 2, nullptr, p.ws.grid[2], nullptr, false, codes, q);
  if (a1.fuse || a1.coarsest_here || a2.nblocks != a1.nblocks) fail(BM_EINVAL, "nested pair: inconsistent levels");
  std::memcpy(out1, &a1, sizeof(a1));
  std::memcpy(out2, &a2, sizeof(a2));
}

template <typename T>
void launch_batch_nest(bool dec, const void* a1, const void* a2, const int64_t* first, int nf, int64_t ntasks,
                       hipStream_t st) {
  if (ntasks <= 0) return;
  if (dec) {
    auto k = k_batch_decompose_nest<T, true>;
    const int nt = Geo<17, sizeof(T)>::NT;
    hipLaunchKernelGGL(k, dim3(resident_grid(k, nt, ntasks)), dim3(nt), 0, st, static_cast<const DecArgs<T>*>(a1),
                       static_cast<const DecArgs<T>*>(a2), first, nf, ntasks);
  } else {
    auto k = k_batch_recompose_nest<T, true>;
    const int nt = Geo<17, sizeof(T), false>::NT;
    hipLaunchKernelGGL(k, dim3(resident_grid(k, nt, ntasks)), dim3(nt), 0, st, static_cast<const RecArgs<T>*>(a1),
                       static_cast<const RecArgs<T>*>(a2), first, nf, ntasks);
  }
  BM_HIP(hipGetLastError());
}

}  // namespace

// Arguments of a field's nested pair (17-node level 1, 9-node level 2) for
// the batched nest launch: out1 gets level 1's, out2 level 2's (each
// block_args_size bytes).
void block_nest_args(const bm_plan_s& p, bool dec, const View3& src, void* x, int32_t* codes, const QPrep* q,
                     void* out1, void* out2) {
  if (!nest_pair(p, 1)) fail(BM_EINVAL, "block levels 1, 2 are not a nested 17/9 pair");
  if (dec) {
    if (p.cfg.dtype == BM_F32)
      nest_dec_pair<float>(p, src, codes, q, out1, out2);
    else
      nest_dec_pair<double>(p, src, codes, q, out1, out2);
  } else {
    if (p.cfg.dtype == BM_F32)
      nest_rec_pair<float>(p, x, codes, q, out1, out2);
    else
      nest_rec_pair<double>(p, x, codes, q, out1, out2);
  }
}

void launch_block_batch_nest(int dtype, bool dec, const void* a1, const void* a2, const int64_t* first, int nf,
                             int64_t ntasks, hipStream_t st) {
  if (dtype == BM_F32)
    launch_batch_nest<float>(dec, a1, a2, first, nf, ntasks, st);
  else
    launch_batch_nest<double>(dec, a1, a2, first, nf, ntasks, st);
}

}  // namespace bm
