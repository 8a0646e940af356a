// Shared-face block geometry of the In-cache Block levels (Sec. IV-A), the
// constants of the face-fixed correction, and the per-node pieces (block
// coordinates, Delta classes, quantizer) shared by the block kernels of the
// transform and of its transpose.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace bm {

// ES: bytes per value; DEC: decomposition (else recomposition).  Blocks per
// workgroup: three 9^3 blocks fill 256 lanes; for FP32 decomposition two
// x-neighbouring 17^3 blocks (640 lanes) share the cache lines of their
// common face in one workgroup, which halves the partial-line traffic across
// workgroups.  FP64, and the recomposition (more registers per lane), keep
// one 17^3 block so several workgroups still fit on a CU.
template <int B, int ES = 4, bool DEC = true>
struct Geo {
  static constexpr int BB = B * B;
  static constexpr int MC = (B + 1) / 2;        // coarse nodes per axis
  static constexpr int MI = MC - 2;             // interior coarse nodes per axis
  static constexpr int NB = B <= 9 ? 3 : ((ES == 4 && DEC) ? 2 : 1);
  static constexpr int NT = ((NB * BB + 63) / 64) * 64;
  // LDS per block: decompose UE[MC][B][B] + T1[MI][B][B] (T2 aliases UE, Z aliases T1)
  static constexpr int DEC_LDS = MC * BB + MI * BB;
  // recompose: UC[MC][MC][MC] + T1[MI][B][B] + T2[MI][MI][B] (Z aliases T1)
  static constexpr int REC_LDS = MC * MC * MC + MI * BB + MI * MI * B;
  // transposes: T1[MI][B][B] + T2[MI][MI][B] + Z[MI][MI][MI]; the restriction
  // planes R[MC][B][B] alias the start
  static constexpr int ADJ_WORK = MI * BB + MI * MI * B + MI * MI * MI;
  static constexpr int ADJ_LDS = ADJ_WORK > MC * BB ? ADJ_WORK : MC * BB;
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

// XCD-aware order: hardware workgroup ids go round-robin over the 8 XCDs;
// this map gives each XCD a contiguous run of workgroups so shared faces are
// re-read from the same L2.
__device__ inline int64_t xcd_group(int64_t wg, int64_t per) { return (wg & 7) * per + (wg >> 3); }

// Restriction by the interior rows of P^T M (centre 2J+2) followed by the
// interior tridiagonal solve, on a line of B values: out[J], J < MI.
template <typename T, int B>
__device__ inline void restrict_solve(const T (&w)[B], T (&out)[Geo<B>::MI]) {
  constexpr int MI = Geo<B>::MI;
  constexpr Pivots<MI> P{};
  const T C0 = T(5.0 / 6.0), C1 = T(0.5), C2 = T(1.0 / 12.0);
  T d[MI];
#pragma unroll
  for (int J = 0; J < MI; ++J) {
    const int c = 2 * J + 2;
    const T r = C2 * (w[c - 2] + w[c + 2]) + C1 * (w[c - 1] + w[c + 1]) + C0 * w[c];
    d[J] = J == 0 ? T(3) * r * T(P.v[0]) : (T(3) * r - d[J - 1]) * T(P.v[J]);
  }
  out[MI - 1] = d[MI - 1];
#pragma unroll
  for (int J = MI - 2; J >= 0; --J) out[J] = d[J] - T(P.v[J]) * out[J + 1];
}

// The next level's interpolant along one column (p, q) of a block's coarse
// grid (MC nodes per axis): out[j], j < MC.  rd(J, P, Q) reads the next
// level's coarse node (2J, 2P, 2Q).  The y-x means of the even planes come
// first (x pairs, then y), then pairs along z; the scalings by 1/4 and 1/2
// are exact, so out[j] equals cell_mean over the node's cell bit for bit.
template <typename T, int MC, typename F>
__device__ inline void column_interp(int p, int q, F rd, T (&out)[MC]) {
  constexpr int H = (MC + 1) / 2;
  const int p0 = p >> 1, p1 = (p + 1) >> 1, q0 = q >> 1, q1 = (q + 1) >> 1;
  T I2[H];
#pragma unroll
  for (int J = 0; J < H; ++J) I2[J] = T(0.25) * ((rd(J, p0, q0) + rd(J, p0, q1)) + (rd(J, p1, q0) + rd(J, p1, q1)));
#pragma unroll
  for (int j = 0; j < MC; ++j) out[j] = (j & 1) ? T(0.5) * (I2[j >> 1] + I2[(j >> 1) + 1]) : I2[j >> 1];
}

// 3 (P^T M v) at coarse node k (k < (MC+1)/2) of a line of MC values read
// by v(t) (unit spacing): interior rows {1/12, 1/2, 5/6, 1/2, 1/12} around
// node 2k; the two end rows keep the half on the line's side, 5/12 at the
// end node.
template <typename T, int MC, typename V>
__device__ inline T restrict_half(int k, V v) {
  constexpr int H = (MC + 1) / 2;
  const int c = 2 * k;
  T r;
  if (k == 0)
    r = T(5.0 / 12.0) * v(0) + T(0.5) * v(1) + T(1.0 / 12.0) * v(2);
  else if (k == H - 1)
    r = T(1.0 / 12.0) * v(MC - 3) + T(0.5) * v(MC - 2) + T(5.0 / 12.0) * v(MC - 1);
  else
    r = T(1.0 / 12.0) * (v(c - 2) + v(c + 2)) + T(0.5) * (v(c - 1) + v(c + 1)) + T(5.0 / 6.0) * v(c);
  return T(3) * r;
}

// block coordinates of block index blk
__device__ inline void block_coords(uint32_t blk, const FastDiv& f2, const FastDiv& f1, const int64_t nb[3],
                                    int64_t& bz, int64_t& by, int64_t& bx) {
  const uint32_t t = f2.div(blk);
  bx = int64_t(blk) - int64_t(t) * nb[2];
  const uint32_t z = f1.div(t);
  by = int64_t(t) - int64_t(z) * nb[1];
  bz = z;
}

// position class of a local coordinate: first face 0, interior 1, last face 2
template <int B>
__device__ inline int pos_class(int c) {
  return c == 0 ? 0 : (c == B - 1 ? 2 : 1);
}

// The Delta-table entries (27 classes per block) of one z-column: a node takes
// the smallest Delta (largest 1/Delta) of the blocks that contain it.  Entries
// for z = 0, for 0 < z < B-1 and for z = B-1.
template <int B>
__device__ inline void column_class(const double* tab, int64_t blk, int y, int x, double out[3]) {
  const double* t = tab + blk * 27 + pos_class<B>(y) * 3 + pos_class<B>(x);
  out[0] = t[0];
  out[1] = t[9];
  out[2] = t[18];
}

template <int B>
__device__ inline int zcase(int z) { return z == 0 ? 0 : (z == B - 1 ? 2 : 1); }

// q = rint(c * (1/Delta)) in FP64.  A code outside int32 sets bit kFlagRange
// of bad, a coefficient that is NaN or infinite (non-finite data) sets
// kFlagNonFinite; either way 0 is written.  skip: a placeholder (zero) is
// written instead and nothing is checked.
template <typename T>
__device__ inline int32_t quant(T c, double inv, bool skip, unsigned& bad) {
  const double v = rint(mul_rn(double(c), inv));
  const bool ok = fabs(v) <= 2147483647.0;
  if (!ok && !skip) bad |= code_flag(double(c));
  return (ok && !skip) ? int32_t(v) : 0;
}

}  // namespace bm
