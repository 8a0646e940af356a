// One wavefront solves one line of the coarse mass-matrix system of a global
// level (Sec. II-B): 3 Mc x = rhs, where 3 Mc = tridiag(1, 4, 1) with end
// diagonals 2 (linear elements, unit spacing, natural ends).
//
// Lane l owns the q = ceil(m / 64) consecutive unknowns starting at l * q.
// Both Thomas sweeps are first-order affine recurrences,
//   forward   d_J = -inv_J d_{J-1} + inv_J rhs_J,
//   backward  x_J = -inv_J x_{J+1} + d_J,
// with inv_J the reciprocal pivots.  Each lane folds its run into one affine
// map, a 64-lane scan of the maps (wave shuffles) gives each lane its
// incoming value, and the lane replays its run.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bm {

constexpr int kLineQ = 9;   // unknowns per lane: lines of up to 64 * 9 coarse nodes

// Affine map x -> A x + B; inclusive scan composing lower lanes first.
template <typename T>
__device__ inline void scan_up(T& A, T& B, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T Ap = __shfl_up(A, off, 64);
    const T Bp = __shfl_up(B, off, 64);
    if (lane >= off) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
}

// The same, composing higher lanes first.
template <typename T>
__device__ inline void scan_down(T& A, T& B, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T An = __shfl_down(A, off, 64);
    const T Bn = __shfl_down(B, off, 64);
    if (lane + off < 64) {
      B = A * Bn + B;
      A = A * An;
    }
  }
}

// rhs(J) returns the right-hand side of row J (already scaled by 3);
// out(J, x) receives the solution.  Every rhs is read before any out is
// called, so the two may refer to the same storage.
template <typename T, typename Rhs, typename Out>
__device__ inline void wave_thomas(int64_t m, const double* inv, int lane, Rhs rhs, Out out) {
  const int q = int((m + 63) / 64);
  const int64_t J0 = int64_t(lane) * q;
  T f[kLineQ], al[kLineQ];
  T A = T(1), B = T(0);
#pragma unroll
  for (int j = 0; j < kLineQ; ++j) {
    const int64_t J = J0 + j;
    if (j < q && J < m) {
      const T iv = T(inv[J]);
      al[j] = J == 0 ? T(0) : -iv;
      f[j] = rhs(J) * iv;
      A = al[j] * A;
      B = al[j] * B + f[j];
    }
  }
  scan_up(A, B, lane);
  T din = __shfl_up(B, 1, 64);
  if (lane == 0) din = T(0);
#pragma unroll
  for (int j = 0; j < kLineQ; ++j) {
    if (j < q && J0 + j < m) {
      din = al[j] * din + f[j];
      f[j] = din;   // f now holds d_J
    }
  }
  A = T(1);
  B = T(0);
#pragma unroll
  for (int j = kLineQ - 1; j >= 0; --j) {
    const int64_t J = J0 + j;
    if (j < q && J < m) {
      al[j] = J == m - 1 ? T(0) : -T(inv[J]);
      A = al[j] * A;
      B = al[j] * B + f[j];
    }
  }
  scan_down(A, B, lane);
  T xin = __shfl_down(B, 1, 64);
  if (lane == 63) xin = T(0);
#pragma unroll
  for (int j = kLineQ - 1; j >= 0; --j) {
    const int64_t J = J0 + j;
    if (j < q && J < m) {
      xin = al[j] * xin + f[j];
      out(J, xin);
    }
  }
}

}  // namespace bm
