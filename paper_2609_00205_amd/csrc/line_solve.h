// Line solves of the coarse mass-matrix system of a global level (Sec. II-B):
// 3 Mc x = rhs, where 3 Mc = tridiag(1, 4, 1) with end diagonals 2 (linear
// elements, unit spacing, natural ends).
//
// A group of lanes solves one line; lane r of the group owns the q
// consecutive unknowns starting at r * q.  Both Thomas sweeps are
// first-order affine recurrences,
//   forward   d_J = -inv_J d_{J-1} + inv_J rhs_J,
//   backward  x_J = -inv_J x_{J+1} + d_J,
// with inv_J the reciprocal pivots.  Each lane folds its run into one affine
// map, a scan of the maps across the group gives each lane its incoming
// value, and the lane replays its run.  Lines of up to 16 * kRowQ coarse
// nodes use 16-lane groups (one DPP row: the scan is four row shifts, no
// LDS traffic), four lines per wavefront; longer lines use the whole
// wavefront and shuffles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bm {

constexpr int kLineQ = 9;    // 64-lane groups: unknowns per lane, lines of up to 576 coarse nodes
constexpr int kRowQ = 17;    // 16-lane groups: unknowns per lane, lines of up to 272 coarse nodes

// Value of the lane selected by a DPP row control (row_shr / row_shl within
// 16-lane rows); lanes with no source in their row get `old`.
template <int CTRL>
__device__ inline float dpp_row(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ inline double dpp_row(double old, double v) {
  const unsigned long long o = __double_as_longlong(old), s = __double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(int(unsigned(o)), int(unsigned(s)), CTRL, 0xf, 0xf, false));
  const unsigned hi =
      unsigned(__builtin_amdgcn_update_dpp(int(unsigned(o >> 32)), int(unsigned(s >> 32)), CTRL, 0xf, 0xf, false));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// One step of an affine-map scan: compose this lane's map after the map of
// the lane CTRL selects (identity where there is none).
template <int CTRL, typename T>
__device__ inline void row_step(T& A, T& B) {
  const T Ap = dpp_row<CTRL>(T(1), A);
  const T Bp = dpp_row<CTRL>(T(0), B);
  B = A * Bp + B;
  A = A * Ap;
}

// inclusive scans within 16-lane rows: lower lanes first (row_shr) or higher
// lanes first (row_shl)
template <typename T>
__device__ inline void row_scan_up(T& A, T& B) {
  row_step<0x111>(A, B);
  row_step<0x112>(A, B);
  row_step<0x114>(A, B);
  row_step<0x118>(A, B);
}

template <typename T>
__device__ inline void row_scan_down(T& A, T& B) {
  row_step<0x101>(A, B);
  row_step<0x102>(A, B);
  row_step<0x104>(A, B);
  row_step<0x108>(A, B);
}

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
__device__ inline void wave_thomas(int64_t m, const T* inv, int lane, Rhs rhs, Out out) {
  const int q = int((m + 63) / 64);
  const int64_t J0 = int64_t(lane) * q;
  T f[kLineQ], al[kLineQ];
  T A = T(1), B = T(0);
#pragma unroll
  for (int j = 0; j < kLineQ; ++j) {
    const int64_t J = J0 + j;
    if (j < q && J < m) {
      const T iv = inv[J];
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
      al[j] = J == m - 1 ? T(0) : -inv[J];
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

// The same solve by a 16-lane row (r = lane within the row), m <= 16 * Q.
template <typename T, int Q, typename Rhs, typename Out>
__device__ inline void row_thomas(int m, const T* inv, int r, Rhs rhs, Out out) {
  const int q = (m + 15) >> 4;
  const int J0 = r * q;
  T f[Q], al[Q];
  T A = T(1), B = T(0);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int J = J0 + j;
    if (j < q && J < m) {
      const T iv = inv[J];
      al[j] = J == 0 ? T(0) : -iv;
      f[j] = rhs(J) * iv;
      A = al[j] * A;
      B = al[j] * B + f[j];
    }
  }
  row_scan_up(A, B);
  T din = dpp_row<0x111>(T(0), B);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if (j < q && J0 + j < m) {
      din = al[j] * din + f[j];
      f[j] = din;
    }
  }
  A = T(1);
  B = T(0);
#pragma unroll
  for (int j = Q - 1; j >= 0; --j) {
    const int J = J0 + j;
    if (j < q && J < m) {
      al[j] = J == m - 1 ? T(0) : -inv[J];
      A = al[j] * A;
      B = al[j] * B + f[j];
    }
  }
  row_scan_down(A, B);
  T xin = dpp_row<0x101>(T(0), B);
#pragma unroll
  for (int j = Q - 1; j >= 0; --j) {
    const int J = J0 + j;
    if (j < q && J < m) {
      xin = al[j] * xin + f[j];
      out(J, xin);
    }
  }
}

// Solves lines 0..wv-1 of a tile with the NTHREADS / 64 wavefronts of a
// workgroup.  rhs(w, J) reads the right-hand side of row J of line w;
// out(w, J, x) receives the solution.  Q > 0: 16-lane rows with up to Q
// unknowns per lane (m <= 16 Q; registers scale with Q, so the launcher picks
// the smallest Q that fits); Q = 0: a wavefront per line.  Every lane of a
// wavefront takes part in its scans: a row past the last line repeats a
// valid line and writes nothing.
inline int row_q_for(int64_t m) {
  // (11 for the 161-node lines of a 321-node axis: 16 x 11 = 176 slots
  // instead of 272 shortens every lane's sweeps; measured 3% on the 8^3
  // hybrid's fused step at 512^3, whose global axes are 321 nodes long)
  return m <= 48 ? 3 : m <= 80 ? 5 : m <= 144 ? 9 : m <= 176 ? 11 : m <= 16 * kRowQ ? kRowQ : 0;
}

template <typename T, int NTHREADS, int Q, typename Rhs, typename Out>
__device__ inline void solve_lines(int m, const T* inv, int wv, int tid, Rhs rhs, Out out) {
  constexpr int NW = NTHREADS / 64;
  const int lane = tid & 63, wave = tid >> 6;
  if constexpr (Q > 0) {
    const int r = lane & 15;
    for (int w0 = wave * 4; w0 < wv; w0 += NW * 4) {
      const int w = w0 + (lane >> 4);
      const int wr = w < wv ? w : w0;
      row_thomas<T, Q>(m, inv, r, [&](int J) { return rhs(wr, J); }, [&](int J, T x) {
        if (w < wv) out(w, J, x);
      });
    }
  } else {
    for (int w = wave; w < wv; w += NW)
      wave_thomas<T>(m, inv, lane, [&](int64_t J) { return rhs(w, int(J)); },
                     [&](int64_t J, T x) { out(w, int(J), x); });
  }
}

// Lines per workgroup tile of a line pass: a power of two <= 64 whose LDS
// tile (line_elems values per line) stays within 40 KiB, halved while the
// launch would have fewer than 1024 tiles (four per CU; short grids still
// spread over the 256 CUs, and wider tiles keep more lines per load), and no
// wider than the nq lines available.
inline int tile_width(int64_t line_elems, size_t esize, int64_t np, int64_t nq) {
  int W = 64;
  while (W > 1 && line_elems * (W + 1) * int64_t(esize) > 40960) W >>= 1;
  while (W > 1 && np * ((nq + W - 1) / W) < 1024) W >>= 1;
  while (W > 1 && W / 2 >= nq) W >>= 1;
  return W;
}

}  // namespace bm
