// Shared-face block geometry of the In-cache Block levels (Sec. IV-A) and
// the constants of the face-fixed correction, used by the block kernels of
// the transform and of its transpose.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bm {

template <int B>
struct Geo {
  static constexpr int BB = B * B;
  static constexpr int MC = (B + 1) / 2;        // coarse nodes per axis
  static constexpr int MI = MC - 2;             // interior coarse nodes per axis
  static constexpr int NB = B <= 9 ? 3 : 1;     // blocks per workgroup
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

}  // namespace bm
