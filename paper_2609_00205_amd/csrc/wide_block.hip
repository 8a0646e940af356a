// In-cache Block levels with b = 33 (Sec. IV-A; the block sizes of the
// hybrid hierarchy, Sec. IV-B).
//
// The level is the same face-fixed block step as for b = 9 and 17 (details
// from the multilinear interpolant of the block's coarse nodes; correction
// z = K_x K_y K_z w over the 15 interior coarse rows per axis; every node
// written once, by its owner).  A 33^3 block does not fit one workgroup the
// way a 17^3 block does: one z-column per lane would take 1089 lanes, and the
// FP64 block alone is 281 KiB, more than a CU's LDS.  So the block is cut
// along x into two halves of 17 columns, x in [0, 16] and [16, 32] (column 16
// is computed by both and stored by the first), and a level runs as
//   columns  per half: z-columns in registers; the multilinear details from
//            the half's coarse nodes (LDS); the z pass into LDS; the y pass,
//            whose 15 x 15 values per column go to a scratch array;
//   coarse   per block: the x pass over that array, then the 15^3 interior
//            coarse nodes of the compact coarse grid: decomposition adds z to
//            u_C, recomposition turns c into u_C = c - z in place;
//   interp   per half, recomposition only: u = interpolant(u_C) + w.
// Compared with the one-kernel 17^3 form this moves 15/33 of a value per
// node (the y-pass result) through HBM twice more, and the recomposition
// reads its coefficients twice.

#include <algorithm>
#include <cstring>

#include "block.h"
#include "internal.h"

namespace bm {
namespace {

constexpr int B = 33;
constexpr int MC = Geo<B>::MC;        // 17 coarse nodes per axis
constexpr int MI = Geo<B>::MI;        // 15 interior coarse nodes per axis
constexpr int HW = 17;                // columns per half along x
constexpr int HC = 9;                 // coarse columns per half along x
constexpr int NCOL = B * HW;          // 561 columns per half
constexpr int NT1 = 576;              // lanes of a half's workgroup (9 wavefronts)
constexpr int NT2 = 256;              // lanes of a block's coarse-node workgroup
constexpr int T2B = MI * MI * B;      // scratch values per block

template <typename T>
struct WideArgs {
  // decomposition source (level 1: the logical input, read with clamp or zero fill)
  const T* src;
  int64_t sn[3], ss[3];
  int first, zero_pad;
  // this level's coefficients (in place in the padded array), or their codes
  T* coeff;
  int32_t* codes;
  int64_t cs[3];
  // compact coarse grid G^s
  T* cgrid;
  int64_t cn[3];
  // y-pass result per block, [MI][MI][B]
  T* t2;
  // recomposition output (cropped to on)
  T* out;
  int64_t on[3], os[3];
  int64_t nb[3];
  uint32_t nblocks;
  int64_t per1, per2;     // XCD runs of the half and block launches
  FastDiv fnb2, fnb1;
  QTab tab, ctab;
  int coarsest_here;
  int64_t* flag;
};

// dequantized (or plain) coefficients of one block column, in registers
template <typename T, bool Q>
__device__ inline void load_coeff_column(const WideArgs<T>& a, uint32_t blk, int y, int x, int64_t off, T (&w)[B]) {
  if (!Q) {
    const T* col = a.coeff + off;
#pragma unroll
    for (int z = 0; z < B; ++z) w[z] = col[z * a.cs[0]];
  } else {
    const int32_t* col = a.codes + off;
    int32_t qv[B];
#pragma unroll
    for (int z = 0; z < B; ++z) qv[z] = col[z * a.cs[0]];
    double dd[3];
    column_class<B>(a.tab.cdel, blk, y, x, dd);
#pragma unroll
    for (int z = 0; z < B; ++z) w[z] = T(mul_rn(double(qv[z]), dd[zcase<B>(z)]));
  }
}

// Column step: block half g (block g/2, half g%2) with NT1 lanes; lds holds
// MI * B * HW values (decomposition: the half's coarse nodes UC[MC][MC][HC],
// then T1[MI][B][HW]).
template <typename T, bool DEC, bool Q>
__device__ __attribute__((always_inline)) inline void wide_columns(const WideArgs<T>& a, int64_t g, T* lds) {
  const uint32_t blk = uint32_t(g >> 1);
  const int h = int(g & 1);
  const int tid = threadIdx.x;
  const bool act = tid < NCOL;
  const int y = act ? tid / HW : 0, xl = act ? tid - (tid / HW) * HW : 0;
  const int x = 16 * h + xl;
  int64_t bz, by, bx;
  block_coords(blk, a.fnb2, a.fnb1, a.nb, bz, by, bx);
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  const bool ecol = ((y | x) & 1) == 0;
  // stored by this half (column 16 by the first), then the shared-face rule
  const bool own = act && (h == 0 || xl > 0) && (y < B - 1 || by == a.nb[1] - 1) && (x < B - 1 || bx == a.nb[2] - 1);
  const bool lastz = bz == a.nb[0] - 1;
  const int64_t off = oz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2];
  T v[B];
  if (DEC) {
    T* UC = lds;
    double iv[3];
    if (Q && act) column_class<B>(a.tab.cinv, blk, y, x, iv);
    if (act) {
      if (!a.first || (oz + B <= a.sn[0] && gy < a.sn[1] && gx < a.sn[2])) {
        const T* col = a.src + oz * a.ss[0] + gy * a.ss[1] + gx * a.ss[2];
#pragma unroll
        for (int z = 0; z < B; ++z) v[z] = col[z * a.ss[0]];
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
      if (ecol) {
#pragma unroll
        for (int j = 0; j < MC; ++j) UC[(j * MC + (y >> 1)) * HC + (xl >> 1)] = v[2 * j];
      }
    }
    __syncthreads();
    if (act) {
      // details u - interpolant, final at once; v keeps u_C on the coarse nodes
      const int cy0 = y >> 1, cy1 = (y + 1) >> 1, cx0 = xl >> 1, cx1 = (xl + 1) >> 1;
      T I2[MC];
#pragma unroll
      for (int j = 0; j < MC; ++j) {
        const T* pl = UC + j * MC * HC;
        I2[j] = T(0.25) * ((pl[cy0 * HC + cx0] + pl[cy0 * HC + cx1]) + (pl[cy1 * HC + cx0] + pl[cy1 * HC + cx1]));
      }
#pragma unroll
      for (int z = 0; z < B; ++z) {
        if (z & 1)
          v[z] = v[z] - T(0.5) * (I2[z >> 1] + I2[(z >> 1) + 1]);
        else if (!ecol)
          v[z] = v[z] - I2[z >> 1];
      }
      if (own) {
        // coarse nodes of an even column get a placeholder (u_C, or code 0)
        // that a later level or the coarsest values overwrite; the plane
        // z = B-1 belongs to the next block unless this is the last one
        if (!Q) {
          T* dst = a.coeff + off;
#pragma unroll
          for (int z = 0; z < B - 1; ++z) dst[z * a.cs[0]] = v[z];
          if (lastz) dst[(B - 1) * a.cs[0]] = v[B - 1];
        } else {
          int32_t* dst = a.codes + off;
          unsigned bad = 0;
#pragma unroll
          for (int z = 0; z < B - 1; ++z) dst[z * a.cs[0]] = quant(v[z], iv[zcase<B>(z)], ecol && !(z & 1), bad);
          if (lastz) dst[(B - 1) * a.cs[0]] = quant(v[B - 1], iv[2], ecol, bad);
          if (bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), (unsigned long long)bad);
        }
        if (ecol) {
          // u_C into the compact coarse grid; the coarse kernel adds z
          T* cdst = a.cgrid + ((oz >> 1) * a.cn[1] + (gy >> 1)) * a.cn[2] + (gx >> 1);
#pragma unroll
          for (int j = 0; j < MC - 1; ++j) cdst[j * a.cn[1] * a.cn[2]] = v[2 * j];
          if (lastz) cdst[(MC - 1) * a.cn[1] * a.cn[2]] = v[B - 1];
        }
      }
#pragma unroll
      for (int z = 0; z < B; z += 2)
        if (ecol) v[z] = T(0);   // w is zero on the coarse nodes
    }
    __syncthreads();             // UC is dead: T1 takes its place
  } else {
    if (act) {
      load_coeff_column<T, Q>(a, blk, y, x, off, v);
      if (ecol) {
#pragma unroll
        for (int z = 0; z < B; z += 2) v[z] = T(0);
      }
    }
  }
  // z pass of the correction: T1[J][y][xl]
  T* T1 = lds;
  if (act) {
    T o[MI];
    restrict_solve<T, B>(v, o);
#pragma unroll
    for (int J = 0; J < MI; ++J) T1[(J * B + y) * HW + xl] = o[J];
  }
  __syncthreads();
  // y pass over the lines (J, xl) this half stores
  if (tid < MI * HW) {
    const int J = tid / HW, c = tid - (tid / HW) * HW;
    if (h == 0 || c > 0) {
      T line[B], o[MI];
#pragma unroll
      for (int yy = 0; yy < B; ++yy) line[yy] = T1[(J * B + yy) * HW + c];
      restrict_solve<T, B>(line, o);
      T* dst = a.t2 + int64_t(blk) * T2B + J * MI * B + 16 * h + c;
#pragma unroll
      for (int I = 0; I < MI; ++I) dst[I * B] = o[I];
    }
  }
}

template <typename T, bool DEC, bool Q>
__global__ __launch_bounds__(NT1) void k_wide_columns(WideArgs<T> a) {
  __shared__ T lds[MI * B * HW];
  const int64_t g = xcd_group(blockIdx.x, a.per1);
  if (g >= 2 * int64_t(a.nblocks)) return;
  wide_columns<T, DEC, Q>(a, g, lds);
}

// Coarse step: block g with NT2 lanes.  x pass, then the interior coarse
// nodes (and, at the last level of a quantized hierarchy, the codes of all of
// the block's coarse nodes).  S holds T2B values: T2[MI][MI][B]; the x pass
// leaves Z[J][I][K] in the first MI of each row.
template <typename T, bool DEC, bool Q>
__device__ __attribute__((always_inline)) inline void wide_coarse(const WideArgs<T>& a, int64_t g, T* S) {
  const uint32_t blk = uint32_t(g);
  const int tid = threadIdx.x;
  const T* src = a.t2 + int64_t(blk) * T2B;
  for (int i = tid; i < T2B; i += NT2) S[i] = src[i];
  __syncthreads();
  if (tid < MI * MI) {
    T line[B], o[MI];
#pragma unroll
    for (int x = 0; x < B; ++x) line[x] = S[tid * B + x];
    restrict_solve<T, B>(line, o);
#pragma unroll
    for (int K = 0; K < MI; ++K) S[tid * B + K] = o[K];   // the row is this lane's alone
  }
  __syncthreads();
  int64_t bz, by, bx;
  block_coords(blk, a.fnb2, a.fnb1, a.nb, bz, by, bx);
  const int64_t c0 = bz * (MC - 1), c1 = by * (MC - 1), c2 = bx * (MC - 1);
  const int64_t cpl = a.cn[1] * a.cn[2];
  if (!(Q && a.coarsest_here)) {
    for (int i = tid; i < MI * MI * MI; i += NT2) {
      const int J = i / (MI * MI), r = i - J * MI * MI, I = r / MI, K = r - I * MI;
      T* c = a.cgrid + (c0 + J + 1) * cpl + (c1 + I + 1) * a.cn[2] + (c2 + K + 1);
      const T z = S[(J * MI + I) * B + K];
      *c = DEC ? *c + z : *c - z;
    }
    return;
  }
  // codes of the coarsest values: every coarse node the block owns
  const int64_t oz = bz * (B - 1), oy = by * (B - 1), ox = bx * (B - 1);
  unsigned bad = 0;
  for (int i = tid; i < MC * MC * MC; i += NT2) {
    const int j = i / (MC * MC), r = i - j * MC * MC, k1 = r / MC, k2 = r - k1 * MC;
    const bool owned = (j < MC - 1 || bz == a.nb[0] - 1) && (k1 < MC - 1 || by == a.nb[1] - 1) &&
                       (k2 < MC - 1 || bx == a.nb[2] - 1);
    if (!owned) continue;
    const bool inner = j >= 1 && j <= MC - 2 && k1 >= 1 && k1 <= MC - 2 && k2 >= 1 && k2 <= MC - 2;
    const T z = inner ? S[((j - 1) * MI + (k1 - 1)) * B + (k2 - 1)] : T(0);
    const int cls = pos_class<B>(2 * j) * 9 + pos_class<B>(2 * k1) * 3 + pos_class<B>(2 * k2);
    const int64_t off = (oz + 2 * j) * a.cs[0] + (oy + 2 * k1) * a.cs[1] + (ox + 2 * k2) * a.cs[2];
    T* c = a.cgrid + (c0 + j) * cpl + (c1 + k1) * a.cn[2] + (c2 + k2);
    if (DEC) {
      a.codes[off] = quant(T(*c + z), a.ctab.cinv[int64_t(blk) * 27 + cls], false, bad);
    } else {
      const T cv = T(mul_rn(double(a.codes[off]), a.ctab.cdel[int64_t(blk) * 27 + cls]));
      *c = cv - z;
    }
  }
  if (DEC && bad) atomicOr(reinterpret_cast<unsigned long long*>(a.flag), (unsigned long long)bad);
}

template <typename T, bool DEC, bool Q>
__global__ __launch_bounds__(NT2) void k_wide_coarse(WideArgs<T> a) {
  __shared__ T S[T2B];
  const int64_t g = xcd_group(blockIdx.x, a.per2);
  if (g >= int64_t(a.nblocks)) return;
  wide_coarse<T, DEC, Q>(a, g, S);
}

// Interpolation step of the recomposition: block half g with NT1 lanes; UC
// holds the half's coarse values [MC][MC][HC].  Lanes leave early only after
// the step's one barrier.
template <typename T, bool Q>
__device__ __attribute__((always_inline)) inline void wide_interp(const WideArgs<T>& a, int64_t g, T* UC) {
  const uint32_t blk = uint32_t(g >> 1);
  const int h = int(g & 1);
  const int tid = threadIdx.x;
  int64_t bz, by, bx;
  block_coords(blk, a.fnb2, a.fnb1, a.nb, bz, by, bx);
  const int64_t cpl = a.cn[1] * a.cn[2];
  {
    const T* cs = a.cgrid + bz * (MC - 1) * cpl + by * (MC - 1) * a.cn[2] + bx * (MC - 1) + 8 * h;
    for (int i = tid; i < MC * MC * HC; i += NT1) {
      const int j = i / (MC * HC), r = i - j * MC * HC, I = r / HC, K = r - I * HC;
      UC[i] = cs[j * cpl + I * a.cn[2] + K];
    }
  }
  __syncthreads();
  if (tid >= NCOL) return;
  const int y = tid / HW, xl = tid - (tid / HW) * HW;
  const int x = 16 * h + xl;
  if (h == 1 && xl == 0) return;   // column 16 is the first half's
  const int64_t oz = bz * (B - 1), gy = by * (B - 1) + y, gx = bx * (B - 1) + x;
  const bool owny = (y < B - 1 || by == a.nb[1] - 1) && gy < a.on[1];
  const bool ownx = (x < B - 1 || bx == a.nb[2] - 1) && gx < a.on[2];
  if (!(owny && ownx)) return;
  const bool ecol = ((y | x) & 1) == 0;
  const bool lastz = bz == a.nb[0] - 1;
  T w[B];
  load_coeff_column<T, Q>(a, blk, y, x, oz * a.cs[0] + gy * a.cs[1] + gx * a.cs[2], w);
  // the y-x interpolant of even plane j, formed as the z sweep reaches it
  // (holding all MC planes would spill in FP64)
  const int cy0 = y >> 1, cy1 = (y + 1) >> 1, cx0 = xl >> 1, cx1 = (xl + 1) >> 1;
  auto plane = [&](int j) {
    const T* pl = UC + j * MC * HC;
    return T(0.25) * ((pl[cy0 * HC + cx0] + pl[cy0 * HC + cx1]) + (pl[cy1 * HC + cx0] + pl[cy1 * HC + cx1]));
  };
  T* dst = a.out + oz * a.os[0] + gy * a.os[1] + gx * a.os[2];
  T lo = plane(0);
#pragma unroll
  for (int z = 0; z < B; ++z) {
    T u;
    if (z & 1) {
      const T hi = plane((z >> 1) + 1);
      u = T(0.5) * (lo + hi) + w[z];
      lo = hi;
    } else {
      u = ecol ? lo : lo + w[z];
    }
    if ((z < B - 1 || lastz) && oz + z < a.on[0]) dst[z * a.os[0]] = u;
  }
}

template <typename T, bool Q>
__global__ __launch_bounds__(NT1) void k_wide_interp(WideArgs<T> a) {
  __shared__ T UC[MC * MC * HC];
  const int64_t g = xcd_group(blockIdx.x, a.per1);
  if (g >= 2 * int64_t(a.nblocks)) return;
  wide_interp<T, Q>(a, g, UC);
}

// Many fields in one persistent launch per step: task k is half (columns,
// interp) or block (coarse) k - first[f] of field f; the field index is
// uniform over the workgroup and its record is read with scalar loads.

template <typename T, bool DEC, bool Q>
__global__ __launch_bounds__(NT1) void k_batch_wide_columns(const WideArgs<T>* __restrict__ fa,
                                                            const int64_t* __restrict__ first, int nf,
                                                            int64_t ntasks) {
  __shared__ T lds[MI * B * HW];
  for (int64_t k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const int f = __builtin_amdgcn_readfirstlane(task_field(first, nf, k));
    wide_columns<T, DEC, Q>(fa[f], k - first[f], lds);
    __syncthreads();
  }
}

template <typename T, bool DEC, bool Q>
__global__ __launch_bounds__(NT2) void k_batch_wide_coarse(const WideArgs<T>* __restrict__ fa,
                                                           const int64_t* __restrict__ first, int nf, int64_t ntasks) {
  __shared__ T S[T2B];
  for (int64_t k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const int f = __builtin_amdgcn_readfirstlane(task_field(first, nf, k));
    wide_coarse<T, DEC, Q>(fa[f], k - first[f], S);
    __syncthreads();
  }
}

template <typename T, bool Q>
__global__ __launch_bounds__(NT1) void k_batch_wide_interp(const WideArgs<T>* __restrict__ fa,
                                                           const int64_t* __restrict__ first, int nf, int64_t ntasks) {
  __shared__ T UC[MC * MC * HC];
  for (int64_t k = blockIdx.x; k < ntasks; k += gridDim.x) {
    const int f = __builtin_amdgcn_readfirstlane(task_field(first, nf, k));
    wide_interp<T, Q>(fa[f], k - first[f], UC);
    __syncthreads();
  }
}


template <typename T>
WideArgs<T> wide_args(const bm_plan_s& p, int s, void* coeff, int32_t* codes, void* cgrid, const QPrep* q) {
  const Level& L = p.lv[s - 1];
  WideArgs<T> a{};
  a.coeff = static_cast<T*>(coeff);
  a.codes = codes;
  const View3 cv = level_view(p, s, q ? static_cast<void*>(codes) : coeff);
  for (int k = 0; k < 3; ++k) {
    a.cs[k] = cv.s[k];
    a.cn[k] = L.m[k];
    a.nb[k] = L.nb[k];
  }
  a.cgrid = static_cast<T*>(cgrid);
  const int64_t nblocks = L.nb[0] * L.nb[1] * L.nb[2];
  if (nblocks >= (int64_t(1) << 31)) fail(BM_EUNSUPPORTED, "too many blocks");
  if (size_t(nblocks) * T2B > p.ws.t_elems) fail(BM_EINVAL, "plan workspace too small for 33^3 blocks");
  a.nblocks = uint32_t(nblocks);
  a.t2 = static_cast<T*>(p.ws.t1);
  a.per1 = (2 * nblocks + 7) / 8;
  a.per2 = (nblocks + 7) / 8;
  a.fnb2 = FastDiv(uint32_t(L.nb[2]));
  a.fnb1 = FastDiv(uint32_t(L.nb[1]));
  if (q) {
    a.tab = q->lv[s - 1];
    a.coarsest_here = (p.M == 0 && s == p.L) ? 1 : 0;
    if (a.coarsest_here) a.ctab = q->lv[kCoarseSlotHost];
    a.flag = q->flag;
  }
  return a;
}

template <typename T>
void launch_wide_dec(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout,
                     int32_t* codes, const QPrep* q, hipStream_t st) {
  WideArgs<T> a = wide_args<T>(p, s, coeff, codes, cout, q);
  a.src = static_cast<const T*>(src.ptr);
  for (int k = 0; k < 3; ++k) {
    a.sn[k] = src.n[k];
    a.ss[k] = src.s[k];
  }
  a.first = first;
  a.zero_pad = p.cfg.pad_mode == 1;
  const dim3 g1(unsigned(8 * a.per1)), g2(unsigned(8 * a.per2));
  if (q) {
    hipLaunchKernelGGL((k_wide_columns<T, true, true>), g1, dim3(NT1), 0, st, a);
    hipLaunchKernelGGL((k_wide_coarse<T, true, true>), g2, dim3(NT2), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_wide_columns<T, true, false>), g1, dim3(NT1), 0, st, a);
    hipLaunchKernelGGL((k_wide_coarse<T, true, false>), g2, dim3(NT2), 0, st, a);
  }
  BM_HIP(hipGetLastError());
}

template <typename T>
void launch_wide_rec(const bm_plan_s& p, int s, const void* coeff, void* cin, void* out, bool last,
                     const int32_t* codes, const QPrep* q, hipStream_t st) {
  WideArgs<T> a = wide_args<T>(p, s, const_cast<void*>(coeff), const_cast<int32_t*>(codes), cin, q);
  a.out = static_cast<T*>(out);
  const int64_t* on = last ? p.dims : p.lv[s - 1].n;
  for (int k = 0; k < 3; ++k) a.on[k] = on[k];
  a.os[0] = on[1] * on[2];
  a.os[1] = on[2];
  a.os[2] = 1;
  const dim3 g1(unsigned(8 * a.per1)), g2(unsigned(8 * a.per2));
  if (q) {
    hipLaunchKernelGGL((k_wide_columns<T, false, true>), g1, dim3(NT1), 0, st, a);
    hipLaunchKernelGGL((k_wide_coarse<T, false, true>), g2, dim3(NT2), 0, st, a);
    hipLaunchKernelGGL((k_wide_interp<T, true>), g1, dim3(NT1), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_wide_columns<T, false, false>), g1, dim3(NT1), 0, st, a);
    hipLaunchKernelGGL((k_wide_coarse<T, false, false>), g2, dim3(NT2), 0, st, a);
    hipLaunchKernelGGL((k_wide_interp<T, false>), g1, dim3(NT1), 0, st, a);
  }
  BM_HIP(hipGetLastError());
}

template <typename T>
void wide_batch_args_t(const bm_plan_s& p, int s, bool dec, const View3& src, bool first, void* out, int32_t* codes,
                       const QPrep* q, void* dst) {
  WideArgs<T> a = wide_args<T>(p, s, nullptr, codes, p.ws.grid[s], q);
  if (dec) {
    a.src = static_cast<const T*>(src.ptr);
    for (int k = 0; k < 3; ++k) {
      a.sn[k] = src.n[k];
      a.ss[k] = src.s[k];
    }
    a.first = first;
    a.zero_pad = p.cfg.pad_mode == 1;
  } else {
    a.out = static_cast<T*>(out);
    const int64_t* on = first ? p.dims : p.lv[s - 1].n;
    for (int k = 0; k < 3; ++k) a.on[k] = on[k];
    a.os[0] = on[1] * on[2];
    a.os[1] = on[2];
    a.os[2] = 1;
  }
  std::memcpy(dst, &a, sizeof(a));
}

template <typename T>
void launch_wide_batch_t(bool dec, const void* args, const int64_t* first_half, const int64_t* first_block, int nf,
                         int64_t nhalf, int64_t nblock, hipStream_t st) {
  if (nblock <= 0) return;
  const auto* fa = static_cast<const WideArgs<T>*>(args);
  if (dec) {
    auto kc = k_batch_wide_columns<T, true, true>;
    auto ko = k_batch_wide_coarse<T, true, true>;
    hipLaunchKernelGGL(kc, dim3(resident_grid(kc, NT1, nhalf)), dim3(NT1), 0, st, fa, first_half, nf, nhalf);
    hipLaunchKernelGGL(ko, dim3(resident_grid(ko, NT2, nblock)), dim3(NT2), 0, st, fa, first_block, nf, nblock);
  } else {
    auto kc = k_batch_wide_columns<T, false, true>;
    auto ko = k_batch_wide_coarse<T, false, true>;
    auto ki = k_batch_wide_interp<T, true>;
    hipLaunchKernelGGL(kc, dim3(resident_grid(kc, NT1, nhalf)), dim3(NT1), 0, st, fa, first_half, nf, nhalf);
    hipLaunchKernelGGL(ko, dim3(resident_grid(ko, NT2, nblock)), dim3(NT2), 0, st, fa, first_block, nf, nblock);
    hipLaunchKernelGGL(ki, dim3(resident_grid(ki, NT1, nhalf)), dim3(NT1), 0, st, fa, first_half, nf, nhalf);
  }
  BM_HIP(hipGetLastError());
}

}  // namespace

size_t wide_args_size(const bm_plan_s& p) {
  return p.cfg.dtype == BM_F32 ? sizeof(WideArgs<float>) : sizeof(WideArgs<double>);
}

void wide_batch_args(const bm_plan_s& p, int s, bool dec, const View3& src, bool first, void* out, int32_t* codes,
                     const QPrep* q, void* dst) {
  if (p.lv[s - 1].b != B) fail(BM_EINVAL, "not a 33-node block level");
  if (p.cfg.dtype == BM_F32)
    wide_batch_args_t<float>(p, s, dec, src, first, out, codes, q, dst);
  else
    wide_batch_args_t<double>(p, s, dec, src, first, out, codes, q, dst);
}

void launch_wide_batch(int dtype, bool dec, const void* args, const int64_t* first_half, const int64_t* first_block,
                       int nf, int64_t nhalf, int64_t nblock, hipStream_t st) {
  if (dtype == BM_F32)
    launch_wide_batch_t<float>(dec, args, first_half, first_block, nf, nhalf, nblock, st);
  else
    launch_wide_batch_t<double>(dec, args, first_half, first_block, nf, nhalf, nblock, st);
}

size_t wide_scratch_elems(const int64_t nb[3]) { return size_t(nb[0] * nb[1] * nb[2]) * T2B; }

void wide_decompose(const bm_plan_s& p, int s, const View3& src, bool first, void* coeff, void* cout, int32_t* codes,
                    const QPrep* q, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    launch_wide_dec<float>(p, s, src, first, coeff, cout, codes, q, st);
  else
    launch_wide_dec<double>(p, s, src, first, coeff, cout, codes, q, st);
}

void wide_recompose(const bm_plan_s& p, int s, const void* coeff, void* cin, void* out, bool last,
                    const int32_t* codes, const QPrep* q, hipStream_t st) {
  if (p.cfg.dtype == BM_F32)
    launch_wide_rec<float>(p, s, coeff, cin, out, last, codes, q, st);
  else
    launch_wide_rec<double>(p, s, coeff, cin, out, last, codes, q, st);
}

}  // namespace bm
