// Lossless stage: canonical Huffman coding of the quantization codes
// (the paper's pipeline ends with Huffman stages for outliers, histogram,
// codebook, encoding; Sec. IV-B).
//
// Symbols: q + 2^15 for |q| < 2^15, else the escape symbol 0 with the
// value q kept as an outlier, in raster order: an outlier's position is
// that of its escape symbol, and per-chunk outlier offsets locate the
// outliers of each chunk (stream version 3).  Code lengths come from
// Huffman's algorithm merging the two smallest (weight, smallest symbol in
// the subtree) keys, so the tree is unique; lengths above 32 are cut to 32
// and the longest codes below 32 are lengthened (largest symbol first) until
// Kraft's sum is <= 1.  Codes are canonical in (length, symbol) order.
// The stream is cut into chunks of 4096 symbols, each packed MSB-first into
// 32-bit words and starting on a word boundary.
//
// GPU work: an LDS-privatised histogram; bit counts and encode with a
// workgroup of 256 threads per chunk (16 consecutive symbols per thread,
// their bit offsets from a workgroup scan, LDS atomic ORs into the chunk's
// words); decode with four wavefronts per chunk.  Decoding a chunk is split
// over its 256 lanes by bit position: lane l owns the codewords that start in
// the l-th 1/256 of the chunk's bits.  Where that first codeword starts is
// only known once lane l - 1 has decoded, so every lane first decodes its part
// from a guessed start (the part's first bit) and hands its end position to
// the next lane; the hand-over is repeated, re-decoding only the lanes whose
// start changed, until no start changes, which is the exact decomposition
// (the fixed point of "start of lane l + 1 = end of lane l from the start of
// lane l", reached in at most 256 rounds).  Huffman codes resynchronise within
// a few codewords from a wrong start, so a few rounds are the rule
// (self-synchronising parallel decoding, as in Weissenberger and Schmidt,
// ICPP 2018).  The codebook is built on the host.

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <mutex>

#include "internal.h"

namespace bm {
namespace {

constexpr int R = 1 << 15;
constexpr int NSYM = 2 * R;
constexpr int CHUNK = 4096;
constexpr int LMAX = 32;
constexpr int HW = 4096;             // LDS histogram window: symbols [R - HW, R + HW)
constexpr int DLB = 11;              // decode lookup bits
constexpr int ET = 256;              // threads per chunk in the bit count and the encode
constexpr int EPT = CHUNK / ET;      // consecutive symbols per thread there
constexpr uint32_t kNoPos = 0xFFFFFFFFu;   // decode position after an invalid code
constexpr size_t kLdsCap = 64 * 1024;      // LDS bytes a decode workgroup may take

using clk = std::chrono::steady_clock;
inline double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

__device__ inline uint32_t sym_of(int32_t q) { return (q > -R && q < R) ? uint32_t(q + R) : 0u; }

// LDS bins: [0, 2 HW) for symbols R-HW .. R+HW-1, bin 2 HW for the escape
// symbol; everything else (rare) goes straight to the global histogram.
__global__ __launch_bounds__(256) void k_hist(const int32_t* codes, int64_t n, unsigned long long* hist) {
  __shared__ uint32_t h[2 * HW + 1];
  for (int i = threadIdx.x; i < 2 * HW + 1; i += 256) h[i] = 0;
  __syncthreads();
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const uint32_t s = sym_of(codes[i]);
    const int64_t k = int64_t(s) - (R - HW);
    if (s == 0)
      atomicAdd(&h[2 * HW], 1u);
    else if (k >= 0 && k < 2 * HW)
      atomicAdd(&h[k], 1u);
    else
      atomicAdd(&hist[s], 1ull);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * HW; i += 256)
    if (h[i]) atomicAdd(&hist[R - HW + i], (unsigned long long)h[i]);
  if (threadIdx.x == 0 && h[2 * HW]) atomicAdd(&hist[0], (unsigned long long)h[2 * HW]);
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) p[i] = 0;
}

__device__ inline uint32_t wave_incl_scan(uint32_t v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

__device__ inline uint32_t wave_excl_scan(uint32_t v, int lane) { return wave_incl_scan(v, lane) - v; }

// The EPT consecutive codes [i0, i0 + EPT) of a chunk of cnt codes at p
// (0 past cnt); VEC: 16-byte loads (p is 16-byte aligned).
template <bool VEC>
__device__ inline void load_run(const int32_t* p, int i0, int cnt, int32_t (&q)[EPT]) {
  if (VEC && i0 + EPT <= cnt) {
    const int4* v = reinterpret_cast<const int4*>(p + i0);
#pragma unroll
    for (int k = 0; k < EPT / 4; ++k) {
      const int4 w = v[k];
      q[4 * k] = w.x;
      q[4 * k + 1] = w.y;
      q[4 * k + 2] = w.z;
      q[4 * k + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < EPT; ++k) q[k] = i0 + k < cnt ? p[i0 + k] : 0;
  }
}

// bits and escapes of each chunk (a workgroup per chunk)
template <bool VEC>
__global__ __launch_bounds__(ET) void k_chunk_bits(const int32_t* codes, int64_t n, const uint8_t* len,
                                                   uint32_t* bits, uint32_t* esc) {
  __shared__ uint32_t part[2][ET / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t c = blockIdx.x, b0 = c * CHUNK;
  const int cnt = int(b0 + CHUNK < n ? CHUNK : n - b0);
  int32_t q[EPT];
  load_run<VEC>(codes + b0, EPT * t, cnt, q);
  uint32_t nb = 0, ne = 0;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    if (EPT * t + k < cnt) {
      const uint32_t s = sym_of(q[k]);
      nb += len[s];
      ne += s == 0;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    nb += __shfl_down(nb, off, 64);
    ne += __shfl_down(ne, off, 64);
  }
  if (lane == 0) {
    part[0][wave] = nb;
    part[1][wave] = ne;
  }
  __syncthreads();
  if (t == 0) {
    uint32_t sb = 0, se = 0;
    for (int w = 0; w < ET / 64; ++w) {
      sb += part[0][w];
      se += part[1][w];
    }
    bits[c] = sb;
    esc[c] = se;
  }
}

// a 32-bit little-endian store; BYTES: four byte stores (a destination that
// is not 4-byte aligned)
template <bool BYTES>
__device__ inline void store32(void* base, uint64_t i, uint32_t v) {
  if (BYTES) {
    uint8_t* p = static_cast<uint8_t*>(base) + 4 * i;
    p[0] = uint8_t(v);
    p[1] = uint8_t(v >> 8);
    p[2] = uint8_t(v >> 16);
    p[3] = uint8_t(v >> 24);
  } else {
    static_cast<uint32_t*>(base)[i] = v;
  }
}

// A workgroup per chunk; thread t codes symbols [16 t, 16 t + 16) of the
// chunk at the bit offset a workgroup scan of the code lengths gives, OR-ing
// each code into the chunk's words in LDS (dynamic size: the longest chunk's
// words).  Code lengths and codes are looked up for all 16 symbols before any
// is placed, so the table reads overlap.
template <bool BYTES, bool VEC>
__global__ __launch_bounds__(ET) void k_encode(const int32_t* codes, int64_t n, const uint8_t* len,
                                               const uint32_t* cw, const uint64_t* woff, const uint64_t* ooff,
                                               void* words, void* oval) {
  extern __shared__ uint32_t out[];
  __shared__ uint32_t part[2][ET / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t c = blockIdx.x, b0 = c * CHUNK;
  const int cnt = int(b0 + CHUNK < n ? CHUNK : n - b0);
  const uint64_t w0 = woff[c];
  const uint32_t nw = uint32_t(woff[c + 1] - w0);
  for (uint32_t i = t; i < nw; i += ET) out[i] = 0;
  int32_t q[EPT];
  load_run<VEC>(codes + b0, EPT * t, cnt, q);
  uint32_t l[EPT], v[EPT];
  uint32_t nb = 0, ne = 0;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    l[k] = 0;
    v[k] = 0;
    if (EPT * t + k < cnt) {
      const uint32_t s = sym_of(q[k]);
      l[k] = len[s];
      v[k] = cw[s];
      ne += s == 0;
    }
    nb += l[k];
  }
  const uint32_t ib = wave_incl_scan(nb, lane), ie = wave_incl_scan(ne, lane);
  if (lane == 63) {
    part[0][wave] = ib;
    part[1][wave] = ie;
  }
  __syncthreads();
  uint32_t p = ib - nb, pe = ie - ne;
  for (int w = 0; w < wave; ++w) {
    p += part[0][w];
    pe += part[1][w];
  }
  uint64_t e = ooff[c] + pe;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    if (l[k] == 0) break;   // past the chunk's end (a coded symbol has a length >= 1)
    const uint32_t w = p >> 5, o = p & 31;
    if (o + l[k] <= 32) {
      atomicOr(&out[w], v[k] << (32 - o - l[k]));
    } else {
      atomicOr(&out[w], v[k] >> (o + l[k] - 32));
      atomicOr(&out[w + 1], v[k] << (64 - o - l[k]));
    }
    p += l[k];
    if (q[k] <= -R || q[k] >= R) store32<BYTES>(oval, e++, uint32_t(q[k]));
  }
  __syncthreads();
  for (uint32_t i = t; i < nw; i += ET) store32<BYTES>(words, w0 + i, out[i]);
}

// ------------------------------------------------------------------ decode
// Tables (built on the host from the code lengths):
// * lut[2^DLB], indexed by the next DLB bits: for a code of l <= DLB bits,
//   its symbol | l << 16; for a prefix whose codes all
//   have one length l > DLB and fill it, kOne | the index of its first code
//   | l << 16 (the code's index is that plus the l - DLB bits after the
//   prefix); for any other prefix of longer codes, kLong | Lmin << 16 |
//   Lmax << 24, the shortest and longest code lengths with that prefix; 0 for
//   a prefix of no code;
// * lastc[L]: the largest 32-bit left-justified code value of length <= L
//   (codes are canonical, so a code of length L is the 32-bit window w with
//   lastc[L - 1] < w <= lastc[L]);
// * offs[L]: index in canonical order of a code of length L minus its value;
// * sorted16: the coded symbols in canonical order (device memory).
constexpr uint32_t kLong = 0x80000000u;
constexpr uint32_t kOne = 0x40000000u;
constexpr int kDecHdrWords = (1 << DLB) + 2 * (LMAX + 1);

struct DecTables {
  const uint32_t* hdr;        // [kDecHdrWords]: lut, lastc, offs
  const uint16_t* sorted16;   // coded symbols in (length, symbol) order
  uint32_t nsorted;           // their count (>= 1)
  uint32_t escidx;            // index of the escape symbol in canonical order (nsorted: none)
};

struct DecLds {
  const uint32_t* lut;
  const uint32_t* lastc;
  const uint32_t* offs;
};

// Decodes the codewords of a chunk that start at x and after, while they
// start before hi.  wl: the chunk's words in LDS followed by two zero words.
// Returns the position of the first codeword at or past hi (x itself when
// x >= hi), or kNoPos at an invalid code; ns counts the codewords decoded.
// With EMIT, emit(k, v, lng, e) receives for the k-th code its symbol (lng
// false: a code of at most DLB bits) or its index in canonical order (lng
// true) and the position where it ends.  Each step reads the two words under
// the position (one LDS instruction) and shifts them, so a step is a dozen
// vector instructions; an invalid code ends the loop through its condition
// (pos = kNoPos), so the loop has a single exit and the common path no branch
// but the rare long-code one.
template <bool EMIT, typename Emit>
__device__ inline uint32_t decode_run(const uint32_t* wl, const DecLds& d, uint32_t x, uint32_t hi, uint32_t& ns,
                                      Emit emit) {
  ns = 0;
  uint32_t pos = x;
  while (pos < hi) {
    const uint32_t i = pos >> 5;   // i + 1 <= nw while pos < hi <= 32 nw
    const uint64_t win = (uint64_t(wl[i]) << 32) | wl[i + 1];
    const uint32_t top = uint32_t((win << (pos & 31)) >> 32);
    const uint32_t lu = d.lut[top >> (32 - DLB)];
    uint32_t l = (lu >> 16) & 63u, v = lu & 0xFFFFu;
    if (lu & kLong) {   // a prefix of codes of several lengths, or one they do not fill (rare)
      const uint32_t lmax = (lu >> 24) & 63u;
      uint32_t lc = d.lastc[l];
      while (top > lc && l < lmax) lc = d.lastc[++l];
      if (EMIT) v = d.offs[l] + (top >> (32 - l));
      if (top > lc) l = 0;
    } else if (EMIT && (lu & kOne)) {
      v += (top << DLB) >> (32 - l + DLB);
    }
    const bool valid = l != 0;
    if (EMIT && valid) emit(ns, v, l > DLB, pos + l);
    ns += valid;
    pos = valid ? pos + l : kNoPos;
  }
  return pos;
}

// Decode: CPW chunks per workgroup, WPC wavefronts (NL = 64 WPC lanes) per
// chunk; chunk lane L owns the codewords that start in the L-th 1/NL of the
// chunk's bits.  LDS: the tables (shared), then per chunk its words
// (wcap + 2), a bit mask of the tile's long codes, a tile of its 4096 symbols
// (uint16; for a code longer than DLB bits its index in canonical order) and
// a small control block.  Rounds of the start hand-over end with workgroup
// barriers (lane 63 of a wavefront hands its end to lane 0 of the next
// through LDS).  The tile is turned into codes by the chunk's wavefronts, a
// segment of 4096 / WPC positions each, 256 at a time: the long codes'
// symbols gathered from sorted16 (only the lanes that hold one load), then
// stored 64 consecutive codes per instruction; an escape's position in the
// chunk goes to rel (in outlier order) and k_outliers puts the outlier values
// in place afterwards, so no lane waits for a load from the outlier array.
// A chunk whose symbols do not decode from its own words (an invalid code,
// too few codewords, a codeword that runs past the chunk's last word) or
// whose escapes do not match its outlier count raises the flag (the caller
// then fails); bits after the chunk's last symbol are not read as symbols.
constexpr int kCtl = 20;   // control words per chunk: hand-over [4], first bad lane [4], wave totals [8], escapes [4]

template <int WPC, int CPW>
__global__ __launch_bounds__(64 * WPC * CPW) void k_decode(const uint32_t* words, const uint64_t* woff, int64_t nch,
                                                           int64_t n, DecTables t, const uint64_t* ooff,
                                                           uint16_t* rel, int32_t* codes, int* err, int wcap) {
  static_assert(WPC == 1 || WPC == 2 || WPC == 4, "1, 2 or 4 wavefronts per chunk");
  constexpr int NL = 64 * WPC, SEG = CHUNK / WPC;
  extern __shared__ uint32_t smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int slot = wave / WPC, wic = wave % WPC, L = wic * 64 + lane;
  const int per = wcap + 2 + CHUNK / 32 + CHUNK / 2 + kCtl;
  uint32_t* flag = smem + kDecHdrWords;                     // [2] workgroup: a start changed in the round
  uint32_t* wl = smem + kDecHdrWords + 2 + slot * per;      // chunk words, two zero words
  uint32_t* lmask = wl + wcap + 2;
  uint16_t* tile = reinterpret_cast<uint16_t*>(lmask + CHUNK / 32);
  uint32_t* ctl = lmask + CHUNK / 32 + CHUNK / 2;
  uint32_t* xch = ctl;        // [WPC] end of each wavefront's lane 63
  uint32_t* fbad = ctl + 4;   // [WPC] first lane of each wavefront that met an invalid code (64: none)
  uint32_t* wtot = ctl + 8;   // [WPC] codewords of each wavefront; [WPC] of lanes up to the first bad one
  uint32_t* esc = ctl + 16;   // [WPC] escapes in each tile segment
  for (int i = tid; i < kDecHdrWords; i += 64 * WPC * CPW) smem[i] = t.hdr[i];
  if (tid < 2) flag[tid] = 0;
  const int64_t c = int64_t(blockIdx.x) * CPW + slot;
  const bool valid = c < nch;   // uniform over the chunk's wavefronts
  uint64_t w0 = 0;
  uint32_t nw = 0;
  if (valid) {
    w0 = woff[c];
    nw = uint32_t(woff[c + 1] - w0);   // <= wcap (checked on the host)
  }
  for (uint32_t i = L; i < nw + 2; i += NL) wl[i] = i < nw ? words[w0 + i] : 0u;
  for (int i = L; i < CHUNK / 32; i += NL) lmask[i] = 0;
  if (L < kCtl) ctl[L] = 0;
  __syncthreads();
  const DecLds d{smem, smem + (1 << DLB), smem + (1 << DLB) + (LMAX + 1)};
  const int64_t b0 = c * CHUNK;
  const uint32_t cnt = valid ? uint32_t(b0 + CHUNK < n ? CHUNK : n - b0) : 0u;
  const uint32_t NB = nw * 32, S = max((NB + NL - 1) / NL, 32u);
  const uint32_t lo = min(uint32_t(L) * S, NB), hi = min(lo + S, NB);
  auto none = [](uint32_t, uint32_t, bool, uint32_t) {};
  // The lanes' start positions: guessed, then handed over until they hold.
  // A lane whose predecessor met an invalid code keeps its own start (a
  // wrong start of the predecessor is the likely cause); lanes up to the
  // first one that ends in an invalid code hold exact starts at the fixed
  // point, and only their symbols are used.
  // Later rounds decode only the lanes whose start changed.
  uint32_t x = lo, ns = 0, end = 0;
  bool ok = false, dirty = true;
  for (int round = 0; round <= NL; ++round) {
    if (dirty) end = decode_run<false>(wl, d, x, hi, ns, none);
    if (lane == 63) xch[wic] = end;
    __syncthreads();
    uint32_t xn = __shfl_up(end, 1, 64);
    if (lane == 0) xn = wic ? xch[wic - 1] : 0u;
    if (xn == kNoPos) xn = x;
    dirty = xn != x;
    if (__any(dirty) && lane == 0) atomicOr(&flag[round & 1], 1u);
    __syncthreads();
    const bool again = flag[round & 1] != 0;
    if (tid == 0) flag[(round + 1) & 1] = 0;
    x = xn;
    if (!again) {
      ok = true;
      break;
    }
  }
  // lanes past the chunk's first one that ends in an invalid code are not used
  const uint64_t badm = __ballot(end == kNoPos);
  const uint32_t fb = badm ? uint32_t(__ffsll((unsigned long long)badm) - 1) : 64u;
  const uint32_t incl = wave_incl_scan(ns, lane);
  if (lane == 63) {
    fbad[wic] = fb;
    wtot[wic] = incl;
  }
  if (fb < 64 && uint32_t(lane) == fb) wtot[4 + wic] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0, lastw = WPC;
  for (int w = 0; w < WPC; ++w) {
    if (lastw == WPC && fbad[w] < 64) lastw = uint32_t(w);
    if (w < wic) before += wtot[w];
  }
  for (int w = 0; w < WPC; ++w) {
    if (uint32_t(w) < lastw) total += wtot[w];
    if (uint32_t(w) == lastw) total += wtot[4 + w];
  }
  const bool used = uint32_t(wic) < lastw || (uint32_t(wic) == lastw && uint32_t(lane) <= fbad[wic]);
  const uint32_t start = before + incl - ns;
  const bool good = valid && ok && total >= cnt;   // uniform over the chunk
  if (valid && !good && L == 0) atomicOr(err, 1);
  bool over = false;   // a codeword of the chunk's symbols runs past its words
  uint32_t ne[WPC] = {};
  if (good && used)
    decode_run<true>(wl, d, x, hi, ns, [&](uint32_t k, uint32_t v, bool lng, uint32_t e) {
      const uint32_t i = start + k;
      if (i < cnt) {
        tile[i] = uint16_t(v);
        if (lng) atomicOr(&lmask[i >> 5], 1u << (i & 31));
        over |= e > NB;
        if (lng ? v == t.escidx : v == 0) {
#pragma unroll
          for (int w = 0; w < WPC; ++w) ne[w] += i / SEG == uint32_t(w);
        }
      }
    });
#pragma unroll
  for (int w = 0; w < WPC; ++w)
    if (ne[w]) atomicAdd(&esc[w], ne[w]);
  if (__any(over) && lane == 0) atomicOr(err, 1);
  __syncthreads();
  if (!good) return;   // no barrier follows
  uint64_t run = ooff[c];
  for (int w = 0; w < wic; ++w) run += esc[w];
  const uint64_t e1 = ooff[c + 1];
  const uint32_t s0 = uint32_t(wic) * SEG, s1 = min(s0 + SEG, cnt);
  for (uint32_t k0 = s0; k0 < s1; k0 += 256) {
    uint32_t s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t i = k0 + 64 * j + lane;
      s[j] = 1u;
      if (i < s1) {
        s[j] = tile[i];
        if ((lmask[i >> 5] >> (i & 31)) & 1u) s[j] = t.sorted16[min(s[j], t.nsorted - 1)];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t i = k0 + 64 * j + lane;
      const uint64_t m = __ballot(s[j] == 0);
      if (s[j] == 0) {
        const uint64_t ei = run + __popcll(m & ((uint64_t(1) << lane) - 1));
        if (ei < e1) rel[ei] = uint16_t(i);
      }
      if (i < s1) codes[b0 + i] = int32_t(s[j]) - R;
      run += __popcll(m);
    }
  }
  // the segment's escapes as counted in the write pass, and all of them the chunk's count
  uint64_t upto = ooff[c];
  for (int w = 0; w <= wic; ++w) upto += esc[w];
  if (lane == 0 && (run != upto || (wic == WPC - 1 && upto != e1))) atomicOr(err, 1);
}

// The outlier values of each chunk to their positions (a workgroup per
// chunk).  Positions are bounded by the chunk's length: a chunk that failed
// to decode may have left its entries of rel unset (the call then fails).
__global__ __launch_bounds__(256) void k_outliers(const uint64_t* ooff, const uint16_t* rel, const int32_t* oval,
                                                  int32_t* codes, int64_t n) {
  const int64_t c = blockIdx.x, b0 = c * CHUNK;
  const uint32_t cnt = uint32_t(b0 + CHUNK < n ? CHUNK : n - b0);
  const uint64_t e0 = ooff[c], e1 = ooff[c + 1];
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const uint32_t r = rel[e];
    if (r < cnt) codes[b0 + r] = oval[e];
  }
}

// ------------------------------------------------------------------ host codebook
// The codebook is built in fixed arrays (no allocation), so the same code
// serves the entry point that may not allocate.

// Work arrays of the code-length construction: the leaves sorted by key
// (weight, symbol), the merged nodes in the order they are made, parents and
// depths of the merge tree.
struct HNode {
  uint64_t w;     // weight
  uint32_t m;     // smallest symbol in the subtree
  uint32_t id;    // node: a symbol, or NSYM + merge number
};
struct LenWork {
  HNode leaf[NSYM], tmp[NSYM], node[NSYM];
  uint32_t digit[2048];
  int32_t parent[2 * NSYM], depth[2 * NSYM], L[NSYM], present[NSYM];
};

inline bool key_less(const HNode& a, const HNode& b) { return a.w != b.w ? a.w < b.w : a.m < b.m; }

// Huffman code lengths of the symbols with hist[s] > 0 (len[s] = 0 for the
// others): merge the two smallest (weight, smallest symbol in the subtree)
// keys until one tree remains; lengths above 32 are cut to 32 and the
// longest codes below 32 are lengthened (largest symbol first) until Kraft's
// sum is <= 1.  The keys are unique, so the tree is.  Two sorted queues give
// the smallest keys in O(n): the leaves sorted by key (a stable radix sort by
// weight of the symbols in ascending order), and the merged nodes in the
// order they are made, which is key order too: merges take keys in
// increasing order, so merged weights do not decrease, and two merged nodes
// of one weight 2w both come from pairs of weight-w nodes taken in
// increasing symbol order, so their smallest symbols increase.
void code_lengths(const uint64_t* hist, uint8_t* len, LenWork& w) {
  std::memset(len, 0, NSYM);
  int np = 0;
  uint64_t wmax = 0;
  for (int s = 0; s < NSYM; ++s)
    if (hist[s]) {
      w.present[np++] = s;
      wmax = std::max(wmax, hist[s]);
    }
  if (np == 0) return;
  if (np == 1) {
    len[w.present[0]] = 1;
    return;
  }
  HNode* A = w.leaf;
  HNode* T = w.tmp;
  for (int k = 0; k < np; ++k) A[k] = HNode{hist[w.present[k]], uint32_t(w.present[k]), uint32_t(w.present[k])};
  for (int sh = 0; sh < 64 && (wmax >> sh) != 0; sh += 11) {   // stable LSD passes of 11 bits
    std::memset(w.digit, 0, sizeof(w.digit));
    for (int k = 0; k < np; ++k) ++w.digit[(A[k].w >> sh) & 2047u];
    uint32_t sum = 0;
    for (int d = 0; d < 2048; ++d) {
      const uint32_t c = w.digit[d];
      w.digit[d] = sum;
      sum += c;
    }
    for (int k = 0; k < np; ++k) T[w.digit[(A[k].w >> sh) & 2047u]++] = A[k];
    std::swap(A, T);
  }
  HNode* B = w.node;
  int ai = 0, bi = 0, bn = 0;
  auto pop = [&]() -> HNode {
    if (ai < np && (bi >= bn || key_less(A[ai], B[bi]))) return A[ai++];
    return B[bi++];
  };
  int next = NSYM;
  for (int k = 0; k < np - 1; ++k) {
    const HNode a = pop(), b = pop();
    w.parent[a.id] = next;
    w.parent[b.id] = next;
    B[bn++] = HNode{a.w + b.w, std::min(a.m, b.m), uint32_t(next)};
    ++next;
  }
  w.depth[next - 1] = 0;
  for (int v = next - 2; v >= NSYM; --v) w.depth[v] = w.depth[w.parent[v]] + 1;  // parents come after children
  int maxl = 0;
  for (int k = 0; k < np; ++k) {
    const int s = w.present[k];
    w.L[s] = w.depth[w.parent[s]] + 1;
    maxl = std::max(maxl, w.L[s]);
  }
  if (maxl > LMAX) {
    uint64_t kraft = 0;
    for (int k = 0; k < np; ++k) {
      const int s = w.present[k];
      if (w.L[s] > LMAX) w.L[s] = LMAX;
      kraft += uint64_t(1) << (LMAX - w.L[s]);
    }
    while (kraft > (uint64_t(1) << LMAX)) {
      int best = -1;
      for (int k = 0; k < np; ++k) {
        const int s = w.present[k];
        if (w.L[s] < LMAX && (best < 0 || w.L[s] > w.L[best] || (w.L[s] == w.L[best] && s > best))) best = s;
      }
      kraft -= uint64_t(1) << (LMAX - w.L[best] - 1);
      w.L[best] += 1;
    }
  }
  for (int k = 0; k < np; ++k) len[w.present[k]] = uint8_t(w.L[w.present[k]]);
}

// Canonical codes in (length, symbol) order; sorted receives the coded
// symbols in that order (a counting sort by length), *nsorted their count.
void canonical(const uint8_t* len, uint32_t* code, uint32_t* sorted, int* nsorted) {
  std::memset(code, 0, NSYM * sizeof(uint32_t));
  uint32_t at[LMAX + 2] = {};
  for (int s = 0; s < NSYM; ++s)
    if (len[s]) ++at[len[s] + 1];
  for (int l = 1; l <= LMAX; ++l) at[l + 1] += at[l];
  const int n = int(at[LMAX + 1]);
  for (int s = 0; s < NSYM; ++s)
    if (len[s]) sorted[at[len[s]]++] = uint32_t(s);
  uint64_t c = 0;
  int prev = 0;
  for (int i = 0; i < n; ++i) {
    const int l = len[sorted[i]];
    if (i) c = (c + 1) << (l - prev);
    code[sorted[i]] = uint32_t(c);
    prev = l;
  }
  *nsorted = n;
}

// stream header; the code-length table lists present symbols only:
// uint16 symbol[npresent] (ascending), then uint8 length[npresent]
struct HuffHeader {
  uint32_t magic, version;
  int64_t n, nchunks, nwords, noutliers, npresent;
};
constexpr uint32_t kHuffMagic = 0x46484D42u;   // "BMHF"

template <typename T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(size_t n) {
    if (n) BM_HIP(hipMalloc(&p, n * sizeof(T)));
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    BM_HIP(hipEventCreate(&a));
    BM_HIP(hipEventCreate(&b));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  double ms() const {
    BM_HIP(hipEventSynchronize(b));
    float t = 0.f;
    BM_HIP(hipEventElapsedTime(&t, a, b));
    return double(t);
  }
};

thread_local bm_lossless_times g_times{};

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

void launch_chunk_bits(const int32_t* codes, int64_t n, int64_t nch, const uint8_t* len, uint32_t* bits,
                       uint32_t* esc, hipStream_t st) {
  if (!nch) return;
  if (aligned16(codes))
    hipLaunchKernelGGL(k_chunk_bits<true>, dim3(unsigned(nch)), dim3(ET), 0, st, codes, n, len, bits, esc);
  else
    hipLaunchKernelGGL(k_chunk_bits<false>, dim3(unsigned(nch)), dim3(ET), 0, st, codes, n, len, bits, esc);
  BM_HIP(hipGetLastError());
}

void launch_encode(const int32_t* codes, int64_t n, int64_t nch, const uint8_t* len, const uint32_t* cw,
                   const uint64_t* woff, const uint64_t* ooff, uint64_t wmax, void* words, void* oval,
                   hipStream_t st) {
  if (!nch) return;
  const size_t shm = size_t(wmax) * 4;
  const bool bytes = (reinterpret_cast<uintptr_t>(words) & 3) != 0;   // oval - words is a multiple of 4
  const bool vec = aligned16(codes);
  const dim3 g{unsigned(nch)}, b{unsigned(ET)};
  if (bytes && vec)
    hipLaunchKernelGGL((k_encode<true, true>), g, b, shm, st, codes, n, len, cw, woff, ooff, words, oval);
  else if (bytes)
    hipLaunchKernelGGL((k_encode<true, false>), g, b, shm, st, codes, n, len, cw, woff, ooff, words, oval);
  else if (vec)
    hipLaunchKernelGGL((k_encode<false, true>), g, b, shm, st, codes, n, len, cw, woff, ooff, words, oval);
  else
    hipLaunchKernelGGL((k_encode<false, false>), g, b, shm, st, codes, n, len, cw, woff, ooff, words, oval);
  BM_HIP(hipGetLastError());
}

constexpr int kDecWpc = 4;   // wavefronts per chunk in the decode
constexpr int kDecCpw = 2;   // chunks per decode workgroup

template <int WPC, int CPW>
void launch_decode(const uint32_t* words, const uint64_t* woff, int64_t nch, int64_t n, const DecTables& t,
                   const uint64_t* ooff, uint16_t* rel, int32_t* codes, int* err, int wcap, hipStream_t st) {
  // LDS: tables, two flags, then per chunk its words (+2), long-code mask, tile and control block
  const size_t per = size_t(wcap) + 2 + CHUNK / 32 + CHUNK / 2 + kCtl;
  const size_t bytes = (size_t(kDecHdrWords) + 2 + CPW * per) * 4;
  if (bytes > kLdsCap) fail(BM_EUNSUPPORTED, "decode workgroup does not fit in LDS");
  hipLaunchKernelGGL((k_decode<WPC, CPW>), dim3(unsigned((nch + CPW - 1) / CPW)), dim3(64 * WPC * CPW), bytes, st,
                     words, woff, nch, n, t, ooff, rel, codes, err, wcap);
}

// CRC-32 (the reflected polynomial 0xEDB88320 with pre- and post-inversion,
// as zlib) of every 16 KiB block of the code words: each lane takes 64
// consecutive bytes with a four-table byte-slicing update, then the
// workgroup folds its 256 lane CRCs in order by a tree whose level k moves
// the left CRC over the right part's 64 * 2^k bytes (crc(A B) = Z(crc(A)) ^
// crc(B), Z linear over GF(2): its 32 columns come with the launch).
struct CrcTree {
  uint32_t m[8][32];
};

__device__ inline uint32_t gf2_mul(const uint32_t (&m)[32], uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 32; ++i)
    if ((v >> i) & 1u) r ^= m[i];
  return r;
}

__global__ __launch_bounds__(256) void k_crc_blocks(const uint4* words, CrcTree t, uint32_t* out) {
  static_assert(kCrcBlock == 256 * 64, "one 64-byte run per lane");
  __shared__ uint32_t tab[4][256];
  __shared__ uint32_t s[256];
  const int tid = threadIdx.x;
  const uint4* q = words + (size_t(blockIdx.x) * 256 + tid) * 4;
  uint4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = q[k];
  uint32_t c = uint32_t(tid);
#pragma unroll
  for (int k = 0; k < 8; ++k) c = (c & 1u) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
  tab[0][tid] = c;
  __syncthreads();
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    c = (c >> 8) ^ tab[0][c & 0xFFu];
    tab[k][tid] = c;
  }
  __syncthreads();
  uint32_t crc = 0xFFFFFFFFu;
  auto step = [&](uint32_t w) {
    crc ^= w;
    crc = tab[3][crc & 0xFFu] ^ tab[2][(crc >> 8) & 0xFFu] ^ tab[1][(crc >> 16) & 0xFFu] ^ tab[0][crc >> 24];
  };
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    step(v[k].x);
    step(v[k].y);
    step(v[k].z);
    step(v[k].w);
  }
  s[tid] = ~crc;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int w = 1 << k;
    if ((tid & (2 * w - 1)) == 0) s[tid] = gf2_mul(t.m[k], s[tid]) ^ s[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[blockIdx.x] = s[0];
}

}  // namespace

// ------------------------------------------------------------------ encoder
// One plan per code array: histogram (device), code lengths and canonical
// codes (host), per-chunk bit and escape counts (device), word and outlier
// offsets (host).  write() encodes with that plan.
struct HuffmanEncoder::Impl {
  const int32_t* codes;
  int64_t n, nch;
  hipStream_t st;
  std::vector<uint8_t> len;
  std::vector<uint32_t> cw, sorted;
  std::vector<uint64_t> woff, ooff;
  std::vector<uint16_t> psym;
  std::vector<uint8_t> plen;
  uint64_t wmax = 0;
  size_t bytes = 0;
  CrcSpan span[2];      // the last write's words and outlier values
  DevBuf<uint8_t> dlen{NSYM};
  DevBuf<uint32_t> dcw{NSYM};
  Impl(const int32_t* c, int64_t n_, hipStream_t s) : codes(c), n(n_), nch((n_ + CHUNK - 1) / CHUNK), st(s) {}
};

HuffmanEncoder::HuffmanEncoder(const int32_t* codes, int64_t n, hipStream_t st) {
  if (n < 0 || (n > 0 && !codes)) fail(BM_EINVAL, "bad code array");
  d_ = std::make_unique<Impl>(codes, n, st);
  Impl& I = *d_;
  bm_lossless_times& T = g_times;
  T.enc_n = n;
  T.enc_hist_ms = T.enc_table_ms = T.enc_sizes_ms = T.enc_encode_ms = T.enc_copy_ms = T.enc_crc_ms = 0.0;
  const int64_t nch = I.nch;
  DevBuf<unsigned long long> hist(NSYM);
  EventPair eh, eb;
  BM_HIP(hipEventRecord(eh.a, st));
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, st, hist.p, int64_t(NSYM));
  if (n) {
    const int64_t g = std::min<int64_t>(2048, (n + 255) / 256);
    hipLaunchKernelGGL(k_hist, dim3(unsigned(g)), dim3(256), 0, st, codes, n, hist.p);
  }
  BM_HIP(hipGetLastError());
  BM_HIP(hipEventRecord(eh.b, st));
  std::vector<uint64_t> h(NSYM);
  BM_HIP(hipMemcpyAsync(h.data(), hist.p, NSYM * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  T.enc_hist_ms = eh.ms();
  const auto t1 = clk::now();
  {
    auto work = std::make_unique<LenWork>();
    I.len.assign(NSYM, 0);
    code_lengths(h.data(), I.len.data(), *work);
  }
  I.cw.assign(NSYM, 0);
  I.sorted.assign(NSYM, 0);
  int ns = 0;
  canonical(I.len.data(), I.cw.data(), I.sorted.data(), &ns);
  I.sorted.resize(ns);
  for (int s = 0; s < NSYM; ++s)
    if (I.len[s]) {
      I.psym.push_back(uint16_t(s));
      I.plen.push_back(I.len[s]);
    }
  T.enc_table_ms = ms_since(t1);
  const auto t2 = clk::now();
  BM_HIP(hipMemcpyAsync(I.dlen.p, I.len.data(), NSYM, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(I.dcw.p, I.cw.data(), NSYM * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  DevBuf<uint32_t> bits(size_t(std::max<int64_t>(nch, 1))), esc(size_t(std::max<int64_t>(nch, 1)));
  BM_HIP(hipEventRecord(eb.a, st));
  launch_chunk_bits(codes, n, nch, I.dlen.p, bits.p, esc.p, st);
  BM_HIP(hipEventRecord(eb.b, st));
  std::vector<uint32_t> hb(nch), he(nch);
  if (nch) {
    BM_HIP(hipMemcpyAsync(hb.data(), bits.p, nch * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    BM_HIP(hipMemcpyAsync(he.data(), esc.p, nch * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  }
  BM_HIP(hipStreamSynchronize(st));
  I.woff.assign(nch + 1, 0);
  I.ooff.assign(nch + 1, 0);
  for (int64_t c = 0; c < nch; ++c) {
    const uint64_t w = (uint64_t(hb[c]) + 31) / 32;
    I.wmax = std::max(I.wmax, w);
    I.woff[c + 1] = I.woff[c] + w;
    I.ooff[c + 1] = I.ooff[c] + he[c];
  }
  T.enc_sizes_ms = ms_since(t2);
  I.bytes = sizeof(HuffHeader) + I.psym.size() * 3 + size_t(nch + 1) * 16 + size_t(I.woff[nch]) * 4 +
            size_t(I.ooff[nch]) * 4;
}

HuffmanEncoder::~HuffmanEncoder() = default;

size_t HuffmanEncoder::bytes() const { return d_->bytes; }
const CrcSpan (&HuffmanEncoder::device_spans() const)[2] { return d_->span; }

namespace {
// the columns of the tree's shifts over 64, 128, ..., 8192 zero bytes
const CrcTree& crc_tree() {
  static const CrcTree t = [] {
    CrcTree r{};
    for (int k = 0; k < 8; ++k) crc32_shift_matrix(uint64_t(64) << k, r.m[k]);
    return r;
  }();
  return t;
}
}  // namespace

void HuffmanEncoder::write(uint8_t* dst, size_t capacity) {
  Impl& I = *d_;
  bm_lossless_times& T = g_times;
  if (I.bytes > capacity) fail(BM_ECAPACITY, "Huffman stream larger than its buffer");
  const int64_t nch = I.nch, nw = int64_t(I.woff[nch]), nout = int64_t(I.ooff[nch]);
  const int64_t np = int64_t(I.psym.size());
  DevBuf<uint64_t> dwoff(nch + 1), dooff(nch + 1);
  DevBuf<uint32_t> dwords(size_t(std::max<int64_t>(nw, 1)));
  DevBuf<int32_t> doval(size_t(std::max<int64_t>(nout, 1)));
  BM_HIP(hipMemcpyAsync(dwoff.p, I.woff.data(), (nch + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, I.st));
  BM_HIP(hipMemcpyAsync(dooff.p, I.ooff.data(), (nch + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, I.st));
  EventPair ee, ec;
  BM_HIP(hipEventRecord(ee.a, I.st));
  launch_encode(I.codes, I.n, nch, I.dlen.p, I.dcw.p, dwoff.p, dooff.p, I.wmax, dwords.p, doval.p, I.st);
  // the CRC-32 of every whole 16 KiB block of the words and of the outlier
  // values, while they are on the device
  const void* dsrc[2] = {dwords.p, doval.p};
  const size_t dbytes[2] = {size_t(nw) * 4, size_t(nout) * 4};
  size_t nblk[2];
  for (int k = 0; k < 2; ++k) nblk[k] = dbytes[k] / kCrcBlock;
  DevBuf<uint32_t> dcrc(std::max<size_t>(nblk[0] + nblk[1], 1));
  for (int k = 0; k < 2; ++k) {
    I.span[k].bytes = dbytes[k];
    I.span[k].block_crc.assign(nblk[k], 0u);
    if (!nblk[k]) continue;
    if (nblk[k] >= (size_t(1) << 31)) fail(BM_EUNSUPPORTED, "Huffman stream too large");
    hipLaunchKernelGGL(k_crc_blocks, dim3(unsigned(nblk[k])), dim3(256), 0, I.st, static_cast<const uint4*>(dsrc[k]),
                       crc_tree(), dcrc.p + (k ? nblk[0] : 0));
    BM_HIP(hipGetLastError());
  }
  BM_HIP(hipEventRecord(ee.b, I.st));
  HuffHeader hh{kHuffMagic, 3, I.n, nch, nw, nout, np};
  uint8_t* o = dst;
  std::memcpy(o, &hh, sizeof(hh));
  o += sizeof(hh);
  if (np) std::memcpy(o, I.psym.data(), size_t(np) * 2);
  o += size_t(np) * 2;
  if (np) std::memcpy(o, I.plen.data(), size_t(np));
  o += size_t(np);
  std::memcpy(o, I.woff.data(), (nch + 1) * 8);
  o += (nch + 1) * 8;
  std::memcpy(o, I.ooff.data(), (nch + 1) * 8);
  o += (nch + 1) * 8;
  BM_HIP(hipEventRecord(ec.a, I.st));
  I.span[0].offset = size_t(o - dst);
  if (nw) BM_HIP(hipMemcpyAsync(o, dwords.p, size_t(nw) * 4, hipMemcpyDeviceToHost, I.st));
  for (int k = 0; k < 2; ++k)
    if (nblk[k])
      BM_HIP(hipMemcpyAsync(I.span[k].block_crc.data(), dcrc.p + (k ? nblk[0] : 0), nblk[k] * 4, hipMemcpyDeviceToHost,
                            I.st));
  o += size_t(nw) * 4;
  I.span[1].offset = size_t(o - dst);
  if (nout) BM_HIP(hipMemcpyAsync(o, doval.p, size_t(nout) * 4, hipMemcpyDeviceToHost, I.st));
  BM_HIP(hipEventRecord(ec.b, I.st));
  BM_HIP(hipStreamSynchronize(I.st));
  T.enc_encode_ms = ee.ms();
  T.enc_copy_ms = ec.ms();
}

size_t huffman_size(const int32_t* codes, int64_t n, hipStream_t st) { return HuffmanEncoder(codes, n, st).bytes(); }

size_t huffman_encode(const int32_t* codes, int64_t n, std::vector<uint8_t>& out, hipStream_t st) {
  HuffmanEncoder e(codes, n, st);
  out.resize(e.bytes());
  e.write(out.data(), out.size());
  return out.size();
}

void set_lossless_crc_ms(double ms) { g_times.enc_crc_ms = ms; }

void huffman_code_lengths(const uint64_t* hist, uint8_t* len) {
  auto work = std::make_unique<LenWork>();
  code_lengths(hist, len, *work);
}

bm_lossless_times lossless_times() { return g_times; }

// ------------------------------------------------------------------ decode (host)
struct HuffmanDecoder::Impl {
  hipStream_t st;
  const uint8_t* in;
  size_t in_bytes;
  int64_t n = 0, nch = 0, nw = 0, nout = 0;
  uint64_t wcap = 0;
  CrcSpan span[2];
  std::vector<uint32_t> hdr;
  std::vector<uint16_t> sorted16;
  std::vector<uint64_t> woff, ooff;
  uint32_t escidx = 0;
  std::unique_ptr<DevBuf<uint32_t>> dhdr, dwords;
  std::unique_ptr<DevBuf<uint16_t>> dsorted, drel;
  std::unique_ptr<DevBuf<uint64_t>> dwoff, dooff;
  std::unique_ptr<DevBuf<int32_t>> doval;
  std::unique_ptr<DevBuf<int>> derr;
  EventPair eu;
  Impl(const uint8_t* i, size_t ib, hipStream_t s) : st(s), in(i), in_bytes(ib) {}
};

HuffmanDecoder::~HuffmanDecoder() = default;

HuffmanDecoder::HuffmanDecoder(const uint8_t* in, size_t in_bytes, hipStream_t st) {
  d_ = std::make_unique<Impl>(in, in_bytes, st);
  Impl& I = *d_;
  bm_lossless_times& T = g_times;
  T.dec_parse_ms = T.dec_upload_ms = T.dec_decode_ms = 0.0;
  const auto t0 = clk::now();
  if (!in || in_bytes < sizeof(HuffHeader)) fail(BM_ECORRUPT, "Huffman stream too short");
  HuffHeader hh;
  std::memcpy(&hh, in, sizeof(hh));
  if (hh.magic != kHuffMagic || hh.version != 3) fail(BM_ECORRUPT, "bad Huffman stream header");
  const int64_t n = hh.n;
  if (n < 0 || hh.nchunks != (n + CHUNK - 1) / CHUNK || hh.nwords < 0 || hh.noutliers < 0 || hh.noutliers > n ||
      hh.npresent < 0 || hh.npresent > NSYM || hh.nwords > (int64_t(1) << 40))
    fail(BM_ECORRUPT, "inconsistent Huffman stream header");
  const int64_t nch = hh.nchunks, nw = hh.nwords, nout = hh.noutliers, np = hh.npresent;
  const size_t need = sizeof(hh) + size_t(np) * 3 + size_t(nch + 1) * 16 + size_t(nw) * 4 + size_t(nout) * 4;
  if (in_bytes < need) fail(BM_ECORRUPT, "Huffman stream truncated");
  const uint8_t* p = in + sizeof(hh);
  std::vector<uint8_t> len(NSYM, 0);
  {
    std::vector<uint16_t> psym(np);
    if (np) std::memcpy(psym.data(), p, size_t(np) * 2);
    for (int64_t k = 0; k < np; ++k) {
      if (k && psym[k] <= psym[k - 1]) fail(BM_ECORRUPT, "code table symbols out of order");
      len[psym[k]] = p[size_t(np) * 2 + k];
      if (len[psym[k]] == 0) fail(BM_ECORRUPT, "zero code length in the table");
    }
  }
  p += size_t(np) * 3;
  std::vector<uint64_t>& woff = I.woff;
  woff.resize(nch + 1);
  std::memcpy(woff.data(), p, (nch + 1) * 8);
  p += (nch + 1) * 8;
  std::vector<uint64_t>& ooff = I.ooff;
  ooff.resize(nch + 1);
  std::memcpy(ooff.data(), p, (nch + 1) * 8);
  p += (nch + 1) * 8;
  if (woff[0] != 0 || ooff[0] != 0 || ooff[nch] != uint64_t(nout)) fail(BM_ECORRUPT, "bad chunk offsets");
  uint64_t wcap = 0;
  for (int64_t c = 0; c < nch; ++c) {
    const uint64_t cnt = uint64_t(std::min<int64_t>(CHUNK, n - c * CHUNK));
    // a chunk of cnt symbols has at most 32 cnt bits
    if (woff[c + 1] < woff[c] || woff[c + 1] > uint64_t(nw) || woff[c + 1] - woff[c] > cnt ||
        ooff[c + 1] < ooff[c] || ooff[c + 1] - ooff[c] > cnt)
      fail(BM_ECORRUPT, "bad chunk offsets");
    wcap = std::max(wcap, woff[c + 1] - woff[c]);
  }
  uint64_t kraft = 0;
  for (int s = 0; s < NSYM; ++s) {
    if (len[s] > LMAX) fail(BM_ECORRUPT, "code length above 32");
    if (len[s]) kraft += uint64_t(1) << (LMAX - len[s]);
  }
  if (kraft > (uint64_t(1) << LMAX)) fail(BM_ECORRUPT, "code lengths violate Kraft's inequality");
  std::vector<uint32_t> cw(NSYM), sorted(NSYM);
  int ns = 0;
  canonical(len.data(), cw.data(), sorted.data(), &ns);
  sorted.resize(ns);
  // decode tables (layout at k_decode)
  std::vector<uint32_t>& hdr = I.hdr;
  hdr.assign(kDecHdrWords, 0);
  std::vector<uint16_t>& sorted16 = I.sorted16;
  sorted16.assign(std::max<size_t>(sorted.size(), 1), 0);
  {
    uint32_t* lut = hdr.data();
    uint32_t* lastc = lut + (1 << DLB);
    uint32_t* offs = lastc + (LMAX + 1);
    uint32_t first[LMAX + 1] = {}, count[LMAX + 1] = {}, base[LMAX + 1] = {};
    for (size_t i = 0; i < sorted.size(); ++i) {
      const uint32_t s = sorted[i], l = len[s];
      sorted16[i] = uint16_t(s);
      if (count[l] == 0) {
        first[l] = cw[s];
        base[l] = uint32_t(i);
      }
      ++count[l];
      if (l <= DLB) {
        const uint32_t lo = cw[s] << (DLB - l), span = 1u << (DLB - l);
        for (uint32_t k = 0; k < span; ++k) lut[lo + k] = s | (l << 16);
      } else {
        uint32_t& e = lut[cw[s] >> (l - DLB)];
        e = e ? ((e & ~(63u << 24)) | (l << 24)) : (kLong | (l << 16) | (l << 24) | uint32_t(i));
      }
    }
    // prefixes of one code length whose codes fill them: length and first index in the entry
    for (uint32_t pf = 0; pf < (1u << DLB); ++pf) {
      const uint32_t e = lut[pf];
      if (!(e & kLong)) continue;
      const uint32_t lmin = (e >> 16) & 63u, lmax = (e >> 24) & 63u, i0 = e & 0xFFFFu;
      if (lmin != lmax || i0 + (1u << (lmin - DLB)) > uint32_t(sorted.size())) continue;
      const uint32_t s0 = sorted[i0], sl = sorted[i0 + (1u << (lmin - DLB)) - 1];
      // the prefix's first code starts it; the 2^(l - DLB)-th code of length l from there ends it
      if (len[sl] == lmin && (cw[s0] >> (lmin - DLB)) == pf && (cw[sl] >> (lmin - DLB)) == pf)
        lut[pf] = kOne | i0 | (lmin << 16);
    }
    uint64_t end = 0;   // left-justified end of the codes of length <= L
    for (int l = 1; l <= LMAX; ++l) {
      if (count[l]) end = (uint64_t(first[l]) + count[l]) << (LMAX - l);
      lastc[l] = end ? uint32_t(end - 1) : 0u;
      offs[l] = base[l] - first[l];
    }
  }
  T.dec_parse_ms = ms_since(t0);
  I.n = n;
  I.nch = nch;
  I.nw = nw;
  I.nout = nout;
  I.wcap = wcap;
  I.dhdr = std::make_unique<DevBuf<uint32_t>>(hdr.size());
  I.dsorted = std::make_unique<DevBuf<uint16_t>>(sorted16.size());
  I.dwoff = std::make_unique<DevBuf<uint64_t>>(nch + 1);
  I.dooff = std::make_unique<DevBuf<uint64_t>>(nch + 1);
  I.dwords = std::make_unique<DevBuf<uint32_t>>(size_t(std::max<int64_t>(nw, 1)));
  I.doval = std::make_unique<DevBuf<int32_t>>(size_t(std::max<int64_t>(nout, 1)));
  I.drel = std::make_unique<DevBuf<uint16_t>>(size_t(std::max<int64_t>(nout, 1)));
  I.derr = std::make_unique<DevBuf<int>>(1);
  BM_HIP(hipEventRecord(I.eu.a, st));
  BM_HIP(hipMemcpyAsync(I.dhdr->p, hdr.data(), hdr.size() * 4, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(I.dsorted->p, sorted16.data(), sorted16.size() * 2, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(I.dwoff->p, woff.data(), (nch + 1) * 8, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(I.dooff->p, ooff.data(), (nch + 1) * 8, hipMemcpyHostToDevice, st));
  I.span[0].offset = size_t(p - in);
  I.span[0].bytes = size_t(nw) * 4;
  if (nw) BM_HIP(hipMemcpyAsync(I.dwords->p, p, size_t(nw) * 4, hipMemcpyHostToDevice, st));
  p += size_t(nw) * 4;
  I.span[1].offset = size_t(p - in);
  I.span[1].bytes = size_t(nout) * 4;
  if (nout) BM_HIP(hipMemcpyAsync(I.doval->p, p, size_t(nout) * 4, hipMemcpyHostToDevice, st));
  BM_HIP(hipEventRecord(I.eu.b, st));
  I.escidx = uint32_t(sorted16.size());
  for (size_t i = 0; i < sorted.size(); ++i)
    if (sorted[i] == 0) I.escidx = uint32_t(i);
}

uint32_t HuffmanDecoder::crc(uint32_t crc) {
  Impl& I = *d_;
  const void* src[2] = {I.dwords->p, I.doval->p};
  size_t nblk[2];
  for (int k = 0; k < 2; ++k) nblk[k] = I.span[k].bytes / kCrcBlock;
  DevBuf<uint32_t> dcrc(std::max<size_t>(nblk[0] + nblk[1], 1));
  for (int k = 0; k < 2; ++k) {
    I.span[k].block_crc.assign(nblk[k], 0u);
    if (!nblk[k]) continue;
    if (nblk[k] >= (size_t(1) << 31)) fail(BM_EUNSUPPORTED, "Huffman stream too large");
    hipLaunchKernelGGL(k_crc_blocks, dim3(unsigned(nblk[k])), dim3(256), 0, I.st, static_cast<const uint4*>(src[k]),
                       crc_tree(), dcrc.p + (k ? nblk[0] : 0));
    BM_HIP(hipGetLastError());
    BM_HIP(hipMemcpyAsync(I.span[k].block_crc.data(), dcrc.p + (k ? nblk[0] : 0), nblk[k] * 4,
                          hipMemcpyDeviceToHost, I.st));
  }
  BM_HIP(hipStreamSynchronize(I.st));
  return crc_with_spans(I.in, I.in_bytes, crc, I.span, 2);
}

void HuffmanDecoder::decode(int32_t* codes, int64_t n) {
  Impl& I = *d_;
  bm_lossless_times& T = g_times;
  if (I.n != n) fail(BM_EINVAL, "symbol count does not match the destination");
  T.dec_n = n;
  const int64_t nch = I.nch;
  const DecTables t{I.dhdr->p, I.dsorted->p, uint32_t(I.sorted16.size()), I.escidx};
  const int zero = 0;
  BM_HIP(hipMemcpyAsync(I.derr->p, &zero, sizeof(int), hipMemcpyHostToDevice, I.st));
  EventPair ed;
  BM_HIP(hipEventRecord(ed.a, I.st));
  if (nch) {
    launch_decode<kDecWpc, kDecCpw>(I.dwords->p, I.dwoff->p, nch, n, t, I.dooff->p, I.drel->p, codes, I.derr->p,
                                    int(I.wcap), I.st);
    BM_HIP(hipGetLastError());
    if (I.nout)
      hipLaunchKernelGGL(k_outliers, dim3(unsigned(nch)), dim3(256), 0, I.st, I.dooff->p, I.drel->p, I.doval->p, codes,
                         n);
    BM_HIP(hipGetLastError());
  }
  BM_HIP(hipEventRecord(ed.b, I.st));
  int herr = 0;
  BM_HIP(hipMemcpyAsync(&herr, I.derr->p, sizeof(int), hipMemcpyDeviceToHost, I.st));
  BM_HIP(hipStreamSynchronize(I.st));
  T.dec_upload_ms = I.eu.ms();
  T.dec_decode_ms = ed.ms();
  if (herr) fail(BM_ECORRUPT, "Huffman stream does not decode");
}

void huffman_decode(const uint8_t* in, size_t in_bytes, int32_t* codes, int64_t n, hipStream_t st) {
  if (!in || in_bytes < sizeof(HuffHeader)) fail(BM_ECORRUPT, "Huffman stream too short");
  HuffHeader hh;
  std::memcpy(&hh, in, sizeof(hh));
  if (hh.magic == kHuffMagic && hh.version == 3 && hh.n != n)
    fail(BM_EINVAL, "symbol count does not match the destination");
  HuffmanDecoder d(in, in_bytes, st);
  d.decode(codes, n);
}

// ------------------------------------------------------------------ stage times
// The encoder's stages timed one by one (the lossless part of the time model
// of Algorithm 1): histogram, code table, chunk sizes + encode, copy-out + CRC.
void huffman_stage_times(const int32_t* codes, int64_t n, hipStream_t st, double ms[4]) {
  HuffmanEncoder e(codes, n, st);
  std::vector<uint8_t> out(e.bytes());
  e.write(out.data(), out.size());
  const auto t0 = clk::now();
  volatile uint32_t crc = stream_crc(e, out.data(), out.size(), 0);
  (void)crc;
  const double crc_ms = ms_since(t0);
  const bm_lossless_times& T = g_times;
  ms[0] = T.enc_hist_ms;
  ms[1] = T.enc_table_ms;
  ms[2] = T.enc_sizes_ms + T.enc_encode_ms;
  ms[3] = T.enc_copy_ms + crc_ms;
}

// ------------------------------------------------------------------ no allocation
// Huffman encoding into a device buffer with every work array fixed in size:
// device scratch in one file-scope array (per GPU, held until the process
// ends), host work arrays static.  Calls share both, so they are serialised
// by a mutex on the host; calls on one GPU must not overlap in time (they
// share that GPU's scratch).

namespace {

constexpr int64_t kNoAllocMaxCh = kNoAllocMaxCodes / CHUNK;
constexpr size_t kScrHist = 0;                                         // uint64 [NSYM]
constexpr size_t kScrLen = kScrHist + size_t(NSYM) * 8;                // uint8  [NSYM]
constexpr size_t kScrCw = kScrLen + size_t(NSYM);                      // uint32 [NSYM]
constexpr size_t kScrBits = kScrCw + size_t(NSYM) * 4;                 // uint32 [chunks]
constexpr size_t kScrEsc = kScrBits + size_t(kNoAllocMaxCh) * 4;       // uint32 [chunks]
constexpr size_t kScrWoff = kScrEsc + size_t(kNoAllocMaxCh) * 4;       // uint64 [chunks + 1]
constexpr size_t kScrOoff = kScrWoff + size_t(kNoAllocMaxCh + 1) * 8;  // uint64 [chunks + 1]
constexpr size_t kScratchBytes = kScrOoff + size_t(kNoAllocMaxCh + 1) * 8;
static_assert(kScrCw % 4 == 0 && kScrWoff % 8 == 0 && kScrOoff % 8 == 0, "scratch alignment");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct NoAllocHost {
  uint64_t hist[NSYM];
  uint8_t len[NSYM];
  uint32_t cw[NSYM], sorted[NSYM];
  uint16_t psym[NSYM];
  uint8_t plen[NSYM];
  uint32_t bits[kNoAllocMaxCh], esc[kNoAllocMaxCh];
  uint64_t woff[kNoAllocMaxCh + 1], ooff[kNoAllocMaxCh + 1];
  LenWork work;
};
NoAllocHost g_na;
std::mutex g_na_mu;
constexpr int kMaxDevices = 64;
unsigned char* g_scratch[kMaxDevices] = {};   // each GPU's copy of `scratch` (device address)

unsigned char* scratch_ptr() {
  int dev = 0;
  BM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(BM_EUNSUPPORTED, "device index beyond 63");
  if (!g_scratch[dev]) {
    void* p = nullptr;
    BM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  return g_scratch[dev];
}

}  // namespace

size_t huffman_encode_noalloc(const int32_t* codes, int64_t n, void* out, size_t capacity, size_t* out_bytes,
                              hipStream_t st) {
  if (n < 0 || n > kNoAllocMaxCodes) fail(BM_EINVAL, "n outside [0, 2^28] for the entry point that does not allocate");
  if (n > 0 && !codes) fail(BM_EINVAL, "null codes");
  std::lock_guard<std::mutex> lock(g_na_mu);
  NoAllocHost& H = g_na;
  unsigned char* scr = scratch_ptr();
  auto* hist = reinterpret_cast<unsigned long long*>(scr + kScrHist);
  auto* dlen = scr + kScrLen;
  auto* dcw = reinterpret_cast<uint32_t*>(scr + kScrCw);
  auto* bits = reinterpret_cast<uint32_t*>(scr + kScrBits);
  auto* esc = reinterpret_cast<uint32_t*>(scr + kScrEsc);
  auto* dwoff = reinterpret_cast<uint64_t*>(scr + kScrWoff);
  auto* dooff = reinterpret_cast<uint64_t*>(scr + kScrOoff);
  const int64_t nch = (n + CHUNK - 1) / CHUNK;
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, st, hist, int64_t(NSYM));
  if (n) {
    const int64_t g = std::min<int64_t>(2048, (n + 255) / 256);
    hipLaunchKernelGGL(k_hist, dim3(unsigned(g)), dim3(256), 0, st, codes, n, hist);
  }
  BM_HIP(hipGetLastError());
  BM_HIP(hipMemcpyAsync(H.hist, hist, sizeof(H.hist), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  code_lengths(H.hist, H.len, H.work);
  int ns = 0;
  canonical(H.len, H.cw, H.sorted, &ns);
  BM_HIP(hipMemcpyAsync(dlen, H.len, sizeof(H.len), hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dcw, H.cw, sizeof(H.cw), hipMemcpyHostToDevice, st));
  launch_chunk_bits(codes, n, nch, dlen, bits, esc, st);
  if (nch) {
    BM_HIP(hipMemcpyAsync(H.bits, bits, size_t(nch) * 4, hipMemcpyDeviceToHost, st));
    BM_HIP(hipMemcpyAsync(H.esc, esc, size_t(nch) * 4, hipMemcpyDeviceToHost, st));
  }
  BM_HIP(hipStreamSynchronize(st));
  H.woff[0] = 0;
  H.ooff[0] = 0;
  uint64_t wmax = 0;
  for (int64_t c = 0; c < nch; ++c) {
    const uint64_t w = (uint64_t(H.bits[c]) + 31) / 32;
    wmax = std::max(wmax, w);
    H.woff[c + 1] = H.woff[c] + w;
    H.ooff[c + 1] = H.ooff[c] + H.esc[c];
  }
  int64_t np = 0;
  for (int s = 0; s < NSYM; ++s)
    if (H.len[s]) {
      H.psym[np] = uint16_t(s);
      H.plen[np] = H.len[s];
      ++np;
    }
  const int64_t nw = int64_t(H.woff[nch]), nout = int64_t(H.ooff[nch]);
  HuffHeader hh{kHuffMagic, 3, n, nch, nw, nout, np};
  const size_t off_tab = sizeof(hh), off_off = off_tab + size_t(np) * 3;
  const size_t off_words = off_off + size_t(nch + 1) * 16, off_out = off_words + size_t(nw) * 4;
  const size_t bytes = off_out + size_t(nout) * 4;
  *out_bytes = bytes;
  if (!out || capacity < bytes) fail(BM_ECAPACITY, "output buffer too small");
  uint8_t* o = static_cast<uint8_t*>(out);
  BM_HIP(hipMemcpyAsync(o, &hh, sizeof(hh), hipMemcpyHostToDevice, st));
  if (np) {
    BM_HIP(hipMemcpyAsync(o + off_tab, H.psym, size_t(np) * 2, hipMemcpyHostToDevice, st));
    BM_HIP(hipMemcpyAsync(o + off_tab + size_t(np) * 2, H.plen, size_t(np), hipMemcpyHostToDevice, st));
  }
  BM_HIP(hipMemcpyAsync(o + off_off, H.woff, size_t(nch + 1) * 8, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(o + off_off + size_t(nch + 1) * 8, H.ooff, size_t(nch + 1) * 8, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dwoff, H.woff, size_t(nch + 1) * 8, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dooff, H.ooff, size_t(nch + 1) * 8, hipMemcpyHostToDevice, st));
  launch_encode(codes, n, nch, dlen, dcw, dwoff, dooff, wmax, o + off_words, o + off_out, st);
  BM_HIP(hipStreamSynchronize(st));
  return bytes;
}

}  // namespace bm
