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
// GPU work: an LDS-privatised histogram, one wavefront per chunk for the
// bit counts and for the encode (LDS atomic ORs into the chunk's words),
// one thread per chunk for decoding (tables and output staged in LDS).  The
// codebook is built on the host.

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
constexpr int HW = 4096;           // LDS histogram window: symbols [R - HW, R + HW)
constexpr int LUTB = 10;           // decode lookup bits

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

// one wavefront per chunk: bit count and escape count
__global__ __launch_bounds__(64) void k_chunk_bits(const int32_t* codes, int64_t n, const uint8_t* len,
                                                   uint32_t* bits, uint32_t* esc) {
  const int64_t c = blockIdx.x;
  const int64_t b0 = c * CHUNK;
  const int64_t b1 = b0 + CHUNK < n ? b0 + CHUNK : n;
  uint32_t nb = 0, ne = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 64) {
    const uint32_t s = sym_of(codes[i]);
    nb += len[s];
    ne += s == 0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    nb += __shfl_down(nb, off, 64);
    ne += __shfl_down(ne, off, 64);
  }
  if (threadIdx.x == 0) {
    bits[c] = nb;
    esc[c] = ne;
  }
}

__device__ inline uint32_t wave_excl_scan(uint32_t v, int lane) {
  uint32_t s = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(s, off, 64);
    if (lane >= off) s += t;
  }
  return s - v;
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

// one wavefront per chunk; lane l codes symbols [64 l, 64 l + 64) of the chunk
template <bool BYTES = false>
__global__ __launch_bounds__(64) void k_encode(const int32_t* codes, int64_t n, const uint8_t* len,
                                               const uint32_t* cw, const uint64_t* woff, const uint64_t* ooff,
                                               void* words, void* oval) {
  __shared__ uint32_t sym[64 * 65];
  __shared__ uint32_t out[CHUNK];
  const int lane = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int64_t b0 = c * CHUNK;
  const int cnt = int(b0 + CHUNK < n ? CHUNK : n - b0);
  const uint64_t w0 = woff[c], nw = woff[c + 1] - w0;
  for (int i = lane; i < CHUNK; i += 64) sym[(i >> 6) * 65 + (i & 63)] = i < cnt ? sym_of(codes[b0 + i]) : 0xFFFFFFFFu;
  for (uint64_t i = lane; i < nw; i += 64) out[i] = 0;
  __syncthreads();
  uint32_t nb = 0, ne = 0;
  for (int k = 0; k < 64; ++k) {
    const uint32_t s = sym[lane * 65 + k];
    if (s != 0xFFFFFFFFu) {
      nb += len[s];
      ne += s == 0;
    }
  }
  uint32_t p = wave_excl_scan(nb, lane);
  uint64_t e = ooff[c] + wave_excl_scan(ne, lane);
  for (int k = 0; k < 64; ++k) {
    const uint32_t s = sym[lane * 65 + k];
    if (s == 0xFFFFFFFFu) break;
    const uint32_t l = len[s], v = cw[s];
    const uint32_t w = p >> 5, o = p & 31;
    if (o + l <= 32) {
      atomicOr(&out[w], v << (32 - o - l));
    } else {
      atomicOr(&out[w], v >> (o + l - 32));
      atomicOr(&out[w + 1], v << (64 - o - l));
    }
    p += l;
    if (s == 0) store32<BYTES>(oval, e++, uint32_t(codes[b0 + lane * 64 + k]));
  }
  __syncthreads();
  for (uint64_t i = lane; i < nw; i += 64) store32<BYTES>(words, w0 + i, out[i]);
}

struct DecTables {
  const uint32_t* lut;        // [1 << LUTB]: symbol | length << 16 (length 0: longer code)
  const uint32_t* first;      // [LMAX + 1] first canonical code of each length
  const uint32_t* count;      // [LMAX + 1]
  const uint32_t* base;       // [LMAX + 1] index of the first symbol of each length in `sorted`
  const uint32_t* sorted;     // symbols in (length, symbol) order
};

// One thread per chunk, 64 chunks per workgroup.  The lookup tables live in
// LDS; decoded symbols go to an LDS tile 64 at a time per lane, and the tile
// is stored one lane's run at a time, so every store instruction writes 64
// consecutive codes (a lane writing straight to its own chunk would put the
// 64 lanes of a store 16 KiB apart).  A lane that meets a malformed stream
// raises the flag and decodes nothing more (the caller then fails).
__global__ __launch_bounds__(64) void k_decode(const uint32_t* words, const uint64_t* woff, int64_t nch, int64_t n,
                                               DecTables t, const uint64_t* ooff, const int32_t* oval,
                                               int32_t* codes, int* err) {
  __shared__ uint32_t lut[1 << LUTB];
  __shared__ uint32_t first[LMAX + 1], count[LMAX + 1], base[LMAX + 1];
  __shared__ int32_t tile[64 * 65];
  const int lane = threadIdx.x;
  for (int i = lane; i < (1 << LUTB); i += 64) lut[i] = t.lut[i];
  if (lane <= LMAX) {
    first[lane] = t.first[lane];
    count[lane] = t.count[lane];
    base[lane] = t.base[lane];
  }
  const int64_t c0 = int64_t(blockIdx.x) * 64;
  const int64_t c = c0 + lane;
  const bool valid = c < nch;
  const int64_t b0 = c * CHUNK;
  const int cnt = valid ? int(b0 + CHUNK < n ? CHUNK : n - b0) : 0;
  const uint64_t w0 = valid ? woff[c] : 0, w1 = valid ? woff[c + 1] : 0;
  // this chunk's outliers, in the order of its escape symbols
  uint64_t e = valid ? ooff[c] : 0;
  const uint64_t e1 = valid ? ooff[c + 1] : 0;
  uint64_t buf = 0;
  int avail = 0;
  uint64_t wp = w0;
  bool bad = false;
  __syncthreads();
  for (int k0 = 0; k0 < CHUNK; k0 += 64) {
    for (int kk = 0; kk < 64; ++kk) {
      const int k = k0 + kk;
      if (bad || k >= cnt) break;
      while (avail <= 32) {
        const uint64_t wv = wp < w1 ? words[wp] : 0u;
        ++wp;
        buf |= wv << (32 - avail);
        avail += 32;
      }
      uint32_t s, l;
      const uint32_t lu = lut[buf >> (64 - LUTB)];
      if ((lu >> 16) != 0) {
        s = lu & 0xFFFFu;
        l = lu >> 16;
      } else {
        l = 0;
        s = 0;
        for (uint32_t L = LUTB + 1; L <= LMAX; ++L) {
          const uint32_t code = uint32_t(buf >> (64 - L));
          if (count[L] && code - first[L] < count[L]) {
            s = t.sorted[base[L] + code - first[L]];
            l = L;
            break;
          }
        }
        if (l == 0) {
          bad = true;
          break;
        }
      }
      buf <<= l;
      avail -= int(l);
      int32_t q;
      if (s == 0) {
        if (e >= e1) {
          bad = true;
          break;
        }
        q = oval[e++];
      } else {
        q = int32_t(s) - R;
      }
      tile[lane * 65 + kk] = q;
    }
    __syncthreads();
    // lane j's 64 codes, written by the whole wavefront
    for (int j = 0; j < 64; ++j) {
      const int64_t cj = c0 + j;
      if (cj >= nch) break;
      const int cntj = int(cj * CHUNK + CHUNK < n ? CHUNK : n - cj * CHUNK);
      if (k0 + lane < cntj) codes[cj * CHUNK + k0 + lane] = tile[j * 65 + lane];
    }
    __syncthreads();
  }
  if (valid && (bad || e != e1)) atomicOr(err, 1);
}

// ------------------------------------------------------------------ host codebook
// The codebook is built in fixed arrays (no allocation), so the same code
// serves the entry point that may not allocate.

// Work arrays of the code-length construction: a binary min-heap of live
// nodes keyed by (weight, smallest symbol in the subtree), parents and depths
// of the merge tree.  The key is unique among live nodes (the smallest symbol
// of a subtree belongs to it alone), so any correct heap pops in one order.
struct LenWork {
  uint64_t hw[NSYM];
  int32_t hmin[NSYM], hid[NSYM];
  int32_t parent[2 * NSYM], depth[2 * NSYM], L[NSYM], present[NSYM];
};

inline bool heap_less(const LenWork& w, int a, int b) {
  return w.hw[a] != w.hw[b] ? w.hw[a] < w.hw[b] : w.hmin[a] < w.hmin[b];
}

inline void heap_swap(LenWork& w, int a, int b) {
  std::swap(w.hw[a], w.hw[b]);
  std::swap(w.hmin[a], w.hmin[b]);
  std::swap(w.hid[a], w.hid[b]);
}

inline void heap_up(LenWork& w, int i) {
  while (i > 0) {
    const int p = (i - 1) / 2;
    if (!heap_less(w, i, p)) break;
    heap_swap(w, i, p);
    i = p;
  }
}

inline void heap_down(LenWork& w, int n, int i) {
  for (;;) {
    const int l = 2 * i + 1, r = l + 1;
    int m = i;
    if (l < n && heap_less(w, l, m)) m = l;
    if (r < n && heap_less(w, r, m)) m = r;
    if (m == i) break;
    heap_swap(w, i, m);
    i = m;
  }
}

// Huffman code lengths of the symbols with hist[s] > 0 (len[s] = 0 for the
// others): merge the two smallest (weight, smallest symbol) keys until one
// tree remains; lengths above 32 are cut to 32 and the longest codes below
// 32 are lengthened (largest symbol first) until Kraft's sum is <= 1.
void code_lengths(const uint64_t* hist, uint8_t* len, LenWork& w) {
  std::memset(len, 0, NSYM);
  int np = 0;
  for (int s = 0; s < NSYM; ++s)
    if (hist[s]) w.present[np++] = s;
  if (np == 0) return;
  if (np == 1) {
    len[w.present[0]] = 1;
    return;
  }
  int hn = 0;
  for (int k = 0; k < np; ++k) {
    const int s = w.present[k];
    w.hw[hn] = hist[s];
    w.hmin[hn] = s;
    w.hid[hn] = s;
    heap_up(w, hn++);
  }
  int next = NSYM;
  while (hn > 1) {
    const uint64_t aw = w.hw[0];
    const int am = w.hmin[0], aid = w.hid[0];
    heap_swap(w, 0, --hn);
    heap_down(w, hn, 0);
    const uint64_t bw = w.hw[0];
    const int bm = w.hmin[0], bid = w.hid[0];
    heap_swap(w, 0, --hn);
    heap_down(w, hn, 0);
    w.parent[aid] = next;
    w.parent[bid] = next;
    w.hw[hn] = aw + bw;
    w.hmin[hn] = std::min(am, bm);
    w.hid[hn] = next;
    heap_up(w, hn++);
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
// symbols in that order, *nsorted their count.
void canonical(const uint8_t* len, uint32_t* code, uint32_t* sorted, int* nsorted) {
  std::memset(code, 0, NSYM * sizeof(uint32_t));
  int n = 0;
  for (int l = 1; l <= LMAX; ++l)
    for (int s = 0; s < NSYM; ++s)
      if (len[s] == l) sorted[n++] = uint32_t(s);
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

}  // namespace

namespace {

// Code table and stream layout of a code array: histogram (device), code
// lengths and canonical codes (host), per-chunk bit and escape counts
// (device), word and outlier offsets (host).
struct StreamPlan {
  std::vector<uint8_t> len;
  std::vector<uint32_t> cw, sorted;
  std::vector<uint64_t> woff, ooff;
  int64_t nch = 0;
};

StreamPlan plan_stream(const int32_t* codes, int64_t n, hipStream_t st, DevBuf<uint8_t>& dlen, DevBuf<uint32_t>& dcw) {
  if (n < 0 || (n > 0 && !codes)) fail(BM_EINVAL, "bad code array");
  StreamPlan sp;
  const int64_t nch = (n + CHUNK - 1) / CHUNK;
  sp.nch = nch;
  DevBuf<unsigned long long> hist(NSYM);
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, st, hist.p, int64_t(NSYM));
  if (n) {
    const int64_t g = std::min<int64_t>(2048, (n + 255) / 256);
    hipLaunchKernelGGL(k_hist, dim3(unsigned(g)), dim3(256), 0, st, codes, n, hist.p);
  }
  BM_HIP(hipGetLastError());
  std::vector<uint64_t> h(NSYM);
  BM_HIP(hipMemcpyAsync(h.data(), hist.p, NSYM * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  {
    auto work = std::make_unique<LenWork>();
    sp.len.assign(NSYM, 0);
    code_lengths(h.data(), sp.len.data(), *work);
  }
  sp.cw.assign(NSYM, 0);
  sp.sorted.assign(NSYM, 0);
  int ns = 0;
  canonical(sp.len.data(), sp.cw.data(), sp.sorted.data(), &ns);
  sp.sorted.resize(ns);
  BM_HIP(hipMemcpyAsync(dlen.p, sp.len.data(), NSYM, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dcw.p, sp.cw.data(), NSYM * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  DevBuf<uint32_t> bits(size_t(std::max<int64_t>(nch, 1))), esc(size_t(std::max<int64_t>(nch, 1)));
  if (nch) hipLaunchKernelGGL(k_chunk_bits, dim3(unsigned(nch)), dim3(64), 0, st, codes, n, dlen.p, bits.p, esc.p);
  BM_HIP(hipGetLastError());
  std::vector<uint32_t> hb(nch), he(nch);
  if (nch) {
    BM_HIP(hipMemcpyAsync(hb.data(), bits.p, nch * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    BM_HIP(hipMemcpyAsync(he.data(), esc.p, nch * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  }
  BM_HIP(hipStreamSynchronize(st));
  sp.woff.assign(nch + 1, 0);
  sp.ooff.assign(nch + 1, 0);
  for (int64_t c = 0; c < nch; ++c) {
    sp.woff[c + 1] = sp.woff[c] + (uint64_t(hb[c]) + 31) / 32;
    sp.ooff[c + 1] = sp.ooff[c] + he[c];
  }
  return sp;
}

size_t stream_bytes(const StreamPlan& sp) {
  int64_t np = 0;
  for (int s = 0; s < NSYM; ++s) np += sp.len[s] != 0;
  return sizeof(HuffHeader) + size_t(np) * 3 + size_t(sp.nch + 1) * 16 + size_t(sp.woff[sp.nch]) * 4 +
         size_t(sp.ooff[sp.nch]) * 4;
}

}  // namespace

size_t huffman_size(const int32_t* codes, int64_t n, hipStream_t st) {
  DevBuf<uint8_t> dlen(NSYM);
  DevBuf<uint32_t> dcw(NSYM);
  return stream_bytes(plan_stream(codes, n, st, dlen, dcw));
}

size_t huffman_encode(const int32_t* codes, int64_t n, std::vector<uint8_t>& out, hipStream_t st) {
  const size_t bytes = huffman_size(codes, n, st);
  out.resize(bytes);
  return huffman_encode_to(codes, n, out.data(), bytes, st);
}

size_t huffman_encode_to(const int32_t* codes, int64_t n, uint8_t* dst, size_t capacity, hipStream_t st) {
  DevBuf<uint8_t> dlen(NSYM);
  DevBuf<uint32_t> dcw(NSYM);
  const StreamPlan sp = plan_stream(codes, n, st, dlen, dcw);
  const int64_t nch = sp.nch;
  const std::vector<uint8_t>& len = sp.len;
  const std::vector<uint64_t>& woff = sp.woff;
  const std::vector<uint64_t>& ooff = sp.ooff;
  const int64_t nw = int64_t(woff[nch]), nout = int64_t(ooff[nch]);
  DevBuf<uint64_t> dwoff(nch + 1), dooff(nch + 1);
  DevBuf<uint32_t> dwords(size_t(std::max<int64_t>(nw, 1)));
  DevBuf<int32_t> doval(size_t(std::max<int64_t>(nout, 1)));
  BM_HIP(hipMemcpyAsync(dwoff.p, woff.data(), (nch + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dooff.p, ooff.data(), (nch + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  if (nch)
    hipLaunchKernelGGL(k_encode<false>, dim3(unsigned(nch)), dim3(64), 0, st, codes, n, dlen.p, dcw.p, dwoff.p,
                       dooff.p, static_cast<void*>(dwords.p), static_cast<void*>(doval.p));
  BM_HIP(hipGetLastError());
  std::vector<uint16_t> psym;
  std::vector<uint8_t> plen;
  for (int s = 0; s < NSYM; ++s)
    if (len[s]) {
      psym.push_back(uint16_t(s));
      plen.push_back(len[s]);
    }
  const int64_t np = int64_t(psym.size());
  HuffHeader hh{kHuffMagic, 3, n, nch, nw, nout, np};
  const size_t bytes = sizeof(hh) + size_t(np) * 3 + (nch + 1) * 16 + size_t(nw) * 4 + size_t(nout) * 4;
  if (bytes > capacity) fail(BM_ECAPACITY, "Huffman stream larger than its buffer");
  uint8_t* o = dst;
  std::memcpy(o, &hh, sizeof(hh));
  o += sizeof(hh);
  if (np) std::memcpy(o, psym.data(), size_t(np) * 2);
  o += size_t(np) * 2;
  if (np) std::memcpy(o, plen.data(), size_t(np));
  o += size_t(np);
  std::memcpy(o, woff.data(), (nch + 1) * 8);
  o += (nch + 1) * 8;
  std::memcpy(o, ooff.data(), (nch + 1) * 8);
  o += (nch + 1) * 8;
  if (nw) BM_HIP(hipMemcpyAsync(o, dwords.p, size_t(nw) * 4, hipMemcpyDeviceToHost, st));
  o += size_t(nw) * 4;
  if (nout) BM_HIP(hipMemcpyAsync(o, doval.p, size_t(nout) * 4, hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  return bytes;
}

void huffman_decode(const uint8_t* in, size_t in_bytes, int32_t* codes, int64_t n, hipStream_t st) {
  if (!in || in_bytes < sizeof(HuffHeader)) fail(BM_ECORRUPT, "Huffman stream too short");
  HuffHeader hh;
  std::memcpy(&hh, in, sizeof(hh));
  if (hh.magic != kHuffMagic || hh.version != 3) fail(BM_ECORRUPT, "bad Huffman stream header");
  if (hh.n != n) fail(BM_EINVAL, "symbol count does not match the destination");
  if (hh.nchunks != (n + CHUNK - 1) / CHUNK || hh.nwords < 0 || hh.noutliers < 0 || hh.noutliers > n ||
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
  std::vector<uint64_t> woff(nch + 1);
  std::memcpy(woff.data(), p, (nch + 1) * 8);
  p += (nch + 1) * 8;
  std::vector<uint64_t> ooff(nch + 1);
  std::memcpy(ooff.data(), p, (nch + 1) * 8);
  p += (nch + 1) * 8;
  if (woff[0] != 0 || ooff[0] != 0 || ooff[nch] != uint64_t(nout)) fail(BM_ECORRUPT, "bad chunk offsets");
  for (int64_t c = 0; c < nch; ++c)
    if (woff[c + 1] < woff[c] || woff[c + 1] > uint64_t(nw) || ooff[c + 1] < ooff[c] ||
        ooff[c + 1] - ooff[c] > uint64_t(CHUNK))
      fail(BM_ECORRUPT, "bad chunk offsets");
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
  std::vector<uint32_t> first(LMAX + 1, 0), count(LMAX + 1, 0), base(LMAX + 1, 0), lut(1u << LUTB, 0);
  for (size_t i = 0; i < sorted.size(); ++i) {
    const int l = len[sorted[i]];
    if (count[l] == 0) {
      first[l] = cw[sorted[i]];
      base[l] = uint32_t(i);
    }
    ++count[l];
    if (l <= LUTB) {
      const uint32_t lo = cw[sorted[i]] << (LUTB - l), span = 1u << (LUTB - l);
      for (uint32_t k = 0; k < span; ++k) lut[lo + k] = sorted[i] | (uint32_t(l) << 16);
    }
  }
  DevBuf<uint32_t> dlut(lut.size()), dfirst(LMAX + 1), dcount(LMAX + 1), dbase(LMAX + 1),
      dsorted(std::max<size_t>(sorted.size(), 1));
  DevBuf<uint64_t> dwoff(nch + 1), dooff(nch + 1);
  DevBuf<uint32_t> dwords(size_t(std::max<int64_t>(nw, 1)));
  DevBuf<int32_t> doval(size_t(std::max<int64_t>(nout, 1)));
  DevBuf<int> derr(1);
  BM_HIP(hipMemcpyAsync(dlut.p, lut.data(), lut.size() * 4, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dfirst.p, first.data(), (LMAX + 1) * 4, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dcount.p, count.data(), (LMAX + 1) * 4, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dbase.p, base.data(), (LMAX + 1) * 4, hipMemcpyHostToDevice, st));
  if (!sorted.empty()) BM_HIP(hipMemcpyAsync(dsorted.p, sorted.data(), sorted.size() * 4, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dwoff.p, woff.data(), (nch + 1) * 8, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dooff.p, ooff.data(), (nch + 1) * 8, hipMemcpyHostToDevice, st));
  if (nw) BM_HIP(hipMemcpyAsync(dwords.p, p, size_t(nw) * 4, hipMemcpyHostToDevice, st));
  p += size_t(nw) * 4;
  if (nout) BM_HIP(hipMemcpyAsync(doval.p, p, size_t(nout) * 4, hipMemcpyHostToDevice, st));
  const int zero = 0;
  BM_HIP(hipMemcpyAsync(derr.p, &zero, sizeof(int), hipMemcpyHostToDevice, st));
  DecTables t{dlut.p, dfirst.p, dcount.p, dbase.p, dsorted.p};
  if (nch)
    hipLaunchKernelGGL(k_decode, dim3(unsigned((nch + 63) / 64)), dim3(64), 0, st, dwords.p, dwoff.p, nch, n, t,
                       dooff.p, doval.p, codes, derr.p);
  BM_HIP(hipGetLastError());
  int herr = 0;
  BM_HIP(hipMemcpyAsync(&herr, derr.p, sizeof(int), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  if (herr) fail(BM_ECORRUPT, "Huffman stream does not decode");
}

// ------------------------------------------------------------------ stage times
// The encoder's stages timed one by one (the lossless part of the time model
// of Algorithm 1): histogram, code table, chunk sizes + encode, copy-out + CRC.
void huffman_stage_times(const int32_t* codes, int64_t n, hipStream_t st, double ms[4]) {
  using clk = std::chrono::steady_clock;
  auto since = [](clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); };
  hipEvent_t e0, e1;
  BM_HIP(hipEventCreate(&e0));
  BM_HIP(hipEventCreate(&e1));
  auto elapsed = [&]() {
    BM_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    BM_HIP(hipEventElapsedTime(&t, e0, e1));
    return double(t);
  };
  const int64_t nch = (n + CHUNK - 1) / CHUNK;
  DevBuf<unsigned long long> hist(NSYM);
  DevBuf<uint8_t> dlen(NSYM);
  DevBuf<uint32_t> dcw(NSYM);
  DevBuf<uint32_t> bits(size_t(std::max<int64_t>(nch, 1))), esc(size_t(std::max<int64_t>(nch, 1)));
  // (0) histogram
  BM_HIP(hipEventRecord(e0, st));
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, st, hist.p, int64_t(NSYM));
  if (n) hipLaunchKernelGGL(k_hist, dim3(unsigned(std::min<int64_t>(2048, (n + 255) / 256))), dim3(256), 0, st, codes, n,
                            hist.p);
  BM_HIP(hipEventRecord(e1, st));
  ms[0] = elapsed();
  // (1) code table on the host
  auto t1 = clk::now();
  std::vector<uint64_t> h(NSYM);
  BM_HIP(hipMemcpyAsync(h.data(), hist.p, NSYM * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  auto work = std::make_unique<LenWork>();
  std::vector<uint8_t> len(NSYM);
  std::vector<uint32_t> cw(NSYM), sorted(NSYM);
  int ns = 0;
  code_lengths(h.data(), len.data(), *work);
  canonical(len.data(), cw.data(), sorted.data(), &ns);
  ms[1] = since(t1);
  // (2) chunk sizes, offsets on the host, encode
  auto t2 = clk::now();
  BM_HIP(hipMemcpyAsync(dlen.p, len.data(), NSYM, hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dcw.p, cw.data(), NSYM * sizeof(uint32_t), hipMemcpyHostToDevice, st));
  if (nch) hipLaunchKernelGGL(k_chunk_bits, dim3(unsigned(nch)), dim3(64), 0, st, codes, n, dlen.p, bits.p, esc.p);
  std::vector<uint32_t> hb(nch), he(nch);
  if (nch) {
    BM_HIP(hipMemcpyAsync(hb.data(), bits.p, nch * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    BM_HIP(hipMemcpyAsync(he.data(), esc.p, nch * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  }
  BM_HIP(hipStreamSynchronize(st));
  std::vector<uint64_t> woff(nch + 1, 0), ooff(nch + 1, 0);
  for (int64_t c = 0; c < nch; ++c) {
    woff[c + 1] = woff[c] + (uint64_t(hb[c]) + 31) / 32;
    ooff[c + 1] = ooff[c] + he[c];
  }
  const int64_t nw = int64_t(woff[nch]), nout = int64_t(ooff[nch]);
  DevBuf<uint64_t> dwoff(nch + 1), dooff(nch + 1);
  DevBuf<uint32_t> dwords(size_t(std::max<int64_t>(nw, 1)));
  DevBuf<int32_t> doval(size_t(std::max<int64_t>(nout, 1)));
  BM_HIP(hipMemcpyAsync(dwoff.p, woff.data(), (nch + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  BM_HIP(hipMemcpyAsync(dooff.p, ooff.data(), (nch + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  if (nch)
    hipLaunchKernelGGL(k_encode<false>, dim3(unsigned(nch)), dim3(64), 0, st, codes, n, dlen.p, dcw.p, dwoff.p,
                       dooff.p, static_cast<void*>(dwords.p), static_cast<void*>(doval.p));
  BM_HIP(hipGetLastError());
  BM_HIP(hipStreamSynchronize(st));
  ms[2] = since(t2);
  // (3) the stream to the host and its CRC
  auto t3 = clk::now();
  std::vector<uint8_t> out(size_t(nw) * 4 + size_t(nout) * 4 + 16);
  if (nw) BM_HIP(hipMemcpyAsync(out.data(), dwords.p, size_t(nw) * 4, hipMemcpyDeviceToHost, st));
  if (nout) BM_HIP(hipMemcpyAsync(out.data() + size_t(nw) * 4, doval.p, size_t(nout) * 4, hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  volatile uint32_t crc = container_crc(out.data(), out.size());
  (void)crc;
  ms[3] = since(t3);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
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
  if (nch) hipLaunchKernelGGL(k_chunk_bits, dim3(unsigned(nch)), dim3(64), 0, st, codes, n, dlen, bits, esc);
  BM_HIP(hipGetLastError());
  if (nch) {
    BM_HIP(hipMemcpyAsync(H.bits, bits, size_t(nch) * 4, hipMemcpyDeviceToHost, st));
    BM_HIP(hipMemcpyAsync(H.esc, esc, size_t(nch) * 4, hipMemcpyDeviceToHost, st));
  }
  BM_HIP(hipStreamSynchronize(st));
  H.woff[0] = 0;
  H.ooff[0] = 0;
  for (int64_t c = 0; c < nch; ++c) {
    H.woff[c + 1] = H.woff[c] + (uint64_t(H.bits[c]) + 31) / 32;
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
  if (nch) {
    void* wd = o + off_words;
    void* od = o + off_out;
    const bool aligned = (reinterpret_cast<uintptr_t>(wd) & 3) == 0;   // off_out - off_words is a multiple of 4
    if (aligned)
      hipLaunchKernelGGL(k_encode<false>, dim3(unsigned(nch)), dim3(64), 0, st, codes, n, dlen, dcw, dwoff, dooff,
                         wd, od);
    else
      hipLaunchKernelGGL(k_encode<true>, dim3(unsigned(nch)), dim3(64), 0, st, codes, n, dlen, dcw, dwoff, dooff,
                         wd, od);
  }
  BM_HIP(hipGetLastError());
  BM_HIP(hipStreamSynchronize(st));
  return bytes;
}

}  // namespace bm
