// extern "C" entry points of libblockmgard: argument checks, error mapping,
// and the self-describing compressed container (Sec. IV pipeline:
// transform -> quantize -> lossless; raw copy of incompressible data,
// Sec. V-F).

#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

bm_plan_s* bm_plan_build(const bm_config* c);
void bm_plan_free(bm_plan_s* p);

namespace {

thread_local std::string g_err;

template <typename F>
bm_status guarded(F&& f) {
  try {
    g_err.clear();
    f();
    return BM_OK;
  } catch (const bm::Error& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return BM_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return BM_EINVAL;
  } catch (...) {
    g_err = "unknown failure";
    return BM_EINVAL;
  }
}

void need(bool ok, const char* what) {
  if (!ok) bm::fail(BM_EINVAL, what);
}

void check_device(const bm_plan_s* p) {
  int d = -1;
  BM_HIP(hipGetDevice(&d));
  if (d != p->device) bm::fail(BM_EINVAL, "the current device is not the plan's device");
}

// CRC-32 (reflected polynomial 0xEDB88320), eight bytes per step with the
// slicing-by-8 tables (Kounavis and Berry): table k maps a byte k positions
// ahead of the end of the word to its contribution; bytes are read in
// little-endian order.
struct Crc32Tables {
  uint32_t t[8][256];
  Crc32Tables() {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      t[0][i] = c;
    }
    for (int k = 1; k < 8; ++k)
      for (uint32_t i = 0; i < 256; ++i) t[k][i] = (t[k - 1][i] >> 8) ^ t[0][t[k - 1][i] & 0xFF];
  }
};

uint32_t crc32(const uint8_t* p, size_t n, uint32_t crc = 0) {
  static const Crc32Tables T;
  crc = ~crc;
  for (; n >= 8; n -= 8, p += 8) {
    uint32_t lo, hi;
    std::memcpy(&lo, p, 4);
    std::memcpy(&hi, p + 4, 4);
    lo ^= crc;
    crc = T.t[7][lo & 0xFF] ^ T.t[6][(lo >> 8) & 0xFF] ^ T.t[5][(lo >> 16) & 0xFF] ^ T.t[4][lo >> 24] ^
          T.t[3][hi & 0xFF] ^ T.t[2][(hi >> 8) & 0xFF] ^ T.t[1][(hi >> 16) & 0xFF] ^ T.t[0][hi >> 24];
  }
  for (; n > 0; --n, ++p) crc = T.t[0][(crc ^ *p) & 0xFF] ^ (crc >> 8);
  return ~crc;
}

// The CRC of a concatenation: crc(A B) = Z(crc(A)) ^ crc(B), where Z shifts
// the CRC register over |B| zero bytes (the pre- and post-inversion cancel).
// Z is a linear map over GF(2); its 32x32 matrix for 2^k zero bits comes
// from squaring the one-bit matrix, and the bits of the byte count choose
// which powers to apply (the combine step of zlib's crc32_combine).
uint32_t gf2_apply(const uint32_t* mat, uint32_t v) {
  uint32_t r = 0;
  for (int i = 0; v; ++i, v >>= 1)
    if (v & 1) r ^= mat[i];
  return r;
}

void gf2_square(uint32_t* sq, const uint32_t* mat) {
  for (int i = 0; i < 32; ++i) sq[i] = gf2_apply(mat, mat[i]);
}

uint32_t crc32_shift(uint32_t crc, uint64_t bytes) {
  if (bytes == 0) return crc;
  uint32_t a[32], b[32];
  a[0] = 0xEDB88320u;                    // one zero bit
  for (int i = 1; i < 32; ++i) a[i] = 1u << (i - 1);
  gf2_square(b, a);                      // two
  gf2_square(a, b);                      // four
  for (;;) {
    gf2_square(b, a);                    // 8, 32, 128, ... bits: one byte times 1, 4, 16, ...
    if (bytes & 1) crc = gf2_apply(b, crc);
    bytes >>= 1;
    if (!bytes) break;
    gf2_square(a, b);                    // 2, 8, 32, ... bytes
    if (bytes & 1) crc = gf2_apply(a, crc);
    bytes >>= 1;
    if (!bytes) break;
  }
  return crc;
}

// crc32 of a large buffer on several host threads, continuing from crc
uint32_t crc32_parallel(const uint8_t* p, size_t n, uint32_t crc) {
  const size_t kMin = size_t(8) << 20;
  unsigned nt = std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  if (n < kMin || nt < 2) return crc32(p, n, crc);
  nt = unsigned(std::min<size_t>(nt, n / (kMin / 4)));
  std::vector<uint32_t> part(nt);
  std::vector<std::thread> th;
  const size_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const size_t lo = std::min(n, t * chunk), hi = std::min(n, lo + chunk);
    th.emplace_back([&, t, lo, hi] { part[t] = crc32(p + lo, hi - lo); });
  }
  for (auto& t : th) t.join();
  for (unsigned t = 0; t < nt; ++t) {
    const size_t lo = std::min(n, t * chunk), hi = std::min(n, lo + chunk);
    crc = crc32_shift(crc, hi - lo) ^ part[t];
  }
  return crc;
}

// container header; payload follows (block tolerances + Huffman stream, or raw data)
struct CHeader {
  uint32_t magic;       // "BMGD"
  uint32_t version;
  uint32_t flags;       // bit 0: raw copy
  int32_t dtype, block, L, M, pad_mode, ndim, nested;
  int64_t dims[3];
  double eta;
  int64_t ntol;         // block tolerance entries
  uint64_t payload;     // bytes after the header
  uint32_t crc;         // CRC32 of header (crc = 0) + payload
  uint32_t pad1;
};
constexpr uint32_t kMagic = 0x44474D42u;   // "BMGD"

bm_config header_config(const CHeader& h) {
  bm_config c{};
  c.ndim = 3;
  c.dims[0] = h.dims[0];
  c.dims[1] = h.dims[1];
  c.dims[2] = h.dims[2];
  c.dtype = h.dtype;
  c.block = h.block;
  c.L = h.L;
  c.M = h.M;
  c.pad_mode = h.pad_mode;
  c.eta = h.eta;
  c.nested = h.nested;
  return c;
}

// The stored block tolerance map must hold positive, finite tolerances (a
// container whose CRC matches can still carry a bad map if it was written
// by other code): BM_ECORRUPT otherwise.
void check_stored_tol(const uint8_t* pl, int64_t ntol) {
  for (int64_t i = 0; i < ntol; ++i) {
    double t;
    std::memcpy(&t, pl + 8 * i, 8);
    if (!(t > 0) || !std::isfinite(t)) bm::fail(BM_ECORRUPT, "stored block tolerance not positive and finite");
  }
}

// header checks; the CRC over header and payload only when check_crc
CHeader parse(const void* in, size_t in_bytes, bool check_crc = true) {
  if (!in || in_bytes < sizeof(CHeader)) bm::fail(BM_ECORRUPT, "buffer shorter than the container header");
  CHeader h;
  std::memcpy(&h, in, sizeof(h));
  if (h.magic != kMagic) bm::fail(BM_ECORRUPT, "bad magic");
  if (h.version != 1) bm::fail(BM_ECORRUPT, "unsupported container version");
  if (h.payload != in_bytes - sizeof(CHeader)) bm::fail(BM_ECORRUPT, "payload size mismatch");
  if (!check_crc) return h;
  CHeader z = h;
  z.crc = 0;
  uint32_t c = crc32(reinterpret_cast<const uint8_t*>(&z), sizeof(z));
  c = crc32_parallel(static_cast<const uint8_t*>(in) + sizeof(CHeader), size_t(h.payload), c);
  if (c != h.crc) bm::fail(BM_ECORRUPT, "CRC mismatch");
  return h;
}

}  // namespace

namespace bm {

// the codes of the padded grid, written by compress and read by decompress
// (the fused paths need no coefficient array)
void ensure_code_buffer(bm_plan_s& p) {
  const size_t n = size_t(p.pdims[0]) * p.pdims[1] * p.pdims[2];
  if (!p.ws.codes) plan_alloc(p, &p.ws.codes, n * sizeof(int32_t));
}

void check_block_tol(bm_plan_s& p, const double* block_tol, hipStream_t st) {
  const int64_t ntol = p.nb1[0] * p.nb1[1] * p.nb1[2];
  std::vector<double> tol(ntol);
  BM_HIP(hipMemcpyAsync(tol.data(), block_tol, ntol * sizeof(double), hipMemcpyDeviceToHost, st));
  BM_HIP(hipStreamSynchronize(st));
  for (double t : tol)
    if (!(t > 0) || !std::isfinite(t)) fail(BM_ENONFINITE, "block tolerances must be positive and finite");
}

struct PendingContainer {
  std::vector<uint8_t> head;   // the header, CRC not set
  std::vector<double> tol;     // block tolerance map
  std::unique_ptr<HuffmanEncoder> enc;
  const void* x = nullptr;     // source of the raw copy (device)
  size_t total = 0;
  hipStream_t st = nullptr;
};

size_t pending_bytes(const PendingContainer& c) { return c.total; }

std::shared_ptr<PendingContainer> plan_container(bm_plan_s& p, const void* x, const double* block_tol, bool too_fine,
                                                 hipStream_t st) {
  const int64_t npad = p.pdims[0] * p.pdims[1] * p.pdims[2];
  const int64_t nlog = p.dims[0] * p.dims[1] * p.dims[2];
  const int64_t ntol = p.nb1[0] * p.nb1[1] * p.nb1[2];
  auto c = std::make_shared<PendingContainer>();
  c->tol.resize(ntol);
  BM_HIP(hipMemcpyAsync(c->tol.data(), block_tol, ntol * sizeof(double), hipMemcpyDeviceToHost, st));
  // the stream is planned once (histogram, code table, chunk sizes); it is
  // encoded when the container is written, straight into the caller's buffer
  const int32_t* codes = static_cast<const int32_t*>(p.ws.codes);
  if (!too_fine) c->enc = std::make_unique<HuffmanEncoder>(codes, npad, st);
  const size_t sb = c->enc ? c->enc->bytes() : 0;
  BM_HIP(hipStreamSynchronize(st));
  CHeader h{};
  h.magic = kMagic;
  h.version = 1;
  h.dtype = p.cfg.dtype;
  h.block = p.cfg.block;
  h.L = p.L;
  h.M = p.M;
  h.pad_mode = p.cfg.pad_mode;
  h.nested = p.cfg.nested;
  h.ndim = 3;
  for (int a = 0; a < 3; ++a) h.dims[a] = p.dims[a];
  h.eta = p.cfg.eta;
  h.ntol = ntol;
  const size_t coded = size_t(ntol) * 8 + sb;
  const size_t raw = size_t(nlog) * p.esize;
  h.flags = (too_fine || coded >= raw) ? 1u : 0u;
  h.payload = h.flags ? raw : coded;
  if (h.flags) c->enc.reset();
  c->head.assign(reinterpret_cast<const uint8_t*>(&h), reinterpret_cast<const uint8_t*>(&h) + sizeof(h));
  c->x = x;
  c->total = sizeof(CHeader) + size_t(h.payload);
  c->st = st;
  return c;
}

void write_pending(PendingContainer& c, void* out) {
  CHeader h;
  std::memcpy(&h, c.head.data(), sizeof(h));
  const size_t ntol = size_t(h.ntol);
  uint8_t* o = static_cast<uint8_t*>(out) + sizeof(CHeader);
  if (h.flags & 1u) {
    BM_HIP(hipMemcpyAsync(o, c.x, size_t(h.payload), hipMemcpyDeviceToHost, c.st));
    BM_HIP(hipStreamSynchronize(c.st));
  } else {
    std::memcpy(o, c.tol.data(), ntol * 8);
    c.enc->write(o + ntol * 8, size_t(h.payload) - ntol * 8);
  }
  h.crc = 0;
  const auto t0 = std::chrono::steady_clock::now();
  uint32_t crc = crc32(reinterpret_cast<const uint8_t*>(&h), sizeof(h));
  if (h.flags & 1u) {
    crc = crc32_parallel(o, size_t(h.payload), crc);
  } else {
    crc = crc32(o, ntol * 8, crc);
    crc = stream_crc(*c.enc, o + ntol * 8, size_t(h.payload) - ntol * 8, crc);
  }
  h.crc = crc;
  if (!(h.flags & 1u))
    set_lossless_crc_ms(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  std::memcpy(out, &h, sizeof(h));
}

bool write_container(bm_plan_s& p, const void* x, const double* block_tol, bool too_fine, void* out,
                     size_t capacity, size_t* needed, hipStream_t st) {
  std::shared_ptr<PendingContainer> c = plan_container(p, x, block_tol, too_fine, st);
  *needed = c->total;
  if (!out || capacity < c->total) return false;
  write_pending(*c, out);
  return true;
}

// Container of the paper's 8^3 form: the same header with flags bit 1 set
// (block = 8, M = 0, zero fill), the level-1 block map, then the Huffman
// stream of the codes (flat layout of bm_p8_decompose), or the raw data.
constexpr uint32_t kFlagP8 = 2u;

bool write_container_p8(bm_p8_s& p, const void* x, const double* block_tol, double eta, bool too_fine, void* out,
                        size_t capacity, size_t* needed, hipStream_t st) {
  int64_t dims[3], nb[3];
  int dtype = 0, L = 0;
  size_t esize = 0;
  p8_info(p, dims, &dtype, &L, &esize);
  p8_block_grid(p, nb);
  const int64_t ntol = nb[0] * nb[1] * nb[2];
  const int64_t nlog = dims[0] * dims[1] * dims[2];
  std::vector<double> tol(ntol);
  BM_HIP(hipMemcpyAsync(tol.data(), block_tol, ntol * sizeof(double), hipMemcpyDeviceToHost, st));
  const int32_t* codes = p8_codes(p);
  const int64_t ncodes = p8_coeff_size(p);
  std::unique_ptr<HuffmanEncoder> enc;
  if (!too_fine) enc = std::make_unique<HuffmanEncoder>(codes, ncodes, st);
  const size_t sb = enc ? enc->bytes() : 0;
  BM_HIP(hipStreamSynchronize(st));
  CHeader h{};
  h.magic = kMagic;
  h.version = 1;
  h.dtype = dtype;
  h.block = 8;
  h.L = L;
  h.M = p8_global_levels(p);
  h.pad_mode = 1;
  h.ndim = 3;
  for (int a = 0; a < 3; ++a) h.dims[a] = dims[a];
  h.eta = eta;
  h.ntol = ntol;
  const size_t coded = size_t(ntol) * 8 + sb;
  const size_t raw = size_t(nlog) * esize;
  h.flags = kFlagP8 | ((too_fine || coded >= raw) ? 1u : 0u);
  h.payload = (h.flags & 1u) ? raw : coded;
  const size_t total = sizeof(CHeader) + size_t(h.payload);
  *needed = total;
  if (!out || capacity < total) return false;
  uint8_t* o = static_cast<uint8_t*>(out) + sizeof(CHeader);
  if (h.flags & 1u) {
    BM_HIP(hipMemcpyAsync(o, x, raw, hipMemcpyDeviceToHost, st));
    BM_HIP(hipStreamSynchronize(st));
  } else {
    std::memcpy(o, tol.data(), size_t(ntol) * 8);
    enc->write(o + size_t(ntol) * 8, sb);
  }
  h.crc = 0;
  const auto t0 = std::chrono::steady_clock::now();
  uint32_t c = crc32(reinterpret_cast<const uint8_t*>(&h), sizeof(h));
  if (h.flags & 1u) {
    c = crc32_parallel(o, size_t(h.payload), c);
  } else {
    c = crc32(o, size_t(ntol) * 8, c);
    c = stream_crc(*enc, o + size_t(ntol) * 8, sb, c);
  }
  h.crc = c;
  if (enc) set_lossless_crc_ms(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  std::memcpy(out, &h, sizeof(h));
  return true;
}

}  // namespace bm

extern "C" {

bm_status bm_plan_create(const bm_config* cfg, bm_plan* out) {
  return guarded([&] {
    need(cfg && out, "null argument");
    *out = bm_plan_build(cfg);
  });
}

bm_status bm_plan_destroy(bm_plan plan) {
  return guarded([&] { bm_plan_free(plan); });
}

bm_status bm_plan_config(bm_plan p, bm_config* cfg) {
  return guarded([&] {
    need(p && cfg, "null argument");
    *cfg = p->cfg;
  });
}

bm_status bm_coeff_shape(bm_plan p, int64_t padded_dims[3]) {
  return guarded([&] {
    need(p && padded_dims, "null argument");
    for (int a = 0; a < 3; ++a) padded_dims[a] = p->pdims[a];
  });
}

bm_status bm_workspace_size(bm_plan p, size_t* bytes) {
  return guarded([&] {
    need(p && bytes, "null argument");
    *bytes = p->dev_bytes;
  });
}

bm_status bm_block_grid(bm_plan p, int64_t nb[3]) {
  return guarded([&] {
    need(p && nb, "null argument");
    for (int a = 0; a < 3; ++a) nb[a] = p->nb1[a];
  });
}

bm_status bm_level_gains(bm_plan p, double* gains) {
  return guarded([&] {
    need(p && gains, "null argument");
    for (int s = 0; s < p->nlev; ++s) gains[s] = p->lv[s].gain;
  });
}

bm_status bm_decompose(bm_plan p, const void* x, void* coeff, hipStream_t st) {
  return guarded([&] {
    need(p && x && coeff, "null argument");
    check_device(p);
    bm::decompose(*p, x, coeff, st);
  });
}

bm_status bm_recompose(bm_plan p, const void* coeff, void* x, hipStream_t st) {
  return guarded([&] {
    need(p && x && coeff, "null argument");
    check_device(p);
    bm::recompose(*p, coeff, x, st);
  });
}

bm_status bm_decompose_adjoint(bm_plan p, const void* gcoeff, void* gx, hipStream_t st) {
  return guarded([&] {
    need(p && gcoeff && gx, "null argument");
    check_device(p);
    bm::decompose_adjoint(*p, gcoeff, gx, st);
  });
}

bm_status bm_recompose_adjoint(bm_plan p, const void* gx, void* gcoeff, hipStream_t st) {
  return guarded([&] {
    need(p && gcoeff && gx, "null argument");
    check_device(p);
    bm::recompose_adjoint(*p, gx, gcoeff, st);
  });
}

bm_status bm_tolmap_from_boxes(bm_plan p, const double* boxes, int nbox, double background, double* block_tol,
                               hipStream_t st) {
  return guarded([&] {
    need(p && block_tol, "null argument");
    check_device(p);
    bm::tolmap_from_boxes(*p, boxes, nbox, background, block_tol, st);
  });
}

bm_status bm_tolmap_from_voxels(bm_plan p, const double* voxel_tol, double* block_tol, hipStream_t st) {
  return guarded([&] {
    need(p && voxel_tol && block_tol, "null argument");
    check_device(p);
    bm::tolmap_from_voxels(*p, voxel_tol, block_tol, st);
  });
}

bm_status bm_quantize_roi(bm_plan p, const void* coeff, const double* block_tol, int32_t* codes, bm_qstats* stats,
                          hipStream_t st) {
  return guarded([&] {
    need(p && coeff && block_tol && codes, "null argument");
    check_device(p);
    bm::quantize(*p, coeff, block_tol, codes, stats, st);
  });
}

bm_status bm_dequantize(bm_plan p, const int32_t* codes, const double* block_tol, void* coeff, hipStream_t st) {
  return guarded([&] {
    need(p && coeff && block_tol && codes, "null argument");
    check_device(p);
    bm::dequantize(*p, codes, block_tol, coeff, st);
  });
}

bm_status bm_decompose_quantize(bm_plan p, const void* x, const double* block_tol, int32_t* codes, bm_qstats* stats,
                                hipStream_t st) {
  return guarded([&] {
    need(p && x && block_tol && codes, "null argument");
    check_device(p);
    bm::decompose_quantize(*p, x, block_tol, codes, stats, st);
  });
}

bm_status bm_dequantize_recompose(bm_plan p, const int32_t* codes, const double* block_tol, void* x, hipStream_t st) {
  return guarded([&] {
    need(p && x && block_tol && codes, "null argument");
    check_device(p);
    bm::dequantize_recompose(*p, codes, block_tol, x, st);
  });
}

bm_status bm_quant_prepare(bm_plan p, const double* block_tol, hipStream_t st) {
  return guarded([&] {
    need(p != nullptr, "null plan");
    if (block_tol) check_device(p);
    bm::quant_keep(*p, block_tol, st);
  });
}

bm_status bm_huffman_encode(const int32_t* codes, int64_t n, void* out, size_t capacity, size_t* out_bytes,
                            hipStream_t st) {
  return guarded([&] {
    need(out_bytes != nullptr, "null out_bytes");
    need(codes || n == 0, "null codes");
    bm::HuffmanEncoder enc(codes, n, st);
    const size_t bytes = enc.bytes();
    *out_bytes = bytes;
    if (!out || capacity < bytes) bm::fail(BM_ECAPACITY, "output buffer too small");
    enc.write(static_cast<uint8_t*>(out), bytes);
  });
}

struct bm_huffman_s {
  std::unique_ptr<bm::HuffmanEncoder> enc;
  int device = 0;
};

bm_status bm_huffman_plan(const int32_t* codes, int64_t n, bm_huffman* out, size_t* out_bytes, hipStream_t st) {
  return guarded([&] {
    need(out && out_bytes, "null argument");
    need(codes || n == 0, "null codes");
    *out = nullptr;
    auto h = std::make_unique<bm_huffman_s>();
    BM_HIP(hipGetDevice(&h->device));
    h->enc = std::make_unique<bm::HuffmanEncoder>(codes, n, st);
    *out_bytes = h->enc->bytes();
    *out = h.release();
  });
}

bm_status bm_huffman_write(bm_huffman h, void* out, size_t capacity, size_t* out_bytes) {
  return guarded([&] {
    need(h && out_bytes, "null argument");
    const size_t bytes = h->enc->bytes();
    *out_bytes = bytes;
    if (!out || capacity < bytes) bm::fail(BM_ECAPACITY, "output buffer too small");
    int dev = 0;
    BM_HIP(hipGetDevice(&dev));
    if (dev != h->device) bm::fail(BM_EINVAL, "handle planned on another device");
    h->enc->write(static_cast<uint8_t*>(out), bytes);
  });
}

bm_status bm_huffman_destroy(bm_huffman h) {
  return guarded([&] { delete h; });
}

bm_status bm_huffman_encode_device(const int32_t* codes, int64_t n, void* out, size_t capacity, size_t* out_bytes,
                                   hipStream_t st) {
  return guarded([&] {
    need(out_bytes != nullptr, "null out_bytes");
    bm::huffman_encode_noalloc(codes, n, out, capacity, out_bytes, st);
  });
}

bm_status bm_huffman_decode(const void* in, size_t in_bytes, int32_t* codes, int64_t n, hipStream_t st) {
  return guarded([&] {
    need(codes || n == 0, "null codes");
    bm::huffman_decode(static_cast<const uint8_t*>(in), in_bytes, codes, n, st);
  });
}

bm_status bm_huffman_code_lengths(const uint64_t* hist, uint8_t* len) {
  return guarded([&] {
    need(hist && len, "null argument");
    bm::huffman_code_lengths(hist, len);
  });
}

bm_status bm_lossless_last_times(bm_lossless_times* out) {
  return guarded([&] {
    need(out != nullptr, "null argument");
    *out = bm::lossless_times();
  });
}

bm_status bm_compress(bm_plan p, const void* x, const double* block_tol, void* out, size_t capacity,
                      size_t* out_bytes, hipStream_t st) {
  return guarded([&] {
    need(p && x && block_tol && out_bytes, "null argument");
    check_device(p);
    p->pending.reset();
    bm::ensure_code_buffer(*p);
    bool too_fine = false;   // codes beyond 32 bits: store the raw data
    bm::check_block_tol(*p, block_tol, st);
    try {
      bm_qstats qs;
      bm::decompose_quantize(*p, x, block_tol, static_cast<int32_t*>(p->ws.codes), &qs, st);
    } catch (const bm::Error& e) {
      if (e.code != BM_ERANGE) throw;
      too_fine = true;
    }
    if (!bm::write_container(*p, x, block_tol, too_fine, out, capacity, out_bytes, st))
      bm::fail(BM_ECAPACITY, "output buffer too small");
  });
}

bm_status bm_compress_plan(bm_plan p, const void* x, const double* block_tol, size_t* out_bytes, hipStream_t st) {
  return guarded([&] {
    need(p && x && block_tol && out_bytes, "null argument");
    check_device(p);
    p->pending.reset();
    bm::ensure_code_buffer(*p);
    bool too_fine = false;   // codes beyond 32 bits: store the raw data
    bm::check_block_tol(*p, block_tol, st);
    try {
      bm_qstats qs;
      bm::decompose_quantize(*p, x, block_tol, static_cast<int32_t*>(p->ws.codes), &qs, st);
    } catch (const bm::Error& e) {
      if (e.code != BM_ERANGE) throw;
      too_fine = true;
    }
    p->pending = bm::plan_container(*p, x, block_tol, too_fine, st);
    *out_bytes = bm::pending_bytes(*p->pending);
  });
}

bm_status bm_compress_write(bm_plan p, void* out, size_t capacity, size_t* out_bytes) {
  return guarded([&] {
    need(p && out_bytes, "null argument");
    if (!p->pending) bm::fail(BM_EINVAL, "no compress planned on this plan (bm_compress_plan)");
    const size_t total = bm::pending_bytes(*p->pending);
    *out_bytes = total;
    if (!out || capacity < total) bm::fail(BM_ECAPACITY, "output buffer too small");
    check_device(p);
    std::shared_ptr<bm::PendingContainer> c = std::move(p->pending);
    bm::write_pending(*c, out);
  });
}

bm_status bm_qoi_deltas(bm_plan p, const void* g, double tol_q, const double* block_tol, double* delta,
                        int64_t* n_set, hipStream_t st) {
  return guarded([&] {
    need(p && g && block_tol && delta, "null argument");
    check_device(p);
    const int64_t n = bm::qoi_deltas(*p, g, tol_q, block_tol, delta, st);
    if (n_set) *n_set = n;
  });
}

bm_status bm_quantize_delta(bm_plan p, const void* coeff, const double* delta, int32_t* codes, bm_qstats* stats,
                            hipStream_t st) {
  return guarded([&] {
    need(p && coeff && delta && codes, "null argument");
    check_device(p);
    bm::quantize_delta(*p, coeff, delta, codes, stats, st);
  });
}

bm_status bm_dequantize_delta(bm_plan p, const int32_t* codes, const double* delta, void* coeff, hipStream_t st) {
  return guarded([&] {
    need(p && coeff && delta && codes, "null argument");
    check_device(p);
    bm::dequantize_delta(*p, codes, delta, coeff, st);
  });
}

bm_status bm_autotune(const bm_config* in, const void* x, const double* voxel_tol, double slack, int reps,
                      bm_config* out, bm_candidate* cands, int cap, int* ncands, hipStream_t st) {
  return guarded([&] {
    need(in && x && voxel_tol && out, "null argument");
    need(cap >= 0 && (cap == 0 || cands), "null candidate table");
    bm_config o{};
    const std::vector<bm_candidate> all = bm::autotune(*in, x, voxel_tol, slack, reps, o, st);
    for (int i = 0; i < cap && i < int(all.size()); ++i) cands[i] = all[i];
    if (ncands) *ncands = int(all.size());
    *out = o;
  });
}

bm_status bm_autotune_budget(const bm_config* in, const void* x, const double* voxel_tol, double budget_ms, int reps,
                             bm_config* out, bm_candidate* cands, int cap, int* ncands, hipStream_t st) {
  return guarded([&] {
    need(in && x && voxel_tol && out, "null argument");
    need(cap >= 0 && (cap == 0 || cands), "null candidate table");
    need(budget_ms > 0.0, "budget must be positive");
    bm_config o{};
    bool fits = false;
    const std::vector<bm_candidate> all = bm::autotune(*in, x, voxel_tol, 0.0, reps, o, st, budget_ms, &fits);
    for (int i = 0; i < cap && i < int(all.size()); ++i) cands[i] = all[i];
    if (ncands) *ncands = int(all.size());
    *out = o;
    if (!fits) bm::fail(BM_ERANGE, "no candidate fits the time budget; *out holds the fastest");
  });
}

bm_status bm_p8_create(const int64_t dims[3], int dtype, int L, bm_p8* out) {
  return guarded([&] {
    need(dims && out, "null argument");
    *out = nullptr;
    *out = bm::p8_create(dims, dtype, L);
  });
}

bm_status bm_p8_create_hybrid(const int64_t dims[3], int dtype, int L, int M, bm_p8* out) {
  return guarded([&] {
    need(dims && out, "null argument");
    *out = nullptr;
    *out = bm::p8_create(dims, dtype, L, M);
  });
}

bm_status bm_p8_destroy(bm_p8 p) {
  return guarded([&] { bm::p8_free(p); });
}

bm_status bm_p8_coeff_size(bm_p8 p, int64_t* elems) {
  return guarded([&] {
    need(p && elems, "null argument");
    *elems = bm::p8_coeff_size(*p);
  });
}

static void p8_check_device(const bm_p8_s* p) {
  int d = -1;
  BM_HIP(hipGetDevice(&d));
  if (d != bm::p8_device(*p)) bm::fail(BM_EINVAL, "the current device is not the plan's device");
}

bm_status bm_p8_decompose(bm_p8 p, const void* x, void* coeff, hipStream_t st) {
  return guarded([&] {
    need(p && x && coeff, "null argument");
    p8_check_device(p);
    bm::p8_decompose(*p, x, coeff, st);
  });
}

bm_status bm_p8_recompose(bm_p8 p, const void* coeff, void* x, hipStream_t st) {
  return guarded([&] {
    need(p && x && coeff, "null argument");
    p8_check_device(p);
    bm::p8_recompose(*p, coeff, x, st);
  });
}

bm_status bm_p8_block_grid(bm_p8 p, int64_t nb[3]) {
  return guarded([&] {
    need(p && nb, "null argument");
    bm::p8_block_grid(*p, nb);
  });
}

bm_status bm_p8_tolmap_from_voxels(bm_p8 p, const double* voxel_tol, double* block_tol, hipStream_t st) {
  return guarded([&] {
    need(p && voxel_tol && block_tol, "null argument");
    p8_check_device(p);
    bm::p8_tolmap_from_voxels(*p, voxel_tol, block_tol, st);
  });
}

bm_status bm_p8_quantize(bm_p8 p, const void* coeff, const double* block_tol, double eta, int32_t* codes,
                         hipStream_t st) {
  return guarded([&] {
    need(p && coeff && block_tol && codes, "null argument");
    p8_check_device(p);
    bm::p8_quantize(*p, coeff, block_tol, eta, codes, st);
  });
}

bm_status bm_p8_dequantize(bm_p8 p, const int32_t* codes, const double* block_tol, double eta, void* coeff,
                           hipStream_t st) {
  return guarded([&] {
    need(p && coeff && block_tol && codes, "null argument");
    p8_check_device(p);
    bm::p8_dequantize(*p, codes, block_tol, eta, coeff, st);
  });
}

bm_status bm_p8_decompose_quantize(bm_p8 p, const void* x, const double* block_tol, double eta, int32_t* codes,
                                   hipStream_t st) {
  return guarded([&] {
    need(p && x && block_tol && codes, "null argument");
    p8_check_device(p);
    bm::p8_decompose_quantize(*p, x, block_tol, eta, codes, st);
  });
}

bm_status bm_p8_dequantize_recompose(bm_p8 p, const int32_t* codes, const double* block_tol, double eta, void* x,
                                     hipStream_t st) {
  return guarded([&] {
    need(p && x && block_tol && codes, "null argument");
    p8_check_device(p);
    bm::p8_dequantize_recompose(*p, codes, block_tol, eta, x, st);
  });
}

bm_status bm_p8_compress(bm_p8 p, const void* x, const double* block_tol, double eta, void* out, size_t capacity,
                         size_t* out_bytes, hipStream_t st) {
  return guarded([&] {
    need(p && x && block_tol && out_bytes, "null argument");
    p8_check_device(p);
    bool too_fine = false;   // codes beyond 32 bits: store the raw data
    try {
      bm::p8_decompose_quantize(*p, x, block_tol, eta, bm::p8_codes(*p), st);
    } catch (const bm::Error& e) {
      if (e.code != BM_ERANGE) throw;
      too_fine = true;
    }
    if (!bm::write_container_p8(*p, x, block_tol, eta, too_fine, out, capacity, out_bytes, st))
      bm::fail(BM_ECAPACITY, "output buffer too small");
  });
}

bm_status bm_batch_create(int nfields, const bm_config* cfgs, bm_batch* out) {
  return guarded([&] {
    need(cfgs && out && nfields > 0, "null argument or empty batch");
    *out = bm::batch_build(nfields, cfgs);
  });
}

bm_status bm_batch_destroy(bm_batch b) {
  return guarded([&] { bm::batch_free(b); });
}

bm_status bm_batch_plan(bm_batch b, int field, bm_plan* out) {
  return guarded([&] {
    need(b && out, "null argument");
    need(field >= 0 && field < bm::batch_size(*b), "field index out of range");
    *out = bm::batch_plan(*b, field);
  });
}

bm_status bm_batch_decompose_quantize(bm_batch b, const void* const* x, const double* const* block_tol,
                                      int32_t* const* codes, int use_graph, int* n_overflow, hipStream_t st) {
  return guarded([&] {
    need(b && x && block_tol && codes, "null argument");
    for (int f = 0; f < bm::batch_size(*b); ++f) {
      need(x[f] && block_tol[f] && codes[f], "null field pointer");
      check_device(bm::batch_plan(*b, f));
    }
    bm::batch_decompose_quantize(*b, x, block_tol, codes, use_graph != 0, st);
    if (n_overflow) {
      std::vector<int> bad;
      *n_overflow = bm::batch_overflows(*b, bad, st);
    }
  });
}

bm_status bm_batch_dequantize_recompose(bm_batch b, const int32_t* const* codes, const double* const* block_tol,
                                        void* const* x, int use_graph, hipStream_t st) {
  return guarded([&] {
    need(b && x && block_tol && codes, "null argument");
    for (int f = 0; f < bm::batch_size(*b); ++f) {
      need(x[f] && block_tol[f] && codes[f], "null field pointer");
      check_device(bm::batch_plan(*b, f));
    }
    bm::batch_dequantize_recompose(*b, codes, block_tol, x, use_graph != 0, st);
  });
}

bm_status bm_batch_compress(bm_batch b, const void* const* x, const double* const* block_tol, void* const* out,
                            const size_t* capacity, size_t* out_bytes, int use_graph, hipStream_t st) {
  return guarded([&] {
    need(b && x && block_tol && out && capacity && out_bytes, "null argument");
    const int nf = bm::batch_size(*b);
    std::vector<int32_t*> codes(nf);
    for (int f = 0; f < nf; ++f) {
      need(x[f] && block_tol[f], "null field pointer");
      bm_plan_s& p = *bm::batch_plan(*b, f);
      check_device(&p);
      bm::check_block_tol(p, block_tol[f], st);
      bm::ensure_code_buffer(p);
      codes[f] = static_cast<int32_t*>(p.ws.codes);
    }
    bm::batch_decompose_quantize(*b, x, block_tol, codes.data(), use_graph != 0, st);
    std::vector<int> bad;
    bm::batch_overflows(*b, bad, st);
    bool short_buf = false;
    for (int f = 0; f < nf; ++f)
      if (!bm::write_container(*bm::batch_plan(*b, f), x[f], block_tol[f], bad[f] != 0, out[f], capacity[f], &out_bytes[f], st))
        short_buf = true;
    if (short_buf) bm::fail(BM_ECAPACITY, "an output buffer is too small (out_bytes holds the sizes needed)");
  });
}

bm_status bm_compressed_config(const void* in, size_t in_bytes, bm_config* cfg) {
  return guarded([&] {
    need(cfg != nullptr, "null cfg");
    *cfg = header_config(parse(in, in_bytes, false));
  });
}

bm_status bm_decompress(const void* in, size_t in_bytes, void* x, hipStream_t st) {
  return guarded([&] {
    need(x != nullptr, "null output");
    const CHeader h = parse(in, in_bytes, false);
    const uint8_t* pl0 = static_cast<const uint8_t*>(in) + sizeof(CHeader);
    CHeader z = h;
    z.crc = 0;
    const uint32_t hcrc = crc32(reinterpret_cast<const uint8_t*>(&z), sizeof(z));
    // the CRC over header and payload is checked before any plan is made: on
    // the host for a raw copy; for a coded payload with the stream's code
    // words and outlier values CRC'd on the device once they are uploaded
    std::unique_ptr<bm::HuffmanDecoder> dec;
    if (h.flags & 1u) {
      if (crc32_parallel(pl0, size_t(h.payload), hcrc) != h.crc) bm::fail(BM_ECORRUPT, "CRC mismatch");
    } else {
      // the stored map is checked before any plan or device buffer is made
      if (h.ntol < 1 || uint64_t(h.ntol) > h.payload / 8) bm::fail(BM_ECORRUPT, "tolerance map size mismatch");
      check_stored_tol(pl0, h.ntol);
      const size_t tb = size_t(h.ntol) * 8;
      dec = std::make_unique<bm::HuffmanDecoder>(pl0 + tb, size_t(h.payload) - tb, st);
      if (dec->crc(crc32(pl0, tb, hcrc)) != h.crc) bm::fail(BM_ECORRUPT, "CRC mismatch");
    }
    if (h.flags & bm::kFlagP8) {
      bm_p8_s* q = bm::p8_create(h.dims, h.dtype, h.L, h.M);
      struct Guard8 {
        bm_p8_s* q;
        double* d = nullptr;
        ~Guard8() {
          if (d) (void)hipFree(d);
          bm::p8_free(q);
        }
      } g8{q};
      const uint8_t* pl = static_cast<const uint8_t*>(in) + sizeof(CHeader);
      int64_t dims[3], nb[3];
      int dtype = 0, L = 0;
      size_t esize = 0;
      bm::p8_info(*q, dims, &dtype, &L, &esize);
      if (h.flags & 1u) {
        if (h.payload != uint64_t(dims[0] * dims[1] * dims[2]) * esize)
          bm::fail(BM_ECORRUPT, "raw payload size mismatch");
        BM_HIP(hipMemcpyAsync(x, pl, size_t(h.payload), hipMemcpyHostToDevice, st));
        BM_HIP(hipStreamSynchronize(st));
        return;
      }
      bm::p8_block_grid(*q, nb);
      const int64_t ntol = nb[0] * nb[1] * nb[2];
      if (h.ntol != ntol || h.payload < uint64_t(ntol) * 8) bm::fail(BM_ECORRUPT, "tolerance map size mismatch");
      BM_HIP(hipMalloc(&g8.d, size_t(ntol) * sizeof(double)));
      BM_HIP(hipMemcpyAsync(g8.d, pl, size_t(ntol) * 8, hipMemcpyHostToDevice, st));
      int32_t* codes = bm::p8_codes(*q);
      dec->decode(codes, bm::p8_coeff_size(*q));
      bm::p8_dequantize_recompose(*q, codes, g8.d, h.eta, x, st);
      BM_HIP(hipStreamSynchronize(st));
      return;
    }
    const bm_config c = header_config(h);
    bm_plan_s* p = bm_plan_build(&c);
    struct Guard {
      bm_plan_s* p;
      double* d = nullptr;
      ~Guard() {
        if (d) (void)hipFree(d);
        bm_plan_free(p);
      }
    } g{p};
    const uint8_t* pl = static_cast<const uint8_t*>(in) + sizeof(CHeader);
    const int64_t nlog = p->dims[0] * p->dims[1] * p->dims[2];
    if (h.flags & 1u) {
      if (h.payload != uint64_t(nlog) * p->esize) bm::fail(BM_ECORRUPT, "raw payload size mismatch");
      BM_HIP(hipMemcpyAsync(x, pl, size_t(h.payload), hipMemcpyHostToDevice, st));
      BM_HIP(hipStreamSynchronize(st));
      return;
    }
    const int64_t ntol = p->nb1[0] * p->nb1[1] * p->nb1[2];
    if (h.ntol != ntol || h.payload < uint64_t(ntol) * 8) bm::fail(BM_ECORRUPT, "tolerance map size mismatch");
    bm::ensure_code_buffer(*p);
    BM_HIP(hipMalloc(&g.d, size_t(ntol) * sizeof(double)));
    BM_HIP(hipMemcpyAsync(g.d, pl, size_t(ntol) * 8, hipMemcpyHostToDevice, st));
    const int64_t npad = p->pdims[0] * p->pdims[1] * p->pdims[2];
    dec->decode(static_cast<int32_t*>(p->ws.codes), npad);
    bm::dequantize_recompose(*p, static_cast<const int32_t*>(p->ws.codes), g.d, x, st);
    BM_HIP(hipStreamSynchronize(st));
  });
}

extern "C++" {
namespace bm {
void drain_timing(bm_plan_s& p) {
  for (auto& e : p.timing.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess &&
        e.slot < int(p.timing.ms.size())) {
      p.timing.ms[e.slot] += ms;
      p.timing.calls[e.slot] += 1;
    }
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  p.timing.pending.clear();
}
uint32_t container_crc(const uint8_t* p, size_t n) { return crc32_parallel(p, n, 0); }

void crc32_shift_matrix(uint64_t bytes, uint32_t out[32]) {
  for (int i = 0; i < 32; ++i) out[i] = crc32_shift(1u << i, bytes);
}

uint32_t crc_with_spans(const uint8_t* buf, size_t n, uint32_t crc, const CrcSpan* spans, int nspans) {
  // the shift over one block as four byte tables: Z(v) = T0[v & 255] ^ T1[..] ^ T2[..] ^ T3[v >> 24]
  static const std::vector<uint32_t> zt = [] {
    uint32_t m[32];
    crc32_shift_matrix(kCrcBlock, m);
    std::vector<uint32_t> t(4 * 256);
    for (int k = 0; k < 4; ++k)
      for (uint32_t b = 0; b < 256; ++b) t[k * 256 + b] = gf2_apply(m, b << (8 * k));
    return t;
  }();
  size_t at = 0;
  for (int i = 0; i < nspans; ++i) {
    const CrcSpan& d = spans[i];
    const size_t done = d.block_crc.size() * kCrcBlock;
    if (d.offset < at || d.offset + d.bytes > n || done > d.bytes)
      fail(BM_EINVAL, "stream CRC: the device parts do not match the stream");
    crc = crc32_parallel(buf + at, d.offset - at, crc);    // host bytes before the span
    // the span: the device's block CRCs in order, then its last partial block
    uint32_t w = 0;
    for (uint32_t b : d.block_crc)
      w = (zt[w & 255u] ^ zt[256 + ((w >> 8) & 255u)] ^ zt[512 + ((w >> 16) & 255u)] ^ zt[768 + (w >> 24)]) ^ b;
    w = crc32_parallel(buf + d.offset + done, d.bytes - done, w);
    crc = crc32_shift(crc, d.bytes) ^ w;
    at = d.offset + d.bytes;
  }
  return crc32_parallel(buf + at, n - at, crc);
}

uint32_t stream_crc(const HuffmanEncoder& e, const uint8_t* stream, size_t n, uint32_t crc) {
  return crc_with_spans(stream, n, crc, e.device_spans(), 2);
}
}  // namespace bm
}  // extern "C++"
using bm::drain_timing;

bm_status bm_model_calibrate(int dtype, int block, bm_model* out, hipStream_t st) {
  return guarded([&] {
    need(out != nullptr, "null model");
    bm_model m{};
    bm::model_calibrate(dtype, block, m, st);
    *out = m;
  });
}

bm_status bm_model_predict(const bm_model* model, const bm_config* cfg, double ms[4]) {
  return guarded([&] {
    need(model && cfg && ms, "null argument");
    double t[4];
    bm::model_predict(*model, *cfg, t);
    for (int k = 0; k < 4; ++k) ms[k] = t[k];
  });
}

bm_status bm_select_levels(const bm_config* in, const bm_model* model, double budget_ms, bm_config* out,
                           bm_candidate* cands, int cap, int* ncands) {
  return guarded([&] {
    need(in && model && out, "null argument");
    std::vector<bm_candidate> c;
    bm_config o{};
    const bool fits = bm::select_levels(*in, *model, budget_ms, o, c);
    *out = o;
    if (ncands) *ncands = int(c.size());
    if (cands)
      for (int k = 0; k < cap && k < int(c.size()); ++k) cands[k] = c[k];
    if (!fits) bm::fail(BM_ERANGE, "no (L, M) fits the time budget; *out holds the fastest predicted");
  });
}

bm_status bm_timing(bm_plan p, int enable) {
  return guarded([&] {
    need(p != nullptr, "null plan");
    drain_timing(*p);
    p->timing.ms.assign(2 * p->nlev + 2, 0.0);
    p->timing.calls.assign(2 * p->nlev + 2, 0);
    p->timing.on = enable != 0;
  });
}

bm_status bm_timing_get(bm_plan p, double* ms, int64_t* calls, int cap, int* n) {
  return guarded([&] {
    need(p && n, "null argument");
    drain_timing(*p);
    const int k = int(p->timing.ms.size());
    *n = k;
    for (int i = 0; i < k && i < cap; ++i) {
      if (ms) ms[i] = p->timing.ms[i];
      if (calls) calls[i] = p->timing.calls[i];
    }
  });
}

const char* bm_status_string(bm_status s) {
  switch (s) {
    case BM_OK: return "ok";
    case BM_EINVAL: return "invalid argument";
    case BM_ENOMEM: return "out of memory";
    case BM_EHIP: return "HIP runtime error";
    case BM_ENONFINITE: return "non-finite value";
    case BM_ECAPACITY: return "output buffer too small";
    case BM_ECORRUPT: return "corrupt stream";
    case BM_ERANGE: return "code out of range";
    case BM_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* bm_last_error(void) { return g_err.c_str(); }

const char* bm_version(void) { return "blockmgard-mi355x 0.1"; }

}  // extern "C"
