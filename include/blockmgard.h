/*
 * blockmgard.h -- C ABI of the BlockMGARD hot path for AMD MI355X (gfx950).
 *
 * The library decomposes a 3D field with a hybrid hierarchy of In-cache
 * Block levels followed by global MGARD levels, quantizes the coefficients
 * under a per-region L-infinity bound, and entropy-codes the result.
 *
 * Paper passages each call implements (BlockMGARD, SC'26):
 *   decompose / recompose ........ Sec. II-B (multilevel decomposition, its
 *                                  exact inverse), Sec. IV-A (In-cache
 *                                  Block levels), Sec. IV-B (hybrid
 *                                  hierarchy of L local + M global levels)
 *   tolerance maps, quantize ..... Sec. IV-C (block-wise tolerance map,
 *                                  conservative propagation, Eq. 2, global
 *                                  budget), Sec. IV-D (per-block
 *                                  reciprocal quantizer), Sec. V-A (REL
 *                                  L-infinity bound)
 *   compress / decompress ........ Sec. IV (transform -> quantize -> lossless
 *                                  pipeline), Sec. IV-B (Huffman stages),
 *                                  Sec. V-F (raw copy of incompressible data)
 *
 * Conventions (apply to every call):
 *   - Arrays are dense, C order [z][y][x], x fastest.  "dims" are {nz,ny,nx}.
 *   - Device pointers are HIP device memory owned by the caller; host
 *     pointers are ordinary host memory owned by the caller.  The library
 *     never frees caller memory.
 *   - A plan owns its constant tables and device workspace, and keeps
 *     state between calls: buffers that first calls allocate
 *     (bm_workspace_size), a kept map's quantizer tables
 *     (bm_quant_prepare), a planned container (bm_compress_plan).  Calls on
 *     one plan must not overlap in time, from one thread on several streams
 *     or from several threads (they share the workspace); different plans
 *     are independent.
 *   - Calls are stream-ordered and asynchronous unless documented as
 *     synchronous.  Passing stream 0 uses the null stream.
 *   - Every call returns a bm_status.  No C++ exception crosses the ABI.
 *     On error, bm_last_error() returns a thread-local message, and no
 *     caller-visible output except an out_bytes size has been written.
 *   - The plan's device is the device current at bm_plan_create; calls
 *     must be made with that device current.
 *   - Environment: BM_PLANE_PASS=0 at bm_plan_create gives the plan one
 *     launch per axis in every global level instead of the plane pass that
 *     runs x and y together (a diagnostic switch: the results are the same
 *     bit for bit, only slower).
 */
#ifndef BLOCKMGARD_H
#define BLOCKMGARD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int bm_status;
enum {
  BM_OK = 0,
  BM_EINVAL = -1,        /* bad argument: shape, block size, levels, null pointer */
  BM_ENOMEM = -2,        /* device or host allocation failed */
  BM_EHIP = -3,          /* a HIP runtime call failed (message names it) */
  BM_ENONFINITE = -4,    /* NaN or Inf in the data or in a tolerance */
  BM_ECAPACITY = -5,     /* output buffer too small; *out_bytes holds the size needed */
  BM_ECORRUPT = -6,      /* compressed stream fails its magic, version, size or CRC check */
  BM_ERANGE = -7,        /* a quantization code does not fit in 32 bits */
  BM_EUNSUPPORTED = -8   /* valid request outside what this library implements */
};

typedef enum { BM_F32 = 0, BM_F64 = 1 } bm_dtype;

/* Plan configuration, filled by the caller and copied by bm_plan_create.
 *   ndim     3 (1 and 2 are accepted as 3D with leading unit dims)
 *   dims     logical dims {nz, ny, nx}
 *   dtype    BM_F32 or BM_F64: the type of data and coefficients
 *   block    b in {9, 17, 33}: nodes per block side of the local levels
 *            (blocks of 2^k+1 nodes share one face with each neighbour);
 *            ignored when L == 0.  b = 33 runs each block level as two
 *            launches (three when recomposing) through a plan-owned scratch
 *            array, its transposes likewise; batches do not take b = 33
 *            (BM_EUNSUPPORTED)
 *   L, M     number of local (In-cache Block) and global levels (Sec. IV-B)
 *   pad_mode 0 = clamp (padded nodes copy the nearest node), 1 = zero fill
 *   eta      safety share of every tolerance kept back for working-precision
 *            rounding, in [0, 0.5); the quantizer uses tau * (1 - eta).
 *   nested   0: every block level re-tiles its grid with b-node blocks.
 *            1: the nested schedule (several block levels inside one block
 *            region, Sec. IV-A): block level s uses (b-1)/2^(s-1)+1-node
 *            blocks, which cover exactly the level-1 block regions; each
 *            level's block must have at least 9 nodes (b = 17: L <= 2;
 *            b = 33: L <= 3), else BM_EINVAL.  Results differ from 0 from
 *            the second block level on.  Batches take it with b = 17
 *            (every field of a batch on one schedule).  Zero-initialised
 *            configs get 0. */
typedef struct {
  int ndim;
  int64_t dims[3];
  int dtype;
  int block;
  int L;
  int M;
  int pad_mode;
  double eta;
  int nested;
} bm_config;

typedef struct bm_plan_s* bm_plan;

/* Per-call quantization statistics (filled synchronously when non-NULL). */
typedef struct {
  int64_t n_codes;       /* number of coefficients quantized (= padded node count) */
  int64_t n_outliers;    /* codes with |q| >= 2^15 (escaped in the Huffman stage) */
  int64_t max_abs_code;  /* max |q| */
} bm_qstats;

/* ---- plans ------------------------------------------------------------ */

/* Validate cfg and build a plan: padded dims, level schedule, per-level
 * gains and device workspace.  The padded length of every axis is the
 * smallest n' >= n on which the L block levels tile exactly and each of the
 * M global levels halves an odd length (lengths <= 2 are left alone).
 * Errors: BM_EINVAL (bad shape/b/L/M/eta, a padded grid of more than 2^40
 * nodes, null), BM_EUNSUPPORTED (a global level would run line solves on an
 * axis of more than 1151 nodes, i.e. more than 576 coarse nodes per line:
 * add a block level), BM_ENOMEM, BM_EHIP. */
bm_status bm_plan_create(const bm_config* cfg, bm_plan* out);

/* Free a plan and its workspace.  NULL is accepted. */
bm_status bm_plan_destroy(bm_plan plan);

/* The configuration the plan was built from (a batch field's L resolved). */
bm_status bm_plan_config(bm_plan plan, bm_config* cfg);

/* Padded dims n' (the coefficient array's dims). */
bm_status bm_coeff_shape(bm_plan plan, int64_t padded_dims[3]);

/* Device memory the plan holds now, in bytes: the workspace built with it
 * (the compact grids of every level after the first, the global levels'
 * pass temporaries, the first global level's partial load vectors, the
 * tolerance maps and quantizer tables, the Thomas pivots) plus buffers that
 * calls add on first use and keep until bm_plan_destroy: the padded code
 * array of bm_compress / bm_compress_plan / bm_decompress and the batch
 * (padded nodes x 4), the padded coefficient array of bm_qoi_deltas and the
 * adjoint's padded gradient (padded nodes x sizeof dtype each), and the
 * quantizer's task table.  The plan
 * owns all of it; a caller cannot supply its own.  Host memory (pinned
 * staging of the box list) is not counted.  Errors: BM_EINVAL (null). */
bm_status bm_workspace_size(bm_plan plan, size_t* bytes);

/* Number of level-1 blocks per axis ({1,1,1} when L == 0): the shape of the
 * block tolerance map taken by the quantizer. */
bm_status bm_block_grid(bm_plan plan, int64_t nblocks[3]);

/* Rounded-up L-infinity gain A_s of the detail coefficients of level s
 * (s = 1..L+M), written to gains[0..L+M-1] (host).  Sec. II-B budget. */
bm_status bm_level_gains(bm_plan plan, double* gains);

/* ---- transform (Sec. II-B, IV-A, IV-B) ---------------------------------- */

/* coeff = D(x).  x: device, logical dims, dtype of the plan.  coeff: device,
 * padded dims, same dtype; every node holds its own coefficient ("in
 * place"): the detail of the level at which the node leaves the grid, or
 * the coarsest value.  Asynchronous on stream; the data are not checked (a
 * NaN or Inf in x gives non-finite coefficients, which the quantizing calls
 * report as BM_ENONFINITE). */
bm_status bm_decompose(bm_plan plan, const void* x, void* coeff, hipStream_t stream);

/* x = R(coeff) = D^{-1}(coeff), cropped to the logical dims.  Asynchronous. */
bm_status bm_recompose(bm_plan plan, const void* coeff, void* x, hipStream_t stream);

/* gx = D^T(gcoeff): gradient of <D(x), gcoeff> with respect to x, the
 * transpose of the linear map of bm_decompose (the levels of Sec. II-B and
 * the block levels of Sec. IV-A, applied in reverse order).  gcoeff: device,
 * padded dims, in-place layout as bm_decompose writes it; gx: device, logical
 * dims, dtype of the plan (overwritten).  Padded nodes' gradients are added
 * into the nodes their clamped value came from (dropped under zero fill).
 * Uses the plan's grid buffers (and, on a padded grid with block levels, one
 * padded-size buffer allocated on first use).  Asynchronous on stream. */
bm_status bm_decompose_adjoint(bm_plan plan, const void* gcoeff, void* gx, hipStream_t stream);

/* gcoeff = R^T(gx): gradient of <R(coeff), gx> with respect to coeff, e.g. the
 * sensitivities of a linear quantity of interest of the reconstruction.
 * gx: device, logical dims; gcoeff: device, padded dims, in-place layout
 * (overwritten).  Asynchronous on stream. */
bm_status bm_recompose_adjoint(bm_plan plan, const void* gx, void* gcoeff, hipStream_t stream);

/* ---- ROI tolerance maps (Sec. IV-C) ------------------------------------- */

/* Level-1 block tolerance map from half-open boxes.  boxes (host): nbox
 * records {z0,y0,x0,z1,y1,x1,abs_tol} in logical node coordinates;
 * background: absolute tolerance elsewhere.  A block takes the minimum over
 * the nodes of its closed range (a partly covered block is strict); padded
 * nodes count as the node they copy.  block_tol (device, double,
 * bm_block_grid entries; 1 entry when L == 0).  Asynchronous.
 * Errors: BM_EINVAL, BM_ENONFINITE (tolerance <= 0 or not finite). */
bm_status bm_tolmap_from_boxes(bm_plan plan, const double* boxes, int nbox, double background,
                               double* block_tol, hipStream_t stream);

/* Level-1 block tolerance map from a per-voxel absolute tolerance (device,
 * double, logical dims): min over each block's closed node range.
 * Asynchronous. */
bm_status bm_tolmap_from_voxels(bm_plan plan, const double* voxel_tol, double* block_tol,
                                hipStream_t stream);

/* ---- quantization (Sec. IV-C, IV-D) ------------------------------------- */

/* codes = rint(c * (1/Delta)) per node (FP64), with Delta = 2 tau (1 - eta) w_s / A_s
 * for a detail of level s and 2 tau (1 - eta) w_c for a coarsest value
 * (Sec. II-B level-dependent budget, Sec. IV-C).  A_s = bm_level_gains.
 * Shares: w_s = (details of level s) / (padded node count) for a block level;
 * the M global levels split (their details) / (node count) equally; w_c =
 * (coarsest values) / (node count); every share below 1/(64 T), T = L + M + 1,
 * is raised to it and the shares are then divided by their sum.  tau is the
 * node's propagated block tolerance at block levels (min over the level's
 * blocks that contain it, block maps propagated by Eq. 2), tau_global = min
 * over the last block level at global levels (and for the coarsest values
 * when M > 0; with M = 0 they keep their node's tau).  coeff: device, padded
 * dims; block_tol: device double map from the calls above; codes: device
 * int32, padded dims.  If stats is non-NULL the call synchronizes the stream
 * and fills it; then a NaN or infinite coefficient returns BM_ENONFINITE and
 * a code beyond int32 range BM_ERANGE. */
bm_status bm_quantize_roi(bm_plan plan, const void* coeff, const double* block_tol, int32_t* codes,
                          bm_qstats* stats, hipStream_t stream);

/* coeff = (dtype)(codes * Delta) with the same Delta.  Asynchronous. */
bm_status bm_dequantize(bm_plan plan, const int32_t* codes, const double* block_tol, void* coeff,
                        hipStream_t stream);

/* Per-coefficient bin widths for a linear quantity of interest Q(x) = <g, x>
 * (the adjoint-guided bounds): s = R^T g gives each coefficient's
 * sensitivity, so quantization moves Q by at most sum |s_i| Delta_i / 2.
 * Every Delta_i is capped by the node's L-inf width cap_i from block_tol (so
 * that map's bounds still hold); below the caps every coefficient takes the
 * same share: |s_i| Delta_i / 2 = min(|s_i| cap_i / 2, lambda), lambda the
 * largest level with sum_i min(|s_i| cap_i / 2, lambda) <= (1 - eta) tol_q
 * (found to the last bit by a bracketing search; no such limit when the caps
 * already fit, and then Delta = cap).  These widths maximise the sum of
 * log Delta_i (the bits saved) under both bounds.  g: device, logical dims,
 * dtype of the plan; delta: device, padded dims, FP64 (written);
 * *n_set (if non-NULL) = the number of coefficients whose width the
 * quantity sets (Delta_i < cap_i).  Synchronous (a few host round trips).
 * Errors: BM_ENONFINITE (tol_q not positive and finite). */
bm_status bm_qoi_deltas(bm_plan plan, const void* g, double tol_q, const double* block_tol, double* delta,
                        int64_t* n_set, hipStream_t stream);

/* Quantization with an explicit per-node Delta (device, padded dims, FP64):
 * q = rint(c * (1 / Delta_i)) in FP64; stats as bm_quantize_roi. */
bm_status bm_quantize_delta(bm_plan plan, const void* coeff, const double* delta, int32_t* codes,
                            bm_qstats* stats, hipStream_t stream);

/* coeff = (dtype)(codes * Delta_i).  Asynchronous. */
bm_status bm_dequantize_delta(bm_plan plan, const int32_t* codes, const double* delta, void* coeff,
                              hipStream_t stream);

/* Fused decompose + quantize (the paper's fused pipeline, Sec. IV-D): the
 * block levels write codes straight from on-chip memory; global-level
 * details are quantized as they are produced.  codes (device int32, padded
 * dims) equal bm_decompose followed by bm_quantize_roi with the same map.
 * If stats is non-NULL the call synchronizes and returns BM_ENONFINITE when
 * x holds a NaN or Inf (it reaches the coefficient of its own node), else
 * BM_ERANGE for a code beyond int32 (n_outliers and max_abs_code are -1:
 * not counted).  Without stats nothing is checked. */
bm_status bm_decompose_quantize(bm_plan plan, const void* x, const double* block_tol, int32_t* codes,
                                bm_qstats* stats, hipStream_t stream);

/* Fused dequantize + recompose: x equals bm_dequantize followed by
 * bm_recompose.  Asynchronous. */
bm_status bm_dequantize_recompose(bm_plan plan, const int32_t* codes, const double* block_tol, void* x,
                                  hipStream_t stream);

/* Keep the quantizer tables of one block tolerance map in the plan (Sec.
 * IV-C: Eq. 2 propagation of the map to every block level, the per-block
 * Delta classes of every level and tau_global).  Every quantizing call
 * (bm_quantize_roi, bm_dequantize, bm_decompose_quantize,
 * bm_dequantize_recompose, bm_compress) builds these tables from its map
 * first, a few launches (about 20 us at 512^3); after this call, calls
 * given the same block_tol pointer use the kept tables instead.  The map's
 * contents must not change while it is kept (call again after changing
 * them), and later calls on another stream must be ordered after this one.
 * A call with another map builds its own tables over the kept ones and
 * drops them; block_tol = NULL drops them.  Stream-ordered. */
bm_status bm_quant_prepare(bm_plan plan, const double* block_tol, hipStream_t stream);

/* ---- lossless stage (Sec. IV-B lossless stages) ----------------------- */

/* Canonical Huffman coding of n int32 codes (device) in raster order.
 * Symbols are q + 2^15 for |q| < 2^15, else the escape symbol 0; the value q
 * of every escaped code is kept as an outlier, in raster order (its position
 * is that of its escape symbol).  Output (host) layout, little endian:
 *   uint32 magic 0x46484D42 ("BMHF"), uint32 version 3,
 *   int64 n, int64 nchunks, int64 nwords, int64 noutliers, int64 npresent,
 *   uint16 symbol[npresent] (ascending), uint8 length[npresent] (code
 *   lengths of the symbols that occur; absent symbols have no code),
 *   uint64 chunk_offsets[nchunks+1] (in words),
 *   uint64 outlier_offsets[nchunks+1] (outliers before each chunk),
 *   uint32 words[nwords] (each chunk of 4096 symbols packed MSB-first,
 *   starting on a word), int32 outlier_value[noutliers].
 * Synchronous.  BM_ECAPACITY sets *out_bytes to the size needed. */
bm_status bm_huffman_encode(const int32_t* codes, int64_t n, void* out, size_t capacity,
                            size_t* out_bytes, hipStream_t stream);

/* bm_huffman_encode in two calls, so a caller that sizes its buffer from the
 * first does not plan the stream twice: bm_huffman_plan runs the histogram,
 * code table and chunk sizes of codes (device, n entries; synchronous) and
 * returns a handle and the stream's exact size; bm_huffman_write encodes into
 * out (host, capacity bytes; synchronous) the bytes bm_huffman_encode
 * writes, and may be called again.  codes must stay allocated and unchanged
 * until the last write.  bm_huffman_destroy frees the handle (NULL is
 * accepted).  Errors: BM_EINVAL (bad n or pointer), BM_ECAPACITY (out too
 * small; *out_bytes holds the size). */
typedef struct bm_huffman_s* bm_huffman;
bm_status bm_huffman_plan(const int32_t* codes, int64_t n, bm_huffman* out, size_t* out_bytes, hipStream_t stream);
bm_status bm_huffman_write(bm_huffman h, void* out, size_t capacity, size_t* out_bytes);
bm_status bm_huffman_destroy(bm_huffman h);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): bm_huffman_encode
 * with the stream written to device memory.  out (device, capacity bytes)
 * receives exactly the bytes bm_huffman_encode writes; codes: device int32,
 * 0 <= n <= 2^28 (else BM_EINVAL).  Nothing is allocated, on the device or the
 * host: the work arrays (histogram, code table, per-chunk bit and escape
 * counts and offsets: 2.3 MiB) live in a fixed device array of the library,
 * one copy per GPU held until the process ends, and in static host arrays.
 * Calls are serialised on the host; calls that overlap in time on one GPU
 * (from other processes or streams) race on that GPU's copy.  Synchronous.
 * BM_ECAPACITY sets *out_bytes to the size needed and writes nothing. */
bm_status bm_huffman_encode_device(const int32_t* codes, int64_t n, void* out, size_t capacity, size_t* out_bytes,
                                   hipStream_t stream);

/* Inverse of bm_huffman_encode into codes (device, n entries).  Synchronous.
 * Each chunk is decoded by one wavefront whose lanes split its bits.
 * Errors: BM_ECORRUPT for a malformed stream (a chunk that does not decode
 * to exactly its 4096 symbols within its own words, or to its outlier
 * count), BM_EINVAL if n mismatches. */
bm_status bm_huffman_decode(const void* in, size_t in_bytes, int32_t* codes, int64_t n,
                            hipStream_t stream);

/* The code lengths of the lossless stage's canonical Huffman code for a
 * symbol histogram, on the host (no GPU; the step the encoder runs between
 * its histogram and its chunk sizes, Sec. IV-B).  hist: 65536 counts
 * (symbol q + 32768 for |q| < 32768, symbol 0 the escape), len: 65536 code
 * lengths out (0 for absent symbols).  Huffman's algorithm merging the two
 * smallest (weight, smallest symbol in the subtree) keys; lengths above 32
 * cut to 32, then the longest codes below 32 lengthened (largest symbol
 * first) until Kraft's sum is <= 1.  Errors: BM_EINVAL for a null pointer. */
bm_status bm_huffman_code_lengths(const uint64_t* hist, uint8_t* len);

/* Stage times (ms) of the calling thread's last Huffman encode (by
 * bm_huffman_encode, bm_compress or bm_batch_compress) and last decode (by
 * bm_huffman_decode or bm_decompress), the lossless stages of Sec. IV-B.
 * Device stages are timed with events on the call's stream, host stages with
 * a steady clock.  Encode: enc_hist (histogram, device), enc_table (code
 * lengths and canonical codes, host), enc_sizes (per-chunk bit and escape
 * counts on the device, offsets on the host), enc_encode (device; with
 * the CRC-32 of each 16 KiB block of the words and outlier values),
 * enc_copy (the stream's words and outliers to the host), enc_crc (the
 * container's CRC-32 from those block CRCs and the host's bytes; 0 outside
 * bm_compress).  Decode:
 * dec_parse (header checks and decode tables, host), dec_upload (tables,
 * offsets, words and outliers to the device), dec_decode (device).  enc_n
 * and dec_n: symbols of those calls (0: none yet).  Never fails. */
typedef struct {
  double enc_hist_ms, enc_table_ms, enc_sizes_ms, enc_encode_ms, enc_copy_ms, enc_crc_ms;
  double dec_parse_ms, dec_upload_ms, dec_decode_ms;
  int64_t enc_n, dec_n;
} bm_lossless_times;
bm_status bm_lossless_last_times(bm_lossless_times* out);

/* ---- end to end (Sec. IV, V-F) -------------------------------------------- */

/* Decompose, quantize with block_tol (device map as above) and Huffman-code x
 * (device) into a self-describing host buffer: header (config, gains),
 * block tolerance map, Huffman stream, CRC-32 (polynomial 0xEDB88320, as
 * zlib) of the header with its CRC field zeroed followed by the payload.  If
 * the coded form is not smaller than the raw data the raw bytes are stored
 * instead (Sec. V-F).  Synchronous.  The stream is planned once (histogram,
 * code table, chunk sizes) and encoded straight into out.  BM_ECAPACITY sets
 * *out_bytes to the size needed (that call plans the stream but does not
 * encode it).
 * BM_ENONFINITE: NaN or Inf in x or in block_tol (nothing is written). */
bm_status bm_compress(bm_plan plan, const void* x, const double* block_tol, void* out,
                      size_t capacity, size_t* out_bytes, hipStream_t stream);

/* bm_compress in two calls, so a caller that sizes its buffer from the
 * result does not decompose, quantize and plan twice.  bm_compress_plan does
 * all but the writing (decompose, quantize, histogram, code table, chunk
 * sizes; synchronous), keeps the pending container in the plan and sets
 * *out_bytes to its exact size; bm_compress_write writes it to out (host,
 * capacity bytes; synchronous) and drops it.  x and block_tol must not change
 * in between (the raw copy reads x when written).  Another bm_compress or
 * bm_compress_plan on the plan drops a pending container; bm_compress_write
 * without one: BM_EINVAL; a buffer too small: BM_ECAPACITY, the container
 * stays pending.  Errors of the plan step as bm_compress. */
bm_status bm_compress_plan(bm_plan plan, const void* x, const double* block_tol, size_t* out_bytes,
                           hipStream_t stream);
bm_status bm_compress_write(bm_plan plan, void* out, size_t capacity, size_t* out_bytes);

/* Read the configuration stored in a compressed buffer (host, synchronous).
 * Checks the header (magic, version, payload size), not the CRC: a call that
 * only sizes the destination does not pay for a pass over the payload;
 * bm_decompress verifies the CRC.  Errors: BM_ECORRUPT. */
bm_status bm_compressed_config(const void* in, size_t in_bytes, bm_config* cfg);

/* Rebuild x (device, logical dims and dtype of the stored config) from a
 * buffer written by bm_compress.  Synchronous.  The CRC is checked before
 * anything is decoded (the stream's words and outlier values in 16 KiB
 * blocks on the device, once uploaded).  Errors: BM_ECORRUPT (bad magic,
 * version, size or CRC, or a stored block tolerance that is not positive
 * and finite). */
bm_status bm_decompress(const void* in, size_t in_bytes, void* x, hipStream_t stream);

/* ---- many fields (the paper's batched multi-field workloads, Sec. V) ------- */

/* A batch of independent fields sharing dtype and block size (each its own
 * dims and L, M).  The fused pipeline of all fields runs as one launch per
 * stage of the quantizer-table preparation, one persistent launch per block
 * level covering the blocks of every field that has that level, and each
 * field's global levels.  With use_graph the sequence is captured once in a
 * HIP graph (per set of bound pointers) and replayed; use_graph needs a
 * stream other than the null stream.  The batch owns one plan per field
 * (bm_batch_plan borrows it: coefficient shapes, tolerance maps); a batch is
 * used from one stream at a time.  With the nested schedule (b = 17, every
 * field) a field's 17- and 9-node levels run as one pair: one persistent
 * launch covers the pairs of all such fields, beside the plain launch of
 * the fields with one block level.  A 33-node level runs its column,
 * coarse (and, recomposing, interpolation) steps as one persistent launch
 * each over the block halves or blocks of every field.  Errors: BM_EINVAL
 * (mixed dtype, block size or schedule, null pointers), BM_EUNSUPPORTED (the
 * nested schedule with b != 17), BM_ENOMEM.  A field config with L = -1
 * takes the most block levels its logical dims tile without padding (at
 * least 1; nested: 2 when they tile, else 1);
 * bm_plan_config of the field's bm_batch_plan returns the resolved config. */
typedef struct bm_batch_s* bm_batch;
bm_status bm_batch_create(int nfields, const bm_config* cfgs, bm_batch* out);
bm_status bm_batch_destroy(bm_batch batch);
bm_status bm_batch_plan(bm_batch batch, int field, bm_plan* out);

/* codes[f] = the fused decompose + ROI quantize of x[f] with block_tol[f]
 * (arrays of nfields device pointers; layouts as bm_decompose_quantize).
 * Asynchronous, unless n_overflow is non-null: then the call waits and
 * stores the number of fields whose codes did not fit in 32 bits, or
 * returns BM_ENONFINITE if a field's data hold a NaN or Inf. */
bm_status bm_batch_decompose_quantize(bm_batch batch, const void* const* x, const double* const* block_tol,
                                      int32_t* const* codes, int use_graph, int* n_overflow, hipStream_t stream);

/* x[f] = the fused dequantize + recompose of codes[f].  Asynchronous. */
bm_status bm_batch_dequantize_recompose(bm_batch batch, const int32_t* const* codes, const double* const* block_tol,
                                        void* const* x, int use_graph, hipStream_t stream);

/* bm_compress of every field: out[f] (host) receives field f's container
 * (capacity[f] bytes available, out_bytes[f] written or needed); a field
 * whose codes overflow is stored raw.  Synchronous.  BM_ECAPACITY if any
 * buffer is too small (out_bytes then holds every needed size). */
bm_status bm_batch_compress(bm_batch batch, const void* const* x, const double* const* block_tol, void* const* out,
                            const size_t* capacity, size_t* out_bytes, int use_graph, hipStream_t stream);

/* ---- choice of (b, L, M) (the hybrid split of Sec. IV-B, by measurement) -- */

typedef struct {
  int block, L, M;        /* block 0: no block levels */
  int status;             /* BM_OK, or BM_ERANGE: codes overflow, stored raw */
  double ms;              /* fused decompose + quantize, median of the repetitions */
  double ratio;           /* raw bytes / container bytes at the given tolerances */
  int nested;             /* 1: the nested block schedule (bm_config.nested) */
  double lossless_ms;     /* Huffman encode of its codes into host memory (histogram, code
                             table, chunk sizes, encode, copy out), host wall time; 0 when
                             the codes overflow */
} bm_candidate;

/* Chooses block size and level split for field x (device, logical dims and
 * dtype of *in) under a per-voxel absolute tolerance (device, logical dims,
 * FP64).  Candidates: pure global M = 1..6; b in {9, 17, 33} with L = 1..4 and
 * M = 0..4, in the plain schedule and, for L >= 2, in the nested one; those
 * the dims admit (a valid plan padding the volume by at most 1/8).  Each is run: median time of `reps` fused decompose + quantize runs
 * and the exact Huffman-coded size.  The fastest candidate whose ratio is at
 * least (1 - slack) times the best ratio wins; *out is *in with block, L, M
 * set.  cands (optional, room for cap entries) receives the measured table
 * and *ncands its length.  Synchronous.  Errors: BM_EINVAL (no admissible
 * candidate, slack outside [0, 1)). */
bm_status bm_autotune(const bm_config* in, const void* x, const double* voxel_tol, double slack, int reps,
                      bm_config* out, bm_candidate* cands, int cap, int* ncands, hipStream_t stream);

/* The same candidates and measurements, chosen by the rule of Algorithm 1
 * (Sec. IV-B) under a time budget: of the candidates whose pipeline time
 * ms + lossless_ms (fused decompose + quantize, then the Huffman encode of
 * their codes) is at most budget_ms, the one with the most global levels M,
 * then the fewest block levels L, then the best ratio (between block sizes).
 * bm_select_levels applies the same rule to predicted times of the same
 * stages.
 * Errors: BM_ERANGE when no candidate fits (*out, the table and *ncands are
 * still filled, *out with the candidate of the shortest pipeline time),
 * BM_EINVAL (budget not positive, no admissible candidate).  Synchronous. */
bm_status bm_autotune_budget(const bm_config* in, const void* x, const double* voxel_tol, double budget_ms, int reps,
                             bm_config* out, bm_candidate* cands, int cap, int* ncands, hipStream_t stream);

/* ---- choice of (L, M) from a time model (Sec. IV-B, Eq. 1, Algorithm 1) -- */

/* Fitted stage times of the pipeline for one dtype and block size (ms, N as
 * noted).  Eq. 1: a block level of N blocks takes 1/Slope + N/TP_peak, i.e.
 * blk_lat_ms + N / blk_tp (blk_tp = TP_peak in blocks per ms, Slope =
 * 1/blk_lat_ms); the last block level before a global level (it forms that
 * level's details and partial load vectors) has its own fit (fblk_*).  A
 * global level of N nodes takes glob_a_ms + glob_b_ms N; the first global
 * level after a block level, which only gathers and solves, fglob_*.
 * Quantization, fitted apart for the local and the global quantizer as
 * Sec. IV-B does: max(q_slope_ms N_s, q_lat_ms) for each block level s (its
 * per-block tables; N_s its grid's nodes), max(gq_slope_ms N, gq_lat_ms)
 * for an all-global hierarchy (N its padded nodes).  Lossless: stage k of the Huffman coder (0
 * histogram, 1 code table, 2 chunk sizes and encode, 3 copy-out and CRC)
 * takes huf_a_ms[k] + huf_b_ms[k] N for N codes. */
typedef struct {
  int dtype, block;
  double blk_lat_ms, blk_tp;
  double fblk_lat_ms, fblk_tp;
  double fglob_a_ms, fglob_b_ms;
  double glob_a_ms, glob_b_ms;
  double q_slope_ms, q_lat_ms;
  double huf_a_ms[4], huf_b_ms[4];
  double gq_slope_ms, gq_lat_ms;
} bm_model;

/* Fits every stage of *out on this device (the device current at the call):
 * each stage runs on synthetic inputs of growing size (cubes of 1 to 32
 * blocks per side, global grids 17^3 to 513^3, 2^16 to 2^26 codes), timed by
 * HIP events and host clocks, and a least-squares line is taken through the
 * (N, time) points.  Synchronous; takes a few seconds and about 2 GB of
 * device memory.  Errors: BM_EINVAL (dtype, block not 9/17/33). */
bm_status bm_model_calibrate(int dtype, int block, bm_model* out, hipStream_t stream);

/* Predicted times of cfg under the model (its dtype and block replace
 * cfg's): ms[0] decomposition (sum over the levels), ms[1] quantization,
 * ms[2] lossless stage, ms[3] their sum.  Host only. */
bm_status bm_model_predict(const bm_model* model, const bm_config* cfg, double ms[4]);

/* Algorithm 1 (Sec. IV-B) on the model's predictions alone: among the (L, M)
 * with L in 0..4, M in 0..6 that the dims admit (a valid plan padding the
 * volume by at most 1/8), those whose predicted total time is at most
 * budget_ms; of them the one with the most global levels M, then the fewest
 * block levels L.  *out = *in with block, L, M set (nested = 0); cands
 * (optional, cap entries) receives every candidate with its predicted time in
 * ms (ratio 0, not measured).  Host only.  BM_ERANGE when none fits (*out
 * then holds the fastest predicted candidate); BM_EINVAL (budget not positive
 * and finite, no admissible candidate). */
bm_status bm_select_levels(const bm_config* in, const bm_model* model, double budget_ms, bm_config* out,
                           bm_candidate* cands, int cap, int* ncands);

/* ---- the paper's own block form (Sec. IV-A, IV-C) ------------------------ */

/* Disjoint 8^3 blocks, each decomposed as one MGARD level (Sec. II-B) with
 * natural ends on its own 8 nodes per axis (coarse nodes 0 2 4 6 7); the
 * 5^3 coarse outputs of a level's blocks, side by side in block order and
 * zero-filled to a multiple of 8, form the next level's grid (Sec. IV-C's
 * re-assembly); L block levels, no global levels.  The input (logical dims,
 * C order, dtype) is read with zero fill up to a multiple of 8 (Sec. IV-D).
 * Coefficients, one flat device array of dtype (bm_p8_coeff_size values):
 * the level arrays s = 1..L (dims n_s, multiples of 8, C order: the details
 * at the fine nodes, 0 at each block's 125 coarse nodes) one after the
 * other, then the coarsest values (dims 5 n_L / 8).  The plan owns the
 * assembled grids between levels: calls on one plan must not overlap.
 * Stream-ordered and asynchronous.  Errors: BM_EINVAL (dims outside
 * [1, 2^31] or a level-1 grid of more than 2^40 nodes, dtype, L outside
 * [1, 8], null), BM_ENOMEM, BM_EHIP. */
typedef struct bm_p8_s* bm_p8;
bm_status bm_p8_create(const int64_t dims[3], int dtype, int L, bm_p8* out);

/* The paper's hybrid with this block form (Sec. IV-B, IV-C; the L = 1,
 * M = 2 default of Sec. V-D): the L block levels, then M global levels
 * (Sec. II-B, natural ends, node index as coordinate) on their assembled
 * coarsest values (dims 5 n_L / 8), extended by clamp per axis to the
 * smallest length on which the M levels halve an odd length.  Coefficients:
 * the level arrays as above, then the global levels' in-place array of that
 * extended grid (bm_p8_coeff_size counts it).  Quantization: the shares of
 * the L block levels, the M global levels (their details split equally) and
 * the coarsest values, proportional to counts, floored at 1/(64 (L+M+1));
 * block details as above, every global coefficient at tau_global (the
 * smallest last-level block tau, Sec. IV-C) with the natural level's gain.
 * Every other bm_p8_* call takes such a plan; M = 0 is bm_p8_create.
 * Errors as bm_p8_create; M outside [0, 16], or a global axis the line
 * solver does not take: BM_EINVAL / BM_EUNSUPPORTED. */
bm_status bm_p8_create_hybrid(const int64_t dims[3], int dtype, int L, int M, bm_p8* out);
bm_status bm_p8_destroy(bm_p8 plan);
bm_status bm_p8_coeff_size(bm_p8 plan, int64_t* elems);
bm_status bm_p8_decompose(bm_p8 plan, const void* x_dev, void* coeff_dev, hipStream_t stream);
bm_status bm_p8_recompose(bm_p8 plan, const void* coeff_dev, void* x_dev, hipStream_t stream);

/* ROI bounds of this form (Sec. IV-C, Fig. 6).  Level-1 block map (blocks
 * per axis = bm_p8_block_grid, C order, FP64, device): the smallest voxel
 * tolerance over a block's real nodes (voxel_tol: logical dims, FP64,
 * absolute L-inf bounds, device).  Eq. 2 on the assembled grids: block I
 * of level s+1 takes the smallest tau of the level-s blocks whose 5^3
 * outputs land in it.  A level's details get Delta = 2 tau (1-eta) w_s / A
 * (A the rounded-up L-inf gain of the natural 8-node level, w_s the
 * level's share, proportional to its count), the coarsest values
 * 2 tau (1-eta) w_c with tau of the block they came from; codes
 * q = rint(c * (1/Delta)) in FP64, int32, one per coefficient (the zero
 * placeholders get 0).  bm_p8_quantize synchronizes the stream and returns
 * BM_ERANGE if a code does not fit in 32 bits; the other calls are
 * asynchronous.  eta in [0, 0.5) (else BM_EINVAL). */
bm_status bm_p8_block_grid(bm_p8 plan, int64_t nb[3]);
bm_status bm_p8_tolmap_from_voxels(bm_p8 plan, const double* voxel_tol_dev, double* block_tol_dev,
                                   hipStream_t stream);
bm_status bm_p8_quantize(bm_p8 plan, const void* coeff_dev, const double* block_tol_dev, double eta,
                         int32_t* codes_dev, hipStream_t stream);
bm_status bm_p8_dequantize(bm_p8 plan, const int32_t* codes_dev, const double* block_tol_dev, double eta,
                           void* coeff_dev, hipStream_t stream);

/* The fused pipeline of this form (Sec. IV-D): the block kernels write the
 * codes of each level's details and, at the last level, of the coarsest
 * values, straight from the block in registers; the recomposition
 * dequantizes on load.  Equal, bit for bit, to bm_p8_quantize after
 * bm_p8_decompose and to bm_p8_recompose after bm_p8_dequantize.
 * bm_p8_decompose_quantize synchronizes (BM_ERANGE as bm_p8_quantize);
 * bm_p8_dequantize_recompose is asynchronous. */
bm_status bm_p8_decompose_quantize(bm_p8 plan, const void* x_dev, const double* block_tol_dev, double eta,
                                   int32_t* codes_dev, hipStream_t stream);
bm_status bm_p8_dequantize_recompose(bm_p8 plan, const int32_t* codes_dev, const double* block_tol_dev, double eta,
                                     void* x_dev, hipStream_t stream);

/* Container of this form (host buffer, the layout of bm_compress): the
 * header with flags bit 1 set (block = 8, M = the plan's global levels,
 * pad_mode = 1), the level-1
 * block map, then the Huffman stream of the fused codes; raw data when a
 * code does not fit in 32 bits or coding does not pay.  Capacity and size
 * query as bm_compress; bm_decompress and bm_compressed_config read it.
 * Synchronous. */
bm_status bm_p8_compress(bm_p8 plan, const void* x_dev, const double* block_tol_dev, double eta, void* out_host,
                         size_t out_capacity, size_t* out_bytes, hipStream_t stream);

/* ---- diagnostics ---------------------------------------------------------- */

/* Per-level timing.  bm_timing(plan, 1) resets the counters and makes every
 * later call on the plan record HIP events on its stream around each level
 * (and around quantize / dequantize); bm_timing(plan, 0) stops recording.
 * bm_timing_get waits for the recorded events and returns, for slot k,
 * total milliseconds ms[k] and number of timed calls calls[k], k < cap:
 *   slot 2(s-1)   decomposition level s (s = 1..L+M; one kernel for a block level)
 *   slot 2(s-1)+1 recomposition level s
 *   slot 2(L+M)   quantize, slot 2(L+M)+1 dequantize.
 * *n receives the number of slots, 2(L+M)+2.  Synchronous. */
bm_status bm_timing(bm_plan plan, int enable);
bm_status bm_timing_get(bm_plan plan, double* ms, int64_t* calls, int cap, int* n);

const char* bm_status_string(bm_status s);
const char* bm_last_error(void);     /* thread-local; "" when no error */
const char* bm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BLOCKMGARD_H */
