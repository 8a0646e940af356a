"""ctypes view of libblockmgard.so (the C ABI declared in include/blockmgard.h).

Argument marshalling only.  If the library has not been built this module
raises on first use: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libblockmgard.so")

BM_F32, BM_F64 = 0, 1
STATUS = {0: "BM_OK", -1: "BM_EINVAL", -2: "BM_ENOMEM", -3: "BM_EHIP", -4: "BM_ENONFINITE",
          -5: "BM_ECAPACITY", -6: "BM_ECORRUPT", -7: "BM_ERANGE", -8: "BM_EUNSUPPORTED"}
BM_ECAPACITY = -5
BM_ERANGE = -7


class BMConfig(C.Structure):
    _fields_ = [("ndim", C.c_int), ("dims", C.c_int64 * 3), ("dtype", C.c_int), ("block", C.c_int),
                ("L", C.c_int), ("M", C.c_int), ("pad_mode", C.c_int), ("eta", C.c_double), ("nested", C.c_int)]


class BMQStats(C.Structure):
    _fields_ = [("n_codes", C.c_int64), ("n_outliers", C.c_int64), ("max_abs_code", C.c_int64)]


class BMCandidate(C.Structure):
    _fields_ = [("block", C.c_int), ("L", C.c_int), ("M", C.c_int), ("status", C.c_int), ("ms", C.c_double),
                ("ratio", C.c_double), ("nested", C.c_int), ("lossless_ms", C.c_double)]


class BMModel(C.Structure):
    _fields_ = [("dtype", C.c_int), ("block", C.c_int), ("blk_lat_ms", C.c_double), ("blk_tp", C.c_double),
                ("fblk_lat_ms", C.c_double), ("fblk_tp", C.c_double), ("fglob_a_ms", C.c_double),
                ("fglob_b_ms", C.c_double), ("glob_a_ms", C.c_double), ("glob_b_ms", C.c_double),
                ("q_slope_ms", C.c_double), ("q_lat_ms", C.c_double), ("huf_a_ms", C.c_double * 4),
                ("huf_b_ms", C.c_double * 4), ("gq_slope_ms", C.c_double), ("gq_lat_ms", C.c_double)]


class BMLosslessTimes(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("enc_hist_ms", "enc_table_ms", "enc_sizes_ms", "enc_encode_ms",
                                          "enc_copy_ms", "enc_crc_ms", "dec_parse_ms", "dec_upload_ms",
                                          "dec_decode_ms")] + [("enc_n", C.c_int64), ("dec_n", C.c_int64)]


class BMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


_lib = None

P = C.c_void_p
_SIGS = {
    "bm_plan_create": [C.POINTER(BMConfig), C.POINTER(P)],
    "bm_plan_destroy": [P],
    "bm_coeff_shape": [P, C.POINTER(C.c_int64)],
    "bm_workspace_size": [P, C.POINTER(C.c_size_t)],
    "bm_model_calibrate": [C.c_int, C.c_int, C.POINTER(BMModel), P],
    "bm_model_predict": [C.POINTER(BMModel), C.POINTER(BMConfig), C.POINTER(C.c_double)],
    "bm_select_levels": [C.POINTER(BMConfig), C.POINTER(BMModel), C.c_double, C.POINTER(BMConfig),
                         C.POINTER(BMCandidate), C.c_int, C.POINTER(C.c_int)],
    "bm_plan_config": [P, C.POINTER(BMConfig)],
    "bm_block_grid": [P, C.POINTER(C.c_int64)],
    "bm_level_gains": [P, C.POINTER(C.c_double)],
    "bm_decompose": [P, P, P, P],
    "bm_recompose": [P, P, P, P],
    "bm_decompose_adjoint": [P, P, P, P],
    "bm_recompose_adjoint": [P, P, P, P],
    "bm_tolmap_from_boxes": [P, C.POINTER(C.c_double), C.c_int, C.c_double, P, P],
    "bm_tolmap_from_voxels": [P, P, P, P],
    "bm_quantize_roi": [P, P, P, P, C.POINTER(BMQStats), P],
    "bm_dequantize": [P, P, P, P, P],
    "bm_huffman_encode": [P, C.c_int64, P, C.c_size_t, C.POINTER(C.c_size_t), P],
    "bm_huffman_decode": [P, C.c_size_t, P, C.c_int64, P],
    "bm_lossless_last_times": [C.POINTER(BMLosslessTimes)],
    "bm_quant_prepare": [P, P, P],
    "bm_p8_create_hybrid": [C.POINTER(C.c_int64), C.c_int, C.c_int, C.c_int, C.POINTER(P)],
    "bm_huffman_plan": [P, C.c_int64, C.POINTER(P), C.POINTER(C.c_size_t), P],
    "bm_huffman_write": [P, P, C.c_size_t, C.POINTER(C.c_size_t)],
    "bm_huffman_destroy": [P],
    "bm_compress_plan": [P, P, P, C.POINTER(C.c_size_t), P],
    "bm_compress_write": [P, P, C.c_size_t, C.POINTER(C.c_size_t)],
    "bm_huffman_code_lengths": [P, P],
    "bm_huffman_encode_device": [P, C.c_int64, P, C.c_size_t, C.POINTER(C.c_size_t), P],
    "bm_compress": [P, P, P, P, C.c_size_t, C.POINTER(C.c_size_t), P],
    "bm_compressed_config": [P, C.c_size_t, C.POINTER(BMConfig)],
    "bm_decompress": [P, C.c_size_t, P, P],
    "bm_decompose_quantize": [P, P, P, P, C.POINTER(BMQStats), P],
    "bm_dequantize_recompose": [P, P, P, P, P],
    "bm_qoi_deltas": [P, P, C.c_double, P, P, C.POINTER(C.c_int64), P],
    "bm_quantize_delta": [P, P, P, P, C.POINTER(BMQStats), P],
    "bm_dequantize_delta": [P, P, P, P, P],
    "bm_autotune": [C.POINTER(BMConfig), P, P, C.c_double, C.c_int, C.POINTER(BMConfig), C.POINTER(BMCandidate),
                    C.c_int, C.POINTER(C.c_int), P],
    "bm_autotune_budget": [C.POINTER(BMConfig), P, P, C.c_double, C.c_int, C.POINTER(BMConfig),
                           C.POINTER(BMCandidate), C.c_int, C.POINTER(C.c_int), P],
    "bm_batch_create": [C.c_int, C.POINTER(BMConfig), C.POINTER(P)],
    "bm_batch_destroy": [P],
    "bm_batch_plan": [P, C.c_int, C.POINTER(P)],
    "bm_batch_decompose_quantize": [P, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.c_int, C.POINTER(C.c_int), P],
    "bm_batch_dequantize_recompose": [P, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.c_int, P],
    "bm_batch_compress": [P, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(C.c_size_t),
                          C.POINTER(C.c_size_t), C.c_int, P],
    "bm_p8_create": [C.POINTER(C.c_int64), C.c_int, C.c_int, C.POINTER(P)],
    "bm_p8_destroy": [P],
    "bm_p8_coeff_size": [P, C.POINTER(C.c_int64)],
    "bm_p8_decompose": [P, P, P, P],
    "bm_p8_recompose": [P, P, P, P],
    "bm_p8_block_grid": [P, C.POINTER(C.c_int64)],
    "bm_p8_tolmap_from_voxels": [P, P, P, P],
    "bm_p8_quantize": [P, P, P, C.c_double, P, P],
    "bm_p8_dequantize": [P, P, P, C.c_double, P, P],
    "bm_p8_decompose_quantize": [P, P, P, C.c_double, P, P],
    "bm_p8_dequantize_recompose": [P, P, P, C.c_double, P, P],
    "bm_p8_compress": [P, P, P, C.c_double, P, C.c_size_t, C.POINTER(C.c_size_t), P],
    "bm_timing": [P, C.c_int],
    "bm_timing_get": [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int, C.POINTER(C.c_int)],
}


def lib():
    """Load the library (once)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_00205_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = C.c_int
        h.bm_status_string.argtypes = [C.c_int]
        h.bm_status_string.restype = C.c_char_p
        h.bm_last_error.argtypes = []
        h.bm_last_error.restype = C.c_char_p
        h.bm_version.argtypes = []
        h.bm_version.restype = C.c_char_p
        _lib = h
    return _lib


def check(status: int) -> None:
    if status != 0:
        raise BMError(status, lib().bm_last_error().decode())


def call(name: str, *args) -> None:
    check(getattr(lib(), name)(*args))
