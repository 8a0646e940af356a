"""Boundary checks that need no GPU: the library loads, exports every entry
point the header declares, and rejects bad arguments with status codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blockmgard.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:bm_status|const char\*)\s+(bm_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2609_00205_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2609_00205_amd import build
        build.build()
    return _lib.lib()


def test_header_declares_the_api():
    names = _declared()
    for n in ["bm_plan_create", "bm_decompose", "bm_recompose", "bm_quantize_roi", "bm_dequantize",
              "bm_compress", "bm_decompress", "bm_huffman_encode", "bm_huffman_decode",
              "bm_decompose_adjoint", "bm_recompose_adjoint", "bm_tolmap_from_boxes", "bm_tolmap_from_voxels"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_status_strings(lib):
    assert lib.bm_status_string(0) == b"ok"
    assert lib.bm_status_string(-6) == b"corrupt stream"
    assert lib.bm_version().startswith(b"blockmgard")


def test_bad_config_rejected_before_touching_a_device(lib):
    from paper_2609_00205_amd._lib import BMConfig
    h = C.c_void_p()
    for cfg in [BMConfig(3, (C.c_int64 * 3)(0, 5, 5), 0, 17, 1, 2, 0, 0.1),      # empty axis
                BMConfig(3, (C.c_int64 * 3)(9, 9, 9), 7, 17, 1, 2, 0, 0.1),      # bad dtype
                BMConfig(3, (C.c_int64 * 3)(9, 9, 9), 0, 12, 1, 2, 0, 0.1),      # block not 2^k+1
                BMConfig(3, (C.c_int64 * 3)(9, 9, 9), 0, 17, 0, 0, 0, 0.1),      # no levels
                BMConfig(3, (C.c_int64 * 3)(9, 9, 9), 0, 17, 1, 2, 0, 0.7),      # eta out of range
                BMConfig(3, (C.c_int64 * 3)(40, 40, 40), 0, 17, 3, 1, 0, 0.1, 1),  # nested: level 3 of 5 nodes
                BMConfig(3, (C.c_int64 * 3)(40, 40, 40), 0, 17, 1, 1, 0, 0.1, 2),   # nested must be 0 or 1
                BMConfig(3, (C.c_int64 * 3)(1 << 31, 1 << 31, 1 << 31), 0, 17, 1, 2, 0, 0.1),   # > 2^40 nodes
                BMConfig(3, (C.c_int64 * 3)(1 << 14, 1 << 14, 1 << 13), 0, 17, 1, 2, 0, 0.1)]:  # 2^41 nodes
        assert lib.bm_plan_create(C.byref(cfg), C.byref(h)) == -1
        assert len(lib.bm_last_error()) > 0
    assert lib.bm_plan_create(None, C.byref(h)) == -1


def test_bad_paper8_config_rejected_before_touching_a_device(lib):
    h = C.c_void_p()
    for dims, dt, L in [((0, 8, 8), 0, 1), ((8, 8, 8), 3, 1), ((8, 8, 8), 0, 0), ((8, 8, 8), 0, 9),
                        ((1 << 31, 1 << 31, 1 << 31), 0, 1), ((1 << 14, 1 << 14, 1 << 13), 0, 1)]:
        assert lib.bm_p8_create((C.c_int64 * 3)(*dims), dt, L, C.byref(h)) == -1, dims
        assert len(lib.bm_last_error()) > 0


def test_corrupt_container_rejected(lib):
    from paper_2609_00205_amd._lib import BMConfig
    cfg = BMConfig()
    assert lib.bm_compressed_config(b"not a stream at all" * 10, 190, C.byref(cfg)) == -6
    assert lib.bm_compressed_config(None, 0, C.byref(cfg)) == -6


def test_null_plan_calls(lib):
    assert lib.bm_decompose(None, None, None, None) == -1
    assert lib.bm_quantize_roi(None, None, None, None, None, None) == -1
    assert lib.bm_plan_destroy(None) == 0
    n = C.c_size_t(7)
    assert lib.bm_workspace_size(None, C.byref(n)) == -1 and n.value == 7
    assert lib.bm_compress_write(None, None, 0, C.byref(n)) == -1
    assert lib.bm_huffman_write(None, None, 0, C.byref(n)) == -1


def test_long_global_axis_rejected_at_plan_creation(lib):
    # global-level line solves take at most 576 coarse nodes per line (axes of at most 1151 nodes)
    from paper_2609_00205_amd._lib import BMConfig
    h = C.c_void_p()
    for dims, b, L, M in [((3, 3, 1153), 17, 0, 1),       # first global level on 1153 nodes
                          ((1153, 5, 5), 17, 0, 2),
                          ((17, 17, 2305), 17, 1, 1)]:    # a block level leaves 1153 nodes
        cfg = BMConfig(3, (C.c_int64 * 3)(*dims), 0, b, L, M, 0, 0.1)
        assert lib.bm_plan_create(C.byref(cfg), C.byref(h)) == -8, dims
        assert b"1151" in lib.bm_last_error()


def _container(tol, flags=0, dims=(9, 9, 9), block=9, L=1, M=1, extra=b"\0" * 64):
    # the container layout of bm_compress: header (CRC over the header with
    # its CRC field zeroed, then the payload), the block map, the stream
    import struct
    import zlib
    payload = struct.pack(f"<{len(tol)}d", *tol) + extra

    def hdr(crc):
        return struct.pack("<III7i3qdqQII", 0x44474D42, 1, flags, 0, block, L, M, 0, 3, 0, *dims, 0.1,
                           len(tol), len(payload), crc, 0)
    crc = zlib.crc32(payload, zlib.crc32(hdr(0)))
    return hdr(crc) + payload


@pytest.mark.parametrize("bad", [0.0, -1e-3, float("inf"), float("nan")])
def test_decompress_rejects_a_bad_stored_tolerance(lib, bad):
    buf = _container([1e-3, bad])
    out = C.c_void_p(1)       # never written: the map is checked before anything else
    assert lib.bm_decompress(buf, len(buf), out, None) == -6
    assert b"tolerance" in lib.bm_last_error()


def test_decompress_rejects_a_map_larger_than_the_payload(lib):
    buf = _container([1e-3] * 4, extra=b"")
    import struct
    b = bytearray(buf)
    struct.pack_into("<q", b, 72, 5)            # ntol beyond the payload (CRC recomputed below)
    import zlib
    struct.pack_into("<I", b, 88, 0)
    crc = zlib.crc32(bytes(b[96:]), zlib.crc32(bytes(b[:96])))
    struct.pack_into("<I", b, 88, crc)
    assert lib.bm_decompress(bytes(b), len(b), C.c_void_p(1), None) == -6


def test_batch_checks_list_lengths():
    # the library reads one pointer per field from each array: the binding
    # refuses lists of another length before building any pointer array
    from paper_2609_00205_amd.api import Batch
    b = Batch.__new__(Batch)
    b.plans = [object(), object()]
    with pytest.raises(ValueError):
        b.decompose_quantize([1], [1, 2])
    with pytest.raises(ValueError):
        b.dequantize_recompose([1, 2], [1, 2], outs=[1])
    with pytest.raises(ValueError):
        b.compress([1, 2, 3], [1, 2])


def _hist_cases():
    rng = np.random.default_rng(9)
    out = []
    for kind in ("ties", "pow2", "wide", "equal", "laplace", "two", "one"):
        h = np.zeros(65536, np.uint64)
        np_ = {"two": 2, "one": 1}.get(kind, 3000 if kind != "laplace" else 65536)
        sym = np.sort(rng.choice(65536, np_, replace=False))
        if kind == "ties":
            h[sym] = rng.integers(1, 4, np_)
        elif kind == "pow2":
            h[sym] = np.uint64(1) << rng.integers(0, 40, np_).astype(np.uint64)
        elif kind == "wide":
            h[sym] = rng.integers(1, 10 ** 6, np_)
        elif kind == "equal":
            h[sym] = 7
        elif kind == "laplace":
            h[:] = (1 + 4e6 * np.exp(-np.abs(np.arange(65536) - 32768) / 300.0)).astype(np.uint64)
        else:
            h[sym] = rng.integers(1, 100, np_)
        out.append((kind, h))
    return out


@pytest.mark.parametrize("kind,hist", _hist_cases(), ids=[k for k, _ in _hist_cases()])
def test_code_lengths_match_oracle(lib, kind, hist):
    """The encoder's host codebook step (bm_huffman_code_lengths: two sorted
    queues) equals the oracle's heap-based Huffman construction, ties, the
    32-bit length cap and a dense 65536-symbol table included."""
    from oracle import huffman as ohf
    from paper_2609_00205_amd import api
    got = api.huffman_code_lengths(hist)
    ref = ohf.code_lengths(hist.astype(np.int64))
    assert np.array_equal(got.astype(np.int64), ref)
    if kind == "pow2":
        assert int(ref.max()) == 32      # the cap is reached


def test_host_buffers_of_every_kind_read_alike(lib):
    # the binding reads a container from bytes, bytearray, a numpy array, a
    # 1-D uint8 host tensor or a memoryview cut from a larger buffer, without
    # a copy where the buffer is writable, and counts bytes, not items
    import numpy as np
    import torch

    from paper_2609_00205_amd import api
    buf = _container([1e-3, 2e-3])
    big = bytearray(buf) + b"\xff" * 100
    kinds = [buf, bytearray(buf), np.frombuffer(bytearray(buf), np.uint8), torch.tensor(list(buf), dtype=torch.uint8),
             memoryview(big)[:len(buf)]]
    for k in kinds:
        assert api._nbytes(k) == len(buf)
        info = api.compressed_config(k)
        assert info["shape"] == (9, 9, 9) and info["block"] == 9 and info["L"] == 1 and info["M"] == 1
    assert api._nbytes(np.zeros(4, np.float64)) == 32
    with pytest.raises(ValueError):
        api._host_view(torch.zeros(4, dtype=torch.int32))
