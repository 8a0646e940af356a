"""The plain method end to end on the small workload: a 65^3 FP32 field of
Gaussian bumps, sine modes and N(0, 1e-3) noise, full global MGARD
decomposition (L = 0, M = 6: 65 -> 33 -> ... -> 2 nodes per axis), uniform
REL 1e-3 bound, Huffman stage, through the C ABI.

The oracle checks the whole pipeline here: coefficients element by element,
codes bit-exact except across a bin edge (the count is printed), the
container's Huffman stream bit-exact against the oracle's coder run on the
GPU's codes, the L-inf bound of the decompressed field, and the ratio.
"""
import struct

import numpy as np
import pytest
import torch

from oracle import huffman as ohf
from oracle import mgard, roi
from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu

SHAPE, B, L, M, REL = (65, 65, 65), 17, 0, 6, 1e-3
HDR = 96   # container header bytes


@pytest.fixture(scope="module")
def c1():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import Plan
    x = synth.workload_small(seed=1)
    assert x.shape == SHAPE and x.dtype == np.float32
    p = Plan(SHAPE, dtype=torch.float32, block=B, L=L, M=M)
    tol = REL * float(np.abs(x).max())
    xd = torch.from_numpy(x).cuda()
    bt = p.tolmap_from_boxes([], tol)
    return x, p, xd, bt, tol


def test_c1_coefficients(c1):
    x, p, xd, bt, tol = c1
    c = p.decompose(xd).cpu().double().numpy()
    ref = mgard.decompose(x.astype(np.float64), B, L, M)
    err = float(np.abs(c - ref).max() / np.abs(x).max())
    print("max rel coefficient error", err)
    assert err <= 1e-6


def test_c1_codes(c1):
    x, p, xd, bt, tol = c1
    h = mgard.hierarchy(SHAPE, B, L, M)
    delta = roi.node_delta(h, tol, p.eta)
    cg = p.decompose(xd)
    co = mgard.decompose(x.astype(np.float64), B, L, M)
    ref = roi.quantize(co, delta)
    fused = p.decompose_quantize(xd, bt).cpu().numpy().astype(np.int64)
    unfused = p.quantize(cg, bt)[0].cpu().numpy().astype(np.int64)
    assert np.array_equal(fused, unfused)
    # given the GPU's own coefficients the codes are bit-exact
    assert np.array_equal(unfused, roi.quantize(cg.cpu().double().numpy(), delta))
    # from the oracle's coefficients they differ only where a bin edge lies between the two
    flips = fused != ref
    print("codes across a bin edge:", int(flips.sum()), "of", fused.size)
    moved = np.abs(cg.cpu().double().numpy() - co) / delta
    r = co * (1.0 / delta)
    edge = np.abs(r - np.floor(r) - 0.5)
    assert np.all(np.abs(fused - ref)[flips] <= 1)
    assert np.all(edge[flips] <= moved[flips] + 1e-9)


def test_c1_container_stream_and_bound(c1):
    from paper_2609_00205_amd import api
    x, p, xd, bt, tol = c1
    codes = p.decompose_quantize(xd, bt).cpu().numpy()
    buf = bytes(p.compress(xd, bt))
    flags, ntol = struct.unpack_from("<I", buf, 8)[0], struct.unpack_from("<q", buf, 72)[0]
    assert flags == 0 and ntol == 1
    assert struct.unpack_from("<d", buf, HDR)[0] == tol
    got = api.parse_huffman(buf[HDR + 8 * ntol:])
    sym, oi, ov = ohf.to_symbols(codes.ravel().astype(np.int64))
    ln = ohf.code_lengths(ohf.histogram(sym))
    words, offs = ohf.encode(sym, ln)
    assert got["n"] == codes.size
    assert np.array_equal(got["lengths"], ln.astype(np.uint8))
    assert np.array_equal(got["offsets"].astype(np.int64), offs)
    assert np.array_equal(got["words"], words)
    assert np.array_equal(got["outlier_value"].astype(np.int64), ov)
    xr = api.decompress(buf).cpu().double().numpy()
    err = float(np.abs(xr - x.astype(np.float64)).max())
    ratio = x.nbytes / len(buf)
    print(f"C1: ratio {ratio:.2f}, max error / bound {err / tol:.3f}")
    assert err <= tol
    assert ratio > 1.0
