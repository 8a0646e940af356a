"""The nested block schedule on the GPU against the oracle's nested mode,
through the C ABI: block level s uses (b-1)/2^(s-1)+1-node blocks over the
level-1 block regions (17 -> 9, 33 -> 17 -> 9).

Same bars as the plain schedule: coefficients within 1e-6 * max|x| (FP32)
and 1e-13 (FP64) of the oracle; codes bit-exact given equal coefficients;
every ROI bound held end to end; transposes by the dot-product identity.
"""
import numpy as np
import pytest
import torch

from oracle import mgard, roi
from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-6, torch.float64: 1e-13}

CASES = [((33, 33, 33), 17, 2, 1, torch.float32),
         ((33, 33, 33), 17, 2, 1, torch.float64),
         ((65, 33, 49), 17, 2, 0, torch.float32),      # block levels only
         ((40, 50, 61), 17, 2, 2, torch.float32),      # ragged
         ((1, 40, 70), 17, 2, 1, torch.float64),       # a 2D field
         ((70, 40, 100), 33, 2, 1, torch.float64),     # 33 -> 17
         ((65, 65, 65), 33, 3, 1, torch.float32),      # 33 -> 17 -> 9
         ((97, 65, 33), 33, 3, 0, torch.float32)]


def _ids(c):
    return "x".join(map(str, c[0])) + f"-b{c[1]}-L{c[2]}M{c[3]}-{str(c[4])[6:]}"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()


def _plan(shape, b, L, M, dt):
    from paper_2609_00205_amd import Plan
    return Plan(shape, dtype=dt, block=b, L=L, M=M, nested=True)


def _np(dt):
    return np.float32 if dt == torch.float32 else np.float64


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_nested_transform_parity(case):
    shape, b, L, M, dt = case
    print("case", _ids(case), flush=True)
    p = _plan(shape, b, L, M, dt)
    h = mgard.hierarchy(shape, b, L, M, nested=True)
    assert p.coeff_shape == h.shape_p
    x = synth.gaussian_random_field(shape, 3.0, seed=31, dtype=np.float64).astype(_np(dt))
    c = p.decompose(torch.from_numpy(x).cuda()).cpu().double().numpy()
    ref = mgard.decompose(x.astype(np.float64), b, L, M, nested=True)
    err = np.abs(c - ref).max() / np.abs(x).max()
    print("max rel coefficient error", err)
    assert err <= TOL[dt]
    # recompose of the oracle's coefficients (plus noise)
    rng = np.random.default_rng(2)
    co = (ref + 0.01 * rng.standard_normal(h.shape_p)).astype(_np(dt))
    out = p.recompose(torch.from_numpy(co).cuda()).cpu().double().numpy()
    rr = mgard.recompose(co.astype(np.float64), shape, b, L, M, nested=True)
    err = np.abs(out - rr).max() / np.abs(rr).max()
    print("max rel recompose error", err)
    assert err <= TOL[dt]
    xr = p.recompose(p.decompose(torch.from_numpy(x).cuda())).cpu().double().numpy()
    assert np.abs(xr - x).max() / np.abs(x).max() <= (2e-6 if dt == torch.float32 else 1e-13)


def _boxes(shape, scale):
    rng = np.random.default_rng(9)
    out = []
    for k in range(2):
        e = [min(s, max(2, s // 5)) for s in shape]
        o = [int(rng.integers(0, s - ee + 1)) for s, ee in zip(shape, e)]
        out.append((o[0], o[1], o[2], o[0] + e[0], o[1] + e[1], o[2] + e[2], scale * 10.0 ** (-3 - k)))
    return out


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_nested_quantizer(case):
    shape, b, L, M, dt = case
    print("case", _ids(case), flush=True)
    p = _plan(shape, b, L, M, dt)
    h = mgard.hierarchy(shape, b, L, M, nested=True)
    assert p.gains == roi.level_gains(h)
    x = synth.gaussian_random_field(shape, 3.0, seed=32, dtype=np.float64)
    scale = float(np.abs(x).max())
    boxes = _boxes(shape, scale)
    vt = roi.voxel_tolerance_from_boxes(shape, boxes, 1e-2 * scale)
    tol1 = roi.block_tolerance(vt, h.shape_p, b)
    bt = p.tolmap_from_boxes(boxes, 1e-2 * scale)
    assert np.array_equal(bt.cpu().numpy().reshape(tol1.shape), tol1)
    # codes bit-exact given the oracle's coefficients
    coeff = mgard.decompose(x, b, L, M, nested=True).astype(_np(dt))
    delta = roi.node_delta(h, tol1, p.eta)
    ref = roi.quantize(coeff.astype(np.float64), delta)
    codes, _ = p.quantize(torch.from_numpy(coeff).cuda(), bt)
    got = codes.cpu().numpy()
    assert np.array_equal(got, ref), int((got != ref).sum())
    # fused pipeline equals the unfused one, and every bound holds
    xd = torch.from_numpy(x).to(dt).cuda()
    cf = p.decompose_quantize(xd, bt)
    cu, _ = p.quantize(p.decompose(xd), bt)
    assert torch.equal(cf, cu), int((cf != cu).sum())
    xr = p.dequantize_recompose(cf, bt)
    assert torch.equal(xr, p.recompose(p.dequantize(cu, bt)))
    err = np.abs(xr.cpu().double().numpy() - xd.cpu().double().numpy())
    print("worst error / bound", float((err / vt).max()))
    assert np.all(err <= vt)


@pytest.mark.parametrize("case", CASES[:3] + CASES[5:7], ids=_ids)
def test_nested_transposes(case):
    shape, b, L, M, dt = case
    dt = torch.float64
    p = _plan(shape, b, L, M, dt)
    h = mgard.hierarchy(shape, b, L, M, nested=True)
    rng = np.random.default_rng(4)
    x = torch.from_numpy(rng.standard_normal(shape)).cuda()
    g = torch.from_numpy(rng.standard_normal(h.shape_p)).cuda()
    lhs = float((p.decompose(x) * g).sum())
    rhs = float((x * p.decompose_adjoint(g)).sum())
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs) + 1e-9
    y = torch.from_numpy(rng.standard_normal(shape)).cuda()
    lhs = float((p.recompose(g) * y).sum())
    rhs = float((g * p.recompose_adjoint(y)).sum())
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs) + 1e-9
    # against the oracle's transpose
    gx = p.decompose_adjoint(g).cpu().numpy()
    ref = mgard.decompose_adjoint(g.cpu().numpy(), shape, b, L, M, nested=True)
    assert np.abs(gx - ref).max() <= 1e-12 * np.abs(ref).max()


def test_nested_container_round_trip():
    from paper_2609_00205_amd import api
    shape, b, L, M = (65, 65, 65), 17, 2, 1
    p = _plan(shape, b, L, M, torch.float32)
    x = synth.gaussian_random_field(shape, 3.0, seed=33, dtype=np.float32)
    scale = float(np.abs(x).max())
    boxes = _boxes(shape, scale)
    bt = p.tolmap_from_boxes(boxes, 1e-2 * scale)
    buf = p.compress(torch.from_numpy(x).cuda(), bt)
    info = api.compressed_config(buf)
    assert info["nested"] and info["L"] == 2
    xr = api.decompress(buf).cpu().double().numpy()
    vt = roi.voxel_tolerance_from_boxes(shape, boxes, 1e-2 * scale)
    assert np.all(np.abs(xr - x.astype(np.float64)) <= vt)


def test_batch_schedule_rules():
    # batches take the nested schedule with b = 17 (its pairs run in one
    # persistent launch); every field shares the schedule; b = 9 nested is refused
    from paper_2609_00205_amd import _lib
    from paper_2609_00205_amd._lib import BMConfig
    import ctypes as C
    lib = _lib.lib()
    h = C.c_void_p()
    ok = (BMConfig * 2)(BMConfig(3, (C.c_int64 * 3)(33, 33, 33), 0, 17, 2, 1, 0, 0.1, 1),
                        BMConfig(3, (C.c_int64 * 3)(65, 33, 17), 0, 17, -1, 0, 0, 0.1, 1))
    assert lib.bm_batch_create(2, ok, C.byref(h)) == 0
    p = C.c_void_p()
    cfg = BMConfig()
    assert lib.bm_batch_plan(h, 1, C.byref(p)) == 0 and lib.bm_plan_config(p, C.byref(cfg)) == 0
    assert cfg.nested == 1 and cfg.L == 2                      # L = -1: both levels of the pair
    assert lib.bm_batch_destroy(h) == 0
    mixed = (BMConfig * 2)(BMConfig(3, (C.c_int64 * 3)(33, 33, 33), 0, 17, 2, 0, 0, 0.1, 1),
                           BMConfig(3, (C.c_int64 * 3)(33, 33, 33), 0, 17, 2, 0, 0, 0.1, 0))
    assert lib.bm_batch_create(2, mixed, C.byref(h)) == -1
    b9 = (BMConfig * 1)(BMConfig(3, (C.c_int64 * 3)(33, 33, 33), 0, 9, 1, 0, 0, 0.1, 1))
    assert lib.bm_batch_create(1, b9, C.byref(h)) == -8
