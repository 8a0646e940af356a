"""GPU decompose / recompose parity with the FP64 oracle, through the C ABI.

Bar: coefficients within 1e-6 * max|x| (FP32) and 1e-13 * max|x| (FP64) of
the oracle on the same seeded input; recomposition of the same coefficient
array within the same bound; round trips back to the input.
"""
import numpy as np
import pytest
import torch

from oracle import mgard
from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-6, torch.float64: 1e-13}

# (shape, b, L, M, dtype, pad_mode)
CASES = [
    ((33, 33, 33), 17, 1, 2, torch.float32, "clamp"),
    ((33, 33, 33), 17, 1, 2, torch.float64, "clamp"),
    ((65, 65, 65), 17, 1, 2, torch.float32, "clamp"),
    ((20, 30, 12), 9, 1, 1, torch.float32, "clamp"),     # ragged: padded to 25 x 33 x 17
    ((20, 30, 12), 9, 1, 1, torch.float64, "zero"),
    ((33, 17, 65), 9, 2, 1, torch.float64, "clamp"),      # two block levels
    ((65, 65, 65), 17, 0, 6, torch.float32, "clamp"),     # pure global down to 2 nodes per axis
    ((9, 5, 33), 9, 0, 4, torch.float64, "clamp"),        # an axis stops coarsening at 2 nodes
    ((65, 33, 49), 17, 1, 0, torch.float32, "clamp"),     # pure local
    ((97, 65, 129), 17, 1, 2, torch.float32, "clamp"),    # 6 x 4 x 8 blocks, global lines of 65
    ((40, 50, 61), 9, 2, 2, torch.float32, "clamp"),      # ragged everywhere
    ((65, 65, 65), 33, 1, 2, torch.float32, "clamp"),     # 33^3 blocks
    ((70, 40, 100), 33, 1, 1, torch.float64, "zero"),     # 33^3 blocks, ragged: padded to 97 x 65 x 129
    ((70, 40, 100), 33, 1, 1, torch.float32, "clamp"),
    ((65, 65, 129), 33, 2, 1, torch.float64, "clamp"),    # two 33^3 block levels
    ((65, 33, 65), 33, 1, 0, torch.float32, "clamp"),     # 33^3 blocks, pure local
    ((129, 97, 97), 17, 0, 2, torch.float32, "clamp"),    # x and y passes fused per z-plane (both levels)
    ((129, 129, 129), 17, 1, 2, torch.float32, "clamp"),  # the same after a block level
    ((1, 40, 70), 9, 1, 1, torch.float32, "clamp"),       # a 2D field: unit z axis padded to one block
    ((1, 40, 70), 9, 1, 1, torch.float64, "zero"),
    ((1, 1, 200), 17, 1, 2, torch.float32, "clamp"),      # a 1D field
    ((3, 3, 3), 9, 0, 1, torch.float64, "clamp"),         # smallest grid that has a level
    ((5, 2, 9), 9, 0, 2, torch.float32, "clamp"),         # an axis of 2 nodes never coarsens
    ((17, 17, 17), 17, 1, 0, torch.float32, "clamp"),     # a single block
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"-b{c[1]}-L{c[2]}M{c[3]}-{str(c[4])[6:]}-{c[5]}"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()   # fails loudly when the library is missing


def _plan(shape, b, L, M, dt, pad):
    from paper_2609_00205_amd import Plan
    return Plan(shape, dtype=dt, block=b, L=L, M=M, pad_mode=pad)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_decompose_parity(case):
    shape, b, L, M, dt, pad = case
    print("case", _ids(case), flush=True)
    x = synth.gaussian_random_field(shape, 3.0, seed=11, dtype=np.float64).astype(
        np.float32 if dt == torch.float32 else np.float64)
    p = _plan(shape, b, L, M, dt, pad)
    xd = torch.from_numpy(x).cuda()
    c = p.decompose(xd).cpu().double().numpy()
    ref = mgard.decompose(x.astype(np.float64), b, L, M, pad_mode=pad)
    assert c.shape == ref.shape
    scale = np.abs(x).max()
    err = np.abs(c - ref).max() / scale
    print("max rel coefficient error", err)
    assert err <= TOL[dt]


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_recompose_parity(case):
    shape, b, L, M, dt, pad = case
    print("case", _ids(case), flush=True)
    rng = np.random.default_rng(5)
    h = mgard.hierarchy(shape, b, L, M)
    # realistic coefficients (the oracle's decomposition of a smooth field) plus noise
    x = synth.gaussian_random_field(shape, 3.0, seed=12, dtype=np.float64)
    coeff = mgard.decompose(x, b, L, M, pad_mode=pad) + 0.01 * rng.standard_normal(h.shape_p)
    coeff = coeff.astype(np.float32 if dt == torch.float32 else np.float64)
    p = _plan(shape, b, L, M, dt, pad)
    out = p.recompose(torch.from_numpy(coeff).cuda()).cpu().double().numpy()
    ref = mgard.recompose(coeff.astype(np.float64), shape, b, L, M)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print("max rel recompose error", err)
    assert err <= TOL[dt]


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_roundtrip(case):
    shape, b, L, M, dt, pad = case
    x = torch.from_numpy(synth.gaussian_random_field(shape, 3.0, seed=13, dtype=np.float64)).to(dt).cuda()
    p = _plan(shape, b, L, M, dt, pad)
    y = p.recompose(p.decompose(x))
    err = (y - x).abs().max().item() / x.abs().max().item()
    assert err <= (2e-6 if dt == torch.float32 else 1e-13)


def test_multilinear_field_has_zero_details():
    from paper_2609_00205_amd import Plan
    shape = (33, 33, 65)
    z, y, x = np.meshgrid(*(np.arange(float(s)) for s in shape), indexing="ij")
    f = (1.5 + 0.02 * x + 0.03 * y - 0.01 * z + 0.001 * x * y * z / 100).astype(np.float64)
    p = Plan(shape, dtype=torch.float64, block=17, L=1, M=2)
    c = p.decompose(torch.from_numpy(f).cuda()).cpu().numpy()
    lev = mgard.node_level(c.shape, 1, 2)
    assert np.abs(c[lev <= 3]).max() < 1e-13 * np.abs(f).max()


def test_repeated_calls_and_streams():
    from paper_2609_00205_amd import Plan
    shape = (65, 65, 65)
    p = Plan(shape, dtype=torch.float32, block=17, L=1, M=2)
    x = torch.from_numpy(synth.gaussian_random_field(shape, 3.0, seed=14)).cuda()
    c0 = p.decompose(x).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())   # calls on one plan must not overlap
    with torch.cuda.stream(s):
        c1 = p.decompose(x)
    s.synchronize()
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        c2 = p.decompose(x)
    torch.cuda.synchronize()
    assert torch.equal(c0, c1) and torch.equal(c0, c2)
