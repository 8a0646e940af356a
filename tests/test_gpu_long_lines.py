"""Global-level line solves on long lines against the FP64 oracle, through
the C ABI: decompose, recompose and both transposes.

The line solver takes a register layout per line length m (coarse nodes per
line): 16-lane groups with 3, 5, 9, 11 or 17 unknowns per lane for m <= 48,
80, 144, 176 or 272, and a whole wavefront for m <= 576.  Short grids reach only the
first two; these cases put the long lines of the full-size workloads on
small grids that the oracle finishes at once:

* L = 0, M = 1 on (3, 3, n), (3, n, 3), (n, 3, 3): one global level whose
  lines along the long axis have m = (n + 1) / 2 = 129, 161, 257, 513 coarse
  nodes (the restriction + solve passes; 161 is the global axis of the 8^3
  form's hybrid at 512^3);
* b = 17, L = 1, M = 1 on (17, 17, n) and its permutations: the first
  global level fused into the block level, whose solve-only passes run on
  the 9 x 9 x (n + 1) / 2 block-coarse grid, lines of (n + 1) / 2 nodes;
* L = 0, M = 2 on (3, 3, 1025): both levels, lines of 513 then 257.

Bar: coefficients within 1e-6 (FP32) and 1e-13 (FP64) of max|x|, as in
``test_gpu_transform.py``; transposes within 2e-6 / 1e-12 of max|ref|.
"""
import numpy as np
import pytest
import torch

from oracle import mgard
from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-6, torch.float64: 1e-13}
TOL_T = {torch.float32: 2e-6, torch.float64: 1e-12}


def _variant(m):
    # the solver's register layout for lines of m coarse nodes (named in the test id)
    return ("Q3" if m <= 48 else "Q5" if m <= 80 else "Q9" if m <= 144 else "Q11" if m <= 176 else "Q17" if m <= 272
            else "Qwave")


def _cases():
    out = []
    for n in (257, 321, 513, 1025):
        m = (n + 1) // 2
        for ax in range(3):
            shape = [3, 3, 3]
            shape[ax] = n
            out.append((tuple(shape), 17, 0, 1, _variant(m)))
            shape17 = [17, 17, 17]
            shape17[ax] = n
            out.append((tuple(shape17), 17, 1, 1, "solve-" + _variant(m)))
    out.append(((3, 3, 1025), 17, 0, 2, "Qwave+Q17"))
    return out


CASES = [c + (dt,) for c in _cases() for dt in (torch.float32, torch.float64)]


def _ids(c):
    return "x".join(map(str, c[0])) + f"-L{c[2]}M{c[3]}-{c[4]}-{str(c[5])[6:]}"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()


def _plan(shape, b, L, M, dt):
    from paper_2609_00205_amd import Plan
    return Plan(shape, dtype=dt, block=b, L=L, M=M)


def _npdt(dt):
    return np.float32 if dt == torch.float32 else np.float64


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_decompose_long_lines(case):
    shape, b, L, M, _, dt = case
    print("case", _ids(case), flush=True)
    x = synth.gaussian_random_field(shape, 3.0, seed=41, dtype=np.float64).astype(_npdt(dt))
    p = _plan(shape, b, L, M, dt)
    c = p.decompose(torch.from_numpy(x).cuda()).cpu().double().numpy()
    ref = mgard.decompose(x.astype(np.float64), b, L, M)
    err = float(np.abs(c - ref).max() / np.abs(x).max())
    print("max rel coefficient error", err)
    assert err <= TOL[dt]


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_recompose_long_lines(case):
    shape, b, L, M, _, dt = case
    print("case", _ids(case), flush=True)
    rng = np.random.default_rng(42)
    h = mgard.hierarchy(shape, b, L, M)
    x = synth.gaussian_random_field(shape, 3.0, seed=43, dtype=np.float64)
    coeff = (mgard.decompose(x, b, L, M) + 0.01 * rng.standard_normal(h.shape_p)).astype(_npdt(dt))
    p = _plan(shape, b, L, M, dt)
    out = p.recompose(torch.from_numpy(coeff).cuda()).cpu().double().numpy()
    ref = mgard.recompose(coeff.astype(np.float64), shape, b, L, M)
    err = float(np.abs(out - ref).max() / np.abs(ref).max())
    print("max rel recompose error", err)
    assert err <= TOL[dt]


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_transposes_long_lines(case):
    shape, b, L, M, _, dt = case
    print("case", _ids(case), flush=True)
    p = _plan(shape, b, L, M, dt)
    rng = np.random.default_rng(44)
    g = rng.standard_normal(p.coeff_shape).astype(_npdt(dt))
    got = p.decompose_adjoint(torch.from_numpy(g).cuda()).cpu().double().numpy()
    ref = mgard.decompose_adjoint(g.astype(np.float64), shape, b, L, M)
    scale = max(1.0, float(np.abs(ref).max()))
    assert float(np.abs(got - ref).max()) <= TOL_T[dt] * scale
    gx = rng.standard_normal(shape).astype(_npdt(dt))
    got = p.recompose_adjoint(torch.from_numpy(gx).cuda()).cpu().double().numpy()
    ref = mgard.recompose_adjoint(gx.astype(np.float64), shape, b, L, M)
    scale = max(1.0, float(np.abs(ref).max()))
    assert float(np.abs(got - ref).max()) <= TOL_T[dt] * scale
