"""GPU transposes D^T and R^T (the adjoint kernels) against the FP64 oracle,
through the C ABI, plus the properties that hold at any size.

Bar: within 2e-6 * max|ref| (FP32) and 1e-12 * max|ref| (FP64) of the
oracle's transposes on the same seeded inputs; <D x, y> = <x, D^T y> and
<R c, g> = <c, R^T g> to rounding (normalised by |D x| |y|) on the GPU alone,
including the full 512^3 FP32 configuration.
"""
import numpy as np
import pytest
import torch

from oracle import mgard
from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 2e-6, torch.float64: 1e-12}

# (shape, b, L, M, dtype, pad_mode)
CASES = [
    ((33, 33, 33), 17, 1, 2, torch.float64, "clamp"),
    ((33, 33, 33), 17, 1, 2, torch.float32, "clamp"),
    ((20, 30, 12), 9, 1, 1, torch.float64, "clamp"),      # ragged: padded to 25 x 33 x 17
    ((20, 30, 12), 9, 1, 1, torch.float32, "zero"),
    ((33, 17, 65), 9, 2, 1, torch.float64, "clamp"),      # two block levels
    ((65, 65, 65), 17, 0, 6, torch.float64, "clamp"),     # pure global down to 2 nodes per axis
    ((30, 9, 20), 17, 0, 3, torch.float64, "clamp"),      # pure global on a padded grid
    ((9, 5, 33), 9, 0, 4, torch.float64, "zero"),         # an axis stops coarsening at 2 nodes
    ((65, 33, 49), 17, 1, 0, torch.float32, "clamp"),     # pure local
    ((97, 65, 129), 17, 1, 2, torch.float32, "clamp"),    # 6 x 4 x 8 blocks
    ((40, 50, 61), 9, 2, 2, torch.float64, "clamp"),      # ragged everywhere
    ((17, 17, 17), 17, 1, 0, torch.float64, "clamp"),     # one block: no shared faces
    ((65, 65, 65), 33, 1, 2, torch.float64, "clamp"),     # 33^3 blocks (split transposes)
    ((70, 40, 100), 33, 1, 1, torch.float32, "zero"),     # 33^3 blocks, ragged: padded to 97 x 65 x 129
    ((65, 65, 129), 33, 2, 1, torch.float64, "clamp"),    # two 33^3 block levels
    ((33, 33, 33), 33, 1, 0, torch.float64, "clamp"),     # a single 33^3 block
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"-b{c[1]}-L{c[2]}M{c[3]}-{str(c[4])[6:]}-{c[5]}"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()


def _plan(shape, b, L, M, dt, pad="clamp"):
    from paper_2609_00205_amd import Plan
    return Plan(shape, dtype=dt, block=b, L=L, M=M, pad_mode=pad)


def _npdt(dt):
    return np.float32 if dt == torch.float32 else np.float64


def _close(got, ref, dt):
    scale = max(1.0, float(np.abs(ref).max()))
    err = float(np.abs(got - ref).max())
    assert err <= TOL[dt] * scale, f"max err {err:.3e} > {TOL[dt]:.0e} * {scale:.3e}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_decompose_adjoint_parity(case):
    shape, b, L, M, dt, pad = case
    print("case", _ids(case), flush=True)
    p = _plan(shape, b, L, M, dt, pad)
    g = np.random.default_rng(21).standard_normal(p.coeff_shape).astype(_npdt(dt))
    got = p.decompose_adjoint(torch.from_numpy(g).cuda()).cpu().double().numpy()
    ref = mgard.decompose_adjoint(g.astype(np.float64), shape, b, L, M, pad_mode=pad)
    assert got.shape == ref.shape == shape
    _close(got, ref, dt)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_recompose_adjoint_parity(case):
    shape, b, L, M, dt, pad = case
    print("case", _ids(case), flush=True)
    p = _plan(shape, b, L, M, dt, pad)
    g = np.random.default_rng(22).standard_normal(shape).astype(_npdt(dt))
    got = p.recompose_adjoint(torch.from_numpy(g).cuda()).cpu().double().numpy()
    ref = mgard.recompose_adjoint(g.astype(np.float64), shape, b, L, M)
    assert got.shape == ref.shape == p.coeff_shape
    _close(got, ref, dt)


def _dot_identity(p, shape, dt, seed, tol):
    rng = np.random.default_rng(seed)
    x = torch.from_numpy(rng.standard_normal(shape).astype(_npdt(dt))).cuda()
    y = torch.from_numpy(rng.standard_normal(p.coeff_shape).astype(_npdt(dt))).cuda()
    dx = p.decompose(x)
    dty = p.decompose_adjoint(y)
    a, b_ = float((dx.double() * y.double()).sum()), float((x.double() * dty.double()).sum())
    scale = float(dx.double().norm() * y.double().norm())
    assert abs(a - b_) <= tol * scale, (a, b_, scale)
    c = y
    rc = p.recompose(c)
    rtx = p.recompose_adjoint(x)
    a, b_ = float((rc.double() * x.double()).sum()), float((c.double() * rtx.double()).sum())
    scale = float(rc.double().norm() * x.double().norm())
    assert abs(a - b_) <= tol * scale, (a, b_, scale)


@pytest.mark.parametrize("case", CASES[:6] + CASES[-4:-2], ids=_ids)
def test_dot_product_identity(case):
    shape, b, L, M, dt, pad = case
    print("case", _ids(case), flush=True)
    _dot_identity(_plan(shape, b, L, M, dt, pad), shape, dt, 23, 1e-13 if dt == torch.float64 else 1e-6)


def test_dot_product_identity_full_size():
    """512^3 FP32, b = 17, L = 1, M = 2: the configuration the throughput is quoted on."""
    shape = (512, 512, 512)
    print("case 512^3 f32 dot identity", flush=True)
    _dot_identity(_plan(shape, 17, 1, 2, torch.float32), shape, torch.float32, 24, 1e-5)
    torch.cuda.empty_cache()


def test_autograd_matches_transposes():
    from paper_2609_00205_amd import DecomposeFn, RecomposeFn
    shape, b, L, M = (33, 33, 33), 17, 1, 2
    p = _plan(shape, b, L, M, torch.float64)
    rng = np.random.default_rng(25)
    x = torch.from_numpy(rng.standard_normal(shape)).cuda().requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal(p.coeff_shape)).cuda()
    (DecomposeFn.apply(x, p) * w).sum().backward()
    ref = mgard.decompose_adjoint(w.cpu().numpy(), shape, b, L, M)
    np.testing.assert_allclose(x.grad.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # a quantity of interest through recomposition: the mean over a sub-box
    c = torch.from_numpy(rng.standard_normal(p.coeff_shape)).cuda().requires_grad_(True)
    RecomposeFn.apply(c, p)[8:24, 4:20, 10:30].mean().backward()
    g = np.zeros(shape)
    g[8:24, 4:20, 10:30] = 1.0 / (16 * 16 * 20)
    ref = mgard.recompose_adjoint(g, shape, b, L, M)
    np.testing.assert_allclose(c.grad.cpu().numpy(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_qoi_finite_difference():
    """Q(c) = mean of R(c) over a sub-box is linear: a difference quotient
    along any direction d equals <R^T g, d> (FP64, 33^3)."""
    shape, b, L, M = (33, 33, 33), 17, 1, 2
    p = _plan(shape, b, L, M, torch.float64)
    rng = np.random.default_rng(26)
    c = torch.from_numpy(rng.standard_normal(p.coeff_shape)).cuda()
    d = torch.from_numpy(rng.standard_normal(p.coeff_shape)).cuda()
    g = torch.zeros(shape, dtype=torch.float64, device="cuda")
    g[8:24, 8:24, 8:24] = 1.0 / 16 ** 3
    s = p.recompose_adjoint(g)

    def q(cc):
        return float((p.recompose(cc) * g).sum())

    h = 1e-3
    fd = (q(c + h * d) - q(c - h * d)) / (2 * h)
    assert abs(fd - float((s * d).sum())) <= 1e-9 * max(1.0, abs(fd))
