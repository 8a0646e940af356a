"""Full-size parity: 512^3 FP32, b = 17, L = 1, M = 2, the configuration the
benchmark times.

The oracle decomposes and recomposes the whole field (about half a minute
each on the host): every coefficient and every reconstructed value is
compared.  Sampled checks it computes one block at a time (level-1 blocks,
level-2 details at sampled nodes) localise a mismatch; the round trip and
every ROI bound hold on the whole field.
"""
import numpy as np
import pytest
import torch

from oracle import mgard, roi
from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu

N, B, L, M = 512, 17, 1, 2


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available()
    from paper_2609_00205_amd import Plan
    x, boxes = synth.workload_roi(N, seed=2)
    p = Plan((N, N, N), dtype=torch.float32, block=B, L=L, M=M)
    xd = torch.from_numpy(x).cuda()
    c = p.decompose(xd)
    torch.cuda.synchronize()
    return x, boxes, p, xd, c


def _pad_block(x, bz, by, bx):
    idx = [np.minimum(np.arange(o * (B - 1), o * (B - 1) + B), N - 1) for o in (bz, by, bx)]
    return x[np.ix_(*idx)].astype(np.float64)


def _oracle_block(x, cache, key):
    if key not in cache:
        cache[key] = mgard.level_decompose(_pad_block(x, *key), [np.arange(float(B))] * 3, True)
    return cache[key]


def test_sampled_level1_blocks(setup):
    x, boxes, p, xd, c = setup
    rng = np.random.default_rng(0)
    nb = 32
    keys = [(0, 0, 0), (nb - 1, nb - 1, nb - 1), (nb - 1, 0, 17)] + \
           [tuple(int(v) for v in rng.integers(0, nb, 3)) for _ in range(13)]
    scale = float(np.abs(x).max())
    cache = {}
    worst = 0.0
    for k in keys:
        ref = _oracle_block(x, cache, k)
        o = [v * (B - 1) for v in k]
        got = c[o[0]:o[0] + B, o[1]:o[1] + B, o[2]:o[2] + B].cpu().double().numpy()
        fine = np.ones((B, B, B), bool)
        fine[::2, ::2, ::2] = False         # coarse nodes hold later levels' coefficients
        worst = max(worst, float(np.abs(got - ref)[fine].max()) / scale)
    print("worst level-1 coefficient error / max|x|:", worst)
    assert worst <= 1e-6


def test_sampled_level2_details(setup):
    x, boxes, p, xd, c = setup
    rng = np.random.default_rng(1)
    scale = float(np.abs(x).max())
    cache = {}

    def u1(q):   # level-1 coarse value at G^1 node q (fine coords 2q)
        f = [2 * v for v in q]
        k = tuple(min(v // (B - 1), 31) for v in f)
        blk = _oracle_block(x, cache, k)
        return blk[tuple(v - kk * (B - 1) for v, kk in zip(f, k))]

    worst = 0.0
    for _ in range(24):
        q = [int(v) for v in rng.integers(0, 257, 3)]
        if all(v % 2 == 0 for v in q):
            q[2] = min(255, q[2] + 1)       # a node that is fine-only at level 2
        lo = [v - (v & 1) for v in q]
        hi = [v + (v & 1) for v in q]
        corners = [(a, b_, d) for a in {lo[0], hi[0]} for b_ in {lo[1], hi[1]} for d in {lo[2], hi[2]}]
        interp = np.mean([u1(cq) for cq in corners])
        ref = u1(q) - interp
        got = float(c[2 * q[0], 2 * q[1], 2 * q[2]])
        worst = max(worst, abs(got - ref) / scale)
    print("worst level-2 detail error / max|x|:", worst)
    assert worst <= 1e-6


def test_roundtrip_and_roi_bounds(setup):
    x, boxes, p, xd, c = setup
    y = p.recompose(c)
    scale = float(xd.abs().max())
    assert float((y - xd).abs().max()) <= 2e-6 * scale
    abs_boxes = [bx + (1e-5 * scale,) for bx in boxes]
    bt = p.tolmap_from_boxes(abs_boxes, 1e-2 * scale)
    codes, st = p.quantize(c, bt)
    xr = p.recompose(p.dequantize(codes, bt))
    err = (xr.double() - xd.double()).abs()
    inside = torch.zeros_like(err, dtype=torch.bool)
    for (z0, y0, x0, z1, y1, x1, tol) in abs_boxes:
        assert float(err[z0:z1, y0:y1, x0:x1].max()) <= tol
        inside[z0:z1, y0:y1, x0:x1] = True
    assert float(err[~inside].max()) <= 1e-2 * scale
    # the block map equals the oracle's
    h = mgard.hierarchy((N, N, N), B, L, M)
    ref = roi.block_tolerance(roi.voxel_tolerance_from_boxes((N, N, N), abs_boxes, 1e-2 * scale), h.shape_p, B)
    assert np.array_equal(bt.cpu().numpy(), ref)


def test_whole_field_decompose_matches_oracle(setup):
    """Every coefficient of the 513^3 array (level-1 details, the first global
    level's solve-only passes on 257-node lines, the second global level,
    the coarsest values) against the oracle's decomposition of the whole
    field."""
    x, boxes, p, xd, c = setup
    print("oracle decomposition of the whole field", flush=True)
    ref = mgard.decompose(x.astype(np.float64), B, L, M)
    got = c.cpu().double().numpy()
    scale = float(np.abs(x).max())
    lev = mgard.node_level(ref.shape, L, M)
    for s in range(1, L + M + 2):
        e = float(np.abs(got[lev == s] - ref[lev == s]).max()) / scale
        print(f"level {s}: max coefficient error / max|x| = {e:.2e}", flush=True)
    err = float(np.abs(got - ref).max()) / scale
    assert err <= 1e-6


def test_whole_field_recompose_matches_oracle(setup):
    """Recomposition of the GPU's own coefficient array, whole field, against
    the oracle's recomposition of the same coefficients."""
    x, boxes, p, xd, c = setup
    y = p.recompose(c).cpu().double().numpy()
    print("oracle recomposition of the whole field", flush=True)
    ref = mgard.recompose(c.cpu().double().numpy(), (N, N, N), B, L, M)
    err = float(np.abs(y - ref).max()) / float(np.abs(ref).max())
    print(f"max recompose error / max|ref| = {err:.2e}")
    assert err <= 1e-6
