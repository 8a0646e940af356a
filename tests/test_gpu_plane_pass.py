"""The plane pass of the global levels (K along x and y of each z-plane in
one launch, from LDS) against the line passes it replaces: a plan created
with BM_PLANE_PASS=0 runs one launch per axis.  Both must give the same
coefficients, reconstructions and codes, bit for bit, on grids whose planes
fit the pass: FP32 and FP64 levels with 3 and 5 unknowns per lane, the fused
first global level's FP64 solve-only planes with 3, 5 and 9, the coarse-node
mask and the codes read on load, and a hierarchy that ends on a global
level (its coarsest values quantized and dequantized by the last pass).
"""
import os

import numpy as np
import pytest
import torch

from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu

CASES = [((65, 65, 65), 17, 0, 3, torch.float32),    # level planes 65^2 -> 33^2, 33^2 -> 17^2 (Q = 3)
         ((65, 65, 65), 17, 0, 2, torch.float64),
         ((129, 129, 129), 17, 1, 2, torch.float32),  # fused solve-only FP64 planes 33^2, then 33^2 -> 17^2
         ((129, 129, 129), 9, 1, 2, torch.float64),
         ((33, 257, 257), 17, 1, 2, torch.float32),   # solve-only 65^2 (Q = 5), then 65^2 -> 33^2
         ((33, 513, 513), 17, 1, 1, torch.float32),   # solve-only 129^2 (Q = 9), the 512^3 step's layout
         ((40, 50, 61), 9, 1, 2, torch.float32)]      # ragged: padded dims, unequal plane sides


def _ids(c):
    return "x".join(map(str, c[0])) + f"-b{c[1]}-L{c[2]}M{c[3]}-{str(c[4])[6:]}"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()


def _plans(shape, b, L, M, dt):
    from paper_2609_00205_amd import Plan
    a = Plan(shape, dtype=dt, block=b, L=L, M=M)
    old = os.environ.get("BM_PLANE_PASS")
    os.environ["BM_PLANE_PASS"] = "0"
    try:
        z = Plan(shape, dtype=dt, block=b, L=L, M=M)
    finally:
        if old is None:
            del os.environ["BM_PLANE_PASS"]
        else:
            os.environ["BM_PLANE_PASS"] = old
    return a, z


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_plane_pass_equals_line_passes(case):
    shape, b, L, M, dt = case
    print("case", _ids(case), flush=True)
    a, z = _plans(shape, b, L, M, dt)
    x = torch.from_numpy(synth.gaussian_random_field(shape, 3.0, seed=71, dtype=np.float64)).to(dt).cuda()
    ca, cz = a.decompose(x), z.decompose(x)
    assert torch.equal(ca, cz), float((ca - cz).abs().max())
    rng = np.random.default_rng(7)
    c = ca + torch.from_numpy(0.01 * rng.standard_normal(tuple(ca.shape))).to(dt).cuda()
    ra, rz = a.recompose(c), z.recompose(c)
    assert torch.equal(ra, rz), float((ra - rz).abs().max())
    sc = float(x.abs().max())
    box = [(2, 2, 2, 2 + shape[0] // 3, 2 + shape[1] // 3, 2 + shape[2] // 3, 1e-5 * sc)]
    ba, bz = a.tolmap_from_boxes(box, 1e-2 * sc), z.tolmap_from_boxes(box, 1e-2 * sc)
    qa, qz = a.decompose_quantize(x, ba), z.decompose_quantize(x, bz)
    assert torch.equal(qa, qz), int((qa != qz).sum())
    xa, xz = a.dequantize_recompose(qa, ba), z.dequantize_recompose(qa, bz)
    assert torch.equal(xa, xz), float((xa - xz).abs().max())
    assert float((xa - x).abs().max()) <= 1e-2 * sc
