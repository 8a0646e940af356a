"""Kept quantizer tables (bm_quant_prepare): calls given the kept map write
the codes and reconstructions of calls that build the tables themselves; a
call with another map builds its own and drops the kept ones; the overflow
flag is still cleared per call (a range error is reported once, not by the
calls after it).
"""
import numpy as np
import pytest
import torch

from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()


CASES = [((33, 33, 33), 17, 1, 2, torch.float32), ((65, 33, 49), 9, 2, 1, torch.float64),
         ((40, 50, 61), 9, 1, 2, torch.float32), ((65, 65, 65), 33, 1, 0, torch.float32)]


@pytest.mark.parametrize("shape,b,L,M,dt", CASES)
def test_kept_tables_equal_built_tables(shape, b, L, M, dt):
    from paper_2609_00205_amd import Plan
    x = torch.from_numpy(synth.gaussian_random_field(shape, 3.0, seed=51, dtype=np.float64)).to(dt).cuda()
    sc = float(x.abs().max())
    p = Plan(shape, dtype=dt, block=b, L=L, M=M)
    bt = p.tolmap_from_boxes([(3, 3, 3, 15, 15, 15, 1e-5 * sc)], 1e-2 * sc)
    bt2 = p.tolmap_from_boxes([], 1e-3 * sc)
    ref = p.decompose_quantize(x, bt).clone()
    ref2 = p.decompose_quantize(x, bt2).clone()
    xr_ref = p.dequantize_recompose(ref, bt).clone()
    p.quant_prepare(bt)
    for _ in range(2):
        assert torch.equal(p.decompose_quantize(x, bt), ref)
        assert torch.equal(p.dequantize_recompose(ref, bt), xr_ref)
    assert torch.equal(p.quantize(p.decompose(x), bt)[0], ref)
    # another map: its own tables, the kept ones dropped; bt works again after
    assert torch.equal(p.decompose_quantize(x, bt2), ref2)
    assert torch.equal(p.decompose_quantize(x, bt), ref)
    p.quant_prepare(bt)
    assert torch.equal(p.dequantize_recompose(ref, bt), xr_ref)
    p.quant_prepare(None)
    assert torch.equal(p.decompose_quantize(x, bt), ref)


def test_overflow_flag_cleared_with_kept_tables():
    from paper_2609_00205_amd import Plan, _lib
    shape = (33, 33, 33)
    x = torch.from_numpy(synth.gaussian_random_field(shape, 3.0, seed=52, dtype=np.float32)).cuda()
    p = Plan(shape, dtype=torch.float32, block=17, L=1, M=2)
    tiny = p.tolmap_from_boxes([], 1e-12)
    ok = p.tolmap_from_boxes([], 1e-3 * float(x.abs().max()))
    p.quant_prepare(tiny)
    with pytest.raises(_lib.BMError) as e:
        p.decompose_quantize(x, tiny, check=True)
    assert e.value.code == -7
    p.quant_prepare(ok)
    p.decompose_quantize(x, ok, check=True)          # no stale range error
    xb = x * 1e9                                      # codes beyond int32 under the kept map
    with pytest.raises(_lib.BMError) as e:
        p.decompose_quantize(xb, ok, check=True)
    assert e.value.code == -7
    p.decompose_quantize(x, ok, check=True)           # cleared again
