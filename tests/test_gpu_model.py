"""The time model calibrated on the device (bm_model_calibrate) and Algorithm 1
on its predictions (bm_select_levels), through the C ABI.  Every fit is
finite and non-negative; predictions of the fused decompose + quantize of a
257^3 field stay within a factor of two of the measured time for the (L, M)
splits the calibration covers (the errors are printed); the budget rule
picks the most global levels that fit."""
import numpy as np
import pytest
import torch

from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import api
    return api.model_calibrate(torch.float32, 17)


def test_fits_are_finite(model):
    for k, v in model.items():
        if k in ("dtype", "block"):
            continue
        vals = v if isinstance(v, list) else [v]
        for x in vals:
            assert np.isfinite(x) and x >= 0, (k, x)
    assert model["blk_tp"] > 0 and model["blk_lat_ms"] > 0


def test_predicted_vs_measured(model):
    from paper_2609_00205_amd import Plan, api
    n = 257
    x = torch.from_numpy(synth.gaussian_random_field((n, n, n), 3.0, seed=51)).cuda()
    worst = 0.0
    for L, M in [(1, 0), (1, 1), (1, 2), (2, 0), (2, 1), (0, 2)]:
        p = Plan((n, n, n), dtype=torch.float32, block=17, L=L, M=M)
        bt = p.tolmap_from_boxes([], 1e-3 * float(x.abs().max()))
        codes = torch.empty(p.coeff_shape, dtype=torch.int32, device="cuda")
        for _ in range(3):
            p.decompose_quantize(x, bt, codes=codes, check=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            p.decompose_quantize(x, bt, codes=codes, check=False)
        e1.record()
        torch.cuda.synchronize()
        meas = e0.elapsed_time(e1) / 10
        pred = api.model_predict(model, (n, n, n), L, M)
        est = pred["decompose"] + pred["quantize"]
        err = abs(est - meas) / meas
        worst = max(worst, err)
        print(f"L={L} M={M}: predicted {est:.4f} ms, measured {meas:.4f} ms ({100 * err:.0f}%)")
        assert 0.5 * meas <= est <= 2.0 * meas
    print("worst relative error", worst)


def test_budget_rule(model):
    from paper_2609_00205_amd import api
    shape = (512, 512, 512)
    _, cands = api.select_levels(shape, 1e9, model)
    best_m = max(c["M"] for c in cands)
    choice, _ = api.select_levels(shape, 1e9, model)
    assert choice["fits"] and choice["M"] == best_m
    assert choice["L"] == min(c["L"] for c in cands if c["M"] == best_m)
    tight = min(c["ms"] for c in cands)
    choice, _ = api.select_levels(shape, tight * 0.5, model)
    assert not choice["fits"]
