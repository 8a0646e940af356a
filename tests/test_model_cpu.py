"""The time model and Algorithm 1 (Sec. IV-B) in the library, host only:
bm_model_predict equals the oracle's predict (Eq. 1 for block levels, lines
for global levels and Huffman stages, max(slope N, T_lat) for quantization)
for hand-made models, and bm_select_levels picks what the oracle's
Algorithm 1 picks from the same candidates under every budget."""
import numpy as np
import pytest
import torch

from oracle import selector

MODELS = [
    {"dtype": torch.float32, "block": 17, "blk_lat_ms": 0.007, "blk_tp": 1.0e5, "fblk_lat_ms": 0.009,
     "fblk_tp": 0.9e5, "fglob_a_ms": 0.03, "fglob_b_ms": 2.0e-9, "glob_a_ms": 0.012, "glob_b_ms": 1.2e-8,
     "q_slope_ms": 1.0e-10, "q_lat_ms": 0.02, "gq_slope_ms": 2.0e-11, "gq_lat_ms": 0.011,
     "huf_a_ms": [0.05, 0.4, 0.1, 0.05], "huf_b_ms": [2e-9, 0.0, 3e-8, 5e-8]},
    {"dtype": torch.float64, "block": 9, "blk_lat_ms": 0.004, "blk_tp": 4.0e5, "fblk_lat_ms": 0.005,
     "fblk_tp": 3.5e5, "fglob_a_ms": 0.02, "fglob_b_ms": 4.0e-9, "glob_a_ms": 0.01, "glob_b_ms": 2.5e-8,
     "q_slope_ms": 3.0e-10, "q_lat_ms": 0.015, "gq_slope_ms": 5.0e-10, "gq_lat_ms": 0.008,
     "huf_a_ms": [0.04, 0.3, 0.08, 0.03], "huf_b_ms": [1e-9, 1e-10, 2e-8, 4e-8]},
    {"dtype": torch.float32, "block": 33, "blk_lat_ms": 0.02, "blk_tp": 2.0e4, "fblk_lat_ms": 0.02,
     "fblk_tp": 2.0e4, "fglob_a_ms": 0.012, "fglob_b_ms": 1.2e-8, "glob_a_ms": 0.012, "glob_b_ms": 1.2e-8,
     "q_slope_ms": 1.0e-10, "q_lat_ms": 0.02, "gq_slope_ms": 2.0e-11, "gq_lat_ms": 0.011,
     "huf_a_ms": [0.05, 0.4, 0.1, 0.05], "huf_b_ms": [2e-9, 0.0, 3e-8, 5e-8]},
]
SHAPES = [(513, 513, 513), (512, 512, 512), (100, 500, 500), (257, 129, 65), (65, 65, 65)]


@pytest.fixture(scope="module")
def lib():
    import os
    from paper_2609_00205_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2609_00205_amd import build
        build.build()
    return _lib.lib()


@pytest.mark.parametrize("mi", range(len(MODELS)))
@pytest.mark.parametrize("shape", SHAPES)
def test_predict_equals_oracle(lib, mi, shape):
    from paper_2609_00205_amd import api
    model = MODELS[mi]
    _, cands = api.select_levels(shape, 1e9, model)
    assert cands
    for c in cands:
        got = api.model_predict(model, shape, c["L"], c["M"])
        ref = selector.predict(shape, model["block"], c["L"], c["M"], model)
        np.testing.assert_allclose([got["decompose"], got["quantize"], got["lossless"], got["total"]], ref,
                                   rtol=1e-12, atol=0)
        assert c["ms"] == pytest.approx(ref[3], rel=1e-12, abs=0)


@pytest.mark.parametrize("mi", range(len(MODELS)))
@pytest.mark.parametrize("shape", SHAPES)
def test_algorithm1_equals_oracle(lib, mi, shape):
    from paper_2609_00205_amd import api
    model = MODELS[mi]
    _, cands = api.select_levels(shape, 1e9, model)
    pairs = [(c["L"], c["M"]) for c in cands]
    pred = {(L, M): selector.predict(shape, model["block"], L, M, model)[3] for (L, M) in pairs}
    times = sorted(pred.values())
    budgets = [times[0] * 0.5] + [0.5 * (a + b) for a, b in zip(times, times[1:])] + [times[-1] * 2]
    for budget in budgets:
        choice, _ = api.select_levels(shape, budget, model)
        ref = selector.select(pairs, lambda L, M: pred[(L, M)], budget)
        if ref is None:
            assert not choice["fits"]
            fastest = min(pairs, key=lambda lm: pred[lm])
            assert (choice["L"], choice["M"]) == fastest
        else:
            assert choice["fits"] and (choice["L"], choice["M"]) == ref, (budget, choice, ref)


def test_candidates_are_valid_hierarchies(lib):
    # every candidate the library offers is a hierarchy the oracle can build,
    # padding the volume by at most 1/8
    from oracle import mgard
    from paper_2609_00205_amd import api
    for shape in SHAPES:
        _, cands = api.select_levels(shape, 1e9, MODELS[0])
        for c in cands:
            h = mgard.hierarchy(shape, 17, c["L"], c["M"])
            assert np.prod(h.shape_p) <= 1.125 * np.prod(shape)
