"""Exact bin widths of the oracle's quantizer against a hand-derived table.

``tests/golden/delta_exact.json`` derives Delta for sampled nodes of three
small cases from the coefficient counts, the 1/(64 T) share floor and the
renormalisation of the budget shares (Sec. II-B level-dependent budget), the
level gains (the dense 3D amplifications of a face-fixed and of a natural
9-node level, and of a natural 8-node level, rounded up to 4 decimals), Eq. 2
propagation and tau_global (Sec. IV-C) and Delta = 2e (Sec. IV-D).  The
comparison is two-sided (relative 1e-13), so a Delta that is too small (a
dropped factor 2, a share divided twice) fails as well as one too large.
"""
import json
import os

import numpy as np
import pytest

from oracle import mgard, paper8, roi

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "delta_exact.json")))
CASES = {c["name"]: c for c in GOLD["cases"]}


def _tau_map(case, nb):
    t = np.full(nb, case["block_tol"]["default"])
    for idx, v in case["block_tol"]["blocks"]:
        t[tuple(idx)] = v
    return t


@pytest.mark.parametrize("name", ["shared_face_17_b9_L1_M1", "shared_face_33_b9_L2_M1"])
@pytest.mark.parametrize("eta,key", [(0.0, "rows_eta0"), (0.1, "rows_eta01")])
def test_shared_face_delta_exact(name, eta, key):
    c = CASES[name]
    h = mgard.hierarchy(tuple(c["shape"]), c["b"], c["L"], c["M"])
    assert h.shape_p == tuple(c["shape"])
    nb = [(n - 1) // (c["b"] - 1) for n in h.shape_p]
    d = roi.node_delta(h, _tau_map(c, nb), eta)
    for pos, what, formula, want in c[key]:
        got = float(d[tuple(pos)])
        assert got == pytest.approx(want, rel=1e-13, abs=0.0), (pos, what, formula, got, want)


def test_shared_face_shares_exact():
    c = CASES["shared_face_33_b9_L2_M1"]
    h = mgard.hierarchy(tuple(c["shape"]), c["b"], c["L"], c["M"])
    assert roi.level_weights(h) == pytest.approx(c["shares"], rel=1e-14, abs=0.0)


def test_shared_face_delta_class_counts():
    # every level-1 detail in the closed node range of the strict block takes its Delta:
    # 9^3 - 5^3 = 604 nodes; every other level-1 detail takes the background one
    c = CASES["shared_face_17_b9_L1_M1"]
    h = mgard.hierarchy(tuple(c["shape"]), c["b"], c["L"], c["M"])
    d = roi.node_delta(h, _tau_map(c, [2, 2, 2]), 0.0)
    lev = mgard.node_level(h.shape_p, 1, 1)
    strict, loose = c["rows_eta0"][0][3], c["rows_eta0"][2][3]
    d1 = d[lev == 1]
    assert d1.size == 17 ** 3 - 9 ** 3
    assert int(np.isclose(d1, strict, rtol=1e-13, atol=0).sum()) == 9 ** 3 - 5 ** 3
    assert int(np.isclose(d1, loose, rtol=1e-13, atol=0).sum()) == d1.size - (9 ** 3 - 5 ** 3)


@pytest.mark.parametrize("eta,key", [(0.0, "rows_eta0"), (0.1, "rows_eta01")])
def test_paper8_delta_exact(eta, key):
    c = CASES["paper8_16_L1"]
    shape = tuple(c["shape"])
    d = paper8.node_delta(shape, c["L"], _tau_map(c, [2, 2, 2]), eta)
    assert d.size == 16 ** 3 + 10 ** 3
    for (part, pos), what, formula, want in c[key]:
        flat = (np.ravel_multi_index(pos, (16, 16, 16)) if part == 0
                else 16 ** 3 + np.ravel_multi_index(pos, (10, 10, 10)))
        got = float(d[flat])
        assert got == pytest.approx(want, rel=1e-13, abs=0.0), (pos, what, formula, got, want)


def test_global_levels_share_equally():
    # 17^3, b = 9, L = 1, M = 2: grids 17^3 -> 9^3 (block level) -> 5^3 -> 3^3 (global levels).
    # The global details number (9^3 - 5^3) + (5^3 - 3^3) = 604 + 98 = 702 of N = 4913; the two
    # global levels take 702 / 4913 / 2 = 351 / 4913 each (Sec. IV-C: tau_global split equally
    # over the M global levels); T = 4, floor 1/256, coarsest 27/4913 is above it and the shares
    # (4184 + 702 + 27) / 4913 sum to 1.  With tau_global = 1e-3 and eta = 0:
    # Delta_s * A_s = 2e-3 * 351 / 4913 for both global levels, A_s the level's gain (pinned to
    # the dense worst case in test_oracle_roi.py).
    h = mgard.hierarchy((17, 17, 17), 9, 1, 2)
    tau = np.full((2, 2, 2), 1e-2)
    tau[1, 1, 0] = 1e-3
    d = roi.node_delta(h, tau, 0.0)
    gains = roi.level_gains(h)
    lev = mgard.node_level(h.shape_p, 1, 2)
    for s in (2, 3):
        got = d[lev == s] * gains[s - 1]
        np.testing.assert_allclose(got, 2e-3 * 351 / 4913, rtol=1e-13, atol=0)
    np.testing.assert_allclose(d[lev == 4], 2e-3 * 27 / 4913, rtol=1e-13, atol=0)
