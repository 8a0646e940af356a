"""Pins of the oracle's ROI map, propagation, budget and quantizer.

* Eq. 2 and Fig. 6 (Sec. IV-C): the coarse block fed by blocks of tolerance
  tau0, tau1, tau2 gets tau2; blocks away from the ROI keep the background.
* Sec. IV-C: a partly covered block takes the stricter tolerance.
* Sec. IV-C: tau_global is the minimum over the last local level.
* Sec. II-B / V-A: the reconstruction error stays within the bound everywhere,
  checked by brute force, including adversarial worst-case errors built
  from the rows of the recomposition matrix (obtained from its transpose).
* The gain A computed from 1D row sums equals the dense brute force.
"""
import numpy as np
import pytest

from oracle import mgard, roi


def test_fig6_propagation():
    t0, t1, t2 = 1e-2, 1e-3, 1e-4
    tol = np.full((1, 1, 8), t0)
    tol[0, 0, 3:5] = [t1, t2]          # adjacent blocks tau0 | tau1 | tau2 | tau0
    nxt = roi.propagate(tol)
    assert nxt.shape == (1, 1, 4)
    # blocks 1 and 2 of the next level receive the tau1/tau2 blocks -> strictest
    assert nxt[0, 0, 1] == t2 and nxt[0, 0, 2] == t2
    # block 0 spans fine blocks 0..2 (+ none before), untouched
    assert nxt[0, 0, 0] == t0
    # block 3 touches fine block 5 (tau0), 6, 7 only
    assert nxt[0, 0, 3] == t0


def test_influence_region_grows_with_levels():
    tol = np.full((16, 16, 16), 1.0)
    tol[7, 7, 7] = 0.1
    tols = roi.level_block_tolerances(tol, 3)
    counts = [int((t < 1).sum()) for t in tols]
    fracs = [c / t.size for c, t in zip(counts, tols)]
    assert counts[0] == 1
    assert fracs[1] > fracs[0] and fracs[2] > fracs[1]


def test_partial_overlap_is_strict():
    shape = (17, 17, 17)
    vt = roi.voxel_tolerance_from_boxes(shape, [(8, 8, 8, 9, 9, 9, 1e-5)], 1e-2)
    bt = roi.block_tolerance(vt, shape, 9)
    # node (8,8,8) is a shared corner of all 8 blocks -> all strict
    assert np.all(bt == 1e-5)
    vt = roi.voxel_tolerance_from_boxes(shape, [(0, 0, 0, 2, 2, 2, 1e-5)], 1e-2)
    bt = roi.block_tolerance(vt, shape, 9)
    assert bt[0, 0, 0] == 1e-5 and (bt == 1e-5).sum() == 1


def test_padded_nodes_copy_source_tolerance():
    shape = (10, 10, 10)             # pads to 17 with b = 9; nodes 10..16 copy node 9
    vt = np.full(shape, 1e-2)
    vt[9, 9, 9] = 1e-6
    bt = roi.block_tolerance(vt, (17, 17, 17), 9)
    # block 1 spans nodes 8..16 (node 9 and its copies); block 0 spans 0..8
    assert bt[1, 1, 1] == 1e-6 and bt[0, 0, 0] == 1e-2 and (bt == 1e-6).sum() == 1
    vt[9, 9, 9] = 1e-2
    vt[8, 8, 8] = 1e-6                # the corner shared by all 8 blocks
    bt = roi.block_tolerance(vt, (17, 17, 17), 9)
    assert np.all(bt == 1e-6)


@pytest.mark.parametrize("coords,ff", [([np.arange(9.0)] * 3, False), ([np.arange(9.0)] * 3, True),
                                        ([np.arange(5.0), np.arange(9.0), np.arange(17.0)], False),
                                        ([np.arange(2.0), np.arange(9.0), np.arange(5.0)], False)])
def test_gain_separable_equals_dense(coords, ff):
    assert roi.amplification(coords, ff) == pytest.approx(roi.amplification_dense(coords, ff), abs=1e-12)


def test_gain_is_the_true_worst_case():
    # the dense gain is attained by the sign pattern of the worst row
    coords = [np.arange(9.0)] * 3
    ops = [mgard.axis_ops(c, True) for c in coords]
    a = [o.P @ o.K for o in ops]
    E = np.eye(729) - np.kron(np.kron(a[0], a[1]), a[2])
    coarse = np.zeros((9, 9, 9), bool)
    coarse[np.ix_(*(o.cidx for o in ops))] = True
    det = ~coarse.ravel()
    row = np.abs(E[:, det]).sum(axis=1).argmax()
    err = np.zeros(729)
    err[det] = np.sign(E[row, det])
    assert (E @ err)[row] == pytest.approx(roi.amplification(coords, True), abs=1e-12)


def _setup(shape, b, L, M, seed, boxes, bg):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    h = mgard.hierarchy(shape, b, L, M)
    vt = roi.voxel_tolerance_from_boxes(shape, boxes, bg)
    tol1 = roi.block_tolerance(vt, h.shape_p, b) if L > 0 else vt.min()
    return x, h, vt, tol1


CASES = [((33, 33, 33), 9, 1, 1, [(2, 3, 4, 10, 12, 9, 1e-4)], 1e-2),
         ((33, 33, 33), 9, 2, 1, [(20, 20, 20, 26, 30, 25, 1e-5)], 1e-2),
         ((33, 17, 33), 9, 2, 0, [(0, 0, 0, 5, 5, 5, 1e-4)], 1e-1),
         ((17, 17, 17), 17, 1, 2, [(9, 9, 9, 12, 12, 12, 1e-5)], 1e-3),
         ((20, 30, 12), 9, 1, 1, [(15, 25, 6, 20, 30, 12, 1e-5)], 1e-3),
         ((17, 9, 33), 9, 0, 3, [], 1e-3)]


@pytest.mark.parametrize("shape,b,L,M,boxes,bg", CASES)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bound_holds_random(shape, b, L, M, boxes, bg, seed):
    x, h, vt, tol1 = _setup(shape, b, L, M, seed, boxes, bg)
    c = mgard.decompose(x, b, L, M)
    delta = roi.node_delta(h, tol1, 0.0)
    q = roi.quantize(c, delta)
    assert np.all(np.abs(c - roi.dequantize(q, delta)) <= delta / 2 * (1 + 1e-12))
    xr = mgard.recompose(roi.dequantize(q, delta), shape, b, L, M)
    assert np.all(np.abs(xr - x) <= vt)


@pytest.mark.parametrize("shape,b,L,M,boxes,bg", CASES)
def test_bound_holds_adversarial(shape, b, L, M, boxes, bg):
    # Worst case: every coefficient off by exactly Delta/2 with the sign of
    # the recomposition row of a target node.  Rows come from R^T e_target.
    x, h, vt, tol1 = _setup(shape, b, L, M, 0, boxes, bg)
    delta = roi.node_delta(h, tol1, 0.0)
    rng = np.random.default_rng(7)
    strict = np.argwhere(vt == vt.min())
    targets = [tuple(strict[0]), tuple(strict[-1])] + [tuple(rng.integers(0, s) for s in shape) for _ in range(4)]
    for t in targets:
        e = np.zeros(shape)
        e[t] = 1.0
        row = mgard.recompose_adjoint(e, shape, b, L, M)
        worst = float(np.sum(np.abs(row) * delta / 2))
        assert worst <= vt[t] * (1 + 1e-12), (t, worst, vt[t])


def test_tau_global_is_min_of_last_local_level():
    tol = np.full((4, 4, 4), 1e-2)
    tol[1, 2, 3] = 1e-6
    tols = roi.level_block_tolerances(tol, 2)
    assert tols[-1].min() == 1e-6
    h = mgard.hierarchy((33, 33, 33), 9, 2, 1)
    d = roi.node_delta(h, tol, 0.0)
    lev = mgard.node_level(h.shape_p, 2, 1)
    A3 = roi.level_gains(h)[2]
    # level-3 share: its count over the 33^3 grid, renormalised after the
    # coarsest share 5^3 / 33^3 is raised to the floor 1/(64 T), T = 4
    floor = 1.0 / 256.0
    raw = [(33 ** 3 - 17 ** 3) / 33 ** 3, (17 ** 3 - 9 ** 3) / 33 ** 3, (9 ** 3 - 5 ** 3) / 33 ** 3, floor]
    w3 = raw[2] / sum(raw)
    got = d[lev == 3]
    assert got.size == 9 ** 3 - 5 ** 3
    np.testing.assert_allclose(got, 1e-6 * 2 * w3 / A3, rtol=1e-13, atol=0)


def test_budget_shares_tighten_as_levels_coarsen():
    # Sec. II-B: level-dependent shares that tighten with coarser levels;
    # Sec. IV-C: the M global levels share their part equally.
    h = mgard.hierarchy((65, 65, 65), 9, 2, 3)
    w = roi.level_weights(h)
    assert sum(w) == pytest.approx(1.0, abs=1e-15)
    assert w[0] > w[1] > w[2]                  # local levels, then the global block
    assert w[2] == w[3] == w[4]                # equal global shares
    # 65 -> 33 -> 17 -> 9 -> 5 -> 3: the coarsest share 27 / 65^3 is below the
    # floor 1/(64 T) and is raised to it before renormalising
    floor = 1 / (64 * 6)
    raw0 = (65 ** 3 - 33 ** 3) / 65 ** 3
    nglob = 17 ** 3 - 3 ** 3
    raw = [raw0, (33 ** 3 - 17 ** 3) / 65 ** 3] + [max(floor, nglob / 65 ** 3 / 3)] * 3 + [max(floor, 27 / 65 ** 3)]
    assert w[0] == pytest.approx(raw0 / sum(raw))
    assert w[5] == pytest.approx(floor / sum(raw))
    assert min(w) >= floor / sum(raw) * (1 - 1e-12)


def test_quantizer_round_half_even_and_reciprocal():
    delta = np.full(6, 0.5)
    c = np.array([0.25, 0.75, -0.25, 1.0, 0.1, -1.3])
    assert list(roi.quantize(c, delta)) == [0, 2, 0, 2, 0, -3]


def test_qoi_level_hand_examples():
    # sum_i min(a_i, lambda) = target, worked by hand
    assert roi.qoi_level(np.array([1.0, 2.0, 3.0]), 4.5) == pytest.approx(1.75, abs=1e-15)   # 1 + 1.75 + 1.75
    assert roi.qoi_level(np.array([3.0, 1.0, 2.0]), 3.0) == pytest.approx(1.0, abs=1e-15)    # 1 + 1 + 1
    assert roi.qoi_level(np.array([0.0, 0.0, 5.0]), 2.0) == pytest.approx(2.0, abs=1e-15)    # zeros take nothing
    assert roi.qoi_level(np.array([1.0, 2.0]), 3.0) is None                                  # the caps fit


@pytest.mark.parametrize("shape,b,L,M,box", [((9, 9, 9), 9, 1, 1, (2, 6)), ((9, 5, 13), 9, 1, 1, (1, 4)),
                                             ((5, 9, 17), 9, 0, 3, (1, 4))])
@pytest.mark.parametrize("bg", [1e-2, 1e-7])
def test_qoi_delta_keeps_the_quantity(shape, b, L, M, box, bg):
    # Q(x) = mean over a sub-box.  Sensitivities by brute force (Q of the
    # recomposition of every unit coefficient) agree with R^T g; the worst
    # case of the quantization errors (every coefficient off by Delta/2 with
    # the sign of its sensitivity) moves Q by exactly tol_q when the
    # quantity binds (bg 1e-2) and by less when every cap fits (bg 1e-7);
    # no width exceeds the map's; widths set by the quantity all carry the
    # same share |s_i| Delta_i / 2; quantizing a random field keeps Q within
    # tol_q and every node within the map's bound.
    rng = np.random.default_rng(3)
    h = mgard.hierarchy(shape, b, L, M)
    lo, hi = box
    g = np.zeros(shape)
    g[lo:hi, lo:hi, lo:hi] = 1.0 / (hi - lo) ** 3
    tol1 = np.full([(n - 1) // (b - 1) for n in h.shape_p], bg) if L > 0 else bg
    tol_q = 1e-6
    delta, nset = roi.qoi_delta(h, tol1, g, tol_q, 0.0)
    npad = int(np.prod(h.shape_p))
    s = np.empty(npad)
    for i in range(npad):
        e = np.zeros(npad)
        e[i] = 1.0
        s[i] = float((g * mgard.recompose(e.reshape(h.shape_p), shape, b, L, M)).sum())
    s = s.reshape(h.shape_p)
    st = mgard.recompose_adjoint(g, shape, b, L, M)
    assert np.abs(s - st).max() <= 1e-14 * np.abs(s).max()
    base = roi.node_delta(h, tol1, 0.0)
    assert np.all(delta <= base)
    worst = float((np.abs(s) * delta / 2).sum())
    if bg == 1e-2:
        assert nset > 0
        assert worst == pytest.approx(tol_q, rel=1e-9)
        share = np.abs(s) * delta / 2
        setq = delta < base
        assert int(setq.sum()) == nset
        assert np.allclose(share[setq], share[setq].max(), rtol=1e-12, atol=0)
        assert np.all(share[~setq] <= share[setq].max() * (1 + 1e-12))
    else:
        assert nset == 0 and np.array_equal(delta, base) and worst <= tol_q
    x = rng.standard_normal(shape)
    c = mgard.decompose(x, b, L, M)
    xr = mgard.recompose(roi.dequantize(roi.quantize(c, delta), delta), shape, b, L, M)
    assert abs(float((g * (xr - x)).sum())) <= tol_q
    assert float(np.abs(xr - x).max()) <= bg
