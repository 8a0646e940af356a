"""Pins of the oracle's paper-literal In-cache Block form (disjoint 8^3
blocks, Sec. IV-A / IV-C) against what the paper prints and what the
mathematics fixes: the working-set constants, hand-derived 8-node
operators, the dense L2 projection of one block, the re-assembly of the
5^3 outputs, multilinear exactness and reconstruction.
"""
import json
import os

import numpy as np
import pytest

from oracle import mgard, paper8

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_working_set():
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    assert paper8.B == g["block_edge"]["value"]
    assert paper8.MC == g["block_coarse_edge"]["value"] == len(paper8.COARSE)
    assert paper8.working_set() == g["working_set_elements"]["value"]
    assert paper8.MC ** 3 == g["coarse_writer_threads"]["value"]
    assert paper8.B ** 3 - paper8.MC ** 3 == g["detail_threads"]["value"]


def test_eight_node_operators_by_hand():
    # linear elements on nodes 0..7, coarse nodes 0 2 4 6 7 (spacings 2 2 2 1)
    ops = mgard.axis_ops(np.arange(8.0), False)
    assert list(ops.cidx) == [0, 2, 4, 6, 7]
    M = mgard.mass_matrix(np.arange(8.0))
    R = ops.P.T @ M
    want = np.zeros((5, 8))
    want[0, :3] = [5 / 12, 1 / 2, 1 / 12]
    want[1, :5] = [1 / 12, 1 / 2, 5 / 6, 1 / 2, 1 / 12]
    want[2, 2:7] = [1 / 12, 1 / 2, 5 / 6, 1 / 2, 1 / 12]
    want[3, 4:] = [1 / 12, 1 / 2, 3 / 4, 1 / 6]
    want[4, 6:] = [1 / 6, 1 / 3]
    assert np.allclose(R, want, atol=1e-15)
    Mc = mgard.mass_matrix(np.array([0.0, 2, 4, 6, 7]))
    assert np.allclose(np.diag(Mc), [2 / 3, 4 / 3, 4 / 3, 1, 1 / 3])
    assert np.allclose(np.diag(Mc, 1), [1 / 3, 1 / 3, 1 / 3, 1 / 6])


def _kron3(a):
    return np.kron(np.kron(a[0], a[1]), a[2])


def test_block_level_is_dense_l2_projection(rng):
    u = rng.standard_normal((8, 8, 8))
    coords = [np.arange(8.0)] * 3
    out = mgard.level_decompose(u, coords, False)
    ops = [mgard.axis_ops(c, False) for c in coords]
    P3 = _kron3([o.P for o in ops])
    M3 = _kron3([mgard.mass_matrix(c) for c in coords])
    c_dense = np.linalg.solve(P3.T @ M3 @ P3, P3.T @ M3 @ u.ravel())
    cid = np.ix_(*(o.cidx for o in ops))
    assert np.allclose(out[cid].ravel(), c_dense, atol=1e-13)


@pytest.mark.parametrize("shape,L,dims,last", [((512, 512, 512), 3, [(512,) * 3, (320,) * 3, (200,) * 3], (125,) * 3),
                                               ((20, 30, 12), 2, [(24, 32, 16), (16, 24, 16)], (10, 15, 10))])
def test_level_dims(shape, L, dims, last):
    d, m = paper8.level_dims(shape, L)
    assert d == dims and m == last


def test_reassembly_places_block_outputs_side_by_side():
    # a field constant on every block: no details, every coarse value is the
    # block's constant, found at [5 b, 5 b + 5) of the next grid
    nb = (2, 3, 2)
    ids = np.arange(np.prod(nb), dtype=float).reshape(nb) + 1.0
    x = np.kron(ids, np.ones((8, 8, 8)))
    c = paper8.decompose(x, 1)
    d, last = paper8.level_dims(x.shape, 1)
    assert np.abs(c[: np.prod(d[0])]).max() < 1e-13
    nxt = c[np.prod(d[0]):].reshape(last)
    assert np.allclose(nxt, np.kron(ids, np.ones((5, 5, 5))), atol=1e-13)


def test_multilinear_first_level_details_vanish():
    z, y, x = np.meshgrid(*(np.arange(float(n)) for n in (16, 24, 16)), indexing="ij")
    f = 0.5 + x - 2 * y + 0.25 * z + 0.1 * x * y - 0.05 * y * z + 0.003 * x * y * z
    c = paper8.decompose(f, 2)
    n1 = 16 * 24 * 16
    assert np.abs(c[:n1]).max() < 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("shape,L", [((16, 16, 16), 1), ((20, 30, 12), 2), ((33, 17, 40), 3)])
def test_reconstruction(shape, L, rng):
    x = rng.standard_normal(shape)
    c = paper8.decompose(x, L)
    assert c.size == paper8.coeff_size(shape, L)
    assert np.abs(paper8.recompose(c, shape, L) - x).max() < 1e-12 * np.abs(x).max()


# --- ROI quantization of the 8^3 form -------------------------------------

def test_propagation_by_assembled_positions(rng):
    # Eq. 2 / Fig. 6 by brute force: every assembled position p came from
    # block p // 5 of the finer level and lies in block p // 8 of the next
    tau = rng.uniform(1e-4, 1e-2, (3, 4, 2))
    m = [5 * n for n in tau.shape]
    nn = [-(-v // 8) for v in m]
    want = np.full(nn, np.inf)
    for p in np.ndindex(*m):
        I = tuple(v // 8 for v in p)
        want[I] = min(want[I], tau[tuple(v // 5 for v in p)])
    assert np.array_equal(paper8.propagate(tau, nn), want)


def test_fig6_strictest_region_wins():
    # three blocks in a row at tau0 > tau1 > tau2: the next-level block that
    # takes outputs of the second and third gets tau2, the first one tau1
    tau = np.array([1e-2, 1e-3, 1e-4]).reshape(1, 1, 3)
    out = paper8.propagate(tau, (1, 1, 2))
    assert out[0, 0, 0] == 1e-3 and out[0, 0, 1] == 1e-4


def test_gain_is_the_dense_worst_case():
    coords = [np.arange(8.0)] * 3
    ops = [mgard.axis_ops(c, False) for c in coords]
    P3 = _kron3([o.P for o in ops])
    K3 = _kron3([o.K for o in ops])
    E = np.eye(512) - P3 @ K3
    coarse = np.zeros((8, 8, 8), bool)
    coarse[np.ix_(*(o.cidx for o in ops))] = True
    det = ~coarse.ravel()
    A = np.abs(E[:, det]).sum(axis=1).max()
    assert paper8.gain() >= A and paper8.gain() - A < 1e-4


def test_shares_sum_to_one():
    w = paper8.weights((100, 70, 33), 3)
    assert abs(sum(w) - 1.0) < 1e-15 and min(w) > 0


@pytest.mark.parametrize("shape,L,seed", [((16, 16, 16), 1, 0), ((20, 30, 12), 2, 1), ((33, 17, 40), 3, 2),
                                          ((40, 40, 40), 2, 3)])
def test_bound_holds(shape, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    vt = np.full(shape, 1e-2)
    z0, y0, x0 = [int(rng.integers(0, max(1, s - 6))) for s in shape]
    vt[z0:z0 + 6, y0:y0 + 6, x0:x0 + 6] = 1e-5
    tau1 = paper8.block_tolerance(vt, L)
    delta = paper8.node_delta(shape, L, tau1, 0.0)
    c = paper8.decompose(x, L)
    q = np.rint(c * (1.0 / delta))
    xr = paper8.recompose(q * delta, shape, L)
    assert np.all(np.abs(xr - x) <= vt)


# ---- the hybrid: block levels, then global levels on the assembled grid ----

HYBRID = [((20, 30, 17), 1, 1), ((20, 30, 17), 1, 2), ((40, 24, 33), 2, 1), ((16, 16, 16), 1, 2)]


@pytest.mark.parametrize("shape,L,M", HYBRID)
def test_hybrid_reconstruction(shape, L, M, rng):
    x = rng.standard_normal(shape)
    c = paper8.decompose_hybrid(x, L, M)
    assert c.size == paper8.hybrid_coeff_size(shape, L, M)
    assert np.abs(paper8.recompose_hybrid(c, shape, L, M) - x).max() < 1e-12


def test_hybrid_without_global_levels_is_the_block_form(rng):
    x = rng.standard_normal((20, 30, 17))
    assert np.array_equal(paper8.decompose_hybrid(x, 2, 0), paper8.decompose(x, 2))
    assert paper8.hybrid_weights((20, 30, 17), 2, 0) == paper8.weights((20, 30, 17), 2)


@pytest.mark.parametrize("shape,L,M", [((16, 24, 40), 1, 1), ((24, 16, 32), 1, 2), ((64, 64, 64), 2, 1)])
def test_hybrid_constant_field(shape, L, M):
    """A constant field on grids the blocks tile without zero fill at every
    level: every detail (block and global) is zero; the global levels'
    coarsest values are the constant and nothing else is non-zero in the
    global array but them (one per node of the coarsest grid)."""
    x = np.full(shape, 3.25)
    c = paper8.decompose_hybrid(x, L, M)
    dims, last = paper8.level_dims(shape, L)
    off = int(sum(np.prod(d) for d in dims))
    assert np.abs(c[:off]).max() < 1e-12
    tail = c[off:]
    n = list(paper8.global_hierarchy(shape, L, M).shape_p)
    for _ in range(M):
        n = [(v + 1) // 2 if v > 2 else v for v in n]
    nz = np.abs(tail) > 1e-12
    assert int(nz.sum()) == int(np.prod(n))
    assert np.abs(tail[nz] - 3.25).max() < 1e-12


def test_hybrid_shares_by_hand():
    """512^3, L = 1, M = 2 (the paper's default split): block details
    64^3 blocks x 387 nodes, the assembled 320^3 grid extended to 321^3,
    global details 321^3 - 81^3 split over two levels, coarsest 81^3, whose
    share 81^3 / N = 0.0032 is raised to the floor 1 / (64 * 4)."""
    w = paper8.hybrid_weights((512, 512, 512), 1, 2)
    N = 512.0 ** 3 + 321.0 ** 3
    ref = [64.0 ** 3 * 387 / N, (321.0 ** 3 - 81.0 ** 3) / N / 2, (321.0 ** 3 - 81.0 ** 3) / N / 2, 1.0 / 256]
    assert 81.0 ** 3 / N < 1.0 / 256 < min(ref[:3])
    ref = [v / sum(ref) for v in ref]
    assert np.allclose(w, ref, rtol=1e-14, atol=0)
    assert paper8.global_hierarchy((512, 512, 512), 1, 2).shape_p == (321, 321, 321)


@pytest.mark.parametrize("shape,L,M,seed", [((16, 16, 16), 1, 1, 0), ((20, 30, 17), 1, 2, 1), ((40, 24, 33), 2, 1, 2),
                                            ((33, 40, 40), 1, 2, 3)])
def test_hybrid_bound_holds(shape, L, M, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    vt = np.full(shape, 1e-2)
    z0, y0, x0 = [int(rng.integers(0, max(1, s - 6))) for s in shape]
    vt[z0:z0 + 6, y0:y0 + 6, x0:x0 + 6] = 1e-5
    tau1 = paper8.block_tolerance(vt, L)
    delta = paper8.hybrid_node_delta(shape, L, M, tau1, 0.0)
    c = paper8.decompose_hybrid(x, L, M)
    q = np.rint(c * (1.0 / delta))
    xr = paper8.recompose_hybrid(q * delta, shape, L, M)
    assert np.all(np.abs(xr - x) <= vt)
    # global coefficients all take tau_global, the strictest block's tau
    dims, _ = paper8.level_dims(shape, L)
    off = int(sum(np.prod(d) for d in dims))
    taus = paper8.level_tolerances(tau1, shape, L)
    assert taus[-1].min() == pytest.approx(1e-5)
    assert np.all(delta[off:] <= 2 * 1e-5)
