"""Pins of the oracle's decomposition against mathematics, not against itself.

Each test checks the oracle against a fact the paper's definitions fix
(Sec. II-B, IV-A, IV-B): a hand-worked example, closed forms (Galerkin
identity, dense L2 projection, Dirichlet-constrained projection), invariants
(multilinear exactness, orthogonality, perfect reconstruction, face
agreement, block locality) and brute-force transposes.
"""
import json
import os

import numpy as np
import pytest

from oracle import mgard

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_coarsening_count_floor_half_plus_one():
    # Sec. II-B: n nodes coarsen to floor(n/2)+1 nodes
    for n in range(3, 70):
        assert len(mgard.coarse_indices(n)) == n // 2 + 1
        c = mgard.coarse_indices(n)
        assert c[0] == 0 and c[-1] == n - 1
    assert list(mgard.coarse_indices(2)) == [0, 1]


def test_paper_block_constants():
    # Sec. IV-A / IV-D: 8^3 block -> 5^3 coarse output, working set 1157
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    b = g["block_edge"]["value"]
    m = len(mgard.coarse_indices(b))
    assert m == g["block_coarse_edge"]["value"]
    ws = b ** 3 + m * b * b + m * m * b + m ** 3
    assert ws == g["working_set_elements"]["value"]
    assert round(ws * 4 / 1000, 2) == g["working_set_kb_fp32"]["value"]
    assert round(ws * 8 / 1000, 2) == g["working_set_kb_fp64"]["value"]
    assert m ** 3 == g["coarse_writer_threads"]["value"]
    assert b ** 3 - m ** 3 == g["detail_threads"]["value"]


@pytest.mark.parametrize("n", [8, 9, 17, 33, 65])
def test_galerkin_identity(n):
    # coarse mass matrix equals P^T M P (nested piecewise-linear spaces)
    x = np.arange(n, dtype=float)
    c = mgard.coarse_indices(n)
    P = mgard.prolongation(x, c)
    M = mgard.mass_matrix(x)
    Mc = mgard.mass_matrix(x[c])
    assert np.allclose(P.T @ M @ P, Mc, atol=1e-14)


@pytest.mark.parametrize("n", [5, 9, 17, 12])
def test_row_sums(n):
    x = np.cumsum(np.r_[0.0, np.linspace(0.5, 1.5, n - 1)])
    M = mgard.mass_matrix(x)
    h = np.diff(x)
    meas = np.r_[h, 0] / 2 + np.r_[0, h] / 2
    assert np.allclose(M.sum(axis=1), meas)          # M 1 = node measures
    ops = mgard.axis_ops(x, False)
    assert np.allclose(ops.K.sum(axis=1), 1.0)        # projection keeps constants
    assert np.allclose(ops.K @ ops.P, np.eye(len(ops.cidx)))  # K P = I


def test_hand_example_n3():
    rows = [l for l in open(os.path.join(GOLD, "hand_example_n3.txt")) if l.strip() and not l.startswith("#")]
    for line in rows:
        left, right = line.split("|")
        u = np.array([float(v) for v in left.split()])
        d, c0, c2 = (float(v) for v in right.split())
        out = mgard.level_decompose(u.reshape(1, 1, 3), [np.zeros(1), np.zeros(1), np.arange(3.0)], False)
        assert out[0, 0, 1] == pytest.approx(d, abs=1e-15)
        assert out[0, 0, 0] == pytest.approx(c0, abs=1e-15)
        assert out[0, 0, 2] == pytest.approx(c2, abs=1e-15)


def _multilinear(shape):
    z, y, x = np.meshgrid(*(np.arange(float(s)) for s in shape), indexing="ij")
    return 1.5 + 2 * x + 3 * y - z + 0.5 * x * y - 0.25 * y * z + 0.1 * x * z + 0.01 * x * y * z


@pytest.mark.parametrize("b,L,M", [(9, 1, 1), (17, 1, 2), (9, 2, 1), (9, 0, 3), (33, 1, 1)])
def test_multilinear_details_vanish(b, L, M):
    shape = {17: (33, 33, 33), 33: (65, 33, 65)}.get(b, (33, 17, 33))
    f = _multilinear(shape)
    c = mgard.decompose(f, b, L, M)
    lev = mgard.node_level(c.shape, L, M)
    scale = np.abs(f).max()
    assert np.abs(c[lev <= L + M]).max() < 1e-13 * scale
    # coarsest values equal the field at the coarsest nodes
    h = mgard.hierarchy(shape, b, L, M)
    g = np.ix_(*h.pos[h.levels])
    assert np.allclose(c[g], f[g], atol=1e-12 * scale)


def _kron3(a):
    return np.kron(np.kron(a[0], a[1]), a[2])


@pytest.mark.parametrize("shape", [(9, 9, 9), (5, 9, 17)])
def test_global_level_is_dense_l2_projection(shape, rng):
    u = rng.standard_normal(shape)
    coords = [np.arange(float(n)) for n in shape]
    out = mgard.level_decompose(u, coords, False)
    ops = [mgard.axis_ops(c, False) for c in coords]
    P3 = _kron3([o.P for o in ops])
    M3 = _kron3([mgard.mass_matrix(c) for c in coords])
    c_dense = np.linalg.solve(P3.T @ M3 @ P3, P3.T @ M3 @ u.ravel())
    cid = np.ix_(*(o.cidx for o in ops))
    assert np.allclose(out[cid].ravel(), c_dense, atol=1e-13)
    # orthogonality: P3^T M3 (u - P3 c) = 0
    r = P3.T @ M3 @ (u.ravel() - P3 @ out[cid].ravel())
    assert np.abs(r).max() < 1e-13
    # details: u - interpolant of u_C at fine-only nodes
    interp = (P3 @ u[cid].ravel()).reshape(shape)
    fine = np.ones(shape, bool)
    fine[cid] = False
    assert np.allclose(out[fine], (u - interp)[fine], atol=1e-14)


@pytest.mark.parametrize("b", [9, 17])
def test_block_level_is_dirichlet_constrained_projection(b, rng):
    # A single block (b = n) with face-fixed correction equals the L2 projection
    # whose coarse values on the block surface are held at the data.
    u = rng.standard_normal((b, b, b))
    coords = [np.arange(float(b))] * 3
    out = mgard.level_decompose(u, coords, True)
    o = mgard.axis_ops(coords[0], False)
    m = len(o.cidx)
    P3 = _kron3([o.P] * 3)
    M3 = _kron3([mgard.mass_matrix(coords[0])] * 3)
    A = P3.T @ M3 @ P3
    rhs = P3.T @ M3 @ u.ravel()
    ci = np.arange(m)
    inner1 = (ci > 0) & (ci < m - 1)
    inner = (inner1[:, None, None] & inner1[None, :, None] & inner1[None, None, :]).ravel()
    uc = u[np.ix_(o.cidx, o.cidx, o.cidx)].ravel()
    c = uc.copy()
    c[inner] = np.linalg.solve(A[np.ix_(inner, inner)], rhs[inner] - A[np.ix_(inner, ~inner)] @ uc[~inner])
    cid = np.ix_(o.cidx, o.cidx, o.cidx)
    assert np.allclose(out[cid].ravel(), c, atol=1e-12)


def test_block_level_33_is_dirichlet_constrained_projection(rng):
    # b = 33: the same constrained projection, with the tensor-product
    # operators applied axis by axis (the dense P3 would hold 35937 x 4913 entries)
    b = 33
    u = rng.standard_normal((b, b, b))
    coords = [np.arange(float(b))] * 3
    out = mgard.level_decompose(u, coords, True)
    o = mgard.axis_ops(coords[0], False)
    m = len(o.cidx)
    M1 = mgard.mass_matrix(coords[0])
    A1 = o.P.T @ M1 @ o.P
    A = _kron3([A1] * 3)
    R = o.P.T @ M1
    rhs = np.einsum("ai,bj,ck,ijk->abc", R, R, R, u, optimize=True).ravel()
    ci = np.arange(m)
    inner1 = (ci > 0) & (ci < m - 1)
    inner = (inner1[:, None, None] & inner1[None, :, None] & inner1[None, None, :]).ravel()
    uc = u[np.ix_(o.cidx, o.cidx, o.cidx)].ravel()
    c = uc.copy()
    c[inner] = np.linalg.solve(A[np.ix_(inner, inner)], rhs[inner] - A[np.ix_(inner, ~inner)] @ uc[~inner])
    cid = np.ix_(o.cidx, o.cidx, o.cidx)
    assert np.allclose(out[cid].ravel(), c, atol=1e-12)


@pytest.mark.parametrize("shape,b,L,M", [((33, 33, 33), 17, 1, 2), ((33, 17, 65), 9, 2, 1),
                                          ((9, 9, 9), 9, 0, 3), ((20, 30, 12), 9, 1, 1),
                                          ((65, 33, 33), 17, 1, 0), ((17, 17, 17), 9, 1, 1),
                                          ((70, 40, 100), 33, 1, 1), ((65, 65, 129), 33, 2, 1),
                                          ((1, 40, 70), 9, 1, 1), ((5, 2, 9), 9, 0, 2), ((3, 3, 3), 9, 0, 1)])
def test_reconstruction(shape, b, L, M, rng):
    x = rng.standard_normal(shape)
    c = mgard.decompose(x, b, L, M)
    h = mgard.hierarchy(shape, b, L, M)
    assert c.shape == h.shape_p                        # non-redundant: one value per node
    xr = mgard.recompose(c, shape, b, L, M)
    assert np.abs(xr - x).max() < 1e-12 * np.abs(x).max()


def test_zero_padding_reconstruction(rng):
    x = rng.standard_normal((20, 30, 12))
    c = mgard.decompose(x, 9, 1, 1, pad_mode="zero")
    xr = mgard.recompose(c, x.shape, 9, 1, 1)
    assert np.abs(xr - x).max() < 1e-12


def test_face_agreement_between_neighbours(rng):
    b = 9
    u = rng.standard_normal((b, b, 2 * b - 1))
    coords = [np.arange(float(b)), np.arange(float(b)), np.arange(2.0 * b - 1)]
    left = mgard.level_decompose(u[:, :, :b], [coords[0], coords[1], coords[2][:b]], True)
    right = mgard.level_decompose(u[:, :, b - 1:], [coords[0], coords[1], coords[2][b - 1:]], True)
    assert np.array_equal(left[:, :, b - 1], right[:, :, 0])


def test_block_locality(rng):
    b = 9
    shape = (17, 17, 17)
    x = rng.standard_normal(shape)
    coords = [np.arange(17.0)] * 3
    base = mgard.local_decompose(x, coords, b)
    j = (3, 11, 5)                     # interior of block (0, 1, 0)
    x2 = x.copy()
    x2[j] += 1.0
    diff = np.abs(mgard.local_decompose(x2, coords, b) - base) > 0
    touched = np.argwhere(diff)
    assert touched[:, 0].max() <= 8 and touched[:, 1].min() >= 8 and touched[:, 2].max() <= 8


def test_block_coarse_grid_is_global_coarse_grid():
    h = mgard.hierarchy((513, 513, 513), 17, 1, 2)
    assert [len(p) for p in h.pos[1]] == [257] * 3
    assert [len(p) for p in h.pos[3]] == [65] * 3
    lev = mgard.node_level((33, 33, 33), 1, 2)
    counts = [int((lev == s).sum()) for s in (1, 2, 3, 4)]
    assert counts == [33 ** 3 - 17 ** 3, 17 ** 3 - 9 ** 3, 9 ** 3 - 5 ** 3, 5 ** 3]


@pytest.mark.parametrize("n,b,L,M,expect", [(512, 17, 1, 2, 513), (65, 17, 0, 6, 65), (500, 9, 1, 2, 505),
                                            (100, 17, 1, 4, 129), (33, 17, 1, 5, 33), (512, 33, 1, 2, 513),
                                            (1000, 33, 1, 2, 1025), (70, 33, 1, 1, 97)])
def test_padding_rule(n, b, L, M, expect):
    assert mgard.padded_length(n, b, L, M) == expect


# --- transposes (adjoint), brute force -----------------------------------

def _dense(fn, nin):
    cols = []
    for i in range(nin):
        e = np.zeros(nin)
        e[i] = 1.0
        cols.append(fn(e).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("shape,b,L,M", [((9, 9, 9), 9, 1, 1), ((9, 5, 9), 5, 1, 1), ((7, 9, 5), 5, 1, 0)])
def test_dense_transpose(shape, b, L, M):
    h = mgard.hierarchy(shape, b, L, M)
    nin = int(np.prod(shape))
    nco = int(np.prod(h.shape_p))
    D = _dense(lambda e: mgard.decompose(e.reshape(shape), b, L, M), nin)
    DT = _dense(lambda g: mgard.decompose_adjoint(g.reshape(h.shape_p), shape, b, L, M), nco)
    assert np.allclose(DT, D.T, atol=1e-12)
    R = _dense(lambda c: mgard.recompose(c.reshape(h.shape_p), shape, b, L, M), nco)
    RT = _dense(lambda g: mgard.recompose_adjoint(g.reshape(shape), shape, b, L, M), nin)
    assert np.allclose(RT, R.T, atol=1e-12)
    assert np.allclose(R @ D, np.eye(nin), atol=1e-12)


@pytest.mark.parametrize("shape,b,L,M", [((33, 33, 33), 17, 1, 2), ((20, 30, 12), 9, 1, 1)])
def test_dot_product_adjoint(shape, b, L, M, rng):
    h = mgard.hierarchy(shape, b, L, M)
    x = rng.standard_normal(shape)
    g = rng.standard_normal(h.shape_p)
    lhs = np.vdot(mgard.decompose(x, b, L, M), g)
    rhs = np.vdot(x, mgard.decompose_adjoint(g, shape, b, L, M))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-10
    c = rng.standard_normal(h.shape_p)
    y = rng.standard_normal(shape)
    lhs = np.vdot(mgard.recompose(c, shape, b, L, M), y)
    rhs = np.vdot(c, mgard.recompose_adjoint(y, shape, b, L, M))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-10
