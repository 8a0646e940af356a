"""Pins of the oracle's nested block schedule (several block levels inside
one block region, Sec. IV-A), against an independent formulation.

In the nested schedule local level s uses blocks of (b-1)/2^(s-1)+1 nodes.
The oracle computes it by re-tiling each level grid with that block size;
the pins here compute it as a recursion inside every level-1 block region
(decompose the block, then decompose the block's own coarse values as one
block, and so on), and check the invariants of the method: exact
reconstruction, vanishing details of multilinear fields, the transposes,
the ROI propagation rule by brute force over node sets, and the L-infinity
bound.
"""
import numpy as np
import pytest

from oracle import mgard, roi


def _recursive_nested(x, b, L, M):
    """Nested decomposition as a recursion per level-1 block region."""
    h = mgard.hierarchy(x.shape, b, L, M, nested=True)
    u = mgard.pad(x, h.shape_p)
    coeff = np.zeros(h.shape_p)
    nb = [(n - 1) // (b - 1) for n in h.shape_p]
    # the coarse values left by the block levels, on the level-L+1 grid
    m = [(n - 1) // (1 << L) + 1 for n in h.shape_p]
    top = np.zeros(m)
    w = (b - 1) >> L
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                o = (bz * (b - 1), by * (b - 1), bx * (b - 1))
                cur = u[o[0]:o[0] + b, o[1]:o[1] + b, o[2]:o[2] + b]
                step = 1
                for s in range(1, L + 1):
                    n = cur.shape[0]
                    out = mgard.level_decompose(cur, [np.arange(float(n))] * 3, True)
                    idx = [o[a] + step * np.arange(n) for a in range(3)]
                    coeff[np.ix_(*idx)] = out
                    cur = out[::2, ::2, ::2]
                    step *= 2
                top[bz * w:bz * w + w + 1, by * w:by * w + w + 1, bx * w:bx * w + w + 1] = cur
    cur = top
    for s in range(L + 1, L + M + 1):
        coords = [p.astype(float) for p in h.pos[s - 1]]
        out = mgard.level_decompose(cur, coords, False)
        coeff[np.ix_(*h.pos[s - 1])] = out
        cur = out[np.ix_(*(mgard.coarse_indices(len(p)) for p in h.pos[s - 1]))]
    coeff[np.ix_(*h.pos[L + M])] = cur
    return coeff


@pytest.mark.parametrize("shape,b,L,M", [((17, 33, 17), 9, 2, 1), ((33, 17, 17), 17, 2, 0),
                                         ((20, 30, 12), 9, 3, 0), ((33, 33, 33), 17, 3, 1)])
def test_nested_equals_recursion_per_block(shape, b, L, M, rng):
    x = rng.standard_normal(shape)
    c = mgard.decompose(x, b, L, M, nested=True)
    r = _recursive_nested(x, b, L, M)
    assert c.shape == r.shape
    assert np.abs(c - r).max() < 1e-13 * np.abs(x).max()


def test_nested_one_level_is_the_plain_schedule(rng):
    x = rng.standard_normal((33, 17, 33))
    assert np.array_equal(mgard.decompose(x, 9, 1, 2, nested=True), mgard.decompose(x, 9, 1, 2))


def test_nested_second_level_differs_from_retiling(rng):
    x = rng.standard_normal((33, 33, 33))
    a = mgard.decompose(x, 9, 2, 1, nested=True)
    b = mgard.decompose(x, 9, 2, 1)
    lev = mgard.node_level(a.shape, 2, 1)
    # level 1 is the same, and so are the level-2 details (interpolation only);
    # the level-2 correction, hence every coarser value, depends on the blocks
    assert np.array_equal(a[lev <= 2], b[lev <= 2])
    assert np.abs(a[lev > 2] - b[lev > 2]).max() > 1e-3


@pytest.mark.parametrize("n,b,L,M,expect", [(40, 17, 2, 0, 49), (512, 17, 2, 1, 513), (20, 9, 3, 0, 25),
                                            (100, 33, 2, 1, 129)])
def test_nested_padding_rule(n, b, L, M, expect):
    # blocks of the first level tile the grid; deeper levels tile the same regions
    assert mgard.padded_length(n, b, L, M, nested=True) == expect


def test_nested_schedule_needs_an_interior_row():
    assert mgard.hierarchy((33, 33, 33), 9, 3, 0, nested=True).block(3) == 3   # 9 -> 5 -> 3
    with pytest.raises(ValueError):
        mgard.hierarchy((33, 33, 33), 9, 4, 0, nested=True)                    # 9 -> 5 -> 3 -> 2


def _multilinear(shape):
    z, y, x = np.meshgrid(*(np.arange(float(n)) for n in shape), indexing="ij")
    return 0.5 + x - 2 * y + 0.25 * z + 0.1 * x * y - 0.05 * y * z + 0.02 * x * z + 0.003 * x * y * z


@pytest.mark.parametrize("shape,b,L,M", [((33, 33, 33), 17, 2, 1), ((17, 33, 17), 9, 3, 1)])
def test_nested_multilinear_details_vanish(shape, b, L, M):
    f = _multilinear(shape)
    c = mgard.decompose(f, b, L, M, nested=True)
    lev = mgard.node_level(c.shape, L, M)
    assert np.abs(c[lev <= L + M]).max() < 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("shape,b,L,M", [((33, 33, 33), 17, 2, 1), ((20, 30, 12), 9, 2, 1), ((65, 33, 33), 33, 2, 1)])
def test_nested_reconstruction_and_transposes(shape, b, L, M, rng):
    h = mgard.hierarchy(shape, b, L, M, nested=True)
    x = rng.standard_normal(shape)
    c = mgard.decompose(x, b, L, M, nested=True)
    assert np.abs(mgard.recompose(c, shape, b, L, M, nested=True) - x).max() < 1e-12 * np.abs(x).max()
    g = rng.standard_normal(h.shape_p)
    lhs = np.vdot(c, g)
    rhs = np.vdot(x, mgard.decompose_adjoint(g, shape, b, L, M, nested=True))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-10
    y = rng.standard_normal(shape)
    lhs = np.vdot(mgard.recompose(g, shape, b, L, M, nested=True), y)
    rhs = np.vdot(g, mgard.recompose_adjoint(y, shape, b, L, M, nested=True))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-10


def _block_nodes(bidx, width):
    """Padded-grid node ranges (inclusive) of a block with `width` cells per side."""
    return [(i * width, (i + 1) * width) for i in bidx]


@pytest.mark.parametrize("nested", [False, True])
def test_propagation_rule_by_node_sets(nested, rng):
    # Eq. 2 by brute force: a next-level block takes the min over the blocks
    # of this level whose node sets (in padded coordinates) meet its own.
    b, nb = 9, (4, 6, 5)
    tol = rng.uniform(1e-4, 1e-2, nb)
    w0 = b - 1                                   # cells of a level-s block (padded units)
    w1 = w0 if nested else 2 * w0                # cells of a level-(s+1) block
    nn = nb if nested else tuple(max(1, n // 2) for n in nb)
    want = np.empty(nn)
    for I in np.ndindex(*nn):
        r1 = _block_nodes(I, w1)
        best = np.inf
        for J in np.ndindex(*nb):
            r0 = _block_nodes(J, w0)
            if all(lo0 <= hi1 and lo1 <= hi0 for (lo0, hi0), (lo1, hi1) in zip(r0, r1)):
                best = min(best, tol[J])
        want[I] = best
    assert np.array_equal(roi.propagate(tol, nested), want)


NESTED_CASES = [((33, 33, 33), 9, 2, 1, [(20, 20, 20, 26, 30, 25, 1e-5)], 1e-2),
                ((33, 17, 33), 9, 3, 0, [(0, 0, 0, 5, 5, 5, 1e-4)], 1e-1),
                ((33, 33, 33), 17, 2, 1, [(9, 9, 9, 12, 12, 12, 1e-5)], 1e-3)]


@pytest.mark.parametrize("shape,b,L,M,boxes,bg", NESTED_CASES)
def test_nested_bound_holds(shape, b, L, M, boxes, bg, rng):
    x = rng.standard_normal(shape)
    h = mgard.hierarchy(shape, b, L, M, nested=True)
    vt = roi.voxel_tolerance_from_boxes(shape, boxes, bg)
    tol1 = roi.block_tolerance(vt, h.shape_p, b)
    delta = roi.node_delta(h, tol1, 0.0)
    c = mgard.decompose(x, b, L, M, nested=True)
    xr = mgard.recompose(roi.dequantize(roi.quantize(c, delta), delta), shape, b, L, M, nested=True)
    assert np.all(np.abs(xr - x) <= vt)
    # worst case: every coefficient off by Delta/2 with the sign of the row
    strict = np.argwhere(vt == vt.min())
    for t in (tuple(strict[0]), tuple(strict[-1]), (0, 0, 0), tuple(s - 1 for s in shape)):
        e = np.zeros(shape)
        e[t] = 1.0
        row = mgard.recompose_adjoint(e, shape, b, L, M, nested=True)
        assert float(np.sum(np.abs(row) * delta / 2)) <= vt[t] * (1 + 1e-12)
