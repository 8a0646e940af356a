"""Oracle: MGARD multilevel decomposition, In-cache Block levels, hybrid hierarchy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain FP64 NumPy; every
operator is a dense matrix built from node coordinates, applied one axis at a
time.  Nothing here is blocked, fused or reordered beyond what the method
states.

Paper passages followed
-----------------------
* Sec. II-B: nested grids G_0 < ... < G_l, a dimension of n nodes coarsens to
  floor(n/2)+1 nodes; each level interpolates coarse -> fine and subtracts
  (multilevel coefficients on the nodes the coarse grid lacks), then corrects
  the coarse values with a mass-matrix solve so the level is an L2 projection;
  multi-D work is a sequence of 1D passes that shrink the array; the
  decomposition is exactly invertible.
* Sec. IV-A: In-cache Block levels; each block is decomposed on its own, the
  working set is the input block plus three shrinking restriction arrays.
* Sec. IV-B: hybrid hierarchy, L local (block) levels then M global levels.
* Sec. IV-D: out-of-range reads of the block kernel are zero-filled (kept as
  the ``pad_mode="zero"`` option; clamp is the default reading).

Readings where the paper is silent
----------------------------------
* Details use the tensor (multilinear) interpolant; the correction is the
  tensor L2 projection computed as restriction passes x, y, z followed by
  tridiagonal solves x, y, z.
* Blocks have 2^k+1 nodes per side and share one face with each neighbour.
  Inside a block the correction rows of the two end coarse nodes of every
  axis are zero and the interior rows solve with the coarse mass matrix
  restricted to interior coarse nodes ("face-fixed").  Face values are then
  functions of face data only, so both neighbours agree and every node of
  the grid stores exactly one coefficient.
* Each local level re-tiles the current grid with b^3 blocks.  A second,
  "nested" schedule is kept as a defined variant (several block levels in
  one on-chip block, Sec. IV-A): local level s uses blocks of
  (b-1)/2^(s-1)+1 nodes, which tile the level-s grid over exactly the
  regions of the level-1 blocks, so every block level of a region works on
  that region's own coarse values.  Its results differ from re-tiling from
  the second block level on.
* Coefficient layout is "in place": one dense array of the padded grid,
  each node holding its own coefficient (detail of the level at which it
  leaves the grid, or the coarsest value).
* Padding per axis: the smallest n' >= n such that every local level tiles
  exactly with b-blocks and every global level halves an odd length (or
  leaves a length <= 2 untouched).  Padded nodes copy the nearest real node
  (clamp) or are zero.

Array convention: 3D arrays are C-order ``[z, y, x]``; "x, y, z" passes
therefore act on axes 2, 1, 0.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# O1 / O2: 1D grids and operators (Sec. II-B)
# --------------------------------------------------------------------------


def coarse_indices(n: int) -> np.ndarray:
    """Indices of the coarse nodes of an n-node axis (Sec. II-B).

    The even indices plus the last node, i.e. floor(n/2)+1 nodes.  An axis
    with n <= 2 is not coarsened any further: all of its nodes stay.
    """
    if n <= 2:
        return np.arange(n)
    idx = list(range(0, n, 2))
    if idx[-1] != n - 1:
        idx.append(n - 1)
    return np.asarray(idx, dtype=np.int64)


def mass_matrix(coords: np.ndarray) -> np.ndarray:
    """Piecewise-linear finite-element mass matrix on 1D nodes ``coords``.

    Diagonal (h_{i-1} + h_i)/3, off-diagonal h_i/6 (exact integrals of products
    of hat functions).
    """
    n = len(coords)
    M = np.zeros((n, n))
    for i in range(n - 1):
        h = float(coords[i + 1] - coords[i])
        M[i, i] += h / 3.0
        M[i + 1, i + 1] += h / 3.0
        M[i, i + 1] += h / 6.0
        M[i + 1, i] += h / 6.0
    return M


def prolongation(coords: np.ndarray, cidx: np.ndarray) -> np.ndarray:
    """Linear interpolation from the coarse nodes ``coords[cidx]`` to all nodes.

    Column J is the coarse hat function of coarse node J evaluated at every
    fine node.
    """
    n, m = len(coords), len(cidx)
    P = np.zeros((n, m))
    cc = coords[cidx]
    for i in range(n):
        x = coords[i]
        j = int(np.searchsorted(cc, x, side="right")) - 1
        if j >= m - 1:
            P[i, m - 1] = 1.0
            continue
        if cc[j] == x:
            P[i, j] = 1.0
            continue
        t = (x - cc[j]) / (cc[j + 1] - cc[j])
        P[i, j] = 1.0 - t
        P[i, j + 1] = t
    return P


@dataclass
class AxisOps:
    """The 1D pieces of one level along one axis.

    ``P``  (n x m) interpolation, ``R`` (rows x n) load-vector operator
    P^T M (only the rows that are solved for), ``Mc`` (rows x rows) the coarse
    mass matrix on those rows, ``rows`` their coarse indices, ``cidx`` the
    coarse nodes.  ``K`` (m x n) is the full correction operator with zero rows
    outside ``rows``.
    """

    n: int
    cidx: np.ndarray
    P: np.ndarray
    R: np.ndarray
    Mc: np.ndarray
    rows: np.ndarray
    K: np.ndarray


def axis_ops(coords: np.ndarray, face_fixed: bool) -> AxisOps:
    """Operators of one level along one axis (Sec. II-B; face rule of Sec. IV-A reading).

    Natural (global) level: K = Mc^{-1} P^T M on all coarse rows.  Face-fixed
    (block) level: the rows of the two end coarse nodes are dropped (their
    correction is zero) and the interior rows use Mc restricted to the
    interior coarse nodes.  An axis of <= 2 nodes is left untouched (identity).
    """
    coords = np.asarray(coords, dtype=np.float64)
    n = len(coords)
    cidx = coarse_indices(n)
    m = len(cidx)
    if n <= 2:
        eye = np.eye(n)
        return AxisOps(n, cidx, eye, np.zeros((0, n)), np.zeros((0, 0)), np.zeros(0, np.int64), eye.copy())
    P = prolongation(coords, cidx)
    M = mass_matrix(coords)
    Mc_full = mass_matrix(coords[cidx])
    PtM = P.T @ M
    if face_fixed:
        rows = np.arange(1, m - 1)
    else:
        rows = np.arange(m)
    R = PtM[rows, :]
    Mc = Mc_full[np.ix_(rows, rows)]
    K = np.zeros((m, n))
    if len(rows):
        K[rows, :] = np.linalg.solve(Mc, R)
    return AxisOps(n, cidx, P, R, Mc, rows, K)


# --------------------------------------------------------------------------
# helpers: apply a matrix / a solve along one axis of a 3D array
# --------------------------------------------------------------------------


def apply_along(A: np.ndarray, arr: np.ndarray, axis: int) -> np.ndarray:
    """Return A applied to every line of ``arr`` along ``axis``."""
    out = np.tensordot(A, arr, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def solve_along(Mc: np.ndarray, arr: np.ndarray, axis: int) -> np.ndarray:
    """Solve Mc y = line for every line of ``arr`` along ``axis``."""
    if Mc.shape[0] == 0:
        return arr
    moved = np.moveaxis(arr, axis, 0)
    shp = moved.shape
    sol = np.linalg.solve(Mc, moved.reshape(shp[0], -1)).reshape(shp)
    return np.moveaxis(sol, 0, axis)


# --------------------------------------------------------------------------
# O3 / O4: one level (Sec. II-B; Sec. IV-A for face-fixed blocks)
# --------------------------------------------------------------------------

X, Y, Z = 2, 1, 0  # axis numbers of the x, y, z passes


def _ops3(coords3, face_fixed):
    return [axis_ops(c, face_fixed) for c in coords3]


def _interp3(ops, uC):
    t = uC
    for ax in (X, Y, Z):
        t = apply_along(ops[ax].P, t, ax)
    return t


def _correction3(ops, w):
    """z = Mc^{-1} P^T M w along x, y, z; rows outside ``rows`` are zero.

    Step order follows Sec. II-B: three shrinking restriction passes (x, then
    y, then z) then the tridiagonal solves (x, then y, then z).
    """
    f = w
    for ax in (X, Y, Z):
        if ops[ax].n > 2:
            f = apply_along(ops[ax].R, f, ax)
    for ax in (X, Y, Z):
        if ops[ax].n > 2:
            f = solve_along(ops[ax].Mc, f, ax)
    # embed the solved rows into the full coarse grid (zeros elsewhere)
    full_shape = tuple(len(o.cidx) for o in ops)
    z = np.zeros(full_shape)
    sel = tuple(o.rows if o.n > 2 else np.arange(o.n) for o in ops)
    z[np.ix_(*sel)] = f
    return z


def level_decompose(u: np.ndarray, coords3: Sequence[np.ndarray], face_fixed: bool) -> np.ndarray:
    """One decomposition level on a grid (Sec. II-B), returned "in place".

    1. u_C = u on the coarse nodes;
    2. w = u - (multilinear interpolant of u_C); w is zero on the coarse nodes
       and holds the multilevel coefficients elsewhere;
    3. f = (P^T M)_x (P^T M)_y (P^T M)_z w (shrinking passes);
    4. z = Mc^{-1} f along x, y, z;
    5. coarse value c = u_C + z.
    The result has w on the fine-only nodes and c on the coarse nodes.
    """
    ops = _ops3(coords3, face_fixed)
    cid = np.ix_(*(o.cidx for o in ops))
    uC = u[cid]
    w = u - _interp3(ops, uC)
    z = _correction3(ops, w)
    out = w.copy()
    out[cid] = uC + z
    return out


def level_recompose(out: np.ndarray, coords3: Sequence[np.ndarray], face_fixed: bool) -> np.ndarray:
    """Inverse of :func:`level_decompose` (Sec. II-B: reverse the operations).

    w = the coefficients with the coarse nodes zeroed, z from w exactly as in
    decomposition, u_C = c - z, u = interpolant(u_C) + w.
    """
    ops = _ops3(coords3, face_fixed)
    cid = np.ix_(*(o.cidx for o in ops))
    c = out[cid]
    w = out.copy()
    w[cid] = 0.0
    z = _correction3(ops, w)
    uC = c - z
    return _interp3(ops, uC) + w


# --------------------------------------------------------------------------
# O4: In-cache Block level on shared-face blocks (Sec. IV-A)
# --------------------------------------------------------------------------


def block_counts(shape: Sequence[int], b: int) -> Tuple[int, int, int]:
    for n in shape:
        if (n - 1) % (b - 1) != 0 or n < b:
            raise ValueError(f"grid {tuple(shape)} does not tile with {b}-node blocks")
    return tuple((n - 1) // (b - 1) for n in shape)


def _block_slices(bidx, b):
    return tuple(slice(i * (b - 1), i * (b - 1) + b) for i in bidx)


def local_decompose(u: np.ndarray, coords3, b: int) -> np.ndarray:
    """In-cache Block level: every b^3 block decomposed on its own (face-fixed).

    Neighbouring blocks share a face; both compute identical face values, so
    writing every block into one array is well defined.
    """
    nb = block_counts(u.shape, b)
    out = np.empty_like(u)
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                sl = _block_slices((bz, by, bx), b)
                cs = [coords3[a][sl[a]] for a in range(3)]
                out[sl] = level_decompose(u[sl], cs, True)
    return out


def local_recompose(out: np.ndarray, coords3, b: int) -> np.ndarray:
    """Inverse of :func:`local_decompose`, block by block."""
    nb = block_counts(out.shape, b)
    u = np.empty_like(out)
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                sl = _block_slices((bz, by, bx), b)
                cs = [coords3[a][sl[a]] for a in range(3)]
                u[sl] = level_recompose(out[sl], cs, True)
    return u


# --------------------------------------------------------------------------
# O5 / O6: padding and the hybrid hierarchy (Sec. IV-B)
# --------------------------------------------------------------------------


def _global_chain_ok(n: int, M: int) -> bool:
    for _ in range(M):
        if n <= 2:
            continue
        if n % 2 == 0:
            return False
        n = (n + 1) // 2
    return True


def level_block(b: int, s: int, nested: bool) -> int:
    """Block size (nodes per side) of local level s: b when every level
    re-tiles its grid, (b-1)/2^(s-1)+1 in the nested schedule."""
    if not nested:
        return b
    w = (b - 1) >> (s - 1)
    if w < 2 or w << (s - 1) != b - 1:
        raise ValueError(f"nested schedule: level {s} of {b}-node blocks has no interior coarse row")
    return w + 1


def padded_length(n: int, b: int, L: int, M: int, nested: bool = False) -> int:
    """Smallest n' >= n on which the L block levels tile and the M global levels halve."""
    if n < 1:
        raise ValueError("empty axis")
    if nested and L > 0:
        level_block(b, L, True)   # validates the schedule
    q = ((b - 1) if nested else (b - 1) * (1 << (L - 1))) if L > 0 else 1
    cand = max(n, (b if L > 0 else 1))
    while True:
        if (cand - 1) % q == 0:
            nl = (cand - 1) // (1 << L) + 1 if L > 0 else cand
            if L == 0 or all(((cand - 1) >> (s - 1)) >= level_block(b, s, nested) - 1 for s in range(1, L + 1)):
                if _global_chain_ok(nl, M):
                    return cand
        cand += 1


def pad(x: np.ndarray, shape_p: Sequence[int], mode: str = "clamp") -> np.ndarray:
    """Extend ``x`` to ``shape_p``: clamp copies the nearest real node, zero fills 0."""
    if mode == "zero":
        xp = np.zeros(shape_p)
        xp[: x.shape[0], : x.shape[1], : x.shape[2]] = x
        return xp
    idx = [np.minimum(np.arange(p), n - 1) for p, n in zip(shape_p, x.shape)]
    return np.asarray(x, dtype=np.float64)[np.ix_(*idx)]


@dataclass
class Hierarchy:
    """Grid bookkeeping of a hybrid hierarchy (Sec. IV-B)."""

    shape: Tuple[int, int, int]          # logical (unpadded) dims
    shape_p: Tuple[int, int, int]        # padded dims
    b: int
    L: int
    M: int
    pos: List[List[np.ndarray]]          # pos[s][axis]: indices of grid G^s in the padded grid
    nested: bool = False                 # nested block schedule (see level_block)

    @property
    def levels(self) -> int:
        return self.L + self.M

    def block(self, s: int) -> int:
        """Block size of local level s (1-based)."""
        return level_block(self.b, s, self.nested)


def hierarchy(shape: Sequence[int], b: int, L: int, M: int, nested: bool = False) -> Hierarchy:
    shape = tuple(int(n) for n in shape)
    if len(shape) != 3:
        raise ValueError("3D grids only")
    if L > 0 and (b < 3 or (b - 1) & (b - 2) != 0):
        raise ValueError("block size must be 2^k+1")
    shape_p = tuple(padded_length(n, b, L, M, nested) for n in shape)
    pos = [[np.arange(n) for n in shape_p]]
    for _ in range(L + M):
        prev = pos[-1]
        pos.append([p[coarse_indices(len(p))] for p in prev])
    return Hierarchy(shape, shape_p, b, L, M, pos, nested)


def decompose(x: np.ndarray, b: int, L: int, M: int, pad_mode: str = "clamp", nested: bool = False) -> np.ndarray:
    """Full hybrid decomposition: L block levels then M global levels (Sec. IV-B).

    Returns the in-place coefficient array on the padded grid.
    """
    h = hierarchy(x.shape, b, L, M, nested)
    cur = pad(np.asarray(x, np.float64), h.shape_p, pad_mode)
    coeff = np.zeros(h.shape_p)
    for s in range(1, h.levels + 1):
        coords = [p.astype(np.float64) for p in h.pos[s - 1]]
        if s <= L:
            out = local_decompose(cur, coords, h.block(s))
        else:
            out = level_decompose(cur, coords, False)
        coeff[np.ix_(*h.pos[s - 1])] = out
        cur = out[np.ix_(*(coarse_indices(len(p)) for p in h.pos[s - 1]))]
    return coeff


def recompose(coeff: np.ndarray, shape: Sequence[int], b: int, L: int, M: int, nested: bool = False) -> np.ndarray:
    """Inverse of :func:`decompose`, cropped back to the logical ``shape``."""
    h = hierarchy(shape, b, L, M, nested)
    if tuple(coeff.shape) != h.shape_p:
        raise ValueError("coefficient array has the wrong shape")
    cur = coeff[np.ix_(*h.pos[h.levels])].astype(np.float64)
    for s in range(h.levels, 0, -1):
        coords = [p.astype(np.float64) for p in h.pos[s - 1]]
        out = coeff[np.ix_(*h.pos[s - 1])].astype(np.float64)
        out[np.ix_(*(coarse_indices(len(p)) for p in h.pos[s - 1]))] = cur
        if s <= L:
            cur = local_recompose(out, coords, h.block(s))
        else:
            cur = level_recompose(out, coords, False)
    n = h.shape
    return cur[: n[0], : n[1], : n[2]]


def node_level(shape_p: Sequence[int], L: int, M: int) -> np.ndarray:
    """Level of every node of the padded grid: s in 1..L+M for a detail of level s,
    L+M+1 for a coarsest value."""
    lev = np.full(tuple(shape_p), L + M + 1, dtype=np.int32)
    pos = [np.arange(n) for n in shape_p]
    for s in range(1, L + M + 1):
        inner = [p[coarse_indices(len(p))] for p in pos]
        grid = np.zeros(tuple(shape_p), bool)
        grid[np.ix_(*pos)] = True
        coarse = np.zeros(tuple(shape_p), bool)
        coarse[np.ix_(*inner)] = True
        lev[grid & ~coarse] = s
        pos = inner
    return lev


# --------------------------------------------------------------------------
# O12: transposes (adjoints) of decompose and recompose
# --------------------------------------------------------------------------


def _level_decompose_T(g: np.ndarray, coords3, face_fixed: bool) -> np.ndarray:
    """Transpose of one level map u -> out.

    out = (I - P3 S) u + S^T S u + S^T K3 (I - P3 S) u, with S the coarse
    selection and K3 the correction operator, so
    out^T g = (I - S^T P3^T)(g + K3^T S g) + S^T S g.
    """
    ops = _ops3(coords3, face_fixed)
    cid = np.ix_(*(o.cidx for o in ops))
    cbar = g[cid]
    t = cbar
    for ax in (X, Y, Z):
        t = apply_along(ops[ax].K.T, t, ax)
    v = g + t
    Ptv = v
    for ax in (X, Y, Z):
        Ptv = apply_along(ops[ax].P.T, Ptv, ax)
    res = v.copy()
    res[cid] -= Ptv
    res[cid] += cbar
    return res


def _level_recompose_T(g: np.ndarray, coords3, face_fixed: bool) -> np.ndarray:
    """Transpose of one recomposition map out -> u.

    u = P3 (S - K3 (I - S^T S)) out + (I - S^T S) out, so with v = P3^T g the
    transpose is: v on the coarse nodes, g - (K3^T v) on the fine-only nodes.
    """
    ops = _ops3(coords3, face_fixed)
    cid = np.ix_(*(o.cidx for o in ops))
    v = g
    for ax in (X, Y, Z):
        v = apply_along(ops[ax].P.T, v, ax)
    t = v
    for ax in (X, Y, Z):
        t = apply_along(ops[ax].K.T, t, ax)
    res = g - t
    res[cid] = v
    return res


def _owner_mask(shape, b, bidx):
    """Nodes of block ``bidx`` that the block owns: a shared face belongs to the
    block that starts on it; the far boundary face belongs to the last block."""
    nb = block_counts(shape, b)
    masks = []
    for a in range(3):
        lo = bidx[a] * (b - 1)
        hi = lo + b - 1 if bidx[a] == nb[a] - 1 else lo + b - 2
        mk = np.zeros(b, bool)
        mk[: hi - lo + 1] = True
        masks.append(mk)
    return masks[0][:, None, None] & masks[1][None, :, None] & masks[2][None, None, :]


def _local_T(g: np.ndarray, coords3, b: int, level_T) -> np.ndarray:
    nb = block_counts(g.shape, b)
    res = np.zeros_like(g)
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                sl = _block_slices((bz, by, bx), b)
                cs = [coords3[a][sl[a]] for a in range(3)]
                gb = np.where(_owner_mask(g.shape, b, (bz, by, bx)), g[sl], 0.0)
                res[sl] += level_T(gb, cs, True)
    return res


def decompose_adjoint(gcoeff: np.ndarray, shape: Sequence[int], b: int, L: int, M: int,
                      pad_mode: str = "clamp", nested: bool = False) -> np.ndarray:
    """D^T: gradient with respect to x of <decompose(x), gcoeff>.

    Levels run in reverse order; the transpose of clamp padding adds every
    padded node's gradient into the node it copied.
    """
    h = hierarchy(shape, b, L, M, nested)
    gcoeff = np.asarray(gcoeff, np.float64)
    # gradient with respect to the coarsest grid
    gcur = gcoeff[np.ix_(*h.pos[h.levels])]
    for s in range(h.levels, 0, -1):
        coords = [p.astype(np.float64) for p in h.pos[s - 1]]
        gout = gcoeff[np.ix_(*h.pos[s - 1])].copy()
        gout[np.ix_(*(coarse_indices(len(p)) for p in h.pos[s - 1]))] = gcur
        if s <= L:
            gcur = _local_T(gout, coords, h.block(s), _level_decompose_T)
        else:
            gcur = _level_decompose_T(gout, coords, False)
    # transpose of padding
    n = h.shape
    gx = np.zeros(n)
    if pad_mode == "zero":
        return gcur[: n[0], : n[1], : n[2]].copy()
    iz, iy, ix = [np.minimum(np.arange(p), q - 1) for p, q in zip(h.shape_p, n)]
    np.add.at(gx, np.ix_(iz, iy, ix), gcur)
    return gx


def recompose_adjoint(gx: np.ndarray, shape: Sequence[int], b: int, L: int, M: int,
                      nested: bool = False) -> np.ndarray:
    """R^T: gradient with respect to the coefficients of <recompose(c), gx>."""
    h = hierarchy(shape, b, L, M, nested)
    gcur = np.zeros(h.shape_p)
    n = h.shape
    gcur[: n[0], : n[1], : n[2]] = gx
    gcoeff = np.zeros(h.shape_p)
    for s in range(1, h.levels + 1):
        coords = [p.astype(np.float64) for p in h.pos[s - 1]]
        if s <= L:
            gout = _local_T(gcur, coords, h.block(s), _level_recompose_T)
        else:
            gout = _level_recompose_T(gcur, coords, False)
        gcoeff[np.ix_(*h.pos[s - 1])] = gout
        gcur = gout[np.ix_(*(coarse_indices(len(p)) for p in h.pos[s - 1]))]
    return gcoeff
