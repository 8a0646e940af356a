"""Oracle: the paper's own In-cache Block form with disjoint 8^3 blocks.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain FP64 NumPy.

Paper passages followed
-----------------------
* Sec. IV-A, Block Size Selection: blocks of 8 x 8 x 8 nodes; the
  dimensional passes shrink the working array 8^3 -> 5x8x8 -> 5x5x8 -> 5^3,
  so an axis of 8 nodes keeps 5 coarse nodes (floor(8/2)+1, Sec. II-B:
  the even indices and the last node, 0 2 4 6 7).
* Sec. IV-C (ROI propagation): the 5^3 coarse outputs of a level's blocks
  are assembled side by side into new 8^3 blocks for the next level, so a
  next-level block can take coarse values of several blocks.
* Sec. IV-D: out-of-range positions are zero-filled.

Readings where the paper is silent
----------------------------------
* Each block is one MGARD level (Sec. II-B) on its own 8 nodes per axis
  with natural ends (the blocks are disjoint, so no face is shared and none
  is held fixed): details on the 387 fine nodes, coarse values
  u_C + Mc^{-1} P^T M w on the 125 coarse nodes.  Node coordinates are the
  block-local indices 0..7 at every level (the operators are the same
  compile-time constants for every block).
* Grid of level s: n_1 = the input dims rounded up to a multiple of 8
  (zero fill); the level's nb = n_s / 8 blocks per axis leave 5 nb coarse
  values per axis, side by side in block order; rounded up to a multiple
  of 8 with zeros they are the next level's grid.  The last level's
  5 nb_L coarse values per axis are the coarsest values (not padded).
* Coefficient layout: the level arrays (dims n_s, the details at the fine
  nodes, 0 at the coarse nodes, whose values live in the next grid), one
  after the other in C order, then the coarsest array.
* Only block levels (no global levels after them).
* ROI bounds (Sec. IV-C): a level-1 block takes the smallest voxel
  tolerance over its real nodes; Eq. 2 on the assembled grids (Fig. 6):
  block I of level s+1 takes the smallest tau over the level-s blocks whose
  5^3 outputs land in it.  Details of level s get half-width
  tau (1-eta) w_s / A with A the rounded-up L-inf gain of the natural
  8-node level and w_s the level's share, the coarsest values
  tau (1-eta) w_c with tau of the block they came from; shares are
  proportional to the number of detail / coarsest coefficients, floored at
  1/(64 T), T = L+1, and renormalised (the rule of the shared-face form).
  Coarsest errors reach the fine nodes through interpolation only (gain 1),
  a level's detail errors with gain A, so every node keeps its bound.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import mgard, roi

B = 8
MC = 5
COARSE = mgard.coarse_indices(B)          # 0 2 4 6 7


def level_dims(shape: Sequence[int], L: int) -> Tuple[List[Tuple[int, int, int]], Tuple[int, int, int]]:
    """Grid dims of levels 1..L (multiples of 8) and of the coarsest array."""
    if len(shape) != 3 or L < 1:
        raise ValueError("3D shape and L >= 1")
    dims = []
    n = tuple(-(-int(d) // B) * B for d in shape)
    for _ in range(L):
        dims.append(n)
        m = tuple(MC * (d // B) for d in n)
        n = tuple(-(-d // B) * B for d in m)
    return dims, m


def coeff_size(shape: Sequence[int], L: int) -> int:
    dims, last = level_dims(shape, L)
    return int(sum(np.prod(d) for d in dims) + np.prod(last))


def _block_level(u: np.ndarray) -> np.ndarray:
    """One MGARD level on one 8^3 block, natural ends, local coordinates 0..7."""
    return mgard.level_decompose(u, [np.arange(float(B))] * 3, False)


def _block_level_inverse(out: np.ndarray) -> np.ndarray:
    return mgard.level_recompose(out, [np.arange(float(B))] * 3, False)


def decompose(x: np.ndarray, L: int) -> np.ndarray:
    """Flat coefficient array (layout above) of x (FP64)."""
    x = np.asarray(x, np.float64)
    dims, last = level_dims(x.shape, L)
    cur = np.zeros(dims[0])
    cur[: x.shape[0], : x.shape[1], : x.shape[2]] = x
    parts = []
    for s in range(L):
        n = dims[s]
        nb = [d // B for d in n]
        lev = np.zeros(n)
        nxt = np.zeros(dims[s + 1] if s + 1 < L else last)
        for bz in range(nb[0]):
            for by in range(nb[1]):
                for bx in range(nb[2]):
                    sl = (slice(B * bz, B * bz + B), slice(B * by, B * by + B), slice(B * bx, B * bx + B))
                    out = _block_level(cur[sl])
                    c = out[np.ix_(COARSE, COARSE, COARSE)]
                    out[np.ix_(COARSE, COARSE, COARSE)] = 0.0
                    lev[sl] = out
                    nxt[MC * bz: MC * bz + MC, MC * by: MC * by + MC, MC * bx: MC * bx + MC] = c
        parts.append(lev.ravel())
        cur = nxt
    parts.append(cur.ravel())
    return np.concatenate(parts)


def recompose(coeff: np.ndarray, shape: Sequence[int], L: int) -> np.ndarray:
    """Inverse of :func:`decompose`, cropped to ``shape``."""
    dims, last = level_dims(shape, L)
    coeff = np.asarray(coeff, np.float64)
    if coeff.size != coeff_size(shape, L):
        raise ValueError("coefficient array has the wrong size")
    offs = np.cumsum([0] + [int(np.prod(d)) for d in dims])
    cur = coeff[offs[L]:].reshape(last)
    for s in range(L - 1, -1, -1):
        n = dims[s]
        nb = [d // B for d in n]
        lev = coeff[offs[s]:offs[s + 1]].reshape(n)
        out = np.zeros(n)
        for bz in range(nb[0]):
            for by in range(nb[1]):
                for bx in range(nb[2]):
                    sl = (slice(B * bz, B * bz + B), slice(B * by, B * by + B), slice(B * bx, B * bx + B))
                    blk = lev[sl].copy()
                    blk[np.ix_(COARSE, COARSE, COARSE)] = cur[MC * bz: MC * bz + MC, MC * by: MC * by + MC,
                                                              MC * bx: MC * bx + MC]
                    out[sl] = _block_level_inverse(blk)
        cur = out
    return cur[: shape[0], : shape[1], : shape[2]]


def working_set() -> int:
    """Elements of a block's working set: input, then the three shrinking passes."""
    return B ** 3 + MC * B * B + MC * MC * B + MC ** 3


# --------------------------------------------------------------------------
# ROI quantization of this form (Sec. IV-C, IV-D)
# --------------------------------------------------------------------------


def block_tolerance(voxel_tol: np.ndarray, L: int) -> np.ndarray:
    """Level-1 block map: the smallest voxel tolerance over a block's real nodes."""
    dims, _ = level_dims(voxel_tol.shape, L)
    nb = [d // B for d in dims[0]]
    out = np.empty(nb)
    for i in range(nb[0]):
        for j in range(nb[1]):
            for k in range(nb[2]):
                out[i, j, k] = voxel_tol[B * i: B * i + B, B * j: B * j + B, B * k: B * k + B].min()
    return out


def propagate(tau: np.ndarray, nb_next: Sequence[int]) -> np.ndarray:
    """Eq. 2 on the assembled grid (Fig. 6): block I of the next level takes the
    smallest tau over the blocks J whose outputs 5J..5J+4 meet 8I..8I+7."""
    out = np.full(tuple(nb_next), np.inf)
    for I in np.ndindex(*nb_next):
        rng = []
        for a in range(3):
            lo, hi = B * I[a] // MC, (B * I[a] + B - 1) // MC
            rng.append(range(lo, min(hi, tau.shape[a] - 1) + 1))
        out[I] = tau[np.ix_(*rng)].min()
    return out


def level_tolerances(tau1: np.ndarray, shape: Sequence[int], L: int) -> List[np.ndarray]:
    dims, _ = level_dims(shape, L)
    taus = [np.asarray(tau1, np.float64)]
    for s in range(1, L):
        taus.append(propagate(taus[-1], [d // B for d in dims[s]]))
    return taus


def gain() -> float:
    """Rounded-up L-inf gain of the details of one natural 8-node level."""
    return roi.round_up4(roi.amplification([np.arange(float(B))] * 3, False))


def weights(shape: Sequence[int], L: int) -> List[float]:
    """Budget shares of the L levels' details and of the coarsest values."""
    dims, last = level_dims(shape, L)
    N = float(sum(np.prod(d) for d in dims) + np.prod(last))
    counts = [float(np.prod(d)) * (B ** 3 - MC ** 3) / B ** 3 for d in dims] + [float(np.prod(last))]
    w = [c / N for c in counts]
    floor = 1.0 / (64.0 * float(L + 1))
    w = [v if v > floor else floor for v in w]
    total = 0.0
    for v in w:
        total += v
    return [v / total for v in w]


def node_delta(shape: Sequence[int], L: int, tau1: np.ndarray, eta: float) -> np.ndarray:
    """Bin width Delta of every coefficient (flat layout of :func:`decompose`)."""
    dims, last = level_dims(shape, L)
    taus = level_tolerances(tau1, shape, L)
    A = gain()
    w = weights(shape, L)
    parts = []
    for s in range(L):
        k = (2.0 * (1.0 - eta)) * w[s] / A
        parts.append((np.kron(taus[s], np.ones((B, B, B))) * k).ravel())
    kc = (2.0 * (1.0 - eta)) * w[L]
    src = [np.arange(n) // MC for n in last]          # block of the last level each value came from
    parts.append((taus[L - 1][np.ix_(*src)] * kc).ravel())
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# The paper's hybrid with this block form (Sec. IV-B, IV-C; Sec. V-D's
# default L = 1, M = 2): L block levels, then M global levels on the
# assembled coarsest grid
# --------------------------------------------------------------------------
#
# Readings: the coarsest values of the block levels (dims 5 nb_L per axis,
# side by side in block order) are the grid the global levels work on, with
# the node index as coordinate (the block levels' own coordinates are block
# local); each global level is one MGARD level with natural ends on the whole
# grid (Sec. II-B), whose axes are extended by clamp to the smallest length
# on which the M levels halve an odd length (the padding rule of the shared-
# face form).  Coefficients: the block levels' arrays, then the global
# levels' in-place array of that extended grid.  Quantization: shares over
# the L block levels, the M global levels (their details split equally) and
# the coarsest values, proportional to counts, floored at 1/(64 T) with
# T = L+M+1 and renormalised; block-level details keep their blocks' taus,
# every global coefficient takes tau_global = the smallest last-level block
# tau (Sec. IV-C), global details with the natural level's gain.  Errors of
# the assembled grid reach the fine nodes through the block levels'
# interpolation only (gain 1), so every node keeps its bound.


def global_hierarchy(shape: Sequence[int], L: int, M: int) -> mgard.Hierarchy:
    """The M global levels on the assembled coarsest grid of L block levels."""
    _, last = level_dims(shape, L)
    return mgard.hierarchy(last, 0, 0, M)


def hybrid_coeff_size(shape: Sequence[int], L: int, M: int) -> int:
    dims, _ = level_dims(shape, L)
    return int(sum(np.prod(d) for d in dims) + np.prod(global_hierarchy(shape, L, M).shape_p))


def decompose_hybrid(x: np.ndarray, L: int, M: int) -> np.ndarray:
    """Block levels, then global levels on their coarsest values (flat, FP64)."""
    if M == 0:
        return decompose(x, L)
    dims, last = level_dims(np.shape(x), L)
    c = decompose(x, L)
    off = int(sum(np.prod(d) for d in dims))
    g = mgard.decompose(c[off:].reshape(last), 0, 0, M)
    return np.concatenate([c[:off], g.ravel()])


def recompose_hybrid(coeff: np.ndarray, shape: Sequence[int], L: int, M: int) -> np.ndarray:
    """Inverse of :func:`decompose_hybrid`, cropped to ``shape``."""
    if M == 0:
        return recompose(coeff, shape, L)
    dims, last = level_dims(shape, L)
    h = global_hierarchy(shape, L, M)
    coeff = np.asarray(coeff, np.float64)
    if coeff.size != hybrid_coeff_size(shape, L, M):
        raise ValueError("coefficient array has the wrong size")
    off = int(sum(np.prod(d) for d in dims))
    g = mgard.recompose(coeff[off:].reshape(h.shape_p), last, 0, 0, M)
    return recompose(np.concatenate([coeff[:off], g.ravel()]), shape, L)


def hybrid_weights(shape: Sequence[int], L: int, M: int) -> List[float]:
    """Shares of the L block levels, the M global levels and the coarsest values."""
    if M == 0:
        return weights(shape, L)
    dims, _ = level_dims(shape, L)
    h = global_hierarchy(shape, L, M)
    sizes = [float(np.prod([len(p) for p in pos])) for pos in h.pos]
    N = float(sum(np.prod(d) for d in dims)) + sizes[0]
    w = [float(np.prod(d)) * (B ** 3 - MC ** 3) / B ** 3 / N for d in dims]
    w += [((sizes[0] - sizes[M]) / N) / float(M)] * M
    w.append(sizes[M] / N)
    floor = 1.0 / (64.0 * float(L + M + 1))
    w = [v if v > floor else floor for v in w]
    total = 0.0
    for v in w:
        total += v
    return [v / total for v in w]


def hybrid_node_delta(shape: Sequence[int], L: int, M: int, tau1: np.ndarray, eta: float) -> np.ndarray:
    """Bin width Delta of every coefficient (flat layout of :func:`decompose_hybrid`)."""
    if M == 0:
        return node_delta(shape, L, tau1, eta)
    dims, _ = level_dims(shape, L)
    taus = level_tolerances(tau1, shape, L)
    A = gain()
    w = hybrid_weights(shape, L, M)
    parts = []
    for s in range(L):
        parts.append((np.kron(taus[s], np.ones((B, B, B))) * roi.kappa(w[s], A, eta)).ravel())
    tg = float(taus[L - 1].min())
    h = global_hierarchy(shape, L, M)
    gains = roi.level_gains(h)
    lev = mgard.node_level(h.shape_p, 0, M)
    k = [roi.kappa(w[L + s], gains[s], eta) for s in range(M)] + [(2.0 * (1.0 - eta)) * w[L + M]]
    parts.append((tg * np.asarray(k)[lev - 1]).ravel())
    return np.concatenate(parts)
