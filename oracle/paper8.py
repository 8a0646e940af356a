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
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import mgard

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
