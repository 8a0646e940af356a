"""Oracle: ROI tolerance maps, conservative propagation, error budget, quantizer.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain FP64 NumPy.

Paper passages followed
-----------------------
* Sec. IV-C, block-wise tolerance assignment: one tolerance per block; a
  block that an ROI only partly overlaps takes the stricter tolerance.
* Sec. IV-C, Eq. 2: a coarse-level block inherits the minimum tolerance of
  the finer-level blocks that contribute to it, applied recursively through
  the L local levels; the global levels get the minimum over the last local
  level.
* Sec. II-B: level-dependent error budget giving an L-infinity bound.
* Sec. IV-D: scalar or per-block reciprocal quantizer (multiply by 1/Delta).
* Sec. V-A: the REL bound is tol * max|u|.

Readings where the paper is silent
----------------------------------
* "Contributes" in Eq. 2 = shares at least one node (shared-face blocks).
* A node's tolerance at a block level is the minimum over the blocks of that
  level that contain it.
* Budget: level s gets the share w_s of every tolerance, w_s proportional to
  the number of coefficients of level s (so the share tightens as levels
  coarsen), the M global levels splitting their part equally; the coarsest
  values get w_c = their count / the total, and the shares sum to 1.  A
  detail of level s gets half-width e = tau (1 - eta) w_s / A_s, where A_s is
  the exact L-infinity gain of that level's detail coefficients in
  reconstruction (max row sum of |I - P3 K3| over detail columns), rounded up
  to 4 decimals; the coarsest values get e = tau (1 - eta) w_c (interpolation
  has gain 1).  Bin width Delta = 2e, q = rint(c * (1/Delta)) in FP64 (round
  half to even), c_hat = q * Delta.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import mgard

# --------------------------------------------------------------------------
# O7: block tolerances and their propagation (Sec. IV-C, Eq. 2)
# --------------------------------------------------------------------------


def voxel_tolerance_from_boxes(shape: Sequence[int], boxes: Sequence[Sequence[float]],
                               background: float) -> np.ndarray:
    """Per-voxel absolute tolerance from half-open boxes {z0,y0,x0,z1,y1,x1,tol}."""
    t = np.full(tuple(shape), float(background))
    for z0, y0, x0, z1, y1, x1, tol in boxes:
        sl = (slice(int(z0), int(z1)), slice(int(y0), int(y1)), slice(int(x0), int(x1)))
        t[sl] = np.minimum(t[sl], tol)
    return t


def block_tolerance(voxel_tol: np.ndarray, shape_p: Sequence[int], b: int) -> np.ndarray:
    """Level-1 block tolerances: min of the voxel tolerance over each block's
    closed node range; padded nodes take the tolerance of the node they copy."""
    n = voxel_tol.shape
    nb = [(p - 1) // (b - 1) for p in shape_p]
    out = np.empty(nb)
    for i in range(nb[0]):
        for j in range(nb[1]):
            for k in range(nb[2]):
                lo = [min(q * (b - 1), nn - 1) for q, nn in zip((i, j, k), n)]
                hi = [min((q + 1) * (b - 1), nn - 1) for q, nn in zip((i, j, k), n)]
                out[i, j, k] = voxel_tol[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1].min()
    return out


def propagate(tol: np.ndarray, nested: bool = False) -> np.ndarray:
    """Eq. 2: block (I,J,K) of the next level takes the min over the blocks of
    this level that share a node with it.

    A next-level block spans two current blocks per axis (2I, 2I+1); the
    blocks 2I-1 and 2I+2 touch it in one face of nodes and contribute too.
    In the nested schedule the next-level block covers the same region as
    block I of this level, so blocks I-1, I, I+1 per axis share its nodes.
    """
    nb = tol.shape
    if nested:
        out = np.empty(nb)
        for I in range(nb[0]):
            for J in range(nb[1]):
                for K in range(nb[2]):
                    out[I, J, K] = tol[max(0, I - 1): I + 2, max(0, J - 1): J + 2, max(0, K - 1): K + 2].min()
        return out
    nn = [max(1, n // 2) for n in nb]
    out = np.empty(nn)
    for I in range(nn[0]):
        for J in range(nn[1]):
            for K in range(nn[2]):
                rz = range(max(0, 2 * I - 1), min(nb[0], 2 * I + 3))
                ry = range(max(0, 2 * J - 1), min(nb[1], 2 * J + 3))
                rx = range(max(0, 2 * K - 1), min(nb[2], 2 * K + 3))
                out[I, J, K] = min(tol[a, c, d] for a in rz for c in ry for d in rx)
    return out


def level_block_tolerances(tol1: np.ndarray, L: int, nested: bool = False) -> List[np.ndarray]:
    """[tau^1, ..., tau^L]: level-1 map and its recursive propagation."""
    tols = [np.asarray(tol1, np.float64)]
    for _ in range(1, L):
        tols.append(propagate(tols[-1], nested))
    return tols


def node_tolerance(tol_s: np.ndarray, grid_shape: Sequence[int], b: int) -> np.ndarray:
    """Per-node tolerance on a level grid: min over the blocks containing the node."""
    # Block i covers nodes [i(b-1), (i+1)(b-1)], so node q lies in blocks
    # ceil(q/(b-1)) - 1 .. floor(q/(b-1)) (clipped): at most two per axis.
    per_axis = []
    for n, nb in zip(grid_shape, tol_s.shape):
        q = np.arange(n)
        lo = np.maximum(0, -(-q // (b - 1)) - 1)
        hi = np.minimum(q // (b - 1), nb - 1)
        per_axis.append((lo, hi))
    out = None
    for iz in per_axis[0]:
        for iy in per_axis[1]:
            for ix in per_axis[2]:
                t = tol_s[np.ix_(iz, iy, ix)]
                out = t if out is None else np.minimum(out, t)
    return out


# --------------------------------------------------------------------------
# O8: per-level amplification and the budget (Sec. II-B)
# --------------------------------------------------------------------------


def amplification_dense(coords3, face_fixed: bool) -> float:
    """A for one level by brute force: the max over rows of the dense matrix
    (I - P3 K3) summed in absolute value over the detail columns."""
    ops = [mgard.axis_ops(np.asarray(c, float), face_fixed) for c in coords3]
    a = [o.P @ o.K for o in ops]
    big = np.kron(np.kron(a[0], a[1]), a[2])
    n = big.shape[0]
    coarse = np.zeros([len(c) for c in coords3], bool)
    coarse[np.ix_(*(o.cidx for o in ops))] = True
    det = ~coarse.ravel()
    E = np.eye(n) - big
    return float(np.abs(E[:, det]).sum(axis=1).max())


def amplification(coords3, face_fixed: bool) -> float:
    """A for one level from 1D row sums (same quantity as the dense form).

    For a row x the detail-column sum of |delta_xy - prod_d a_d(x_d, y_d)| is
    prod S_all - prod S_coarse, plus |1 - prod diag| - |prod diag| when x is
    itself a detail node; S_all / S_coarse are 1D row sums of |a_d| over all /
    coarse columns.  The max runs over the distinct 1D row profiles.
    """
    profs = []
    for c in coords3:
        o = mgard.axis_ops(np.asarray(c, float), face_fixed)
        a = np.abs(o.P @ o.K)
        iscoarse = np.zeros(o.n, bool)
        iscoarse[o.cidx] = True
        s_all = a.sum(axis=1)
        s_c = a[:, iscoarse].sum(axis=1)
        diag = np.diag(o.P @ o.K)
        prof = np.stack([s_all, s_c, diag, iscoarse.astype(float)], axis=1)
        profs.append(np.unique(np.round(prof, 15), axis=0))
    pz, py, px = profs
    best = 0.0
    for rz in pz:
        for ry in py:
            sa = rz[0] * ry[0] * px[:, 0]
            sc = rz[1] * ry[1] * px[:, 1]
            dg = rz[2] * ry[2] * px[:, 2]
            allc = (rz[3] > 0) & (ry[3] > 0) & (px[:, 3] > 0)
            val = sa - sc + np.where(allc, 0.0, np.abs(1.0 - dg) - np.abs(dg))
            best = max(best, float(val.max()))
    return best


def round_up4(a: float) -> float:
    """Round a gain up to 4 decimals (both sides of the parity test use this value).

    A slack of 1e-6 in units of the last decimal keeps a gain that is an exact
    4-decimal number (2.375 for a 3-node level) from being pushed up by
    rounding noise in how it was summed.
    """
    return math.ceil(a * 10000.0 - 1e-6) / 10000.0


def level_gains(h: mgard.Hierarchy) -> List[float]:
    """Rounded-up gain A_s for s = 1..L+M."""
    out = []
    for s in range(1, h.levels + 1):
        if s <= h.L:
            c = [np.arange(h.block(s), dtype=float)] * 3
            out.append(round_up4(amplification(c, True)))
        else:
            c = [np.arange(len(p), dtype=float) for p in h.pos[s - 1]]
            out.append(round_up4(amplification(c, False)))
    return out


def level_weights(h: mgard.Hierarchy) -> List[float]:
    """Share of the L-infinity budget of each level (s = 1..L+M) and of the
    coarsest values (last entry).

    Sec. II-B: the share tightens as the level coarsens; reading: a level's
    share is proportional to the number of coefficients it holds.  Sec. IV-C:
    the M global levels share their part equally.
    """
    N = float(np.prod(h.shape_p))
    sizes = [int(np.prod([len(p) for p in pos])) for pos in h.pos]
    counts = [sizes[s - 1] - sizes[s] for s in range(1, h.levels + 1)]
    w = [0.0] * (h.levels + 1)
    nglob = sum(counts[h.L:])
    for s in range(1, h.levels + 1):
        w[s - 1] = counts[s - 1] / N if s <= h.L else (nglob / N) / float(h.M)
    w[h.levels] = sizes[h.levels] / N
    # no share below 1/(64 T), T = L+M+1: keeps the bins of small, deep
    # levels within reach of 32-bit codes; then renormalise (sequential sum)
    floor = 1.0 / (64.0 * float(h.levels + 1))
    w = [v if v > floor else floor for v in w]
    total = 0.0
    for v in w:
        total += v
    return [v / total for v in w]


def kappa(w: float, A: float, eta: float) -> float:
    """Bin width per unit tolerance for a level with share w and gain A: Delta = tau * kappa."""
    return (2.0 * (1.0 - eta)) * w / A


def node_delta(h: mgard.Hierarchy, tol1, eta: float) -> np.ndarray:
    """Bin width Delta of every node of the padded grid.

    ``tol1`` is the level-1 block map (L >= 1) or a scalar (L == 0).
    """
    L, M = h.L, h.M
    gains = level_gains(h)
    w = level_weights(h)
    lev = mgard.node_level(h.shape_p, L, M)
    delta = np.zeros(h.shape_p)
    if L >= 1:
        tols = level_block_tolerances(np.asarray(tol1, float), L, h.nested)
        tau_global = float(tols[-1].min())
    else:
        tols = []
        tau_global = float(np.min(tol1))
    for s in range(1, L + M + 2):
        grid = np.ix_(*h.pos[s - 1])
        sub_lev = lev[grid]
        mask = sub_lev == s
        if not mask.any():
            continue
        if s <= L:
            tau = node_tolerance(tols[s - 1], [len(p) for p in h.pos[s - 1]], h.block(s))
        elif s == L + M + 1 and M == 0 and L >= 1:
            tau = node_tolerance(tols[L - 1], [len(p) for p in h.pos[L - 1]], h.block(L))
            # coarsest nodes are the coarse nodes of the level-L grid
            tau = tau[np.ix_(*(mgard.coarse_indices(len(p)) for p in h.pos[L - 1]))]
        else:
            tau = np.full([len(p) for p in h.pos[s - 1]], tau_global)
        k = kappa(w[s - 1], gains[s - 1], eta) if s <= L + M else (2.0 * (1.0 - eta)) * w[L + M]
        d = tau * k
        sub = delta[grid]
        sub[mask] = d[mask]
        delta[grid] = sub
    return delta


# --------------------------------------------------------------------------
# O9: reciprocal quantizer (Sec. IV-D)
# --------------------------------------------------------------------------


def quantize(coeff: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """q = rint(c * (1/Delta)) in FP64, int64 result."""
    inv = 1.0 / delta
    return np.rint(np.asarray(coeff, np.float64) * inv).astype(np.int64)


def dequantize(codes: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """c_hat = q * Delta in FP64."""
    return np.asarray(codes, np.float64) * delta


def rel_to_abs(rel: float, x: np.ndarray) -> float:
    """Sec. V-A: the REL bound is tol * max|u|."""
    return float(rel) * float(np.max(np.abs(x)))


# --------------------------------------------------------------------------
# Adjoint-guided bounds for a linear quantity of interest (an addition to the
# method: per-coefficient bin widths from the transpose of recomposition)
# --------------------------------------------------------------------------


def qoi_delta(h: mgard.Hierarchy, tol1, g: np.ndarray, tol_q: float, eta: float) -> Tuple[np.ndarray, int]:
    """Bin widths that keep Q(x) = <g, x> within tol_q after quantization.

    The coefficients' sensitivities are s = R^T g (the recomposition's
    transpose), so quantization moves Q by at most sum |s_i| Delta_i / 2.
    Every Delta_i is capped by the node's L-infinity width from the tolerance
    map (``node_delta``), so the map's bounds still hold.  Reading (the
    widths that maximise the sum of log Delta_i, i.e. the code length saved,
    under the two constraints): each coefficient's share |s_i| Delta_i / 2 is
    the same level lambda, except where the cap is smaller:

        |s_i| Delta_i / 2 = min(a_i, lambda),   a_i = |s_i| cap_i / 2,

    with lambda the root of sum_i min(a_i, lambda) = (1 - eta) tol_q (no root:
    sum a_i <= (1 - eta) tol_q and every coefficient keeps its cap).  The
    root is found plainly: a sorted ascending, the first k with
    prefix_k + a_k (N - k) >= target gives lambda = (target - prefix_k) / (N - k).
    Returns (Delta, number of coefficients whose width the quantity sets,
    i.e. a_i > lambda).
    """
    s = mgard.recompose_adjoint(np.asarray(g, np.float64), h.shape, h.b, h.L, h.M, h.nested)
    cap = node_delta(h, tol1, eta)
    a = np.abs(s) * cap / 2.0
    target = (1.0 - eta) * float(tol_q)
    lam = qoi_level(a.ravel(), target)
    if lam is None:
        return cap, 0
    set_by_q = a > lam
    delta = cap.copy()
    delta[set_by_q] = 2.0 * lam / np.abs(s[set_by_q])
    return delta, int(set_by_q.sum())


def qoi_level(a: np.ndarray, target: float):
    """lambda with sum_i min(a_i, lambda) = target, or None if sum a_i <= target."""
    if float(np.sum(a)) <= target:
        return None
    srt = np.sort(np.asarray(a, np.float64))
    n = srt.size
    prefix = np.concatenate([[0.0], np.cumsum(srt)[:-1]])     # sum of the k smallest
    k = int(np.argmax(prefix + srt * (n - np.arange(n)) >= target))
    return (target - prefix[k]) / (n - k)
