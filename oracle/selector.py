"""Oracle: throughput model (Eq. 1) and automatic (L, M) selection (Algorithm 1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. IV-B: throughput of N concurrent blocks is N / (1/Slope + N/TP_peak);
Algorithm 1 enumerates the valid (L, M) pairs, keeps those whose predicted
decomposition + quantization + lossless time fits the budget, and returns the
pair that is lexicographically largest in (M, -L).
"""
from __future__ import annotations

from typing import Callable, Iterable, Optional, Tuple


def throughput(n: float, slope: float, tp_peak: float) -> float:
    """Eq. 1."""
    return n / (1.0 / slope + n / tp_peak)


def quant_time(n: float, slope: float, t_lat: float) -> float:
    """Sec. IV-B: quantization time max(slope * N, T_latency)."""
    return max(slope * n, t_lat)


def select(candidates: Iterable[Tuple[int, int]],
           predict: Callable[[int, int], float],
           budget: float) -> Optional[Tuple[int, int]]:
    """Algorithm 1: argmax over the feasible pairs of (M, -L)."""
    feasible = [(L, M) for (L, M) in candidates if predict(L, M) <= budget]
    if not feasible:
        return None
    return max(feasible, key=lambda lm: (lm[1], -lm[0]))


def predict(shape, b: int, L: int, M: int, model: dict) -> Tuple[float, float, float, float]:
    """Predicted decomposition, quantization and lossless times (ms) of the
    hybrid hierarchy (b, L, M) on a grid of ``shape`` under a stage model
    (Sec. IV-B: PredictDecompTime from Eq. 1 for block levels and a line in
    the node count for global levels, PredictQuantTime = max(slope N, T_lat)
    fitted apart for local and global quantization, PredictLosslessTime = one
    line per Huffman stage).

    ``model`` keys: blk_lat_ms, blk_tp (Eq. 1 with Slope = 1/blk_lat_ms and
    TP_peak = blk_tp blocks per ms); fblk_lat_ms, fblk_tp for the last block
    level when a global level follows it; glob_a_ms, glob_b_ms and fglob_a_ms,
    fglob_b_ms (the first global level after a block level) per node;
    q_slope_ms, q_lat_ms (the local quantizer, one term per block level on
    that level's grid) and gq_slope_ms, gq_lat_ms (the global one, for an
    all-global hierarchy);
    huf_a_ms[4], huf_b_ms[4] per code.  Block size 33 takes the plain fits
    throughout.
    """
    from . import mgard
    n = [mgard.padded_length(int(d), b, L, M) for d in shape]
    nodes = float(n[0]) * float(n[1]) * float(n[2])
    fused = L > 0 and M > 0 and b != 33
    td = tq = 0.0
    for s in range(1, L + M + 1):
        if s <= L:
            blocks = 1.0
            for v in n:
                blocks *= float((v - 1) // (b - 1))
            if fused and s == L:
                lat, tp = model["fblk_lat_ms"], model["fblk_tp"]
            else:
                lat, tp = model["blk_lat_ms"], model["blk_tp"]
            td += blocks / throughput(blocks, 1.0 / lat, tp)          # = 1/Slope + N / TP_peak
            # local quantization, one term per block level (its tables)
            tq += quant_time(float(n[0]) * float(n[1]) * float(n[2]), model["q_slope_ms"], model["q_lat_ms"])
        else:
            g = float(n[0]) * float(n[1]) * float(n[2])
            if fused and s == L + 1:
                td += model["fglob_a_ms"] + model["fglob_b_ms"] * g
            else:
                td += model["glob_a_ms"] + model["glob_b_ms"] * g
        n = [(v + 1) // 2 if v > 2 else v for v in n]
    if L == 0:
        tq = quant_time(nodes, model["gq_slope_ms"], model["gq_lat_ms"])
    tl = sum(a + bb * nodes for a, bb in zip(model["huf_a_ms"], model["huf_b_ms"]))
    return td, tq, tl, td + tq + tl
