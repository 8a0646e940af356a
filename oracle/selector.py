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
