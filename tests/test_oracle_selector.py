"""Pins of Eq. 1 (throughput model) and Algorithm 1 (Sec. IV-B)."""
import pytest

from oracle import selector


def test_eq1_limits():
    slope, peak = 2.0, 1000.0
    assert selector.throughput(1e-6, slope, peak) == pytest.approx(slope * 1e-6, rel=1e-6)
    assert selector.throughput(1e12, slope, peak) == pytest.approx(peak, rel=1e-6)
    # half of the peak where the two terms are equal: N = peak / slope
    assert selector.throughput(peak / slope, slope, peak) == pytest.approx(peak / 2)


def test_quant_time_floor():
    assert selector.quant_time(10, 1.0, 50.0) == 50.0
    assert selector.quant_time(100, 1.0, 50.0) == 100.0


def test_algorithm1_prefers_more_global_then_fewer_local():
    cands = [(L, M) for L in range(0, 4) for M in range(0, 4) if L + M > 0]
    cost = {(L, M): 1.0 * M + 0.2 * L for (L, M) in cands}
    assert selector.select(cands, lambda L, M: cost[(L, M)], 2.5) == (0, 2)
    assert selector.select(cands, lambda L, M: cost[(L, M)], 100) == (0, 3)
    assert selector.select(cands, lambda L, M: cost[(L, M)], 0.1) is None
