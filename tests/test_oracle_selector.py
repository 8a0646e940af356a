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


def test_predict_by_hand():
    # 513^3, b = 17: level 1 has 32^3 blocks, level 2 (global) a 257^3 grid, level 3 a 129^3 grid
    m = {"blk_lat_ms": 0.01, "blk_tp": 1e5, "fblk_lat_ms": 0.02, "fblk_tp": 5e4, "fglob_a_ms": 0.03,
         "fglob_b_ms": 1e-9, "glob_a_ms": 0.04, "glob_b_ms": 2e-9, "q_slope_ms": 1e-10, "q_lat_ms": 0.5,
         "gq_slope_ms": 3e-9, "gq_lat_ms": 0.25, "huf_a_ms": [1.0, 2.0, 3.0, 4.0], "huf_b_ms": [1e-9, 0.0, 2e-9, 3e-9]}
    nodes = 513.0 ** 3
    # pure block level: Eq. 1 time N / TP(N) = 1/Slope + N/TP_peak
    td, tq, tl, tot = selector.predict((513, 513, 513), 17, 1, 0, m)
    assert td == pytest.approx(0.01 + 32 ** 3 / 1e5, rel=1e-12)
    assert tq == pytest.approx(max(1e-10 * nodes, 0.5), rel=1e-12)
    assert tl == pytest.approx(10.0 + 6e-9 * nodes, rel=1e-12)
    assert tot == pytest.approx(td + tq + tl, rel=1e-12)
    # L = 1, M = 2: the fused block level, the fused first global level, a plain global level
    td, tq, _, _ = selector.predict((513, 513, 513), 17, 1, 2, m)
    assert td == pytest.approx((0.02 + 32 ** 3 / 5e4) + (0.03 + 1e-9 * 257.0 ** 3) + (0.04 + 2e-9 * 129.0 ** 3),
                               rel=1e-12)
    assert tq == pytest.approx(max(1e-10 * nodes, 0.5), rel=1e-12)       # one block level: the local quantizer
    # two block levels (513^3 then 257^3 grids): one local term each
    _, tq, _, _ = selector.predict((513, 513, 513), 17, 2, 1, {**m, "q_lat_ms": 0.001})
    assert tq == pytest.approx(1e-10 * nodes + 1e-10 * 257.0 ** 3, rel=1e-12)
    # all global (L = 0, M = 1): the global quantizer's own fit, 3e-9 N above its floor
    _, tq, _, _ = selector.predict((513, 513, 513), 17, 0, 1, m)
    assert tq == pytest.approx(3e-9 * nodes, rel=1e-12)
