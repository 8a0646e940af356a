"""Pins of the oracle's Huffman stage.

Checked against facts independent of this implementation: decoding inverts
encoding (with a bit-by-bit decoder), Kraft equality for complete codes, the
total coded length equals the sum of internal-node weights of any Huffman
tree (independent of tie-breaking), optimality by brute force on tiny
alphabets, prefix-freeness of the canonical codes, and the 32-bit cap.
"""
import heapq
import itertools

import numpy as np
import pytest

from oracle import huffman as hf


def _geometric_codes(n, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    q = np.rint(rng.laplace(0, scale, n)).astype(np.int64)
    q[:: max(1, n // 17)] += 1 << 16   # a few outliers
    return q


def test_roundtrip_small():
    q = _geometric_codes(9000, 0)
    sym, oi, ov = hf.to_symbols(q)
    ln = hf.code_lengths(hf.histogram(sym))
    stream, off = hf.encode(sym, ln)
    assert len(off) == (len(sym) + hf.CHUNK - 1) // hf.CHUNK + 1
    dec = hf.decode(stream, off, ln, len(sym))
    assert np.array_equal(dec, sym)
    assert np.array_equal(hf.from_symbols(dec, oi, ov), q)


def _huffman_cost(weights):
    h = list(weights)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


@pytest.mark.parametrize("seed", range(5))
def test_kraft_and_total_bits(seed):
    rng = np.random.default_rng(seed)
    hist = np.zeros(hf.NSYM, np.int64)
    syms = rng.choice(hf.NSYM, 300, replace=False)
    hist[syms] = rng.integers(1, 1000, 300)
    hist[syms[:20]] = 1                 # many ties
    ln = hf.code_lengths(hist)
    assert sum(2.0 ** -l for l in ln[ln > 0]) == pytest.approx(1.0, abs=1e-12)
    assert int((ln * hist).sum()) == _huffman_cost(hist[hist > 0])


def test_optimal_by_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(20):
        k = int(rng.integers(2, 6))
        w = rng.integers(1, 50, k)
        hist = np.zeros(hf.NSYM, np.int64)
        hist[:k] = w
        ln = hf.code_lengths(hist)[:k]
        best = min(sum(int(a) * int(b) for a, b in zip(w, L))
                   for L in itertools.product(range(1, k + 1), repeat=k)
                   if sum(2.0 ** -l for l in L) <= 1.0)
        assert int((ln * w).sum()) == best


def test_canonical_prefix_free():
    rng = np.random.default_rng(4)
    hist = np.zeros(hf.NSYM, np.int64)
    hist[rng.choice(hf.NSYM, 100, replace=False)] = rng.integers(1, 10000, 100)
    ln = hf.code_lengths(hist)
    cv = hf.canonical_codes(ln)
    words = [format(int(cv[s]), "0%db" % ln[s]) for s in np.nonzero(ln)[0]]
    for a, b in itertools.permutations(words, 2):
        assert not b.startswith(a)


def test_length_cap():
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    hist = np.zeros(hf.NSYM, np.int64)
    hist[100:140] = fib
    ln = hf.code_lengths(hist)
    assert ln.max() == hf.LMAX
    assert sum(2.0 ** -int(l) for l in ln[ln > 0]) <= 1.0
    sym = np.repeat(np.arange(100, 140), 3)
    stream, off = hf.encode(sym, ln)
    assert np.array_equal(hf.decode(stream, off, ln, len(sym)), sym)


def test_single_symbol():
    sym = np.full(5000, hf.RADIUS)
    ln = hf.code_lengths(hf.histogram(sym))
    assert ln[hf.RADIUS] == 1
    stream, off = hf.encode(sym, ln)
    assert np.array_equal(hf.decode(stream, off, ln, len(sym)), sym)


def test_outlier_offsets_brute_force():
    """Per-chunk outlier offsets equal a direct count of escapes before each chunk."""
    rng = np.random.default_rng(7)
    n, chunk = 1000, 64
    q = rng.integers(-10, 10, n)
    q[rng.choice(n, 37, replace=False)] = 1 << 20
    sym, oi, ov = hf.to_symbols(q)
    off = hf.outlier_offsets(oi, n, chunk)
    nch = (n + chunk - 1) // chunk
    assert len(off) == nch + 1
    for c in range(nch + 1):
        assert off[c] == sum(1 for i in range(min(c * chunk, n)) if sym[i] == 0)
    assert np.array_equal(hf.from_symbols(sym, oi, ov), q)
