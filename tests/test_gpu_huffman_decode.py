"""The wavefront-per-chunk Huffman decoder on streams assembled by hand from
the oracle's encoder (stream version 3, layout in include/blockmgard.h).

The oracle encodes any set of code lengths that satisfies Kraft's
inequality, so these streams reach what Huffman code lengths of real data
rarely do: codes of 13..32 bits (the decoder's path past its lookup table),
incomplete codes (bit patterns that are no codeword, met by lanes that start
decoding at a guessed position), chunks of 4096 words (every code 32 bits),
a single symbol, ragged last chunks.  Every decode is compared with the
symbols that were encoded; small streams also with the oracle's bit-by-bit
decoder.  Malformed chunks (a word missing, an outlier count off by one, an
invalid code among the symbols) fail with BM_ECORRUPT; words after a
chunk's last symbol are ignored, as the oracle's decoder ignores them.
"""
import struct

import numpy as np
import pytest
import torch

from oracle import huffman as ohf

pytestmark = pytest.mark.gpu

R = ohf.RADIUS


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()


def _lengths(pairs):
    ln = np.zeros(ohf.NSYM, np.int64)
    for s, l in pairs:
        ln[s] = l
    assert sum(2.0 ** -l for _, l in pairs) <= 1.0
    return ln


def _assemble(sym, ln, oval, words=None, offs=None, ooffs=None):
    n = len(sym)
    if words is None:
        words, offs = ohf.encode(sym, ln)
    oidx = np.nonzero(sym == 0)[0]
    if ooffs is None:
        ooffs = ohf.outlier_offsets(oidx, n)
    psym = np.nonzero(ln)[0]
    nch = (n + ohf.CHUNK - 1) // ohf.CHUNK
    hdr = struct.pack("<IIqqqqq", 0x46484D42, 3, n, nch, len(words), len(oval), len(psym))
    return (hdr + psym.astype("<u2").tobytes() + ln[psym].astype(np.uint8).tobytes() +
            np.asarray(offs, "<u8").tobytes() + np.asarray(ooffs, "<u8").tobytes() +
            np.asarray(words, "<u4").tobytes() + np.asarray(oval, "<i4").tobytes())


def _case(ln, n, seed, p=None):
    rng = np.random.default_rng(seed)
    present = np.nonzero(ln)[0]
    sym = rng.choice(present, size=n, p=p).astype(np.int64)
    nout = int((sym == 0).sum())
    oval = rng.integers(R, 1 << 30, nout) * rng.choice([-1, 1], nout)
    return sym, oval.astype(np.int64)


def _expected(sym, oval):
    return ohf.from_symbols(sym, np.nonzero(sym == 0)[0], oval)


def _decode(buf, n):
    from paper_2609_00205_amd import api
    return api.huffman_decode(buf, n).cpu().numpy().astype(np.int64)


# complete code with lengths 1..31, 32, 32 (the escape among them)
LONG = _lengths([(R + k, k + 1) for k in range(31)] + [(0, 32), (R + 40, 32)])
# 200 symbols of 32 bits each: an incomplete code, 4096 words per full chunk
MAX32 = _lengths([(R - 100 + k, 32) for k in range(199)] + [(0, 32)])
# incomplete short code (Kraft sum 0.703)
SHORT = _lengths([(R, 2), (R + 1, 2), (0, 3), (R - 1, 4), (R + 7, 6)])
# 13..16-bit codes around short ones: most symbols past a 12-bit lookup table
MID = _lengths([(R, 1), (R + 1, 2), (R + 2, 3)] + [(R + 3 + k, 13) for k in range(200)] +
               [(0, 16)] + [(R - 1 - k, 16) for k in range(100)])

CASES = [("long", LONG, 3 * 4096 + 77, None), ("long-1chunk", LONG, 4096, None), ("max32", MAX32, 2 * 4096 + 1000, None),
         ("short", SHORT, 5 * 4096 + 4095, None), ("mid", MID, 4 * 4096 + 5, None), ("short-1", SHORT, 1, None)]


@pytest.mark.parametrize("name,ln,n,p", CASES, ids=[c[0] for c in CASES])
def test_decode_hand_streams(name, ln, n, p):
    sym, oval = _case(ln, n, seed=len(name) * 7 + n)
    buf = _assemble(sym, ln, oval)
    print("case", name, "n", n, "stream bytes", len(buf), flush=True)
    got = _decode(buf, n)
    assert np.array_equal(got, _expected(sym, oval))
    if n <= 2 * 4096:
        words, offs = ohf.encode(sym, ln)
        assert np.array_equal(ohf.decode(words, offs, ln, n), sym)


def test_decode_single_symbol():
    ln = _lengths([(R + 5, 1)])
    n = 3 * 4096 + 11
    sym = np.full(n, R + 5, np.int64)
    got = _decode(_assemble(sym, ln, np.zeros(0, np.int64)), n)
    assert np.array_equal(got, np.full(n, 5))


def test_decode_skewed_realistic():
    """Huffman lengths of a Laplace histogram with rare outliers (the shape of
    quantization codes), many chunks; the decode equals the encoded codes."""
    from paper_2609_00205_amd import api
    rng = np.random.default_rng(5)
    n = 64 * 4096 + 333
    q = np.rint(rng.laplace(0, 30.0, n)).astype(np.int64)
    q[rng.choice(n, 50, replace=False)] = rng.integers(R, 1 << 29, 50)
    buf = api.huffman_encode(torch.from_numpy(q.astype(np.int32)).cuda())
    assert np.array_equal(_decode(buf, n), q)


def _long_parts(seed=11, n=3 * 4096 + 77):
    sym, oval = _case(LONG, n, seed)
    words, offs = ohf.encode(sym, LONG)
    return sym, oval, words, offs, n


def test_missing_word_rejected():
    from paper_2609_00205_amd import _lib
    sym, oval, words, offs, n = _long_parts()
    # drop the last word of chunk 1 (it holds the end of that chunk's last codeword)
    cut = int(offs[2]) - 1
    w2 = np.delete(words, cut)
    o2 = offs.copy()
    o2[2:] -= 1
    with pytest.raises(_lib.BMError) as e:
        _decode(_assemble(sym, LONG, oval, w2, o2), n)
    assert e.value.code == -6


def test_trailing_word_ignored():
    sym, oval, words, offs, n = _long_parts()
    # a word of ones after chunk 0's symbols: not read as symbols
    w2 = np.insert(words, int(offs[1]), np.uint32(0xFFFFFFFF))
    o2 = offs.copy()
    o2[1:] += 1
    got = _decode(_assemble(sym, LONG, oval, w2, o2), n)
    assert np.array_equal(got, _expected(sym, oval))


def test_outlier_count_mismatch_rejected():
    from paper_2609_00205_amd import _lib
    sym, oval, words, offs, n = _long_parts()
    oo = ohf.outlier_offsets(np.nonzero(sym == 0)[0], n)
    c = int(np.nonzero(np.diff(oo) > 0)[0][0])      # a chunk with an outlier
    oo2 = oo.copy()
    oo2[c + 1] -= 1
    with pytest.raises(_lib.BMError) as e:
        _decode(_assemble(sym, LONG, oval, words, offs, oo2), n)
    assert e.value.code == -6


def test_invalid_code_rejected():
    from paper_2609_00205_amd import _lib
    n = 4096 + 10
    sym, oval = _case(SHORT, n, 3)
    words, offs = ohf.encode(sym, SHORT)
    w2 = words.copy()
    w2[3] = 0xFFFFFFFF      # inside chunk 0; no codeword of SHORT starts with 11
    with pytest.raises(_lib.BMError) as e:
        _decode(_assemble(sym, SHORT, oval, w2, offs), n)
    assert e.value.code == -6
