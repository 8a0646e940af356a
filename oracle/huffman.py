"""Oracle: canonical Huffman coding of quantized codes, chunked MSB-first stream.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper names the lossless stage only by its parts (outlier handling,
histogram, codebook build, encode; Sec. IV-B, citing a GPU Huffman coder).
The format here is the reading used by the library:

* symbol = q + R for |q| < R with R = 2^15; symbol 0 is the escape, and the
  value q of each escaped code is stored on the side in raster order (its
  position is that of its escape symbol; per-chunk counts locate them);
* code lengths from Huffman's algorithm, always merging the two smallest
  (weight, smallest symbol in the subtree) keys, so the tree is unique;
  lengths above 32 are cut to 32 and the longest codes still below 32 are
  lengthened one at a time (largest symbol first) until Kraft's sum is <= 1;
* canonical codes in (length, symbol) order;
* symbols in raster order of the code array, cut into chunks of 4096; each
  chunk is packed MSB-first into 32-bit words and starts on a word boundary;
  a table of chunk start offsets (in words) has nchunks + 1 entries.
"""
from __future__ import annotations

import heapq
from typing import Dict, List, Tuple

import numpy as np

RADIUS = 1 << 15
NSYM = 2 * RADIUS
CHUNK = 4096
LMAX = 32


def to_symbols(codes: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Symbols plus outliers (raster indices, values) for int codes."""
    q = np.asarray(codes, np.int64).ravel()
    inside = np.abs(q) < RADIUS
    sym = np.where(inside, q + RADIUS, 0).astype(np.int64)
    oidx = np.nonzero(~inside)[0].astype(np.int64)
    return sym, oidx, q[oidx]


def from_symbols(sym: np.ndarray, oidx: np.ndarray, oval: np.ndarray) -> np.ndarray:
    q = np.asarray(sym, np.int64) - RADIUS
    q[np.asarray(oidx, np.int64)] = oval
    return q


def outlier_offsets(oidx: np.ndarray, n: int, chunk: int = CHUNK) -> np.ndarray:
    """Number of outliers before each chunk (nchunks + 1 entries)."""
    nch = (n + chunk - 1) // chunk
    counts = np.bincount(np.asarray(oidx, np.int64) // chunk, minlength=nch)[:nch]
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def histogram(sym: np.ndarray) -> np.ndarray:
    return np.bincount(np.asarray(sym, np.int64), minlength=NSYM).astype(np.int64)


def code_lengths(hist: np.ndarray) -> np.ndarray:
    """Huffman code length of every symbol (0 for absent symbols)."""
    hist = np.asarray(hist, np.int64)
    present = [int(s) for s in np.nonzero(hist)[0]]
    lengths = np.zeros(len(hist), np.int64)
    if not present:
        return lengths
    if len(present) == 1:
        lengths[present[0]] = 1
        return lengths
    # heap items: (weight, smallest symbol in subtree, node id)
    heap = [(int(hist[s]), s, s) for s in present]
    heapq.heapify(heap)
    parent: Dict[int, int] = {}
    nxt = len(hist)
    while len(heap) > 1:
        w1, m1, a = heapq.heappop(heap)
        w2, m2, c = heapq.heappop(heap)
        parent[a] = nxt
        parent[c] = nxt
        heapq.heappush(heap, (w1 + w2, min(m1, m2), nxt))
        nxt += 1
    root = heap[0][2]
    depth = {root: 0}

    def d(node):
        if node in depth:
            return depth[node]
        path = []
        while node not in depth:
            path.append(node)
            node = parent[node]
        base = depth[node]
        for k, nd in enumerate(reversed(path)):
            depth[nd] = base + k + 1
        return depth[path[0]]

    for s in present:
        lengths[s] = d(s)
    return limit_lengths(lengths)


def limit_lengths(lengths: np.ndarray) -> np.ndarray:
    lengths = lengths.copy()
    if lengths.max() <= LMAX:
        return lengths
    lengths[lengths > LMAX] = LMAX
    kraft = sum(1 << (LMAX - int(l)) for l in lengths if l > 0)
    while kraft > (1 << LMAX):
        cand = [(int(l), s) for s, l in enumerate(lengths) if 0 < l < LMAX]
        l, s = max(cand)
        lengths[s] = l + 1
        kraft -= 1 << (LMAX - l - 1)
    return lengths


def canonical_codes(lengths: np.ndarray) -> np.ndarray:
    """Canonical code values (MSB-first, ``lengths[s]`` bits) by (length, symbol)."""
    order = sorted((int(l), s) for s, l in enumerate(lengths) if l > 0)
    codes = np.zeros(len(lengths), np.uint64)
    code = 0
    prev = 0
    for i, (l, s) in enumerate(order):
        if i > 0:
            code = (code + 1) << (l - prev)
        else:
            code = 0
        codes[s] = code
        prev = l
    return codes


def encode(sym: np.ndarray, lengths: np.ndarray, chunk: int = CHUNK) -> Tuple[np.ndarray, np.ndarray]:
    """Bitstream words (uint32) and chunk offsets (nchunks+1 word offsets)."""
    sym = np.asarray(sym, np.int64)
    codes = canonical_codes(lengths)
    n = len(sym)
    nch = (n + chunk - 1) // chunk
    words: List[np.ndarray] = []
    offsets = np.zeros(nch + 1, np.int64)
    for c in range(nch):
        s = sym[c * chunk:(c + 1) * chunk]
        ln = lengths[s].astype(np.int64)
        if np.any(ln == 0):
            raise ValueError("symbol without a code")
        cv = codes[s].astype(np.uint64)
        start = np.concatenate([[0], np.cumsum(ln)[:-1]])
        nbits = int(ln.sum())
        nw = (nbits + 31) // 32
        buf = np.zeros(nw + 1, np.uint64)
        w = start // 32
        o = start % 32
        # place each code in a 64-bit window starting at word w
        sh = (64 - o - ln).astype(np.uint64)
        val = cv << sh
        hi = (val >> np.uint64(32)) & np.uint64(0xFFFFFFFF)
        lo = val & np.uint64(0xFFFFFFFF)
        np.bitwise_or.at(buf, w, hi)
        np.bitwise_or.at(buf, w + 1, lo)
        words.append(buf[:nw].astype(np.uint32))
        offsets[c + 1] = offsets[c] + nw
    stream = np.concatenate(words) if words else np.zeros(0, np.uint32)
    return stream, offsets


def decode(stream: np.ndarray, offsets: np.ndarray, lengths: np.ndarray, nsym: int,
           chunk: int = CHUNK) -> np.ndarray:
    """Bit-by-bit canonical decoder (slow; small inputs)."""
    codes = canonical_codes(lengths)
    table = {(int(l), int(codes[s])): s for s, l in enumerate(lengths) if l > 0}
    out = np.empty(nsym, np.int64)
    k = 0
    for c in range(len(offsets) - 1):
        words = stream[offsets[c]:offsets[c + 1]]
        bitpos = 0
        cnt = min(chunk, nsym - c * chunk)
        for _ in range(cnt):
            code, l = 0, 0
            while True:
                wv = int(words[bitpos // 32])
                bit = (wv >> (31 - bitpos % 32)) & 1
                code = (code << 1) | bit
                l += 1
                bitpos += 1
                if (l, code) in table:
                    out[k] = table[(l, code)]
                    k += 1
                    break
                if l > LMAX:
                    raise ValueError("corrupt stream")
    return out
