"""Batched many-field pipeline (one persistent launch per block level,
optionally captured in a HIP graph) against the single-field path and
against the oracle, through the C ABI.

Bar: codes and reconstructions bit-identical to each field's own
bm_decompose_quantize / bm_dequantize_recompose (which the quantizer tests
hold to the oracle); containers byte-identical to bm_compress; graph replays
equal to eager runs on every replay.
"""
import numpy as np
import pytest
import torch

from paper_2609_00205_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()


def _fields(shapes, dt, seed):
    xs = []
    for i, sh in enumerate(shapes):
        x = synth.gaussian_random_field(sh, 3.0, seed=seed + i, dtype=np.float64)
        xs.append(torch.from_numpy(x.astype(np.float32 if dt == torch.float32 else np.float64)).cuda())
    return xs


def _tols(batch, xs, rel_in=1e-5, rel_out=1e-3):
    tols = []
    for p, x in zip(batch.plans, xs):
        s = float(x.abs().max())
        n = p.shape
        box = (n[0] // 4, n[1] // 4, n[2] // 4, n[0] // 2 + 1, n[1] // 2 + 1, n[2] // 2 + 1, rel_in * s)
        tols.append(p.tolmap_from_boxes([box], rel_out * s))
    return tols


CASES = [
    # shapes, dtype, block, L (None: per-field clamp), M
    ([(33, 17, 65), (17, 17, 17), (65, 65, 33), (33, 33, 33), (17, 33, 17)], torch.float32, 17, None, 0),
    ([(33, 17, 65), (65, 33, 33), (17, 17, 17)], torch.float64, 17, None, 0),
    ([(17, 33, 17), (33, 33, 65), (65, 65, 65)], torch.float32, 9, None, 0),
    ([(33, 33, 33), (65, 33, 33), (33, 65, 17)], torch.float32, 17, 1, 2),        # global levels per field
    ([(40, 20, 33), (25, 30, 17)], torch.float32, 9, 1, 1),                       # padded fields
    # nested schedule: a field's 17- and 9-node levels as one pair per launch
    ([(33, 17, 65), (17, 17, 17), (65, 65, 33), (33, 33, 33)], torch.float32, 17, None, 0, True),
    ([(33, 17, 65), (65, 33, 33)], torch.float64, 17, None, 0, True),
    ([(33, 33, 33), (40, 20, 33), (65, 33, 17)], torch.float32, 17, [2, 1, 2], 0, True),   # pairs beside a plain level
    ([(33, 33, 33), (65, 33, 33)], torch.float32, 17, 2, 1, True),                # pairs, then a global level
    # 33-node blocks: column, coarse (and interpolation) steps over all fields
    ([(33, 65, 33), (65, 65, 33), (33, 33, 33)], torch.float32, 33, None, 0),
    ([(65, 33, 33), (33, 33, 65)], torch.float64, 33, 1, 0),
    ([(33, 33, 65), (65, 33, 33), (40, 30, 50)], torch.float32, 33, 1, 1),       # padded, global level
]


def _id(c):
    return f"{len(c[0])}f-{str(c[1])[6:]}-b{c[2]}-L{c[3]}-M{c[4]}" + ("-nested" if len(c) > 5 and c[5] else "")


@pytest.mark.parametrize("case", CASES, ids=_id)
@pytest.mark.parametrize("use_graph", [False, True], ids=["eager", "graph"])
def test_batch_equals_single(case, use_graph):
    from paper_2609_00205_amd import Batch
    shapes, dt, b, L, M = case[:5]
    nested = len(case) > 5 and case[5]
    print("case", _id(case), "graph" if use_graph else "eager", flush=True)
    batch = Batch(shapes, dtype=dt, block=b, L=L, M=M, nested=nested)
    if nested:
        assert all(p.nested for p in batch.plans)
    xs = _fields(shapes, dt, 100)
    tols = _tols(batch, xs)
    codes = [torch.empty(p.coeff_shape, dtype=torch.int32, device="cuda") for p in batch.plans]
    outs = [torch.empty_like(x) for x in xs]
    # two rounds over the same buffers with new values: a graph replays its capture
    for rnd in range(2):
        if rnd:
            for i, x in enumerate(xs):
                x.copy_(_fields([tuple(x.shape)], dt, 500 + i)[0])
        batch.decompose_quantize(xs, tols, codes=codes, use_graph=use_graph)
        batch.dequantize_recompose(codes, tols, outs=outs, use_graph=use_graph)
        torch.cuda.synchronize()
        for p, x, t, c, o in zip(batch.plans, xs, tols, codes, outs):
            ref = p.decompose_quantize(x, t)
            assert torch.equal(c, ref), f"codes differ for field {p.shape} round {rnd}"
            assert torch.equal(o, p.dequantize_recompose(ref, t)), f"reconstruction differs for {p.shape}"


def test_batch_compress_equals_single():
    from paper_2609_00205_amd import Batch, decompress
    shapes = [(33, 17, 65), (17, 17, 17), (65, 65, 33)]
    batch = Batch(shapes, dtype=torch.float32, block=17)
    xs = _fields(shapes, torch.float32, 200)
    tols = _tols(batch, xs)
    bufs = batch.compress(xs, tols, use_graph=True)
    for p, x, t, buf in zip(batch.plans, xs, tols, bufs):
        assert buf == p.compress(x, t)
        xr = decompress(buf)
        err = (xr.double() - x.double()).abs()
        assert float(err.max()) <= float(t.max()) * (1 + 1e-12)


def test_batch_overflow_count():
    from paper_2609_00205_amd import Batch
    shapes = [(17, 17, 17), (33, 17, 17)]
    batch = Batch(shapes, dtype=torch.float64, block=17)
    xs = _fields(shapes, torch.float64, 300)
    xs[1] *= 1e12
    tols = [p.tolmap_from_boxes([], 1e-6) for p in batch.plans]
    _, nbad = batch.decompose_quantize(xs, tols, check=True)
    assert nbad == 1


ORACLE_CASES = [
    ([(33, 17, 65), (65, 33, 33), (17, 33, 17)], torch.float32, 17, None, 0),
    ([(33, 65, 33), (17, 17, 33)], torch.float64, 17, None, 0),
    ([(33, 33, 65), (65, 17, 33)], torch.float32, 9, None, 0),
    ([(33, 33, 33), (65, 33, 33)], torch.float64, 9, 1, 2),          # global levels per field
    ([(33, 17, 65), (65, 33, 33), (17, 33, 17)], torch.float32, 17, None, 0, True),   # nested pairs
    ([(33, 33, 33), (65, 33, 17)], torch.float64, 17, 2, 1, True),
    ([(33, 65, 33), (65, 33, 33)], torch.float32, 33, None, 0),      # 33-node blocks
]


@pytest.mark.parametrize("case", ORACLE_CASES, ids=_id)
def test_batch_matches_oracle(case):
    """Batched codes and reconstructions against the oracle directly.  The
    GPU's coefficients (not an output of the batch) lie within the
    coefficient tolerance e = 1e-6 / 1e-13 of max|x| of the oracle's, so a
    code may differ from the oracle's quantization of its own coefficient by
    at most e / Delta + 1, and where e / Delta < 1/2 only where a bin edge
    lies within e of the oracle's coefficient (count printed);
    reconstructions equal the oracle's recomposition of the dequantized batch
    codes; every voxel within its bound."""
    from oracle import mgard, roi
    from paper_2609_00205_amd import Batch
    shapes, dt, b, L, M = case[:5]
    nested = len(case) > 5 and case[5]
    print("case", _id(case), flush=True)
    batch = Batch(shapes, dtype=dt, block=b, L=L, M=M, nested=nested)
    xs = _fields(shapes, dt, 700)
    tols = _tols(batch, xs)
    codes = batch.decompose_quantize(xs, tols, use_graph=True)
    outs = batch.dequantize_recompose(codes, tols, use_graph=True)
    torch.cuda.synchronize()
    ctol = 1e-6 if dt == torch.float32 else 1e-13
    for p, x, t, c, o in zip(batch.plans, xs, tols, codes, outs):
        xn = x.cpu().double().numpy()
        h = mgard.hierarchy(p.shape, b, p.L, p.M, nested)
        co = mgard.decompose(xn, b, p.L, p.M, nested=nested)
        tol1 = t.cpu().numpy() if p.L > 0 else float(t.cpu().numpy().ravel()[0])
        delta = roi.node_delta(h, tol1, p.eta)
        ref = roi.quantize(co, delta)
        got = c.cpu().numpy().astype(np.int64)
        flips = got != ref
        r = co * (1.0 / delta)
        edge = np.abs(r - np.floor(r) - 0.5) * delta
        scale = float(np.abs(xn).max())
        print(f"field {p.shape} L={p.L}: codes across a bin edge {int(flips.sum())} of {got.size}")
        reach = ctol * scale / delta
        assert np.all(np.abs(got - ref) <= reach + 1)
        near = flips & (reach < 0.5)
        assert np.all(edge[near] <= ctol * scale)
        xr_ref = mgard.recompose(roi.dequantize(got, delta), p.shape, b, p.L, p.M, nested)
        on = o.cpu().double().numpy()
        assert float(np.abs(on - xr_ref).max()) <= ctol * max(scale, float(np.abs(xr_ref).max()))
        n = p.shape
        box = (n[0] // 4, n[1] // 4, n[2] // 4, n[0] // 2 + 1, n[1] // 2 + 1, n[2] // 2 + 1, 1e-5 * scale)
        vt = roi.voxel_tolerance_from_boxes(n, [box], 1e-3 * scale)
        assert np.all(np.abs(on - xn) <= vt)
