"""The entry point that allocates nothing (bm_huffman_encode_device), through
the C ABI: its stream equals bm_huffman_encode's byte for byte, on two calls
in a row (the second smaller, so stale work arrays of the first would show),
into an aligned and a misaligned device destination; a short buffer returns
BM_ECAPACITY with the size needed and writes nothing; n beyond the fixed
maximum is refused before any device work."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _codes(n, seed, scale=4.0):
    rng = np.random.default_rng(seed)
    q = np.rint(rng.laplace(0, scale, n)).astype(np.int64)
    k = max(1, n // 5000)
    q[rng.choice(n, k, replace=False)] = rng.integers(-(1 << 20), 1 << 20, k)
    return torch.from_numpy(q.astype(np.int32)).cuda()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_00205_amd import _lib
    _lib.lib()


@pytest.mark.parametrize("offset", [0, 1, 3], ids=["aligned", "off1", "off3"])
def test_no_alloc_encoder_equals_encoder(offset):
    from paper_2609_00205_amd import api
    for n, seed in [(1_000_003, 1), (50_001, 2), (4096, 3), (1, 4)]:
        print("n", n, "offset", offset, flush=True)
        codes = _codes(n, seed)
        ref = bytes(api.huffman_encode(codes))
        buf = torch.full((len(ref) + 64 + offset,), 0xAB, dtype=torch.uint8, device="cuda")
        out = buf[offset:]
        nb = api.huffman_encode_device(codes, out)
        torch.cuda.synchronize()
        assert nb == len(ref)
        assert bytes(out[:nb].cpu().numpy().tobytes()) == ref
        assert bool((out[nb:] == 0xAB).all()) and bool((buf[:offset] == 0xAB).all())
        dec = api.huffman_decode(ref, n)
        assert torch.equal(dec, codes)


def test_no_alloc_encoder_short_buffer_and_limit():
    from paper_2609_00205_amd import api, _lib
    codes = _codes(100_000, 5)
    ref = bytes(api.huffman_encode(codes))
    out = torch.full((len(ref) - 1,), 0x5A, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.BMError) as e:
        api.huffman_encode_device(codes, out)
    assert e.value.code == -5 and e.value.needed == len(ref)
    assert bool((out == 0x5A).all())
    # beyond 2^28 codes: refused before any device work (the pointer is not read)
    import ctypes as C
    got = C.c_size_t(0)
    st = _lib.lib().bm_huffman_encode_device(C.c_void_p(codes.data_ptr()), (1 << 28) + 1,
                                            C.c_void_p(out.data_ptr()), out.numel(), C.byref(got), None)
    assert st == -1
