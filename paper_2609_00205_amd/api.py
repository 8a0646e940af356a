"""Torch-facing wrappers over the C ABI: device memory and streams come from
PyTorch; every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import BMConfig, BMQStats, call

_DT = {torch.float32: _lib.BM_F32, torch.float64: _lib.BM_F64}
_TD = {_lib.BM_F32: torch.float32, _lib.BM_F64: torch.float64}

# Share of each tolerance kept back for working-precision rounding.
DEFAULT_ETA = {torch.float32: 0.1, torch.float64: 1e-6}


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _writable(buf: bytearray):
    """A ctypes view of a bytearray the library writes into (no copy)."""
    return (C.c_char * len(buf)).from_buffer(buf)


def _take(buf: bytearray, n: int) -> bytearray:
    """buf cut to its first n bytes, in place (the size queries are exact, so
    normally nothing is cut and nothing is copied)."""
    if n < len(buf):
        del buf[n:]
    return buf


def _host_view(buf) -> memoryview:
    """A byte memoryview of a host buffer: any bytes-like object, or a
    contiguous uint8 CPU tensor (pinned ones included), without a copy."""
    if isinstance(buf, torch.Tensor):
        if buf.is_cuda or buf.dtype != torch.uint8 or not buf.is_contiguous() or buf.dim() != 1:
            raise ValueError("a tensor buffer must be a contiguous 1-D uint8 host tensor")
        buf = buf.numpy()
    return memoryview(buf).cast("B")


def _nbytes(buf) -> int:
    return len(buf) if isinstance(buf, bytes) else _host_view(buf).nbytes


def _readable(buf):
    """A pointer argument for a bytes-like container (bytes, bytearray,
    memoryview, a uint8 host tensor)."""
    if isinstance(buf, bytes):
        return buf
    mv = _host_view(buf)
    if mv.readonly:
        return bytes(mv)
    return (C.c_char * mv.nbytes).from_buffer(mv)


def _need(t: torch.Tensor, dtype, shape, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Plan:
    """A decomposition plan: dims, dtype, block size b, L local + M global levels.

    nested=True selects the nested block schedule: block level s uses
    (b-1)/2^(s-1)+1-node blocks over the level-1 block regions (each at
    least 9 nodes per side)."""

    def __init__(self, shape: Sequence[int], dtype=torch.float32, block: int = 17, L: int = 1, M: int = 2,
                 pad_mode: str = "clamp", eta: Optional[float] = None, device=None, nested: bool = False):
        shape = tuple(int(s) for s in shape)
        if len(shape) != 3:
            raise ValueError("3D shapes only")
        self.shape = shape
        self.dtype = dtype
        self.block, self.L, self.M = block, L, M
        self.eta = DEFAULT_ETA[dtype] if eta is None else float(eta)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        cfg = BMConfig(3, (C.c_int64 * 3)(*shape), _DT[dtype], block, L, M, 1 if pad_mode == "zero" else 0, self.eta,
                       int(bool(nested)))
        self.nested = bool(nested)
        self._cfg = cfg
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            call("bm_plan_create", C.byref(cfg), C.byref(h))
        self._h = h
        self._owned = True
        self._query()

    @classmethod
    def _borrow(cls, handle: C.c_void_p, cfg: BMConfig, device) -> "Plan":
        """A view of a plan owned elsewhere (a field of a Batch)."""
        self = cls.__new__(cls)
        self.shape = tuple(int(v) for v in cfg.dims)
        self.dtype = _TD[cfg.dtype]
        self.block, self.L, self.M = cfg.block, cfg.L, cfg.M
        self.nested = bool(cfg.nested)
        self.eta = cfg.eta
        self.device = device
        self._cfg = cfg
        self._h = handle
        self._owned = False
        self._query()
        return self

    def _query(self):
        h, L, M = self._h, self.L, self.M
        pd = (C.c_int64 * 3)()
        call("bm_coeff_shape", h, pd)
        self.coeff_shape = tuple(pd)
        nb = (C.c_int64 * 3)()
        call("bm_block_grid", h, nb)
        self.block_grid = tuple(nb)
        g = (C.c_double * (L + M))()
        call("bm_level_gains", h, g)
        self.gains = list(g)

    @property
    def workspace_bytes(self) -> int:
        """Device memory the plan holds now (bm_workspace_size)."""
        n = C.c_size_t(0)
        call("bm_workspace_size", self._h, C.byref(n))
        return int(n.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and getattr(self, "_owned", False):
            try:
                _lib.lib().bm_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # -- transform -----------------------------------------------------------
    def decompose(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        _need(x, self.dtype, self.shape, "x")
        if out is None:
            out = torch.empty(self.coeff_shape, dtype=self.dtype, device=x.device)
        _need(out, self.dtype, self.coeff_shape, "out")
        call("bm_decompose", self._h, _ptr(x), _ptr(out), _stream(stream))
        return out

    def recompose(self, coeff: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        _need(coeff, self.dtype, self.coeff_shape, "coeff")
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device=coeff.device)
        _need(out, self.dtype, self.shape, "out")
        call("bm_recompose", self._h, _ptr(coeff), _ptr(out), _stream(stream))
        return out

    def decompose_adjoint(self, gcoeff: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        _need(gcoeff, self.dtype, self.coeff_shape, "gcoeff")
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device=gcoeff.device)
        _need(out, self.dtype, self.shape, "out")
        call("bm_decompose_adjoint", self._h, _ptr(gcoeff), _ptr(out), _stream(stream))
        return out

    def recompose_adjoint(self, gx: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        _need(gx, self.dtype, self.shape, "gx")
        if out is None:
            out = torch.empty(self.coeff_shape, dtype=self.dtype, device=gx.device)
        _need(out, self.dtype, self.coeff_shape, "out")
        call("bm_recompose_adjoint", self._h, _ptr(gx), _ptr(out), _stream(stream))
        return out

    # -- ROI and quantization -----------------------------------------------
    def tolmap_from_boxes(self, boxes: Sequence[Sequence[float]], background: float, stream=None) -> torch.Tensor:
        flat = [float(v) for b in boxes for v in b]
        arr = (C.c_double * max(1, len(flat)))(*flat)
        out = torch.empty(self.block_grid, dtype=torch.float64, device=self.device)
        call("bm_tolmap_from_boxes", self._h, arr, len(boxes), float(background), _ptr(out), _stream(stream))
        return out

    def tolmap_from_voxels(self, voxel_tol: torch.Tensor, stream=None) -> torch.Tensor:
        _need(voxel_tol, torch.float64, self.shape, "voxel_tol")
        out = torch.empty(self.block_grid, dtype=torch.float64, device=self.device)
        call("bm_tolmap_from_voxels", self._h, _ptr(voxel_tol), _ptr(out), _stream(stream))
        return out

    def quantize(self, coeff: torch.Tensor, block_tol: torch.Tensor, codes: Optional[torch.Tensor] = None,
                 stats: bool = True, stream=None):
        _need(coeff, self.dtype, self.coeff_shape, "coeff")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        if codes is None:
            codes = torch.empty(self.coeff_shape, dtype=torch.int32, device=coeff.device)
        _need(codes, torch.int32, self.coeff_shape, "codes")
        st = BMQStats()
        call("bm_quantize_roi", self._h, _ptr(coeff), _ptr(block_tol), _ptr(codes),
             C.byref(st) if stats else None, _stream(stream))
        return codes, ({"n_codes": st.n_codes, "n_outliers": st.n_outliers, "max_abs_code": st.max_abs_code}
                       if stats else None)

    def dequantize(self, codes: torch.Tensor, block_tol: torch.Tensor, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
        _need(codes, torch.int32, self.coeff_shape, "codes")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        if out is None:
            out = torch.empty(self.coeff_shape, dtype=self.dtype, device=codes.device)
        _need(out, self.dtype, self.coeff_shape, "out")
        call("bm_dequantize", self._h, _ptr(codes), _ptr(block_tol), _ptr(out), _stream(stream))
        return out

    # -- adjoint-guided bounds for a linear quantity of interest ---------------
    def qoi_deltas(self, g: torch.Tensor, tol_q: float, block_tol: torch.Tensor, stream=None):
        """Per-node Delta keeping <g, x> within tol_q (capped by the block map's
        L-inf Delta); returns (delta, number of coefficients whose width the
        quantity sets, i.e. below the cap)."""
        _need(g, self.dtype, self.shape, "g")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        delta = torch.empty(self.coeff_shape, dtype=torch.float64, device=g.device)
        n = C.c_int64(0)
        call("bm_qoi_deltas", self._h, _ptr(g), float(tol_q), _ptr(block_tol), _ptr(delta), C.byref(n),
             _stream(stream))
        return delta, n.value

    def quantize_delta(self, coeff: torch.Tensor, delta: torch.Tensor, codes: Optional[torch.Tensor] = None,
                       stats: bool = True, stream=None):
        _need(coeff, self.dtype, self.coeff_shape, "coeff")
        _need(delta, torch.float64, self.coeff_shape, "delta")
        if codes is None:
            codes = torch.empty(self.coeff_shape, dtype=torch.int32, device=coeff.device)
        _need(codes, torch.int32, self.coeff_shape, "codes")
        st = BMQStats()
        call("bm_quantize_delta", self._h, _ptr(coeff), _ptr(delta), _ptr(codes), C.byref(st) if stats else None,
             _stream(stream))
        return codes, ({"n_codes": st.n_codes, "n_outliers": st.n_outliers, "max_abs_code": st.max_abs_code}
                       if stats else None)

    def dequantize_delta(self, codes: torch.Tensor, delta: torch.Tensor, out: Optional[torch.Tensor] = None,
                         stream=None) -> torch.Tensor:
        _need(codes, torch.int32, self.coeff_shape, "codes")
        _need(delta, torch.float64, self.coeff_shape, "delta")
        if out is None:
            out = torch.empty(self.coeff_shape, dtype=self.dtype, device=codes.device)
        _need(out, self.dtype, self.coeff_shape, "out")
        call("bm_dequantize_delta", self._h, _ptr(codes), _ptr(delta), _ptr(out), _stream(stream))
        return out

    def decompose_quantize(self, x: torch.Tensor, block_tol: torch.Tensor, codes: Optional[torch.Tensor] = None,
                           check: bool = True, stream=None) -> torch.Tensor:
        """Fused decompose + ROI quantize: codes equal quantize(decompose(x))."""
        _need(x, self.dtype, self.shape, "x")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        if codes is None:
            codes = torch.empty(self.coeff_shape, dtype=torch.int32, device=x.device)
        _need(codes, torch.int32, self.coeff_shape, "codes")
        st = BMQStats()
        call("bm_decompose_quantize", self._h, _ptr(x), _ptr(block_tol), _ptr(codes),
             C.byref(st) if check else None, _stream(stream))
        return codes

    def quant_prepare(self, block_tol: Optional[torch.Tensor], stream=None) -> None:
        """Keep the quantizer tables of block_tol in the plan (bm_quant_prepare):
        later quantizing calls given this same tensor skip building them.  Its
        contents must not change meanwhile; None drops the kept tables."""
        if block_tol is not None:
            _need(block_tol, torch.float64, self.block_grid, "block_tol")
        call("bm_quant_prepare", self._h, _ptr(block_tol) if block_tol is not None else None, _stream(stream))

    def dequantize_recompose(self, codes: torch.Tensor, block_tol: torch.Tensor, out: Optional[torch.Tensor] = None,
                             stream=None) -> torch.Tensor:
        """Fused dequantize + recompose: equals recompose(dequantize(codes))."""
        _need(codes, torch.int32, self.coeff_shape, "codes")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device=codes.device)
        _need(out, self.dtype, self.shape, "out")
        call("bm_dequantize_recompose", self._h, _ptr(codes), _ptr(block_tol), _ptr(out), _stream(stream))
        return out

    # -- per-level timing ------------------------------------------------------
    def timing(self, enable: bool) -> None:
        """Start (reset) or stop recording HIP events around each level."""
        call("bm_timing", self._h, 1 if enable else 0)

    def timing_get(self) -> dict:
        """{"decompose": [ms per level s=1..], "recompose": [...], "quantize": ms, "dequantize": ms,
        "calls": {...}}: totals since timing(True)."""
        k = 2 * (self.L + self.M) + 2
        ms = (C.c_double * k)()
        calls = (C.c_int64 * k)()
        n = C.c_int(0)
        call("bm_timing_get", self._h, ms, calls, k, C.byref(n))
        nl = self.L + self.M
        return {"decompose": [ms[2 * s] for s in range(nl)], "recompose": [ms[2 * s + 1] for s in range(nl)],
                "quantize": ms[2 * nl], "dequantize": ms[2 * nl + 1],
                "calls": {"decompose": [calls[2 * s] for s in range(nl)],
                          "recompose": [calls[2 * s + 1] for s in range(nl)],
                          "quantize": calls[2 * nl], "dequantize": calls[2 * nl + 1]}}

    # -- end to end ----------------------------------------------------------
    def compress(self, x: torch.Tensor, block_tol: torch.Tensor, stream=None, out=None):
        """The container of x under block_tol (bm_compress_plan, then
        bm_compress_write).  Returns a new bytearray of its exact size; or,
        given ``out`` (a writable host buffer: bytearray, numpy array,
        memoryview, or a contiguous 1-D uint8 CPU tensor, e.g. pinned and
        reused, which takes the stream's copy at full PCIe rate), writes into
        it and returns a memoryview of the bytes written.  An ``out`` too
        small raises BMError (BM_ECAPACITY) with the size needed in
        ``.needed`` (the plan stays pending, nothing is written)."""
        _need(x, self.dtype, self.shape, "x")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        # planned once (bm_compress_plan), written into a buffer of its exact size
        need = C.c_size_t(0)
        call("bm_compress_plan", self._h, _ptr(x), _ptr(block_tol), C.byref(need), _stream(stream))
        if out is not None:
            mv = _host_view(out)
            if mv.readonly:
                raise ValueError("out must be writable")
            if mv.nbytes < need.value:
                err = _lib.BMError(_lib.BM_ECAPACITY, f"out holds {mv.nbytes} bytes, the container needs {need.value}")
                err.needed = int(need.value)
                raise err
            got = C.c_size_t(0)
            view = (C.c_char * mv.nbytes).from_buffer(mv)
            call("bm_compress_write", self._h, view, mv.nbytes, C.byref(got))
            del view
            return mv[:got.value]
        buf = bytearray(need.value)
        got = C.c_size_t(0)
        view = _writable(buf)
        call("bm_compress_write", self._h, view, need.value, C.byref(got))
        del view
        return _take(buf, got.value)


def compressed_config(buf) -> dict:
    cfg = BMConfig()
    call("bm_compressed_config", _readable(buf), _nbytes(buf), C.byref(cfg))
    return {"shape": tuple(cfg.dims), "dtype": _TD[cfg.dtype], "block": cfg.block, "L": cfg.L, "M": cfg.M,
            "pad_mode": cfg.pad_mode, "eta": cfg.eta, "nested": bool(cfg.nested)}


def decompress(buf, device=None, stream=None) -> torch.Tensor:
    info = compressed_config(buf)
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = torch.empty(info["shape"], dtype=info["dtype"], device=dev)
    call("bm_decompress", _readable(buf), _nbytes(buf), _ptr(out), _stream(stream))
    return out


def huffman_encode(codes: torch.Tensor, stream=None) -> bytearray:
    """The Huffman stream of int32 device codes (bm_huffman_plan, then
    bm_huffman_write into a buffer of the stream's exact size)."""
    _need(codes, torch.int32, None, "codes")
    need = C.c_size_t(0)
    h = C.c_void_p()
    call("bm_huffman_plan", _ptr(codes), codes.numel(), C.byref(h), C.byref(need), _stream(stream))
    try:
        buf = bytearray(need.value)
        got = C.c_size_t(0)
        view = _writable(buf)
        call("bm_huffman_write", h, view, need.value, C.byref(got))
        del view
    finally:
        _lib.lib().bm_huffman_destroy(h)
    return _take(buf, got.value)


def huffman_encode_device(codes: torch.Tensor, out: torch.Tensor, stream=None) -> int:
    """bm_huffman_encode into a device byte tensor (the entry point that
    allocates nothing); returns the stream size.  When out is too small the
    BMError (BM_ECAPACITY) carries the size needed in ``.needed``."""
    if codes.dtype != torch.int32 or not codes.is_cuda or not codes.is_contiguous():
        raise ValueError("codes: contiguous int32 device tensor")
    if out.dtype != torch.uint8 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out: contiguous uint8 device tensor")
    got = C.c_size_t(0)
    st = _lib.lib().bm_huffman_encode_device(_ptr(codes), int(codes.numel()), _ptr(out), int(out.numel()),
                                             C.byref(got), _stream(stream))
    if st != 0:
        err = _lib.BMError(st, _lib.lib().bm_last_error().decode())
        err.needed = int(got.value)
        raise err
    return int(got.value)


def huffman_decode(buf, n: int, device=None, stream=None) -> torch.Tensor:
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = torch.empty(n, dtype=torch.int32, device=dev)
    call("bm_huffman_decode", _readable(buf), _nbytes(buf), _ptr(out), n, _stream(stream))
    return out


def huffman_code_lengths(hist):
    """Code lengths (uint8 [65536]) of the lossless stage for a histogram of
    65536 symbol counts (bm_huffman_code_lengths; host only)."""
    import numpy as np
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    if h.shape != (65536,):
        raise ValueError("hist: 65536 counts")
    out = np.zeros(65536, np.uint8)
    call("bm_huffman_code_lengths", h.ctypes.data, out.ctypes.data)
    return out


def lossless_times() -> dict:
    """Stage times (ms) of this thread's last Huffman encode and decode
    (bm_lossless_last_times): enc_hist, enc_table, enc_sizes, enc_encode,
    enc_copy, enc_crc, dec_parse, dec_upload, dec_decode, plus enc_n, dec_n."""
    t = _lib.BMLosslessTimes()
    call("bm_lossless_last_times", C.byref(t))
    return {f: getattr(t, f) for f, _ in t._fields_}


def parse_huffman(buf: bytes) -> dict:
    """Split a bm_huffman_encode stream into its arrays (layout in blockmgard.h)."""
    import numpy as np
    hdr = np.frombuffer(buf, dtype=np.int64, count=6, offset=0)
    magic = int(np.frombuffer(buf, dtype=np.uint32, count=1)[0])
    n, nch, nw, nout, npres = (int(v) for v in hdr[1:6])
    o = 48
    psym = np.frombuffer(buf, np.uint16, npres, o); o += 2 * npres
    plen = np.frombuffer(buf, np.uint8, npres, o); o += npres
    lengths = np.zeros(65536, np.uint8)
    lengths[psym.astype(np.int64)] = plen
    offsets = np.frombuffer(buf, np.uint64, nch + 1, o); o += 8 * (nch + 1)
    ooffsets = np.frombuffer(buf, np.uint64, nch + 1, o); o += 8 * (nch + 1)
    words = np.frombuffer(buf, np.uint32, nw, o); o += 4 * nw
    oval = np.frombuffer(buf, np.int32, nout, o)
    return {"magic": magic, "n": n, "nchunks": nch, "lengths": lengths, "offsets": offsets, "words": words,
            "outlier_offsets": ooffsets, "outlier_value": oval}


def autotune(x: torch.Tensor, voxel_tol: torch.Tensor, slack: float = 0.05, reps: int = 3,
             pad_mode: str = "clamp", eta: Optional[float] = None, stream=None, budget_ms: Optional[float] = None):
    """Measured choice of (block, L, M) for field x under the per-voxel absolute
    tolerance voxel_tol (FP64, same shape).  Returns (choice, candidates):
    choice = {"block", "L", "M", "nested"}; candidates = the measured table.

    budget_ms: choose by the rule of Algorithm 1 instead (most global levels,
    then fewest block levels, among the candidates whose pipeline time, fused
    decompose + quantize ("ms") plus the Huffman encode of their codes
    ("lossless_ms"), fits); choice["fits"] tells whether any did (if not, the
    candidate of the shortest pipeline time is returned)."""
    if x.dtype not in _DT:
        raise ValueError("x must be float32 or float64")
    _need(x, x.dtype, None, "x")
    _need(voxel_tol, torch.float64, tuple(x.shape), "voxel_tol")
    eta = DEFAULT_ETA[x.dtype] if eta is None else float(eta)
    cfg = BMConfig(3, (C.c_int64 * 3)(*x.shape), _DT[x.dtype], 17, 1, 1, 1 if pad_mode == "zero" else 0, eta)
    out = BMConfig()
    cap = 128
    table = (_lib.BMCandidate * cap)()
    n = C.c_int(0)
    fits = None
    if budget_ms is None:
        call("bm_autotune", C.byref(cfg), _ptr(x), _ptr(voxel_tol), float(slack), int(reps), C.byref(out), table,
             cap, C.byref(n), _stream(stream))
    else:
        st = _lib.lib().bm_autotune_budget(C.byref(cfg), _ptr(x), _ptr(voxel_tol), float(budget_ms), int(reps),
                                           C.byref(out), table, cap, C.byref(n), _stream(stream))
        if st not in (0, _lib.BM_ERANGE):
            _lib.check(st)
        fits = st == 0
    cands = [{"block": table[i].block, "L": table[i].L, "M": table[i].M, "status": table[i].status,
              "ms": table[i].ms, "ratio": table[i].ratio, "nested": bool(table[i].nested),
              "lossless_ms": table[i].lossless_ms}
             for i in range(min(n.value, cap))]
    choice = {"block": out.block, "L": out.L, "M": out.M, "nested": bool(out.nested)}
    if fits is not None:
        choice["fits"] = fits
    return choice, cands


_MODEL_KEYS = ["blk_lat_ms", "blk_tp", "fblk_lat_ms", "fblk_tp", "fglob_a_ms", "fglob_b_ms", "glob_a_ms",
               "glob_b_ms", "q_slope_ms", "q_lat_ms", "gq_slope_ms", "gq_lat_ms"]


def _model_struct(model: dict) -> "_lib.BMModel":
    m = _lib.BMModel()
    m.dtype = _DT[model["dtype"]] if not isinstance(model["dtype"], int) else model["dtype"]
    m.block = int(model["block"])
    for k in _MODEL_KEYS:
        setattr(m, k, float(model[k]))
    for k in range(4):
        m.huf_a_ms[k] = float(model["huf_a_ms"][k])
        m.huf_b_ms[k] = float(model["huf_b_ms"][k])
    return m


def model_calibrate(dtype=torch.float32, block: int = 17, stream=None) -> dict:
    """Stage fits of the time model on the current device (bm_model_calibrate)."""
    m = _lib.BMModel()
    call("bm_model_calibrate", _DT[dtype], int(block), C.byref(m), _stream(stream))
    out = {"dtype": dtype, "block": m.block}
    for k in _MODEL_KEYS:
        out[k] = float(getattr(m, k))
    out["huf_a_ms"] = [float(m.huf_a_ms[k]) for k in range(4)]
    out["huf_b_ms"] = [float(m.huf_b_ms[k]) for k in range(4)]
    return out


def _cfg(shape, dtype, block, L=1, M=0):
    return BMConfig(3, (C.c_int64 * 3)(*[int(v) for v in shape]), _DT[dtype], int(block), int(L), int(M), 0,
                    DEFAULT_ETA[dtype])


def model_predict(model: dict, shape, L: int, M: int) -> dict:
    """Predicted stage times (ms) of (model's block, L, M) on shape (bm_model_predict)."""
    ms = (C.c_double * 4)()
    cfg = _cfg(shape, model["dtype"], model["block"], L, M)
    call("bm_model_predict", C.byref(_model_struct(model)), C.byref(cfg), ms)
    return {"decompose": ms[0], "quantize": ms[1], "lossless": ms[2], "total": ms[3]}


def select_levels(shape, budget_ms: float, model: dict):
    """Algorithm 1 on the model's predictions (bm_select_levels): returns
    ({"block", "L", "M", "fits"}, [{"block", "L", "M", "ms"}...])."""
    cfg = _cfg(shape, model["dtype"], model["block"])
    out = BMConfig()
    cap = 64
    table = (_lib.BMCandidate * cap)()
    n = C.c_int(0)
    st = _lib.lib().bm_select_levels(C.byref(cfg), C.byref(_model_struct(model)), float(budget_ms), C.byref(out),
                                     table, cap, C.byref(n))
    if st not in (0, _lib.BM_ERANGE):
        _lib.check(st)
    cands = [{"block": table[i].block, "L": table[i].L, "M": table[i].M, "ms": table[i].ms}
             for i in range(min(n.value, cap))]
    return {"block": out.block, "L": out.L, "M": out.M, "fits": st == 0}, cands


class Paper8Plan:
    """The paper's own block form: disjoint 8^3 blocks, L block levels whose
    5^3 coarse outputs are re-assembled into the next level's blocks, then M
    global levels on the assembled coarsest grid (the paper's hybrid; M = 0:
    block levels only).  Coefficients are one flat array (see
    ``bm_p8_create`` and ``bm_p8_create_hybrid``)."""

    def __init__(self, shape: Sequence[int], dtype=torch.float32, L: int = 1, M: int = 0, device=None):
        shape = tuple(int(s) for s in shape)
        if len(shape) != 3:
            raise ValueError("3D shapes only")
        self.shape, self.dtype, self.L, self.M = shape, dtype, int(L), int(M)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            call("bm_p8_create_hybrid", (C.c_int64 * 3)(*shape), _DT[dtype], self.L, self.M, C.byref(h))
        self._h = h
        n = C.c_int64(0)
        call("bm_p8_coeff_size", h, C.byref(n))
        self.coeff_size = int(n.value)
        nb = (C.c_int64 * 3)()
        call("bm_p8_block_grid", h, nb)
        self.block_grid = tuple(nb)
        self.eta = DEFAULT_ETA[dtype]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.lib().bm_p8_destroy(h)
            except Exception:   # interpreter shutdown: the library may be gone already
                pass
            self._h = None

    def decompose(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        _need(x, self.dtype, self.shape, "x")
        if out is None:
            out = torch.empty(self.coeff_size, dtype=self.dtype, device=x.device)
        _need(out, self.dtype, (self.coeff_size,), "out")
        call("bm_p8_decompose", self._h, _ptr(x), _ptr(out), _stream(stream))
        return out

    def recompose(self, coeff: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        _need(coeff, self.dtype, (self.coeff_size,), "coeff")
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device=coeff.device)
        _need(out, self.dtype, self.shape, "out")
        call("bm_p8_recompose", self._h, _ptr(coeff), _ptr(out), _stream(stream))
        return out

    def tolmap_from_voxels(self, voxel_tol: torch.Tensor, stream=None) -> torch.Tensor:
        """Level-1 block map from a per-voxel absolute bound (FP64, logical dims)."""
        _need(voxel_tol, torch.float64, self.shape, "voxel_tol")
        out = torch.empty(self.block_grid, dtype=torch.float64, device=voxel_tol.device)
        call("bm_p8_tolmap_from_voxels", self._h, _ptr(voxel_tol), _ptr(out), _stream(stream))
        return out

    def quantize(self, coeff: torch.Tensor, block_tol: torch.Tensor, stream=None) -> torch.Tensor:
        _need(coeff, self.dtype, (self.coeff_size,), "coeff")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        codes = torch.empty(self.coeff_size, dtype=torch.int32, device=coeff.device)
        call("bm_p8_quantize", self._h, _ptr(coeff), _ptr(block_tol), self.eta, _ptr(codes), _stream(stream))
        return codes

    def dequantize(self, codes: torch.Tensor, block_tol: torch.Tensor, stream=None) -> torch.Tensor:
        _need(codes, torch.int32, (self.coeff_size,), "codes")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        out = torch.empty(self.coeff_size, dtype=self.dtype, device=codes.device)
        call("bm_p8_dequantize", self._h, _ptr(codes), _ptr(block_tol), self.eta, _ptr(out), _stream(stream))
        return out

    def decompose_quantize(self, x: torch.Tensor, block_tol: torch.Tensor, codes: Optional[torch.Tensor] = None,
                           stream=None) -> torch.Tensor:
        """Fused: equal to quantize(decompose(x))."""
        _need(x, self.dtype, self.shape, "x")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        if codes is None:
            codes = torch.empty(self.coeff_size, dtype=torch.int32, device=x.device)
        _need(codes, torch.int32, (self.coeff_size,), "codes")
        call("bm_p8_decompose_quantize", self._h, _ptr(x), _ptr(block_tol), self.eta, _ptr(codes), _stream(stream))
        return codes

    def dequantize_recompose(self, codes: torch.Tensor, block_tol: torch.Tensor, out: Optional[torch.Tensor] = None,
                             stream=None) -> torch.Tensor:
        """Fused: equal to recompose(dequantize(codes))."""
        _need(codes, torch.int32, (self.coeff_size,), "codes")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        if out is None:
            out = torch.empty(self.shape, dtype=self.dtype, device=codes.device)
        _need(out, self.dtype, self.shape, "out")
        call("bm_p8_dequantize_recompose", self._h, _ptr(codes), _ptr(block_tol), self.eta, _ptr(out),
             _stream(stream))
        return out

    def compress(self, x: torch.Tensor, block_tol: torch.Tensor, stream=None) -> bytearray:
        """Container (header, block map, Huffman stream); ``decompress`` reads it."""
        _need(x, self.dtype, self.shape, "x")
        _need(block_tol, torch.float64, self.block_grid, "block_tol")
        need = C.c_size_t(0)
        st = _stream(stream)
        try:
            call("bm_p8_compress", self._h, _ptr(x), _ptr(block_tol), self.eta, None, 0, C.byref(need), st)
        except _lib.BMError as e:
            if e.code != -5:
                raise
        buf = bytearray(need.value)
        got = C.c_size_t(0)
        view = _writable(buf)
        call("bm_p8_compress", self._h, _ptr(x), _ptr(block_tol), self.eta, view, need.value, C.byref(got), st)
        del view
        return _take(buf, got.value)


class Batch:
    """Many fields of one dtype and block size through the fused pipeline in
    few launches (one persistent launch per block level for all fields; for
    33-node blocks one per step of the split block), optionally captured once
    in a HIP graph and replayed.

    L: per-field block levels (default: the most each shape tiles without
    padding, chosen by the library); M: global levels (int or per field);
    nested: the nested block schedule for every field (b = 17: a field's
    17- and 9-node levels run as one pair in one persistent launch).
    """

    def __init__(self, shapes: Sequence[Sequence[int]], dtype=torch.float32, block: int = 17, L=None, M=0,
                 pad_mode: str = "clamp", eta: Optional[float] = None, device=None, nested: bool = False):
        shapes = [tuple(int(v) for v in sh) for sh in shapes]
        nf = len(shapes)
        Ls = [-1] * nf if L is None else ([int(L)] * nf if isinstance(L, int) else [int(v) for v in L])
        Ms = [int(M)] * nf if isinstance(M, int) else [int(v) for v in M]
        self.dtype = dtype
        self.eta = DEFAULT_ETA[dtype] if eta is None else float(eta)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        cfgs = (BMConfig * nf)()
        for i, sh in enumerate(shapes):
            cfgs[i] = BMConfig(3, (C.c_int64 * 3)(*sh), _DT[dtype], block, Ls[i], Ms[i],
                               1 if pad_mode == "zero" else 0, self.eta, 1 if nested else 0)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            call("bm_batch_create", nf, cfgs, C.byref(h))
        self._h = h
        self._cfgs = cfgs
        self.plans = []
        for i in range(nf):
            ph = C.c_void_p()
            call("bm_batch_plan", h, i, C.byref(ph))
            resolved = BMConfig()
            call("bm_plan_config", ph, C.byref(resolved))
            self.plans.append(Plan._borrow(ph, resolved, self.device))
        self._graph_stream = None

    def __len__(self):
        return len(self.plans)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.lib().bm_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    @staticmethod
    def _ptrs(ts) -> "C.Array":
        return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def _run(self, fn, use_graph: bool, stream):
        """Graph capture needs a stream other than the null stream: use a side
        stream ordered after the caller's."""
        cur = stream if stream is not None else torch.cuda.current_stream()
        if not use_graph or cur.cuda_stream != 0:
            return fn(C.c_void_p(cur.cuda_stream))
        if self._graph_stream is None:
            self._graph_stream = torch.cuda.Stream()
        side = self._graph_stream
        side.wait_stream(cur)
        r = fn(C.c_void_p(side.cuda_stream))
        cur.wait_stream(side)
        return r

    def _same_len(self, **lists):
        # the library reads one pointer per field from every array
        for name, v in lists.items():
            if v is not None and len(v) != len(self.plans):
                raise ValueError(f"{name}: {len(v)} entries for a batch of {len(self.plans)} fields")

    def decompose_quantize(self, xs, block_tols, codes=None, use_graph: bool = False, check: bool = False,
                           stream=None):
        """codes[f] = fused decompose + ROI quantize of xs[f]; with check, the
        number of fields whose codes overflowed int32 is returned as well."""
        self._same_len(xs=xs, block_tols=block_tols, codes=codes)
        for p, x, t in zip(self.plans, xs, block_tols):
            _need(x, p.dtype, p.shape, "x")
            _need(t, torch.float64, p.block_grid, "block_tol")
        if codes is None:
            codes = [torch.empty(p.coeff_shape, dtype=torch.int32, device=x.device) for p, x in zip(self.plans, xs)]
        for p, c in zip(self.plans, codes):
            _need(c, torch.int32, p.coeff_shape, "codes")
        nbad = C.c_int(0)
        self._run(lambda st: call("bm_batch_decompose_quantize", self._h, self._ptrs(xs), self._ptrs(block_tols),
                                  self._ptrs(codes), int(use_graph), C.byref(nbad) if check else None, st),
                  use_graph, stream)
        return (codes, nbad.value) if check else codes

    def dequantize_recompose(self, codes, block_tols, outs=None, use_graph: bool = False, stream=None):
        self._same_len(codes=codes, block_tols=block_tols, outs=outs)
        for p, c, t in zip(self.plans, codes, block_tols):
            _need(c, torch.int32, p.coeff_shape, "codes")
            _need(t, torch.float64, p.block_grid, "block_tol")
        if outs is None:
            outs = [torch.empty(p.shape, dtype=p.dtype, device=c.device) for p, c in zip(self.plans, codes)]
        for p, o in zip(self.plans, outs):
            _need(o, p.dtype, p.shape, "out")
        self._run(lambda st: call("bm_batch_dequantize_recompose", self._h, self._ptrs(codes),
                                  self._ptrs(block_tols), self._ptrs(outs), int(use_graph), st), use_graph, stream)
        return outs

    def compress(self, xs, block_tols, use_graph: bool = False, stream=None) -> list:
        nf = len(self.plans)
        self._same_len(xs=xs, block_tols=block_tols)
        for p, x, t in zip(self.plans, xs, block_tols):
            _need(x, p.dtype, p.shape, "x")
            _need(t, torch.float64, p.block_grid, "block_tol")
        cap = (C.c_size_t * nf)(*[64 + int(x.numel()) * x.element_size() * 2 + 8 * int(t.numel()) + (1 << 20)
                                  for x, t in zip(xs, block_tols)])
        bufs = [bytearray(int(c)) for c in cap]
        views = [_writable(b) for b in bufs]
        outp = (C.c_void_p * nf)(*[C.addressof(v) for v in views])
        got = (C.c_size_t * nf)()
        self._run(lambda st: call("bm_batch_compress", self._h, self._ptrs(xs), self._ptrs(block_tols), outp, cap,
                                  got, int(use_graph), st), use_graph, stream)
        del views   # (the buffers cannot be cut while they are exported)
        return [_take(b, got[i]) for i, b in enumerate(bufs)]
