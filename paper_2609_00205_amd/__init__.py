"""BlockMGARD hot path for AMD MI355X (gfx950).

The computation lives in ``libblockmgard.so`` (hand-written HIP kernels
behind the C ABI in ``include/blockmgard.h``); this package only marshals
arguments.  Importing it does not load the library; the first call does,
and raises if the library has not been built.
"""
__all__ = ["Plan", "Paper8Plan", "Batch", "autotune", "decompress", "compressed_config", "huffman_encode",
           "huffman_decode", "huffman_encode_device", "lossless_times", "huffman_code_lengths", "model_calibrate", "model_predict",
           "select_levels", "DecomposeFn", "RecomposeFn"]


def __getattr__(name):
    if name in ("DecomposeFn", "RecomposeFn"):
        from . import autograd
        return getattr(autograd, name)
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
