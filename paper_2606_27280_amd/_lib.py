"""ctypes declarations of the libhnsearch C ABI (include/hnsearch.h).

Only argument marshalling lives here.  Loading fails loudly when the HIP
library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhnsearch.so")

HN_OK = 0
HN_ERR_INVALID_ARG = -1
HN_ERR_NOT_NORMALIZED = -2
HN_ERR_OOM = -3
HN_ERR_DEVICE = -4
HN_ERR_UNSUPPORTED = -5

HN_PREC_FP32, HN_PREC_BF16, HN_PREC_FP8, HN_PREC_INT8 = 0, 1, 2, 3
HN_SEED_PLAIN, HN_SEED_LEARNED, HN_SEED_WINDOW = 0, 1, 2
HN_SEED_SCAN_BF16, HN_SEED_SCAN_FP32 = 0, 1
HN_MLP_IN, HN_MLP_H, HN_MLP_OUT, HN_MLP_PARAMS = 128, 256, 512, 230400
HN_BUILD_NO_VALIDATE = 1 << 0
HN_NOALLOC_SCRATCH_BYTES = 64 << 20

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_dbl = ctypes.c_double


class SearchOpts(ctypes.Structure):
    _fields_ = [("precision", _i32), ("seed", _i32), ("query_tiles", _i32),
                ("chunk_blocks", _i32), ("survivor_cap", _i64), ("beta", _dbl),
                ("seed_scan", _i32)]


class SearchAux(ctypes.Structure):
    _fields_ = [("seed_idx", _vp), ("seed_sim", _vp), ("threshold", _vp),
                ("survivors", _vp), ("slack", _vp)]


class SearchStats(ctypes.Structure):
    _fields_ = [("survivors", _i64), ("overflow_queries", _i64)]


class AdamWOpts(ctypes.Structure):
    _fields_ = [("lr", _dbl), ("beta1", _dbl), ("beta2", _dbl), ("eps", _dbl),
                ("weight_decay", _dbl)]


class HNError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("hnsearch error %d: %s" % (code, msg))
        self.code = code


# name -> (restype, argtypes); every symbol include/hnsearch.h declares
SIGNATURES = {
    "hn_build_index": (_i32, [_vp, _i64, _i32, _i32, _dbl, _u32, _vp, ctypes.POINTER(_vp)]),
    "hn_free_index": (None, [_vp]),
    "hn_index_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                             ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]),
    "hn_search_top1": (_i32, [_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(SearchOpts),
                              ctypes.POINTER(SearchAux), ctypes.POINTER(SearchStats), _vp]),
    "hn_search_top1_noalloc": (_i32, [_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(SearchOpts),
                                      ctypes.POINTER(SearchAux), _vp]),
    "hn_search_topk": (_i32, [_vp, _vp, _i64, _i32, _vp, _vp, ctypes.POINTER(SearchOpts), _vp]),
    "hn_filter_survivors": (_i32, [_vp, _vp, _i64, _vp, _vp, _i64, ctypes.POINTER(_i64), _vp,
                                   ctypes.POINTER(SearchOpts), _vp]),
    "hn_scan_scores": (_i32, [_vp, _vp, _i64, _i32, _vp, _vp]),
    "hn_bruteforce_top1": (_i32, [_vp, _i64, _i32, _vp, _i64, _vp, _vp, _vp]),
    "hn_profile_begin": (_i32, [_vp]),
    "hn_profile_end": (_i32, [_vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_dbl),
                              ctypes.POINTER(_i64), _i32, ctypes.POINTER(_i32)]),
    "hn_mlp_forward": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "hn_mlp_grad": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "hn_mlp_adamw": (_i32, [_vp, _vp, _vp, _vp, _i64, _i32, ctypes.POINTER(AdamWOpts), _vp]),
    "hn_seed_train": (_i32, [_vp, _vp, _vp, _i64, _i32, _i32, ctypes.POINTER(AdamWOpts), _vp,
                             _vp]),
    "hn_kmeanspp": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "hn_seed_labels": (_i32, [_vp, _vp, _i32, _vp, _i64, _vp, _vp]),
    "hn_set_seed_model": (_i32, [_vp, _vp, _vp, _i32, _vp]),
    "hn_layer_forward": (_i32, [_vp, _i64, _i32, _i32, _dbl, _vp, _vp, _vp]),
    "hn_layer_backward": (_i32, [_vp, _vp, _i64, _i32, _i32, _dbl, _vp, _vp]),
    "hn_multi_plan_create": (_i32, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_i64),
                                    ctypes.POINTER(SearchOpts), ctypes.POINTER(_vp)]),
    "hn_multi_search": (_i32, [_vp, _vp, _vp, _vp, _i32, _vp]),
    "hn_multi_plan_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                  ctypes.POINTER(_i32)]),
    "hn_multi_plan_free": (None, [_vp]),
    "hn_multi_batch_times": (_i32, [_vp, ctypes.POINTER(_dbl), _vp]),
    "hn_set_memory_budget": (_i32, [_i64]),
    "hn_memory_held": (_i64, []),
    "hn_release_scratch": (_i32, [_vp]),
    "hn_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libhnsearch.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libhnsearch.so is not built (expected at %s); run "
                "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != HN_OK:
        msg = lib().hn_last_error()
        raise HNError(rc, msg.decode() if msg else "")
