"""Python binding of libckks_lt.so, the MI355X library for homomorphic linear
transformations in RNS-CKKS (triple-hoisted BSGS, Algorithm 2 of arXiv
2605.17222, and the plain BSGS / diagonal methods it is compared with).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libckks_lt.so.  Device buffers are torch tensors (uint64 words held
in int64 tensors on a ROCm device); streams are torch.cuda streams.  The
functions keep the names and argument order of include/ckks_lt.h.  If the
library is not built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libckks_lt.so")

CKKS_OK = 0
CKKS_E_INVALID_ARG = -1
CKKS_E_UNSUPPORTED = -2
CKKS_E_WORKSPACE = -3
CKKS_E_DEVICE = -4
CKKS_E_NOMEM = -5
CKKS_E_TIMEOUT = -6
CKKS_E_CANCELLED = -7
CKKS_PENDING = 1
CKKS_RUNNING = 2

CKKS_SERVER_DEVICE = 0
CKKS_SERVER_SIMULATED = 1

CKKS_LT_NAIVE = 0
CKKS_LT_BSGS = 1
CKKS_LT_TH_BSGS = 2
CKKS_LT_DH_BSGS = 3

EXPORTED = [
    "ckks_strerror", "ckks_params_create", "ckks_params_destroy", "ckks_params_info", "ckks_lt_workspace_size",
    "ckks_lt_eval", "ckks_op_ntt", "ckks_op_decompose", "ckks_op_moddown", "ckks_op_rescale",
    "ckks_op_workspace_size", "ckks_op_keyswitch", "ckks_op_automorph", "ckks_profile_enable", "ckks_profile_read",
    "ckks_lt_batch_workspace_size", "ckks_lt_eval_batch", "ckks_lt_cost_model", "ckks_lt_autotune",
    "ckks_lt_predict", "ckks_server_create", "ckks_server_add_ring", "ckks_server_submit", "ckks_server_poll",
    "ckks_server_result", "ckks_server_cancel", "ckks_server_wait_all", "ckks_server_stats", "ckks_server_destroy",
    "ckks_encode_workspace_size", "ckks_encode", "ckks_th_traffic_model", "ckks_packed_poly_bytes", "ckks_pack",
    "ckks_lt_eval_noalloc",
]

# Largest workspace ckks_lt_eval_noalloc serves (its per-device scratch array).
CKKS_LT_NOALLOC_MAX_WS = 64 << 20

KERNELS = ["ntt_fwd_col", "ntt_fwd_row", "ntt_inv_row", "ntt_inv_col", "bconv", "keyswitch", "ptmac",
           "automorph", "keyswitch_gather", "encode_fft", "ksmac"]


class CkksError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, strerror(code), code))


_u64p = ctypes.POINTER(ctypes.c_uint64)


class ParamsDesc(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_int), ("n_q", ctypes.c_int), ("q", _u64p), ("n_p", ctypes.c_int),
                ("p", _u64p), ("dnum", ctypes.c_int), ("psi", _u64p)]


class Ct(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("scale", ctypes.c_double), ("c0", ctypes.c_void_p),
                ("c1", ctypes.c_void_p)]


class Diags(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int), ("n2", ctypes.c_int), ("n3", ctypes.c_int), ("n_diag", ctypes.c_int),
                ("pt", ctypes.POINTER(ctypes.c_void_p)), ("pt_scale", ctypes.c_double), ("stride", ctypes.c_int),
                ("centre", ctypes.c_int), ("slots", ctypes.POINTER(ctypes.c_void_p)), ("pt_packed", ctypes.c_int)]


class EncodeItem(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_void_p), ("rot", ctypes.c_int32), ("out", ctypes.c_void_p),
                ("coef", ctypes.c_void_p)]


class RotKeys(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("rot", ctypes.POINTER(ctypes.c_int32)),
                ("key", ctypes.POINTER(ctypes.c_void_p)), ("packed", ctypes.c_int)]


class LtCost(ctypes.Structure):
    _fields_ = [("modmul", ctypes.c_double), ("ntt_limbs", ctypes.c_double), ("decompose", ctypes.c_double),
                ("moddown", ctypes.c_double), ("keyswitch", ctypes.c_double), ("keys", ctypes.c_int),
                ("key_bytes", ctypes.c_double), ("pt_bytes", ctypes.c_double)]


class LtRates(ctypes.Structure):
    _fields_ = [("ntt_limb_s", ctypes.c_double), ("bconv_product_s", ctypes.c_double),
                ("hbm_bytes_per_s", ctypes.c_double), ("layer_s", ctypes.c_double)]


class LtItem(ctypes.Structure):
    _fields_ = [("in_", Ct), ("diags", Diags), ("keys", ctypes.POINTER(RotKeys)), ("out", Ct),
                ("status", ctypes.c_int)]


class ThParallelism(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int) for f in ("m1", "l1", "m2", "l2", "m3", "m4", "l3", "m5", "l4", "m6", "l5")]


class ThTraffic(ctypes.Structure):
    _fields_ = [("phase_limbs", ctypes.c_double * 6), ("twiddle_limbs", ctypes.c_double),
                ("matrix_limbs", ctypes.c_double), ("key_limbs", ctypes.c_double), ("read_limbs", ctypes.c_double),
                ("write_limbs", ctypes.c_double), ("total_limbs", ctypes.c_double), ("total_bytes", ctypes.c_double)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("backend", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t), ("max_batch", ctypes.c_int),
                ("max_inflight", ctypes.c_int), ("queue_timeout_s", ctypes.c_double),
                ("simulated_service_s", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("ring", ctypes.c_int), ("in_", Ct), ("diags", Diags), ("out", Ct), ("sim_ws_bytes", ctypes.c_size_t)]


class ServerStat(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_long), ("failed", ctypes.c_long), ("rejected", ctypes.c_long),
                ("queued", ctypes.c_long), ("inflight", ctypes.c_long), ("batches", ctypes.c_long),
                ("max_batch", ctypes.c_long), ("max_inflight", ctypes.c_long), ("arena_in_use", ctypes.c_size_t),
                ("arena_peak", ctypes.c_size_t), ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("mean_s", ctypes.c_double), ("span_s", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built.

    torch is imported first: its wheel carries its own HIP runtime, and the
    library's HIP calls must bind to that same runtime (loaded first, it
    serves both), or the process would start two runtimes on one device and
    torch's tensors and streams would belong to the other one."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libckks_lt.so is not built (run paper_2605_17222_amd/build.py)")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        L.ckks_strerror.restype = ctypes.c_char_p
        L.ckks_strerror.argtypes = [ctypes.c_int]
        L.ckks_params_create.argtypes = [ctypes.POINTER(ParamsDesc), ctypes.POINTER(ctypes.c_void_p)]
        L.ckks_params_destroy.argtypes = [ctypes.c_void_p]
        L.ckks_params_destroy.restype = None
        L.ckks_params_info.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int)] * 3
        L.ckks_params_info.restype = None
        L.ckks_lt_workspace_size.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Diags), ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_size_t)]
        L.ckks_lt_eval.argtypes = [ctypes.c_void_p, ctypes.POINTER(Ct), ctypes.POINTER(Diags),
                                   ctypes.POINTER(RotKeys), ctypes.c_int, ctypes.POINTER(Ct), ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.c_void_p]
        L.ckks_lt_eval_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(Ct), ctypes.POINTER(Diags),
                                           ctypes.POINTER(RotKeys), ctypes.c_int, ctypes.POINTER(Ct),
                                           ctypes.c_void_p]
        L.ckks_op_ntt.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]
        L.ckks_op_decompose.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.ckks_op_moddown.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.ckks_op_rescale.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.ckks_op_workspace_size.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.ckks_op_keyswitch.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        L.ckks_op_automorph.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        L.ckks_profile_enable.argtypes = [ctypes.c_int]
        L.ckks_profile_read.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        L.ckks_lt_batch_workspace_size.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(LtItem),
                                                   ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.ckks_lt_eval_batch.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(LtItem), ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.ckks_lt_cost_model.argtypes = [ctypes.c_int] * 8 + [ctypes.POINTER(LtCost)]
        L.ckks_lt_predict.argtypes = [ctypes.c_int] * 8 + [ctypes.POINTER(LtRates), ctypes.POINTER(ctypes.c_double)]
        L.ckks_lt_autotune.argtypes = [ctypes.c_int] * 6 + [ctypes.POINTER(LtRates)] + \
            [ctypes.POINTER(ctypes.c_int)] * 3 + [ctypes.POINTER(ctypes.c_double)]
        L.ckks_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(ctypes.c_void_p)]
        L.ckks_server_add_ring.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(RotKeys),
                                           ctypes.POINTER(ctypes.c_int)]
        L.ckks_server_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.ckks_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_double)]
        L.ckks_server_result.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Ct)]
        L.ckks_server_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.ckks_server_wait_all.argtypes = [ctypes.c_void_p]
        L.ckks_server_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ServerStat)]
        L.ckks_server_destroy.argtypes = [ctypes.c_void_p]
        L.ckks_server_destroy.restype = None
        L.ckks_th_traffic_model.argtypes = [ctypes.c_int] * 8 + [ctypes.POINTER(ThParallelism),
                                                                 ctypes.POINTER(ThTraffic)]
        L.ckks_packed_poly_bytes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]
        L.ckks_pack.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.ckks_encode_workspace_size.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.ckks_encode.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(EncodeItem), ctypes.c_double,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().ckks_strerror(code).decode()
    except RuntimeError:
        return "error %d" % code


def _check(code: int, what: str):
    if code != CKKS_OK:
        raise CkksError(code, what)


def _ptr(t) -> Optional[int]:
    """Device address of a tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Params:
    """Owns a ckks_params* created by ckks_params_create."""

    def __init__(self, handle: int, log_n: int, q: Sequence[int], p: Sequence[int]):
        self.handle = handle
        self.log_n = log_n
        self.n = 1 << log_n
        self.q = tuple(q)
        self.p = tuple(p)
        self.alpha = len(p)
        self.max_level = len(q) - 1

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                lib().ckks_params_destroy(ctypes.c_void_p(self.handle))
            except Exception:
                pass
            self.handle = None

    @property
    def _as_parameter_(self):
        return ctypes.c_void_p(self.handle)


def ckks_params_create(log_n: int, q: Sequence[int], p: Sequence[int], dnum: int,
                       psi: Optional[Sequence[int]] = None) -> Params:
    qa = (ctypes.c_uint64 * len(q))(*q)
    pa = (ctypes.c_uint64 * len(p))(*p)
    psa = (ctypes.c_uint64 * len(psi))(*psi) if psi is not None else None
    d = ParamsDesc(log_n, len(q), ctypes.cast(qa, _u64p), len(p), ctypes.cast(pa, _u64p), dnum,
                   ctypes.cast(psa, _u64p) if psa is not None else None)
    h = ctypes.c_void_p()
    _check(lib().ckks_params_create(ctypes.byref(d), ctypes.byref(h)), "ckks_params_create")
    return Params(h.value, log_n, q, p)


def ckks_params_info(params: Params) -> Tuple[int, int, int]:
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib().ckks_params_info(params, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


class Packed:
    """A device buffer in the packed layout of ckks_pack (a uint8 tensor):
    pass it wherever a key or a TH-BSGS plaintext goes."""

    def __init__(self, t):
        self.t = t

    def data_ptr(self) -> int:
        return self.t.data_ptr()


def _all_packed(xs) -> bool:
    xs = [x for x in xs if x is not None]
    packed = [isinstance(x, Packed) for x in xs]
    if any(packed) and not all(packed):
        raise ValueError("packed and unpacked operands cannot be mixed in one call")
    return bool(xs) and all(packed)


def _diags(split: Sequence[int], pts: Sequence, pt_scale: float, stride: int = 1, centre: int = 0,
           onfly: bool = False):
    """onfly: pts holds slot vectors (complex128 device tensors of N/2
    entries, or None) that the library encodes itself; Packed plaintexts set
    pt_packed."""
    n1, n2, n3 = (list(split) + [1, 1])[:3]
    arr = (ctypes.c_void_p * max(1, len(pts)))(*[_ptr(x) for x in pts])
    p = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    return Diags(n1, n2, n3, len(pts), None if onfly else p, pt_scale, stride, centre, p if onfly else None,
                 0 if onfly else int(_all_packed(pts))), arr


def _keys(keys: Optional[Dict[int, object]]):
    keys = keys or {}
    rots = sorted(keys)
    r = (ctypes.c_int32 * max(1, len(rots)))(*rots)
    k = (ctypes.c_void_p * max(1, len(rots)))(*[_ptr(keys[x]) for x in rots])
    return RotKeys(len(rots), ctypes.cast(r, ctypes.POINTER(ctypes.c_int32)),
                   ctypes.cast(k, ctypes.POINTER(ctypes.c_void_p)), int(_all_packed(list(keys.values())))), (r, k)


def ckks_lt_workspace_size(params: Params, level: int, split: Sequence[int], pts: Sequence, algo: int,
                           stride: int = 1, centre: int = 0, onfly: bool = False) -> int:
    d, keep = _diags(split, pts, 1.0, stride, centre, onfly)
    out = ctypes.c_size_t()
    _check(lib().ckks_lt_workspace_size(params, level, ctypes.byref(d), algo, ctypes.byref(out)),
           "ckks_lt_workspace_size")
    return out.value


def ckks_lt_eval_noalloc(params: Params, level: int, scale: float, c0, c1, split: Sequence[int], pts: Sequence,
                         pt_scale: float, keys: Optional[Dict[int, object]], algo: int, out0, out1, stream=None,
                         stride: int = 1, centre: int = 0, onfly: bool = False) -> Tuple[int, float]:
    """ckks_lt_eval with the library's per-device scratch as its workspace
    (no device allocation; workspaces above CKKS_LT_NOALLOC_MAX_WS raise
    CKKS_E_WORKSPACE).  Returns (out level, out scale)."""
    cin = Ct(level, scale, _ptr(c0), _ptr(c1))
    cout = Ct(level - 1, 0.0, _ptr(out0), _ptr(out1))
    d, keep1 = _diags(split, pts, pt_scale, stride, centre, onfly)
    k, keep2 = _keys(keys)
    _check(lib().ckks_lt_eval_noalloc(params, ctypes.byref(cin), ctypes.byref(d), ctypes.byref(k), algo,
                                      ctypes.byref(cout), _stream(stream)), "ckks_lt_eval_noalloc")
    return cout.level, cout.scale


def ckks_lt_eval(params: Params, level: int, scale: float, c0, c1, split: Sequence[int], pts: Sequence,
                 pt_scale: float, keys: Optional[Dict[int, object]], algo: int, out0, out1, ws, ws_bytes: int,
                 stream=None, stride: int = 1, centre: int = 0, onfly: bool = False) -> Tuple[int, float]:
    """Enqueue out = LT(in); returns (out level, out scale).  onfly: pts are
    slot vectors encoded by the library with pt_scale."""
    cin = Ct(level, scale, _ptr(c0), _ptr(c1))
    cout = Ct(level - 1, 0.0, _ptr(out0), _ptr(out1))
    d, keep1 = _diags(split, pts, pt_scale, stride, centre, onfly)
    k, keep2 = _keys(keys)
    _check(lib().ckks_lt_eval(params, ctypes.byref(cin), ctypes.byref(d), ctypes.byref(k), algo,
                              ctypes.byref(cout), _ptr(ws), ws_bytes, _stream(stream)), "ckks_lt_eval")
    return cout.level, cout.scale


class BatchItem:
    """One LT of a batch (device buffers as tensors or int addresses)."""

    def __init__(self, level, scale, c0, c1, split, pts, pt_scale, keys, out0, out1, stride=1, centre=0,
                 onfly=False):
        self.level, self.scale, self.c0, self.c1 = level, scale, c0, c1
        self.stride, self.centre, self.onfly = stride, centre, onfly
        self.split, self.pts, self.pt_scale, self.keys = split, pts, pt_scale, keys
        self.out0, self.out1 = out0, out1
        self.status = None
        self.out_level, self.out_scale = None, None


def _items(items: Sequence[BatchItem]):
    arr = (LtItem * max(1, len(items)))()
    keep = []
    for t, it in enumerate(items):
        d, k1 = _diags(it.split, it.pts, it.pt_scale, it.stride, it.centre, it.onfly)
        ks, k2 = _keys(it.keys)
        keep += [d, k1, ks, k2]
        arr[t].in_ = Ct(it.level, it.scale, _ptr(it.c0), _ptr(it.c1))
        arr[t].diags = d
        arr[t].keys = ctypes.pointer(ks)
        arr[t].out = Ct(it.level - 1, 0.0, _ptr(it.out0), _ptr(it.out1))
        arr[t].status = 0
    return arr, keep


def ckks_lt_batch_workspace_size(params: Params, items: Sequence[BatchItem], algo: int) -> int:
    arr, keep = _items(items)
    out = ctypes.c_size_t()
    _check(lib().ckks_lt_batch_workspace_size(params, len(items), arr, algo, ctypes.byref(out)),
           "ckks_lt_batch_workspace_size")
    return out.value


def ckks_lt_eval_batch(params: Params, items: Sequence[BatchItem], algo: int, ws, ws_bytes: int, stream=None) -> int:
    """Enqueue every item; fills each item's status, out_level and out_scale.
    Returns the call's code (raises only on argument marshalling errors)."""
    arr, keep = _items(items)
    code = lib().ckks_lt_eval_batch(params, len(items), arr, algo, _ptr(ws), ws_bytes, _stream(stream))
    for t, it in enumerate(items):
        it.status = arr[t].status
        it.out_level, it.out_scale = arr[t].out.level, arr[t].out.scale
    return code


class Server:
    """Owns a ckks_server handle; the ctypes arrays of registered rings are
    kept alive here for the server's lifetime."""

    def __init__(self, budget_bytes: int, max_batch: int = 8, max_inflight: int = 2, simulated: bool = False,
                 queue_timeout_s: float = 0.0, simulated_service_s: float = 0.0):
        cfg = ServerCfg(CKKS_SERVER_SIMULATED if simulated else CKKS_SERVER_DEVICE, budget_bytes, max_batch,
                        max_inflight, queue_timeout_s, simulated_service_s)
        h = ctypes.c_void_p()
        _check(lib().ckks_server_create(ctypes.byref(cfg), ctypes.byref(h)), "ckks_server_create")
        self.handle = h
        self._keep = []

    @property
    def _as_parameter_(self):
        return self.handle

    def close(self):
        if self.handle:
            lib().ckks_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ckks_server_add_ring(server: Server, params: Optional[Params], keys: Optional[Dict[int, object]]) -> int:
    k, keep = _keys(keys)
    server._keep += [k, keep]
    rid = ctypes.c_int()
    _check(lib().ckks_server_add_ring(server, params, ctypes.byref(k), ctypes.byref(rid)), "ckks_server_add_ring")
    return rid.value


def ckks_server_submit(server: Server, ring: int, level: int = 0, scale: float = 0.0, c0=None, c1=None,
                       split: Sequence[int] = (1, 1, 1), pts: Sequence = (), pt_scale: float = 0.0, out0=None,
                       out1=None, sim_ws_bytes: int = 0, stride: int = 1, centre: int = 0,
                       onfly: bool = False) -> int:
    """Queue one TH-BSGS LT; returns the request id (raises if refused)."""
    d, keep = _diags(split, pts, pt_scale, stride, centre, onfly)
    rq = Request(ring, Ct(level, scale, _ptr(c0), _ptr(c1)), d, Ct(level - 1, 0.0, _ptr(out0), _ptr(out1)),
                 sim_ws_bytes)
    rid = ctypes.c_uint64()
    _check(lib().ckks_server_submit(server, ctypes.byref(rq), ctypes.byref(rid)), "ckks_server_submit")
    return rid.value


def ckks_server_poll(server: Server, rid: int) -> Tuple[int, float]:
    """(status, latency seconds or -1)."""
    st, lat = ctypes.c_int(), ctypes.c_double()
    _check(lib().ckks_server_poll(server, rid, ctypes.byref(st), ctypes.byref(lat)), "ckks_server_poll")
    return st.value, lat.value


def ckks_server_result(server: Server, rid: int) -> Tuple[int, float]:
    """(level, scale) of a finished request's output."""
    c = Ct()
    _check(lib().ckks_server_result(server, rid, ctypes.byref(c)), "ckks_server_result")
    return c.level, c.scale


def ckks_server_cancel(server: Server, rid: int) -> int:
    return lib().ckks_server_cancel(server, rid)


def ckks_server_wait_all(server: Server):
    _check(lib().ckks_server_wait_all(server), "ckks_server_wait_all")


def ckks_server_stats(server: Server) -> dict:
    st = ServerStat()
    _check(lib().ckks_server_stats(server, ctypes.byref(st)), "ckks_server_stats")
    return {f: getattr(st, f) for f, _ in ServerStat._fields_}


def ckks_lt_cost_model(log_n: int, level: int, alpha: int, algo: int, split: Sequence[int], word_bits: int = 64) -> dict:
    n1, n2, n3 = (list(split) + [1, 1])[:3]
    c = LtCost()
    _check(lib().ckks_lt_cost_model(log_n, level, alpha, algo, n1, n2, n3, word_bits, ctypes.byref(c)),
           "ckks_lt_cost_model")
    return {f: getattr(c, f) for f, _ in LtCost._fields_}


def ckks_th_traffic_model(log_n: int, level: int, alpha: int, split: Sequence[int], n_diag: int, word_bits: int,
                          par: dict) -> dict:
    """Off-chip limbs of the paper's memory-optimized data path (Table III) for
    the parallelism parameters par (keys m1 l1 m2 l2 m3 m4 l3 m5 l4 m6 l5)."""
    n1, n2, n3 = split
    p = ThParallelism(*[int(par.get(f, 1)) for f, _ in ThParallelism._fields_])
    t = ThTraffic()
    _check(lib().ckks_th_traffic_model(log_n, level, alpha, n1, n2, n3, n_diag, word_bits, ctypes.byref(p),
                                       ctypes.byref(t)), "ckks_th_traffic_model")
    out = {f: getattr(t, f) for f, _ in ThTraffic._fields_ if f != "phase_limbs"}
    out["phase_limbs"] = list(t.phase_limbs)
    return out


def ckks_lt_predict(log_n: int, level: int, alpha: int, algo: int, split: Sequence[int], n_diag: int,
                    rates: Optional[Tuple[float, float, float, float]] = None) -> float:
    """Predicted device seconds of one LT (the library's model)."""
    n1, n2, n3 = (list(split) + [1, 1])[:3]
    t = ctypes.c_double()
    r = ctypes.byref(LtRates(*rates)) if rates else None
    _check(lib().ckks_lt_predict(log_n, level, alpha, algo, n1, n2, n3, n_diag, r, ctypes.byref(t)),
           "ckks_lt_predict")
    return t.value


def ckks_lt_autotune(log_n: int, level: int, alpha: int, algo: int, n_diag: int, max_keys: int = 0,
                     rates: Optional[Tuple[float, float, float, float]] = None):
    """(split, predicted seconds) chosen by the library's cost model."""
    a, b, c, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    r = ctypes.byref(LtRates(*rates)) if rates else None
    _check(lib().ckks_lt_autotune(log_n, level, alpha, algo, n_diag, max_keys, r, ctypes.byref(a), ctypes.byref(b),
                                  ctypes.byref(c), ctypes.byref(t)), "ckks_lt_autotune")
    return (a.value, b.value, c.value), t.value


def ckks_packed_poly_bytes(params: Params) -> int:
    out = ctypes.c_size_t()
    _check(lib().ckks_packed_poly_bytes(params, ctypes.byref(out)), "ckks_packed_poly_bytes")
    return out.value


def ckks_pack(params: Params, polys, stream=None) -> Packed:
    """Packs full PQ polynomials (device int64 tensor [..., alpha+L+1, N]; a
    key [beta_max, 2, kmax, N] or a plaintext [kmax, N]) into a new Packed."""
    import torch
    kmax = params.alpha + params.max_level + 1
    if not polys.is_contiguous() or tuple(polys.shape[-2:]) != (kmax, params.n):
        raise ValueError("ckks_pack: need a contiguous [..., %d, %d] tensor, got %s" % (kmax, params.n,
                                                                                      tuple(polys.shape)))
    count = polys.numel() // (kmax * params.n)
    out = torch.empty(count * ckks_packed_poly_bytes(params), dtype=torch.uint8, device=polys.device)
    _check(lib().ckks_pack(params, count, _ptr(polys), _ptr(out), _stream(stream)), "ckks_pack")
    return Packed(out)


def ckks_encode_workspace_size(params: Params, count: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().ckks_encode_workspace_size(params, count, ctypes.byref(out)), "ckks_encode_workspace_size")
    return out.value


def ckks_encode(params: Params, slots: Sequence, rots: Sequence[int], scale: float, first_prime: int, n_limbs: int,
                outs: Sequence, ws, ws_bytes: int, coefs: Optional[Sequence] = None, stream=None):
    """Enqueue the encoding of slot vectors slots[i] (complex128 device
    tensors of N/2 entries) as rot(z, rots[i]) into outs[i] ([n_limbs][N]
    NTT form); coefs[i] (int64 [N] or None) receives the integers."""
    n = len(slots)
    arr = (EncodeItem * max(1, n))()
    for i in range(n):
        arr[i] = EncodeItem(_ptr(slots[i]), int(rots[i]), _ptr(outs[i]), _ptr(coefs[i]) if coefs else None)
    _check(lib().ckks_encode(params, n, arr, scale, first_prime, n_limbs, _ptr(ws), ws_bytes, _stream(stream)),
           "ckks_encode")


def ckks_op_ntt(params: Params, forward: bool, first_prime: int, n_limbs: int, x, out, stream=None):
    _check(lib().ckks_op_ntt(params, 1 if forward else 0, first_prime, n_limbs, _ptr(x), _ptr(out),
                             _stream(stream)), "ckks_op_ntt")


def ckks_op_workspace_size(params: Params, level: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().ckks_op_workspace_size(params, level, ctypes.byref(out)), "ckks_op_workspace_size")
    return out.value


def ckks_op_decompose(params: Params, level: int, x, digits, ws, ws_bytes: int, stream=None):
    _check(lib().ckks_op_decompose(params, level, _ptr(x), _ptr(digits), _ptr(ws), ws_bytes, _stream(stream)),
           "ckks_op_decompose")


def ckks_op_moddown(params: Params, level: int, rescale: bool, x, out, ws, ws_bytes: int, stream=None):
    _check(lib().ckks_op_moddown(params, level, 1 if rescale else 0, _ptr(x), _ptr(out), _ptr(ws), ws_bytes,
                                 _stream(stream)), "ckks_op_moddown")


def ckks_op_rescale(params: Params, level: int, x, out, ws, ws_bytes: int, stream=None):
    _check(lib().ckks_op_rescale(params, level, _ptr(x), _ptr(out), _ptr(ws), ws_bytes, _stream(stream)),
           "ckks_op_rescale")


def ckks_op_keyswitch(params: Params, level: int, digits, key, rot: int, add, out_a, out_b, stream=None):
    _check(lib().ckks_op_keyswitch(params, level, _ptr(digits), _ptr(key), rot, _ptr(add), _ptr(out_a),
                                   _ptr(out_b), _stream(stream)), "ckks_op_keyswitch")


def ckks_op_automorph(params: Params, rot: int, n_limbs: int, x, out, stream=None):
    _check(lib().ckks_op_automorph(params, rot, n_limbs, _ptr(x), _ptr(out), _stream(stream)),
           "ckks_op_automorph")


def ckks_profile_enable(mask: int):
    _check(lib().ckks_profile_enable(mask), "ckks_profile_enable")


def ckks_profile_read(kernel: int) -> Tuple[int, float, float]:
    """(launches, total ms, total algorithmic bytes) recorded for one kernel."""
    n, ms, b = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    _check(lib().ckks_profile_read(kernel, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)),
           "ckks_profile_read")
    return n.value, ms.value, b.value


# ---- tensor helpers (host <-> device copies of uint64 words) -------------------

def to_device(a, device="cuda"):
    """numpy uint64 array -> int64 torch tensor on the device (same bits)."""
    import numpy as np
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint64:
        raise TypeError("to_device: need uint64 words, got %s" % a.dtype)
    return torch.from_numpy(a.view(np.int64)).to(device)


def to_host(t):
    """int64 torch tensor -> numpy uint64 array (same bits)."""
    import numpy as np
    return t.detach().cpu().numpy().view(np.uint64)


def empty(shape, device="cuda"):
    import torch
    return torch.empty(shape, dtype=torch.int64, device=device)
