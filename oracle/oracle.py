"""ctypes binding of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pcc_oracle.c")
_LIB_NAME = "liborc.so"

MODE_VP, MODE_SC, MODE_HF = 0, 1, 2
NONE, SAFE, PB, PC = 0, 1, 2, 3
_MODES = {"vp": 0, "sc": 1, "hf": 2}


def lib_path() -> str:
    return os.path.join(HERE, _LIB_NAME)


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liborc.so with gcc."""
    out = lib_path()
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-Wno-unused-parameter", "-o", tmp, SRC, "-ldl", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


class _Params(C.Structure):
    _fields_ = [("b", C.c_double), ("xi", C.c_double), ("mode", C.c_int32),
                ("m_bits", C.c_int32), ("optimizer", C.c_int32),
                ("margin_policy", C.c_int32), ("lr", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double),
                ("adam_eps", C.c_double), ("max_iters", C.c_int64),
                ("loss_tol", C.c_double), ("box", C.c_double * 3)]


class _Consts(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("rs", "rv", "b2", "rs2", "rv2", "eps_q", "qstep", "delta_q",
                 "xi_p", "delta_t", "bm", "bp", "bm2", "bp2")]


class _Pair(C.Structure):
    _fields_ = [("i", C.c_uint32), ("j", C.c_uint32), ("d2", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int64),
                ("n_pairs", C.c_int64), ("n_safe", C.c_int64), ("n_pb", C.c_int64),
                ("n_pc", C.c_int64), ("n_active", C.c_int64),
                ("n_editable", C.c_int64), ("n_flagged", C.c_int64),
                ("loss0", C.c_double), ("loss_final", C.c_double),
                ("viol0", C.c_int64), ("viol_final", C.c_int64),
                ("labels", C.POINTER(C.c_int32)), ("safe_labels", C.POINTER(C.c_int32)),
                ("n_a", C.c_int64), ("a_i", C.POINTER(C.c_uint32)),
                ("a_j", C.POINTER(C.c_uint32)), ("a_type", C.POINTER(C.c_uint8)),
                ("a_thr", C.POINTER(C.c_uint8)),
                ("n_e", C.c_int64), ("e_ids", C.POINTER(C.c_uint32)),
                ("p", C.POINTER(C.c_double)), ("loss_hist", C.POINTER(C.c_double)),
                ("viol_hist", C.POINTER(C.c_int64)), ("stream", C.POINTER(C.c_uint8)),
                ("stream_len", C.c_int64)]


_lib = None
_F3 = C.POINTER(C.c_float) * 3


def _load():
    global _lib
    if _lib is None:
        path = lib_path()
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(path)
        lib.orc_params_default.argtypes = [C.POINTER(_Params)]
        lib.orc_constants.argtypes = [C.POINTER(_Params), C.c_double, C.POINTER(_Consts)]
        lib.orc_classify.argtypes = [C.c_double, C.POINTER(_Consts)]
        lib.orc_classify.restype = C.c_int
        lib.orc_pairs.argtypes = [C.c_int64, _F3, C.POINTER(C.c_double), C.c_double,
                                  C.POINTER(C.POINTER(_Pair))]
        lib.orc_pairs.restype = C.c_int64
        lib.orc_components.argtypes = [C.c_int64, C.POINTER(_Pair), C.c_int64,
                                       C.POINTER(_Consts), C.c_int, C.POINTER(C.c_int32)]
        lib.orc_select.argtypes = [C.c_int, C.c_int64, C.POINTER(_Pair), C.c_int64,
                                   C.POINTER(_Consts), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), _F3, C.POINTER(C.c_double),
                                   C.POINTER(C.POINTER(C.c_uint32)),
                                   C.POINTER(C.POINTER(C.c_uint32)),
                                   C.POINTER(C.POINTER(C.c_uint8))]
        lib.orc_select.restype = C.c_int64
        lib.orc_correct.argtypes = [C.c_int64, _F3, _F3, C.POINTER(_Params), C.POINTER(_Result)]
        lib.orc_correct.restype = C.c_int
        lib.orc_correct_multi.argtypes = [C.c_int64, _F3, _F3, C.POINTER(_Params),
                                          C.POINTER(C.c_double), C.c_int32,
                                          C.POINTER(C.c_int32), C.POINTER(_Result)]
        lib.orc_correct_multi.restype = C.c_int
        lib.orc_result_free.argtypes = [C.POINTER(_Result)]
        lib.orc_decode.argtypes = [C.POINTER(C.c_uint8), C.c_int64, C.c_int64, _F3, _F3]
        lib.orc_decode.restype = C.c_int
        lib.orc_fof_labels.argtypes = [C.c_int64, _F3, C.c_double, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32)]
        lib.orc_fof_labels.restype = C.c_int
        lib.orc_free.argtypes = [C.c_void_p]
        _lib = lib
    return _lib


def _soa(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.ndim == 2 and a.shape[0] == 3
    ptrs = _F3(*[a[k].ctypes.data_as(C.POINTER(C.c_float)) for k in range(3)])
    return a, ptrs


def _box(box) -> C.Array:
    return (C.c_double * 3)(*[float(v) for v in (box or (0.0, 0.0, 0.0))])


def _params(b, xi, mode=MODE_HF, m_bits=16, optimizer="adam", lr=1e-3, beta1=0.9,
            beta2=0.999, adam_eps=1e-8, max_iters=0, loss_tol=0.0, box=None,
            margin="safe") -> _Params:
    p = _Params()
    _load().orc_params_default(C.byref(p))
    p.b, p.xi = float(b), float(xi)
    p.mode = _MODES[mode] if isinstance(mode, str) else int(mode)
    p.m_bits = int(m_bits)
    p.optimizer = {"adam": 0, "sgd": 1}[optimizer]
    p.margin_policy = {"safe": 0, "paper": 1}[margin]
    p.lr, p.beta1, p.beta2, p.adam_eps = lr, beta1, beta2, adam_eps
    p.max_iters = int(max_iters)
    p.loss_tol = float(loss_tol)
    for k, v in enumerate(box or (0.0, 0.0, 0.0)):
        p.box[k] = float(v)
    return p


def constants(b, xi, m_bits=16, maxabs=1.0, margin="safe") -> Dict[str, float]:
    p = _params(b, xi, m_bits=m_bits, margin=margin)
    c = _Consts()
    _load().orc_constants(C.byref(p), float(maxabs), C.byref(c))
    return {k: getattr(c, k) for k, _ in _Consts._fields_}


def _consts_struct(d: Dict[str, float]) -> _Consts:
    c = _Consts()
    for k, _ in _Consts._fields_:
        setattr(c, k, d[k])
    return c


def classify(d2, consts: Dict[str, float]) -> np.ndarray:
    lib = _load()
    c = _consts_struct(consts)
    d2 = np.atleast_1d(np.asarray(d2, dtype=np.float64))
    return np.array([lib.orc_classify(float(v), C.byref(c)) for v in d2], dtype=np.int8)


def pairs(pos: np.ndarray, box=None, r2: float = 0.0):
    """All pairs i < j within sqrt(r2): (i, j, d2) sorted by (i, j)."""
    lib = _load()
    pos, ptr = _soa(pos)
    out = C.POINTER(_Pair)()
    n = pos.shape[1]
    cnt = lib.orc_pairs(n, ptr, _box(box), float(r2), C.byref(out))
    if cnt < 0:
        raise MemoryError("oracle pair search")
    if cnt == 0:
        lib.orc_free(out)
        return (np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.float64))
    buf = np.ctypeslib.as_array(C.cast(out, C.POINTER(C.c_uint8)), shape=(cnt * 16,)).copy()
    lib.orc_free(out)
    rec = buf.view(np.dtype([("i", "<u4"), ("j", "<u4"), ("d2", "<f8")]))
    return rec["i"].copy(), rec["j"].copy(), rec["d2"].copy()


def _pair_array(i, j, d2):
    arr = np.zeros(len(i), dtype=np.dtype([("i", "<u4"), ("j", "<u4"), ("d2", "<f8")]))
    arr["i"], arr["j"], arr["d2"] = i, j, d2
    return arr


def components(n, i, j, d2, consts, which: str) -> np.ndarray:
    """which = 'safe' (safe links) or 'fof' (all links)."""
    lib = _load()
    arr = _pair_array(i, j, d2)
    lab = np.zeros(max(n, 1), dtype=np.int32)
    lib.orc_components(n, arr.ctypes.data_as(C.POINTER(_Pair)), len(arr),
                       C.byref(_consts_struct(consts)), 0 if which == "safe" else 1,
                       lab.ctypes.data_as(C.POINTER(C.c_int32)))
    return lab[:n]


def select(mode, n, i, j, d2, consts, safe_labels, fof_labels, recon, box=None):
    lib = _load()
    arr = _pair_array(i, j, d2)
    recon, rptr = _soa(recon)
    ai = C.POINTER(C.c_uint32)()
    aj = C.POINTER(C.c_uint32)()
    at = C.POINTER(C.c_uint8)()
    sl = np.ascontiguousarray(safe_labels, dtype=np.int32)
    fl = np.ascontiguousarray(fof_labels, dtype=np.int32)
    na = lib.orc_select(_MODES[mode] if isinstance(mode, str) else int(mode), n,
                        arr.ctypes.data_as(C.POINTER(_Pair)), len(arr),
                        C.byref(_consts_struct(consts)),
                        sl.ctypes.data_as(C.POINTER(C.c_int32)),
                        fl.ctypes.data_as(C.POINTER(C.c_int32)), rptr, _box(box),
                        C.byref(ai), C.byref(aj), C.byref(at))
    res = (np.ctypeslib.as_array(ai, shape=(max(na, 1),))[:na].copy(),
           np.ctypeslib.as_array(aj, shape=(max(na, 1),))[:na].copy(),
           np.ctypeslib.as_array(at, shape=(max(na, 1),))[:na].copy())
    for ptr in (ai, aj, at):
        lib.orc_free(ptr)
    return res


@dataclasses.dataclass
class OracleResult:
    status: int
    iters: int
    stats: Dict[str, float]
    labels: np.ndarray
    safe_labels: np.ndarray
    a_i: np.ndarray
    a_j: np.ndarray
    a_type: np.ndarray
    a_thr: np.ndarray       # threshold index of each active pair
    e_ids: np.ndarray
    p: np.ndarray           # (3, N) float64
    loss_hist: np.ndarray
    viol_hist: np.ndarray
    stream: bytes


def _arr(ptr, n, dtype):
    if n <= 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def correct(orig, recon, b, xi, mode=MODE_HF, box=None, **kw) -> OracleResult:
    """The correction at one linking length b, or at several (b a sequence:
    the union of every threshold's constraints); with several, the result's
    labels_all holds the FoF labels at each b."""
    lib = _load()
    orig, optr = _soa(orig)
    recon, rptr = _soa(recon)
    n = orig.shape[1]
    multi = isinstance(b, (list, tuple, np.ndarray))
    p = _params(b[0] if multi else b, xi, mode=mode, box=box, **kw)
    r = _Result()
    labels_all = None
    if multi:
        bl = (C.c_double * len(b))(*[float(v) for v in b])
        labels_all = np.zeros((len(b), max(n, 1)), dtype=np.int32)
        st = lib.orc_correct_multi(n, optr, rptr, C.byref(p), bl, len(b),
                                   labels_all.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(r))
    else:
        st = lib.orc_correct(n, optr, rptr, C.byref(p), C.byref(r))
    try:
        if st < 0:
            raise ValueError("oracle rejected the input: status %d" % st)
        stats = {k: getattr(r, k) for k in ("n_pairs", "n_safe", "n_pb", "n_pc", "n_active",
                                             "n_editable", "n_flagged", "loss0",
                                             "loss_final", "viol0", "viol_final")}
        res = OracleResult(
            status=r.status, iters=r.iters, stats=stats,
            labels=_arr(r.labels, n, np.int32), safe_labels=_arr(r.safe_labels, n, np.int32),
            a_i=_arr(r.a_i, r.n_a, np.uint32), a_j=_arr(r.a_j, r.n_a, np.uint32),
            a_type=_arr(r.a_type, r.n_a, np.uint8), a_thr=_arr(r.a_thr, r.n_a, np.uint8),
            e_ids=_arr(r.e_ids, r.n_e, np.uint32),
            p=_arr(r.p, 3 * n, np.float64).reshape(3, n),
            loss_hist=_arr(r.loss_hist, r.iters + 1, np.float64),
            viol_hist=_arr(r.viol_hist, r.iters + 1, np.int64),
            stream=bytes(_arr(r.stream, r.stream_len, np.uint8).tobytes()))
    finally:
        lib.orc_result_free(C.byref(r))
    if multi:
        res.labels_all = labels_all[:, :n]
    return res


def decode(stream: bytes, recon: np.ndarray) -> np.ndarray:
    lib = _load()
    recon, rptr = _soa(recon)
    n = recon.shape[1]
    out = np.zeros((3, n), dtype=np.float32)
    optr = _F3(*[out[k].ctypes.data_as(C.POINTER(C.c_float)) for k in range(3)])
    buf = np.frombuffer(stream, dtype=np.uint8).copy()
    st = lib.orc_decode(buf.ctypes.data_as(C.POINTER(C.c_uint8)), len(buf), n, rptr, optr)
    if st != 0:
        raise ValueError("oracle decode failed: %d" % st)
    return out


def fof_labels(pos: np.ndarray, b: float, box=None) -> np.ndarray:
    lib = _load()
    pos, ptr = _soa(pos)
    n = pos.shape[1]
    lab = np.zeros(max(n, 1), dtype=np.int32)
    if lib.orc_fof_labels(n, ptr, float(b), _box(box), lab.ctypes.data_as(C.POINTER(C.c_int32))):
        raise MemoryError("oracle fof")
    return lab[:n]
