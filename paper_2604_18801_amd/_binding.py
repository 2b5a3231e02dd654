"""ctypes binding of libpcc.so (include/pcc.h): argument marshalling only.

Device arrays are torch tensors on the GPU (torch supplies device memory and
the current HIP stream); host arrays are numpy.  Every computation happens in
the library; when it is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PCC_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("PCC_LIBRARY") or os.path.join(HERE, "libpcc.so")

OK, NOT_CONVERGED = 0, 1
MODES = {"vp": 0, "sc": 1, "hf": 2}
MEM_HOST, MEM_DEVICE = 0, 1
NSTAGES = 10
NKERNELS = 8
KERNEL_NAMES = ("pair_classify", "pair_count", "pair_write", "pgd_step", "pgd_finalize",
                "cell_sort", "pair_csr_sort", "forest")
STAGE_NAMES = ("input_scan", "cell_build", "pair_pass", "labels", "selection", "csr", "pgd",
               "encode_device", "lossless_host", "total_wall")


class PccError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("pcc status %d: %s" % (status, msg))
        self.status = status


class Particles(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("n", C.c_int64),
                ("memspace", C.c_int32), ("reserved", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("b", C.c_double), ("xi", C.c_double), ("mode", C.c_int32),
                ("m_bits", C.c_int32), ("optimizer", C.c_int32), ("margin_policy", C.c_int32),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("adam_eps", C.c_double), ("max_iters", C.c_int64), ("loss_tol", C.c_double),
                ("box", C.c_double * 3)]


class Outputs(C.Structure):
    _fields_ = [("labels", C.c_void_p), ("stream", C.c_void_p), ("stream_cap", C.c_size_t),
                ("stream_len", C.POINTER(C.c_size_t)), ("debug_xyz", C.c_void_p),
                ("loss_trace", C.c_void_p), ("viol_trace", C.c_void_p), ("trace_cap", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_safe", C.c_int64), ("n_pb", C.c_int64),
                ("n_pc", C.c_int64), ("n_active", C.c_int64), ("n_editable", C.c_int64),
                ("n_flagged", C.c_int64), ("iters", C.c_int64), ("loss0", C.c_double),
                ("loss_final", C.c_double), ("viol0", C.c_int64), ("viol_final", C.c_int64),
                ("bytes_flags", C.c_int64), ("bytes_codes", C.c_int64),
                ("bytes_stream", C.c_int64), ("t_stage_ms", C.c_double * NSTAGES),
                ("kernel_ms", C.c_double * NKERNELS), ("kernel_launches", C.c_int64 * NKERNELS),
                ("pgd_rows_evaluated", C.c_int64), ("pgd_incidences_evaluated", C.c_int64)]


class Job(C.Structure):
    _fields_ = [("orig", Particles), ("recon", Particles), ("params", Params), ("out", Outputs)]


class JobResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("stats", Stats),
                ("t_submit_ms", C.c_double), ("t_start_ms", C.c_double),
                ("t_finish_ms", C.c_double), ("batch_jobs", C.c_int32), ("worker", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_inflight", C.c_int32), ("n_streams", C.c_int32)]


_TUNE_MAX = 32


class TuneReport(C.Structure):
    _fields_ = [("cell_pct", C.c_int32), ("dense_cell", C.c_int32), ("graph_iters", C.c_int32),
                ("n_trials", C.c_int32), ("trial_kind", C.c_int32 * _TUNE_MAX),
                ("trial_cell_pct", C.c_int32 * _TUNE_MAX),
                ("trial_dense_cell", C.c_int32 * _TUNE_MAX),
                ("trial_graph_iters", C.c_int32 * _TUNE_MAX),
                ("trial_ms", C.c_double * _TUNE_MAX)]


PENDING = 2


_lib = None


def lib() -> C.CDLL:
    """Load libpcc.so (built by __graft_entry__.build or build_lib.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpcc.so is not built (run __graft_entry__.build())")
        # PyTorch ships its own HIP runtime under the same soname as the
        # system's; loading torch first makes libpcc.so bind to that one, so
        # the process has a single HIP runtime whatever the import order
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.pcc_version.restype = C.c_int
        L.pcc_status_string.restype = C.c_char_p
        L.pcc_status_string.argtypes = [C.c_int32]
        L.pcc_last_error.restype = C.c_char_p
        L.pcc_context_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
        L.pcc_context_destroy.argtypes = [C.c_void_p]
        L.pcc_params_init.argtypes = [C.POINTER(Params)]
        L.pcc_params_init.restype = None
        L.pcc_stream_bound.argtypes = [C.c_int64, C.POINTER(Params)]
        L.pcc_stream_bound.restype = C.c_size_t
        L.pcc_correct.argtypes = [C.c_void_p, C.POINTER(Particles), C.POINTER(Particles),
                                  C.POINTER(Params), C.POINTER(Outputs), C.POINTER(Stats),
                                  C.c_void_p]
        L.pcc_correct_multi.argtypes = [C.c_void_p, C.POINTER(Particles), C.POINTER(Particles),
                                        C.POINTER(Params), C.POINTER(C.c_double), C.c_int32,
                                        C.POINTER(Outputs), C.POINTER(Stats), C.c_void_p]
        L.pcc_correct_batch.argtypes = [C.c_void_p, C.POINTER(Job), C.c_int32,
                                        C.POINTER(JobResult), C.c_void_p]
        L.pcc_decode.argtypes = [C.c_void_p, C.c_size_t, C.POINTER(Particles), C.c_void_p,
                                 C.c_void_p, C.c_void_p]
        L.pcc_fof_labels.argtypes = [C.c_void_p, C.POINTER(Particles), C.c_double,
                                     C.POINTER(C.c_double), C.c_void_p, C.c_void_p]
        L.pcc_fof_labels_noalloc.argtypes = [C.c_void_p, C.POINTER(Particles), C.c_double,
                                             C.POINTER(C.c_double), C.c_void_p, C.c_void_p]
        L.pcc_workspace_query.argtypes = [C.c_void_p, C.POINTER(Particles), C.POINTER(Particles),
                                          C.POINTER(Params), C.POINTER(C.c_size_t), C.c_void_p]
        L.pcc_fof_labels_noalloc_max_n.argtypes = []
        L.pcc_fof_labels_noalloc_max_n.restype = C.c_int64
        L.pcc_context_set.argtypes = [C.c_void_p, C.c_int32, C.c_int64]
        L.pcc_context_get.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64)]
        L.pcc_debug_set.argtypes = [C.c_int32, C.c_int64]
        L.pcc_debug_get.argtypes = [C.c_int32, C.POINTER(C.c_int64)]
        L.pcc_autotune.argtypes = [C.c_void_p, C.POINTER(Job), C.c_int32, C.c_int32,
                                   C.POINTER(TuneReport), C.c_void_p]
        L.pcc_debug_fetch.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                      C.POINTER(C.c_int64)]
        L.pcc_decode_device.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(Particles),
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.pcc_server_create.argtypes = [C.c_void_p, C.POINTER(ServerConfig),
                                        C.POINTER(C.c_void_p)]
        L.pcc_server_submit.argtypes = [C.c_void_p, C.POINTER(Job), C.POINTER(C.c_uint64)]
        L.pcc_server_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(JobResult)]
        L.pcc_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int64, C.POINTER(JobResult)]
        L.pcc_server_cancel.argtypes = [C.c_void_p, C.c_uint64]
        L.pcc_server_drain.argtypes = [C.c_void_p]
        L.pcc_server_destroy.argtypes = [C.c_void_p]
        for name in ("pcc_context_create", "pcc_context_destroy", "pcc_correct",
                     "pcc_correct_multi", "pcc_correct_batch", "pcc_decode", "pcc_fof_labels",
                     "pcc_fof_labels_noalloc", "pcc_workspace_query", "pcc_debug_fetch",
                     "pcc_context_set", "pcc_context_get", "pcc_autotune", "pcc_decode_device",
                     "pcc_debug_set", "pcc_debug_get", "pcc_server_create", "pcc_server_submit",
                     "pcc_server_poll", "pcc_server_wait", "pcc_server_cancel",
                     "pcc_server_drain", "pcc_server_destroy"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _check(status: int) -> int:
    if status < 0:
        raise PccError(status, lib().pcc_last_error().decode() or
                       lib().pcc_status_string(status).decode())
    return status


def stats_dict(s: Stats) -> Dict:
    d = {k: getattr(s, k) for k, _ in Stats._fields_
         if k not in ("t_stage_ms", "kernel_ms", "kernel_launches")}
    d["t_stage_ms"] = {STAGE_NAMES[k]: s.t_stage_ms[k] for k in range(NSTAGES)}
    d["kernel_ms"] = {KERNEL_NAMES[k]: s.kernel_ms[k] for k in range(NKERNELS)}
    d["kernel_launches"] = {KERNEL_NAMES[k]: s.kernel_launches[k] for k in range(NKERNELS)}
    return d


def make_params(b: float, xi: float, mode="hf", box=None, m_bits=16, optimizer="adam",
                lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8, max_iters=0, loss_tol=0.0,
                margin="safe") -> Params:
    p = Params()
    lib().pcc_params_init(C.byref(p))
    p.b, p.xi = float(b), float(xi)
    p.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    p.m_bits = int(m_bits)
    p.optimizer = {"adam": 0, "sgd": 1}[optimizer]
    p.margin_policy = {"safe": 0, "paper": 1}[margin]
    p.lr, p.beta1, p.beta2, p.adam_eps = float(lr), float(beta1), float(beta2), float(adam_eps)
    p.max_iters = int(max_iters)
    p.loss_tol = float(loss_tol)
    for k, v in enumerate(box or (0.0, 0.0, 0.0)):
        p.box[k] = float(v)
    return p


def _view(a) -> Tuple[Particles, object]:
    """Particles view of a (3, N) float32 array: torch GPU tensor or numpy."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if a.dtype != torch.float32 or a.dim() != 2 or a.shape[0] != 3:
                raise ValueError("expected a (3, N) float32 tensor")
            a = a.contiguous()
            mem = MEM_DEVICE if a.is_cuda else MEM_HOST
            base, st = a.data_ptr(), a.stride(0) * a.element_size()
            return Particles(base, base + st, base + 2 * st, a.shape[1], mem, 0), a
    except ImportError:
        pass
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2 or a.shape[0] != 3:
        raise ValueError("expected a (3, N) float32 array")
    base, st = a.ctypes.data, a.strides[0]
    return Particles(base, base + st, base + 2 * st, a.shape[1], MEM_HOST, 0), a


def _trace_buffers(out: "Outputs", k: int):
    """Host buffers of a k-entry loss / violation trace, set into out."""
    if k <= 0:
        return None, None
    tl = np.zeros(k, dtype=np.float64)
    tv = np.zeros(k, dtype=np.int64)
    out.loss_trace, out.viol_trace, out.trace_cap = tl.ctypes.data, tv.ctypes.data, k
    return tl, tv


def _trace_results(stats: Dict, tl, tv):
    if tl is None:
        return
    m = min(len(tl), int(stats["iters"]) + 1)
    stats["loss_trace"] = tl[:m].copy()
    stats["viol_trace"] = tv[:m].copy()


def _stream_handle(on_device: bool):
    if not on_device:
        return None
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class _JobBuffers:
    """A pcc_job built from a job dict (orig, recon, b, xi; optional mode,
    box, opts, debug_xyz) together with the Python objects that own its
    buffers, which must live until the job has finished."""

    def __init__(self, jd: Dict):
        po, ko = _view(jd["orig"])
        pr, kr = _view(jd["recon"])
        self.on_device = po.memspace == MEM_DEVICE
        params = make_params(jd["b"], jd["xi"], mode=jd.get("mode", "hf"), box=jd.get("box"),
                             **dict(jd.get("opts", {})))
        cap = lib().pcc_stream_bound(po.n, C.byref(params))
        self.sbuf = np.zeros(max(cap, 1), dtype=np.uint8)
        self.slen = C.c_size_t(0)
        if self.on_device:
            import torch
            self.lab = torch.empty(max(po.n, 1), dtype=torch.int32, device=ko.device)
            lptr = self.lab.data_ptr()
        else:
            self.lab = np.zeros(max(po.n, 1), dtype=np.int32)
            lptr = self.lab.ctypes.data
        self.dbg = np.zeros((3, max(po.n, 1)), dtype=np.float64) if jd.get("debug_xyz") else None
        self.n = po.n
        self.keep = (ko, kr)
        self.job = Job()
        self.job.orig, self.job.recon, self.job.params = po, pr, params
        self.job.out = Outputs(lptr, self.sbuf.ctypes.data, cap, C.pointer(self.slen),
                               self.dbg.ctypes.data if self.dbg is not None else None)

    def result(self, r: "JobResult"):
        st = stats_dict(r.stats)
        st["status"] = r.status
        for k in ("t_submit_ms", "t_start_ms", "t_finish_ms", "batch_jobs", "worker"):
            st[k] = getattr(r, k)
        if self.dbg is not None:
            st["debug_xyz"] = self.dbg[:, : self.n]
        return r.status, bytes(self.sbuf[: self.slen.value]), self.lab[: self.n], st


class Context:
    """A library context bound to one GPU."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().pcc_context_create(int(device), C.byref(h)))
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().pcc_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    _OPTIONS = {"kernel_timing": 1, "graph_iters": 2, "exact_pairs": 3, "cell_pct": 4,
                "dense_cell": 5, "workspace_high_water": 6}

    def set_option(self, key: str, value: int):
        _check(lib().pcc_context_set(self._h, self._OPTIONS[key], int(value)))

    def get_option(self, key: str) -> int:
        v = C.c_int64(0)
        _check(lib().pcc_context_get(self._h, self._OPTIONS[key], C.byref(v)))
        return v.value

    def autotune(self, jobs: Sequence[Dict], graph: bool = True) -> Dict:
        """Times the jobs (dicts as for correct_batch) under candidate
        scheduling knobs and keeps the fastest on this context; returns the
        choice and every trial."""
        cj = (Job * len(jobs))()
        held = []
        on_dev = False
        for k, jd in enumerate(jobs):
            h = _JobBuffers(jd)
            cj[k] = h.job
            on_dev |= h.on_device
            held.append(h)
        rep = TuneReport()
        _check(lib().pcc_autotune(self._h, cj, len(jobs), 0 if graph else 1, C.byref(rep),
                                  _stream_handle(on_dev)))
        trials = [{"kind": ("pre_pgd_stages", "correction")[rep.trial_kind[t]],
                   "cell_pct": rep.trial_cell_pct[t], "dense_cell": rep.trial_dense_cell[t],
                   "graph_iters": rep.trial_graph_iters[t], "ms": rep.trial_ms[t]}
                  for t in range(rep.n_trials)]
        return {"cell_pct": rep.cell_pct, "dense_cell": rep.dense_cell,
                "graph_iters": rep.graph_iters, "trials": trials}

    # ------------------------------------------------------------------
    def correct(self, orig, recon, b: float, xi: float, mode="hf", box=None, labels=True,
                debug_xyz=False, stream_cap: Optional[int] = None, trace: int = 0, **opts):
        """Alg. 1 on one snapshot.  Returns (stream bytes, labels, stats);
        labels live where `orig` lives; stats['status'] is 0 or 1.  With
        trace = K > 0, stats['loss_trace'] / ['viol_trace'] hold the loss of
        Eq. 3 and the violated-constraint count of the first K evaluations."""
        po, ko = _view(orig)
        pr, kr = _view(recon)
        n = po.n
        params = make_params(b, xi, mode=mode, box=box, **opts)
        cap = int(stream_cap) if stream_cap is not None else lib().pcc_stream_bound(n, C.byref(params))
        sbuf = np.zeros(max(cap, 1), dtype=np.uint8)
        slen = C.c_size_t(0)
        lab = None
        lab_ptr = None
        if labels:
            if po.memspace == MEM_DEVICE:
                import torch
                lab = torch.empty(max(n, 1), dtype=torch.int32, device=ko.device)
                lab_ptr = lab.data_ptr()
            else:
                lab = np.zeros(max(n, 1), dtype=np.int32)
                lab_ptr = lab.ctypes.data
        dbg = np.zeros((3, max(n, 1)), dtype=np.float64) if debug_xyz else None
        out = Outputs(lab_ptr, sbuf.ctypes.data, cap, C.pointer(slen),
                      dbg.ctypes.data if dbg is not None else None)
        tl, tv = _trace_buffers(out, trace)
        st = Stats()
        status = lib().pcc_correct(self._h, C.byref(po), C.byref(pr), C.byref(params),
                                   C.byref(out), C.byref(st),
                                   _stream_handle(po.memspace == MEM_DEVICE))
        _check(status)
        stats = stats_dict(st)
        stats["status"] = status
        res_lab = lab[:n] if lab is not None else None
        if dbg is not None:
            stats["debug_xyz"] = dbg[:, :n]
        _trace_results(stats, tl, tv)
        return bytes(sbuf[: slen.value]), res_lab, stats

    def workspace_query(self, orig, recon, b: float, xi: float, mode="hf", box=None,
                        **opts) -> int:
        """Bound of the device workspace bytes correct() would take."""
        po, ko = _view(orig)
        pr, kr = _view(recon)
        params = make_params(b, xi, mode=mode, box=box, **opts)
        out = C.c_size_t(0)
        _check(lib().pcc_workspace_query(self._h, C.byref(po), C.byref(pr), C.byref(params),
                                         C.byref(out), _stream_handle(po.memspace == MEM_DEVICE)))
        return int(out.value)

    def workspace_high_water(self) -> int:
        """Device workspace bytes the last call on this context used at most."""
        return self.get_option("workspace_high_water")

    def correct_multi(self, orig, recon, b_list: Sequence[float], xi: float, mode="hf",
                      box=None, labels=True, debug_xyz=False, **opts):
        """One snapshot corrected for every linking length in b_list at once.
        Returns (stream bytes, labels (len(b_list), N) or None, stats)."""
        if not 1 <= len(b_list) <= 8:
            raise ValueError("correct_multi takes 1 to 8 linking lengths")
        po, ko = _view(orig)
        pr, kr = _view(recon)
        n, nb = po.n, len(b_list)
        params = make_params(float(b_list[0]), xi, mode=mode, box=box, **opts)
        cap = lib().pcc_stream_bound(n, C.byref(params))
        sbuf = np.zeros(max(cap, 1), dtype=np.uint8)
        slen = C.c_size_t(0)
        lab = None
        lab_ptr = None
        if labels:
            if po.memspace == MEM_DEVICE:
                import torch
                lab = torch.empty((nb, max(n, 1)), dtype=torch.int32, device=ko.device)
                lab_ptr = lab.data_ptr()
            else:
                lab = np.zeros((nb, max(n, 1)), dtype=np.int32)
                lab_ptr = lab.ctypes.data
            if n == 0:
                lab_ptr = None
        dbg = np.zeros((3, max(n, 1)), dtype=np.float64) if debug_xyz else None
        out = Outputs(lab_ptr, sbuf.ctypes.data, cap, C.pointer(slen),
                      dbg.ctypes.data if dbg is not None else None)
        bl = (C.c_double * max(nb, 1))(*[float(v) for v in b_list])
        st = Stats()
        status = lib().pcc_correct_multi(self._h, C.byref(po), C.byref(pr), C.byref(params), bl,
                                         nb, C.byref(out), C.byref(st),
                                         _stream_handle(po.memspace == MEM_DEVICE))
        _check(status)
        stats = stats_dict(st)
        stats["status"] = status
        if dbg is not None:
            stats["debug_xyz"] = dbg[:, :n]
        res_lab = lab[:, :n] if lab is not None else None
        return bytes(sbuf[: slen.value]), res_lab, stats

    def correct_batch(self, jobs: Sequence[Dict]):
        """jobs: dicts with orig, recon, b, xi and optional mode, box, opts.
        Returns a list of (status, stream bytes, labels, stats)."""
        cj = (Job * len(jobs))()
        held = []
        on_dev = False
        for k, jd in enumerate(jobs):
            h = _JobBuffers(jd)
            cj[k] = h.job
            on_dev |= h.on_device
            held.append(h)
        res = (JobResult * len(jobs))()
        lib().pcc_correct_batch(self._h, cj, len(jobs), res, _stream_handle(on_dev))
        return [h.result(res[k]) for k, h in enumerate(held)]

    def decode_device(self, stream: bytes, recon):
        """Apply an edit stream to a (3, N) float32 reconstruction on this
        GPU; returns a new (3, N) device tensor (bitwise equal to decode())."""
        import torch
        pr, kr = _view(recon)
        if pr.memspace != MEM_DEVICE:
            raise ValueError("decode_device takes a device tensor; use decode() for host arrays")
        out = torch.empty((3, max(pr.n, 1)), dtype=torch.float32, device=kr.device)
        buf = np.frombuffer(stream, dtype=np.uint8).copy()
        _check(lib().pcc_decode_device(self._h, buf.ctypes.data, len(buf), C.byref(pr),
                                       out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                                       _stream_handle(True)))
        return out[:, : pr.n]

    def fof_labels(self, pts, b: float, box=None, labels=None):
        return self._fof(lib().pcc_fof_labels, pts, b, box, labels)

    def fof_labels_noalloc(self, pts, b: float, box=None, labels=None):
        """pcc_fof_labels_noalloc: the same labels with no device allocation
        in the library (pass `labels`, an int32 buffer of N entries in the
        memspace of pts, to allocate nothing here either)."""
        return self._fof(lib().pcc_fof_labels_noalloc, pts, b, box, labels)

    def _fof(self, fn, pts, b, box, labels):
        p, keep = _view(pts)
        n = p.n
        if labels is not None:
            lab = labels
            ptr = lab.data_ptr() if p.memspace == MEM_DEVICE else lab.ctypes.data
        elif p.memspace == MEM_DEVICE:
            import torch
            lab = torch.empty(max(n, 1), dtype=torch.int32, device=keep.device)
            ptr = lab.data_ptr()
        else:
            lab = np.zeros(max(n, 1), dtype=np.int32)
            ptr = lab.ctypes.data
        bx = (C.c_double * 3)(*[float(v) for v in (box or (0.0, 0.0, 0.0))])
        _check(fn(self._h, C.byref(p), float(b), bx, C.c_void_p(ptr),
                  _stream_handle(p.memspace == MEM_DEVICE)))
        return lab[:n]

    def debug_fetch(self, job: int, what: str):
        code = {"active_i": 1, "active_j": 2, "active_type": 3, "safe_labels": 4,
                "editable": 5, "active_thr": 6, "cell_start": 7, "neighbors": 8}[what]
        dtype = {1: np.uint32, 2: np.uint32, 3: np.uint8, 4: np.int32, 5: np.uint32,
                 6: np.uint8, 7: np.uint32, 8: np.uint32}[code]
        cnt = C.c_int64(0)
        _check(lib().pcc_debug_fetch(self._h, int(job), code, None, 0, C.byref(cnt)))
        buf = np.zeros(max(cnt.value, 1), dtype=dtype)
        _check(lib().pcc_debug_fetch(self._h, int(job), code, buf.ctypes.data, cnt.value,
                                     C.byref(cnt)))
        return buf[: cnt.value]


def inject_alloc_failure(after: int):
    """Test hook: the workspace allocation after `after` more successful ones
    fails as if the device were out of memory (-1 switches it off)."""
    _check(lib().pcc_debug_set(1, int(after)))


def fof_labels_noalloc_max_n() -> int:
    """Largest point count pcc_fof_labels_noalloc accepts."""
    return int(lib().pcc_fof_labels_noalloc_max_n())


def noalloc_high_water() -> int:
    """Bytes of the static scratch the last pcc_fof_labels_noalloc used."""
    v = C.c_int64(0)
    _check(lib().pcc_debug_get(2, C.byref(v)))
    return v.value


def alloc_failure_countdown() -> int:
    v = C.c_int64(0)
    _check(lib().pcc_debug_get(1, C.byref(v)))
    return v.value


class Server:
    """Served form: a queue of jobs run in batches by worker threads on the
    context's GPU.  submit() returns a ticket; poll() / wait() return None
    while the job is pending, else (status, stream bytes, labels, stats) with
    the submit / start / finish times (ms since the server started) in
    stats.  Device inputs are synchronised on the current stream at submit."""

    def __init__(self, ctx: Context, hbm_budget: int = 0, max_inflight: int = 0,
                 n_streams: int = 0):
        cfg = ServerConfig(int(hbm_budget), int(max_inflight), int(n_streams))
        h = C.c_void_p()
        _check(lib().pcc_server_create(ctx._h, C.byref(cfg), C.byref(h)))
        self._h = h
        self._ctx = ctx
        self._held: Dict[int, _JobBuffers] = {}

    def submit(self, **jd) -> int:
        hb = _JobBuffers(jd)
        if hb.on_device:
            import torch
            torch.cuda.current_stream().synchronize()
        tk = C.c_uint64(0)
        _check(lib().pcc_server_submit(self._h, C.byref(hb.job), C.byref(tk)))
        self._held[tk.value] = hb
        return tk.value

    def _finish(self, ticket: int, status: int, r: "JobResult"):
        if status == PENDING:
            return None
        hb = self._held.pop(ticket)
        return hb.result(r)

    def poll(self, ticket: int):
        r = JobResult()
        status = lib().pcc_server_poll(self._h, C.c_uint64(ticket), C.byref(r))
        if status == -1 and ticket not in self._held:
            _check(status)
        return self._finish(ticket, status, r)

    def wait(self, ticket: int, timeout_ms: int = -1):
        r = JobResult()
        status = lib().pcc_server_wait(self._h, C.c_uint64(ticket), int(timeout_ms), C.byref(r))
        if status == -1 and ticket not in self._held:
            _check(status)
        return self._finish(ticket, status, r)

    def cancel(self, ticket: int) -> bool:
        """True if the job was removed before it started."""
        return lib().pcc_server_cancel(self._h, C.c_uint64(ticket)) == 0

    def drain(self):
        _check(lib().pcc_server_drain(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().pcc_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode(stream: bytes, recon: np.ndarray) -> np.ndarray:
    """Apply an edit stream to a host (3, N) float32 reconstruction."""
    pr, kr = _view(np.asarray(recon, dtype=np.float32))
    n = pr.n
    out = np.zeros((3, max(n, 1)), dtype=np.float32)
    buf = np.frombuffer(stream, dtype=np.uint8).copy()
    _check(lib().pcc_decode(buf.ctypes.data, len(buf), C.byref(pr), out[0].ctypes.data,
                            out[1].ctypes.data, out[2].ctypes.data))
    return out[:, :n]


def version() -> int:
    return lib().pcc_version()
