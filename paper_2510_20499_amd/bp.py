"""Python binding of libbp.so: argument marshalling only.

Every step of propagation and probing runs in the HIP library.  PyTorch
provides device memory (float64/int32 CUDA tensors on ROCm) and the current
stream.  If the library is missing this module raises at import; there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbp.so")

BP_OK, BP_INFEASIBLE, BP_ROUND_LIMIT = 0, 1, 2
BP_EINVAL, BP_ENOMEM, BP_EDEVICE, BP_ECAPACITY, BP_ESTATE, BP_ECANCELED = -1, -2, -3, -4, -5, -6
COMPLETION_CANCELLED = 1
FLAG_FORCE_EXACT, FLAG_TIME_KERNELS, FLAG_HOST_ROUNDS, FLAG_COUNT_VARS, FLAG_BATCH_SLOTS = 1, 2, 4, 8, 16
FLAG_FULL_ROWS = 32
FLAG_LV_DENSE = 64

EXPORTS = ["bp_options_default", "bp_load", "bp_propagate", "bp_propagate_batch", "bp_probe",
           "bp_get_base", "bp_kernel_stats", "bp_device_bytes", "bp_free", "bp_last_error",
           "bp_server_create", "bp_server_submit", "bp_server_run", "bp_server_poll",
           "bp_server_results", "bp_server_info", "bp_server_pool_info", "bp_server_destroy", "bp_autotune",
           "bp_scores", "bp_probe_order", "bp_round", "bp_scores_noalloc", "bp_repair",
           "bp_autotune_batch", "bp_debug_fail_alloc", "bp_server_cancel", "bp_server_expire",
           "bp_server_add_instance", "bp_server_evict"]
REQ_PROBE, REQ_PROPAGATE = 0, 1


class Sparse(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("ptr", C.c_void_p), ("idx", C.c_void_p), ("val", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("feastol", C.c_double), ("inttol", C.c_double), ("tau", C.c_double),
                ("max_rounds", C.c_int32), ("flags", C.c_uint32),
                ("heavy_threshold", C.c_int32), ("rounds_per_launch", C.c_int32),
                ("probe_slots", C.c_int32), ("heavy_chunk", C.c_int32),
                ("repair_calls", C.c_int32), ("repair_attempts", C.c_int32),
                ("repair_shifts", C.c_int32), ("lv_grid", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("rounds", C.c_int32), ("nnz_propagated", C.c_int64),
                ("n_infeasible_rows", C.c_int32), ("infeasible_var", C.c_int32),
                ("infeasible_row", C.c_int64)]

    def as_dict(self):
        return dict(status=self.status, rounds=self.rounds, nnz_propagated=self.nnz_propagated,
                    n_infeasible_rows=self.n_infeasible_rows,
                    infeasible_row=self.infeasible_row, infeasible_var=self.infeasible_var)


class ProbeOut(C.Structure):
    _fields_ = [("status", C.c_void_p), ("rounds", C.c_void_p), ("nnz", C.c_void_p),
                ("off", C.c_void_p), ("var", C.c_void_p), ("lb", C.c_void_p),
                ("ub", C.c_void_p), ("cap", C.c_int64), ("required", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("ms", C.c_double), ("launches", C.c_int64), ("rows", C.c_int64),
                ("nnz", C.c_int64), ("vars_read", C.c_int64), ("vars_written", C.c_int64),
                ("rows_kept", C.c_int64), ("nnz_kept", C.c_int64), ("apply_ms", C.c_double),
                ("apply_entries", C.c_int64), ("apply_colent", C.c_int64), ("apply_corr", C.c_int64),
                ("rows_union", C.c_int64), ("nnz_union", C.c_int64), ("lv_corr_chunks", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("instance", C.c_int32), ("kind", C.c_int32), ("count", C.c_int32),
                ("reserved", C.c_int32), ("vars", C.c_void_p), ("lb", C.c_void_p),
                ("ub", C.c_void_p)]


class Completion(C.Structure):
    _fields_ = [("id", C.c_int64), ("instance", C.c_int32), ("kind", C.c_int32),
                ("jobs", C.c_int32), ("flags", C.c_int32), ("submit_us", C.c_double),
                ("done_us", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("heavy_threshold", C.c_int32), ("heavy_chunk", C.c_int32),
                ("rounds_per_launch", C.c_int32), ("probe_slots", C.c_int32),
                ("ms", C.c_double), ("trials", C.c_int32), ("from_cache", C.c_int32),
                ("lv_grid", C.c_int32)]


class ScoresOut(C.Structure):
    _fields_ = [("nviol", C.c_void_p), ("maxviol", C.c_void_p), ("minunit", C.c_void_p),
                ("slack_score", C.c_void_p)]


class Cache(C.Structure):
    _fields_ = [("vars", C.c_void_p), ("k", C.c_int32), ("status", C.c_void_p), ("off", C.c_void_p),
                ("var", C.c_void_p), ("lb", C.c_void_p), ("ub", C.c_void_p)]


class RoundResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("bulks", C.c_int32), ("singles", C.c_int32),
                ("recoveries", C.c_int32), ("fixed", C.c_int32), ("iterations", C.c_int32),
                ("nnz_propagated", C.c_int64), ("repairs", C.c_int32), ("repaired", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class RepairResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("attempts", C.c_int32), ("shifts", C.c_int32),
                ("reason", C.c_int32), ("nnz_propagated", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libbp error %d: %s" % (code, msg))
        self.code = code


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libbp.so is not built (run paper_2510_20499_amd/build.py or "
                          "__graft_entry__.build())")
    lib = C.CDLL(path)
    lib.bp_options_default.argtypes = [C.POINTER(Options)]
    lib.bp_options_default.restype = None
    lib.bp_load.argtypes = [C.POINTER(Sparse), C.POINTER(Sparse), C.c_void_p, C.c_void_p,
                            C.c_void_p, C.POINTER(Options), C.c_void_p, C.POINTER(C.c_void_p)]
    lib.bp_load.restype = C.c_int
    lib.bp_propagate.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                 C.POINTER(Result), C.c_void_p]
    lib.bp_propagate.restype = C.c_int
    lib.bp_propagate_batch.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.POINTER(Result), C.c_void_p]
    lib.bp_propagate_batch.restype = C.c_int
    lib.bp_probe.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(ProbeOut), C.c_void_p]
    lib.bp_probe.restype = C.c_int
    lib.bp_scores.restype = C.c_int
    lib.bp_scores.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(ScoresOut), C.c_void_p]
    lib.bp_repair.restype = C.c_int
    lib.bp_repair.argtypes = [C.c_void_p] + [C.c_void_p] * 4 + [C.c_int32, C.c_int32,
                                                                 C.POINTER(RepairResult), C.c_void_p]
    lib.bp_scores_noalloc.restype = C.c_int
    lib.bp_scores_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(ScoresOut),
                                      C.c_void_p]
    lib.bp_probe_order.restype = C.c_int
    lib.bp_probe_order.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_void_p, C.c_void_p]
    lib.bp_round.restype = C.c_int
    lib.bp_round.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.POINTER(Cache), C.POINTER(RoundResult), C.c_void_p]
    lib.bp_get_base.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.bp_get_base.restype = C.c_int
    lib.bp_kernel_stats.argtypes = [C.c_void_p, C.POINTER(Stats), C.c_int]
    lib.bp_kernel_stats.restype = C.c_int
    lib.bp_device_bytes.argtypes = [C.c_void_p]
    lib.bp_device_bytes.restype = C.c_int64
    lib.bp_free.argtypes = [C.c_void_p]
    lib.bp_free.restype = None
    lib.bp_last_error.argtypes = []
    lib.bp_last_error.restype = C.c_char_p
    lib.bp_server_create.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Options), C.c_int64,
                                     C.c_void_p, C.POINTER(C.c_void_p)]
    lib.bp_server_create.restype = C.c_int
    lib.bp_server_submit.argtypes = [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_int64)]
    lib.bp_server_submit.restype = C.c_int
    lib.bp_server_run.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
    lib.bp_server_run.restype = C.c_int
    lib.bp_server_poll.argtypes = [C.c_void_p, C.POINTER(Completion), C.c_int32,
                                   C.POINTER(C.c_int32)]
    lib.bp_server_poll.restype = C.c_int
    lib.bp_server_results.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 10 + \
                                     [C.c_int64, C.POINTER(C.c_int64)]
    lib.bp_server_results.restype = C.c_int
    lib.bp_server_info.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    lib.bp_server_info.restype = C.c_int
    lib.bp_server_pool_info.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
    lib.bp_server_pool_info.restype = C.c_int
    lib.bp_autotune.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                C.c_char_p, C.POINTER(Tuning), C.c_void_p]
    lib.bp_autotune.restype = C.c_int
    lib.bp_autotune_batch.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_char_p, C.POINTER(Tuning), C.c_void_p]
    lib.bp_autotune_batch.restype = C.c_int
    lib.bp_server_destroy.argtypes = [C.c_void_p]
    lib.bp_server_destroy.restype = None
    lib.bp_server_cancel.argtypes = [C.c_void_p, C.c_int64]
    lib.bp_server_cancel.restype = C.c_int
    lib.bp_server_expire.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_int32)]
    lib.bp_server_expire.restype = C.c_int
    lib.bp_server_add_instance.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]
    lib.bp_server_add_instance.restype = C.c_int
    lib.bp_server_evict.argtypes = [C.c_void_p, C.c_int32]
    lib.bp_server_evict.restype = C.c_int
    lib.bp_debug_fail_alloc.argtypes = [C.c_int64]
    lib.bp_debug_fail_alloc.restype = C.c_int
    return lib


_LIB = load_library()


def lib():
    return _LIB


def debug_fail_alloc(k: int):
    """bp_debug_fail_alloc: make the k-th device allocation from now on fail
    with BP_ENOMEM (k = 0 disarms)."""
    _check(_LIB.bp_debug_fail_alloc(int(k)))


def _check(rc):
    if rc < 0:
        raise BPError(rc, _LIB.bp_last_error().decode())
    return rc


def default_options(**kw) -> Options:
    o = Options()
    _LIB.bp_options_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _dptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Instance:
    """A constraint matrix resident on the device (bp_load)."""

    def __init__(self, inst: dict, options: Options = None, with_csc: bool = False, stream=None):
        self.m = int(inst["m"])
        self.n = int(inst["n"])
        self._rp = _host(inst["row_ptr"], np.int64)
        self._col = _host(inst["col"], np.int32)
        self._val = _host(inst["val"], np.float64)
        self._lo = _host(inst["lo"], np.float64)
        self._hi = _host(inst["hi"], np.float64)
        self._vt = _host(inst["vtype"], np.uint8)
        self.nnz = int(self._rp[-1])
        csr = Sparse(self.m, self.n, self.nnz, self._rp.ctypes.data, self._col.ctypes.data,
                     self._val.ctypes.data)
        csc_p = None
        if with_csc:
            order = np.argsort(self._col, kind="stable")
            rows = np.repeat(np.arange(self.m, dtype=np.int32), np.diff(self._rp))
            self._crow = np.ascontiguousarray(rows[order])
            self._cval = np.ascontiguousarray(self._val[order])
            self._cptr = np.zeros(self.n + 1, np.int64)
            np.cumsum(np.bincount(self._col, minlength=self.n), out=self._cptr[1:])
            csc = Sparse(self.m, self.n, self.nnz, self._cptr.ctypes.data,
                         self._crow.ctypes.data, self._cval.ctypes.data)
            csc_p = C.byref(csc)
        self.options = options or default_options()
        h = C.c_void_p()
        _check(_LIB.bp_load(C.byref(csr), csc_p, self._lo.ctypes.data, self._hi.ctypes.data,
                            self._vt.ctypes.data, C.byref(self.options), _stream_ptr(stream),
                            C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _LIB.bp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self) -> int:
        return int(_LIB.bp_device_bytes(self._h))

    def propagate(self, lb: torch.Tensor, ub: torch.Tensor, changed: torch.Tensor = None,
                  stream=None) -> dict:
        """bp_propagate: lb/ub are float64 device tensors, updated in place."""
        assert lb.dtype == torch.float64 and ub.dtype == torch.float64
        assert lb.is_cuda and ub.is_cuda and lb.is_contiguous() and ub.is_contiguous()
        assert lb.numel() == self.n and ub.numel() == self.n
        r = Result()
        if changed is None:
            rc = _LIB.bp_propagate(self._h, _dptr(lb), _dptr(ub), None, 0, C.byref(r),
                                   _stream_ptr(stream))
        else:
            assert changed.dtype == torch.int32 and changed.is_cuda and changed.is_contiguous()
            # A non-null pointer marks a warm start even for an empty list.
            ptr = _dptr(changed) if changed.numel() else C.c_void_p(lb.data_ptr())
            rc = _LIB.bp_propagate(self._h, _dptr(lb), _dptr(ub), ptr, changed.numel(),
                                   C.byref(r), _stream_ptr(stream))
        _check(rc)
        return r.as_dict()

    def propagate_batch(self, lb: torch.Tensor, ub: torch.Tensor, changed_ptr: torch.Tensor = None,
                        changed_idx: torch.Tensor = None, stream=None) -> list:
        """bp_propagate_batch: lb/ub are [B, n] float64 device tensors."""
        B = lb.shape[0]
        assert lb.shape == (B, self.n) and ub.shape == (B, self.n)
        assert lb.is_contiguous() and ub.is_contiguous()
        res = (Result * max(B, 1))()
        cp = _dptr(changed_ptr) if changed_ptr is not None else None
        ci = _dptr(changed_idx) if changed_idx is not None and changed_idx.numel() else None
        _check(_LIB.bp_propagate_batch(self._h, B, _dptr(lb), _dptr(ub), cp, ci, res,
                                       _stream_ptr(stream)))
        return [res[j].as_dict() for j in range(B)]

    def probe(self, vars_: torch.Tensor, cap: int = None, stream=None) -> dict:
        """bp_probe: double probing of the integer variables in vars_ (int32
        device): binaries at 0 and 1, other integers by two half-intervals."""
        k = vars_.numel()
        dev = vars_.device
        cap = cap if cap is not None else max(1024, 64 * 2 * k)
        while True:
            o = dict(status=torch.empty(2 * k, dtype=torch.int8, device=dev),
                     rounds=torch.empty(2 * k, dtype=torch.int32, device=dev),
                     nnz=torch.empty(2 * k, dtype=torch.int64, device=dev),
                     off=torch.empty(2 * k + 1, dtype=torch.int64, device=dev),
                     var=torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                     lb=torch.empty(max(cap, 1), dtype=torch.float64, device=dev),
                     ub=torch.empty(max(cap, 1), dtype=torch.float64, device=dev))
            po = ProbeOut(o["status"].data_ptr(), o["rounds"].data_ptr(), o["nnz"].data_ptr(),
                          o["off"].data_ptr(), o["var"].data_ptr(), o["lb"].data_ptr(),
                          o["ub"].data_ptr(), cap, 0)
            rc = _LIB.bp_probe(self._h, _dptr(vars_) if k else None, k, C.byref(po),
                               _stream_ptr(stream))
            if rc == BP_ECAPACITY:
                cap = int(po.required)
                continue
            _check(rc)
            tot = int(po.required)
            for key in ("var", "lb", "ub"):
                o[key] = o[key][:tot]
            return o

    def _bounds_ok(self, lb, ub):
        for t in (lb, ub):
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
            assert t.numel() == self.n

    def scores(self, lb: torch.Tensor, ub: torch.Tensor, stream=None, out: dict = None,
               noalloc: bool = False) -> dict:
        """bp_scores (bp_scores_noalloc with noalloc=True): probe-priority and
        implied-slack scores of every variable at the float64 device bounds
        lb/ub, into `out` (nviol int32, maxviol / minunit / slack_score
        float64, each [n] on the device) or new tensors."""
        self._bounds_ok(lb, ub)
        dev = lb.device
        if out is None:
            out = dict(nviol=torch.empty(self.n, dtype=torch.int32, device=dev),
                       maxviol=torch.empty(self.n, dtype=torch.float64, device=dev),
                       minunit=torch.empty(self.n, dtype=torch.float64, device=dev),
                       slack_score=torch.empty(self.n, dtype=torch.float64, device=dev))
        for key, dt in (("nviol", torch.int32), ("maxviol", torch.float64),
                        ("minunit", torch.float64), ("slack_score", torch.float64)):
            t = out[key]
            assert t.dtype == dt and t.is_cuda and t.is_contiguous() and t.numel() == self.n
        so = ScoresOut(out["nviol"].data_ptr(), out["maxviol"].data_ptr(),
                       out["minunit"].data_ptr(), out["slack_score"].data_ptr())
        fn = _LIB.bp_scores_noalloc if noalloc else _LIB.bp_scores
        _check(fn(self._h, _dptr(lb), _dptr(ub), C.byref(so), _stream_ptr(stream)))
        return out

    def probe_order(self, vars_: torch.Tensor, lb: torch.Tensor, ub: torch.Tensor,
                    stream=None) -> torch.Tensor:
        """bp_probe_order: vars_ (int32 device) sorted into probe order by
        the scores at lb/ub."""
        self._bounds_ok(lb, ub)
        k = vars_.numel()
        assert vars_.dtype == torch.int32 and vars_.is_cuda and vars_.is_contiguous()
        order = torch.empty(max(k, 1), dtype=torch.int32, device=vars_.device)
        _check(_LIB.bp_probe_order(self._h, _dptr(lb), _dptr(ub), _dptr(vars_) if k else None, k,
                                   _dptr(order), _stream_ptr(stream)))
        return order[:k]

    def round(self, lb: torch.Tensor, ub: torch.Tensor, x: torch.Tensor, draws: torch.Tensor,
              cache: dict = None, stream=None) -> dict:
        """bp_round: bound-propagation rounding of the integer variables of
        the box lb/ub (updated in place) towards x with the draws [2n]; cache
        is an optional dict of device tensors vars, status, off, var, lb, ub
        (bp_probe's output for vars)."""
        self._bounds_ok(lb, ub)
        for t in (x, draws):
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
        assert x.numel() == self.n and draws.numel() == 2 * self.n
        cp = None
        if cache is not None:
            k = cache["vars"].numel()
            cs = Cache(cache["vars"].data_ptr() if k else None, k, cache["status"].data_ptr(),
                       cache["off"].data_ptr(),
                       cache["var"].data_ptr() if cache["var"].numel() else None,
                       cache["lb"].data_ptr() if cache["lb"].numel() else None,
                       cache["ub"].data_ptr() if cache["ub"].numel() else None)
            cp = C.byref(cs)
        r = RoundResult()
        _check(_LIB.bp_round(self._h, _dptr(lb), _dptr(ub), _dptr(x), _dptr(draws), cp, C.byref(r),
                             _stream_ptr(stream)))
        d = r.as_dict()
        if self.options.repair_calls == 0:
            # no repair configured: the counts are always 0
            del d["repairs"], d["repaired"]
        return d

    def repair(self, lb: torch.Tensor, ub: torch.Tensor, lb0: torch.Tensor, ub0: torch.Tensor,
               max_shifts: int = 64, max_attempts: int = 8, stream=None) -> dict:
        """bp_repair: the repair procedure on the box lb/ub (updated in place
        when repaired) inside the original box lb0/ub0."""
        self._bounds_ok(lb, ub)
        self._bounds_ok(lb0, ub0)
        r = RepairResult()
        _check(_LIB.bp_repair(self._h, _dptr(lb), _dptr(ub), _dptr(lb0), _dptr(ub0), int(max_shifts),
                              int(max_attempts), C.byref(r), _stream_ptr(stream)))
        return r.as_dict()

    def autotune(self, lb: torch.Tensor, ub: torch.Tensor, vars_: torch.Tensor = None,
                 cache_path: str = None, stream=None) -> dict:
        """bp_autotune on a cold propagation from (lb, ub) and, if given, a
        probe of vars_; the chosen schedule stays in the instance."""
        t = Tuning()
        k = 0 if vars_ is None else vars_.numel()
        _check(_LIB.bp_autotune(self._h, _dptr(lb), _dptr(ub),
                                _dptr(vars_) if k else None, k,
                                cache_path.encode() if cache_path else None, C.byref(t),
                                _stream_ptr(stream)))
        return dict(heavy_threshold=t.heavy_threshold, heavy_chunk=t.heavy_chunk,
                    rounds_per_launch=t.rounds_per_launch, probe_slots=t.probe_slots,
                    ms=t.ms, trials=t.trials, from_cache=bool(t.from_cache))

    def autotune_batch(self, lb: torch.Tensor, ub: torch.Tensor, changed_ptr: torch.Tensor = None,
                       changed_idx: torch.Tensor = None, cache_path: str = None, stream=None) -> dict:
        """bp_autotune_batch on the batch (lb, ub [B, n]; left unchanged) with
        its changed lists; the chosen schedule stays in the instance."""
        assert lb.dim() == 2 and lb.shape == ub.shape and lb.shape[1] == self.n
        t = Tuning()
        _check(_LIB.bp_autotune_batch(self._h, lb.shape[0], _dptr(lb), _dptr(ub),
                                      _dptr(changed_ptr) if changed_ptr is not None else None,
                                      _dptr(changed_idx) if changed_idx is not None else None,
                                      cache_path.encode() if cache_path else None, C.byref(t),
                                      _stream_ptr(stream)))
        return dict(lv_grid=t.lv_grid, rounds_per_launch=t.rounds_per_launch, ms=t.ms,
                    trials=t.trials, from_cache=bool(t.from_cache))

    def base(self, stream=None):
        lb = torch.empty(self.n, dtype=torch.float64, device="cuda")
        ub = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(_LIB.bp_get_base(self._h, _dptr(lb), _dptr(ub), _stream_ptr(stream)))
        return lb, ub

    def kernel_stats(self, reset: bool = False) -> dict:
        s = Stats()
        _check(_LIB.bp_kernel_stats(self._h, C.byref(s), 1 if reset else 0))
        return dict(ms=s.ms, launches=s.launches, rows=s.rows, nnz=s.nnz,
                    vars_read=s.vars_read, vars_written=s.vars_written,
                    rows_kept=s.rows_kept, nnz_kept=s.nnz_kept, apply_ms=s.apply_ms,
                    apply_entries=s.apply_entries, apply_colent=s.apply_colent,
                    apply_corr=s.apply_corr, rows_union=s.rows_union, nnz_union=s.nnz_union,
                    lv_corr_chunks=s.lv_corr_chunks)


class Server:
    """Continuous-batching server over loaded instances (bp_server_*)."""

    def __init__(self, instances, budget_bytes: int, options: Options = None, stream=None):
        self._insts = list(instances)  # keep them alive
        arr = (C.c_void_p * len(self._insts))(*[i._h.value for i in self._insts])
        h = C.c_void_p()
        _check(_LIB.bp_server_create(arr, len(self._insts),
                                     C.byref(options) if options is not None else None,
                                     int(budget_bytes), _stream_ptr(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _LIB.bp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        """Slots over all pools, bytes of a slot sized for every instance,
        and per pool its slots, bytes per slot and instances."""
        s, b = C.c_int32(), C.c_int64()
        _check(_LIB.bp_server_info(self._h, C.byref(s), C.byref(b)))
        npools = C.c_int32()
        _check(_LIB.bp_server_pool_info(self._h, -1, C.byref(npools), None, None, None))
        pools = []
        for q in range(npools.value):
            ps, pb, pi = C.c_int32(), C.c_int64(), C.c_int32()
            _check(_LIB.bp_server_pool_info(self._h, q, None, C.byref(ps), C.byref(pb), C.byref(pi)))
            pools.append(dict(slots=ps.value, bytes_per_slot=pb.value, instances=pi.value))
        return dict(slots=s.value, bytes_per_slot=b.value, pools=pools)

    def submit(self, instance: int, kind: int, vars_, lb=None, ub=None) -> int:
        v = np.ascontiguousarray(vars_, dtype=np.int32)
        lbp = ubp = None
        keep = [v]
        if kind == REQ_PROPAGATE:
            lbp = np.ascontiguousarray(lb, dtype=np.float64)
            ubp = np.ascontiguousarray(ub, dtype=np.float64)
            keep += [lbp, ubp]
        r = Request(instance, kind, v.size, 0, v.ctypes.data if v.size else None,
                    lbp.ctypes.data if lbp is not None and lbp.size else None,
                    ubp.ctypes.data if ubp is not None and ubp.size else None)
        rid = C.c_int64()
        _check(_LIB.bp_server_submit(self._h, C.byref(r), C.byref(rid)))
        return rid.value

    def run(self, rounds: int) -> int:
        busy = C.c_int32()
        _check(_LIB.bp_server_run(self._h, rounds, C.byref(busy)))
        return busy.value

    def poll(self, max_items: int = 4096):
        buf = (Completion * max_items)()
        n = C.c_int32()
        _check(_LIB.bp_server_poll(self._h, buf, max_items, C.byref(n)))
        return [dict(id=buf[i].id, instance=buf[i].instance, kind=buf[i].kind, jobs=buf[i].jobs,
                     cancelled=bool(buf[i].flags & COMPLETION_CANCELLED),
                     submit_us=buf[i].submit_us, done_us=buf[i].done_us) for i in range(n.value)]

    def add_instance(self, instance) -> int:
        """bp_server_add_instance: serve one more loaded Instance; returns
        its index."""
        t = C.c_int32()
        _check(_LIB.bp_server_add_instance(self._h, instance._h, C.byref(t)))
        while len(self._insts) <= t.value:
            self._insts.append(None)
        self._insts[t.value] = instance
        return t.value

    def evict(self, index: int):
        """bp_server_evict: stop serving instance `index` (BP_ESTATE while it
        has unfinished requests)."""
        _check(_LIB.bp_server_evict(self._h, index))
        self._insts[index] = None

    def cancel(self, rid: int):
        """bp_server_cancel: take a request that still waits in the host
        queue out of it (BPError with BP_ESTATE once its jobs are on the
        device)."""
        _check(_LIB.bp_server_cancel(self._h, rid))

    def expire(self, max_wait_us: float) -> int:
        """bp_server_expire: cancel the host-queued requests that waited
        longer than max_wait_us; returns how many."""
        n = C.c_int32()
        _check(_LIB.bp_server_expire(self._h, float(max_wait_us), C.byref(n)))
        return n.value

    def results(self, rid: int, jobs: int) -> dict:
        req = C.c_int64()
        cap = 0
        while True:
            st = np.zeros(jobs, np.int8)
            rd = np.zeros(jobs, np.int32)
            nz = np.zeros(jobs, np.int64)
            nb = np.zeros(jobs, np.int32)
            br = np.zeros(jobs, np.int32)
            bv = np.zeros(jobs, np.int32)
            off = np.zeros(jobs + 1, np.int64)
            var = np.zeros(max(cap, 1), np.int32)
            lb = np.zeros(max(cap, 1))
            ub = np.zeros(max(cap, 1))
            rc = _LIB.bp_server_results(self._h, rid, st.ctypes.data, rd.ctypes.data,
                                        nz.ctypes.data, nb.ctypes.data, br.ctypes.data,
                                        bv.ctypes.data, off.ctypes.data, var.ctypes.data,
                                        lb.ctypes.data, ub.ctypes.data, cap, C.byref(req))
            if rc == BP_ECAPACITY:
                cap = int(req.value)
                continue
            _check(rc)
            tot = int(off[-1])
            return dict(status=st, rounds=rd, nnz=nz, n_infeasible_rows=nb, infeasible_row=br,
                        infeasible_var=bv, off=off, var=var[:tot], lb=lb[:tot], ub=ub[:tot])


# ---------------------------------------------------------------------------
# Probing cache files (bp_probe output kept for later rounding calls)
# ---------------------------------------------------------------------------
CACHE_KEYS = ("vars", "status", "rounds", "nnz", "off", "var", "lb", "ub")


def _cache_sha256(arrays: dict) -> str:
    import hashlib
    h = hashlib.sha256()
    for k in CACHE_KEYS:
        a = np.ascontiguousarray(arrays[k])
        h.update(k.encode())
        h.update(str(a.dtype).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def save_probe_cache(path: str, vars_: torch.Tensor, probe_out: dict, instance_sha256: str = None) -> str:
    """Write a probing cache (the probed variables and Instance.probe's
    output) to ``path`` (.npz) with a manifest ``path + '.sha256.json'``
    holding the content digest and, if given, the digest of the instance it
    was computed on.  Returns the content digest."""
    import json
    arrays = {"vars": vars_.detach().cpu().numpy()}
    for k in CACHE_KEYS[1:]:
        arrays[k] = probe_out[k].detach().cpu().numpy()
    with open(path, "wb") as fh:
        np.savez(fh, **arrays)
    digest = _cache_sha256(arrays)
    with open(path + ".sha256.json", "w") as fh:
        json.dump({"sha256": digest, "instance_sha256": instance_sha256,
                   "probes": int(arrays["vars"].size)}, fh, indent=1, sort_keys=True)
    return digest


def load_probe_cache(path: str, device="cuda", instance_sha256: str = None) -> dict:
    """Read a cache written by save_probe_cache into device tensors (the dict
    Instance.round takes as ``cache``).  ValueError if the content does not
    match its manifest, or the manifest names another instance than
    ``instance_sha256``."""
    import json
    with np.load(path, allow_pickle=False) as z:
        arrays = {k: z[k] for k in CACHE_KEYS}
    with open(path + ".sha256.json") as fh:
        man = json.load(fh)
    if _cache_sha256(arrays) != man["sha256"]:
        raise ValueError("probing cache %s does not match its manifest" % path)
    if instance_sha256 is not None and man.get("instance_sha256") != instance_sha256:
        raise ValueError("probing cache %s was computed on another instance" % path)
    k = int(arrays["vars"].size)
    off = arrays["off"]
    if off.size != 2 * k + 1 or arrays["status"].size != 2 * k or int(off[-1]) != arrays["var"].size:
        raise ValueError("probing cache %s has inconsistent sizes" % path)
    return {key: torch.from_numpy(a).to(device) for key, a in arrays.items()}
