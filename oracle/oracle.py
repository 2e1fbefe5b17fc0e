"""ctypes front end of the C oracle ``bp_oracle.c`` (test infrastructure only).

The C file is compiled with gcc, without FMA contraction and without fast
math, into ``liborc.so`` next to it.  Nothing here is shared with the GPU
library: the two sides only receive the same seeded input arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bp_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

BP_OK, BP_INFEASIBLE, BP_ROUND_LIMIT = 0, 1, 2
MODE_WORKLIST, MODE_DEFINITION = 0, 1


@dataclass
class Options:
    feastol: float = 1e-6
    inttol: float = 1e-6
    tau: float = 1e-3
    max_rounds: int = 1000


class _Inst(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("lo", C.c_void_p), ("hi", C.c_void_p), ("vtype", C.c_void_p)]


class _Opt(C.Structure):
    _fields_ = [("feastol", C.c_double), ("inttol", C.c_double), ("tau", C.c_double),
                ("max_rounds", C.c_int32)]


class _Res(C.Structure):
    _fields_ = [("status", C.c_int32), ("rounds", C.c_int32), ("nnz_propagated", C.c_int64),
                ("n_infeasible_rows", C.c_int32), ("infeasible_row", C.c_int64),
                ("infeasible_var", C.c_int32)]


class _RoundRes(C.Structure):
    _fields_ = [("status", C.c_int32), ("bulks", C.c_int32), ("singles", C.c_int32),
                ("recoveries", C.c_int32), ("fixed", C.c_int32), ("iterations", C.c_int32),
                ("nnz_propagated", C.c_int64), ("repairs", C.c_int32), ("repaired", C.c_int32)]


class _RepairLimits(C.Structure):
    _fields_ = [("calls", C.c_int32), ("attempts", C.c_int32), ("shifts", C.c_int32)]


class _RepairRes(C.Structure):
    _fields_ = [("status", C.c_int32), ("attempts", C.c_int32), ("shifts", C.c_int32),
                ("reason", C.c_int32), ("nnz_propagated", C.c_int64)]


_lib = None


def compile_to(src: str, out: str) -> str:
    """gcc -O2, no FMA contraction, no fast math."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle when the library is missing or older than its source."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_to(SRC, LIB)
    return LIB


def bind(path: str):
    """Load an oracle library built from ``bp_oracle.c`` (or a variant of it)."""
    lib = C.CDLL(path)
    lib.orc_exact_sum.restype = C.c_double
    lib.orc_exact_sum.argtypes = [C.c_void_p, C.c_int64]
    lib.orc_validate.restype = C.c_int
    lib.orc_validate.argtypes = [C.POINTER(_Inst)]
    lib.orc_propagate.restype = C.c_int
    lib.orc_propagate.argtypes = [C.POINTER(_Inst), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int64, C.POINTER(_Opt), C.c_int, C.POINTER(_Res)]
    lib.orc_probe_box.restype = C.c_int
    lib.orc_probe_box.argtypes = [C.c_double, C.c_double, C.c_int, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]
    lib.orc_probe.restype = C.c_int
    lib.orc_probe.argtypes = [C.POINTER(_Inst), C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_int32, C.POINTER(_Opt), C.c_int] + [C.c_void_p] * 8 + \
                             [C.c_int64, C.POINTER(C.c_int64)]
    lib.orc_scores.restype = C.c_int
    lib.orc_scores.argtypes = [C.POINTER(_Inst), C.c_void_p, C.c_void_p, C.POINTER(_Opt)] + \
                              [C.c_void_p] * 4
    lib.orc_probe_order.restype = C.c_int
    lib.orc_probe_order.argtypes = [C.POINTER(_Inst), C.c_void_p, C.c_void_p, C.POINTER(_Opt),
                                    C.c_void_p, C.c_int32, C.c_void_p]
    lib.orc_round.restype = C.c_int
    lib.orc_round.argtypes = [C.POINTER(_Inst), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_int32] + [C.c_void_p] * 6 + [C.POINTER(_Opt),
                                                                C.POINTER(_RepairLimits),
                                                                C.POINTER(_RoundRes)]
    lib.orc_repair.restype = C.c_int
    lib.orc_repair.argtypes = [C.POINTER(_Inst), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int32, C.c_int32, C.POINTER(_Opt), C.POINTER(_RepairRes)]
    return lib


def load():
    global _lib
    if _lib is None:
        build()
        _lib = bind(LIB)
    return _lib




def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class _Held:
    """Keeps contiguous copies alive while the C side reads them."""

    def __init__(self, inst):
        self.row_ptr = np.ascontiguousarray(inst["row_ptr"], dtype=np.int64)
        self.col = np.ascontiguousarray(inst["col"], dtype=np.int32)
        self.val = np.ascontiguousarray(inst["val"], dtype=np.float64)
        self.lo = np.ascontiguousarray(inst["lo"], dtype=np.float64)
        self.hi = np.ascontiguousarray(inst["hi"], dtype=np.float64)
        self.vtype = np.ascontiguousarray(inst["vtype"], dtype=np.uint8)
        self.s = _Inst(int(inst["m"]), int(inst["n"]), int(self.row_ptr[-1]),
                       _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val), _ptr(self.lo),
                       _ptr(self.hi), _ptr(self.vtype))


def _opt(o):
    o = o or Options()
    return _Opt(o.feastol, o.inttol, o.tau, o.max_rounds)


def exact_sum(x, lib=None) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float((lib or load()).orc_exact_sum(_ptr(x), x.size))


def validate(inst, lib=None) -> int:
    h = _Held(inst)
    return int((lib or load()).orc_validate(C.byref(h.s)))


def propagate(inst, lb=None, ub=None, changed=None, opts: Options = None,
              mode: int = MODE_WORKLIST, lib=None):
    """Round-synchronous propagation.  Returns (result dict, lb, ub)."""
    lib = lib or load()
    h = _Held(inst)
    lb = np.array(inst["lb"] if lb is None else lb, dtype=np.float64, copy=True)
    ub = np.array(inst["ub"] if ub is None else ub, dtype=np.float64, copy=True)
    res = _Res()
    if changed is None:
        rc = lib.orc_propagate(C.byref(h.s), _ptr(lb), _ptr(ub), None, -1,
                                  C.byref(_opt(opts)), mode, C.byref(res))
    else:
        ch = np.ascontiguousarray(changed, dtype=np.int32)
        rc = lib.orc_propagate(C.byref(h.s), _ptr(lb), _ptr(ub),
                                  _ptr(ch) if ch.size else C.c_void_p(1), ch.size,
                                  C.byref(_opt(opts)), mode, C.byref(res))
    if rc < 0:
        raise ValueError("oracle propagate failed with code %d" % rc)
    out = dict(status=res.status, rounds=res.rounds, nnz_propagated=res.nnz_propagated,
               n_infeasible_rows=res.n_infeasible_rows, infeasible_row=res.infeasible_row,
               infeasible_var=res.infeasible_var)
    return out, lb, ub


def probe(inst, base_lb, base_ub, vars_, opts: Options = None, mode: int = MODE_WORKLIST,
          lib=None):
    """Double probing of integer variables around the base (Section 2.2).
    Probe 2t+h restricts vars[t] to probe_box(l, u, h): x = h for a binary,
    the halves split at (l + u) / 2 for a boxed integer, x = l / x >= l + 1
    (x <= u - 1 / x = u) for a one-sided one.  Returns a dict of arrays:
    status/rounds/nnz/n_infeasible_rows per probe, off[2k+1] and the
    concatenated implied (var, lb, ub) lists."""
    lib = lib or load()
    h = _Held(inst)
    base_lb = np.ascontiguousarray(base_lb, dtype=np.float64)
    base_ub = np.ascontiguousarray(base_ub, dtype=np.float64)
    vs = np.ascontiguousarray(vars_, dtype=np.int32)
    k = vs.size
    st = np.zeros(2 * k, np.int8)
    rd = np.zeros(2 * k, np.int32)
    nz = np.zeros(2 * k, np.int64)
    nir = np.zeros(2 * k, np.int32)
    off = np.zeros(2 * k + 1, np.int64)
    cap = 1 << 16
    while True:
        iv = np.zeros(cap, np.int32)
        il = np.zeros(cap)
        iu = np.zeros(cap)
        req = C.c_int64(0)
        rc = lib.orc_probe(C.byref(h.s), _ptr(base_lb), _ptr(base_ub), _ptr(vs), k,
                              C.byref(_opt(opts)), mode, _ptr(st), _ptr(rd), _ptr(nz),
                              _ptr(nir), _ptr(off), _ptr(iv), _ptr(il), _ptr(iu), cap,
                              C.byref(req))
        if rc == -4:
            cap = int(req.value)
            continue
        if rc < 0:
            raise ValueError("oracle probe failed with code %d" % rc)
        tot = int(off[-1])
        return dict(status=st, rounds=rd, nnz=nz, n_infeasible_rows=nir, off=off,
                    var=iv[:tot].copy(), lb=il[:tot].copy(), ub=iu[:tot].copy())


def probe_box(l, u, h, lib=None):
    """The box (lo, hi) probe h in {0, 1} restricts an integer variable with
    base bounds [l, u] to, before intersecting with [l, u]; None for a
    variable with no finite bound."""
    lib = lib or load()
    a, b = C.c_double(), C.c_double()
    if lib.orc_probe_box(float(l), float(u), int(h), C.byref(a), C.byref(b)) != 0:
        return None
    return a.value, b.value


def _bounds(inst, lb, ub):
    lb = np.ascontiguousarray(inst["lb"] if lb is None else lb, dtype=np.float64)
    ub = np.ascontiguousarray(inst["ub"] if ub is None else ub, dtype=np.float64)
    return lb, ub


def scores(inst, lb=None, ub=None, opts: Options = None, lib=None):
    """Probe-priority and implied-slack scores of every variable at (lb, ub)
    (Sections 2.2 and 2.3): nviol (rows violated when the variable's
    contribution flips between its bounds; only variables whose column mixes
    signs and whose bounds are finite), maxviol (the largest such violation),
    minunit (smallest slack / |a| over the finite row sides without infinite
    terms) and slack_score (S = sum of (a / slack)^2 over the same sides)."""
    lib = lib or load()
    h = _Held(inst)
    lb, ub = _bounds(inst, lb, ub)
    n = int(inst["n"])
    out = dict(nviol=np.zeros(n, np.int32), maxviol=np.zeros(n), minunit=np.zeros(n),
               slack_score=np.zeros(n))
    rc = lib.orc_scores(C.byref(h.s), _ptr(lb), _ptr(ub), C.byref(_opt(opts)),
                        _ptr(out["nviol"]), _ptr(out["maxviol"]), _ptr(out["minunit"]),
                        _ptr(out["slack_score"]))
    if rc < 0:
        raise ValueError("oracle scores failed with code %d" % rc)
    return out


def probe_order(inst, vars_, lb=None, ub=None, opts: Options = None, lib=None):
    """The listed variables in probe order (Section 2.2): more violated rows
    first, then the larger maximum violation, the smaller minimum unit slack,
    the smaller index."""
    lib = lib or load()
    h = _Held(inst)
    lb, ub = _bounds(inst, lb, ub)
    vs = np.ascontiguousarray(vars_, dtype=np.int32)
    order = np.zeros(max(vs.size, 1), np.int32)
    rc = lib.orc_probe_order(C.byref(h.s), _ptr(lb), _ptr(ub), C.byref(_opt(opts)), _ptr(vs),
                             vs.size, _ptr(order))
    if rc < 0:
        raise ValueError("oracle probe order failed with code %d" % rc)
    return order[:vs.size]


def repair(inst, lb, ub, lb0=None, ub0=None, max_shifts: int = 64, max_attempts: int = 8,
           opts: Options = None, lib=None):
    """Repair procedure (Section 2.3; Algorithm 1's Run-Repair-Procedure) of
    the box (lb, ub) inside the original box (lb0, ub0), default the
    instance's bounds.  Returns (result dict, lb, ub): the repaired box, or
    the given one when the repair fails."""
    lib = lib or load()
    h = _Held(inst)
    lb = np.array(lb, dtype=np.float64, copy=True)
    ub = np.array(ub, dtype=np.float64, copy=True)
    lb0 = np.ascontiguousarray(inst["lb"] if lb0 is None else lb0, dtype=np.float64)
    ub0 = np.ascontiguousarray(inst["ub"] if ub0 is None else ub0, dtype=np.float64)
    r = _RepairRes()
    rc = lib.orc_repair(C.byref(h.s), _ptr(lb), _ptr(ub), _ptr(lb0), _ptr(ub0), int(max_shifts),
                        int(max_attempts), C.byref(_opt(opts)), C.byref(r))
    if rc < 0:
        raise ValueError("oracle repair failed with code %d" % rc)
    out = dict(status=r.status, attempts=r.attempts, shifts=r.shifts, reason=r.reason,
               nnz_propagated=r.nnz_propagated)
    return out, lb, ub


def round_(inst, x, draws, lb=None, ub=None, cache=None, opts: Options = None, lib=None,
           repair=None):
    """Bound-propagation rounding (Algorithm 1 without the LP polish) of the
    integer variables of the box (lb, ub) towards the point x, with the
    uniform draws draws[2j + h] for the two candidate bulks, an optional
    probing cache of binaries (dict with vars and the probe() output) and
    optional repair limits (calls, attempts, shifts); without them no
    repair runs.  Returns (result dict, lb, ub)."""
    lib = lib or load()
    h = _Held(inst)
    lb = np.array(inst["lb"] if lb is None else lb, dtype=np.float64, copy=True)
    ub = np.array(inst["ub"] if ub is None else ub, dtype=np.float64, copy=True)
    x = np.ascontiguousarray(x, dtype=np.float64)
    draws = np.ascontiguousarray(draws, dtype=np.float64)
    if cache is None:
        k = 0
        arrs = [np.zeros(1, np.int32), np.zeros(2, np.int8), np.zeros(3, np.int64),
                np.zeros(1, np.int32), np.zeros(1), np.zeros(1)]
    else:
        vs = np.ascontiguousarray(cache["vars"], dtype=np.int32)
        k = vs.size
        arrs = [vs, np.ascontiguousarray(cache["status"], dtype=np.int8),
                np.ascontiguousarray(cache["off"], dtype=np.int64),
                np.ascontiguousarray(cache["var"], dtype=np.int32) if len(cache["var"]) else np.zeros(1, np.int32),
                np.ascontiguousarray(cache["lb"], dtype=np.float64) if len(cache["lb"]) else np.zeros(1),
                np.ascontiguousarray(cache["ub"], dtype=np.float64) if len(cache["ub"]) else np.zeros(1)]
    r = _RoundRes()
    rp = None if repair is None else C.byref(_RepairLimits(*[int(v) for v in repair]))
    rc = lib.orc_round(C.byref(h.s), _ptr(lb), _ptr(ub), _ptr(x), _ptr(draws), k,
                       *[_ptr(a) for a in arrs], C.byref(_opt(opts)), rp, C.byref(r))
    if rc < 0:
        raise ValueError("oracle round failed with code %d" % rc)
    out = dict(status=r.status, bulks=r.bulks, singles=r.singles, recoveries=r.recoveries,
               fixed=r.fixed, iterations=r.iterations, nnz_propagated=r.nnz_propagated)
    if repair is not None:
        out.update(repairs=r.repairs, repaired=r.repaired)
    return out, lb, ub
