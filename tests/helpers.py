"""Shared test helpers: golden fixtures, brute force and an exact-rational
Gauss-Seidel propagator written independently of the C oracle."""
from __future__ import annotations

import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np

from paper_2510_20499_amd import gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _f(x):
    return float(x)  # json strings "inf"/"-inf" → float


def load_golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        d = json.load(fh)
    inst = gen.from_rows(d["n"], [(c, v) for c, v in d["rows"]],
                         [_f(x) for x in d["lo"]], [_f(x) for x in d["hi"]], d["vtype"],
                         [_f(x) for x in d["lb"]], [_f(x) for x in d["ub"]])
    return inst, d


def rows_of(inst):
    rp, c, v = inst["row_ptr"], inst["col"], inst["val"]
    return [(c[rp[k]:rp[k + 1]], v[rp[k]:rp[k + 1]]) for k in range(inst["m"])]


def feasible_points(inst, lb=None, ub=None):
    """All integer points of the box that satisfy every row (micro only)."""
    lb = inst["lb"] if lb is None else lb
    ub = inst["ub"] if ub is None else ub
    doms = [range(int(lb[i]), int(ub[i]) + 1) for i in range(inst["n"])]
    rows = rows_of(inst)
    out = []
    for x in itertools.product(*doms):
        ok = True
        for k, (c, v) in enumerate(rows):
            s = sum(int(v[t]) * x[c[t]] for t in range(len(c)))
            if s < inst["lo"][k] or s > inst["hi"][k]:
                ok = False
                break
        if ok:
            out.append(x)
    return out


def exact_gs_fixed_point(inst, lb=None, ub=None, inttol=Fraction(1, 10**6)):
    """Pure-integer greatest fixed point by Gauss-Seidel sweeps in exact
    rational arithmetic: rows are visited one at a time and every tightening
    is applied at once (a different schedule from round-synchronous rounds).
    Returns (feasible, lb, ub) with Fractions; feasible False when the box
    became empty."""
    lb = [Fraction(int(x)) for x in (inst["lb"] if lb is None else lb)]
    ub = [Fraction(int(x)) for x in (inst["ub"] if ub is None else ub)]
    rows = rows_of(inst)
    lo = inst["lo"]
    hi = inst["hi"]
    changed = True
    while changed:
        changed = False
        for k, (c, v) in enumerate(rows):
            a = [Fraction(int(t)) for t in v]
            idx = [int(t) for t in c]
            # Upper side: sum a x <= hi.
            if math.isfinite(hi[k]):
                g = Fraction(hi[k])
                for t, i in enumerate(idx):
                    rest = sum((a[s] * (lb[j] if a[s] > 0 else ub[j])) for s, j in enumerate(idx) if s != t)
                    bound = (g - rest) / a[t]
                    if a[t] > 0:
                        nb = math.floor(bound + inttol)
                        if nb < ub[i]:
                            ub[i] = Fraction(nb); changed = True
                    else:
                        nb = math.ceil(bound - inttol)
                        if nb > lb[i]:
                            lb[i] = Fraction(nb); changed = True
                    if lb[i] > ub[i]:
                        return False, lb, ub
            if math.isfinite(lo[k]):
                g = Fraction(lo[k])
                for t, i in enumerate(idx):
                    rest = sum((a[s] * (ub[j] if a[s] > 0 else lb[j])) for s, j in enumerate(idx) if s != t)
                    bound = (g - rest) / a[t]
                    if a[t] > 0:
                        nb = math.ceil(bound - inttol)
                        if nb > lb[i]:
                            lb[i] = Fraction(nb); changed = True
                    else:
                        nb = math.floor(bound + inttol)
                        if nb < ub[i]:
                            ub[i] = Fraction(nb); changed = True
                    if lb[i] > ub[i]:
                        return False, lb, ub
    # A row may still be violated with all its bounds fixed (no tightening
    # possible): check activity bounds once more.
    for k, (c, v) in enumerate(rows):
        mn = sum(Fraction(int(a)) * (lb[i] if a > 0 else ub[i]) for i, a in zip(c, v))
        mx = sum(Fraction(int(a)) * (ub[i] if a > 0 else lb[i]) for i, a in zip(c, v))
        if mn > hi[k] or mx < lo[k]:
            return False, lb, ub
    return True, lb, ub


def implied_dict(P, p):
    a, b = int(P["off"][p]), int(P["off"][p + 1])
    return {int(P["var"][t]): (float(P["lb"][t]), float(P["ub"][t])) for t in range(a, b)}


def rel_close(a, b, tol=1e-9):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    same = (a == b)
    scale = np.maximum(1.0, np.abs(np.where(np.isfinite(a), a, 0.0)))
    with np.errstate(invalid="ignore"):
        near = np.abs(a - b) <= tol * scale
    return bool(np.all(same | near))
