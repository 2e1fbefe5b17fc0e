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


def load_golden_cases(name):
    """A fixture holding several small hand-computed cases: [(inst, case)]."""
    with open(os.path.join(GOLDEN, name + ".json")) as fh:
        d = json.load(fh)
    out = []
    for c in d["cases"]:
        inst = gen.from_rows(c["n"], [(cc, v) for cc, v in c["rows"]],
                             [_f(x) for x in c["lo"]], [_f(x) for x in c["hi"]], c["vtype"],
                             [_f(x) for x in c["lb"]], [_f(x) for x in c["ub"]])
        out.append((inst, c))
    return out


def bits(a):
    """Bit patterns of doubles (tells +0.0 from -0.0)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64)).view(np.int64)


RESULT_FIELDS = ("status", "rounds", "nnz_propagated", "n_infeasible_rows", "infeasible_row",
                 "infeasible_var")


def case_mismatch(c, r, lb, ub):
    """None if a propagation result (r, lb, ub) is the hand-computed cold
    result of fixture case c (bounds bit for bit when feasible), else a
    description of the first difference."""
    exp = c["cold"]
    for f in RESULT_FIELDS:
        if r[f] != exp[f]:
            return "%s: %s got %r want %r" % (c["name"], f, r[f], exp[f])
    if "lb" in exp:
        if not np.array_equal(bits(lb), bits([_f(x) for x in exp["lb"]])):
            return "%s: lb %r want %r" % (c["name"], list(lb), exp["lb"])
        if not np.array_equal(bits(ub), bits([_f(x) for x in exp["ub"]])):
            return "%s: ub %r want %r" % (c["name"], list(ub), exp["ub"])
    return None


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


# ---------------------------------------------------------------------------
# Slack filter of the row kernels, restated for tests.  A row none of whose
# candidates can be taken skips its candidate pass on the GPU; the rule must
# never skip a row the definition would let tighten a bound.
# ---------------------------------------------------------------------------
INF = math.inf


def filter_width(a, lb, ub):
    """Width of one nonzero: |a| (ub - lb + 1 + 2^-50 max|bound|) (1 + 2^-40),
    in the kernels' operation order (each step rounded to double)."""
    d = ub - lb
    d = d + 1.0
    d = d + max(abs(lb), abs(ub)) * 2.0 ** -50
    return (abs(a) * d) * (1.0 + 2.0 ** -40)


def filter_quiet(minfin, maxfin, nmin, nmax, lo, hi, rng):
    """The kernels' decision that no candidate of a row can be taken."""
    fin = rng < INF
    qhi = hi == INF or nmin >= 2 or (nmin == 0 and fin and hi - minfin >= rng)
    qlo = lo == -INF or nmax >= 2 or (nmax == 0 and fin and maxfin - lo >= rng)
    return qhi and qlo


def slack_edge_instance(seed, count=300, naive=False, lengths=(1, 7)):
    """Rows with disjoint variables whose slack is placed at the slack
    filter's threshold, give or take a few ulps to 1e-3 relative: binaries,
    integers with non-integral bounds, continuous variables of magnitude up
    to 1e13 with small domains, coefficients of magnitude 1e-3..1e3.
    naive=True places the slack at max |a| (ub - lb) instead (the threshold
    without the integer unit and the rounding margins).  Returns the
    instance and, per row, (minfin, maxfin, width).  Row lengths are
    uniform in [lengths[0], lengths[1])."""
    rs = np.random.default_rng(seed)
    rows, lo, hi, vt, lb, ub, info = [], [], [], [], [], [], []
    eps = [0.0, 2.0 ** -52, -2.0 ** -52, 2.0 ** -45, -2.0 ** -45, 2.0 ** -40, -2.0 ** -40,
           1e-9, -1e-9, 1e-3, -1e-3]
    n = 0
    for _ in range(count):
        L = int(rs.integers(lengths[0], lengths[1]))
        cols = list(range(n, n + L))
        n += L
        vals, ls, us = [], [], []
        for _ in range(L):
            kind = int(rs.integers(0, 4))
            if kind == 0:
                l, u, t = 0.0, 1.0, 1
            elif kind == 1:
                l = float(rs.integers(-5, 5)) + float(rs.choice([0.0, 0.25, 0.5]))
                u = l + float(rs.integers(1, 8)) + float(rs.choice([0.0, 0.3]))
                t = 1
            elif kind == 2:
                c = float(rs.choice([-1.0, 1.0])) * 10.0 ** rs.uniform(6, 13)
                l, u, t = c, c + 10.0 ** rs.uniform(-4, 2), 0
            else:
                l = rs.uniform(-100, 0)
                u, t = l + rs.uniform(0, 200), 0
            vals.append(float(rs.choice([-1.0, 1.0])) * 10.0 ** rs.uniform(-3, 3))
            ls.append(float(l))
            us.append(float(u))
            vt.append(t)
        tmin = [a * l if a > 0 else a * u for a, l, u in zip(vals, ls, us)]
        tmax = [a * u if a > 0 else a * l for a, l, u in zip(vals, ls, us)]
        mn, mx = math.fsum(tmin), math.fsum(tmax)
        if naive:
            w = max(abs(a) * (u - l) for a, l, u in zip(vals, ls, us))
        else:
            w = max(filter_width(a, l, u) for a, l, u in zip(vals, ls, us))
        kind = int(rs.integers(0, 3))  # 0: a.x <= hi, 1: lo <= a.x, 2: both
        h = mn + w * (1.0 + eps[int(rs.integers(len(eps)))]) if kind != 1 else INF
        g = mx - w * (1.0 + eps[int(rs.integers(len(eps)))]) if kind != 0 else -INF
        if g > h:  # both sides at the threshold would cross: keep the upper one
            g = -INF
        rows.append((cols, vals))
        lo.append(g)
        hi.append(h)
        lb.extend(ls)
        ub.extend(us)
        info.append((mn, mx, max(filter_width(a, l, u) for a, l, u in zip(vals, ls, us))))
    inst = gen.from_rows(n, rows, lo, hi, vt, lb, ub)
    return inst, info


def stack_instances(parts):
    """Block-diagonal instance of the given instances (disjoint variables)."""
    rows, lo, hi, vt, lb, ub = [], [], [], [], [], []
    n = 0
    for inst in parts:
        rp = inst["row_ptr"]
        for k in range(inst["m"]):
            rows.append((inst["col"][rp[k]:rp[k + 1]] + n, inst["val"][rp[k]:rp[k + 1]]))
        lo.extend(inst["lo"])
        hi.extend(inst["hi"])
        vt.extend(inst["vtype"])
        lb.extend(inst["lb"])
        ub.extend(inst["ub"])
        n += inst["n"]
    return gen.from_rows(n, rows, lo, hi, vt, lb, ub)


def row_instance(inst, k):
    """Row k alone, over its own variables."""
    rp = inst["row_ptr"]
    c = inst["col"][rp[k]:rp[k + 1]]
    v = inst["val"][rp[k]:rp[k + 1]]
    return gen.from_rows(len(c), [(np.arange(len(c)), v)], [inst["lo"][k]], [inst["hi"][k]],
                         inst["vtype"][c], inst["lb"][c], inst["ub"][c])


def keep_rows(inst, ks):
    """The rows ks of inst (variables unchanged; others become empty columns)."""
    rp = inst["row_ptr"]
    rows = [(inst["col"][rp[k]:rp[k + 1]], inst["val"][rp[k]:rp[k + 1]]) for k in ks]
    return gen.from_rows(inst["n"], rows, inst["lo"][ks], inst["hi"][ks], inst["vtype"],
                         inst["lb"], inst["ub"])



def box_extremes(inst, k, lb, ub, fix=None):
    """Exact minimum and maximum of row k's activity over the box, with
    variable fix = (j, value) held at value.  The activity is separable, so
    each term ranges between its values at the two ends of its interval (a
    product with an infinite end is infinite).  None for an unbounded side."""
    rp = inst["row_ptr"]
    lo, hi = Fraction(0), Fraction(0)
    for i, a in zip(inst["col"][rp[k]:rp[k + 1]], inst["val"][rp[k]:rp[k + 1]]):
        ends = [fix[1]] if fix is not None and i == fix[0] else [lb[i], ub[i]]
        vals = [math.copysign(INF, a) * math.copysign(1.0, b) if math.isinf(b)
                else Fraction(float(a)) * Fraction(float(b)) for b in ends]
        tmin, tmax = min(vals), max(vals)
        lo = None if lo is None or tmin == -INF else lo + tmin
        hi = None if hi is None or tmax == INF else hi + tmax
    return lo, hi


def brute_scores(inst, lb, ub, feastol=1e-6):
    """Scores from their meaning, in exact rationals: the row's extreme
    activities over the box with the variable held at the bound that pushes
    the row hardest; slack = distance from the extreme activity to the side."""
    n, m = inst["n"], inst["m"]
    rp, col, val = inst["row_ptr"], inst["col"], inst["val"]
    signs = [set() for _ in range(n)]
    for p in range(len(col)):
        signs[col[p]].add(val[p] > 0)
    nviol = [0] * n
    maxviol = [Fraction(0)] * n
    units = [[] for _ in range(n)]
    terms = [[] for _ in range(n)]
    for k in range(m):
        mn, mx = box_extremes(inst, k, lb, ub)
        hi, lo = inst["hi"][k], inst["lo"][k]
        sides = []
        if not math.isinf(hi) and mn is not None:
            sides.append(Fraction(float(hi)) - mn)
        if not math.isinf(lo) and mx is not None:
            sides.append(mx - Fraction(float(lo)))
        for p in range(rp[k], rp[k + 1]):
            j, a = int(col[p]), float(val[p])
            for sl in sides:
                units[j].append(sl / abs(Fraction(a)))
                terms[j].append(None if sl == 0 else (Fraction(a) / sl) ** 2)
            if len(signs[j]) == 2 and not math.isinf(lb[j]) and not math.isinf(ub[j]):
                push_up = ub[j] if a > 0 else lb[j]      # raises the minimum activity
                push_down = lb[j] if a > 0 else ub[j]    # lowers the maximum activity
                worst = None
                if not math.isinf(hi):
                    fmn, _ = box_extremes(inst, k, lb, ub, fix=(j, push_up))
                    if fmn is not None and fmn - Fraction(float(hi)) > Fraction(feastol):
                        worst = fmn - Fraction(float(hi))
                if not math.isinf(lo):
                    _, fmx = box_extremes(inst, k, lb, ub, fix=(j, push_down))
                    if fmx is not None and Fraction(float(lo)) - fmx > Fraction(feastol):
                        e = Fraction(float(lo)) - fmx
                        worst = e if worst is None or e > worst else worst
                if worst is not None:
                    nviol[j] += 1
                    maxviol[j] = max(maxviol[j], worst)
    return nviol, maxviol, units, terms


def round_scenarios():
    """The hand-traced rounding scenarios of tests/golden/w6_round.json:
    (name, instance, spec) with spec holding x, draws, the expected counts
    and final values, and an optional hand-written cache."""
    with open(os.path.join(GOLDEN, "w6_round.json")) as fh:
        d = json.load(fh)
    out = []
    for key in ("A", "B", "C", "D"):
        s = d[key]
        inst = gen.from_rows(s["n"], [(c, v) for c, v in s["rows"]], [_f(x) for x in s["lo"]],
                             [_f(x) for x in s["hi"]], s["vtype"], [_f(x) for x in s["lb"]],
                             [_f(x) for x in s["ub"]])
        if "cache" in s:
            s = dict(s)
            s["cache"] = {k: np.asarray(v) for k, v in s["cache"].items()}
        out.append((key, inst, s))
    return out


def row_violations(inst, x, tol=0.0):
    """Rows of inst violated at the point x (exact for integer data)."""
    rp, col, val = inst["row_ptr"], inst["col"], inst["val"]
    bad = []
    for k in range(inst["m"]):
        s = sum(Fraction(float(val[p])) * Fraction(float(x[col[p]])) for p in range(rp[k], rp[k + 1]))
        lo, hi = inst["lo"][k], inst["hi"][k]
        if (not math.isinf(lo) and s < Fraction(float(lo)) - Fraction(tol)) or \
                (not math.isinf(hi) and s > Fraction(float(hi)) + Fraction(tol)):
            bad.append(k)
    return bad


def repair_cases():
    """The hand-traced repair cases of tests/golden/w8_repair.json:
    [(instance, case)]; the instance's bounds are the original box, the
    case holds the given box, the limits and the expected result."""
    return load_golden_cases("w8_repair")


def repair_round_scenario():
    """The hand-traced rounding-with-repair scenario of w8_repair.json:
    (instance, spec)."""
    with open(os.path.join(GOLDEN, "w8_repair.json")) as fh:
        s = json.load(fh)["rounding"]
    inst = gen.from_rows(s["n"], [(c, v) for c, v in s["rows"]], [_f(x) for x in s["lo"]],
                         [_f(x) for x in s["hi"]], s["vtype"], [_f(x) for x in s["lb"]],
                         [_f(x) for x in s["ub"]])
    return inst, s


def repair_case_mismatch(c, r, lb, ub):
    """None if a repair result matches hand-traced case c, else the first
    difference."""
    if r != c["result"]:
        return "%s: result %r want %r" % (c["name"], r, c["result"])
    if not np.array_equal(bits(lb), bits([_f(x) for x in c["final_lb"]])):
        return "%s: lb %r want %r" % (c["name"], list(lb), c["final_lb"])
    if not np.array_equal(bits(ub), bits([_f(x) for x in c["final_ub"]])):
        return "%s: ub %r want %r" % (c["name"], list(ub), c["final_ub"])
    return None


def single_row_repair_instance(seed):
    """A pure-integer instance of one row (2-5 variables, coefficients in
    [-5, 5] without 0, original domains inside {0..6}) and a point of the
    domains that violates the row: (instance, point)."""
    rng = np.random.default_rng(1000 + seed)
    while True:
        n = int(rng.integers(2, 6))
        lb = rng.integers(0, 3, size=n).astype(np.float64)
        ub = lb + rng.integers(1, 5, size=n)
        a = (rng.integers(1, 6, size=n) * np.where(rng.integers(0, 2, size=n) == 0, -1, 1)).astype(np.float64)
        x = np.array([rng.integers(int(lb[i]), int(ub[i]) + 1) for i in range(n)], dtype=np.float64)
        s = float(np.dot(a, x))
        gap = float(rng.integers(1, 7))
        if rng.integers(0, 2) == 0:
            lo, hi = -math.inf, s - gap
        else:
            lo, hi = s + gap, math.inf
        inst = gen.from_rows(n, [(list(range(n)), a)], [lo], [hi], [1] * n, lb, ub)
        return inst, x


def brute_single_row_repair(inst, x):
    """What one shift must do on a single violated row, by enumeration with
    exact integers: for each variable, the move towards feasibility by the
    fewest units that makes the row hold, or the farthest one the original
    domain allows; its score is the exact change of the row's violation.
    Returns (index, new value) of the lowest negative score (smallest index
    on ties) or None."""
    a = [int(v) for v in inst["val"]]
    lo, hi = inst["lo"][0], inst["hi"][0]
    X = [int(v) for v in x]
    s = sum(ai * xi for ai, xi in zip(a, X))

    def viol(t):
        if not math.isinf(hi) and t > hi:
            return t - int(hi)
        if not math.isinf(lo) and t < lo:
            return int(lo) - t
        return 0

    e = viol(s)
    best = None
    for j, aj in enumerate(a):
        # the direction that lowers the violation
        want_down = (not math.isinf(hi) and s > hi)
        step = -1 if (aj > 0) == want_down else 1
        v = X[j]
        lim = int(inst["lb"][j]) if step < 0 else int(inst["ub"][j])
        moves = []
        w = v + step
        while (w >= lim) if step < 0 else (w <= lim):
            moves.append(w)
            if viol(s + aj * (w - v)) == 0:
                break
            w += step
        if not moves:
            continue
        w = moves[-1]
        score = viol(s + aj * (w - v)) - e
        if score < 0 and (best is None or score < best[0]):
            best = (score, j, w)
    return None if best is None else (best[1], float(best[2]))
