"""Planted mistakes in the CPU oracle must be caught by its pins.

Each mutant is a one-line textual change of ``oracle/bp_oracle.c`` (a
dropped term, a wrong sign or index, a swapped operand), compiled on the CPU
into a temporary library.  The pins (worked examples, brute force, exact
Gauss-Seidel, closed forms, planted-point invariants) are run against it
and at least one must fail.
"""
import math
import os
from fractions import Fraction
import tempfile

import numpy as np
import pytest

import oracle
from helpers import (_f, brute_scores, brute_single_row_repair, case_mismatch, exact_gs_fixed_point,
                     feasible_points, implied_dict, load_golden, load_golden_cases, repair_case_mismatch,
                     repair_cases, repair_round_scenario, round_scenarios, row_violations,
                     single_row_repair_instance)
from paper_2510_20499_amd import gen

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "bp_oracle.c")

MUTANTS = {
    "own_term_sign": ("v = r + t;", "v = r - t;"),
    "own_term_dropped": ("v = r + t;", "v = r;"),
    "activity_bounds_swapped": ("double bmin = a > 0.0 ? lb[i] : ub[i];",
                                "double bmin = a > 0.0 ? ub[i] : lb[i];"),
    "no_integer_floor": ("if (is_int) c = floor(c + o->inttol);", "if (is_int) c = floor(c);"),
    "inttol_sign": ("if (is_int) c = ceil(c - o->inttol);", "if (is_int) c = ceil(c + o->inttol);"),
    "threshold_sign": ("return cand < old - o->tau * fmax(1.0, fabs(old));",
                       "return cand < old + o->tau * fmax(1.0, fabs(old));"),
    "inf_count_rule": ("} else if (own_inf && act->ninf_min == 1) {",
                       "} else if (own_inf && act->ninf_min == 0) {"),
    "row_test_tolerance": ("if (act->ninf_min == 0 && act->minfin > I->hi[k] + o->feastol) return 1;",
                           "if (act->ninf_min == 0 && act->minfin > I->hi[k] + 1.0) return 1;"),
    "worklist_skips_first_row": (
        "for (int64_t p = w.col_ptr[i]; p < w.col_ptr[i + 1]; ++p) add_row(I, &w, w.col_row[p], &nrows);\n        }\n    }",
        "for (int64_t p = w.col_ptr[i] + 1; p < w.col_ptr[i + 1]; ++p) add_row(I, &w, w.col_row[p], &nrows);\n        }\n    }"),
    "division_operand": ("double c = v / a;", "double c = v / fabs(a);"),
    "probe_split_rounded_down": ("double c = ceil((l + u) / 2.0);", "double c = floor((l + u) / 2.0);"),
    "probe_one_sided_step": ("else { *nl = l + 1.0; *nu = u; }", "else { *nl = l; *nu = u; }"),
    "flip_direction": ("const double d = a * b_max - a * b_min;",
                       "const double d = a * b_min - a * b_max;"),
    "flip_without_mixed_signs": ("if (sign[j] == 3 && !isinf(lb[j])", "if (sign[j] != 0 && !isinf(lb[j])"),
    "slack_from_max_activity": ("const double slack_hi = hi_ok ? I->hi[k] - A->minfin : 0.0;",
                                "const double slack_hi = hi_ok ? I->hi[k] - A->maxfin : 0.0;"),
    "unit_slack_inverted": ("double u = slack_lo / fabs(a);", "double u = fabs(a) / slack_lo;"),
    "square_dropped": ("double t = s * s;", "double t = fabs(s);"),
    "bulk_last_singles": ("int64_t bulk = (recovery || R <= 36) ? 1", "int64_t bulk = (recovery || R <= 35) ? 1"),
    "bulk_size_floor": ("(int64_t)ceil(sqrt((double)R))", "(int64_t)floor(sqrt((double)R))"),
    "random_rounding_band": ("if (f > 0.25 && f < 0.75) v = u < f", "if (f > 0.35 && f < 0.75) v = u < f"),
    "random_rounding_direction": ("v = u < f ? fl + 1.0 : fl;", "v = u < f ? fl : fl + 1.0;"),
    "implied_slack_ascending": ("if (a->key != b->key) return a->key > b->key ? -1 : 1;",
                                "if (a->key != b->key) return a->key < b->key ? -1 : 1;"),
    "no_recovery_mode": ("if (!recovery && !infeasible) {", "if (0) {"),
    "cache_conflicts_kept": ("if (keep[t] && !(box_l[j] <= val[h][t] && val[h][t] <= box_u[j])) keep[t] = 0;",
                             "(void)j;"),
    # crossing rule, infeasibility evidence and signed zeros (fixture w7)
    "snap_deleted": ("} else {\n                    nl = nu;\n                }", "} else {\n                }"),
    "snap_reversed": ("} else {\n                    nl = nu;\n                }",
                      "} else {\n                    nu = nl;\n                }"),
    "crossing_without_feastol": ("if (is_int || nl - nu > o->feastol) {", "if (is_int || nl - nu > 0.0) {"),
    "integer_crossing_snapped": ("if (is_int || nl - nu > o->feastol) {", "if (nl - nu > o->feastol) {"),
    "largest_bad_row_worklist": (
        "if (row_infeasible(I, k, &act, o)) {\n                    n_bad += 1;\n                    if (bad_row < 0 || k < bad_row) bad_row = k;",
        "if (row_infeasible(I, k, &act, o)) {\n                    n_bad += 1;\n                    if (bad_row < 0 || k > bad_row) bad_row = k;"),
    "largest_bad_row_definition": (
        "if (row_infeasible(I, k, &acts[k], o)) {\n                    n_bad += 1;\n                    if (bad_row < 0 || k < bad_row) bad_row = k;",
        "if (row_infeasible(I, k, &acts[k], o)) {\n                    n_bad += 1;\n                    if (bad_row < 0 || k > bad_row) bad_row = k;"),
    "largest_crossed_var": ("if (bad_var < 0 || i < bad_var) bad_var = i;", "if (bad_var < 0 || i > bad_var) bad_var = i;"),
    "infeasible_row_count_one": ("res->n_infeasible_rows = (int32_t)n_bad;", "res->n_infeasible_rows = 1;"),
    "no_canonical_zero": ("static double canon(double x) { return x == 0.0 ? 0.0 : x; }",
                          "static double canon(double x) { return x; }"),
    "row_precedence_dropped": ("if (n_bad) {\n            /* Step 3: the round ends with the row evidence. */",
                               "if (0) {\n            /* Step 3: the round ends with the row evidence. */"),
    "order_violation_direction": ("if (a->maxviol != b->maxviol) return a->maxviol > b->maxviol ? -1 : 1;",
                                  "if (a->maxviol != b->maxviol) return a->maxviol < b->maxviol ? -1 : 1;"),
    # repair procedure (fixture w8_repair, single-row brute force, micro invariants)
    "repair_first_violated_row": ("if (e > eb) { eb = e; kb = k; }", "if (e > 0.0 && kb < 0) { eb = e; kb = k; }"),
    "repair_shift_sign": ("double r = hi_side ? (-e) / a : e / a;", "double r = hi_side ? e / a : e / a;"),
    "repair_no_unit_minimum": ("if (mag < 1.0) mag = 1.0;", "(void)0;"),
    "repair_inttol_sign": ("double mag = ceil(fabs(r) - o->inttol);", "double mag = ceil(fabs(r) + o->inttol);"),
    "repair_no_upper_limit": ("if (d > 0.0 && !isinf(u0) && d > u0 - v) d = u0 - v;", "(void)u0;"),
    "repair_no_lower_limit": ("if (d < 0.0 && !isinf(l0) && d < l0 - v) d = l0 - v;", "(void)l0;"),
    "repair_ties_to_larger_index": ("if (jb < 0 || score < sb) { jb = j; sb = score; vbest = nv; }",
                                    "if (jb < 0 || score <= sb) { jb = j; sb = score; vbest = nv; }"),
    "repair_zero_score_accepted": ("if (jb < 0 || !(sb < 0.0)) { res->reason = 1; goto done; }",
                                   "if (jb < 0 || !(sb <= 0.0)) { res->reason = 1; goto done; }"),
    "repair_score_ignores_other_rows": ("diffs[nd++] = e1 - e0;", "if (r == kb) diffs[nd++] = e1 - e0;"),
    "repair_shifts_unfixed": ("if (!fixed[j] || !repair_shift(", "if (!I->vtype[j] || !repair_shift("),
    "repair_restart_from_the_box": ("if (pr.rounds > 1) {\n            /* the same propagation stopped",
                                    "if (0) {\n            /* the same propagation stopped"),
    "repair_restart_after_d_rounds": ("o2.max_rounds = pr.rounds - 1;", "o2.max_rounds = pr.rounds;"),
    "repair_attempt_limit_late": ("if (res->attempts >= max_attempts) { res->reason = 3; goto done; }",
                                  "if (res->attempts > max_attempts) { res->reason = 3; goto done; }"),
    "round_repair_never_called": ("if (infeasible && rp && res->repairs < rp->calls) {",
                                  "if (0 && infeasible && rp && res->repairs < rp->calls) {"),
    "round_repair_keeps_mark": ("res->repaired += 1;\n                infeasible = 0;",
                                "res->repaired += 1;"),
    "round_repair_from_current_box": ("orc_repair(I, lb, ub, start_l, start_u,", "orc_repair(I, lb, ub, lb, ub,"),
}


def _pins_hold(lib) -> bool:
    try:
        for mode in (oracle.MODE_WORKLIST, oracle.MODE_DEFINITION):
            for inst, c in load_golden_cases("w7"):
                r, lb, ub = oracle.propagate(inst, mode=mode, lib=lib)
                if case_mismatch(c, r, lb, ub) is not None:
                    return False
        for name in ("w1", "w2", "w3", "w4"):
            inst, d = load_golden(name)
            r, lb, ub = oracle.propagate(inst, lib=lib)
            c = d["cold"]
            if (r["status"], r["rounds"], r["nnz_propagated"]) != (c["status"], c["rounds"], c["nnz_propagated"]):
                return False
            if list(lb) != [float(x) for x in c["lb"]] or list(ub) != [float(x) for x in c["ub"]]:
                return False
            P = oracle.probe(inst, lb, ub, d["probe_vars"], lib=lib)
            for p, exp in enumerate(d["probes"]):
                if (P["status"][p], P["rounds"][p], P["nnz"][p]) != (exp["status"], exp["rounds"], exp["nnz"]):
                    return False
                if "n_infeasible_rows" in exp and P["n_infeasible_rows"][p] != exp["n_infeasible_rows"]:
                    return False
                want = {int(v): (float(a), float(b)) for v, a, b in exp["implied"]}
                if implied_dict(P, p) != want:
                    return False
        for seed in range(120):
            inst = gen.make_micro(seed)
            F = feasible_points(inst)
            r, lb, ub = oracle.propagate(inst, lib=lib)
            if r["status"] == oracle.BP_INFEASIBLE:
                if F:
                    return False
                continue
            for x in F:
                if not all(lb[i] <= x[i] <= ub[i] for i in range(inst["n"])):
                    return False
            ok, glb, gub = exact_gs_fixed_point(inst)
            if not ok or [float(x) for x in glb] != list(lb) or [float(x) for x in gub] != list(ub):
                return False
        for seed in range(5):
            inst = gen.make("tiny", seed)
            r, lb, ub = oracle.propagate(inst, lib=lib)
            x = inst["xstar"]
            if r["status"] != oracle.BP_OK or not ((lb <= x + 1e-6).all() and (x <= ub + 1e-6).all()):
                return False
        inst = gen.make("tiny_inf", 0)
        r, lb, ub = oracle.propagate(inst, lib=lib)
        x = inst["xstar"]
        if r["status"] != oracle.BP_OK or not ((lb <= x + 1e-6).all() and (x <= ub + 1e-6).all()):
            return False
        n = 6
        a = [1.5, 2.0, 3.0, 0.7, 5.0, 9.0]
        g = 10.0
        inst = gen.from_rows(n, [(list(range(n)), a)], [-math.inf], [g], [1] * n, [0.0] * n, [30.0] * n)
        r, lb, ub = oracle.propagate(inst, lib=lib)
        if list(ub) != [min(30.0, math.floor(g / a[j] + 1e-6)) for j in range(n)]:
            return False
        # 0.3 / 0.1 evaluates to 2.9999999999999996: the integer tolerance
        # gives x <= 3, and symmetrically x >= 3 from 0.1 x >= 0.3.
        inst = gen.from_rows(1, [([0], [0.1])], [-math.inf], [0.3], [1], [0.0], [10.0])
        if list(oracle.propagate(inst, lib=lib)[2]) != [3.0]:
            return False
        inst = gen.from_rows(1, [([0], [0.1])], [0.3], [math.inf], [1], [0.0], [10.0])
        if list(oracle.propagate(inst, lib=lib)[1]) != [3.0]:
            return False
        # priority scores: the hand-computed fixture and their exact meaning
        inst, d = load_golden("w5_scores")
        S = oracle.scores(inst, lib=lib)
        if (list(S["nviol"]) != d["nviol"] or list(S["maxviol"]) != [float(x) for x in d["maxviol"]]
                or list(S["minunit"]) != [float(x) for x in d["minunit"]]
                or list(S["slack_score"]) != [float(x) for x in d["slack_score"]]):
            return False
        for vs, exp in d["orders"]:
            if list(oracle.probe_order(inst, vs, lib=lib)) != exp:
                return False
        for seed in range(40):
            inst = gen.make_micro(seed)
            S = oracle.scores(inst, lib=lib)
            nviol, maxviol, units, terms = brute_scores(inst, inst["lb"], inst["ub"])
            if list(S["nviol"]) != nviol or [Fraction(x) for x in S["maxviol"]] != maxviol:
                return False
            for j in range(inst["n"]):
                if S["minunit"][j] != (float(min(units[j])) if units[j] else math.inf):
                    return False
                exact = None if any(t is None for t in terms[j]) else sum(terms[j], Fraction(0))
                if (exact is None) != (S["slack_score"][j] == math.inf):
                    return False
                if exact is not None and abs(Fraction(S["slack_score"][j]) - exact) > exact / 2 ** 49:
                    return False
        # rounding driver: the hand-traced scenarios, the planted point
        for _, inst, s in round_scenarios():
            r, lb, ub = oracle.round_(inst, s["x"], s["draws"], lib=lib)
            if r != s["expect"] or list(lb) != [float(v) for v in s["final"]]:
                return False
            if "cache" in s:
                r, lb, ub = oracle.round_(inst, s["x"], s["draws"], cache=s["cache"], lib=lib)
                if r != s["expect_cache"]:
                    return False
        for seed in range(3):
            inst = gen.make("tiny", seed)
            r0, lb, ub = oracle.propagate(inst, lib=lib)
            xs = inst["xstar"]
            ints = inst["vtype"] == 1
            d = np.random.default_rng(seed).random(2 * inst["n"])
            r, l2, u2 = oracle.round_(inst, xs, d, lb, ub, lib=lib)
            if r["status"] != oracle.BP_OK or not np.array_equal(l2[ints], xs[ints]):
                return False
        # repair: the hand-traced cases and rounding, single-row brute force,
        # micro invariants
        for inst, c in repair_cases():
            r, lb, ub = oracle.repair(inst, [_f(x) for x in c["box_lb"]], [_f(x) for x in c["box_ub"]],
                                      max_shifts=c["max_shifts"], max_attempts=c["max_attempts"], lib=lib)
            if repair_case_mismatch(c, r, lb, ub) is not None:
                return False
        inst, s = repair_round_scenario()
        r0, lb, ub = oracle.propagate(inst, lib=lib)
        r, l2, u2 = oracle.round_(inst, s["x"], s["draws"], lb, ub, repair=s["repair_limits"], lib=lib)
        if r != s["expect"] or list(l2) != s["final_lb"] or list(u2) != s["final_ub"]:
            return False
        for seed in range(200):
            inst, x = single_row_repair_instance(seed)
            r, lb, ub = oracle.repair(inst, x, x, max_shifts=1, max_attempts=1, lib=lib)
            want = brute_single_row_repair(inst, x)
            if want is None:
                if r["status"] != oracle.BP_INFEASIBLE or r["reason"] != 1:
                    return False
                continue
            y = x.copy()
            y[want[0]] = want[1]
            if not row_violations(inst, y):
                if r["status"] != oracle.BP_OK or list(lb) != list(y):
                    return False
            elif r["status"] != oracle.BP_INFEASIBLE or r["reason"] != 2:
                return False
        for seed in range(120):
            inst = gen.make_micro(seed)
            n = inst["n"]
            rng = np.random.default_rng(seed)
            x = np.array([rng.integers(int(inst["lb"][i]), int(inst["ub"][i]) + 1) for i in range(n)],
                         dtype=np.float64)
            r, lb, ub = oracle.repair(inst, x, x, lib=lib)
            if r["status"] == oracle.BP_OK:
                if row_violations(inst, lb) or (not row_violations(inst, x) and r["shifts"] != 0):
                    return False
            elif not np.array_equal(lb, x):
                return False
    except (ValueError, ZeroDivisionError, OverflowError):
        return False
    return True


def test_unmutated_oracle_passes_pins():
    assert _pins_hold(oracle.load())


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_mutant_is_caught(mutant):
    src = open(SRC).read()
    old, new = MUTANTS[mutant]
    assert src.count(old) >= 1, mutant
    mutated = src.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as d:
        cpath = os.path.join(d, "mut.c")
        with open(cpath, "w") as fh:
            fh.write(mutated)
        lib = oracle.bind(oracle.compile_to(cpath, os.path.join(d, "libmut.so")))
        assert not _pins_hold(lib), "pins did not catch mutant %s" % mutant
