"""Bound-propagation rounding on the GPU (bp_round) against the CPU oracle on
the same seeded inputs (box, fractional point, draws, probing cache computed
by the oracle): every counter, the status and the final box bit-identical."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import bp, dev
from helpers import round_scenarios
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu


def _cache_dev(P):
    return {"vars": dev(np.asarray(P["vars"], np.int32), torch.int32),
            "status": dev(np.asarray(P["status"], np.int8), torch.int8),
            "off": dev(np.asarray(P["off"], np.int64), torch.int64),
            "var": dev(np.asarray(P["var"], np.int32), torch.int32),
            "lb": dev(np.asarray(P["lb"], np.float64), torch.float64),
            "ub": dev(np.asarray(P["ub"], np.float64), torch.float64)}


def _gpu_round(I, lb, ub, x, draws, cache=None):
    tl, tu = dev(lb, torch.float64), dev(ub, torch.float64)
    r = I.round(tl, tu, dev(x, torch.float64), dev(draws, torch.float64),
                None if cache is None else _cache_dev(cache))
    torch.cuda.synchronize()
    return r, tl.cpu().numpy(), tu.cpu().numpy()


def _same(inst, lb, ub, x, draws, cache=None, what=""):
    I = bp().Instance(inst)
    rg, lg, ug = _gpu_round(I, lb, ub, x, draws, cache)
    ro, lo, uo = oracle.round_(inst, x, draws, lb, ub, cache=cache)
    assert rg == ro, (what, rg, ro)
    assert np.array_equal(lg.view(np.int64), lo.view(np.int64)), (what, np.nonzero(lg != lo)[0][:5])
    assert np.array_equal(ug.view(np.int64), uo.view(np.int64)), (what, np.nonzero(ug != uo)[0][:5])
    return rg


@pytest.mark.parametrize("key", ["A", "B", "C", "D"])
def test_golden_w6_round(key):
    sc = {k: (inst, s) for k, inst, s in round_scenarios()}
    inst, s = sc[key]
    I = bp().Instance(inst)
    x, d = np.asarray(s["x"], float), np.asarray(s["draws"], float)
    r, lb, ub = _gpu_round(I, inst["lb"], inst["ub"], x, d)
    assert r == s["expect"]
    assert list(lb) == [float(v) for v in s["final"]] and list(ub) == list(lb)
    if "cache" in s:
        r, lb, ub = _gpu_round(I, inst["lb"], inst["ub"], x, d, s["cache"])
        assert r == s["expect_cache"]
        assert list(lb) == [float(v) for v in s["final"]]


def _point(inst, lb, ub, seed, noise=0.4):
    rng = np.random.default_rng(seed)
    x = np.clip(inst["xstar"] + rng.normal(0.0, noise, inst["n"]), lb, ub)
    return x, rng.random(2 * inst["n"])


@pytest.mark.parametrize("name,seed", [("tiny", 0), ("tiny", 1), ("tiny", 4), ("tiny_inf", 2)])
def test_tiny_instances(name, seed):
    inst = gen.make(name, seed)
    r0, lb, ub = oracle.propagate(inst)
    x, d = _point(inst, lb, ub, seed)
    _same(inst, lb, ub, x, d, what="%s/%d" % (name, seed))
    cand = np.nonzero((inst["vtype"] == 1) & (lb == 0) & (ub == 1))[0][:60].astype(np.int32)
    P = oracle.probe(inst, lb, ub, cand)
    P["vars"] = cand
    _same(inst, lb, ub, x, d, cache=P, what="%s/%d cache" % (name, seed))


def _micro_feasible_seeds(count=30):
    """The first `count` micro seeds whose root (oracle) is not infeasible:
    rounding starts from a root box."""
    out = []
    seed = 0
    while len(out) < count:
        if oracle.propagate(gen.make_micro(seed))[0]["status"] != oracle.BP_INFEASIBLE:
            out.append(seed)
        seed += 1
    return out


@pytest.mark.parametrize("seed", _micro_feasible_seeds())
def test_micro_instances(seed):
    inst = gen.make_micro(seed)
    r0, lb, ub = oracle.propagate(inst)
    assert r0["status"] != oracle.BP_INFEASIBLE
    rng = np.random.default_rng(seed)
    x = lb + rng.random(inst["n"]) * (ub - lb)
    _same(inst, lb, ub, x, rng.random(2 * inst["n"]), what="micro %d" % seed)


@pytest.mark.parametrize("seed", [3, 5])
def test_single_workload_scaled(seed):
    """Bulks of ceil(sqrt R) up to ~50 variables on 3000 variables with
    heavy rows; a cache of 200 binaries."""
    inst = gen.make("single", seed, scale=0.02)
    r0, lb, ub = oracle.propagate(inst)
    x, d = _point(inst, lb, ub, seed)
    r = _same(inst, lb, ub, x, d, what="single %d" % seed)
    assert r["bulks"] > 0
    cand = np.nonzero((inst["vtype"] == 1) & (lb == 0) & (ub == 1))[0][:200].astype(np.int32)
    P = oracle.probe(inst, lb, ub, cand)
    P["vars"] = cand
    _same(inst, lb, ub, x, d, cache=P, what="single %d cache" % seed)


def test_planted_point_on_the_gpu():
    inst = gen.make("single", 2, scale=0.02)
    r0, lb, ub = oracle.propagate(inst)
    xs = inst["xstar"]
    d = np.random.default_rng(1).random(2 * inst["n"])
    I = bp().Instance(inst)
    r, l2, u2 = _gpu_round(I, lb, ub, xs, d)
    ints = inst["vtype"] == 1
    assert r["status"] == bp().BP_OK and r["recoveries"] == 0
    assert np.array_equal(l2[ints], xs[ints]) and np.array_equal(u2[ints], xs[ints])


def test_edge_cases_and_errors():
    # no integer variable left to fix
    inst = gen.from_rows(2, [([0, 1], [1.0, 1.0])], [-math.inf], [3.0], [0, 1], [0.0, 2.0], [5.0, 2.0])
    I = bp().Instance(inst)
    r, lb, ub = _gpu_round(I, inst["lb"], inst["ub"], np.array([1.0, 2.0]), np.zeros(4))
    assert r["iterations"] == 0 and r["status"] == bp().BP_OK and r["fixed"] == 1
    inst = gen.make("tiny", 5)
    I = bp().Instance(inst)
    n = inst["n"]
    x = np.clip(inst["xstar"], inst["lb"], inst["ub"])
    d = np.full(2 * n, 0.5)
    bad_x = x.copy()
    bad_x[3] = np.nan
    with pytest.raises(bp().BPError):
        _gpu_round(I, inst["lb"], inst["ub"], bad_x, d)
    bad_d = d.copy()
    bad_d[7] = 1.0
    with pytest.raises(bp().BPError):
        _gpu_round(I, inst["lb"], inst["ub"], x, bad_d)
    P = {"vars": np.array([n], np.int32), "status": np.zeros(2, np.int8), "off": np.zeros(3, np.int64),
         "var": np.zeros(0, np.int32), "lb": np.zeros(0), "ub": np.zeros(0)}
    with pytest.raises(bp().BPError):
        _gpu_round(I, inst["lb"], inst["ub"], x, d, P)
    # the instance still propagates as before after a rounding call
    tl, tu = dev(inst["lb"], torch.float64), dev(inst["ub"], torch.float64)
    rg = I.propagate(tl, tu)
    ro, lo, uo = oracle.propagate(inst)
    assert (rg["status"], rg["rounds"], rg["nnz_propagated"]) == (ro["status"], ro["rounds"], ro["nnz_propagated"])


def test_round_limit_counts_as_not_infeasible():
    """With two rounds per propagation many bulks stop at the round limit;
    such a bulk is accepted like a feasible one, on both sides."""
    inst = gen.make("single", 6, scale=0.02)
    r0, lb, ub = oracle.propagate(inst)
    x, d = _point(inst, lb, ub, 6)
    I = bp().Instance(inst, bp().default_options(max_rounds=2))
    rg, lg, ug = _gpu_round(I, lb, ub, x, d)
    oo = oracle.Options()
    oo.max_rounds = 2
    ro, lo, uo = oracle.round_(inst, x, d, lb, ub, opts=oo)
    assert rg == ro
    assert np.array_equal(lg.view(np.int64), lo.view(np.int64))
    assert np.array_equal(ug.view(np.int64), uo.view(np.int64))
