"""Probe-priority and implied-slack scores on the GPU (bp_scores,
bp_probe_order) against the CPU oracle on the same seeded inputs: violation
counts and the probe order bit-exact; the floating-point scores bit-exact
too, since each is a fixed sequence of IEEE operations on correctly rounded
activities (no fused multiply-add on either side)."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import bp, dev
from helpers import load_golden, slack_edge_instance
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu

FIELDS = ("nviol", "maxviol", "minunit", "slack_score")


def _gpu_scores(I, lb, ub):
    out = I.scores(dev(lb, torch.float64), dev(ub, torch.float64))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(g, o, what):
    for f in FIELDS:
        a, b = g[f], o[f]
        assert a.shape == b.shape, (what, f)
        if f == "nviol":
            assert np.array_equal(a, b), (what, f, np.nonzero(a != b)[0][:5])
        else:
            # bitwise (views as integers: +inf, +0.0 and values alike)
            ai, bi = a.view(np.int64), b.view(np.int64)
            bad = np.nonzero(ai != bi)[0]
            assert bad.size == 0, (what, f, bad[:5], a[bad[:5]], b[bad[:5]])


def _check(inst, lb=None, ub=None, what=""):
    lb = inst["lb"] if lb is None else lb
    ub = inst["ub"] if ub is None else ub
    I = bp().Instance(inst)
    _same(_gpu_scores(I, lb, ub), oracle.scores(inst, lb, ub), what)
    return I


def test_golden_w5():
    inst, d = load_golden("w5_scores")
    I = bp().Instance(inst)
    g = _gpu_scores(I, inst["lb"], inst["ub"])
    assert list(g["nviol"]) == d["nviol"]
    assert list(g["maxviol"]) == [float(x) for x in d["maxviol"]]
    assert list(g["minunit"]) == [float(x) for x in d["minunit"]]
    assert list(g["slack_score"]) == [float(x) for x in d["slack_score"]]
    tl, tu = dev(inst["lb"], torch.float64), dev(inst["ub"], torch.float64)
    for vs, exp in d["orders"]:
        order = I.probe_order(dev(np.asarray(vs, np.int32), torch.int32), tl, tu)
        assert order.cpu().tolist() == exp


@pytest.mark.parametrize("name,seed", [("tiny", 0), ("tiny", 1), ("tiny_inf", 2), ("tiny_inf", 5)])
def test_small_instances(name, seed):
    inst = gen.make(name, seed)
    _check(inst, what="%s/%d original" % (name, seed))
    r, lb, ub = oracle.propagate(inst)
    assert r["status"] == oracle.BP_OK
    _check(inst, lb, ub, what="%s/%d base" % (name, seed))


@pytest.mark.parametrize("seed", range(0, 40, 3))
def test_micro_instances(seed):
    inst = gen.make_micro(seed)
    _check(inst, what="micro %d" % seed)


@pytest.mark.parametrize("scale,longest", [(0.02, 512), (0.06, 1024)])
def test_single_workload_scaled(scale, longest):
    """Ragged bins; at the larger scale rows of several thousand nonzeros
    (chunked)."""
    inst = gen.make("single", 4, scale=scale)
    assert np.diff(inst["row_ptr"]).max() > longest
    _check(inst, what="single %.2f" % scale)


def test_single_workload_full_size():
    """The full single-instance workload (rows up to ~47k nonzeros, split in
    chunks of 4096), at its original bounds and at its propagated base."""
    inst = gen.make("single", 0)
    I = _check(inst, what="single full")
    r, lb, ub = oracle.propagate(inst)
    _same(_gpu_scores(I, lb, ub), oracle.scores(inst, lb, ub), "single full base")


def test_probe_workload_scaled():
    inst = gen.make("probe", 2, scale=0.01)
    _check(inst, what="probe 0.01")


@pytest.mark.parametrize("seed", [0, 1])
def test_slack_edges(seed):
    """Slacks placed at a few ulps of the filter threshold, mixed types."""
    inst = slack_edge_instance(seed, count=200)[0]
    _check(inst, what="edge %d" % seed)


def test_cancellation_uses_exact_activities():
    """Rows whose terms cancel beyond double-double (1e32, 1e16, 1, ...):
    the certified sum fails and the exact accumulator decides."""
    n = 6
    rows = [([0, 1, 2, 3, 4], [1e32, 1e16, 1.0, -1e32, -1e16]),
            ([0, 3, 5], [1e32, -1e32, 3.0]),
            ([1, 4, 5], [1e16, -1e16, -1.0])]
    inst = gen.from_rows(n, rows, [-math.inf, -5.0, -math.inf], [4.0, math.inf, 2.0],
                         [0] * n, [1.0, 1.0, 1.0, 1.0, 1.0, 0.0], [1.0, 1.0, 1.0, 1.0, 1.0, 2.0])
    _check(inst, what="cancel")


def test_empty_columns_and_free_rows():
    """A variable in no row, a row with no finite side, an empty row."""
    rows = [([0, 1], [1.0, -2.0]), ([1, 2], [3.0, 1.0]), ([], [])]
    inst = gen.from_rows(4, rows, [-math.inf, -math.inf, 0.0], [math.inf, 4.0, 1.0],
                         [1, 1, 0, 0], [0.0, 0.0, 0.0, -1.0], [3.0, 2.0, 5.0, 1.0])
    _check(inst, what="empty")


@pytest.mark.parametrize("k", [1, 2, 1000, 4097])
def test_probe_order_matches_oracle(k):
    inst = gen.make("single", 1, scale=0.05)
    rng = np.random.default_rng(k)
    vs = rng.integers(0, inst["n"], size=k).astype(np.int32)  # repeats allowed
    I = bp().Instance(inst)
    tl, tu = dev(inst["lb"], torch.float64), dev(inst["ub"], torch.float64)
    order = I.probe_order(dev(vs, torch.int32), tl, tu).cpu().numpy()
    assert np.array_equal(order, oracle.probe_order(inst, vs))


def test_probe_order_of_every_integer_of_the_single_workload():
    inst = gen.make("single", 0)
    r, lb, ub = oracle.propagate(inst)
    vs = np.nonzero(inst["vtype"] == 1)[0].astype(np.int32)
    I = bp().Instance(inst)
    order = I.probe_order(dev(vs, torch.int32), dev(inst["lb"], torch.float64),
                          dev(inst["ub"], torch.float64)).cpu().numpy()
    assert np.array_equal(order, oracle.probe_order(inst, vs))


def test_errors_and_state():
    """Out-of-range ids and NaN bounds are rejected; an empty list is fine;
    scoring leaves propagation results unchanged."""
    inst = gen.make("tiny", 3)
    I = bp().Instance(inst)
    tl, tu = dev(inst["lb"], torch.float64), dev(inst["ub"], torch.float64)
    with pytest.raises(bp().BPError):
        I.probe_order(dev(np.array([0, inst["n"]], np.int32), torch.int32), tl, tu)
    assert I.probe_order(torch.zeros(0, dtype=torch.int32, device="cuda"), tl, tu).numel() == 0
    bad = inst["lb"].copy()
    bad[4] = np.nan
    with pytest.raises(bp().BPError):
        I.scores(dev(bad, torch.float64), tu)
    lb, ub = dev(inst["lb"], torch.float64), dev(inst["ub"], torch.float64)
    r = I.propagate(lb, ub)
    ro, lo, uo = oracle.propagate(inst)
    assert r["status"] == ro["status"] and r["rounds"] == ro["rounds"]
    _same(_gpu_scores(I, inst["lb"], inst["ub"]), oracle.scores(inst), "after propagate")
