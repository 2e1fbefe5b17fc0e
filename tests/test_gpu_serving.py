"""Serving (continuous batching over several resident instances): every
request's results match the CPU oracle, and are the same when the request
is served alone and in the mix."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, bp, dev, gpu_base, gpu_propagate
from helpers import rel_close
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu


def _instances():
    insts = [gen.make("tiny", 0), gen.make("tiny_inf", 1), gen.make("single", 2, scale=0.02),
             gen.make("probe", 0, scale=0.003), gen.make("single", 3, scale=0.05)]
    loaded, bases = [], []
    for inst in insts:
        I = bp().Instance(inst, bp().default_options(heavy_threshold=2048))
        r, lb, ub = gpu_propagate(I, inst)
        ro, olb, oub = oracle.propagate(inst)
        assert ro["status"] == oracle.BP_OK
        assert_same(inst, r, lb, ub, ro, olb, oub, "serving root")
        gpu_base(I, olb, oub)  # both sides serve from the oracle's root
        loaded.append(I)
        bases.append((olb, oub))
    return insts, loaded, bases


def _requests(insts, bases, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        t = int(rng.integers(0, len(insts)))
        inst = insts[t]
        lb, ub = bases[t]
        bins = np.nonzero((inst["vtype"] == 1) & (lb == 0) & (ub == 1))[0]
        if rng.uniform() < 0.5 and bins.size:
            k = int(min(bins.size, np.exp(rng.uniform(0, np.log(64)))))
            vs = np.sort(rng.choice(bins, size=max(k, 1), replace=False)).astype(np.int32)
            reqs.append((t, bp().REQ_PROBE, vs, None, None))
        else:
            ints = np.nonzero((inst["vtype"] == 1) & (lb < ub))[0]
            k = max(1, int(0.01 * max(bins.size, 1)))
            k = min(k, ints.size)
            vs = np.sort(rng.choice(ints, size=k, replace=False)).astype(np.int32)
            val = np.rint(rng.uniform(lb[vs], ub[vs]))
            reqs.append((t, bp().REQ_PROPAGATE, vs, val, val))
    return reqs


def _oracle_result(inst, base, req):
    t, kind, vs, lo, hi = req
    lb, ub = base
    if kind == bp().REQ_PROBE:
        return oracle.probe(inst, lb, ub, vs)
    nlb, nub = lb.copy(), ub.copy()
    nlb[vs] = np.maximum(lb[vs], lo)
    nub[vs] = np.minimum(ub[vs], hi)
    changed = vs[(nlb[vs] != lb[vs]) | (nub[vs] != ub[vs])]
    r, flb, fub = oracle.propagate(inst, nlb, nub, changed=changed)
    diff = np.nonzero((flb != lb) | (fub != ub))[0]
    if r["status"] == oracle.BP_INFEASIBLE:
        diff = diff[:0]
    return dict(status=np.array([r["status"]]), rounds=np.array([r["rounds"]]),
                nnz=np.array([r["nnz_propagated"]]),
                n_infeasible_rows=np.array([r["n_infeasible_rows"]]),
                infeasible_row=np.array([r["infeasible_row"]]),
                infeasible_var=np.array([r["infeasible_var"]]),
                off=np.array([0, diff.size]), var=diff.astype(np.int32), lb=flb[diff], ub=fub[diff])


def _same(a, b, inst, what, evidence=False):
    for f in ("status", "rounds", "nnz", "off", "var"):
        assert np.array_equal(np.asarray(a[f]), np.asarray(b[f])), (what, f, a[f], b[f])
    if evidence:
        for f in ("n_infeasible_rows", "infeasible_row", "infeasible_var"):
            assert np.array_equal(np.asarray(a[f]), np.asarray(b[f])), (what, f, a[f], b[f])
    integ = inst["vtype"][np.asarray(a["var"], dtype=np.int64)] == 1 if len(a["var"]) else np.zeros(0, bool)
    assert np.array_equal(np.asarray(a["lb"])[integ], np.asarray(b["lb"])[integ]), what
    assert np.array_equal(np.asarray(a["ub"])[integ], np.asarray(b["ub"])[integ]), what
    assert rel_close(np.asarray(a["lb"])[~integ], np.asarray(b["lb"])[~integ]), what
    assert rel_close(np.asarray(a["ub"])[~integ], np.asarray(b["ub"])[~integ]), what


def _serve(loaded, reqs, budget, rounds_per_step=8, waves=1, opts=None):
    S = bp().Server(loaded, budget, opts)
    ids = []
    # submit in `waves` batches, running between them (requests arrive
    # while others are on the device)
    chunks = np.array_split(np.arange(len(reqs)), waves)
    for c in chunks:
        for j in c:
            t, kind, vs, lo, hi = reqs[j]
            ids.append(S.submit(t, kind, vs, lo, hi))
        S.run(rounds_per_step)
    busy = 1
    guard = 0
    while busy:
        busy = S.run(rounds_per_step)
        guard += 1
        assert guard < 10000
    done = {c["id"]: c for c in S.poll(100000)}
    assert len(done) == len(reqs)
    out = []
    for j, rid in enumerate(ids):
        t, kind, vs, lo, hi = reqs[j]
        jobs = 2 * vs.size if kind == bp().REQ_PROBE else 1
        out.append(S.results(rid, jobs))
    return S, out, done


def test_serving_mix_matches_oracle_and_alone():
    insts, loaded, bases = _instances()
    reqs = _requests(insts, bases, 60, seed=3)
    S, mix, done = _serve(loaded, reqs, budget=256 << 20, waves=4)
    # two classes (300 and 3000-7500 variables), each with its own slots
    pools = S.info()["pools"]
    assert len(pools) == 2 and [p["instances"] for p in pools] == [2, 3]
    assert pools[0]["bytes_per_slot"] < pools[1]["bytes_per_slot"]
    for j, req in enumerate(reqs):
        t = req[0]
        want = _oracle_result(insts[t], bases[t], req)
        _same(mix[j], want, insts[t], "req%d" % j, evidence=req[1] == bp().REQ_PROPAGATE)
    # alone: a subset served one request per server run
    for j in range(0, len(reqs), 7):
        _, alone, _ = _serve(loaded, [reqs[j]], budget=64 << 20)
        _same(alone[0], mix[j], insts[reqs[j][0]], "alone%d" % j,
              evidence=reqs[j][1] == bp().REQ_PROPAGATE)


@pytest.mark.parametrize("full_rows", [False, True])
def test_serving_heavy_rows_incremental_and_full(full_rows):
    """Heavy rows of serving slots keep exact corrections over their
    instance's base rows (cleared per changed variable when a probe
    retires, all at once after a long fixing list), or, with FULL_ROWS, are
    summed chunk by chunk; both match the oracle on a pool of six slots
    that every slot reuses for many jobs."""
    insts, loaded, bases = _instances()
    reqs = _requests(insts, bases, 40, seed=21)
    t = 4  # the instance with heavy rows (5 rows over the threshold of 2048)
    inst = insts[t]
    lb, ub = bases[t]
    assert (np.diff(inst["row_ptr"]) > 2048).sum() >= 5
    ints = np.nonzero((inst["vtype"] == 1) & (lb < ub))[0]
    rng = np.random.default_rng(5)
    for _ in range(6):
        vs = np.sort(rng.choice(ints, size=min(400, ints.size), replace=False)).astype(np.int32)
        val = np.rint(rng.uniform(lb[vs], ub[vs]))
        reqs.append((t, bp().REQ_PROPAGATE, vs, val, val))
    opts = bp().default_options(heavy_threshold=2048)
    if full_rows:
        opts.flags |= bp().FLAG_FULL_ROWS
    per_slot = bp().Server(loaded, 1 << 40, opts).info()["bytes_per_slot"]
    S, out, done = _serve(loaded, reqs, budget=6 * per_slot, waves=3, opts=opts)
    assert S.info()["slots"] == 6
    for j, req in enumerate(reqs):
        want = _oracle_result(insts[req[0]], bases[req[0]], req)
        _same(out[j], want, insts[req[0]], "req%d" % j, evidence=req[1] == bp().REQ_PROPAGATE)


def test_serving_small_pool_and_validation():
    insts, loaded, bases = _instances()
    reqs = _requests(insts, bases, 25, seed=9)
    # a pool of 3 slots: requests wait for slots and refill them
    info_budget = bp().Server(loaded, 1 << 40).info()["bytes_per_slot"]
    S, mix, _ = _serve(loaded, reqs, budget=3 * info_budget, rounds_per_step=3, waves=3)
    assert S.info()["slots"] == 3
    for j, req in enumerate(reqs):
        t = req[0]
        _same(mix[j], _oracle_result(insts[t], bases[t], req), insts[t], "small%d" % j)
    with pytest.raises(bp().BPError):
        S.submit(99, bp().REQ_PROBE, np.array([0], np.int32))
    cont = np.nonzero(insts[0]["vtype"] == 0)[0][:1].astype(np.int32)
    with pytest.raises(bp().BPError):
        S.submit(0, bp().REQ_PROBE, cont)
    with pytest.raises(bp().BPError):
        S.submit(0, bp().REQ_PROPAGATE, np.array([1, 1], np.int32), np.zeros(2), np.ones(2))


def test_serving_infeasible_fixings():
    insts, loaded, bases = _instances()
    t = 0
    lb, ub = bases[t]
    bins = np.nonzero((insts[t]["vtype"] == 1) & (lb == 0) & (ub == 1))[0]
    # a value outside the base box: infeasible before any round
    fixed1 = np.nonzero((insts[t]["vtype"] == 1) & (lb == ub))[0]
    reqs = []
    if fixed1.size:
        v = fixed1[:1].astype(np.int32)
        reqs.append((t, bp().REQ_PROPAGATE, v, lb[v] + 1, lb[v] + 1))
    # many binaries fixed to 1 at once: typically infeasible after rounds
    vs = np.sort(bins[:40]).astype(np.int32)
    reqs.append((t, bp().REQ_PROPAGATE, vs, np.ones(vs.size), np.ones(vs.size)))
    _, mix, _ = _serve(loaded, reqs, budget=64 << 20)
    for j, req in enumerate(reqs):
        _same(mix[j], _oracle_result(insts[t], bases[t], req), insts[t], "inf%d" % j, evidence=True)


def test_serving_trickle_arrivals():
    """Requests arrive one at a time between short steps, with idle steps
    on an empty server before and between them: every job is still
    admitted (the job counter never runs past the end of the list) and
    every result matches the oracle."""
    insts, loaded, bases = _instances()
    reqs = _requests(insts, bases, 30, seed=21)
    opts = bp().default_options(rounds_per_launch=2)
    per_slot = bp().Server(loaded, 1 << 40, opts).info()["bytes_per_slot"]
    S = bp().Server(loaded, 4 * per_slot, opts)
    assert S.info()["slots"] == 4
    assert S.run(8) == 0  # idle steps before anything arrives
    ids = []
    for j, (t, kind, vs, lo, hi) in enumerate(reqs):
        ids.append(S.submit(t, kind, vs, lo, hi))
        S.run(2)  # the next request arrives while this one may still run
        if j == len(reqs) // 2:
            guard = 0
            while S.run(2):
                guard += 1
                assert guard < 10000
            assert S.run(8) == 0  # idle again, then more arrivals
    guard = 0
    while S.run(2):
        guard += 1
        assert guard < 10000
    done = {c["id"] for c in S.poll(100000)}
    assert done == set(ids)
    for j, rid in enumerate(ids):
        t, kind, vs, lo, hi = reqs[j]
        jobs = 2 * vs.size if kind == bp().REQ_PROBE else 1
        _same(S.results(rid, jobs), _oracle_result(insts[t], bases[t], reqs[j]), insts[t],
              "trickle%d" % j, evidence=kind == bp().REQ_PROPAGATE)



def test_serving_integer_probes():
    """Probe requests of general integers (half-intervals) in the mix."""
    insts, loaded, bases = _instances()
    rng = np.random.default_rng(31)
    reqs = []
    for t in range(len(insts)):
        lb, ub = bases[t]
        ints = np.nonzero((insts[t]["vtype"] == 1) & (lb < ub) & (ub - lb > 1))[0]
        if ints.size == 0:
            continue
        for _ in range(3):
            k = int(min(ints.size, rng.integers(1, 40)))
            vs = np.sort(rng.choice(ints, size=k, replace=False)).astype(np.int32)
            reqs.append((t, bp().REQ_PROBE, vs, None, None))
    assert len(reqs) >= 6
    _, mix, _ = _serve(loaded, reqs, budget=128 << 20, waves=2)
    for j, req in enumerate(reqs):
        t = req[0]
        _same(mix[j], _oracle_result(insts[t], bases[t], req), insts[t], "intprobe%d" % j)


def _drain(S):
    guard = 0
    while S.run(8):
        guard += 1
        assert guard < 10000
    return {c["id"]: c for c in S.poll(100000)}


def _check_requests(S, done, ids, reqs, insts, bases, what):
    for rid, q in zip(ids, reqs):
        t = q[0]
        got = S.results(rid, done[rid]["jobs"])
        _same(got, _oracle_result(insts[t], bases[t], q), insts[t], "%s %d" % (what, rid),
              evidence=q[1] == bp().REQ_PROPAGATE)


def test_serving_add_and_evict_instances():
    insts, loaded, bases = _instances()
    # the slots are sized by the instances given at creation; every row
    # bin of tiny_inf fits them
    S = bp().Server([loaded[4], loaded[0], loaded[2]], 1 << 28)
    order = [4, 0, 2]  # server index -> _instances() index
    reqs = [q for q in _requests(insts, bases, 40, seed=21) if q[0] in order][:12]
    local = [(order.index(q[0]),) + q[1:] for q in reqs]
    ids = [S.submit(*q) for q in local]
    busy = {order.index(q[0]) for q in reqs}
    for t in busy:  # instances with queued requests stay
        with pytest.raises(bp().BPError) as e:
            S.evict(t)
        assert e.value.code == bp().BP_ESTATE
    done = _drain(S)
    _check_requests(S, done, ids, reqs, insts, bases, "before eviction")
    S.evict(1)
    S.evict(2)
    vs = np.array([0], np.int32)
    with pytest.raises(bp().BPError) as e:
        S.submit(1, bp().REQ_PROBE, vs)
    assert e.value.code == bp().BP_EINVAL
    with pytest.raises(bp().BPError) as e:
        S.evict(1)
    assert e.value.code == bp().BP_EINVAL
    # freed indices are taken in order
    assert S.add_instance(loaded[1]) == 1
    assert S.add_instance(loaded[2]) == 2
    order = [4, 1, 2]
    with pytest.raises(bp().BPError) as e:
        S.add_instance(loaded[1])
    assert e.value.code == bp().BP_EINVAL
    reqs = [q for q in _requests(insts, bases, 60, seed=22) if q[0] in order][:18]
    local = [(order.index(q[0]),) + q[1:] for q in reqs]
    ids = [S.submit(*q) for q in local]
    done = _drain(S)
    _check_requests(S, done, ids, reqs, insts, bases, "after adding")
    # an instance larger than the slots is refused
    big = gen.make("single", 6, scale=0.2)
    B = bp().Instance(big, bp().default_options(heavy_threshold=2048))
    r, lb, ub = gpu_propagate(B, big)
    assert r["status"] == bp().BP_OK
    with pytest.raises(bp().BPError) as e:
        S.add_instance(B)
    assert e.value.code == bp().BP_ECAPACITY
