"""Incremental activities of heavy rows (bp_propagate of one vector): the
exact sums of each heavy row are corrected by every accepted bound change
instead of being recomputed from the row's nonzeros.  Outcome, rounds,
propagated nonzeros, evidence and bounds must match the oracle, and be
bit-identical to the full recomputation (BP_FLAG_FULL_ROWS)."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_same, bp, gpu_propagate
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu
INF = math.inf


def _dense_instance(seed, n=3000, dense=4, m_short=2500, frac_inf=0.25):
    """A few rows longer than the smallest heavy threshold (1024) with mixed
    signs and sides close to their activity range, so that they tighten
    bounds and are not filtered as quiet; many short rows; a quarter of the
    variables with one infinite bound, tightened to finite values as the
    rounds go."""
    rng = np.random.default_rng(seed)
    vtype = (rng.random(n) < 0.6).astype(np.uint8)
    lb = np.where(vtype == 1, 0.0, -50.0)
    ub = np.where(vtype == 1, rng.integers(1, 11, n).astype(float), 50.0)
    inf = rng.random(n) < frac_inf
    side = rng.random(n) < 0.5
    lb[inf & side] = -INF
    ub[inf & ~side] = INF
    x = np.where(np.isfinite(lb), lb, ub - 3.0) + rng.random(n) * 2.0  # a point the rows keep
    x = np.where(vtype == 1, np.clip(np.round(x), lb, ub), np.clip(x, lb, ub))
    rows, lo, hi = [], [], []
    for _ in range(dense):
        L = int(rng.integers(1100, 2600))
        cols = np.sort(rng.choice(n, size=L, replace=False))
        vals = rng.choice([-1.0, 1.0], L) * rng.uniform(0.5, 4.0, L)
        act = float(vals @ x[cols])
        rows.append((cols, vals))
        lo.append(act - rng.uniform(1.0, 20.0) if rng.random() < 0.5 else -INF)
        hi.append(act + rng.uniform(1.0, 20.0))
    for _ in range(m_short):
        L = int(rng.integers(2, 7))
        cols = np.sort(rng.choice(n, size=L, replace=False))
        vals = rng.choice([-1.0, 1.0], L) * rng.integers(1, 6, L).astype(float)
        act = float(vals @ x[cols])
        rows.append((cols, vals))
        lo.append(act - rng.uniform(0.0, 3.0) if rng.random() < 0.3 else -INF)
        hi.append(act + rng.uniform(0.0, 3.0))
    return gen.from_rows(n, rows, lo, hi, vtype, lb, ub)


def _orc(o):
    return oracle.Options(feastol=o.feastol, inttol=o.inttol, tau=o.tau, max_rounds=o.max_rounds)


def _three_ways(inst, lb=None, ub=None, changed=None, what="", **kw):
    """Incremental, full recomputation and the oracle on the same input."""
    o_inc = bp().default_options(heavy_threshold=1024, **kw)
    o_full = bp().default_options(heavy_threshold=1024, **kw)
    o_full.flags |= bp().FLAG_FULL_ROWS
    ri, li, ui = gpu_propagate(bp().Instance(inst, o_inc), inst, lb, ub, changed)
    rf, lf, uf = gpu_propagate(bp().Instance(inst, o_full), inst, lb, ub, changed)
    ro, lo, uo = oracle.propagate(inst, lb, ub, changed=changed, opts=_orc(o_inc))
    assert_same(inst, ri, li, ui, ro, lo, uo, what + " incremental")
    assert ri == rf, (what, ri, rf)
    if ri["status"] != bp().BP_INFEASIBLE:
        assert np.array_equal(li.view(np.int64), lf.view(np.int64)), what
        assert np.array_equal(ui.view(np.int64), uf.view(np.int64)), what
    return ri, li, ui


@pytest.mark.parametrize("seed", range(6))
def test_dense_rows_cold(seed):
    inst = _dense_instance(seed)
    assert (np.diff(inst["row_ptr"]) > 1024).sum() >= 3
    r, _, _ = _three_ways(inst, what="dense%d" % seed)
    assert r["rounds"] >= 2


@pytest.mark.parametrize("seed", range(3))
def test_dense_rows_warm_fixings(seed):
    """Warm starts from the oracle's fixed point with a few variables fixed:
    the first round builds the accumulators, later rounds correct them."""
    inst = _dense_instance(10 + seed)
    r0, lb, ub = oracle.propagate(inst)
    if r0["status"] != oracle.BP_OK:
        pytest.skip("infeasible root")
    rng = np.random.default_rng(seed)
    ints = np.nonzero((inst["vtype"] == 1) & (lb < ub) & np.isfinite(lb) & np.isfinite(ub))[0]
    for count in (1, 5, 40):
        pick = np.sort(rng.choice(ints, size=min(count, ints.size), replace=False)).astype(np.int32)
        l2, u2 = lb.copy(), ub.copy()
        v = np.round(rng.uniform(lb[pick], ub[pick]))
        l2[pick] = v
        u2[pick] = v
        _three_ways(inst, l2, u2, pick, what="warm%d/%d" % (seed, count))


@pytest.mark.parametrize("max_rounds", [1, 2, 3, 7])
def test_round_limit(max_rounds):
    inst = _dense_instance(21)
    _three_ways(inst, what="limit%d" % max_rounds, max_rounds=max_rounds)


def test_force_exact_with_incremental_rows():
    inst = _dense_instance(22)
    o = bp().default_options(heavy_threshold=1024)
    o.flags |= bp().FLAG_FORCE_EXACT
    r, l, u = gpu_propagate(bp().Instance(inst, o), inst)
    ro, lo, uo = oracle.propagate(inst)
    assert_same(inst, r, l, u, ro, lo, uo, "force-exact")


@pytest.mark.parametrize("scale,chunk", [(0.05, 256), (0.2, 1024)])
def test_single_workload_scaled_many_heavy_rows(scale, chunk):
    """Scan rounds (large first updates) rebuild the accumulators; later
    rounds correct them; many chunks per row."""
    inst = gen.make("single", 3, scale=scale)
    _three_ways(inst, what="single %.2f" % scale, heavy_chunk=chunk)


def test_infeasible_after_fixings():
    inst = _dense_instance(30)
    r0, lb, ub = oracle.propagate(inst)
    if r0["status"] != oracle.BP_OK:
        pytest.skip("infeasible root")
    ints = np.nonzero((inst["vtype"] == 1) & (lb < ub) & np.isfinite(ub))[0][:400].astype(np.int32)
    l2, u2 = lb.copy(), ub.copy()
    l2[ints] = ub[ints]
    r, _, _ = _three_ways(inst, l2, ub.copy(), ints, what="infeasible")
    assert r["status"] in (bp().BP_INFEASIBLE, bp().BP_OK)


def test_repeated_calls_reuse_the_engine():
    """Accumulators start from zero in every call (cold after warm, warm
    after cold)."""
    inst = _dense_instance(40)
    I = bp().Instance(inst, bp().default_options(heavy_threshold=1024))
    ro, lo, uo = oracle.propagate(inst)
    for _ in range(3):
        r, l, u = gpu_propagate(I, inst)
        assert_same(inst, r, l, u, ro, lo, uo, "repeat")
        if ro["status"] == oracle.BP_OK:
            r2, l2, u2 = gpu_propagate(I, inst, lo, uo, np.zeros(0, np.int32))
            assert r2["rounds"] == 0


@pytest.mark.parametrize("B,flags", [(2, 0), (5, 0), (16, "slots")])
@pytest.mark.parametrize("cold", [True, False])
def test_several_vectors_keep_their_own_accumulators(B, flags, cold):
    """Calls of up to 16 vectors on the slot engine: on a cold start every
    vector's heavy rows keep accumulators of their own (warm starts of
    several vectors recompute their rows); results per vector match the
    oracle and the full recomputation."""
    import torch
    from gpu_util import dev
    inst = _dense_instance(50 + B)
    r0, lb, ub = oracle.propagate(inst)
    if r0["status"] != oracle.BP_OK:
        pytest.skip("infeasible root")
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=B, frac=0.01, seed=B)
    ptr = np.zeros(B + 1, np.int64)
    ptr[1:] = np.cumsum([c.size for c in changed])
    idx = np.concatenate(changed).astype(np.int32)
    outs = []
    for full in (False, True):
        o = bp().default_options(heavy_threshold=1024)
        if flags == "slots":
            o.flags |= bp().FLAG_BATCH_SLOTS
        if full:
            o.flags |= bp().FLAG_FULL_ROWS
        I = bp().Instance(inst, o)
        tl, tu = dev(LB, torch.float64), dev(UB, torch.float64)
        if cold:
            res = I.propagate_batch(tl, tu)
        else:
            res = I.propagate_batch(tl, tu, dev(ptr, torch.int64), dev(idx, torch.int32))
        torch.cuda.synchronize()
        outs.append((res, tl.cpu().numpy(), tu.cpu().numpy()))
    (ri, li, ui), (rf, lf, uf) = outs
    assert ri == rf
    for v in range(B):
        ro, lo, uo = oracle.propagate(inst, LB[v], UB[v], changed=None if cold else changed[v])
        assert_same(inst, ri[v], li[v], ui[v], ro, lo, uo, "batch %d v%d" % (B, v))
        if ri[v]["status"] != bp().BP_INFEASIBLE:
            assert np.array_equal(li[v].view(np.int64), lf[v].view(np.int64))
            assert np.array_equal(ui[v].view(np.int64), uf[v].view(np.int64))


@pytest.mark.parametrize("name", ["dense", "single"])
def test_successive_calls_on_one_instance(name):
    """Many calls on one instance, one and two vectors, some ending
    infeasible (a crossed variable leaves queued rows to drain, possibly in
    a rebuild round): no queue flag or accumulator state may leak into the
    next call."""
    import torch
    from gpu_util import dev
    inst = _dense_instance(60) if name == "dense" else gen.make("single", 0, scale=0.2)
    thr = 1024 if name == "dense" else 8192
    r0, lb, ub = oracle.propagate(inst)
    if r0["status"] != oracle.BP_OK:
        pytest.skip("infeasible root")
    I = bp().Instance(inst, bp().default_options(heavy_threshold=thr))
    rng = np.random.default_rng(7)
    ints = np.nonzero((inst["vtype"] == 1) & (lb < ub) & np.isfinite(lb) & np.isfinite(ub))[0]
    for t in range(24):
        B = 1 + t % 2
        k = [3, 40, 300, 1200][t % 4]
        LB, UB, changed = [], [], []
        for v in range(B):
            pick = np.sort(rng.choice(ints, size=min(k, ints.size), replace=False)).astype(np.int32)
            l2, u2 = lb.copy(), ub.copy()
            val = np.round(rng.uniform(lb[pick], ub[pick]))
            l2[pick] = val
            u2[pick] = val
            changed.append(pick)
            LB.append(l2)
            UB.append(u2)
        LB, UB = np.array(LB), np.array(UB)
        ptr = np.zeros(B + 1, np.int64)
        ptr[1:] = np.cumsum([c.size for c in changed])
        tl, tu = dev(LB, torch.float64), dev(UB, torch.float64)
        res = I.propagate_batch(tl, tu, dev(ptr, torch.int64), dev(np.concatenate(changed), torch.int32))
        torch.cuda.synchronize()
        gl, gu = tl.cpu().numpy(), tu.cpu().numpy()
        for v in range(B):
            ro, lo, uo = oracle.propagate(inst, LB[v], UB[v], changed=changed[v])
            assert_same(inst, res[v], gl[v], gu[v], ro, lo, uo, "call %d v%d" % (t, v))


def test_byte_accounting_counters():
    """The counters behind the roofline figures: heavy rows tested from
    their accumulators and their unread nonzeros (zero with the full
    recomputation), the update kernel's entries, column entries and
    corrections, and both kernels' event times."""
    import torch
    from gpu_util import dev
    inst = gen.make("single", 3, scale=0.2)
    stats = {}
    for full in (False, True):
        flags = bp().FLAG_COUNT_VARS | bp().FLAG_TIME_KERNELS | (bp().FLAG_FULL_ROWS if full else 0)
        I = bp().Instance(inst, bp().default_options(flags=flags))
        tl, tu = dev(inst["lb"], torch.float64), dev(inst["ub"], torch.float64)
        r = I.propagate(tl, tu)
        stats[full] = (r, I.kernel_stats(reset=True))
    (ri, si), (rf, sf) = stats[False], stats[True]
    assert ri == rf
    assert si["rows"] == sf["rows"] and si["nnz"] == sf["nnz"] == ri["nnz_propagated"]
    assert sf["rows_kept"] == 0 and sf["nnz_kept"] == 0 and sf["apply_corr"] == 0
    assert 0 < si["rows_kept"] <= si["rows"] and 0 < si["nnz_kept"] <= si["nnz"]
    assert si["apply_corr"] > 0 and si["vars_read"] < sf["vars_read"]
    for s in (si, sf):
        assert s["apply_entries"] >= s["vars_written"] > 0 and s["apply_colent"] > 0
        assert s["launches"] >= ri["rounds"] and s["ms"] > 0 and s["apply_ms"] > 0


def test_host_rounds_and_probe_engine_reuse():
    """Host-driven rounds, and a plain propagation on the engine a probe
    call sized for its slots (no scan rounds there): both keep incremental
    heavy rows and match the oracle."""
    import torch
    from gpu_util import dev, gpu_base
    inst = _dense_instance(70)
    ro, lo, uo = oracle.propagate(inst)
    o = bp().default_options(heavy_threshold=1024)
    o.flags |= bp().FLAG_HOST_ROUNDS
    r, l, u = gpu_propagate(bp().Instance(inst, o), inst)
    assert_same(inst, r, l, u, ro, lo, uo, "host rounds")
    if ro["status"] != oracle.BP_OK:
        return
    I = bp().Instance(inst, bp().default_options(heavy_threshold=1024, probe_slots=64))
    gpu_base(I, lo, uo)
    bins = np.nonzero((inst["vtype"] == 1) & (lo == 0) & (uo == 1))[0][:40].astype(np.int32)
    G = I.probe(dev(bins, torch.int32))
    torch.cuda.synchronize()
    O = oracle.probe(inst, lo, uo, bins)
    assert np.array_equal(G["status"].cpu().numpy(), O["status"])
    assert np.array_equal(G["nnz"].cpu().numpy(), O["nnz"])
    for seed in range(3):
        rng = np.random.default_rng(seed)
        ints = np.nonzero((inst["vtype"] == 1) & (lo < uo) & np.isfinite(lo) & np.isfinite(uo))[0]
        pick = np.sort(rng.choice(ints, size=25, replace=False)).astype(np.int32)
        l2, u2 = lo.copy(), uo.copy()
        l2[pick] = np.round(rng.uniform(lo[pick], uo[pick]))
        u2[pick] = l2[pick]
        rg, lg, ug = gpu_propagate(I, inst, l2, u2, pick)
        r2, lo2, uo2 = oracle.propagate(inst, l2, u2, changed=pick)
        assert_same(inst, rg, lg, ug, r2, lo2, uo2, "after probe %d" % seed)
        rg, lg, ug = gpu_propagate(I, inst, l2, u2)
        r2, lo2, uo2 = oracle.propagate(inst, l2, u2)
        assert_same(inst, rg, lg, ug, r2, lo2, uo2, "cold after probe %d" % seed)
