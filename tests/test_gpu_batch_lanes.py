"""Batched propagation with one vector per lane (bp_propagate_batch with 16
or more vectors): each vector's outcome, rounds, propagated nonzeros,
evidence and bounds match the oracle run on that vector alone, and the slot
engine's results for the same batch.  Each case runs with whole records
and, where the instance has a base box (overlay = True: the oracle's root,
or the instance's bounds, handed over by a warm start with an empty change
list), with vectors read as overlays on it."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, bp, dev, gpu_base
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu


def _batch(I, LB, UB, changed=None):
    tl, tu = dev(LB, torch.float64), dev(UB, torch.float64)
    if changed is None:
        res = I.propagate_batch(tl, tu)
    else:
        ptr = np.zeros(len(changed) + 1, np.int64)
        ptr[1:] = np.cumsum([c.size for c in changed])
        idx = np.concatenate(changed).astype(np.int32) if ptr[-1] else np.zeros(1, np.int32)
        res = I.propagate_batch(tl, tu, dev(ptr, torch.int64), dev(idx, torch.int32))
    torch.cuda.synchronize()
    return res, tl.cpu().numpy(), tu.cpu().numpy()


def _check(inst, res, GL, GU, LB, UB, changed, what, opts=None):
    for v in range(len(res)):
        ro, lo, uo = oracle.propagate(inst, LB[v], UB[v],
                                      changed=None if changed is None else changed[v], opts=opts)
        assert_same(inst, res[v], GL[v], GU[v], ro, lo, uo, "%s v%d" % (what, v))


def _instance(inst, overlay, lb, ub, **opt):
    I = bp().Instance(inst, bp().default_options(**opt) if opt else None)
    if overlay:
        gpu_base(I, lb, ub)
    return I


def _root(inst):
    r, lb, ub = oracle.propagate(inst)
    assert r["status"] == oracle.BP_OK
    return lb, ub


@pytest.mark.parametrize("overlay", [False, True])
@pytest.mark.parametrize("B,frac", [(16, 0.05), (70, 0.01), (130, 0.002)])
def test_fix_vectors_match_oracle(B, frac, overlay):
    """Ragged groups (70, 130 vectors), mostly infeasible (5% fixed) to
    mostly feasible (0.2% fixed) candidates."""
    inst = gen.make("single", 5, scale=0.02)
    lb, ub = _root(inst)
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=B, frac=frac, seed=B)
    I = _instance(inst, overlay, lb, ub)
    res, GL, GU = _batch(I, LB, UB, changed)
    _check(inst, res, GL, GU, LB, UB, changed, "fix%d" % B)
    assert len({r["status"] for r in res}) >= 1


@pytest.mark.parametrize("overlay", [False, True])
def test_long_rows_in_chunks(overlay):
    """Rows of several chunks (dense rows of the scaled single workload)."""
    inst = gen.make("single", 7, scale=0.06)
    assert np.diff(inst["row_ptr"]).max() > 1024
    lb, ub = _root(inst)
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=24, frac=0.003, seed=3)
    I = _instance(inst, overlay, lb, ub)
    res, GL, GU = _batch(I, LB, UB, changed)
    _check(inst, res, GL, GU, LB, UB, changed, "long")


@pytest.mark.parametrize("overlay", [False, True])
def test_cold_vectors_and_slot_engine_agree(overlay):
    """Cold start of different boxes; the slot engine (BP_FLAG_BATCH_SLOTS)
    gives bit-identical results and bounds."""
    inst = gen.make("single", 2, scale=0.02)
    rng = np.random.default_rng(4)
    B = 40
    LB = np.repeat(inst["lb"][None], B, 0)
    UB = np.repeat(inst["ub"][None], B, 0)
    ints = np.nonzero((inst["vtype"] == 1) & (inst["ub"] > inst["lb"]))[0]
    for v in range(1, B):
        pick = rng.choice(ints, size=3, replace=False)
        UB[v, pick] = np.maximum(LB[v, pick], UB[v, pick] - 1)
    I = _instance(inst, overlay, inst["lb"], inst["ub"])
    res, GL, GU = _batch(I, LB, UB)
    _check(inst, res, GL, GU, LB, UB, None, "cold")
    Is = bp().Instance(inst, bp().default_options(flags=bp().FLAG_BATCH_SLOTS))
    rs, SL, SU = _batch(Is, LB, UB)
    assert rs == res
    # bounds are specified (and compared) unless the outcome is infeasible
    ok = np.array([r["status"] != oracle.BP_INFEASIBLE for r in res])
    assert ok.sum() >= B // 3
    assert np.array_equal(SL[ok], GL[ok]) and np.array_equal(SU[ok], GU[ok])
    # the lane engine leaves an infeasible vector's bounds as given
    assert np.array_equal(GL[~ok], LB[~ok]) and np.array_equal(GU[~ok], UB[~ok])


@pytest.mark.parametrize("overlay", [False, True])
def test_probe_workload_rows(overlay):
    """Set-cover and big-M rows."""
    inst = gen.make("probe", 1, scale=0.004)
    lb, ub = _root(inst)
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=64, frac=0.002, seed=9)
    I = _instance(inst, overlay, lb, ub)
    res, GL, GU = _batch(I, LB, UB, changed)
    _check(inst, res, GL, GU, LB, UB, changed, "probe")


@pytest.mark.parametrize("overlay", [False, True])
def test_edge_cases(overlay):
    """Crossed boxes, empty and repeated changed lists, infinite bounds, the
    round limit, and a second call on the same buffers."""
    inst = gen.make("tiny_inf", 3)
    lb, ub = inst["lb"].copy(), inst["ub"].copy()
    B = 33
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=B, frac=0.05, seed=5)
    LB[3, 7], UB[3, 7] = 5.0, 2.0                      # crossed box
    changed[4] = np.zeros(0, np.int32)                 # nothing to do
    changed[5] = np.concatenate([changed[5], changed[5][:3]])  # repeats
    I = _instance(inst, overlay, lb, ub)
    res, GL, GU = _batch(I, LB, UB, changed)
    _check(inst, res, GL, GU, LB, UB, changed, "edge")
    assert res[3]["status"] == oracle.BP_INFEASIBLE and res[4]["rounds"] == 0
    # again, fewer vectors, on the buffers of the first call
    res2, GL2, GU2 = _batch(I, LB[:17], UB[:17], changed[:17])
    assert res2 == res[:17]
    assert np.array_equal(GL2, GL[:17]) and np.array_equal(GU2, GU[:17])
    # round limit
    Ir = _instance(inst, overlay, lb, ub, max_rounds=1)
    rr, RL, RU = _batch(Ir, LB, UB, changed)
    oo = oracle.Options()
    oo.max_rounds = 1
    for v in range(B):
        ro, lo, uo = oracle.propagate(inst, LB[v], UB[v], changed=changed[v], opts=oo)
        assert_same(inst, rr[v], RL[v], RU[v], ro, lo, uo, "limit v%d" % v)


def test_force_exact_and_counting_change_nothing():
    inst = gen.make("single", 11, scale=0.01)
    lb, ub = _root(inst)
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=20, frac=0.01, seed=2)
    ref, RL, RU = _batch(bp().Instance(inst), LB, UB, changed)
    for flags in (bp().FLAG_FORCE_EXACT, bp().FLAG_COUNT_VARS, bp().FLAG_HOST_ROUNDS):
        res, GL, GU = _batch(bp().Instance(inst, bp().default_options(flags=flags)), LB, UB, changed)
        assert res == ref, flags
        assert np.array_equal(GL, RL) and np.array_equal(GU, RU), flags


def test_overlay_and_dense_agree_bit_for_bit():
    """The same batch with the overlay (a base box) and with whole records
    (BP_FLAG_LV_DENSE): identical results and bounds, also on a second call
    after the base moved."""
    inst = gen.make("single", 3, scale=0.03)
    lb, ub = _root(inst)
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=100, frac=0.004, seed=6)
    ref, RL, RU = _batch(_instance(inst, False, lb, ub), LB, UB, changed)
    for flags in (0, bp().FLAG_LV_DENSE):
        I = _instance(inst, True, lb, ub, flags=flags)
        res, GL, GU = _batch(I, LB, UB, changed)
        assert res == ref, flags
        assert np.array_equal(GL, RL) and np.array_equal(GU, RU), flags
        # a base that differs from every vector in many places: still exact
        gpu_base(I, inst["lb"], inst["ub"])
        res, GL, GU = _batch(I, LB, UB, changed)
        assert res == ref, flags
        assert np.array_equal(GL, RL) and np.array_equal(GU, RU), flags


def test_long_rows_as_base_plus_corrections():
    """Dense rows queued by most vectors of each group, every vector fixing
    a few variables of the base: their chunks are summed as the chunk's sums
    at the base bounds plus each vector's corrections (counted), and every
    result matches the oracle.  When the base moves, the chunk sums are
    taken again, and the results match on the new base too."""
    inst = gen.make("single", 7, scale=0.06)
    assert np.diff(inst["row_ptr"]).max() > 1024
    lb, ub = _root(inst)
    I = _instance(inst, True, lb, ub)
    for step in range(2):
        LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=128, frac=0.002, seed=40 + step)
        I.kernel_stats(reset=True)
        res, GL, GU = _batch(I, LB, UB, changed)
        assert I.kernel_stats(reset=True)["lv_corr_chunks"] > 0
        _check(inst, res, GL, GU, LB, UB, changed, "corr%d" % step)
        # a new base: the fixed point of one feasible vector
        v = next(j for j, r in enumerate(res) if r["status"] == oracle.BP_OK)
        ro, lb, ub = oracle.propagate(inst, LB[v], UB[v], changed=changed[v])
        assert ro["status"] == oracle.BP_OK
        gpu_base(I, lb, ub)
