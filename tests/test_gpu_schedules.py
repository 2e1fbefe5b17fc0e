"""Schedule invariance: every row-split schedule the autotuner may choose
(heavy-row threshold, heavy chunk size, rounds per graph, probe slots)
returns bit-identical results; the autotuner keeps a schedule and its cache
round-trips."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, bp, dev, gpu_propagate
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ht,hc,rpl", [(1024, 256, 1), (2048, 512, 4), (4096, 1024, 8),
                                        (8192, 4096, 16), (32768, 2048, 32)])
def test_schedules_give_identical_results(ht, hc, rpl):
    inst = gen.make("single", 6, scale=0.2)
    ro, lo, uo = oracle.propagate(inst)
    I = bp().Instance(inst, bp().default_options(heavy_threshold=ht, heavy_chunk=hc,
                                                 rounds_per_launch=rpl))
    rg, lg, ug = gpu_propagate(I, inst)
    assert_same(inst, rg, lg, ug, ro, lo, uo, "schedule %d/%d/%d" % (ht, hc, rpl))
    assert np.array_equal(lg, lo) and np.array_equal(ug, uo)


def test_autotune_and_cache():
    inst = gen.make("single", 7, scale=0.1)
    I = bp().Instance(inst)
    lb = dev(inst["lb"], torch.float64)
    ub = dev(inst["ub"], torch.float64)
    _, blb, bub = oracle.propagate(inst)
    vs = gen.pick_probe_vars(inst, blb, bub, 40, seed=2)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        t = I.autotune(lb, ub, dev(vs, torch.int32), cache_path=path)
        assert t["trials"] > 10 and not t["from_cache"]
        assert (lb.cpu().numpy() == inst["lb"]).all()  # inputs untouched
        # results with the chosen schedule still match the oracle
        r, lg, ug = gpu_propagate(I, inst)
        ro, lo, uo = oracle.propagate(inst)
        assert_same(inst, r, lg, ug, ro, lo, uo, "tuned")
        G = I.probe(dev(vs, torch.int32))
        O = oracle.probe(inst, lo, uo, vs)
        assert np.array_equal(G["var"].cpu().numpy(), O["var"])
        assert np.array_equal(G["status"].cpu().numpy(), O["status"])
        # a new instance of the same matrix reads the cache
        I2 = bp().Instance(inst)
        t2 = I2.autotune(lb, ub, dev(vs, torch.int32), cache_path=path)
        assert t2["from_cache"] and t2["trials"] == 0
        for key in ("heavy_threshold", "heavy_chunk", "rounds_per_launch", "probe_slots"):
            assert t2[key] == t[key]
        r2, lg2, ug2 = gpu_propagate(I2, inst)
        assert_same(inst, r2, lg2, ug2, ro, lo, uo, "cached")
        # later lines for the same key with schedules the engine does not
        # support (zero or unaligned chunks, a tiny threshold) are ignored
        with open(path) as f:
            key = f.readline().split()[0]
        with open(path, "a") as f:
            f.write("%s 4096 0 8 512 1.0\n%s 4096 300 8 512 1.0\n%s 16 1024 8 512 1.0\n" % (key, key, key))
        I3 = bp().Instance(inst)
        t3 = I3.autotune(lb, ub, dev(vs, torch.int32), cache_path=path)
        assert t3["from_cache"]
        for k in ("heavy_threshold", "heavy_chunk", "rounds_per_launch", "probe_slots"):
            assert t3[k] == t[k]


@pytest.mark.parametrize("grid", [256, 1024, 8192])
def test_lane_grids_give_identical_results(grid):
    """The lane engine's workgroups per round kernel change nothing."""
    inst = gen.make("single", 4, scale=0.02)
    _, lb, ub = oracle.propagate(inst)
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=40, frac=0.004, seed=8)
    ptr = np.zeros(41, np.int64)
    ptr[1:] = np.cumsum([c.size for c in changed])
    idx = np.concatenate(changed).astype(np.int32)
    out = []
    for g in (0, grid):
        I = bp().Instance(inst, bp().default_options(lv_grid=g))
        tl, tu = dev(LB, torch.float64), dev(UB, torch.float64)
        res = I.propagate_batch(tl, tu, dev(ptr, torch.int64), dev(idx, torch.int32))
        torch.cuda.synchronize()
        out.append((res, tl.cpu().numpy(), tu.cpu().numpy()))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])


def test_autotune_batch_and_cache():
    """bp_autotune_batch times the batch itself, leaves the inputs alone,
    keeps a lane schedule that gives the oracle's results, and its cache
    round-trips."""
    inst = gen.make("single", 9, scale=0.02)
    _, lb, ub = oracle.propagate(inst)
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=48, frac=0.003, seed=4)
    ptr = np.zeros(49, np.int64)
    ptr[1:] = np.cumsum([c.size for c in changed])
    idx = np.concatenate(changed).astype(np.int32)
    tl, tu = dev(LB, torch.float64), dev(UB, torch.float64)
    pd, idd = dev(ptr, torch.int64), dev(idx, torch.int32)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        I = bp().Instance(inst)
        t = I.autotune_batch(tl, tu, pd, idd, cache_path=path)
        assert t["trials"] >= 6 and not t["from_cache"] and t["lv_grid"] in (1024, 2048, 4096, 8192)
        assert np.array_equal(tl.cpu().numpy(), LB) and np.array_equal(tu.cpu().numpy(), UB)
        res = I.propagate_batch(tl, tu, pd, idd)
        torch.cuda.synchronize()
        GL, GU = tl.cpu().numpy(), tu.cpu().numpy()
        for v in range(48):
            ro, lo, uo = oracle.propagate(inst, LB[v], UB[v], changed=changed[v])
            assert_same(inst, res[v], GL[v], GU[v], ro, lo, uo, "tuned batch v%d" % v)
        I2 = bp().Instance(inst)
        t2 = I2.autotune_batch(dev(LB, torch.float64), dev(UB, torch.float64), pd, idd, cache_path=path)
        assert t2["from_cache"] and t2["trials"] == 0
        assert (t2["lv_grid"], t2["rounds_per_launch"]) == (t["lv_grid"], t["rounds_per_launch"])
