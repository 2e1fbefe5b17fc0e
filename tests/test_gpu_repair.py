"""The repair procedure on the GPU (bp_repair, and bp_round with repairs on
a marked path) against the CPU oracle on the same inputs: outcome, attempts,
shifts, reason and propagated nonzeros equal; integer bounds bit for bit;
continuous bounds within 1e-9 relative (they come from propagation).  Also
the hand-traced cases of tests/golden/w8_repair.json, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import bp, dev
from helpers import _f, bits, rel_close, repair_case_mismatch, repair_cases, repair_round_scenario
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu


def _gpu_repair(I, lb, ub, lb0, ub0, shifts=64, attempts=8):
    tl, tu = dev(lb, torch.float64), dev(ub, torch.float64)
    r = I.repair(tl, tu, dev(lb0, torch.float64), dev(ub0, torch.float64), shifts, attempts)
    torch.cuda.synchronize()
    return r, tl.cpu().numpy(), tu.cpu().numpy()


def _same_box(inst, gl, gu, ol, ou, what):
    integ = inst["vtype"] == 1
    assert np.array_equal(bits(gl[integ]), bits(ol[integ])), (what, "integer lb")
    assert np.array_equal(bits(gu[integ]), bits(ou[integ])), (what, "integer ub")
    assert rel_close(gl[~integ], ol[~integ]), (what, "continuous lb")
    assert rel_close(gu[~integ], ou[~integ]), (what, "continuous ub")


def _both(inst, lb, ub, lb0=None, ub0=None, shifts=64, attempts=8, what=""):
    lb0 = inst["lb"] if lb0 is None else lb0
    ub0 = inst["ub"] if ub0 is None else ub0
    I = bp().Instance(inst)
    rg, gl, gu = _gpu_repair(I, lb, ub, lb0, ub0, shifts, attempts)
    ro, ol, ou = oracle.repair(inst, lb, ub, lb0, ub0, max_shifts=shifts, max_attempts=attempts)
    assert rg == ro, (what, rg, ro)
    _same_box(inst, gl, gu, ol, ou, what)
    return rg


def test_golden_w8_cases():
    for inst, c in repair_cases():
        I = bp().Instance(inst)
        r, gl, gu = _gpu_repair(I, np.asarray([_f(x) for x in c["box_lb"]]),
                                np.asarray([_f(x) for x in c["box_ub"]]), inst["lb"], inst["ub"],
                                c["max_shifts"], c["max_attempts"])
        assert repair_case_mismatch(c, r, gl, gu) is None, repair_case_mismatch(c, r, gl, gu)


def test_golden_w8_rounding_with_repair():
    inst, s = repair_round_scenario()
    r0, lb, ub = oracle.propagate(inst)
    for limits, exp, fl, fu in ((s["repair_limits"], s["expect"], s["final_lb"], s["final_ub"]),
                                (None, s["expect_no_repair"], s["final_lb_no_repair"],
                                 s["final_ub_no_repair"])):
        o = bp().default_options()
        if limits:
            o.repair_calls, o.repair_attempts, o.repair_shifts = limits
        I = bp().Instance(inst, o)
        tl, tu = dev(lb, torch.float64), dev(ub, torch.float64)
        r = I.round(tl, tu, dev(s["x"], torch.float64), dev(s["draws"], torch.float64))
        torch.cuda.synchronize()
        assert r == exp, (r, exp)
        assert tl.cpu().tolist() == fl and tu.cpu().tolist() == fu


@pytest.mark.parametrize("seed", range(0, 120, 3))
def test_micro_instances(seed):
    """All variables fixed at a point of the domains, then the first half."""
    inst = gen.make_micro(seed)
    n = inst["n"]
    rng = np.random.default_rng(seed)
    x = np.array([rng.integers(int(inst["lb"][i]), int(inst["ub"][i]) + 1) for i in range(n)],
                 dtype=np.float64)
    _both(inst, x, x, what="micro %d all fixed" % seed)
    k = max(1, n // 2)
    bl, bu = inst["lb"].copy(), inst["ub"].copy()
    bl[:k] = x[:k]
    bu[:k] = x[:k]
    _both(inst, bl, bu, what="micro %d half fixed" % seed)
    _both(inst, x, x, shifts=1, attempts=1, what="micro %d one shift" % seed)


@pytest.mark.parametrize("scale,seed", [(0.02, 0), (0.02, 1), (0.05, 2)])
def test_scaled_single_workload(scale, seed):
    """Rows of up to a few thousand nonzeros (chunked activities), real
    coefficients: a seeded 30% of the integer variables fixed to random
    values of their root box, repaired against the root box."""
    inst = gen.make("single", seed, scale=scale)
    r0, lb, ub = oracle.propagate(inst)
    rng = np.random.default_rng(seed)
    ints = np.nonzero((inst["vtype"] == 1) & (lb < ub))[0]
    pick = rng.choice(ints, size=int(0.3 * ints.size), replace=False)
    bl, bu = lb.copy(), ub.copy()
    v = np.floor(lb[pick] + rng.random(pick.size) * (ub[pick] - lb[pick] + 1))
    v = np.minimum(v, ub[pick])
    bl[pick] = v
    bu[pick] = v
    r = _both(inst, bl, bu, lb, ub, what="single %.2f/%d" % (scale, seed))
    assert r["attempts"] >= 1 or r["reason"] in (1, 2)


@pytest.mark.parametrize("scale,seed", [(0.02, 0), (0.02, 2), (0.05, 2)])
def test_rounding_with_repairs(scale, seed):
    """bp_round on the scaled single-instance workload with up to three
    repairs on a marked path, against the oracle's rounding with the same
    limits: counts, repairs and final box equal."""
    inst = gen.make("single", 0, scale=scale)
    r0, lb, ub = oracle.propagate(inst)
    rng = np.random.default_rng(seed)
    x = np.clip(inst["xstar"] + rng.normal(0.0, 0.4, inst["n"]), lb, ub)
    d = rng.random(2 * inst["n"])
    o = bp().default_options(repair_calls=3, repair_attempts=8, repair_shifts=64)
    I = bp().Instance(inst, o)
    tl, tu = dev(lb, torch.float64), dev(ub, torch.float64)
    r = I.round(tl, tu, dev(x, torch.float64), dev(d, torch.float64))
    torch.cuda.synchronize()
    ro, ol, ou = oracle.round_(inst, x, d, lb, ub, repair=(3, 8, 64))
    assert r == ro, (r, ro)
    assert np.array_equal(bits(tl.cpu().numpy()), bits(ol)) and np.array_equal(bits(tu.cpu().numpy()), bits(ou))


def test_errors_leave_the_box():
    inst = gen.make_micro(3)
    I = bp().Instance(inst)
    bl, bu = inst["lb"] - 1.0, inst["ub"].copy()
    tl, tu = dev(bl, torch.float64), dev(bu, torch.float64)
    l0, u0 = dev(inst["lb"], torch.float64), dev(inst["ub"], torch.float64)
    with pytest.raises(bp().BPError) as e:
        I.repair(tl, tu, l0, u0)
    assert e.value.code == bp().BP_EINVAL
    with pytest.raises(bp().BPError):
        I.repair(l0.clone(), u0.clone(), l0, u0, 64, 0)
    nan = inst["lb"].copy()
    nan[0] = np.nan
    with pytest.raises(bp().BPError):
        I.repair(dev(nan, torch.float64), u0.clone(), l0, u0)
    torch.cuda.synchronize()
    assert np.array_equal(tl.cpu().numpy(), bl)
