"""GPU-side helpers for the parity tests: run the HIP library through its
C ABI on seeded inputs and compare with the CPU oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from helpers import bits, rel_close

INT_FIELDS = ("status", "rounds", "nnz_propagated", "n_infeasible_rows", "infeasible_row",
              "infeasible_var")


def bp():
    from paper_2510_20499_amd import bp as _bp
    return _bp


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def gpu_propagate(I, inst, lb=None, ub=None, changed=None):
    lb = inst["lb"] if lb is None else lb
    ub = inst["ub"] if ub is None else ub
    tl = dev(lb, torch.float64)
    tu = dev(ub, torch.float64)
    ch = None if changed is None else dev(np.asarray(changed, np.int32), torch.int32)
    r = I.propagate(tl, tu, ch)
    torch.cuda.synchronize()
    return r, tl.cpu().numpy(), tu.cpu().numpy()


def assert_same(inst, rg, lg, ug, ro, lo, uo, what=""):
    """Parity rule: identical outcome, counters and evidence; integer bounds
    bit-exact; continuous bounds within 1e-9 relative (max(1,|x|) scale).
    Bounds are not compared after an infeasible outcome."""
    for f in INT_FIELDS:
        assert rg[f] == ro[f], (what, f, rg, ro)
    if ro["status"] == oracle.BP_INFEASIBLE:
        return
    integ = inst["vtype"] == 1
    # bit patterns, so that a stored -0.0 differs from +0.0
    assert np.array_equal(bits(lg[integ]), bits(lo[integ])), (what, "integer lb")
    assert np.array_equal(bits(ug[integ]), bits(uo[integ])), (what, "integer ub")
    assert rel_close(lg[~integ], lo[~integ]), (what, "continuous lb")
    assert rel_close(ug[~integ], uo[~integ]), (what, "continuous ub")
    for g, o in ((lg[~integ], lo[~integ]), (ug[~integ], uo[~integ])):
        z = o == 0.0
        assert np.array_equal(np.signbit(g[z]), np.signbit(o[z])), (what, "sign of a zero bound")


def gpu_base(I, lb, ub):
    """Make bounds the oracle computed the instance's base: a warm start
    with an empty change list propagates nothing and keeps them.  The
    stored base is read back and checked bit for bit, so both sides start
    from the same input."""
    tl = dev(lb, torch.float64)
    tu = dev(ub, torch.float64)
    r = I.propagate(tl, tu, torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert r["status"] == 0 and r["rounds"] == 0, r
    bl, bu = I.base()
    torch.cuda.synchronize()
    assert np.array_equal(bl.cpu().numpy().view(np.int64), np.asarray(lb, np.float64).view(np.int64))
    assert np.array_equal(bu.cpu().numpy().view(np.int64), np.asarray(ub, np.float64).view(np.int64))


def both(I, inst, lb=None, ub=None, changed=None, opts=None, what=""):
    rg, lg, ug = gpu_propagate(I, inst, lb, ub, changed)
    ro, lo, uo = oracle.propagate(inst, lb, ub, changed=changed, opts=opts)
    assert_same(inst, rg, lg, ug, ro, lo, uo, what)
    return rg, lg, ug
