"""bp_scores_noalloc (the scores entry point that allocates no device
memory; its work buffers are a static device array) against bp_scores on
the same inputs: bit for bit, on two calls in a row, the second on a
smaller instance, so that anything the first call left in the shared array
would show.  Also: the size limit and the NaN check."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_util import bp, dev
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu

FIELDS = ("nviol", "maxviol", "minunit", "slack_score")


def _out(n, fill):
    return dict(nviol=torch.full((n,), -7, dtype=torch.int32, device="cuda"),
                maxviol=torch.full((n,), fill, dtype=torch.float64, device="cuda"),
                minunit=torch.full((n,), fill, dtype=torch.float64, device="cuda"),
                slack_score=torch.full((n,), fill, dtype=torch.float64, device="cuda"))


def _bits(t):
    a = t.cpu().numpy()
    return a if a.dtype == np.int32 else a.view(np.int64)


def _compare(inst, lb, ub, what):
    I = bp().Instance(inst)
    tl, tu = dev(lb, torch.float64), dev(ub, torch.float64)
    ref = I.scores(tl, tu, out=_out(inst["n"], -1.0))
    got = I.scores(tl, tu, out=_out(inst["n"], 12345.0), noalloc=True)
    torch.cuda.synchronize()
    for f in FIELDS:
        a, b = _bits(got[f]), _bits(ref[f])
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, (what, f, bad[:5])
    return I, ref


def test_noalloc_matches_bp_scores_twice_second_smaller():
    # first call: the single-instance workload at a third of its size, with
    # rows longer than 1024 nonzeros (chunked partial sums) and a box tightened
    # by a propagation, so that slacks and violations are non-trivial
    big = gen.make("single", 0, scale=0.3)
    I = bp().Instance(big)
    tl, tu = dev(big["lb"], torch.float64), dev(big["ub"], torch.float64)
    r = I.propagate(tl, tu)
    assert r["status"] == 0
    lb1, ub1 = tl.cpu().numpy(), tu.cpu().numpy()
    del I
    _, ref1 = _compare(big, lb1, ub1, "first (larger) instance")
    assert int((ref1["nviol"] > 0).sum()) > 0
    # second call, smaller instance: every output must come from this call
    small = gen.make("tiny", 3)
    _compare(small, small["lb"], small["ub"], "second (smaller) instance")
    # and a third on the first instance again at its initial bounds
    _compare(big, big["lb"], big["ub"], "first instance again, initial box")


def test_noalloc_rejects_an_instance_beyond_the_limit():
    limit = 64 << 20  # BP_SCORES_NOALLOC_MAX_BYTES
    n = limit // 16 + 1024  # packed bounds alone exceed the static array
    inst = gen.from_rows(n, [([0, n - 1], [1.0, 1.0])], [-np.inf], [1.0],
                         np.zeros(n, np.uint8), np.zeros(n), np.ones(n))
    I = bp().Instance(inst)
    tl, tu = dev(inst["lb"], torch.float64), dev(inst["ub"], torch.float64)
    out = _out(n, 3.5)
    with pytest.raises(bp().BPError) as e:
        I.scores(tl, tu, out=out, noalloc=True)
    assert e.value.code == bp().BP_EINVAL
    assert "static array" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out["maxviol"] == 3.5).all()) and bool((out["nviol"] == -7).all())
    # the allocating entry point still serves it
    ref = I.scores(tl, tu)
    torch.cuda.synchronize()
    assert int(ref["nviol"].sum()) == 0


def test_noalloc_rejects_nan_bounds():
    inst = gen.make("tiny", 1)
    I = bp().Instance(inst)
    lb = inst["lb"].copy()
    lb[5] = np.nan
    out = _out(inst["n"], 2.5)
    with pytest.raises(bp().BPError) as e:
        I.scores(dev(lb, torch.float64), dev(inst["ub"], torch.float64), out=out, noalloc=True)
    assert e.value.code == bp().BP_EINVAL
    torch.cuda.synchronize()
    assert bool((out["minunit"] == 2.5).all())
