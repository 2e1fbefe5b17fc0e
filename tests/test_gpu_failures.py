"""Failure handling forced from the host: device allocations made to fail
one at a time (bp_debug_fail_alloc) unwind cleanly, leak nothing and leave
the caller's bounds untouched; queued serving requests can be cancelled or
expire.  Every kernel still runs to its normal end: the failures happen in
host code before launches."""
import time

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, bp, dev, gpu_propagate
from paper_2510_20499_amd import gen
from test_gpu_serving import _instances, _oracle_result, _requests, _same

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _disarm():
    bp().debug_fail_alloc(0)
    yield
    bp().debug_fail_alloc(0)


def _enomem(fn):
    """Run fn; True if it failed with BP_ENOMEM, False if it succeeded."""
    try:
        fn()
    except bp().BPError as e:
        assert e.code == bp().BP_ENOMEM, e
        assert "injected" in str(e), e
        return False
    return True


def _free_bytes():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_load_fails_at_every_allocation_without_leaking():
    inst = gen.make("single", 0, scale=0.5)
    opts = bp().default_options(heavy_threshold=2048)
    bp().Instance(inst, opts).close()  # first use of the runtime's own pools
    before = _free_bytes()
    failures = 0
    for k in range(1, 200):
        bp().debug_fail_alloc(k)
        held = []
        if _enomem(lambda: held.append(bp().Instance(inst, opts))):
            held[0].close()
            break
        failures += 1
    else:
        pytest.fail("bp_load never succeeded")
    bp().debug_fail_alloc(0)  # k was past the last allocation of the load
    assert failures >= 9  # CSR, CSC, sides, types, bins, base ...
    after = _free_bytes()
    assert before - after < 16 << 20, (before, after)
    # the library still works: a load and a cold propagation match the oracle
    I = bp().Instance(inst, opts)
    r, lb, ub = gpu_propagate(I, inst)
    ro, olb, oub = oracle.propagate(inst)
    assert_same(inst, r, lb, ub, ro, olb, oub, "after injected load failures")


def test_propagate_fails_cleanly_then_recovers():
    inst = gen.make("single", 1, scale=0.05)
    I = bp().Instance(inst, bp().default_options(heavy_threshold=1024))
    ro, olb, oub = oracle.propagate(inst)
    lb0, ub0 = inst["lb"].copy(), inst["ub"].copy()
    failures = 0
    for k in range(1, 400):
        tl, tu = dev(lb0, torch.float64), dev(ub0, torch.float64)
        bp().debug_fail_alloc(k)
        out = []
        ok = _enomem(lambda: out.append(I.propagate(tl, tu)))
        torch.cuda.synchronize()
        if ok:
            bp().debug_fail_alloc(0)
            assert_same(inst, out[0], tl.cpu().numpy(), tu.cpu().numpy(), ro, olb, oub,
                        "first propagation after %d injected failures" % failures)
            break
        failures += 1
        # the failed call left the caller's bounds as they were
        assert np.array_equal(tl.cpu().numpy(), lb0) and np.array_equal(tu.cpu().numpy(), ub0)
    else:
        pytest.fail("bp_propagate never succeeded")
    assert failures >= 10  # the engine's work buffers
    # a second call allocates nothing more and is unaffected by an armed hook
    bp().debug_fail_alloc(1)
    r, lb, ub = gpu_propagate(I, inst)
    assert_same(inst, r, lb, ub, ro, olb, oub, "warm engine")
    bp().debug_fail_alloc(0)


def test_batch_and_probe_fail_cleanly_then_recover():
    inst = gen.make("tiny", 3)
    I = bp().Instance(inst)
    r, lb, ub = gpu_propagate(I, inst)
    assert r["status"] == bp().BP_OK
    bins = np.nonzero((inst["vtype"] == 1) & (lb == 0) & (ub == 1))[0][:24].astype(np.int32)
    want = oracle.probe(inst, lb, ub, bins)
    vs = dev(bins, torch.int32)
    for k in range(1, 100):
        bp().debug_fail_alloc(k)
        out = []
        if _enomem(lambda: out.append(I.probe(vs))):
            break
    else:
        pytest.fail("bp_probe never succeeded")
    bp().debug_fail_alloc(0)
    got = {key: t.cpu().numpy() for key, t in out[0].items()}
    for f in ("status", "rounds", "nnz", "off", "var"):
        assert np.array_equal(got[f], want[f]), f
    # 64 vectors, one per lane: fix 8 binaries of each to the planted point
    B = 64
    rng = np.random.default_rng(5)
    LB = np.tile(lb, (B, 1))
    UB = np.tile(ub, (B, 1))
    for v in range(B):
        f = rng.choice(bins, size=8, replace=False)
        LB[v, f] = UB[v, f] = inst["xstar"][f]
    for k in range(1, 100):
        tl, tu = dev(LB, torch.float64), dev(UB, torch.float64)
        bp().debug_fail_alloc(k)
        res = []
        if _enomem(lambda: res.append(I.propagate_batch(tl, tu))):
            break
        assert np.array_equal(tl.cpu().numpy(), LB) and np.array_equal(tu.cpu().numpy(), UB)
    else:
        pytest.fail("bp_propagate_batch never succeeded")
    bp().debug_fail_alloc(0)
    gl, gu = tl.cpu().numpy(), tu.cpu().numpy()
    for v in range(0, B, 9):
        ro, olb, oub = oracle.propagate(inst, LB[v], UB[v])
        assert_same(inst, res[0][v], gl[v], gu[v], ro, olb, oub, "vector %d" % v)


def test_server_create_fails_cleanly():
    insts, loaded, bases = _instances()
    # every allocation of the server's pools (engine and job storage each)
    for k in range(1, 400):
        bp().debug_fail_alloc(k)
        held = []
        if _enomem(lambda: held.append(bp().Server(loaded, 1 << 28))):
            break
    else:
        pytest.fail("bp_server_create never succeeded")
    bp().debug_fail_alloc(0)
    S = held[0]
    reqs = _requests(insts, bases, 6, seed=11)
    ids = [S.submit(*q) for q in reqs]
    guard = 0
    while S.run(8) and guard < 10000:
        guard += 1
    done = {c["id"]: c for c in S.poll()}
    for rid, q in zip(ids, reqs):
        assert not done[rid]["cancelled"]
        got = S.results(rid, done[rid]["jobs"])
        _same(got, _oracle_result(insts[q[0]], bases[q[0]], q), insts[q[0]], "request %d" % rid)


def test_server_cancel_and_expire_queued_requests():
    insts, loaded, bases = _instances()
    S = bp().Server(loaded, 1 << 28)
    reqs = _requests(insts, bases, 10, seed=3)
    ids = [S.submit(*q) for q in reqs]
    cancelled = {ids[1], ids[4], ids[9]}
    for rid in sorted(cancelled):
        S.cancel(rid)
    with pytest.raises(bp().BPError) as e:
        S.cancel(ids[1])  # already finished (as cancelled)
    assert e.value.code == bp().BP_ESTATE
    with pytest.raises(bp().BPError) as e:
        S.cancel(10 ** 9)
    assert e.value.code == bp().BP_EINVAL
    guard = 0
    while S.run(8) and guard < 10000:
        guard += 1
    done = {c["id"]: c for c in S.poll()}
    assert set(done) == set(ids)
    for rid, q in zip(ids, reqs):
        if rid in cancelled:
            assert done[rid]["cancelled"]
            with pytest.raises(bp().BPError) as e:
                S.results(rid, done[rid]["jobs"])
            assert e.value.code == bp().BP_ECANCELED
        else:
            assert not done[rid]["cancelled"]
            got = S.results(rid, done[rid]["jobs"])
            _same(got, _oracle_result(insts[q[0]], bases[q[0]], q), insts[q[0]], "request %d" % rid)
            with pytest.raises(bp().BPError) as e:
                S.cancel(rid)
            assert e.value.code == bp().BP_ESTATE
    # queue timeout: requests that waited longer than the limit are cancelled
    old = [S.submit(*q) for q in reqs[:3]]
    time.sleep(0.05)
    new = [S.submit(*q) for q in reqs[3:5]]
    assert S.expire(20_000.0) == len(old)  # 20 ms
    guard = 0
    while S.run(8) and guard < 10000:
        guard += 1
    done = {c["id"]: c for c in S.poll()}
    assert all(done[r]["cancelled"] for r in old)
    for rid, q in zip(new, reqs[3:5]):
        assert not done[rid]["cancelled"]
        got = S.results(rid, done[rid]["jobs"])
        _same(got, _oracle_result(insts[q[0]], bases[q[0]], q), insts[q[0]], "late request %d" % rid)
