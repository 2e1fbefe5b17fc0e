"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.  Outcome, rounds, propagated nonzeros and evidence
must be identical, integer bounds bit-exact and continuous bounds within
1e-9 relative."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, both, bp, dev, gpu_propagate
from helpers import (case_mismatch, keep_rows, load_golden, load_golden_cases, row_instance,
                     slack_edge_instance, stack_instances)
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu
INF = math.inf


def _opts(**kw):
    return bp().default_options(**kw)


def _orc_opts(o):
    return oracle.Options(feastol=o.feastol, inttol=o.inttol, tau=o.tau, max_rounds=o.max_rounds)


@pytest.mark.parametrize("name", ["w1", "w2", "w3"])
@pytest.mark.parametrize("rounds", ["graph", "host"])
def test_golden_cold_and_second_call(name, rounds):
    inst, d = load_golden(name)
    flags = bp().FLAG_HOST_ROUNDS if rounds == "host" else 0
    I = bp().Instance(inst, _opts(flags=flags))
    rg, lg, ug = both(I, inst, what=name)
    assert rg["rounds"] == d["cold"]["rounds"]
    assert rg["nnz_propagated"] == d["cold"]["nnz_propagated"]
    assert list(lg) == [float(x) for x in d["cold"]["lb"]]
    assert list(ug) == [float(x) for x in d["cold"]["ub"]]
    r2, _, _ = both(I, inst, lg, ug, what=name + " second")
    assert r2["rounds"] == d["second_cold"]["rounds"]


@pytest.mark.parametrize("rounds", ["graph", "host"])
def test_golden_w7_crossing_evidence_and_signed_zeros(rounds):
    # Hand-computed crossing, evidence and signed-zero cases: the GPU gives
    # the fixture's result itself (bounds bit for bit) and the oracle's.
    flags = bp().FLAG_HOST_ROUNDS if rounds == "host" else 0
    for inst, c in load_golden_cases("w7"):
        I = bp().Instance(inst, _opts(flags=flags))
        rg, lg, ug = both(I, inst, what=c["name"])
        assert case_mismatch(c, rg, lg, ug) is None, case_mismatch(c, rg, lg, ug)


@pytest.mark.parametrize("seed", range(10))
def test_tiny(seed):
    inst = gen.make("tiny", seed)
    I = bp().Instance(inst)
    both(I, inst, what="tiny%d" % seed)


@pytest.mark.parametrize("seed", range(5))
def test_tiny_inf(seed):
    inst = gen.make("tiny_inf", seed)
    I = bp().Instance(inst)
    both(I, inst, what="tiny_inf%d" % seed)


@pytest.mark.parametrize("seed", range(40))
def test_micro_including_infeasible(seed):
    inst = gen.make_micro(seed)
    I = bp().Instance(inst)
    both(I, inst, what="micro%d" % seed)


@pytest.mark.parametrize("scale,seed", [(0.01, 0), (0.02, 1), (0.05, 2), (0.1, 0)])
def test_single_scaled(scale, seed):
    # Scaled-down single-instance workload: power-law rows plus dense rows
    # that exceed the heavy threshold at scale >= 0.1.
    inst = gen.make("single", seed, scale=scale)
    I = bp().Instance(inst)
    both(I, inst, what="single%g" % scale)


def test_single_heavy_paths_small_threshold():
    # A low heavy threshold sends the dense rows through the chunked path and
    # mid rows through the one-workgroup path.
    inst = gen.make("single", 3, scale=0.02)
    I = bp().Instance(inst, _opts(heavy_threshold=1024))
    both(I, inst, what="heavy1024")


def test_heavy_rows_many_chunks():
    # 256-nonzero chunks: the dense rows of the full single-instance workload
    # split into up to ~200 chunks, more than one partial per merging lane.
    inst = gen.make("single", 0, scale=0.5)
    I = bp().Instance(inst, _opts(heavy_chunk=256, heavy_threshold=2048))
    both(I, inst, what="chunks256")


def test_probe_workload_scaled():
    inst = gen.make("probe", 0, scale=0.004)
    I = bp().Instance(inst)
    both(I, inst, what="probe-scaled")


@pytest.mark.parametrize("name,scale", [("tiny", 1.0), ("single", 0.02)])
def test_force_exact_path(name, scale):
    # Every activity through the fixed-point accumulator: identical results.
    inst = gen.make(name, 0, scale=scale) if name != "tiny" else gen.make("tiny", 0)
    I = bp().Instance(inst, _opts(flags=bp().FLAG_FORCE_EXACT))
    both(I, inst, what="exact-" + name)


def test_cancellation_rows_take_exact_path():
    # Terms 2^106, 2^53, 1, -2^106, -2^53 sum to exactly 1; a double-double
    # accumulation loses the 1, so the certificate fails and the exact path
    # decides.  The bound of the last variable depends on that sum.
    n = 6
    vals = [2.0 ** 106, 2.0 ** 53, 1.0, -(2.0 ** 106), -(2.0 ** 53), 1.0]
    rows = [(list(range(n)), vals)]
    lb = [1.0, 1.0, 1.0, 1.0, 1.0, 0.0]
    ub = [1.0, 1.0, 1.0, 1.0, 1.0, 10.0]
    inst = gen.from_rows(n, rows, [-INF], [4.5], [1, 1, 1, 1, 1, 1], lb, ub)
    I = bp().Instance(inst)
    rg, lg, ug = both(I, inst, what="cancel")
    assert ug[5] == 3.0  # 4.5 - 1 = 3.5 -> floor 3


def test_warm_start_changed_list():
    inst = gen.make("single", 4, scale=0.02)
    I = bp().Instance(inst)
    r, lb, ub = both(I, inst, what="root")
    rng = np.random.default_rng(0)
    ints = np.nonzero((inst["vtype"] == 1) & (lb < ub))[0]
    pick = np.sort(rng.choice(ints, size=min(50, ints.size), replace=False))
    lb2, ub2 = lb.copy(), ub.copy()
    val = np.rint(rng.uniform(lb2[pick], ub2[pick]))
    lb2[pick] = val
    ub2[pick] = val
    both(I, inst, lb2, ub2, changed=pick.astype(np.int32), what="warm")
    # empty change list: nothing to do
    rg, _, _ = gpu_propagate(I, inst, lb, ub, changed=np.zeros(0, np.int32))
    assert rg["rounds"] == 0 and rg["status"] == 0


def test_round_limit_and_box_check():
    n = 30
    rows = [([i, i + 1], [1.0, -1.0]) for i in range(n - 1)]
    inst = gen.from_rows(n, rows, [-INF] * (n - 1), [-1.0] * (n - 1), [1] * n, [0.0] * n,
                         [100.0] * n)
    o = _opts(max_rounds=5)
    I = bp().Instance(inst, o)
    rg, lg, ug = gpu_propagate(I, inst)
    ro, lo, uo = oracle.propagate(inst, opts=_orc_opts(o))
    assert ro["status"] == oracle.BP_ROUND_LIMIT
    assert_same(inst, rg, lg, ug, ro, lo, uo, "round-limit")
    assert np.array_equal(lg, lo) and np.array_equal(ug, uo)
    I2 = bp().Instance(inst)
    both(I2, inst, what="chain")
    lb = inst["lb"].copy(); ub = inst["ub"].copy()
    lb[7] = 5.0; ub[7] = 4.0
    both(I2, inst, lb, ub, what="crossed box")


def test_empty_rows_and_instance():
    inst = gen.from_rows(1, [([], []), ([0], [2.0])], [-INF, -INF], [-1.0, 3.0], [1], [0], [5])
    I = bp().Instance(inst)
    both(I, inst, what="empty-row-infeasible")
    inst = gen.from_rows(3, [], [], [], [1, 0, 1], [0, 0, 0], [1, 1, 1])
    I = bp().Instance(inst)
    r, lg, ug = both(I, inst, what="no rows")
    assert r["rounds"] == 0


def test_with_given_csc_and_validation():
    inst = gen.make("tiny", 3)
    I = bp().Instance(inst, with_csc=True)
    both(I, inst, what="csc")
    bad = dict(inst)
    bad["val"] = inst["val"].copy()
    bad["val"][5] = 0.0
    with pytest.raises(bp().BPError) as e:
        bp().Instance(bad)
    assert e.value.code == bp().BP_EINVAL


def test_full_single_workload():
    """The single-instance workload at full size (m=100k, n=150k, ~1M nnz),
    cold start, in the configuration the benchmark times."""
    inst = gen.make("single", 0)
    I = bp().Instance(inst)
    both(I, inst, what="single-full")


def test_batch_matches_single_vectors():
    inst = gen.make("single", 5, scale=0.02)
    I = bp().Instance(inst)
    r, lb, ub = both(I, inst, what="root")
    LB, UB, changed = gen.bulk_fix_vectors(inst, lb, ub, count=6, frac=0.05, seed=1)
    ptr = np.zeros(len(changed) + 1, np.int64)
    ptr[1:] = np.cumsum([c.size for c in changed])
    idx = np.concatenate(changed).astype(np.int32)
    tl, tu = dev(LB, torch.float64), dev(UB, torch.float64)
    res = I.propagate_batch(tl, tu, dev(ptr, torch.int64), dev(idx, torch.int32))
    torch.cuda.synchronize()
    GL, GU = tl.cpu().numpy(), tu.cpu().numpy()
    for v in range(len(changed)):
        ro, lo, uo = oracle.propagate(inst, LB[v], UB[v], changed=changed[v])
        assert_same(inst, res[v], GL[v], GU[v], ro, lo, uo, "batch%d" % v)
    # cold batch
    tl, tu = dev(np.repeat(inst["lb"][None], 3, 0), torch.float64), dev(np.repeat(inst["ub"][None], 3, 0), torch.float64)
    res = I.propagate_batch(tl, tu)
    ro, lo, uo = oracle.propagate(inst)
    for v in range(3):
        assert_same(inst, res[v], tl[v].cpu().numpy(), tu[v].cpu().numpy(), ro, lo, uo, "coldbatch")


@pytest.mark.parametrize("seed", [0, 1])
def test_slack_filter_edges(seed):
    """Rows whose slack sits at the slack filter's threshold, and at the
    naive threshold max |a| (ub - lb) where some rows do tighten, in light,
    block and heavy rows: the rows the kernels skip and the rows they
    process must both give the oracle's result."""
    parts = [slack_edge_instance(seed, 300)[0],
             slack_edge_instance(seed + 10, 300, naive=True)[0],
             slack_edge_instance(seed + 20, 12, lengths=(1500, 6000))[0],
             slack_edge_instance(seed + 30, 12, naive=True, lengths=(1500, 6000))[0]]
    inst = stack_instances(parts)
    # rows that are infeasible on their own would end the run in its first
    # rounds; keep the others so that every bound is compared
    ok = [k for k in range(inst["m"]) if oracle.propagate(row_instance(inst, k))[0]["status"] == 0]
    inst = keep_rows(inst, ok)
    r0, lb0, ub0 = oracle.propagate(inst)
    assert r0["status"] == 0 and r0["rounds"] >= 2
    assert ((lb0 != inst["lb"]) | (ub0 != inst["ub"])).sum() >= 20  # some rows do tighten
    for thr in (2048, 8192):
        I = bp().Instance(inst, bp().default_options(heavy_threshold=thr, heavy_chunk=512))
        both(I, inst, what="slack-edge thr=%d" % thr)
