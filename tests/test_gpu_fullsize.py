"""Parity at the full sizes of the measured workloads, in the launch
configurations the benchmark times: the probe workload (m=500k, n=1M, 8M
nonzeros; 4096 binaries probed together on 512 slots), the bulk workload
(m=2M, n=3M, 20M nonzeros; 256 fix-and-propagate vectors in one call on the
one-vector-per-lane engine) and the serving mix (64 resident instances, 2000
requests, slot pool sized by a 64 GiB budget).

The oracle computes every input both sides start from and, one by one, a
seeded sample of the outputs; the remaining outputs are checked through
properties that hold at any size (list order and bounds inside the base box
for probes, the first round's nonzero count for bulk vectors)."""
import math

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_same, bp, dev, gpu_base, gpu_propagate
from helpers import rel_close
from paper_2510_20499_amd import gen

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _probe_slice(G, p):
    a, b = int(G["off"][p]), int(G["off"][p + 1])
    return G["var"][a:b], G["lb"][a:b], G["ub"][a:b]


def test_probe_workload_full_size():
    _say("full size: probe workload, seed 0")
    inst = gen.make("probe", 0)
    n = inst["n"]
    ro, olb, oub = oracle.propagate(inst)
    assert ro["status"] == oracle.BP_OK
    I = bp().Instance(inst)
    # the cold root on the GPU, whole vectors compared
    rg, glb, gub = gpu_propagate(I, inst)
    assert_same(inst, rg, glb, gub, ro, olb, oub, "probe-workload root")
    gpu_base(I, olb, oub)
    vs = gen.pick_probe_vars(inst, olb, oub, 4096, seed=0)
    assert vs.size == 4096 and I.options.probe_slots == 512
    G = I.probe(dev(vs, torch.int32))
    torch.cuda.synchronize()
    G = {k: v.cpu().numpy() for k, v in G.items()}
    st, off = G["status"], G["off"]
    # properties of all 8192 probes
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == G["var"].size
    integ = inst["vtype"] == 1
    for p in range(2 * vs.size):
        v, l, u = _probe_slice(G, p)
        if st[p] == bp().BP_INFEASIBLE:
            assert v.size == 0, p
            continue
        assert np.all(np.diff(v) > 0), p
        assert np.all(l >= olb[v]) and np.all(u <= oub[v]) and np.all((l != olb[v]) | (u != oub[v])), p
        t, h = divmod(p, 2)
        assert vs[t] in v and l[v == vs[t]][0] == h and u[v == vs[t]][0] == h, p
        iv = integ[v]
        assert np.all(l[iv] == np.round(l[iv])) and np.all(u[iv] == np.round(u[iv])), p
    # sampled probes, one by one in the oracle: a seeded draw of 64
    # binaries, every binary with a probe found infeasible and the one with
    # the most rounds
    rng = np.random.default_rng(11)
    pick = set(rng.choice(vs.size, size=64, replace=False).tolist())
    pick |= set((np.nonzero(st == bp().BP_INFEASIBLE)[0] // 2).tolist())
    pick.add(int(np.argmax(G["rounds"]) // 2))
    pick = sorted(pick)
    O = oracle.probe(inst, olb, oub, vs[pick])
    for j, t in enumerate(pick):
        for h in (0, 1):
            p, q = 2 * t + h, 2 * j + h
            what = "probe var %d at %d" % (vs[t], h)
            assert st[p] == O["status"][q], what
            assert G["rounds"][p] == O["rounds"][q], what
            assert G["nnz"][p] == O["nnz"][q], what
            v, l, u = _probe_slice(G, p)
            a, b = int(O["off"][q]), int(O["off"][q + 1])
            assert np.array_equal(v, O["var"][a:b]), what
            iv = integ[v]
            assert np.array_equal(l[iv], O["lb"][a:b][iv]) and np.array_equal(u[iv], O["ub"][a:b][iv]), what
            assert rel_close(l[~iv], O["lb"][a:b][~iv]) and rel_close(u[~iv], O["ub"][a:b][~iv]), what
    # scores of all variables and the probe order of the unfixed integers
    # at the root, as the benchmark runs them
    S = I.scores(dev(olb, torch.float64), dev(oub, torch.float64))
    So = oracle.scores(inst, olb, oub)
    for f in ("nviol", "maxviol", "minunit", "slack_score"):
        g = S[f].cpu().numpy()
        assert np.array_equal(g.view(np.int64) if g.dtype == np.float64 else g,
                              So[f].view(np.int64) if So[f].dtype == np.float64 else So[f]), f
    un = np.nonzero(integ & (olb < oub))[0].astype(np.int32)
    order = I.probe_order(dev(un, torch.int32), dev(olb, torch.float64), dev(oub, torch.float64))
    assert np.array_equal(order.cpu().numpy(), oracle.probe_order(inst, un, olb, oub))
    assert n == 1000000


def _first_round_nnz(inst, rowid, changed):
    """Nonzeros of the rows holding a changed variable: what a warm start
    processes in its first round.  rowid[p] is the row of nonzero p."""
    mark = np.zeros(inst["n"], bool)
    mark[changed] = True
    rows = np.unique(rowid[mark[inst["col"]]])
    rp = inst["row_ptr"]
    return int((rp[rows + 1] - rp[rows]).sum())


def test_bulk_workload_full_size():
    _say("full size: bulk workload, seed 0")
    inst = gen.make("bulk", 0)
    n = inst["n"]
    # The base: three rounds of the cold root propagation (the full root
    # runs into the round limit; three rounds keep the oracle to seconds).
    oo = oracle.Options()
    oo.max_rounds = 3
    ro, olb, oub = oracle.propagate(inst, opts=oo)
    assert ro["status"] == oracle.BP_ROUND_LIMIT
    I3 = bp().Instance(inst, bp().default_options(max_rounds=3))
    rg, glb, gub = gpu_propagate(I3, inst)
    assert_same(inst, rg, glb, gub, ro, olb, oub, "bulk-workload three rounds")
    assert np.array_equal(glb, olb) and np.array_equal(gub, oub)
    del I3
    B = 256
    lists = gen.bulk_fix_lists(inst, olb, oub, B, frac=0.05, seed=0)
    ptr = np.zeros(B + 1, np.int64)
    ptr[1:] = np.cumsum([p.size for p, _ in lists])
    idx = np.concatenate([p for p, _ in lists])
    vals = np.concatenate([v for _, v in lists])
    I = bp().Instance(inst)
    gpu_base(I, olb, oub)  # the lanes read the vectors as overlays on it
    d = torch.device("cuda:0")
    LB = dev(olb, torch.float64).expand(B, -1).contiguous()
    UB = dev(oub, torch.float64).expand(B, -1).contiguous()
    flat = torch.tensor(np.repeat(np.arange(B), np.diff(ptr)) * n + idx, device=d)
    LB.view(-1)[flat] = dev(vals, torch.float64)
    UB.view(-1)[flat] = dev(vals, torch.float64)
    res = I.propagate_batch(LB, UB, dev(ptr, torch.int64), dev(idx, torch.int32))
    torch.cuda.synchronize()
    assert len(res) == B
    # every vector: outcome and evidence well formed; a vector that ends in
    # its first round propagated exactly the rows of its fixed variables
    rowid = np.repeat(np.arange(inst["m"], dtype=np.int32), np.diff(inst["row_ptr"]))
    for v in range(0, B, 8):
        r = res[v]
        assert r["status"] in (bp().BP_OK, bp().BP_INFEASIBLE, bp().BP_ROUND_LIMIT), r
        if r["status"] == bp().BP_INFEASIBLE:
            assert (0 <= r["infeasible_row"] < inst["m"]) or (0 <= r["infeasible_var"] < n), r
        if r["rounds"] == 1:
            assert r["nnz_propagated"] == _first_round_nnz(inst, rowid, lists[v][0]), v
    # sampled vectors, one by one in the oracle: every sixteenth and the last
    for v in list(range(0, B, 16)) + [B - 1]:
        p, val = lists[v]
        lb, ub = olb.copy(), oub.copy()
        lb[p] = val
        ub[p] = val
        rv, lv, uv = oracle.propagate(inst, lb, ub, changed=p)
        assert_same(inst, res[v], LB[v].cpu().numpy(), UB[v].cpu().numpy(), rv, lv, uv,
                    "bulk vector %d" % v)


def test_bulk_root_against_the_oracle_record():
    """The benchmark's bulk root: a cold propagation of the full bulk
    workload from its initial bounds, 1000 rounds (the round limit), against
    what the oracle computed once (tests/golden/bulk_root.json, written by
    make_bulk_root.py): outcome, rounds, propagated nonzeros and evidence
    equal; integer bounds bit for bit through their sha256; continuous
    bounds bit for bit through theirs, else a seeded sample of 4096 within
    1e-9 relative."""
    import hashlib
    import json
    import os
    _say("full size: bulk root against the oracle's record")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bulk_root.json")) as fh:
        rec = json.load(fh)

    def digest(lb, ub):
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(lb, dtype="<f8").tobytes())
        h.update(np.ascontiguousarray(ub, dtype="<f8").tobytes())
        return h.hexdigest()

    inst = gen.make("bulk", 0)
    assert digest(inst["lb"], inst["ub"]) == rec["input_sha256"], "generator output changed"
    assert int(inst["col"].size) == rec["nnz"]
    I = bp().Instance(inst)
    rg, glb, gub = gpu_propagate(I, inst)
    for f, v in rec["result"].items():
        assert rg[f] == v, (f, rg, rec["result"])
    integ = inst["vtype"] == 1
    assert digest(glb[integ], gub[integ]) == rec["integer_bounds_sha256"]
    if digest(glb[~integ], gub[~integ]) != rec["continuous_bounds_sha256"]:
        smp = rec["continuous_sample"]
        v = np.asarray(smp["var"])
        assert rel_close(glb[v], np.asarray(smp["lb"])) and rel_close(gub[v], np.asarray(smp["ub"]))


def test_serving_mix_full_size():
    _say("full size: serving mix, seed 0")
    insts = gen.make_serving(0, count=64, m_hi=1e6)
    rng = np.random.default_rng(5)
    small = [t for t, x in enumerate(insts) if x["m"] <= 100000]
    checked = set(rng.choice(small, size=6, replace=False).tolist())
    loaded, bases = [], []
    for t, inst in enumerate(insts):
        I = bp().Instance(inst)
        if t in checked:
            ro, lb, ub = oracle.propagate(inst)
            assert ro["status"] == oracle.BP_OK
            gpu_base(I, lb, ub)
        else:
            r, lb, ub = gpu_propagate(I, inst)
            assert r["status"] == bp().BP_OK
        loaded.append(I)
        bases.append((lb, ub))
    # the benchmark's request mix
    rr = np.random.default_rng(17)
    reqs = []
    for _ in range(2000):
        t = int(rr.integers(0, len(insts)))
        lb, ub = bases[t]
        bins = np.nonzero((insts[t]["vtype"] == 1) & (lb == 0) & (ub == 1))[0]
        if rr.uniform() < 0.5:
            k = max(1, int(round(0.01 * bins.size)))
            vs = np.sort(rr.choice(bins, size=min(k, bins.size), replace=False)).astype(np.int32)
            val = rr.integers(0, 2, size=vs.size).astype(np.float64)
            reqs.append((t, bp().REQ_PROPAGATE, vs, val))
        else:
            k = int(round(math.exp(rr.uniform(0, math.log(512)))))
            vs = np.sort(rr.choice(bins, size=min(k, bins.size), replace=False)).astype(np.int32)
            reqs.append((t, bp().REQ_PROBE, vs, None))
    S = bp().Server(loaded, 64 << 30, bp().default_options(rounds_per_launch=4))
    pools = S.info()["pools"]
    # classes by size, each with its own slot footprint, all at the slot cap
    assert len(pools) >= 2 and sum(p["instances"] for p in pools) == len(insts)
    assert all(p["slots"] == 512 for p in pools)
    sizes = [p["bytes_per_slot"] for p in pools]
    assert sizes == sorted(sizes) and sizes[-1] > 8 * sizes[0]
    ids = [S.submit(t, kind, vs, val, val) for t, kind, vs, val in reqs]
    guard = 0
    while S.run(4):
        guard += 1
        assert guard < 100000
    done = {c["id"] for c in S.poll(100000)}
    assert done == set(ids)
    sample = [j for j, r in enumerate(reqs) if r[0] in checked]
    sample = sorted(rng.choice(sample, size=min(40, len(sample)), replace=False).tolist())
    _say("serving: %d requests checked against the oracle" % len(sample))
    integ_of = [x["vtype"] == 1 for x in insts]
    for j in sample:
        t, kind, vs, val = reqs[j]
        inst, (lb, ub) = insts[t], bases[t]
        jobs = 2 * vs.size if kind == bp().REQ_PROBE else 1
        g = S.results(ids[j], jobs)
        if kind == bp().REQ_PROBE:
            O = oracle.probe(inst, lb, ub, vs)
            want = dict(status=O["status"], rounds=O["rounds"], nnz=O["nnz"], off=O["off"],
                        var=O["var"], lb=O["lb"], ub=O["ub"])
        else:
            nlb, nub = lb.copy(), ub.copy()
            nlb[vs] = np.maximum(lb[vs], val)
            nub[vs] = np.minimum(ub[vs], val)
            changed = vs[(nlb[vs] != lb[vs]) | (nub[vs] != ub[vs])]
            r, flb, fub = oracle.propagate(inst, nlb, nub, changed=changed)
            diff = np.nonzero((flb != lb) | (fub != ub))[0]
            if r["status"] == oracle.BP_INFEASIBLE:
                diff = diff[:0]
            want = dict(status=[r["status"]], rounds=[r["rounds"]], nnz=[r["nnz_propagated"]],
                        off=[0, diff.size], var=diff, lb=flb[diff], ub=fub[diff])
        what = "request %d (instance %d, kind %d)" % (j, t, kind)
        for f in ("status", "rounds", "nnz", "off", "var"):
            assert np.array_equal(np.asarray(g[f]), np.asarray(want[f])), (what, f)
        gv = np.asarray(g["var"], dtype=np.int64)
        iv = integ_of[t][gv] if gv.size else np.zeros(0, bool)
        gl, gu = np.asarray(g["lb"]), np.asarray(g["ub"])
        assert np.array_equal(gl[iv], np.asarray(want["lb"])[iv]), what
        assert np.array_equal(gu[iv], np.asarray(want["ub"])[iv]), what
        assert rel_close(gl[~iv], np.asarray(want["lb"])[~iv]), what
        assert rel_close(gu[~iv], np.asarray(want["ub"])[~iv]), what
    S.close()


@pytest.mark.parametrize("name", ["single", "bulk"])
def test_incremental_rows_over_long_runs(name):
    """The cold root of the full single-instance workload (79 rounds) and of
    the bulk workload (1000 rounds, the round limit): incremental heavy rows
    and the full recomputation (BP_FLAG_FULL_ROWS) give the same outcome,
    rounds and propagated nonzeros, and the same bounds bit for bit, after
    every correction of a long run."""
    _say("full size: incremental rows over a long run, %s" % name)
    inst = gen.make(name, 0)
    out = []
    for full in (False, True):
        o = bp().default_options()
        if full:
            o.flags |= bp().FLAG_FULL_ROWS
        I = bp().Instance(inst, o)
        out.append(gpu_propagate(I, inst))
        del I
    (ri, li, ui), (rf, lf, uf) = out
    assert ri == rf, (ri, rf)
    assert np.array_equal(li.view(np.int64), lf.view(np.int64))
    assert np.array_equal(ui.view(np.int64), uf.view(np.int64))
    if name == "single":
        ro, lo, uo = oracle.propagate(inst)
        assert_same(inst, ri, li, ui, ro, lo, uo, "single full, incremental")
