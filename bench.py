"""Benchmark: bound propagation on the single-instance workload (one GPU).

A step is one cold propagation to the fixed point of the single-instance
workload (m=100k rows, n=150k variables, ~1M nonzeros, power-law rows plus
~20 dense rows of 10k-50k nonzeros), from the initial bounds, with the
changed-row worklist: every row in the first round, then only the rows of
variables whose bounds changed.  The instance and the initial bounds are
resident in device memory before the timed region; each step restores the
initial bounds with a device-to-device copy and calls bp_propagate.

Output: one JSON line with propagated nonzeros per second, the roofline of
the activity kernel (algorithmic bytes per launch over its HIP-event time,
with the measured HBM traffic when the kernel sources match) and the CPU
oracle timed on a bounded sample of the same workload.  The same line
carries the batched forms: double probing of 4096 binaries of the probe
workload, bulk fix-and-propagate of 256 vectors of the bulk workload, and
serving a Poisson request stream over 64 resident instances (p50/p99),
each against its one-at-a-time baseline on the same GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E datasheet peak


# HBM traffic per launch of the kernels the roofline records cover, from
# rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs (one counter per run;
# the commands are in profiles/), averaged over the named launches and scaled
# by what the same counters read for a 1 GiB device copy (FETCH_SIZE x2.0,
# WRITE_SIZE x1.0).  The figures belong to the library sources they were
# measured on (SOURCES_SHA256, see sources_sha256()): when any source
# differs, the bench line reports null.
SOURCES_SHA256 = "985df3f92fc5e8fe51e0824fd58dda8f099c01bfcdb958d13e696e7a43788c40"
TRAFFIC = {
    # single-instance workload, `bench.py --profile-steps 5`: 5 cold calls of
    # 79 working launches each (KiB per working launch)
    "plain k_rows": {"fetch_kib": 1851.30, "write_kib": 194.19, "fetch_scale": 2.0, "write_scale": 1.0},
    "plain k_apply": {"fetch_kib": 403.82, "write_kib": 179.62, "fetch_scale": 2.0, "write_scale": 1.0},
    # probe workload, `bench.py --only-probe --profile-probe 3`: 4 batched
    # calls of 8192 probes on 2048 slots, 15 working launches each
    "probe k_rows": {"fetch_kib": 15505.34, "write_kib": 343.61, "fetch_scale": 2.0, "write_scale": 1.0,
                     "schedule": {"heavy_threshold": 8192, "heavy_chunk": 4096, "probe_slots": 2048}},
    # bulk workload, `bench.py --only-bulk --profile-bulk 2 --bulk-schedule
    # G,16`: 3 calls of 256 vectors, one working launch each; one record per
    # lane-engine grid G the tuner chooses between
    "bulk k_lv_rows": [
        {"fetch_kib": 21053940.33, "write_kib": 463640.53, "fetch_scale": 2.0, "write_scale": 1.0,
         "schedule": {"lv_grid": 4096}},
        {"fetch_kib": 21028913.88, "write_kib": 470956.22, "fetch_scale": 2.0, "write_scale": 1.0,
         "schedule": {"lv_grid": 8192}},
    ],
}


def sources_sha256():
    """sha256 over the library's kernel sources and build script, in name
    order: what the traffic records were measured on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2510_20499_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "paper_2510_20499_amd", "build.py"))
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(hashlib.sha256(fh.read()).digest())
    return h.hexdigest()


def measured_traffic(key, schedule=None):
    """HBM bytes per launch for TRAFFIC[key], or None when there is no
    record, the sources changed since the counters were taken, or the
    record names a schedule (the tuned knobs that change the kernel's work)
    that `schedule` does not match.  A key may hold one record per
    schedule."""
    recs = TRAFFIC.get(key)
    if recs is None or SOURCES_SHA256 is None or sources_sha256() != SOURCES_SHA256:
        return None
    for t in recs if isinstance(recs, list) else [recs]:
        if all(schedule is not None and schedule.get(k) == v for k, v in t.get("schedule", {}).items()):
            return int((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024)
    return None


def log(msg):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(msg, file=sys.stderr, flush=True)


METRIC = "propagated nnz/s (batched vs plain) + HBM GB/s; p50/p99 probe latency"

# Oracle threads of the all-cores CPU baselines: the host's cores, at most
# the 16 a one-GPU share of the machine holds.
CPU_POOL_MAX = 16


def inst_sha256(inst):
    """sha256 of an instance's arrays (row pointers, columns, coefficients,
    sides, types, bounds), as generated: what the record was measured on
    (the digest the instance files' manifests carry)."""
    from paper_2510_20499_amd import gen
    return gen.digest(inst)


def cpu_info():
    """Host CPU model and logical core count (recorded with every CPU leg)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def oracle_pool(fn, items):
    """Run fn over items on a pool of threads, each calling the unchanged
    single-threaded oracle (its C calls release the interpreter lock).
    Returns (results, wall seconds, threads)."""
    from concurrent.futures import ThreadPoolExecutor
    threads = max(1, min(CPU_POOL_MAX, os.cpu_count() or 1, len(items)))
    t = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        out = list(ex.map(fn, items))
    return out, time.perf_counter() - t, threads


def fresh(*ts):
    """Clones of device tensors (a call's in/out bounds)."""
    return tuple(t.clone() for t in ts)


def kernel_roofline(bp, inst, call, reps=5, kernel="k_rows", **opt):
    """Roofline of the activity kernel (k_rows, or k_lv_rows for batches of
    one vector per lane) for one call `call(I)`.

    Time: HIP events recorded around each k_rows launch (rounds driven from
    the host so every launch is bracketed), averaged over `reps` calls.
    Bytes: what the method must move per launch -- 12 B per nonzero (int32
    column + f64 coefficient), 24 B per row (row pointer + two sides), 16 B
    per distinct bound record read -- counted by an instrumented run of the
    same call and divided by the launches per call.  A queued heavy row
    tested from its incremental accumulators costs their 2 x 68 limbs
    (1088 B) instead, and its nonzeros count only when its candidates had
    to read them."""
    Ic = bp.Instance(inst, bp.default_options(flags=bp.FLAG_COUNT_VARS, **opt))
    call(Ic)
    cs = Ic.kernel_stats(reset=True)
    del Ic
    It = bp.Instance(inst, bp.default_options(flags=bp.FLAG_TIME_KERNELS, **opt))
    call(It)  # warm
    It.kernel_stats(reset=True)
    for _ in range(reps):
        call(It)
    ts = It.kernel_stats(reset=True)
    del It
    launches = ts["launches"] / reps
    alg_bytes_per_call = (12 * (cs["nnz"] - cs["nnz_kept"]) + 24 * cs["rows"] + 16 * cs["vars_read"]
                          + 1088 * cs["rows_kept"])
    bytes_per_launch = alg_bytes_per_call / max(launches, 1)
    avg_launch_ms = ts["ms"] / max(ts["launches"], 1)
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": None,
           "kernel": kernel, "avg_launch_us": round(avg_launch_ms * 1e3, 3),
           "launches_per_call": launches, "alg_bytes_per_launch": int(bytes_per_launch)}
    if ts.get("apply_ms", 0.0) > 0.0:
        # k_apply: per changed-list entry 73 B (entry, candidate keys read and
        # reset, bound record, column pointers, type), 16 B per accepted bound
        # written, 25 B per column entry walked (row id, row pointers, bin,
        # row flag), 8 B per queued row, 56 B per heavy-row correction
        # (coefficient and limb updates)
        ab = (73 * cs["apply_entries"] + 16 * cs["vars_written"] + 25 * cs["apply_colent"]
              + 8 * cs["rows"] + 56 * cs["apply_corr"]) / max(launches, 1)
        a_ms = ts["apply_ms"] / max(ts["launches"], 1)
        a_ach = ab / (a_ms * 1e-3) / 1e9
        out["apply"] = {"bound": "hbm", "achieved": round(a_ach, 2), "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": round(a_ach / HBM_PEAK_GBPS, 5), "traffic": None,
                        "kernel": "k_apply", "avg_launch_us": round(a_ms * 1e3, 3),
                        "launches_per_call": launches, "alg_bytes_per_launch": int(ab)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many plain steps (for profilers) and exit")
    ap.add_argument("--skip-probe", action="store_true",
                    help="skip the batched double-probing measurement")
    ap.add_argument("--probe-vars", type=int, default=4096)
    ap.add_argument("--probe-schedule", default="8192,4096,32,2048",
                    help="heavy_threshold,heavy_chunk,rounds_per_launch,probe_slots of the probe leg "
                         "(the schedule bp_autotune chooses on this workload); empty: tune it")
    ap.add_argument("--probe-plain", type=int, default=256,
                    help="binaries probed one call at a time for the plain baseline")
    ap.add_argument("--skip-serving", action="store_true",
                    help="skip the serving measurement (64-instance mix, Poisson requests)")
    ap.add_argument("--only-serving", action="store_true")
    ap.add_argument("--serve-instances", type=int, default=64)
    ap.add_argument("--serve-mmax", type=float, default=1e6)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-rounds", type=int, default=4,
                    help="rounds per server step between admissions")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only copy a device buffer of this many MiB 5 times (a kernel of "
                         "known traffic, for scaling hardware byte counters) and exit")
    ap.add_argument("--skip-bulk", action="store_true",
                    help="skip the bulk-rounding (fix-and-propagate batch) measurement")
    ap.add_argument("--only-bulk", action="store_true")
    ap.add_argument("--bulk-vectors", type=int, default=256)
    ap.add_argument("--bulk-steps", type=int, default=3)
    ap.add_argument("--bulk-plain", type=int, default=16,
                    help="vectors propagated one call at a time for the plain baseline")
    ap.add_argument("--profile-probe", type=int, default=0,
                    help="only the probe leg's root and this many batched calls (counter runs)")
    ap.add_argument("--bulk-schedule", default="",
                    help="lv_grid,rounds_per_launch for --profile-bulk (the tuned schedule)")
    ap.add_argument("--profile-bulk", type=int, default=0,
                    help="run only this many batched bulk calls (no tuning, no baselines; "
                         "for profilers) and exit")
    ap.add_argument("--only-probe", action="store_true",
                    help="run only the double-probing measurement (for profilers)")
    ap.add_argument("--probe-cpu", type=int, default=16,
                    help="binaries the oracle probes for a CPU probing rate (0: skip)")
    ap.add_argument("--skip-tiny", action="store_true",
                    help="skip the Tiny workload (propagation and double probing of 150 binaries)")
    ap.add_argument("--bulk-light", type=float, default=0.002,
                    help="fraction of the unfixed integers each vector of the multi-round bulk leg "
                         "fixes (0: skip that leg)")
    ap.add_argument("--bulk-fp-rounds", type=int, default=5000,
                    help="round limit of the fixed-point root of the multi-round bulk leg")
    ap.add_argument("--bulk-cpu", type=int, default=8,
                    help="bulk vectors the oracle propagates one thread for the CPU baseline (0: skip)")
    ap.add_argument("--skip-round", action="store_true",
                    help="skip the bound-propagation rounding measurement")
    ap.add_argument("--only-round", action="store_true")
    ap.add_argument("--only-tiny", action="store_true")
    ap.add_argument("--round-reps", type=int, default=2)
    ap.add_argument("--round-cpu-scale", type=float, default=0.2,
                    help="scale of the single-instance workload the oracle rounds for the "
                         "CPU baseline (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_20499_amd import bp, gen

    if args.only_probe:
        print(json.dumps({"probe_batched": bench_probe(args, bp, gen, torch, np)}), flush=True)
        return
    if args.only_tiny:
        print(json.dumps({"tiny": bench_tiny(args, bp, gen, torch, np)}), flush=True)
        return
    if args.only_round:
        print(json.dumps({"rounding": bench_round(args, bp, gen, torch, np)}), flush=True)
        return
    if args.copy_calibrate:
        nb = args.copy_calibrate << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb, "copies": 5}), flush=True)
        return
    if args.only_bulk:
        print(json.dumps({"bulk_batched": bench_bulk(args, bp, gen, torch, np)}), flush=True)
        return
    if args.only_serving:
        print(json.dumps({"serving": bench_serving(args, bp, gen, torch, np)}), flush=True)
        return

    dev = torch.device("cuda:0")
    inst = gen.make("single", args.seed)
    m, n, nnz = inst["m"], inst["n"], int(inst["row_ptr"][-1])
    I = bp.Instance(inst)
    lb0 = torch.tensor(inst["lb"], dtype=torch.float64, device=dev)
    ub0 = torch.tensor(inst["ub"], dtype=torch.float64, device=dev)
    lb = torch.empty_like(lb0)
    ub = torch.empty_like(ub0)

    def step():
        lb.copy_(lb0)
        ub.copy_(ub0)
        return I.propagate(lb, ub)

    if args.profile_steps:
        for _ in range(args.profile_steps):
            r = step()
        torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "result": r}), flush=True)
        return

    for _ in range(args.warmup):
        r0 = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_nnz = 0
    for _ in range(args.steps):
        r = step()
        total_nnz += r["nnz_propagated"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert r["status"] == bp.BP_OK and r == r0
    value = total_nnz / dt

    roofline = kernel_roofline(bp, inst, lambda J: J.propagate(*fresh(lb0, ub0)))
    roofline["traffic"] = measured_traffic("plain k_rows")
    other = roofline.pop("apply", None)
    if other is not None:
        other["traffic"] = measured_traffic("plain k_apply")
        # the roofline is the kernel with the larger share of a call
        if other["avg_launch_us"] > roofline["avg_launch_us"]:
            roofline, other = other, roofline

    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        import oracle
        reps_cpu = 0
        t_cpu = 0.0
        nnz_cpu = 0
        while reps_cpu < 1 or (t_cpu < 10.0 and reps_cpu < 5):
            tc = time.perf_counter()
            ro, _, _ = oracle.propagate(inst)
            t_cpu += time.perf_counter() - tc
            nnz_cpu += ro["nnz_propagated"]
            reps_cpu += 1
        assert ro["nnz_propagated"] == r["nnz_propagated"] and ro["rounds"] == r["rounds"]
        cpu = {"value": nnz_cpu / t_cpu, "unit": "nnz/s", "cores": 1, "kind": "oracle",
               "sample": "%d cold propagation(s) of the full single-instance workload, "
                         "worklist mode, one thread" % reps_cpu, "host": cpu_info()}
        outs, wall, thr = oracle_pool(lambda _: oracle.propagate(inst)[0]["nnz_propagated"],
                                      list(range(min(CPU_POOL_MAX, os.cpu_count() or 1))))
        cpu_all = {"value": sum(outs) / wall, "unit": "nnz/s", "cores": thr, "kind": "oracle",
                   "sample": "%d independent cold propagations of the full single-instance "
                             "workload, one per thread, unchanged single-threaded oracle" % len(outs),
                   "host": cpu_info()}
        log("cpu: one thread %.3g nnz/s, %d threads %.3g nnz/s" % (cpu["value"], thr, cpu_all["value"]))

    tiny = None if args.skip_tiny else bench_tiny(args, bp, gen, torch, np)
    rounding = None if args.skip_round else bench_round(args, bp, gen, torch, np, inst=inst, I=I)
    probe = None if args.skip_probe else bench_probe(args, bp, gen, torch, np)
    bulk = None if args.skip_bulk else bench_bulk(args, bp, gen, torch, np)
    serving = None if args.skip_serving else bench_serving(args, bp, gen, torch, np)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator standing in for MIPLIB2017)",
        "config": {"workload": "single-instance plain propagation: m=%d, n=%d, nnz=%d, cold start "
                               "to fixed point with changed-row worklist" % (m, n, nnz),
                   "m": m, "n": n, "nnz": nnz, "seed": args.seed, "sha256": inst_sha256(inst),
                   "rounds": r["rounds"], "nnz_propagated_per_step": r["nnz_propagated"],
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "roofline_other": other,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "batched_vs_plain": {
            "probe": None if probe is None else {
                k: probe[k] for k in ("batched_nnz_per_s", "plain_nnz_per_s", "batched_probes_per_s",
                                      "plain_probes_per_s", "batched_over_plain")},
            "bulk": None if bulk is None else {
                k: bulk[k] for k in ("batched_nnz_per_s", "plain_nnz_per_s", "batched_vectors_per_s",
                                     "plain_vectors_per_s", "batched_over_plain")},
            "serving": None if serving is None else {
                k: serving[k] for k in ("saturated_requests_per_s", "throughput_over_fifo")},
        },
        "tiny": tiny,
        "rounding": rounding,
        "probe_batched": probe,
        "bulk_batched": bulk,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


def bench_tiny(args, bp, gen, torch, np):
    """The Tiny workload (m=200, n=300: 150 binaries, 100 integers in
    [0, 10], 50 continuous; 4-6 nonzeros per row, integer coefficients),
    seeds 0-9: a cold propagation to the fixed point, then double probing of
    all 150 binaries around it, with the instance resident.  Latency-bound:
    reported as time per instance and rounds, beside the oracle doing the
    same on one thread."""
    dev = torch.device("cuda:0")
    seeds = list(range(10))
    gpu_ms, rounds, nnz, probes, tuned = [], [], 0, 0, []
    insts = [gen.make("tiny", s) for s in seeds]
    for inst in insts:
        I = bp.Instance(inst)
        lb0 = torch.tensor(inst["lb"], dtype=torch.float64, device=dev)
        ub0 = torch.tensor(inst["ub"], dtype=torch.float64, device=dev)
        binv = np.nonzero((inst["vtype"] == 1) & (inst["lb"] == 0) & (inst["ub"] == 1))[0].astype(np.int32)
        bins = torch.tensor(binv, dtype=torch.int32, device=dev)
        # the schedule (rounds per graph, probe slots) tuned on this
        # instance's own propagation and probe, before timing
        t = I.autotune(*fresh(lb0, ub0), bins)
        tuned.append({k: t[k] for k in ("rounds_per_launch", "probe_slots")})

        def call():
            lb, ub = fresh(lb0, ub0)
            r = I.propagate(lb, ub)
            G = I.probe(bins)
            torch.cuda.synchronize()
            return r, G

        call()  # warm
        t = time.perf_counter()
        reps = 20
        for _ in range(reps):
            r, G = call()
        gpu_ms.append((time.perf_counter() - t) / reps * 1e3)
        rounds.append(r["rounds"])
        nnz += r["nnz_propagated"] + int(G["nnz"].sum().item())
        probes += 2 * binv.size
        del I
    res = {"workload": "tiny: m=200, n=300 (150 binaries), seeds 0-9; cold propagation to the "
                       "fixed point, then double probing of all 150 binaries",
           "ms_per_instance_median": float(np.median(gpu_ms)),
           "ms_per_instance": [round(x, 4) for x in gpu_ms],
           "rounds": rounds, "probes_per_instance": probes // len(seeds), "schedules": tuned,
           "nnz_per_s": nnz / (sum(gpu_ms) * 1e-3)}
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        for inst in insts:
            ro, lo, uo = oracle.propagate(inst)
            binv = np.nonzero((inst["vtype"] == 1) & (inst["lb"] == 0) & (inst["ub"] == 1))[0]
            oracle.probe(inst, lo, uo, binv.astype(np.int32))
        tc = (time.perf_counter() - t) / len(insts)
        res["cpu_baseline"] = {"value": tc * 1e3, "unit": "ms per instance", "cores": 1,
                               "kind": "oracle", "sample": "the same ten instances, one thread",
                               "host": cpu_info()}
    log("tiny: %.3f ms per instance (median), oracle %s ms"
        % (res["ms_per_instance_median"], res.get("cpu_baseline", {}).get("value")))
    return res


def _round_inputs(inst, lb, ub, seed, np):
    """Seeded fractional point (the planted point plus N(0, 0.4) noise,
    clipped into the root box; no LP relaxation is solved here) and draws."""
    rng = np.random.default_rng(seed + 77)
    x = np.clip(inst["xstar"] + rng.normal(0.0, 0.4, inst["n"]), lb, ub)
    return x, rng.random(2 * inst["n"])


def bench_round(args, bp, gen, torch, np, inst=None, I=None):
    """Bound-propagation rounding (bp_round: Algorithm 1 without repair and
    LP polish) of every integer variable of the single-instance workload from
    its root fixed point, with a probing cache of 1024 binaries chosen by
    bp_probe_order.  CPU baseline: the oracle's rounding of the same kind of
    input on the workload scaled by --round-cpu-scale, timed beside the GPU
    on that same scaled input."""
    dev = torch.device("cuda:0")
    if inst is None:
        inst = gen.make("single", args.seed)
        I = bp.Instance(inst)

    def setup(inst, I, kc):
        lb = torch.tensor(inst["lb"], dtype=torch.float64, device=dev)
        ub = torch.tensor(inst["ub"], dtype=torch.float64, device=dev)
        assert I.propagate(lb, ub)["status"] == bp.BP_OK
        x, d = _round_inputs(inst, lb.cpu().numpy(), ub.cpu().numpy(), args.seed, np)
        xd = torch.tensor(x, dtype=torch.float64, device=dev)
        dd = torch.tensor(d, dtype=torch.float64, device=dev)
        cache = None
        if kc:
            lbh, ubh = lb.cpu().numpy(), ub.cpu().numpy()
            bins = np.nonzero((inst["vtype"] == 1) & (lbh == 0) & (ubh == 1))[0].astype(np.int32)
            order = I.probe_order(torch.tensor(bins, device=dev), lb, ub)
            pv = order[:min(kc, bins.size)].contiguous()
            G = I.probe(pv)
            cache = dict(vars=pv, status=G["status"], off=G["off"], var=G["var"], lb=G["lb"],
                         ub=G["ub"])
        return lb, ub, xd, dd, cache

    lb0, ub0, xd, dd, cache = setup(inst, I, 1024)
    lb, ub = lb0.clone(), ub0.clone()
    R = I.round(lb, ub, xd, dd, cache)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.round_reps):
        lb.copy_(lb0)
        ub.copy_(ub0)
        R = I.round(lb, ub, xd, dd, cache)
    torch.cuda.synchronize()
    tr = (time.perf_counter() - t0) / args.round_reps
    res = {"workload": "rounding of the %d integer variables of the single-instance workload "
                       "(m=%d, n=%d) from its root fixed point; cache of %d binaries"
                       % (int((inst["vtype"] == 1).sum()), inst["m"], inst["n"],
                          0 if cache is None else cache["vars"].numel()),
           "round_ms": tr * 1e3, "result": R,
           "nnz_propagated_per_s": R["nnz_propagated"] / tr,
           "steps_per_s": R["iterations"] / tr}
    log("rounding: %.1f ms per call, %d steps (%d bulk), status %d"
        % (tr * 1e3, R["iterations"], R["bulks"], R["status"]))
    if args.round_cpu_scale > 0:
        import oracle
        small = gen.make("single", args.seed, scale=args.round_cpu_scale)
        Is = bp.Instance(small)
        slb, sub, sx, sd, _ = setup(small, Is, 0)
        l2, u2 = slb.clone(), sub.clone()
        Is.round(l2, u2, sx, sd)
        torch.cuda.synchronize()
        l2.copy_(slb)
        u2.copy_(sub)
        tg = time.perf_counter()
        Rg = Is.round(l2, u2, sx, sd)
        torch.cuda.synchronize()
        tg = time.perf_counter() - tg
        _, olb, oub = oracle.propagate(small)
        tc = time.perf_counter()
        Ro, _, _ = oracle.round_(small, sx.cpu().numpy(), sd.cpu().numpy(), olb, oub)
        tc = time.perf_counter() - tc
        assert Ro == Rg, (Ro, Rg)
        res["cpu_baseline"] = {"value": tc * 1e3, "unit": "ms per rounding call", "cores": 1,
                               "kind": "oracle", "gpu_ms_same_input": tg * 1e3,
                               "sample": "one rounding of the single-instance workload scaled by "
                                         "%g (n=%d), no cache, one thread; the GPU result on that "
                                         "input is identical" % (args.round_cpu_scale, small["n"])}
    return res


def bench_probe(args, bp, gen, torch, np):
    """Double probing on the probe workload (m=500k, n=1M, ~8M nnz, 70%
    binaries, set-cover and big-M rows): a seeded sample of unfixed binaries
    of the root fixed point, each probed at 0 and 1.  Plain: one bp_probe
    call per binary (k = 1).  Batched: one call for all of them, slots
    refilled at round boundaries."""
    dev = torch.device("cuda:0")
    inst = gen.make("probe", args.seed)
    sched = None
    if args.probe_schedule:  # the given schedule
        ht, hc, rk, ps = (int(x) for x in args.probe_schedule.split(","))
        sched = dict(heavy_threshold=ht, heavy_chunk=hc, rounds_per_launch=rk, probe_slots=ps)
    I = bp.Instance(inst, bp.default_options(**(sched or {})))
    lb0 = torch.tensor(inst["lb"], dtype=torch.float64, device=dev)
    ub0 = torch.tensor(inst["ub"], dtype=torch.float64, device=dev)
    lb, ub = fresh(lb0, ub0)
    root = I.propagate(lb, ub)
    assert root["status"] == bp.BP_OK
    vs = gen.pick_probe_vars(inst, lb.cpu().numpy(), ub.cpu().numpy(), args.probe_vars, seed=args.seed)
    k = int(vs.size)
    vars_d = torch.tensor(vs, dtype=torch.int32, device=dev)
    if sched is None and not args.profile_probe:
        # --probe-schedule "": the schedule (row split, rounds per graph,
        # probe slots) tuned on this instance's cold propagation and on these
        # probes, before timing; the tuner leaves the base at the root
        t = I.autotune(*fresh(lb0, ub0), vars_d)
        sched = {key: t[key] for key in ("heavy_threshold", "heavy_chunk", "rounds_per_launch", "probe_slots")}
        log("probe: tuned schedule %s (%d trials)" % (sched, t["trials"]))
    # batched
    G = I.probe(vars_d)  # warm (sizes the output buffers)
    cap = int(G["off"][-1].item()) + 16
    torch.cuda.synchronize()
    if args.profile_probe:
        # counter runs: only batched calls after the root
        for _ in range(args.profile_probe):
            G = I.probe(vars_d, cap=cap)
        torch.cuda.synchronize()
        return {"profile_probe": args.profile_probe, "nnz_per_call": int(G["nnz"].sum().item())}
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        G = I.probe(vars_d, cap=cap)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    nnz_b = int(G["nnz"].sum().item())
    rounds = G["rounds"].cpu().numpy()
    # plain: one binary per call, on an instance with the default schedule
    # (the batch's tuned graphs of many rounds would only slow calls of a
    # round or two)
    kp = min(args.probe_plain, k)
    Ip = bp.Instance(inst)
    lp, up = fresh(lb0, ub0)
    assert Ip.propagate(lp, up)["status"] == bp.BP_OK
    Ip.probe(vars_d[:1], cap=cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nnz_p = 0
    for t in range(kp):
        Gp = Ip.probe(vars_d[t:t + 1], cap=cap)
        nnz_p += int(Gp["nnz"].sum().item())
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    del Ip
    res = {
        "workload": "double probing: m=%d, n=%d, nnz=%d; %d binaries x {0,1} = %d bound vectors"
                    % (inst["m"], inst["n"], int(inst["row_ptr"][-1]), k, 2 * k),
        "sha256": inst_sha256(inst),
        "batched_probes_per_s": 2 * k / tb,
        "batched_nnz_per_s": nnz_b / tb,
        "batched_ms": tb * 1e3,
        "plain_probes_per_s": 2 * kp / tp,
        "plain_nnz_per_s": nnz_p / tp,
        "batched_over_plain": (2 * k / tb) / (2 * kp / tp),
        "probe_slots": int(sched["probe_slots"] if sched else I.options.probe_slots),
        "schedule": sched,
        "rounds_mean": float(rounds.mean()), "rounds_max": int(rounds.max()),
        "nnz_per_probe_mean": nnz_b / (2 * k),
        "implied_entries": int(G["off"][-1].item()),
        "infeasible_probes": int((G["status"] == bp.BP_INFEASIBLE).sum().item()),
    }
    res["roofline"] = probe_roofline(bp, inst, lb, ub, vars_d, cap, tb, torch, sched)
    res["roofline"]["traffic"] = measured_traffic("probe k_rows", sched)
    log("probe: batched %.2f ms, k_rows %.1f GB/s (%.4f of peak), call %.1f GB/s"
        % (tb * 1e3, res["roofline"]["achieved"], res["roofline"]["frac"],
           res["roofline"]["call_alg_GBps"]))
    res["scores"] = bench_scores(args, bp, inst, I, lb, ub, torch, np)
    if args.probe_cpu:
        import oracle
        _, olb, oub = oracle.propagate(inst)
        kc = min(args.probe_cpu, k)
        tc = time.perf_counter()
        O = oracle.probe(inst, olb, oub, vs[:kc])
        tc = time.perf_counter() - tc
        res["cpu_baseline"] = {"value": 2 * kc / tc, "unit": "probes/s", "cores": 1,
                               "kind": "oracle", "nnz_per_s": float(O["nnz"].sum()) / tc,
                               "sample": "%d binaries x {0,1} of the same sample, around the "
                                         "oracle's own root fixed point, one thread" % kc,
                               "host": cpu_info()}
        per = args.probe_cpu
        chunks = [vs[kc + j * per: kc + (j + 1) * per] for j in range(min(CPU_POOL_MAX, os.cpu_count() or 1))]
        chunks = [c for c in chunks if c.size]
        outs, wall, thr = oracle_pool(lambda c: float(oracle.probe(inst, olb, oub, c)["nnz"].sum()), chunks)
        nb = sum(c.size for c in chunks)
        res["cpu_baseline_all_cores"] = {
            "value": 2 * nb / wall, "unit": "probes/s", "cores": thr, "kind": "oracle",
            "nnz_per_s": sum(outs) / wall,
            "sample": "%d further binaries x {0,1} of the same sample, %d per thread, unchanged "
                      "single-threaded oracle" % (nb, per), "host": cpu_info()}
    return res


def probe_roofline(bp, inst, lb, ub, vars_d, cap, t_call, torch, sched=None):
    """Roofline of the activity kernel k_rows in the batched double probing.
    Bytes (the algorithmic count for a batch): the matrix term once per row
    and round over the union of the slots' worklists -- 12 B per nonzero and
    24 B per row -- plus, per vector, 16 B per distinct bound record read
    and 1088 B of accumulator limbs per heavy row tested from them (a heavy
    row's nonzeros count in the union only when its candidates are read);
    counted by an instrumented run of the same call (the base of the
    instrumented instance is the same root), divided by its launches.  Time:
    HIP events around every k_rows launch (rounds driven from the host),
    average over the launches of one call.  Also the whole call's
    algorithmic bytes (bound records written too) over its measured time."""
    def run(flags):
        J = bp.Instance(inst, bp.default_options(flags=flags, **(sched or {})))
        l2, u2 = fresh(lb, ub)
        J.propagate(l2, u2, torch.zeros(0, dtype=torch.int32, device=lb.device))
        J.kernel_stats(reset=True)
        J.probe(vars_d, cap=cap)
        torch.cuda.synchronize()
        st = J.kernel_stats(reset=True)
        del J
        return st

    cs = run(bp.FLAG_COUNT_VARS)
    run(bp.FLAG_TIME_KERNELS)  # warm
    ts = run(bp.FLAG_TIME_KERNELS)
    launches = max(ts["launches"], 1)
    rows_bytes = (12 * cs["nnz_union"] + 24 * cs["rows_union"] + 16 * cs["vars_read"]
                  + 1088 * cs["rows_kept"])
    per_launch = rows_bytes / launches
    avg_ms = ts["ms"] / launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    call_bytes = rows_bytes + 16 * cs["vars_written"]
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": None, "kernel": "k_rows",
            "avg_launch_us": round(avg_ms * 1e3, 3), "launches_per_call": ts["launches"],
            "alg_bytes_per_launch": int(per_launch),
            "union_rows": cs["rows_union"], "union_nnz": cs["nnz_union"],
            "task_rows": cs["rows"], "task_nnz": cs["nnz"], "vars_read": cs["vars_read"],
            "heavy_rows_kept": cs["rows_kept"],
            "call_alg_bytes": int(call_bytes), "call_alg_GBps": round(call_bytes / t_call / 1e9, 2),
            "call_frac": round(call_bytes / t_call / 1e9 / HBM_PEAK_GBPS, 5),
            "k_rows_share_of_call": round(ts["ms"] * 1e-3 / t_call, 3)}


def bench_scores(args, bp, inst, I, lb, ub, torch, np):
    """Probe priority and implied-slack scores (bp_scores) of every variable
    of the probe workload at its root fixed point, and the probe order
    (bp_probe_order) of all its unfixed integer variables.  Algorithmic
    bytes of a scores call: 24 per nonzero (column index and value read once
    in the row pass and once more, as CSC row and value, in the column pass),
    76 per row (row pointer, activity record written and read, row sides,
    bin list) and 100 per variable (bounds read and packed, column pointer,
    bounds again, the four outputs)."""
    m, n, nnz = int(inst["m"]), int(inst["n"]), int(inst["row_ptr"][-1])
    S = I.scores(lb, ub)  # warm: builds the CSC values and the chunk table
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        S = I.scores(lb, ub)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / reps
    lbh, ubh = lb.cpu().numpy(), ub.cpu().numpy()
    cand = np.nonzero((inst["vtype"] == 1) & (ubh > lbh))[0].astype(np.int32)
    cand_d = torch.tensor(cand, dtype=torch.int32, device=lb.device)
    order = I.probe_order(cand_d, lb, ub)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        order = I.probe_order(cand_d, lb, ub)
    torch.cuda.synchronize()
    to = (time.perf_counter() - t0) / 3
    alg = 24 * nnz + 76 * m + 100 * n
    res = {"workload": "scores of all %d variables (m=%d, nnz=%d) at the root fixed point; "
                       "probe order of its %d unfixed integers" % (n, m, nnz, cand.size),
           "scores_ms": ts * 1e3, "alg_bytes": alg, "effective_GBps": alg / ts / 1e9,
           "frac_of_hbm": alg / ts / 8e12, "order_ms": to * 1e3, "order_vars": int(cand.size),
           "vars_violating": int((S["nviol"] > 0).sum().item())}
    if args.probe_cpu:
        import oracle
        tc = time.perf_counter()
        oracle.scores(inst, lbh, ubh)
        tc = time.perf_counter() - tc
        res["cpu_baseline"] = {"value": tc * 1e3, "unit": "ms per scores call", "cores": 1,
                               "kind": "oracle", "sample": "one scores call of the oracle on the "
                                                           "same instance and bounds, one thread"}
    log("scores: %.3f ms per call, order of %d vars %.3f ms" % (ts * 1e3, cand.size, to * 1e3))
    return res


def bench_bulk(args, bp, gen, torch, np):
    """Bulk-rounding fix-and-propagate on the bulk workload (m=2M, n=3M,
    50% binary, 30% integer in [0,1000], ~20M nnz): B bound vectors per
    call, each the root with a seeded 5% of the unfixed integer variables
    fixed to rint(U[lb, ub]), propagated from their changed lists with
    bp_propagate_batch.  The schedule comes from the autotuners: the
    slot-engine knobs from a cold propagation (bp_autotune), the lane
    engine's workgroups per round kernel and rounds per graph from this
    batch (bp_autotune_batch).  Plain: the same vectors one per call."""
    dev = torch.device("cuda:0")
    B = args.bulk_vectors
    t = time.perf_counter()
    inst = gen.make("bulk", args.seed)
    log("bulk: instance generated in %.1f s" % (time.perf_counter() - t))
    t = time.perf_counter()
    I = bp.Instance(inst)
    torch.cuda.synchronize()
    t_load = time.perf_counter() - t
    lb0 = torch.tensor(inst["lb"], dtype=torch.float64, device=dev)
    ub0 = torch.tensor(inst["ub"], dtype=torch.float64, device=dev)
    if args.profile_bulk:
        # counter runs: the schedule the bench line's tuner chose, given
        tune = dict(trials=0)
        opt_kw = {}
        if args.bulk_schedule:
            g, r = (int(x) for x in args.bulk_schedule.split(","))
            opt_kw = dict(lv_grid=g, rounds_per_launch=r)
            I.close()
            I = bp.Instance(inst, bp.default_options(**opt_kw))
    else:
        tune = I.autotune(lb0, ub0)
        opt_kw = dict(heavy_threshold=tune["heavy_threshold"], heavy_chunk=tune["heavy_chunk"],
                      rounds_per_launch=tune["rounds_per_launch"])
    log("bulk: loaded in %.1f s, tuned %s" % (t_load, opt_kw))
    # Root bounds: the cold propagation's result.  At this size the root
    # may stop at the round limit; its bounds are still valid (every
    # tightening is implied), so they serve as the root of the candidates.
    rl, ru = fresh(lb0, ub0)
    root = I.propagate(rl, ru)
    assert root["status"] in (bp.BP_OK, bp.BP_ROUND_LIMIT), root
    # the root becomes the instance's base (a warm start with an empty change
    # list): the batched calls then read each candidate as an overlay on it
    empty = torch.zeros(0, dtype=torch.int32, device=dev)
    assert I.propagate(*fresh(rl, ru), empty)["rounds"] == 0
    # cold root propagation at this size (plain path)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps_cold = 0 if args.profile_bulk else 3
    r = root
    for _ in range(reps_cold):
        r = I.propagate(*fresh(lb0, ub0))
    torch.cuda.synchronize()
    t_cold = (time.perf_counter() - t) / max(reps_cold, 1)
    lists = gen.bulk_fix_lists(inst, rl.cpu().numpy(), ru.cpu().numpy(), B, frac=0.05, seed=args.seed)
    ptr = np.zeros(B + 1, np.int64)
    ptr[1:] = np.cumsum([p.size for p, _ in lists])
    idx = torch.tensor(np.concatenate([p for p, _ in lists]), dtype=torch.int32, device=dev)
    vals = torch.tensor(np.concatenate([v for _, v in lists]), dtype=torch.float64, device=dev)
    vec = torch.repeat_interleave(torch.arange(B, device=dev), torch.tensor(np.diff(ptr), device=dev))
    flat = vec * inst["n"] + idx.long()
    ptr_d = torch.tensor(ptr, dtype=torch.int64, device=dev)
    LB = torch.empty(B, inst["n"], dtype=torch.float64, device=dev)
    UB = torch.empty_like(LB)

    def restore():
        LB.copy_(rl.expand(B, -1))
        UB.copy_(ru.expand(B, -1))
        LB.view(-1)[flat] = vals
        UB.view(-1)[flat] = vals

    def batch_call(J):
        restore()
        return J.propagate_batch(LB, UB, ptr_d, idx)

    log("bulk: %d vectors of %d fixings ready" % (B, int(ptr[1])))
    if not args.profile_bulk:
        # the lane engine's schedule, timed on this batch itself
        restore()
        tb_tune = I.autotune_batch(LB, UB, ptr_d, idx)
        opt_kw.update(lv_grid=tb_tune["lv_grid"], rounds_per_launch=tb_tune["rounds_per_launch"])
        tune["trials"] += tb_tune["trials"]
        log("bulk: lane schedule %s" % tb_tune)
    res = batch_call(I)  # warm
    torch.cuda.synchronize()
    if args.profile_bulk:
        for _ in range(args.profile_bulk):
            res = batch_call(I)
        torch.cuda.synchronize()
        return {"profile_bulk": args.profile_bulk,
                "nnz_per_call": sum(x["nnz_propagated"] for x in res)}
    tb = 0.0
    for _ in range(args.bulk_steps):
        restore()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = I.propagate_batch(LB, UB, ptr_d, idx)
        torch.cuda.synchronize()
        tb += time.perf_counter() - t
    tb /= args.bulk_steps
    nnz_b = sum(x["nnz_propagated"] for x in res)
    status = np.array([x["status"] for x in res])
    rounds = np.array([x["rounds"] for x in res])
    log("bulk: batched %.1f ms per call" % (tb * 1e3))
    # plain: the first vectors, one per call
    kp = max(1, min(args.bulk_plain, B))  # at least one vector: the plain rate is reported
    L1 = torch.empty(1, inst["n"], dtype=torch.float64, device=dev)
    U1 = torch.empty_like(L1)
    tp = 0.0
    nnz_p = 0
    for v in range(-1, kp):
        w = max(v, 0)
        a, b = int(ptr[w]), int(ptr[w + 1])
        sel = idx[a:b].long()
        L1[0].copy_(rl)
        U1[0].copy_(ru)
        L1[0, sel] = vals[a:b]
        U1[0, sel] = vals[a:b]
        p1 = torch.tensor([0, b - a], dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r1 = I.propagate_batch(L1, U1, p1, idx[a:b])
        torch.cuda.synchronize()
        if v >= 0:  # v = -1 is a warm-up call
            tp += time.perf_counter() - t
            nnz_p += r1[0]["nnz_propagated"]
            assert r1[0] == res[v], (v, r1[0], res[v])
    log("bulk: plain %.2f ms per vector" % (tp / kp * 1e3))
    def with_base(J):
        # the base is set once per instance, before the counted or timed
        # calls (its warm start runs no round of the lane kernels)
        if not getattr(J, "bench_base_set", False):
            J.propagate(*fresh(rl, ru), empty)
            J.kernel_stats(reset=True)
            J.bench_base_set = True
        return batch_call(J)

    roof = kernel_roofline(bp, inst, with_base, reps=2, kernel="k_lv_rows", **opt_kw)
    roof["traffic"] = measured_traffic("bulk k_lv_rows", opt_kw)
    cpu = cpu_all = None
    if args.bulk_cpu and not args.no_cpu_baseline:
        # The oracle's own root of this size takes minutes, so the CPU legs
        # start from its first three rounds (a valid box of the same
        # workload); the vectors fix 5% of its unfixed integers as above.
        import oracle
        oo = oracle.Options()
        oo.max_rounds = 3
        t = time.perf_counter()
        _, olb, oub = oracle.propagate(inst, opts=oo)
        t_root3 = time.perf_counter() - t
        olists = gen.bulk_fix_lists(inst, olb, oub, B, frac=0.05, seed=args.seed)

        def one(v):
            p, val = olists[v]
            l2, u2 = olb.copy(), oub.copy()
            l2[p] = val
            u2[p] = val
            return oracle.propagate(inst, l2, u2, changed=p)[0]["nnz_propagated"]

        kc = min(args.bulk_cpu, B)
        t = time.perf_counter()
        nn = sum(one(v) for v in range(kc))
        tc = time.perf_counter() - t
        cpu = {"value": kc / tc, "unit": "vectors/s", "cores": 1, "kind": "oracle",
               "nnz_per_s": nn / tc,
               "extrapolated_ms_per_%d_vectors" % B: tc / kc * B * 1e3,
               "sample": "%d of the %d vectors (fixing 5%% each), from the oracle's first three "
                         "root rounds (%.1f s, not included), one thread; a call of %d vectors "
                         "extrapolated" % (kc, B, t_root3, B), "host": cpu_info()}
        items = list(range(kc, min(B, kc + 2 * min(CPU_POOL_MAX, os.cpu_count() or 1))))
        outs, wall, thr = oracle_pool(one, items)
        cpu_all = {"value": len(items) / wall, "unit": "vectors/s", "cores": thr, "kind": "oracle",
                   "nnz_per_s": sum(outs) / wall,
                   "sample": "%d further vectors, two per thread, unchanged single-threaded oracle"
                             % len(items), "host": cpu_info()}
        log("bulk: oracle %.2f vectors/s one thread, %.2f on %d threads" % (cpu["value"], cpu_all["value"], thr))
    light = None
    if args.bulk_light > 0:
        del LB, UB
        light = bench_bulk_light(args, bp, gen, torch, np, inst, lb0, ub0, opt_kw, B)
    return {
        "sha256": inst_sha256(inst),
        "multi_round_leg": light,
        "workload": "bulk rounding: m=%d, n=%d, nnz=%d; %d vectors per call, each fixing %d "
                    "integer variables (5%%) and propagating"
                    % (inst["m"], inst["n"], int(inst["row_ptr"][-1]), B, int(ptr[1])),
        "batched_nnz_per_s": nnz_b / tb, "batched_ms": tb * 1e3,
        "batched_vectors_per_s": B / tb,
        "plain_nnz_per_s": nnz_p / tp, "plain_vectors_per_s": kp / tp,
        "batched_over_plain": (B / tb) / (kp / tp),
        "infeasible": int((status == bp.BP_INFEASIBLE).sum()),
        "rounds_mean": float(rounds.mean()), "rounds_max": int(rounds.max()),
        "nnz_per_vector_mean": nnz_b / B,
        "root_cold": {"ms": t_cold * 1e3, "rounds": r["rounds"], "status": r["status"],
                      "nnz_per_s": r["nnz_propagated"] / t_cold},
        "load_s": t_load, "schedule": opt_kw, "tune_trials": tune["trials"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
    }


def bench_bulk_light(args, bp, gen, torch, np, inst, lb0, ub0, opt_kw, B):
    """Multi-round bulk leg: the root propagated to its fixed point (the bulk
    workload's cold root needs 1223 rounds; the round limit here is
    --bulk-fp-rounds), which becomes the instance's base; then B vectors,
    each fixing a seeded --bulk-light fraction of its unfixed integer
    variables to the planted point's values (random values in the bounds
    make every vector infeasible in its first round), so that the vectors
    stay feasible and propagate for several rounds."""
    dev = lb0.device
    o = dict(opt_kw, max_rounds=args.bulk_fp_rounds)
    I = bp.Instance(inst, bp.default_options(**o))
    fl, fu = fresh(lb0, ub0)
    t = time.perf_counter()
    fp = I.propagate(fl, fu)
    torch.cuda.synchronize()
    t_fp = time.perf_counter() - t
    assert fp["status"] == bp.BP_OK, fp
    lists = gen.bulk_fix_lists(inst, fl.cpu().numpy(), fu.cpu().numpy(), B, frac=args.bulk_light,
                               seed=args.seed + 1, point=inst["xstar"])
    ptr = np.zeros(B + 1, np.int64)
    ptr[1:] = np.cumsum([p.size for p, _ in lists])
    idx = torch.tensor(np.concatenate([p for p, _ in lists]), dtype=torch.int32, device=dev)
    vals = torch.tensor(np.concatenate([v for _, v in lists]), dtype=torch.float64, device=dev)
    vec = torch.repeat_interleave(torch.arange(B, device=dev), torch.tensor(np.diff(ptr), device=dev))
    flat = vec * inst["n"] + idx.long()
    ptr_d = torch.tensor(ptr, dtype=torch.int64, device=dev)
    LB = torch.empty(B, inst["n"], dtype=torch.float64, device=dev)
    UB = torch.empty_like(LB)
    empty = torch.zeros(0, dtype=torch.int32, device=dev)

    def call(J):
        if not getattr(J, "bench_base_set", False):
            J.propagate(*fresh(fl, fu), empty)
            J.kernel_stats(reset=True)
            J.bench_base_set = True
        LB.copy_(fl.expand(B, -1))
        UB.copy_(fu.expand(B, -1))
        LB.view(-1)[flat] = vals
        UB.view(-1)[flat] = vals
        return J.propagate_batch(LB, UB, ptr_d, idx)

    res = call(I)  # warm
    torch.cuda.synchronize()
    tb = 0.0
    reps = 3
    for _ in range(reps):
        LB.copy_(fl.expand(B, -1))
        UB.copy_(fu.expand(B, -1))
        LB.view(-1)[flat] = vals
        UB.view(-1)[flat] = vals
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = I.propagate_batch(LB, UB, ptr_d, idx)
        torch.cuda.synchronize()
        tb += time.perf_counter() - t
    tb /= reps
    nnz_b = sum(x["nnz_propagated"] for x in res)
    status = np.array([x["status"] for x in res])
    rounds = np.array([x["rounds"] for x in res])
    log("bulk light: %.1f ms per call, rounds mean %.2f, %d infeasible"
        % (tb * 1e3, rounds.mean(), int((status == bp.BP_INFEASIBLE).sum())))
    # plain: the first vectors one per call (bp_propagate warm starts from
    # the same base, with their fixings as the changed list)
    kp = min(args.bulk_plain, B)
    I.propagate(*fresh(fl, fu), empty)
    torch.cuda.synchronize()
    tp, nnz_p = 0.0, 0
    for v in range(kp):
        p, val = lists[v]
        l1, u1 = fresh(fl, fu)
        pd = torch.tensor(p, dtype=torch.int32, device=dev)
        vd = torch.tensor(val, dtype=torch.float64, device=dev)
        l1[pd.long()] = vd
        u1[pd.long()] = vd
        torch.cuda.synchronize()
        t = time.perf_counter()
        r1 = I.propagate(l1, u1, pd)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t
        nnz_p += r1["nnz_propagated"]
        assert r1 == res[v], (v, r1, res[v])
    log("bulk light: plain %.2f ms per vector" % (tp / max(kp, 1) * 1e3))
    roof = kernel_roofline(bp, inst, call, reps=2, kernel="k_lv_rows", **o)
    del LB, UB
    return {"workload": "bulk rounding from the fixed-point root (%d rounds): %d vectors per call, "
                        "each fixing %d integer variables (%.1f%%) to the planted point's values "
                        "and propagating"
                        % (fp["rounds"], B, int(ptr[1]), 100 * args.bulk_light),
            "root_fixed_point": {"rounds": fp["rounds"], "ms": t_fp * 1e3},
            "batched_ms": tb * 1e3, "batched_nnz_per_s": nnz_b / tb, "batched_vectors_per_s": B / tb,
            "plain_vectors_per_s": kp / tp if kp else None,
            "plain_nnz_per_s": nnz_p / tp if kp else None,
            "batched_over_plain": (B / tb) / (kp / tp) if kp else None,
            "plain_sample": "the first %d vectors, one bp_propagate per vector" % kp,
            "infeasible": int((status == bp.BP_INFEASIBLE).sum()),
            "rounds_mean": float(rounds.mean()), "rounds_max": int(rounds.max()),
            "nnz_per_vector_mean": nnz_b / B, "roofline": roof}


def bench_serving(args, bp, gen, torch, np):
    """Serving: seeded instances with m log-uniform in [1e3, mmax] (n = 1.5 m,
    nnz ~ 8 m), resident on the device; a seeded request trace, instance
    uniform, half propagate requests (1% of the unfixed binaries fixed to a
    random 0/1) and half probe requests (k = round(exp(U[0, ln 512])) unfixed
    binaries).  C is the saturated rate (all requests queued at once); then
    Poisson arrivals at 0.5 C and 0.9 C report p50/p99 latency.  Baseline:
    the same requests served one at a time in arrival order (FIFO) with
    bp_propagate / bp_probe, its latency derived from measured service times
    and the same arrival trace as the server's run at that load."""
    import math
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    insts = gen.make_serving(args.seed, count=args.serve_instances, m_hi=args.serve_mmax)
    t_gen = time.perf_counter() - t_gen
    log("serving: %d instances generated in %.1f s" % (len(insts), t_gen))
    loaded, bases = [], []
    for inst in insts:
        I = bp.Instance(inst)
        lb = torch.tensor(inst["lb"], dtype=torch.float64, device=dev)
        ub = torch.tensor(inst["ub"], dtype=torch.float64, device=dev)
        r = I.propagate(lb, ub)
        assert r["status"] == bp.BP_OK
        loaded.append(I)
        bases.append((lb.cpu().numpy(), ub.cpu().numpy()))
    rng = np.random.default_rng(args.seed + 17)
    reqs = []
    for _ in range(args.serve_requests):
        t = int(rng.integers(0, len(insts)))
        lb, ub = bases[t]
        bins = np.nonzero((insts[t]["vtype"] == 1) & (lb == 0) & (ub == 1))[0]
        if rng.uniform() < 0.5:
            k = max(1, int(round(0.01 * bins.size)))
            vs = np.sort(rng.choice(bins, size=min(k, bins.size), replace=False)).astype(np.int32)
            val = rng.integers(0, 2, size=vs.size).astype(np.float64)
            reqs.append((t, bp.REQ_PROPAGATE, vs, val))
        else:
            k = int(round(math.exp(rng.uniform(0, math.log(512)))))
            vs = np.sort(rng.choice(bins, size=min(k, bins.size), replace=False)).astype(np.int32)
            reqs.append((t, bp.REQ_PROBE, vs, None))
    nnz_total = sum(int(i["row_ptr"][-1]) for i in insts)
    opts = bp.default_options(rounds_per_launch=args.serve_rounds)
    budget = 64 << 30
    S = bp.Server(loaded, budget, opts)
    info = S.info()
    S.close()
    log("serving: instances resident, %d requests, %d slots of %d bytes"
        % (len(reqs), info["slots"], info["bytes_per_slot"]))
    for q, pl in enumerate(info["pools"]):
        log("  pool %d: %d instances, %d slots of %d bytes" % (q, pl["instances"], pl["slots"], pl["bytes_per_slot"]))

    def run_trace(arrivals):
        """arrivals: seconds from start (None: all at once).  Returns
        (elapsed s, latencies us, jobs, nnz)."""
        S0 = bp.Server(loaded, budget, opts)
        ids = {}
        sub_py = {}
        i = 0
        n = len(reqs)
        done = {}
        t0 = time.perf_counter()
        t_note = t_last = t0
        while len(done) < n:
            now = time.perf_counter() - t0
            while i < n and (arrivals is None or arrivals[i] <= now):
                t, kind, vs, val = reqs[i]
                sub_py[i] = time.perf_counter()
                rid = S0.submit(t, kind, vs, val, val)
                ids[rid] = i
                i += 1
            busy = S0.run(args.serve_rounds)
            got = S0.poll(100000)
            for c in got:
                done[ids[c["id"]]] = c
            tn = time.perf_counter()
            if got:
                t_last = tn
            if tn - t_note > 5.0:
                log("  serving: %d/%d done, %d submitted, %d unfinished, %.1f s"
                    % (len(done), n, i, busy, tn - t0))
                t_note = tn
            if busy and tn - t_last > 60.0:
                raise RuntimeError("serving made no progress for 60 s (%d/%d done, %d unfinished)"
                                   % (len(done), n, busy))
            if busy == 0 and i < n and arrivals is not None:
                wait = arrivals[i] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
        elapsed = time.perf_counter() - t0
        # Latency from arrival to the server observing the last job done.
        # The server stamps in its own clock; the submit stamp of each
        # request maps the arrival time onto it.
        lat = []
        for j in range(n):
            arr_py = t0 + (0.0 if arrivals is None else arrivals[j])
            off_us = done[j]["submit_us"] - sub_py[j] * 1e6
            lat.append(done[j]["done_us"] - (arr_py * 1e6 + off_us))
        S0.close()
        return elapsed, np.array(lat)

    # saturated rate
    el_sat, lat_sat = run_trace(None)
    C = len(reqs) / el_sat
    log("serving: saturated %.1f requests/s" % C)
    out = {"workload": "%d instances, m log-uniform [1e3, %g], %d nnz resident; %d requests "
                       "(50%% propagate fixing 1%% of binaries, 50%% probe k~exp U[0, ln 512])"
                       % (len(insts), args.serve_mmax, nnz_total, len(reqs)),
           "sha256_of_instance_digests": __import__("hashlib").sha256(
               "".join(inst_sha256(x) for x in insts).encode()).hexdigest(),
           "slots": info["slots"], "bytes_per_slot": info["bytes_per_slot"], "pools": info["pools"],
           "generate_s": t_gen, "saturated_requests_per_s": C,
           "saturated_p50_ms": float(np.percentile(lat_sat, 50)) / 1e3,
           "saturated_p99_ms": float(np.percentile(lat_sat, 99)) / 1e3}
    # one Poisson arrival trace per load, served both by the server and by
    # the FIFO baseline below
    traces = {frac: np.cumsum(rng.exponential(1.0 / (frac * C), size=len(reqs))) for frac in (0.5, 0.9)}
    for frac in (0.5, 0.9):
        arrivals = traces[frac]
        el, lat = run_trace(arrivals)
        log("serving: load %g done in %.1f s" % (frac, el))
        out["load_%g" % frac] = {"offered_per_s": frac * C, "served_per_s": len(reqs) / el,
                                 "p50_ms": float(np.percentile(lat, 50)) / 1e3,
                                 "p99_ms": float(np.percentile(lat, 99)) / 1e3}
    # FIFO one-at-a-time baseline: the service time of every request alone,
    # measured instance by instance on a fresh instance (its engine memory
    # is released before the next one; service times do not depend on the
    # order), after one warm-up probe and propagation.  Propagate requests
    # use a one-vector batch, which leaves the base unchanged, as the server
    # does.
    svc = np.zeros(len(reqs))
    t_fifo = time.perf_counter()
    by_inst = {}
    for j, rq in enumerate(reqs):
        by_inst.setdefault(rq[0], []).append(j)
    done_n = 0

    def serve_one(J, lb0, ub0, kind, vs, val):
        if kind == bp.REQ_PROBE:
            J.probe(torch.tensor(vs, dtype=torch.int32, device=dev))
        else:
            lb = torch.tensor(lb0, device=dev)[None].clone()
            ub = torch.tensor(ub0, device=dev)[None].clone()
            vv = torch.tensor(vs, dtype=torch.long, device=dev)
            vals = torch.tensor(val, device=dev)
            lb[0, vv] = torch.maximum(lb[0, vv], vals)
            ub[0, vv] = torch.minimum(ub[0, vv], vals)
            ptr = torch.tensor([0, len(vs)], dtype=torch.int64, device=dev)
            J.propagate_batch(lb, ub, ptr, torch.tensor(vs, dtype=torch.int32, device=dev))
        torch.cuda.synchronize()

    for t, js in sorted(by_inst.items()):
        J = bp.Instance(insts[t])
        lb0, ub0 = bases[t]
        J.propagate(torch.tensor(lb0, device=dev), torch.tensor(ub0, device=dev))  # base
        first = reqs[js[0]]
        serve_one(J, lb0, ub0, bp.REQ_PROBE, first[2][:1] if first[1] == bp.REQ_PROBE else
                  np.nonzero((insts[t]["vtype"] == 1) & (lb0 == 0) & (ub0 == 1))[0][:1].astype(np.int32),
                  None)
        for j in js:
            _, kind, vs, val = reqs[j]
            ts = time.perf_counter()
            serve_one(J, lb0, ub0, kind, vs, val)
            svc[j] = time.perf_counter() - ts
            done_n += 1
            if time.perf_counter() - t_fifo > 5.0:
                log("  fifo baseline: %d/%d requests" % (done_n, len(reqs)))
                t_fifo = time.perf_counter()
        del J
        torch.cuda.synchronize()
    base = {"saturated_requests_per_s": len(reqs) / svc.sum()}
    for frac in (0.5, 0.9):
        arrivals = traces[frac]
        finish = np.zeros(len(reqs))
        tcur = 0.0
        for j in range(len(reqs)):
            tcur = max(tcur, arrivals[j]) + svc[j]
            finish[j] = tcur
        lat = (finish - arrivals) * 1e3
        base["load_%g" % frac] = {"p50_ms": float(np.percentile(lat, 50)),
                                  "p99_ms": float(np.percentile(lat, 99))}
    out["fifo_one_at_a_time"] = base
    out["throughput_over_fifo"] = C / base["saturated_requests_per_s"]
    return out


if __name__ == "__main__":
    main()
