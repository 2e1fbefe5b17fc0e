"""Write bulk_root.json: the CPU oracle's cold propagation of the full bulk
workload (m=2M rows, n=3M variables, ~20M nonzeros, seed 0) from its
initial bounds, with the default options (1000-round limit).

The bound vectors are too large to store, so the file keeps the outcome,
the counters and the evidence, sha256 digests of the bounds (integer
variables and continuous variables apart, each as the little-endian bytes
of lb then ub), and the bounds of a seeded sample of continuous variables
for a comparison within tolerance.  Only the oracle computes anything
here; the generator supplies the input.  Runs for about ten minutes on one
core:  python tests/golden/make_bulk_root.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2510_20499_amd import gen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bulk_root.json")
SAMPLE = 4096


def digest(lb, ub):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(lb, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(ub, dtype="<f8").tobytes())
    return h.hexdigest()


def main():
    t0 = time.time()
    inst = gen.make("bulk", 0)
    print("generated in %.1f s: m=%d n=%d nnz=%d" % (time.time() - t0, inst["m"], inst["n"],
                                                     inst["col"].size), flush=True)
    t0 = time.time()
    r, lb, ub = oracle.propagate(inst)
    secs = time.time() - t0
    print("oracle: %s in %.1f s" % (r, secs), flush=True)
    integ = inst["vtype"] == 1
    cont = np.nonzero(~integ)[0]
    rng = np.random.default_rng(20251023)
    pick = np.sort(rng.choice(cont, size=min(SAMPLE, cont.size), replace=False))
    rec = dict(
        workload="bulk, seed 0, cold start from the initial bounds, default options",
        m=int(inst["m"]), n=int(inst["n"]), nnz=int(inst["col"].size),
        input_sha256=digest(inst["lb"], inst["ub"]),
        result={k: int(v) for k, v in r.items()},
        integer_bounds_sha256=digest(lb[integ], ub[integ]),
        continuous_bounds_sha256=digest(lb[~integ], ub[~integ]),
        continuous_sample=dict(var=pick.tolist(), lb=[float(x) for x in lb[pick]],
                               ub=[float(x) for x in ub[pick]]),
        oracle_seconds=round(secs, 1),
    )
    with open(OUT, "w") as fh:
        json.dump(rec, fh)
        fh.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
