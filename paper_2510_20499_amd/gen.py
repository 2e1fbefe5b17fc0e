"""Seeded synthetic MILP instances for bound propagation and probing.

This module only draws inputs.  It holds none of the propagation arithmetic:
it builds a constraint matrix, row sides and variable bounds from a numpy
``PCG64`` stream, and both the GPU path and the CPU oracle are fed the same
arrays.  The paper evaluates on MIPLIB2017 (Section 3), which is not used
here; the instances below stand in for it.  Their shape follows the paper's
observation (Section 2.1, load-balancing paragraph) that constraints and
variables carry a median of 6-9 terms on average, with large variability:
most rows are short (truncated power law), a few are dense (10k-50k terms).

An instance is a dict with

* ``m``, ``n``: rows and variables;
* ``row_ptr`` (int64[m+1]), ``col`` (int32[nnz], ascending per row),
  ``val`` (float64[nnz], no explicit zeros): the CSR matrix;
* ``lo``, ``hi`` (float64[m]): row sides, ``lo <= a.x <= hi`` with +-inf for
  one-sided rows;
* ``vtype`` (uint8[n]): 0 continuous, 1 integer (binaries are integers in
  [0, 1]);
* ``lb``, ``ub`` (float64[n]): initial variable bounds;
* ``xstar`` (float64[n]): the planted point every row is built around.
"""
from __future__ import annotations

import math

import numpy as np

INF = float("inf")

# Workloads (sizes as given for the benchmark configurations).
CONFIGS = {
    # Tiny: m=200, n=300 (150 binary, 100 integer [0,10], 50 continuous
    # [0,100]), 4-6 nnz per row, integer coefficients in [-5,5]\{0}, rows
    # a.x <= a.x* + U[0,3].
    "tiny": dict(m=200, n=300, frac_bin=0.5, frac_int=1.0 / 3.0, u_int=10,
                 u_cont=100.0, kind="tiny"),
    # Single instance, plain path: m=100k, n=150k (60% B, 20% I[0,100],
    # 20% C[0,1e4]), ~1M nnz, power-law rows plus ~20 dense rows.
    "single": dict(m=100_000, n=150_000, frac_bin=0.6, frac_int=0.2,
                   u_int=100, u_cont=1e4, nnz=1_000_000, dense=20,
                   kind="generic"),
    # Batched double probing: m=500k, n=1M (70% B), 8M nnz, with set-cover
    # rows (0/1 coefficients, >= 1) and big-M rows (one coefficient 1e4).
    "probe": dict(m=500_000, n=1_000_000, frac_bin=0.7, frac_int=0.15,
                  u_int=100, u_cont=1e4, nnz=8_000_000, dense=100,
                  frac_setcover=0.30, frac_bigm=0.05, kind="generic"),
    # Bulk rounding: m=2M, n=3M (50% B, 30% I[0,1000]), 20M nnz.
    "bulk": dict(m=2_000_000, n=3_000_000, frac_bin=0.5, frac_int=0.3,
                 u_int=1000, u_cont=1e4, nnz=20_000_000, dense=400,
                 kind="generic"),
}


def _stream(seed: int, n_streams: int = 8):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n_streams)]


def _power_law_lmax(mean_target: float, lmin: int = 2, alpha: float = 1.5,
                    cap: int = 4096) -> int:
    """Smallest L_max such that the truncated power law P(L) ~ L^-alpha on
    [lmin, L_max] has mean >= mean_target (integer search)."""
    best = lmin
    for lmax in range(lmin, cap + 1):
        L = np.arange(lmin, lmax + 1, dtype=np.float64)
        w = L ** (-alpha)
        mean = float((w * L).sum() / w.sum())
        best = lmax
        if mean >= mean_target:
            break
    return best


def _power_law_lengths(rng, count: int, lmax: int, lmin: int = 2,
                       alpha: float = 1.5) -> np.ndarray:
    L = np.arange(lmin, lmax + 1, dtype=np.int64)
    w = L.astype(np.float64) ** (-alpha)
    w /= w.sum()
    return rng.choice(L, size=count, p=w)


def _draw_supports(rng, lengths: np.ndarray, pools: list, pool_of_row: np.ndarray):
    """Draw, for every row, ``lengths[r]`` distinct column indices from the
    pool ``pools[pool_of_row[r]]`` (an int array of candidate columns).

    Returns (row_ptr, col) with columns ascending inside each row."""
    m = lengths.shape[0]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int64)
    row_of = np.repeat(np.arange(m, dtype=np.int64), lengths)
    big = 4096  # rows longer than this are drawn one by one without replacement
    long_rows = np.nonzero(lengths > big)[0]
    short_mask = lengths[row_of] <= big
    for p, pool in enumerate(pools):
        sel = short_mask & (pool_of_row[row_of] == p)
        idx = np.nonzero(sel)[0]
        if idx.size:
            col[idx] = pool[rng.integers(0, pool.size, size=idx.size)]
    for r in long_rows:
        pool = pools[pool_of_row[r]]
        a, b = row_ptr[r], row_ptr[r + 1]
        col[a:b] = np.sort(rng.choice(pool, size=b - a, replace=False))
    # Resample duplicates inside short rows until every row's support is a set.
    n_cols = int(max(int(pool.max()) for pool in pools if pool.size)) + 1
    for _ in range(200):
        key = row_of * n_cols + col
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(nnz, dtype=bool)
        dup[order[1:][ks[1:] == ks[:-1]]] = True
        if not dup.any():
            break
        di = np.nonzero(dup)[0]
        for p, pool in enumerate(pools):
            sel = di[pool_of_row[row_of[di]] == p]
            if sel.size:
                col[sel] = pool[rng.integers(0, pool.size, size=sel.size)]
    else:  # pragma: no cover - pools far too small for the requested lengths
        raise RuntimeError("could not draw distinct supports")
    # Sort columns inside rows.
    key = row_of * n_cols + col
    col = col[np.argsort(key, kind="stable")]
    return row_ptr, col.astype(np.int32)


def _var_types(rng, n, frac_bin, frac_int, u_int, u_cont, cont_int_point=False):
    n_bin = int(round(frac_bin * n))
    n_int = int(round(frac_int * n))
    perm = rng.permutation(n)
    kind = np.full(n, 2, dtype=np.int8)  # 0 bin, 1 int, 2 cont
    kind[perm[:n_bin]] = 0
    kind[perm[n_bin:n_bin + n_int]] = 1
    vtype = (kind < 2).astype(np.uint8)
    lb = np.zeros(n)
    ub = np.where(kind == 0, 1.0, np.where(kind == 1, float(u_int), float(u_cont)))
    return kind, vtype, lb, ub


def _planted_point(rng, kind, u_int, u_cont, cont_integer):
    n = kind.shape[0]
    x = np.empty(n)
    b = kind == 0
    x[b] = rng.integers(0, 2, size=int(b.sum()))
    i = kind == 1
    x[i] = rng.integers(0, u_int + 1, size=int(i.sum()))
    c = kind == 2
    if cont_integer:
        x[c] = rng.integers(0, int(u_cont) + 1, size=int(c.sum()))
    else:
        x[c] = rng.uniform(0.0, u_cont, size=int(c.sum()))
    return x


def _row_activity_at(row_ptr, col, val, x):
    prod = val * x[col]
    m = row_ptr.shape[0] - 1
    out = np.zeros(m)
    nz = row_ptr[1:] > row_ptr[:-1]
    out[nz] = np.add.reduceat(prod, row_ptr[:-1][nz])
    return out


def make_tiny(seed: int = 0, m: int = 200, n: int = 300, inf_frac: float = 0.0):
    """The Tiny workload: integer coefficients, all rows ``a.x <= a.x* + d``.

    ``inf_frac`` > 0 gives that fraction of the continuous variables one
    infinite bound (half lose ub, half lose lb), exercising the infinite
    contribution counts."""
    rs = _stream(seed)
    cfg = CONFIGS["tiny"]
    n_bin = int(round(n * 0.5))
    n_int = int(round(n / 3.0))
    kind, vtype, lb, ub = _var_types(rs[0], n, n_bin / n, n_int / n,
                                     cfg["u_int"], cfg["u_cont"])
    x = _planted_point(rs[1], kind, cfg["u_int"], cfg["u_cont"], True)
    lengths = rs[2].integers(4, 7, size=m)
    row_ptr, col = _draw_supports(rs[3], lengths, [np.arange(n)], np.zeros(m, np.int64))
    nnz = int(row_ptr[-1])
    val = rs[4].integers(1, 6, size=nnz).astype(np.float64)
    val *= np.where(rs[4].integers(0, 2, size=nnz) == 0, -1.0, 1.0)
    s = _row_activity_at(row_ptr, col, val, x)
    hi = s + rs[5].uniform(0.0, 3.0, size=m)
    lo = np.full(m, -INF)
    if inf_frac > 0:
        cont = np.nonzero(kind == 2)[0]
        k = int(round(inf_frac * cont.size))
        pick = rs[6].permutation(cont)[:k]
        half = k // 2
        ub[pick[:half]] = INF
        lb[pick[half:]] = -INF
    return dict(m=m, n=n, row_ptr=row_ptr, col=col, val=val, lo=lo, hi=hi,
                vtype=vtype, lb=lb, ub=ub, xstar=x, kind=kind)


def make_generic(seed: int = 0, m: int = 100_000, n: int = 150_000,
                 frac_bin: float = 0.6, frac_int: float = 0.2, u_int: int = 100,
                 u_cont: float = 1e4, nnz: int = 1_000_000, dense: int = 20,
                 frac_setcover: float = 0.0, frac_bigm: float = 0.0,
                 dense_len=(10_000, 50_000), sides=(0.85, 0.10, 0.05), **_):
    """Power-law rows with real coefficients in [-100, 100].

    ``dense`` rows get a length uniform on ``dense_len`` (capped at n/2); the
    other rows follow P(L) ~ L^-1.5 on [2, L_max] with L_max chosen so the
    expected total is ``nnz``.  Set-cover rows use binaries only, coefficient
    1 and ``>= 1`` (each holds a binary with x* = 1); big-M rows are generic
    rows with one extra binary of coefficient -1e4.  Generic sides are
    ``<=`` / ``>=`` / ranged in the ``sides`` proportions, each with a slack
    drawn from U[0, 3] around a.x*."""
    rs = _stream(seed)
    kind, vtype, lb, ub = _var_types(rs[0], n, frac_bin, frac_int, u_int, u_cont)
    x = _planted_point(rs[1], kind, u_int, u_cont, False)
    dlo, dhi = dense_len
    dhi = min(dhi, n // 2)
    dlo = min(dlo, dhi)
    dense = min(dense, m)
    dense_lengths = rs[2].integers(dlo, dhi + 1, size=dense) if dense else np.zeros(0, np.int64)
    rest = m - dense
    mean_rest = max(2.0, (nnz - float(dense_lengths.sum())) / max(rest, 1))
    lmax = _power_law_lmax(mean_rest)
    lengths = np.concatenate([_power_law_lengths(rs[2], rest, lmax), dense_lengths]).astype(np.int64)
    # Place dense rows at seeded positions.
    perm = rs[3].permutation(m)
    lengths = lengths[np.argsort(perm, kind="stable")]
    is_dense = np.zeros(m, dtype=bool)
    is_dense[perm[rest:]] = True  # positions holding the dense lengths
    # Row roles: 0 generic, 1 set-cover, 2 big-M (dense rows stay generic).
    role = np.zeros(m, dtype=np.int8)
    cand = np.nonzero(~is_dense)[0]
    cand = rs[4].permutation(cand)
    n_sc = int(round(frac_setcover * m))
    n_bm = int(round(frac_bigm * m))
    role[cand[:n_sc]] = 1
    role[cand[n_sc:n_sc + n_bm]] = 2
    bins = np.nonzero(kind == 0)[0]
    pools = [np.arange(n), bins]
    pool_of_row = (role == 1).astype(np.int64)
    # Big-M rows draw their generic part one shorter, then get the extra binary.
    gl = lengths.copy()
    gl[role == 2] = np.maximum(gl[role == 2] - 1, 1)
    row_ptr, col = _draw_supports(rs[5], gl, pools, pool_of_row)
    nnz_g = int(row_ptr[-1])
    val = rs[6].uniform(-100.0, 100.0, size=nnz_g)
    while True:
        z = val == 0.0
        if not z.any():
            break
        val[z] = rs[6].uniform(-100.0, 100.0, size=int(z.sum()))
    row_of = np.repeat(np.arange(m), np.diff(row_ptr))
    val[role[row_of] == 1] = 1.0
    # Set-cover rows: force one member with x* = 1.
    sc_rows = np.nonzero(role == 1)[0]
    if sc_rows.size:
        ones = bins[x[bins] == 1.0]
        for r in sc_rows:
            a, b = row_ptr[r], row_ptr[r + 1]
            seg = col[a:b]
            if not (x[seg] == 1.0).any():
                choice = ones[rs[7].integers(0, ones.size)]
                if choice not in seg:
                    seg = np.sort(np.concatenate([seg[1:], [choice]]))
                    col[a:b] = seg.astype(np.int32)
    # Big-M rows: append one binary not already present with coefficient -1e4.
    bm_rows = np.nonzero(role == 2)[0]
    if bm_rows.size:
        new_len = np.diff(row_ptr).copy()
        new_len[bm_rows] += 1
        new_ptr = np.zeros(m + 1, dtype=np.int64)
        np.cumsum(new_len, out=new_ptr[1:])
        new_col = np.empty(int(new_ptr[-1]), dtype=np.int32)
        new_val = np.empty(int(new_ptr[-1]))
        # copy old rows
        keep = np.ones(int(new_ptr[-1]), dtype=bool)
        extra_pos = new_ptr[bm_rows + 1] - 1
        keep[extra_pos] = False
        new_col[keep] = col
        new_val[keep] = val
        extra = bins[rs[7].integers(0, bins.size, size=bm_rows.size)]
        for t, r in enumerate(bm_rows):
            a, b = row_ptr[r], row_ptr[r + 1]
            seg = col[a:b]
            e = extra[t]
            while e in seg:
                e = bins[rs[7].integers(0, bins.size)]
            segv = val[a:b]
            merged_c = np.concatenate([seg, [e]]).astype(np.int32)
            merged_v = np.concatenate([segv, [-1e4]])
            o = np.argsort(merged_c, kind="stable")
            na, nb = new_ptr[r], new_ptr[r + 1]
            new_col[na:nb] = merged_c[o]
            new_val[na:nb] = merged_v[o]
        row_ptr, col, val = new_ptr, new_col, new_val
    s = _row_activity_at(row_ptr, col, val, x)
    lo = np.full(m, -INF)
    hi = np.full(m, INF)
    u = rs[7].uniform(size=m)
    d1 = rs[7].uniform(0.0, 3.0, size=m)
    d2 = rs[7].uniform(0.0, 3.0, size=m)
    le = u < sides[0]
    ge = (u >= sides[0]) & (u < sides[0] + sides[1])
    rg = u >= sides[0] + sides[1]
    hi[le] = s[le] + d1[le]
    lo[ge] = s[ge] - d1[ge]
    lo[rg] = s[rg] - d1[rg]
    hi[rg] = s[rg] + d2[rg]
    sc = role == 1
    lo[sc] = 1.0
    hi[sc] = INF
    return dict(m=m, n=n, row_ptr=row_ptr, col=col.astype(np.int32), val=val,
                lo=lo, hi=hi, vtype=vtype, lb=lb, ub=ub, xstar=x, kind=kind)


def make(name: str, seed: int = 0, scale: float = 1.0):
    """Instance of a named workload; ``scale`` < 1 shrinks m, n, nnz and the
    dense-row count/length proportionally (for tests at reduced size)."""
    if name in ("tiny", "tiny_inf"):
        return make_tiny(seed, inf_frac=0.1 if name == "tiny_inf" else 0.0)
    cfg = dict(CONFIGS[name])
    if scale != 1.0:
        cfg["m"] = max(8, int(cfg["m"] * scale))
        cfg["n"] = max(8, int(cfg["n"] * scale))
        cfg["nnz"] = max(16, int(cfg["nnz"] * scale))
        cfg["dense_len"] = (max(64, int(10_000 * scale)), max(64, int(50_000 * scale)))
    return make_generic(seed, **cfg)


def make_serving(seed: int = 0, count: int = 64, m_lo: float = 1e3, m_hi: float = 1e6):
    """Serving mix: ``count`` instances with m log-uniform in [m_lo, m_hi],
    n = 1.5 m, nnz ~ 8 m, dense rows round(2e-4 m); same generator as the
    single-instance workload."""
    rng = _stream(seed)[0]
    out = []
    for t in range(count):
        m = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        n = int(round(1.5 * m))
        d = int(round(2e-4 * m))
        out.append(make_generic(seed * 1000 + t + 1, m=m, n=n, frac_bin=0.6,
                                frac_int=0.2, u_int=100, u_cont=1e4,
                                nnz=8 * m, dense=d))
    return out


def make_micro(seed: int, n: int = None, m: int = None):
    """Pure-integer micro instance for brute force: n <= 8 variables with
    domains inside {0..3}, m <= 6 rows, integer coefficients in [-5, 5].
    Sides are drawn around a random point with a slack that may be negative,
    so some instances are infeasible."""
    rng = _stream(seed)[0]
    if n is None:
        n = int(rng.integers(2, 9))
    if m is None:
        m = int(rng.integers(1, 7))
    lb = rng.integers(0, 2, size=n).astype(np.float64)
    ub = np.minimum(3.0, lb + rng.integers(0, 3, size=n))
    vtype = np.ones(n, dtype=np.uint8)
    rows_c, rows_v = [], []
    for _ in range(m):
        L = int(rng.integers(1, min(n, 5) + 1))
        c = np.sort(rng.choice(n, size=L, replace=False))
        v = rng.integers(1, 6, size=L) * np.where(rng.integers(0, 2, size=L) == 0, -1, 1)
        rows_c.append(c)
        rows_v.append(v.astype(np.float64))
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(c) for c in rows_c])
    col = np.concatenate(rows_c).astype(np.int32)
    val = np.concatenate(rows_v)
    x = np.array([rng.integers(int(lb[i]), int(ub[i]) + 1) for i in range(n)], dtype=np.float64)
    s = _row_activity_at(row_ptr, col, val, x)
    lo = np.full(m, -INF)
    hi = np.full(m, INF)
    for k in range(m):
        t = int(rng.integers(0, 3))
        slack = float(rng.integers(-2, 3))
        if t == 0:
            hi[k] = s[k] + slack
        elif t == 1:
            lo[k] = s[k] - slack
        else:
            lo[k] = s[k] - abs(slack)
            hi[k] = s[k] + float(rng.integers(0, 3))
    return dict(m=m, n=n, row_ptr=row_ptr, col=col, val=val, lo=lo, hi=hi,
                vtype=vtype, lb=lb, ub=ub, xstar=x)


def from_rows(n, rows, lo, hi, vtype, lb, ub):
    """Instance from a list of (cols, vals) rows (small hand-written cases)."""
    m = len(rows)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(c) for c, _ in rows])
    col = np.concatenate([np.asarray(c, dtype=np.int32) for c, _ in rows]) if m else np.zeros(0, np.int32)
    val = np.concatenate([np.asarray(v, dtype=np.float64) for _, v in rows]) if m else np.zeros(0)
    return dict(m=m, n=n, row_ptr=row_ptr, col=col.astype(np.int32), val=val,
                lo=np.asarray(lo, dtype=np.float64), hi=np.asarray(hi, dtype=np.float64),
                vtype=np.asarray(vtype, dtype=np.uint8), lb=np.asarray(lb, dtype=np.float64),
                ub=np.asarray(ub, dtype=np.float64))


def pick_probe_vars(inst, lb, ub, k: int, seed: int = 0):
    """Seeded sample of k binaries that are unfixed in the bounds (lb, ub)."""
    rng = _stream(seed + 7919)[0]
    binm = (inst["vtype"] == 1) & (lb == 0.0) & (ub == 1.0)
    cand = np.nonzero(binm)[0]
    k = min(k, cand.size)
    return np.sort(rng.choice(cand, size=k, replace=False)).astype(np.int32)


def bulk_fix_lists(inst, lb, ub, count: int, frac: float = 0.05, seed: int = 0, point=None):
    """Bulk-rounding candidates as fixing lists: for each of ``count``
    vectors, a seeded ``frac`` of the unfixed integer variables (sorted) and
    their values rint(U[lb, ub]), or, with ``point``, the point's values
    rounded and clipped into [lb, ub] (the planted point gives candidates
    that stay feasible).  Returns a list of (vars int32, values)."""
    rng = _stream(seed + 104729)[0]
    ints = np.nonzero(inst["vtype"] == 1)[0]
    ints = ints[np.isfinite(lb[ints]) & np.isfinite(ub[ints]) & (lb[ints] < ub[ints])]
    k = int(round(frac * ints.size))
    out = []
    for _ in range(count):
        pick = np.sort(rng.choice(ints, size=k, replace=False))
        if point is None:
            val = np.rint(rng.uniform(lb[pick], ub[pick]))
        else:
            val = np.clip(np.rint(point[pick]), lb[pick], ub[pick])
        out.append((pick.astype(np.int32), val))
    return out


def bulk_fix_vectors(inst, lb, ub, count: int, frac: float = 0.05, seed: int = 0):
    """Bulk-rounding candidates as dense bound vectors: (LB[count, n],
    UB[count, n], changed lists), the fixings of bulk_fix_lists applied to
    (lb, ub)."""
    LB = np.repeat(lb[None, :], count, axis=0)
    UB = np.repeat(ub[None, :], count, axis=0)
    changed = []
    for v, (pick, val) in enumerate(bulk_fix_lists(inst, lb, ub, count, frac, seed)):
        LB[v, pick] = val
        UB[v, pick] = val
        changed.append(pick)
    return LB, UB, changed


# ---------------------------------------------------------------------------
# Instance files: an .npz of the arrays plus a sha256 manifest beside it.
# ---------------------------------------------------------------------------
ARRAYS = ("row_ptr", "col", "val", "lo", "hi", "vtype", "lb", "ub")


def digest(inst) -> str:
    """sha256 over the instance's arrays (row pointers, columns,
    coefficients, sides, types, bounds) in that order, as their bytes."""
    import hashlib
    h = hashlib.sha256()
    for k in ARRAYS:
        h.update(np.ascontiguousarray(inst[k]).tobytes())
    return h.hexdigest()


def _manifest(inst) -> dict:
    import hashlib
    return {"m": int(inst["m"]), "n": int(inst["n"]), "sha256": digest(inst),
            "arrays": {k: {"dtype": str(np.asarray(inst[k]).dtype),
                           "shape": list(np.asarray(inst[k]).shape),
                           "sha256": hashlib.sha256(np.ascontiguousarray(inst[k]).tobytes()).hexdigest()}
                       for k in ARRAYS}}


def save(inst, path: str) -> str:
    """Write the instance to ``path`` (.npz, uncompressed) and its manifest
    to ``path + '.sha256.json'``; returns the instance digest."""
    import json
    arrays = {k: np.ascontiguousarray(inst[k]) for k in ARRAYS}
    if "xstar" in inst:
        arrays["xstar"] = np.ascontiguousarray(inst["xstar"])
    with open(path, "wb") as fh:
        np.savez(fh, m=np.int64(inst["m"]), n=np.int64(inst["n"]), **arrays)
    man = _manifest(inst)
    with open(path + ".sha256.json", "w") as fh:
        json.dump(man, fh, indent=1, sort_keys=True)
    return man["sha256"]


def load(path: str, verify: bool = True) -> dict:
    """Read an instance written by ``save``; with ``verify`` every array is
    checked against the manifest (ValueError on a mismatch or a missing
    manifest)."""
    import json
    with np.load(path, allow_pickle=False) as z:
        inst = {k: z[k] for k in z.files}
    inst["m"] = int(inst["m"])
    inst["n"] = int(inst["n"])
    if verify:
        try:
            with open(path + ".sha256.json") as fh:
                want = json.load(fh)
        except FileNotFoundError:
            raise ValueError("no manifest beside %s" % path)
        got = _manifest(inst)
        if got != want:
            bad = [k for k in ARRAYS if got["arrays"][k] != want["arrays"].get(k)]
            raise ValueError("instance %s does not match its manifest (%s)"
                             % (path, ", ".join(bad) or "sizes"))
    return inst
