// bp_lv.h -- batched propagation of many bound vectors of one instance,
// one vector per lane (part of bp_engine.hip's translation unit; the C ABI
// entry is bp_propagate_batch in include/bp.h).
//
// The rounds are those of the slot engine (Section 2.1 activities and
// bound updates, restricted to changed constraints), with the bound vectors
// of a batch laid side by side: the bound record of variable i in vector v
// sits at bnd[i * V + v].  A wave serves 64 consecutive vectors (a group):
// for a queued (row, group) task it reads each nonzero's column and
// coefficient once, as wave-uniform values, and the 64 vectors' bound
// records of that column as one contiguous 1 KB load.  The matrix is read
// once per group instead of once per vector, and no bound gather touches a
// line that holds no other vector's record.
//
// Worklists are 64-bit masks: rmask[par][g][k] has bit l set when vector
// g*64+l has row k queued.  The first vector to queue (k, g) appends k to
// the group's task list; the mask deduplicates the rest.  Rows of up to
// LV_SHORT nonzeros are one task; longer rows are split into chunks of
// LV_CHUNK nonzeros whose per-lane partial sums a second kernel combines.
// Per-vector counters and evidence are accumulated in lane registers and
// flushed once per wave, so no counter is hit by more than one atomic per
// wave.  Arithmetic, the order-free integer atomics, the certified sums
// and the exact fallback are those of the slot engine: a vector's result
// is the same whichever engine runs it.
//
// Overlay mode (the instance has a base box, as the bulk-rounding
// candidates do: each is the base with a few fixings): a vector's record of
// variable i is its own record only where dmask[g][i] has its lane set (it
// differs from the base), else the base's record.  A (row, group) task then
// reads per nonzero an 8-byte mask word and the 16-byte base record, both
// shared by the whole group (and the base by every group), and own records
// only for the lanes that differ: instead of 1 KB per nonzero and group,
// the records the vectors actually changed.
#pragma once

namespace bp {

// Nonzeros per chunk of a long row: every chunk task merges the partial
// states of all chunks of its row, so shorter chunks trade that merge
// (quadratic in the chunk count) against parallelism.  1024 was the
// fastest of 256-4096 on the bulk workload (both legs).
#ifndef BP_LV_CHUNK
#define BP_LV_CHUNK 1024
#endif
#ifndef BP_LV_UNROLL
#define BP_LV_UNROLL 8
#endif
#ifndef BP_LV_WAVES
#define BP_LV_WAVES 4  // waves per SIMD the row kernel's register budget targets
#endif
constexpr int LV_SHORT = 64;             // rows up to this length: one task
// Chunks queued for at most this many vectors of a group split their
// nonzeros over the wave, one vector at a time (lv_chunk_few; also the
// merge and candidates of k_lv_heavy).  1, 2, 4, 8, 16, 32 and 48 were
// timed on the multi-round bulk workload: 4 was the fastest.
#ifndef BP_LV_FEW
#define BP_LV_FEW 4
#endif
constexpr int LV_FEW = BP_LV_FEW;
constexpr int LV_CHUNK = BP_LV_CHUNK;    // nonzeros per chunk of longer rows
constexpr int LV_MAX_GROUPS = 128;       // batches of up to 8192 vectors
constexpr int LV_UNROLL = BP_LV_UNROLL;  // bound loads issued together

struct LvVec {
    int32_t state, status, rounds;
    int32_t row_bad_min, row_bad_count, var_bad_min;
    unsigned long long nnz, pending_rows, pending_nnz;
};

struct LvCtl {
    uint32_t round, done, active, pad_;
    uint32_t nshort[2][LV_MAX_GROUPS];  // short-row tasks per parity and group
    uint32_t nlong[2][LV_MAX_GROUPS];   // chunk tasks per parity and group
    uint32_t nchg[LV_MAX_GROUPS];       // variables with candidates this round
    unsigned long long stat_rows, stat_nnz, stat_vars, stat_written;
    unsigned long long stat_corr;  // chunk tasks summed as base plus corrections
};

struct LvParams {
    DInst I;
    double feastol, inttol, tau;
    int32_t force_exact, count_vars, max_rounds;
    int32_t B, V, NG;
    int32_t m, n;
    double2 *bnd;        // [n][V]
    const double2 *base; // [n] base records (overlay mode), else null
    uint64_t *dmask;     // [NG][n] lanes whose own record is valid (overlay mode)
    longlong2 *cand;     // [n][V] (lower key, upper key)
    uint64_t *vmask;     // [NG][n] vectors with a candidate for the variable
    uint64_t *rmask[2];  // [NG][m] vectors that have the row queued
    int32_t *qs[2];      // [NG][m] short-row tasks
    int2 *ql[2];         // [NG][lcap] chunk tasks (row, chunk)
    int64_t lcap;        // chunk tasks per group and parity (every chunk of every long row)
    Acc *lpart;          // [NG][lcap][2][64] per-lane partial (min, max) states
    double *lrng;        // [NG][lcap][64] per-lane partial widths
    uint64_t *lmask;     // [NG][lcap] queued vectors of the chunk's row
    int32_t *chg;        // [NG][n] variables with candidates this round
    uint64_t *touched;   // [NG][n] bound records read this round (counting only)
    uint32_t *rtouch;    // [m / 32] rows read this round by any group (counting only)
    LvVec *vec;          // [V]
    uint32_t *vbad;      // [V] vector has an infeasible row this round (set early, read relaxed)
    LvCtl *ctl;
    // overlay mode: each long-row chunk's sums at the base bounds, so that a
    // chunk whose nonzeros are mostly unchanged in every lane is summed as
    // the base plus each lane's corrections (null: always summed whole)
    const int32_t *lchunk0;  // [m] chunk id of chunk 0 of a long row
    const Acc *lbase;        // [chunks][2] (min, max) states at the base bounds
    const double *lbw;       // [chunks] largest nonzero width at the base bounds
};

// A vector with an infeasible row in the current round finishes at its end
// with row evidence and unspecified bounds: its candidates can change
// nothing, so they are skipped once the flag is seen.  The flag only goes
// from 0 to 1 within a round; a stale read merely computes them anyway.
__device__ __forceinline__ bool lv_known_bad(const LvParams &P, int v) {
    return __hip_atomic_load(&P.vbad[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

__device__ __forceinline__ void lv_mark_bad(const LvParams &P, int v, bool bad, bool &flagged) {
    if (bad && !flagged) {
        __hip_atomic_store(&P.vbad[v], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        flagged = true;
    }
}

__device__ __forceinline__ int rl_i32(int x, int t) { return __builtin_amdgcn_readlane(x, t); }
__device__ __forceinline__ uint64_t rl_u64(uint64_t x, int t) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, t);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), t);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double rl_f64(double x, int t) {
    long long b = __double_as_longlong(x);
    int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, t);
    int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), t);
    return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The record of variable i for the lane's vector v (group g): its own, or
// in overlay mode the base's where its lane is not marked.  The mask word
// and the base record are the same for the whole wave.
__device__ __forceinline__ double2 lv_rec(const LvParams &P, int g, int i, int v) {
    if (!P.base) return P.bnd[(size_t)i * P.V + v];
    const uint64_t dm = P.dmask[(size_t)g * P.n + i];
    const double2 b0 = P.base[i];
    return ((dm >> (v & 63)) & 1ull) ? P.bnd[(size_t)i * P.V + v] : b0;
}

// Wave-local buffer of appends to one list: lane j holds the j-th pending
// entry; 64 entries (or the end of the wave's work) cost one atomic.
struct WaveBuf {
    int32_t val;
    int n;  // wave-uniform
};

__device__ __forceinline__ void wbuf_flush(WaveBuf &w, uint32_t *counter, int32_t *list) {
    if (w.n == 0) return;
    uint32_t base = 0;
    if (__lane_id() == 0) base = atomicAdd(counter, (uint32_t)w.n);
    base = __shfl(base, 0, 64);
    if (__lane_id() < w.n) list[base + __lane_id()] = w.val;
    w.n = 0;
}

// Append x (a wave-uniform value) to the buffer.
__device__ __forceinline__ void wbuf_push(WaveBuf &w, int32_t x, uint32_t *counter, int32_t *list) {
    if (__lane_id() == w.n) w.val = x;
    w.n += 1;
    if (w.n == 64) wbuf_flush(w, counter, list);
}

// Exact activity of one side of row [p0, p1) for the vector of this lane.
// The arrays come by value (not the parameter block by reference, which
// would make every lane copy it to scratch memory on entry).
__device__ __noinline__ double lv_exact_side(const double *val, const int32_t *col,
                                             const double2 *bnd, const double2 *base,
                                             const uint64_t *dm, int64_t V, int v, int64_t p0,
                                             int64_t p1, bool maxside) {
    SuperAcc S;
    sa_zero(S);
    for (int64_t p = p0; p < p1; ++p) {
        double a = val[p];
        const int i = col[p];
        double2 b = (base && !((dm[i] >> (v & 63)) & 1ull)) ? base[i] : bnd[(size_t)i * V + v];
        double bb = (a > 0.0) != maxside ? b.x : b.y;
        if (!isinf(bb)) sa_add(S, a * bb);
    }
    return canon0(sa_round(S));
}

// Per-wave counts of a counting run: row tasks, their nonzeros, distinct
// bound records read.  Flushed once per wave.
struct LvCount {
    unsigned long long rows, nnz, vars;
};

__device__ __forceinline__ void lv_count_read(const LvParams &P, int g, int i, uint64_t live,
                                              LvCount &K) {
    if (!P.count_vars || live == 0) return;
    uint64_t old = 0;
    if (__lane_id() == 0) old = atomicOr((unsigned long long *)&P.touched[(size_t)g * P.n + i], live);
    old = __shfl(old, 0, 64);
    K.vars += (unsigned long long)__popcll(live & ~old);
}

// The matrix term counts a row once per round over all groups (the row is
// shared by the whole batch).
__device__ __forceinline__ void lv_count_row(const LvParams &P, int k, int64_t len, LvCount &K) {
    if (!P.count_vars) return;
    uint32_t old = 0;
    if (__lane_id() == 0) old = atomicOr(&P.rtouch[k >> 5], 1u << (k & 31));
    old = __shfl(old, 0, 64);
    if (!((old >> (k & 31)) & 1u)) {
        K.rows += 1;
        K.nnz += (unsigned long long)len;
    }
}

__device__ __forceinline__ void lv_count_flush(const LvParams &P, const LvCount &K) {
    if (!P.count_vars || __lane_id() != 0) return;
    if (K.rows) atomicAdd(&P.ctl->stat_rows, K.rows);
    if (K.nnz) atomicAdd(&P.ctl->stat_nnz, K.nnz);
    if (K.vars) atomicAdd(&P.ctl->stat_vars, K.vars);
}

// Bound records of the nonzeros t0 .. t0 + LV_UNROLL - 1 of a block (column
// of nonzero t in lane t of cj) for the lane's vector when `need`, issued
// together: in overlay mode the mask words and base records first (the
// same for the whole wave), then the own records of the marked lanes.
__device__ __forceinline__ void lv_load(const LvParams &P, int g, int v, bool need, int cj, int t0,
                                        int len, double2 (&b)[LV_UNROLL]) {
    if (!P.base) {
#pragma unroll
        for (int u = 0; u < LV_UNROLL; ++u) {
            b[u] = make_double2(0.0, 0.0);
            if (t0 + u < len && need) b[u] = P.bnd[(size_t)rl_i32(cj, t0 + u) * P.V + v];
        }
        return;
    }
    uint64_t dm[LV_UNROLL];
    const uint64_t *dg = P.dmask + (size_t)g * P.n;
#pragma unroll
    for (int u = 0; u < LV_UNROLL; ++u) {
        dm[u] = 0ull;
        b[u] = make_double2(0.0, 0.0);
        if (t0 + u < len) {
            const int i = rl_i32(cj, t0 + u);
            dm[u] = dg[i];
            b[u] = P.base[i];
        }
    }
#pragma unroll
    for (int u = 0; u < LV_UNROLL; ++u)
        if (t0 + u < len && need && ((dm[u] >> (v & 63)) & 1ull))
            b[u] = P.bnd[(size_t)rl_i32(cj, t0 + u) * P.V + v];
}

// The two sides' terms of one nonzero, as add_terms computes them but
// without branches: an infinite bound is counted and adds +0.0, which
// leaves the state's exact value and error bound as they were (at most
// the sign of a zero sum changes, and results store zeros as +0.0).
__device__ __forceinline__ void lv_add_terms(Acc &mn, Acc &mx, double a, double lb, double ub) {
    const bool pos = a > 0.0;
    const double bmin = pos ? lb : ub, bmax = pos ? ub : lb;
    const bool imin = isinf(bmin), imax = isinf(bmax);
    mn.ninf += imin ? 1 : 0;
    mx.ninf += imax ? 1 : 0;
    acc_add(mn, imin ? 0.0 : a * bmin);
    acc_add(mx, imax ? 0.0 : a * bmax);
}

// The two sides' terms of one nonzero at the given bounds taken out again
// (the exact negations of what lv_add_terms adds; an infinite bound is
// uncounted).
__device__ __forceinline__ void lv_sub_terms(Acc &mn, Acc &mx, double a, double lb, double ub) {
    const bool pos = a > 0.0;
    const double bmin = pos ? lb : ub, bmax = pos ? ub : lb;
    const bool imin = isinf(bmin), imax = isinf(bmax);
    mn.ninf -= imin ? 1 : 0;
    mx.ninf -= imax ? 1 : 0;
    acc_add(mn, imin ? 0.0 : -(a * bmin));
    acc_add(mx, imax ? 0.0 : -(a * bmax));
}

// Activity over nonzeros [q0, q1) of a row (at most 64 per block), for the
// lanes in `live`.  Columns and coefficients are loaded once per block,
// one per lane, and broadcast; bound records are loaded LV_UNROLL at a time.
__device__ __forceinline__ void lv_accumulate(const LvParams &P, int g, int v, bool live,
                                              uint64_t livemask, int64_t q0, int64_t q1, Acc &mn,
                                              Acc &mx, double &wmax, LvCount &K) {
    for (int64_t b0 = q0; b0 < q1; b0 += 64) {
        const int len = (int)min((int64_t)64, q1 - b0);
        int cj = 0;
        double aj = 0.0;
        if (__lane_id() < len) {
            cj = P.I.col[b0 + __lane_id()];
            aj = P.I.val[b0 + __lane_id()];
        }
        for (int t0 = 0; t0 < len; t0 += LV_UNROLL) {
            double2 b[LV_UNROLL];
            lv_load(P, g, v, live, cj, t0, len, b);
#pragma unroll
            for (int u = 0; u < LV_UNROLL; ++u) {
                if (t0 + u < len) {
                    // every lane accumulates, without branches; the states
                    // of lanes that are not live are never read
                    double a = rl_f64(aj, t0 + u);
                    lv_add_terms(mn, mx, a, b[u].x, b[u].y);
                    wmax = fmax(wmax, nz_width(a, b[u].x, b[u].y));
                    lv_count_read(P, g, rl_i32(cj, t0 + u), livemask, K);
                }
            }
        }
    }
}

// Candidates of nonzeros [q0, q1) for the lanes in `want`; variables that
// receive a significant candidate are marked in vmask and listed.
__device__ __forceinline__ void lv_candidates(const LvParams &P, int g, int v, bool want,
                                              const RowAct &R, int64_t q0, int64_t q1, WaveBuf &wb) {
    if (__ballot(want) == 0) return;
    for (int64_t b0 = q0; b0 < q1; b0 += 64) {
        const int len = (int)min((int64_t)64, q1 - b0);
        int cj = 0;
        double aj = 0.0;
        if (__lane_id() < len) {
            cj = P.I.col[b0 + __lane_id()];
            aj = P.I.val[b0 + __lane_id()];
        }
        for (int t0 = 0; t0 < len; t0 += LV_UNROLL) {
            double2 b[LV_UNROLL];
            lv_load(P, g, v, want, cj, t0, len, b);
#pragma unroll
            for (int u = 0; u < LV_UNROLL; ++u) {
                if (t0 + u < len) {
                    const int i = rl_i32(cj, t0 + u);
                    const double a = rl_f64(aj, t0 + u);
                    bool pass = false;
                    if (want) {
                        const bool is_int = P.I.vtype[i] != 0;
                        double cl, cu;
                        nz_candidates(R, a, b[u].x, b[u].y, is_int, P.inttol, cl, cu);
                        longlong2 *cp = &P.cand[(size_t)i * P.V + v];
                        if (take_lower(is_int, cl, b[u].x, P.tau)) {
                            atomicMax(&cp->x, dkey(canon0(cl)));
                            pass = true;
                        }
                        if (take_upper(is_int, cu, b[u].y, P.tau)) {
                            atomicMin(&cp->y, dkey(canon0(cu)));
                            pass = true;
                        }
                    }
                    const uint64_t pm = __ballot(pass);
                    if (pm) {
                        uint64_t old = 0;
                        if (__lane_id() == 0)
                            old = atomicOr((unsigned long long *)&P.vmask[(size_t)g * P.n + i], pm);
                        old = __shfl(old, 0, 64);
                        if (old == 0) wbuf_push(wb, i, &P.ctl->nchg[g], P.chg + (size_t)g * P.n);
                    }
                }
            }
        }
    }
}

// Candidates of nonzeros [q0, q1) for few vectors (the lanes in wantmask):
// one vector at a time, the wave spread over the nonzeros.  The same keys,
// masks and changed-list entries as lv_candidates: a variable enters the
// group's list once, from the first vector whose bit it gets.
__device__ void lv_candidates_few(const LvParams &P, int g, uint64_t wantmask, const RowAct &R, int64_t q0,
                                  int64_t q1) {
    const int lane = __lane_id();
    const uint64_t *dg = P.dmask + (size_t)g * P.n;
    for (uint64_t rest = wantmask; rest; rest &= rest - 1) {
        const int vl = __ffsll((long long)rest) - 1;  // uniform
        const size_t v = (size_t)g * 64 + vl;
        RowAct Rv;
        Rv.lo = __shfl(R.lo, vl, 64);
        Rv.hi = __shfl(R.hi, vl, 64);
        Rv.minfin = __shfl(R.minfin, vl, 64);
        Rv.maxfin = __shfl(R.maxfin, vl, 64);
        Rv.rng = __shfl(R.rng, vl, 64);
        Rv.nmin = __shfl(R.nmin, vl, 64);
        Rv.nmax = __shfl(R.nmax, vl, 64);
        for (int64_t b0 = q0; b0 < q1; b0 += 64) {
            const int64_t p = b0 + lane;
            bool push = false;
            int i = 0;
            if (p < q1) {
                i = P.I.col[p];
                const double a = P.I.val[p];
                double2 b;
                if (P.base) b = ((dg[i] >> vl) & 1ull) ? P.bnd[(size_t)i * P.V + v] : P.base[i];
                else b = P.bnd[(size_t)i * P.V + v];
                const bool is_int = P.I.vtype[i] != 0;
                double cl, cu;
                nz_candidates(Rv, a, b.x, b.y, is_int, P.inttol, cl, cu);
                longlong2 *cp = &P.cand[(size_t)i * P.V + v];
                bool pass = false;
                if (take_lower(is_int, cl, b.x, P.tau)) {
                    atomicMax(&cp->x, dkey(canon0(cl)));
                    pass = true;
                }
                if (take_upper(is_int, cu, b.y, P.tau)) {
                    atomicMin(&cp->y, dkey(canon0(cu)));
                    pass = true;
                }
                if (pass)
                    push = atomicOr((unsigned long long *)&P.vmask[(size_t)g * P.n + i], 1ull << vl) == 0ull;
            }
            const uint64_t pm = __ballot(push);
            if (pm) {
                uint32_t at = 0;
                if (lane == 0) at = atomicAdd(&P.ctl->nchg[g], (uint32_t)__popcll(pm));
                at = __shfl(at, 0, 64);
                if (push) P.chg[(size_t)g * P.n + at + lane_rank(pm)] = i;
            }
        }
    }
}

// Certified activities of the lane's vector, with the exact fallback.
__device__ __forceinline__ void lv_finish_act(const LvParams &P, int v, bool live, Acc &mn, Acc &mx,
                                              int64_t p0, int64_t p1, RowAct &R) {
    R.nmin = mn.ninf;
    R.nmax = mx.ninf;
    R.minfin = 0.0;
    R.maxfin = 0.0;
    bool ok_min = live && !P.force_exact && acc_certify(mn, R.minfin);
    bool ok_max = live && !P.force_exact && acc_certify(mx, R.maxfin);
    const uint64_t *dm = P.base ? P.dmask + (size_t)(v >> 6) * P.n : nullptr;
    if (live && !ok_min) R.minfin = lv_exact_side(P.I.val, P.I.col, P.bnd, P.base, dm, P.V, v, p0, p1, false);
    if (live && !ok_max) R.maxfin = lv_exact_side(P.I.val, P.I.col, P.bnd, P.base, dm, P.V, v, p0, p1, true);
}

// One short row for the 64 vectors of group g: activity, row test and
// candidates in one task.
__device__ void lv_short_row(const LvParams &P, int par, int g, int v, bool active, int k,
                             int &bad_min, int &bad_cnt, bool &flagged, WaveBuf &wb, LvCount &K) {
    uint64_t *mp = &P.rmask[par][(size_t)g * P.m + k];
    const uint64_t word = *mp;
    const uint64_t livemask = word & __ballot(active);
    const bool live = (livemask >> __lane_id()) & 1ull;
    const bool kb = live && lv_known_bad(P, v);
    const int64_t p0 = P.I.row_ptr[k], p1 = P.I.row_ptr[k + 1];
    const double2 sd = P.I.side[k];
    if (__lane_id() == 0) *mp = 0ull;  // the word is queued again only by a later round
    lv_count_row(P, k, p1 - p0, K);
    Acc mn, mx;
    acc_zero(mn);
    acc_zero(mx);
    double wmax = 0.0;
    lv_accumulate(P, g, v, live, livemask, p0, p1, mn, mx, wmax, K);
    RowAct R;
    lv_finish_act(P, v, live, mn, mx, p0, p1, R);
    R.lo = sd.x;
    R.hi = sd.y;
    R.rng = wmax;
    bool bad = false;
    if (live) {
        bad = row_bad(R, P.feastol);
        if (bad) {
            bad_min = min(bad_min, k);
            bad_cnt += 1;
        }
        lv_mark_bad(P, v, bad, flagged);
    }
    const bool want = live && !bad && !kb && !flagged && !row_quiet(R);
    lv_candidates(P, g, v, want, R, p0, p1, wb);
}

// Chunk activity when the row is queued for few vectors of the group: the
// wave splits the chunk's nonzeros instead of the vectors, one live vector
// at a time, and the lanes' states are merged across the wave.  The sums
// are correctly rounded exact sums, so the certified values are those of
// the one-lane-per-vector loop; lane l ends with the state of vector l (a
// zero state when l is not live).  Distinct records read are counted once
// per nonzero for the whole live mask, as that loop counts them.
__device__ void lv_chunk_few(const LvParams &P, int g, uint64_t livemask, int64_t q0, int64_t q1, Acc &own_mn,
                             Acc &own_mx, double &own_w, LvCount &K) {
    const int lane = __lane_id();
    acc_zero(own_mn);
    acc_zero(own_mx);
    own_w = 0.0;
    const uint64_t *dg = P.dmask + (size_t)g * P.n;
    unsigned long long reads = 0;
    bool first = true;
    for (uint64_t rest = livemask; rest; rest &= rest - 1, first = false) {
        const int vl = __ffsll((long long)rest) - 1;  // uniform
        const size_t v = (size_t)g * 64 + vl;
        Acc mn, mx;
        acc_zero(mn);
        acc_zero(mx);
        double w = 0.0;
        for (int64_t p = q0 + lane; p < q1; p += 64) {
            const int i = P.I.col[p];
            const double a = P.I.val[p];
            double2 b;
            if (P.base) b = ((dg[i] >> vl) & 1ull) ? P.bnd[(size_t)i * P.V + v] : P.base[i];
            else b = P.bnd[(size_t)i * P.V + v];
            lv_add_terms(mn, mx, a, b.x, b.y);
            w = fmax(w, nz_width(a, b.x, b.y));
            if (first && P.count_vars) {
                const uint64_t old = atomicOr((unsigned long long *)&P.touched[(size_t)g * P.n + i], livemask);
                reads += (unsigned long long)__popcll(livemask & ~old);
            }
        }
        acc_group_reduce<64>(mn);
        acc_group_reduce<64>(mx);
        w = group_max<64>(w);
        if (lane == vl) {
            own_mn = mn;
            own_mx = mx;
            own_w = w;
        }
    }
    if (P.count_vars) {
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) reads += __shfl_xor(reads, o, 64);
        if (lane == 0) K.vars += reads;
    }
}

// Chunk partial states as the chunk's sums at the base bounds (chunk id
// `id`) plus each lane's corrections: for every nonzero whose variable some
// live lane has changed (its mask bit set; the word is the same for the
// whole wave, so unchanged nonzeros cost no arithmetic), those lanes add
// their own terms and take out the base terms.  The exact sums are those of
// the lane's own records over the chunk.  The width is the base's, or a
// changed nonzero's own when larger: a bound on the lane's widths.
__device__ void lv_chunk_corr(const LvParams &P, int g, int v, uint64_t livemask, int64_t q0, int64_t q1,
                              int64_t id, Acc &mn, Acc &mx, double &wmax) {
    const int lane = __lane_id();
    const uint64_t *dg = P.dmask + (size_t)g * P.n;
    acc_zero(mn);
    acc_zero(mx);
    double w = 0.0;
    for (int64_t b0 = q0; b0 < q1; b0 += 64) {
        const int64_t p = b0 + lane;
        int i = 0;
        double a = 0.0;
        uint64_t dm = 0;
        if (p < q1) {
            i = P.I.col[p];
            a = P.I.val[p];
            dm = dg[i] & livemask;
        }
        uint64_t any = __ballot(dm != 0);
        while (any) {
            const int q = __ffsll((long long)any) - 1;  // uniform
            any &= any - 1;
            const uint64_t wq = rl_u64(dm, q);
            const int iq = rl_i32(i, q);
            const double aq = rl_f64(a, q);
            const double2 bb = P.base[iq];
            if ((wq >> lane) & 1ull) {
                const double2 bo = P.bnd[(size_t)iq * P.V + v];
                lv_add_terms(mn, mx, aq, bo.x, bo.y);
                lv_sub_terms(mn, mx, aq, bb.x, bb.y);
                w = fmax(w, nz_width(aq, bo.x, bo.y));
            }
        }
    }
    const Acc bmn = P.lbase[2 * id], bmx = P.lbase[2 * id + 1];
    acc_merge(mn, bmn.s, bmn.c, bmn.e, bmn.ninf);
    acc_merge(mx, bmx.s, bmx.c, bmx.e, bmx.ninf);
    wmax = fmax(w, P.lbw[id]);
}

// Chunk c of a long row: per-lane partial states.
__device__ void lv_chunk_activity(const LvParams &P, int par, int g, int v, bool active, uint32_t u,
                                  LvCount &K) {
    const int2 rec = P.ql[par][(size_t)g * P.lcap + u];
    const int k = rec.x, c = rec.y;
    const uint64_t livemask = P.rmask[par][(size_t)g * P.m + k] & __ballot(active);
    const bool live = (livemask >> __lane_id()) & 1ull;
    const int64_t r0 = P.I.row_ptr[k], r1 = P.I.row_ptr[k + 1];
    const int64_t q0 = r0 + (int64_t)c * LV_CHUNK, q1 = min(r1, q0 + (int64_t)LV_CHUNK);
    if (__lane_id() == 0) P.lmask[(size_t)g * P.lcap + u] = livemask;
    if (c == 0) lv_count_row(P, k, r1 - r0, K);
    Acc mn, mx;
    double wmax = 0.0;
    bool corr = false;
    if (__popcll(livemask) > LV_FEW && P.lbase && !P.count_vars) {
        // base plus corrections when fewer than half of the chunk's
        // nonzeros are changed in some live lane (each costs four terms
        // there, two in the whole sum); counting runs sum whole
        const uint64_t *dg = P.dmask + (size_t)g * P.n;
        int64_t dirty = 0;
        for (int64_t b0 = q0; b0 < q1; b0 += 64) {
            const int64_t p = b0 + __lane_id();
            const bool d = p < q1 && (dg[P.I.col[p]] & livemask) != 0;
            dirty += __popcll(__ballot(d));
        }
        corr = 2 * dirty < q1 - q0;
    }
    if (__popcll(livemask) <= LV_FEW) {
        lv_chunk_few(P, g, livemask, q0, q1, mn, mx, wmax, K);
    } else if (corr) {
        lv_chunk_corr(P, g, v, livemask, q0, q1, (int64_t)P.lchunk0[k] + c, mn, mx, wmax);
        if (__lane_id() == 0) atomicAdd(&P.ctl->stat_corr, 1ull);
    } else {
        acc_zero(mn);
        acc_zero(mx);
        lv_accumulate(P, g, v, live, livemask, q0, q1, mn, mx, wmax, K);
    }
    const size_t base = ((size_t)g * P.lcap + u) * 128;
    P.lpart[base + __lane_id()] = mn;
    P.lpart[base + 64 + __lane_id()] = mx;
    P.lrng[((size_t)g * P.lcap + u) * 64 + __lane_id()] = wmax;
}

// Row kernel: chunk partials of long rows, then short rows.  Grid (x, NG).
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(BP_LV_WAVES))) k_lv_rows(LvParams P) {
    LvCtl *C = P.ctl;
    if (C->done) return;
    const int par = C->round & 1;
    const int g = blockIdx.y;
    const int v = g * 64 + __lane_id();
    const bool active = P.vec[v].state == SLOT_ACTIVE;
    const uint32_t nw = gridDim.x * (WG / 64);
    const uint32_t w = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    const uint32_t nl = C->nlong[par][g], ns = C->nshort[par][g];
    int bad_min = NONE, bad_cnt = 0;
    bool flagged = false;
    WaveBuf wb;
    wb.val = 0;
    wb.n = 0;
    LvCount K = {0ull, 0ull, 0ull};
    for (uint32_t t = w; t < nl + ns; t += nw) {
        if (t < nl) lv_chunk_activity(P, par, g, v, active, t, K);
        else lv_short_row(P, par, g, v, active, P.qs[par][(size_t)g * P.m + (t - nl)], bad_min, bad_cnt,
                          flagged, wb, K);
    }
    wbuf_flush(wb, &C->nchg[g], P.chg + (size_t)g * P.n);
    lv_count_flush(P, K);
    if (bad_cnt) {
        atomicMin(&P.vec[v].row_bad_min, bad_min);
        atomicAdd(&P.vec[v].row_bad_count, bad_cnt);
    }
}

// Long rows: each chunk task combines the row's partials (lane-wise, in
// chunk order), tests the row and computes the chunk's candidates.
__global__ void __launch_bounds__(WG) k_lv_heavy(LvParams P) {
    LvCtl *C = P.ctl;
    if (C->done) return;
    const int par = C->round & 1;
    const int g = blockIdx.y;
    const int v = g * 64 + __lane_id();
    const bool active = P.vec[v].state == SLOT_ACTIVE;
    const uint32_t nw = gridDim.x * (WG / 64);
    const uint32_t w = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    const uint32_t nl = C->nlong[par][g];
    int bad_min = NONE, bad_cnt = 0;
    bool flagged = false;
    WaveBuf wb;
    wb.val = 0;
    wb.n = 0;
    for (uint32_t u = w; u < nl; u += nw) {
        const int2 rec = P.ql[par][(size_t)g * P.lcap + u];
        const int k = rec.x, c = rec.y;
        const uint64_t livemask = P.lmask[(size_t)g * P.lcap + u];
        const bool live = ((livemask >> __lane_id()) & 1ull) && active;
        const bool kb = live && lv_known_bad(P, v);
        const int64_t r0 = P.I.row_ptr[k], r1 = P.I.row_ptr[k + 1];
        const int nch = (int)((r1 - r0 + LV_CHUNK - 1) / LV_CHUNK);
        const uint32_t u0 = u - (uint32_t)c;
        if (c == 0 && __lane_id() == 0) P.rmask[par][(size_t)g * P.m + k] = 0ull;
        Acc A, Bm;
        acc_zero(A);
        acc_zero(Bm);
        double wmax = 0.0;
        const uint64_t lm = __ballot(live);
        if (__popcll(lm) <= LV_FEW) {
            // few live vectors: one at a time, the lanes over the row's
            // chunks, then a merge across the wave (exact sums: the
            // certified values do not depend on the merge order)
            for (uint64_t rest = lm; rest; rest &= rest - 1) {
                const int vl = __ffsll((long long)rest) - 1;  // uniform
                Acc a1, b1;
                acc_zero(a1);
                acc_zero(b1);
                double w1 = 0.0;
                for (int j = __lane_id(); j < nch; j += 64) {
                    const size_t base = ((size_t)g * P.lcap + u0 + j) * 128;
                    const Acc a = P.lpart[base + vl], b = P.lpart[base + 64 + vl];
                    acc_merge(a1, a.s, a.c, a.e, a.ninf);
                    acc_merge(b1, b.s, b.c, b.e, b.ninf);
                    w1 = fmax(w1, P.lrng[((size_t)g * P.lcap + u0 + j) * 64 + vl]);
                }
                acc_group_reduce<64>(a1);
                acc_group_reduce<64>(b1);
                w1 = group_max<64>(w1);
                if (__lane_id() == vl) {
                    A = a1;
                    Bm = b1;
                    wmax = w1;
                }
            }
        } else {
            for (int j = 0; j < nch; ++j) {
                const size_t base = ((size_t)g * P.lcap + u0 + j) * 128;
                Acc a = P.lpart[base + __lane_id()], b = P.lpart[base + 64 + __lane_id()];
                acc_merge(A, a.s, a.c, a.e, a.ninf);
                acc_merge(Bm, b.s, b.c, b.e, b.ninf);
                wmax = fmax(wmax, P.lrng[((size_t)g * P.lcap + u0 + j) * 64 + __lane_id()]);
            }
        }
        RowAct R;
        lv_finish_act(P, v, live, A, Bm, r0, r1, R);
        const double2 sd = P.I.side[k];
        R.lo = sd.x;
        R.hi = sd.y;
        R.rng = wmax;
        bool bad = false;
        if (live) {
            bad = row_bad(R, P.feastol);
            if (bad && c == 0) {
                bad_min = min(bad_min, k);
                bad_cnt += 1;
            }
            lv_mark_bad(P, v, bad, flagged);
        }
        const bool want = live && !bad && !kb && !flagged && !row_quiet(R);
        const int64_t q0 = r0 + (int64_t)c * LV_CHUNK, q1 = min(r1, q0 + (int64_t)LV_CHUNK);
        const uint64_t wantmask = __ballot(want);
        if (__popcll(wantmask) <= LV_FEW) {
            if (wantmask) lv_candidates_few(P, g, wantmask, R, q0, q1);
        } else {
            lv_candidates(P, g, v, want, R, q0, q1, wb);
        }
    }
    wbuf_flush(wb, &C->nchg[g], P.chg + (size_t)g * P.n);
    if (bad_cnt) {
        atomicMin(&P.vec[v].row_bad_min, bad_min);
        atomicAdd(&P.vec[v].row_bad_count, bad_cnt);
    }
}

// Bound updates of the round's candidates, and the rows of every changed
// variable queued for the next round.  With seed = 1 (before the first
// round) the listed variables count as changed for the vectors in their
// masks and their rows go to the first round's queues.  Grid (x, NG).
__global__ void __launch_bounds__(WG) k_lv_apply(LvParams P, int seed) {
    LvCtl *C = P.ctl;
    if (!seed && C->done) return;
    const int tgt = seed ? 0 : ((C->round & 1) ^ 1);
    const int g = blockIdx.y;
    const int lane = __lane_id();
    const int v = g * 64 + lane;
    const double INF = __builtin_inf();
    const LvVec &Vv = P.vec[v];
    const bool active = Vv.state == SLOT_ACTIVE && (seed || Vv.row_bad_count == 0);
    const uint32_t nw = gridDim.x * (WG / 64);
    const uint32_t w = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    const uint32_t total = C->nchg[g];
    unsigned long long my_rows = 0, my_nnz = 0;
    int var_bad = NONE;
    uint32_t written = 0;
    for (uint32_t e = w; e < total; e += nw) {
        const int i = P.chg[(size_t)g * P.n + e];
        uint64_t *vm = &P.vmask[(size_t)g * P.n + i];
        const uint64_t mask = *vm;
        const bool mine = (mask >> lane) & 1ull;
        bool go = false;
        if (seed) {
            go = mine && active;
        } else {
            longlong2 *cp = &P.cand[(size_t)i * P.V + v];
            long long kl = 0, ku = 0;
            if (mine) {
                kl = cp->x;
                ku = cp->y;
                *cp = make_longlong2(dkey(-INF), dkey(INF));
            }
            if (mine && active) {
                double2 *bp = &P.bnd[(size_t)i * P.V + v];
                const double2 b = lv_rec(P, g, i, v);
                const bool is_int = P.I.vtype[i] != 0;
                const double L = dunkey(kl), U = dunkey(ku);
                double nl = b.x, nu = b.y;
                bool ch = false;
                if (take_upper(is_int, U, b.y, P.tau)) { nu = canon0(U); ch = true; }
                if (take_lower(is_int, L, b.x, P.tau)) { nl = canon0(L); ch = true; }
                if (ch && nl > nu) {
                    if (is_int || nl - nu > P.feastol) var_bad = min(var_bad, i);
                    else nl = nu;
                }
                if (ch) {
                    *bp = make_double2(nl, nu);
                    go = true;
                }
            }
        }
        if (lane == 0) *vm = 0ull;
        const uint64_t gm = __ballot(go);
        written += __popcll(gm);
        if (gm == 0) continue;
        // overlay mode: the written records are the lanes' own from now on
        // (one wave handles a (variable, group) pair in a round)
        if (P.base && !seed && lane == 0) P.dmask[(size_t)g * P.n + i] |= gm;
        const int64_t c0 = P.I.col_ptr[i], c1 = P.I.col_ptr[i + 1];
        for (int64_t j0 = c0; j0 < c1; j0 += 64) {
            const int64_t j = j0 + lane;
            const bool has = j < c1;
            int k = 0;
            int64_t len = 0;
            uint64_t newb = 0;
            bool first = false;
            if (has) {
                k = P.I.col_row[j];
                len = P.I.row_ptr[k + 1] - P.I.row_ptr[k];
                const uint64_t old =
                    atomicOr((unsigned long long *)&P.rmask[tgt][(size_t)g * P.m + k], gm);
                newb = gm & ~old;
                first = old == 0;
            }
            // queue (k, g) once: short rows as one task, long rows as chunks
            const bool qshort = first && len <= LV_SHORT;
            const uint64_t sm = __ballot(qshort);
            if (sm) {
                const int leader = __ffsll((long long)sm) - 1;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(&C->nshort[tgt][g], (uint32_t)__popcll(sm));
                base = __shfl(base, leader, 64);
                if (qshort) P.qs[tgt][(size_t)g * P.m + base + lane_rank(sm)] = k;
            }
            if (first && len > LV_SHORT) {
                const int nch = (int)((len + LV_CHUNK - 1) / LV_CHUNK);
                uint32_t base = atomicAdd(&C->nlong[tgt][g], (uint32_t)nch);
                for (int c = 0; c < nch; ++c) P.ql[tgt][(size_t)g * P.lcap + base + c] = make_int2(k, c);
            }
            // per-vector counts of the newly queued rows
            uint64_t any = __ballot(newb != 0);
            while (any) {
                const int t = __ffsll((long long)any) - 1;
                any &= any - 1;
                const uint64_t nb = (uint64_t)(uint32_t)rl_i32((int)(uint32_t)newb, t) |
                                    ((uint64_t)(uint32_t)rl_i32((int)(uint32_t)(newb >> 32), t) << 32);
                const int lt = rl_i32((int)len, t);
                if ((nb >> lane) & 1ull) {
                    my_rows += 1;
                    my_nnz += (unsigned long long)lt;
                }
            }
        }
    }
    if (my_rows) {
        atomicAdd(&P.vec[v].pending_rows, my_rows);
        atomicAdd(&P.vec[v].pending_nnz, my_nnz);
    }
    if (var_bad != NONE) atomicMin(&P.vec[v].var_bad_min, var_bad);
    if (lane == 0 && written && !seed) atomicAdd(&C->stat_written, (unsigned long long)written);
}

// Round end for every vector (one workgroup).
__global__ void __launch_bounds__(WG) k_lv_end(LvParams P) {
    LvCtl *C = P.ctl;
    if (C->done) return;
    const int par = C->round & 1;
    __shared__ uint32_t s_active;
    if (threadIdx.x == 0) s_active = 0;
    __syncthreads();
    for (int v = threadIdx.x; v < P.V; v += WG) {
        LvVec &S = P.vec[v];
        P.vbad[v] = 0u;
        if (S.state != SLOT_ACTIVE) continue;
        bool fin = true;
        if (S.row_bad_count > 0 || S.var_bad_min != NONE) {
            S.status = 1;
        } else if (S.pending_rows == 0) {
            S.status = 0;
        } else if ((uint32_t)S.rounds >= (uint32_t)P.max_rounds) {
            S.status = 2;
        } else {
            fin = false;
            S.rounds += 1;
            S.nnz += S.pending_nnz;
            if (!P.count_vars) {  // counting runs count the tasks themselves
                atomicAdd(&C->stat_rows, S.pending_rows);
                atomicAdd(&C->stat_nnz, S.pending_nnz);
            }
            S.pending_rows = 0;
            S.pending_nnz = 0;
            atomicAdd(&s_active, 1u);
        }
        if (fin) S.state = SLOT_FREE;
    }
    if (P.count_vars) {
        size_t words = (size_t)P.NG * P.n;
        for (size_t t = threadIdx.x; t < words; t += WG) P.touched[t] = 0ull;
        for (size_t t = threadIdx.x; t < (size_t)(P.m + 31) / 32; t += WG) P.rtouch[t] = 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int g = 0; g < P.NG; ++g) {
            C->nshort[par][g] = 0;
            C->nlong[par][g] = 0;
            C->nchg[g] = 0;
        }
        C->active = s_active;
        C->round = C->round + 1;
        if (s_active == 0) C->done = 1;
    }
}

// ---------------------------------------------------------------------------
// Set-up kernels
// ---------------------------------------------------------------------------

// Bounds in: [B][n] row-major vectors to the [n][V] layout through a
// 64 x 64 LDS tile; crossed and NaN boxes per vector.  With a base
// (overlay mode) only records that differ from it are stored, and the
// lanes that hold one are marked in dmask.
__global__ void __launch_bounds__(WG) k_lv_pack(const double *lb, const double *ub, double2 *bnd,
                                                int32_t n, int32_t B, int32_t V, const uint8_t *vtype,
                                                double feastol, int32_t *box, const double2 *base,
                                                uint64_t *dmask) {
    __shared__ double2 tile[64][65];
    const int64_t tiles_i = (n + 63) / 64;
    const int ngv = V / 64;
    for (int64_t t = blockIdx.x; t < tiles_i * ngv; t += gridDim.x) {
        const int64_t i0 = (t / ngv) * 64;
        const int v0 = (int)(t % ngv) * 64;
        // read: 4 waves, each lane one variable, rows of vectors
        for (int r = threadIdx.x >> 6; r < 64; r += WG / 64) {
            const int v = v0 + r;
            const int64_t i = i0 + __lane_id();
            double2 b = make_double2(0.0, 0.0);
            if (v < B && i < n) {
                b = make_double2(canon0(lb[(size_t)v * n + i]), canon0(ub[(size_t)v * n + i]));
                if (isnan(b.x) || isnan(b.y)) atomicOr(&box[2 * v + 1], 1);
                const double slack = vtype[i] ? 0.0 : feastol;
                if (b.x > b.y + slack) atomicMin(&box[2 * v], (int32_t)i);
            }
            tile[r][__lane_id()] = b;
        }
        __syncthreads();
        for (int c = threadIdx.x >> 6; c < 64; c += WG / 64) {
            const int64_t i = i0 + c;
            if (i >= n) continue;  // wave-uniform
            const double2 t = tile[__lane_id()][c];
            if (!base) {
                bnd[(size_t)i * V + v0 + __lane_id()] = t;
                continue;
            }
            const double2 b0 = base[i];
            const bool d = v0 + __lane_id() < B && (t.x != b0.x || t.y != b0.y);
            if (d) bnd[(size_t)i * V + v0 + __lane_id()] = t;
            const uint64_t m = __ballot(d);
            if (__lane_id() == 0) dmask[(size_t)(v0 >> 6) * n + i] = m;
        }
        __syncthreads();
    }
}

// Bounds out: [n][V] back to [B][n].  In overlay mode only the records the
// vectors hold of their own are written (the others equal the base, and
// so the input, which the arrays still hold).
__global__ void __launch_bounds__(WG) k_lv_unpack(const double2 *bnd, double *lb, double *ub,
                                                  int32_t n, int32_t B, int32_t V, const uint8_t *wmask,
                                                  const uint64_t *dmask) {
    __shared__ double2 tile[64][65];
    __shared__ uint64_t dms[64];
    const int64_t tiles_i = (n + 63) / 64;
    const int ngv = V / 64;
    for (int64_t t = blockIdx.x; t < tiles_i * ngv; t += gridDim.x) {
        const int64_t i0 = (t / ngv) * 64;
        const int v0 = (int)(t % ngv) * 64;
        // vectors whose bounds are written back (uniform over the tile)
        if (__ballot(wmask[v0 + __lane_id()] != 0) == 0) continue;
        for (int c = threadIdx.x >> 6; c < 64; c += WG / 64) {
            const int64_t i = i0 + c;
            const uint64_t dm = (dmask && i < n) ? dmask[(size_t)(v0 >> 6) * n + i] : ~0ull;
            const bool own = (dm >> __lane_id()) & 1ull;
            tile[__lane_id()][c] = (i < n && own) ? bnd[(size_t)i * V + v0 + __lane_id()] : make_double2(0.0, 0.0);
            if (__lane_id() == 0) dms[c] = dm;
        }
        __syncthreads();
        for (int r = threadIdx.x >> 6; r < 64; r += WG / 64) {
            const int v = v0 + r;
            const int64_t i = i0 + __lane_id();
            if (v < B && i < n && wmask[v] && ((dms[__lane_id()] >> r) & 1ull)) {
                const double2 b = tile[r][__lane_id()];
                lb[(size_t)v * n + i] = b.x;
                ub[(size_t)v * n + i] = b.y;
            }
        }
        __syncthreads();
    }
}

__global__ void k_lv_fill_cand(longlong2 *c, size_t N) {
    const double INF = __builtin_inf();
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N; j += (size_t)gridDim.x * blockDim.x)
        c[j] = make_longlong2(dkey(-INF), dkey(INF));
}

// 64 x 64 bit matrix held one row per lane (bit c of lane r's word is
// element (r, c)) transposed across the wave: lane c ends with column c.
// Stage j exchanges bit j of the row index with bit j of the column index
// (the off-diagonal j x j blocks of every 2j x 2j block swap); the six
// exchanges commute and together transpose.
__device__ __forceinline__ uint64_t wave_bit_transpose(uint64_t x) {
    const uint64_t M[6] = {0xAAAAAAAAAAAAAAAAull, 0xCCCCCCCCCCCCCCCCull, 0xF0F0F0F0F0F0F0F0ull,
                           0xFF00FF00FF00FF00ull, 0xFFFF0000FFFF0000ull, 0xFFFFFFFF00000000ull};
    const int lane = __lane_id();
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int j = 1 << s;
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, j, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), j, 64);
        const uint64_t y = ((uint64_t)hi << 32) | lo;
        x = (lane & j) ? ((x & M[s]) | ((y & M[s]) >> j)) : ((x & ~M[s]) | ((y & ~M[s]) << j));
    }
    return x;
}

// Bounds in, overlay mode: the same records, flags and mask words as
// k_lv_pack with a base, read without a transpose through LDS.  Tile: 64
// variables x one group; each wave takes 16 vectors, one coalesced load of
// lb and of ub per vector, compares with the base and ballots; the 64
// ballots (bit c: variable i0 + c) are transposed into one mask word per
// variable.  Only differing records are written.
__global__ void __launch_bounds__(WG) k_lv_pack_overlay(const double *lb, const double *ub, double2 *bnd,
                                                        int32_t n, int32_t B, int32_t V,
                                                        const uint8_t *vtype, double feastol, int32_t *box,
                                                        const double2 *base, uint64_t *dmask) {
    __shared__ uint64_t words[64];
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int64_t tiles_i = (n + 63) / 64;
    const int ngv = V / 64;
    for (int64_t t = blockIdx.x; t < tiles_i * ngv; t += gridDim.x) {
        const int64_t i0 = (t / ngv) * 64;
        const int v0 = (int)(t % ngv) * 64;
        const int64_t i = i0 + lane;
        const bool iin = i < n;
        double2 b0 = make_double2(0.0, 0.0);
        double slack = 0.0;
        if (iin) {
            b0 = base[i];
            slack = vtype[i] ? 0.0 : feastol;
        }
        // the wave's 16 vectors: every load issued before any use
        double l[16], u[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int v = v0 + wave * 16 + q;
            l[q] = 0.0;
            u[q] = 0.0;
            if (v < B && iin) {
                l[q] = lb[(size_t)v * n + i];
                u[q] = ub[(size_t)v * n + i];
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = wave * 16 + q, v = v0 + r;
            bool d = false;
            if (v < B && iin) {
                const double lq = canon0(l[q]), uq = canon0(u[q]);
                if (isnan(lq) || isnan(uq)) atomicOr(&box[2 * v + 1], 1);
                if (lq > uq + slack) atomicMin(&box[2 * v], (int32_t)i);
                d = lq != b0.x || uq != b0.y;
                if (d) bnd[(size_t)i * V + v] = make_double2(lq, uq);
            }
            const uint64_t m = __ballot(d);
            if (lane == 0) words[r] = m;
        }
        __syncthreads();
        if (wave == 0) {
            const uint64_t col = wave_bit_transpose(words[lane]);
            if (iin) dmask[(size_t)(v0 >> 6) * n + i] = col;
        }
        __syncthreads();
    }
}

// Every long-row chunk's (min, max) states and largest nonzero width at the
// base bounds (one wave per chunk; chunk id = index in the chunk table).
__global__ void __launch_bounds__(WG) k_lv_base_chunks(DInst I, const int2 *chunks, int64_t nchunks,
                                                       Acc *lbase, double *lbw) {
    const int64_t nw = (int64_t)gridDim.x * (WG / 64);
    for (int64_t id = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6); id < nchunks; id += nw) {
        const int2 ck = chunks[id];
        const int64_t r0 = I.row_ptr[ck.x], r1 = I.row_ptr[ck.x + 1];
        const int64_t q0 = r0 + (int64_t)ck.y * LV_CHUNK, q1 = min(r1, q0 + (int64_t)LV_CHUNK);
        Acc mn, mx;
        acc_zero(mn);
        acc_zero(mx);
        double w = 0.0;
        for (int64_t p = q0 + __lane_id(); p < q1; p += 64) {
            const double a = I.val[p];
            const double2 b = I.base[I.col[p]];
            lv_add_terms(mn, mx, a, b.x, b.y);
            w = fmax(w, nz_width(a, b.x, b.y));
        }
        acc_group_reduce<64>(mn);
        acc_group_reduce<64>(mx);
        w = group_max<64>(w);
        if (__lane_id() == 0) {
            lbase[2 * id] = mn;
            lbase[2 * id + 1] = mx;
            lbw[id] = w;
        }
    }
}

__global__ void k_lv_fill_u64(uint64_t *p, size_t N) {
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N; j += (size_t)gridDim.x * blockDim.x)
        p[j] = 0ull;
}

// Vectors: active unless their box is crossed (box[2v] != NONE).
__global__ void k_lv_reset(LvParams P, const int32_t *box) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < P.V; v += gridDim.x * blockDim.x) {
        LvVec &S = P.vec[v];
        S.state = (v < P.B && box[2 * v] == NONE) ? SLOT_ACTIVE : SLOT_FREE;
        S.status = 0;
        S.rounds = 0;
        S.row_bad_min = NONE;
        S.row_bad_count = 0;
        S.var_bad_min = NONE;
        S.nnz = 0;
        S.pending_rows = 0;
        S.pending_nnz = 0;
        P.vbad[v] = 0u;
    }
}

// Cold start: every row queued for every active vector.  short_rows and
// long_chunks list the instance's rows by class (long rows as (row, chunk)).
__global__ void k_lv_seed_cold(LvParams P, const int32_t *short_rows, int64_t nshort,
                               const int2 *long_chunks, int64_t nlong) {
    const int g = blockIdx.y;
    uint64_t lanes = 0;
    for (int l = 0; l < 64; ++l)
        if (P.vec[g * 64 + l].state == SLOT_ACTIVE) lanes |= 1ull << l;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nshort; j += (int64_t)gridDim.x * blockDim.x) {
        const int k = short_rows[j];
        P.qs[0][(size_t)g * P.m + j] = k;
        P.rmask[0][(size_t)g * P.m + k] = lanes;
    }
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nlong; j += (int64_t)gridDim.x * blockDim.x) {
        const int2 r = long_chunks[j];
        P.ql[0][(size_t)g * P.lcap + j] = r;
        if (r.y == 0) P.rmask[0][(size_t)g * P.m + r.x] = lanes;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.ctl->nshort[0][g] = (uint32_t)(lanes ? nshort : 0);
        P.ctl->nlong[0][g] = (uint32_t)(lanes ? nlong : 0);
    }
}

// Warm start: the listed variables of every vector (entries of
// changed_idx, vector v owning [ptr[v], ptr[v+1])) are marked in vmask and
// listed once per group; k_lv_apply with seed = 1 then queues their rows.
// lists = 0: only the (group, variable) masks are set (the rows are then
// queued by k_lv_seed_rows, and the masks cleared whole afterwards).
__global__ void k_lv_seed_vars(LvParams P, const int32_t *vars, const int64_t *ptr, int64_t e0,
                               int64_t total, int lists) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += stride) {
        const int64_t e = e0 + base + threadIdx.x;  // entry of vars; ptr is absolute
        const bool has = base + threadIdx.x < total;
        int v = 0, i = 0;
        bool first = false;
        if (has) {
            int lo = 0, hi = P.B;
            while (hi - lo > 1) {
                int mid = (lo + hi) / 2;
                if (ptr[mid] <= e) lo = mid;
                else hi = mid;
            }
            v = lo;
            i = vars[e];
            if (P.vec[v].state == SLOT_ACTIVE) {
                const uint64_t bit = 1ull << (v & 63);
                unsigned long long *w = (unsigned long long *)&P.vmask[(size_t)(v >> 6) * P.n + i];
                if (lists) first = atomicOr(w, bit) == 0;
                else atomicOr(w, bit);
            }
        }
        if (!lists) continue;  // uniform
        // one atomic per wave when the wave's new entries share a group
        const int g = v >> 6;
        const uint64_t fm = __ballot(first);
        if (fm) {
            const int leader = __ffsll((long long)fm) - 1;
            const int g0 = __shfl(g, leader, 64);
            if (__ballot(first && g != g0) == 0) {
                uint32_t b = 0;
                if (__lane_id() == leader) b = atomicAdd(&P.ctl->nchg[g0], (uint32_t)__popcll(fm));
                b = __shfl(b, leader, 64);
                if (first) P.chg[(size_t)g0 * P.n + b + lane_rank(fm)] = i;
            } else if (first) {
                uint32_t slot = atomicAdd(&P.ctl->nchg[g], 1u);
                P.chg[(size_t)g * P.n + slot] = i;
            }
        }
    }
}

// Warm start by rows (large changed lists): row k is queued for the
// vectors in the OR of its variables' masks.  One wave per row; no atomics
// on the masks.  Grid (x, NG).
__global__ void __launch_bounds__(WG) k_lv_seed_rows(LvParams P) {
    const int g = blockIdx.y;
    const int lane = __lane_id();
    const int v = g * 64 + lane;
    const uint64_t activemask = __ballot(P.vec[v].state == SLOT_ACTIVE);
    const uint32_t nw = gridDim.x * (WG / 64);
    const uint32_t w = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    unsigned long long my_rows = 0, my_nnz = 0;
    WaveBuf wb;
    wb.val = 0;
    wb.n = 0;
    for (uint32_t k = w; k < (uint32_t)P.m; k += nw) {
        const int64_t p0 = P.I.row_ptr[k], p1 = P.I.row_ptr[k + 1];
        uint64_t acc = 0;
        for (int64_t j = p0 + lane; j < p1; j += 64) acc |= P.vmask[(size_t)g * P.n + P.I.col[j]];
        uint32_t lo = (uint32_t)acc, hi = (uint32_t)(acc >> 32);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo |= (uint32_t)__shfl_xor((int)lo, o, 64);
            hi |= (uint32_t)__shfl_xor((int)hi, o, 64);
        }
        const uint64_t mask = (((uint64_t)hi << 32) | lo) & activemask;
        if (mask == 0) continue;
        const int64_t len = p1 - p0;
        if (lane == 0) P.rmask[0][(size_t)g * P.m + k] = mask;
        if (len <= LV_SHORT) {
            wbuf_push(wb, (int32_t)k, &P.ctl->nshort[0][g], P.qs[0] + (size_t)g * P.m);
        } else {
            const int nch = (int)((len + LV_CHUNK - 1) / LV_CHUNK);
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&P.ctl->nlong[0][g], (uint32_t)nch);
            base = __shfl(base, 0, 64);
            for (int c = lane; c < nch; c += 64) P.ql[0][(size_t)g * P.lcap + base + c] = make_int2((int)k, c);
        }
        if ((mask >> lane) & 1ull) {
            my_rows += 1;
            my_nnz += (unsigned long long)len;
        }
    }
    wbuf_flush(wb, &P.ctl->nshort[0][g], P.qs[0] + (size_t)g * P.m);
    if (my_rows) {
        atomicAdd(&P.vec[v].pending_rows, my_rows);
        atomicAdd(&P.vec[v].pending_nnz, my_nnz);
    }
}

// After seeding: first-round counters of every vector.
__global__ void k_lv_seed_finish(LvParams P, int cold, long long nnz) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < P.V; v += gridDim.x * blockDim.x) {
        LvVec &S = P.vec[v];
        if (S.state != SLOT_ACTIVE) continue;
        if (cold) {
            S.pending_rows = (unsigned long long)P.m;
            S.pending_nnz = (unsigned long long)nnz;
        }
        if (S.pending_rows == 0) {
            S.state = SLOT_FREE;
            S.status = 0;
        } else if (P.max_rounds <= 0) {
            S.state = SLOT_FREE;
            S.status = 2;
        } else {
            S.rounds = 1;
            S.nnz = S.pending_nnz;
            if (!P.count_vars) {
                atomicAdd(&P.ctl->stat_rows, S.pending_rows);
                atomicAdd(&P.ctl->stat_nnz, S.pending_nnz);
            }
            S.pending_rows = 0;
            S.pending_nnz = 0;
        }
    }
}

// After seeding: clear the variable lists, set the done flag.
__global__ void k_lv_start(LvParams P) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int v = threadIdx.x; v < P.V; v += blockDim.x)
        if (P.vec[v].state == SLOT_ACTIVE) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int g = 0; g < P.NG; ++g) P.ctl->nchg[g] = 0;
        P.ctl->done = any ? 0u : 1u;
        P.ctl->active = any ? 1u : 0u;
    }
}

// After the last round: rows queued for a round that never ran leave their
// mask words set; clear them so the masks start empty next time.
__global__ void k_lv_cleanup(LvParams P) {
    const int par = P.ctl->round & 1;
    const int g = blockIdx.y;
    const uint32_t ns = P.ctl->nshort[par][g], nl = P.ctl->nlong[par][g];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ns + nl; t += gridDim.x * blockDim.x) {
        const int k = t < ns ? P.qs[par][(size_t)g * P.m + t] : P.ql[par][(size_t)g * P.lcap + (t - ns)].x;
        P.rmask[par][(size_t)g * P.m + k] = 0ull;
    }
}

__global__ void k_lv_cleanup_counts(LvParams P) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int p = 0; p < 2; ++p)
            for (int g = 0; g < P.NG; ++g) {
                P.ctl->nshort[p][g] = 0;
                P.ctl->nlong[p][g] = 0;
            }
        for (int g = 0; g < P.NG; ++g) P.ctl->nchg[g] = 0;
    }
}

}  // namespace bp

// Device buffers of the one-vector-per-lane engine (sized for V lanes; a
// call with fewer vectors uses the same buffers with a smaller stride).
struct LvEngine {
    int32_t Vcap = 0;
    int64_t lcap = 0, nshort = 0, nlong = 0;
    bool have_touched = false;
    // long-row chunks at the base bounds (overlay mode): chunk id of each
    // long row's chunk 0, the chunks' states and widths, and the base
    // version they were summed for
    DevBuf lchunk0, lbase, lbw;
    int64_t lb_version = -1;
    DevBuf bnd, cand, vmask, dmask, rmask[2], qs[2], ql[2], lpart, lrng, lmask, chg, touched, rtouch, vec, vbad,
        ctl, box, wmask;
    DevBuf short_rows, long_chunks;  // cold-start tasks of the instance
    hipGraphExec_t graph = nullptr;
    int graph_rounds = 0;
    bp::LvParams graph_params;
    ~LvEngine() {
        if (graph) (void)hipGraphExecDestroy(graph);
    }
};
