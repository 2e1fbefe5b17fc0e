// bp_kernels.h -- HIP kernels for round-synchronous bound propagation.
//
// One round (the paper's Section 2.1: activities of the constraints, then
// bound updates) runs as kernels over a slot table.  A slot is one bound
// vector in flight: the vector of bp_propagate, one candidate of
// bp_propagate_batch, one probe of bp_probe, or one job of a serving
// request.  Slots may belong to different instances (serving); each slot's
// per-variable arrays have a fixed stride sized for the largest instance.
//
//   k_rows   (activity + candidates) every queued (slot, row) task of the
//            round: the row activity, the row infeasibility test and, for
//            light and block rows, the candidates of every nonzero,
//            scattered as order-independent 64-bit integer atomic min/max
//            into the slot's candidate array.  Only candidates that pass
//            the threshold against the round-start bounds are scattered:
//            the threshold is monotone in the candidate, so the tightest
//            candidate passes iff some candidate passes.  Heavy rows only
//            produce chunk partials here.
//   k_heavy  (candidates of heavy rows) combines the partials of each row,
//            tests it, and scatters the candidates of each chunk.
//   k_apply  (bound update) each (slot, variable) that received a
//            candidate: acceptance, crossing test, new bounds, and the rows
//            of the variable's column queued for the next round (the
//            paper's "propagation on changed constraints", Section 1).
//   k_end    per-slot round end (one workgroup).
//   k_retire (jobs only) results of finished jobs, slot restore, admission
//            of the next jobs into free slots.
//
// Rows are binned by length (logarithmic radix binning, Section 2.1 load
// balancing): bin b <= 10 holds rows of length in (2^(b-1), 2^b] and is
// processed by groups of G = min(64, 2^b) lanes of a 64-lane wave; bin 11
// holds rows up to the heavy threshold, one 256-lane workgroup per row;
// bin 12 holds heavy rows, split into chunks across workgroups.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bp_sum.h"
#include "bp_carry.h"

namespace bp {

constexpr int NLIGHT = 11;          // bins 0..10
constexpr int BIN_BLOCK = 11;
constexpr int BIN_HEAVY = 12;
constexpr int NBIN = 13;
constexpr int WG = 256;             // workgroup size of every kernel
constexpr int32_t NONE = 0x7fffffff;
constexpr int FILT_WORDS = 1024;    // 32768-bit dirty filter per slot (4 KB)
// A single bound vector spreads its changed list over this many stripes,
// one counter each, chosen by workgroup index: every such counter is hit by
// an eighth of the waves (same-address atomics serialise).
constexpr int NSTRIPE = 8;

enum : int32_t { SLOT_FREE = 0, SLOT_ACTIVE = 1, SLOT_DRAINING = 2 };

// Device view of one instance (read-only during propagation).
struct DInst {
    int32_t m, n;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
    const double2 *side;    // (lo, hi)
    const int64_t *col_ptr;
    const int32_t *col_row;
    const uint8_t *vtype;
    const uint8_t *rbin;
    const double2 *base;    // base bounds (jobs read them as an overlay)
    // heavy rows (incremental activities)
    const int32_t *hidx;    // [m] heavy index of a row, -1 for the others
    const double *cval;     // [nnz] coefficients in column order
    // the heavy rows at the base bounds (null until computed for the
    // current base): limbs [H][2][HL], infinite counts [H][2], widths [H]
    const long long *hblimb;
    const int32_t *hbinf;
    const double *hbwid;
};

// Per-slot bookkeeping.
struct SlotInfo {
    int32_t state;
    int32_t status;
    int32_t rounds;
    int32_t row_bad_min;
    int32_t row_bad_count;
    int32_t var_bad_min;
    int32_t pending_rows;
    int32_t job;        // job or vector index
    unsigned long long nnz;
    unsigned long long pending_nnz;
    int32_t retire;     // finished at the last round end, results not yet written
    int32_t inst;       // instance of the slot
    // Assigned by the round end of a job engine (valid while Ctl::claims is
    // set): the next job of a slot that is free (CLAIM_NONE: none left), and
    // the staging offset and completion-ring position of a finished job.
    int32_t claim;
    uint32_t ring_pos;
    unsigned long long stage_off;
};
constexpr int32_t CLAIM_NONE = -1;

// Round control block (one per engine).
struct Ctl {
    uint32_t round;             // rounds started by the engine (parity = round & 1)
    uint32_t done;
    uint32_t qcount[2][NBIN];   // queue lengths per parity
    uint32_t hchunks[2];        // heavy chunks per parity
    uint32_t nchanged[NSTRIPE]; // (slot, var) entries of the current round, per stripe
    uint32_t active;            // slots active or draining after the last round end
    uint32_t finished;          // slots finished at the last round end
    uint32_t max_rounds;
    uint32_t nslots;
    // jobs are admitted in order into free slots
    uint32_t next_job;
    uint32_t total_jobs;
    uint32_t done_jobs;              // entries of the completion ring
    uint32_t claims;                 // the slots' claim / staging fields are assigned
    unsigned long long stage_count;  // implied entries staged so far
    // cumulative counters (byte accounting)
    unsigned long long stat_rows;    // row tasks at round starts
    unsigned long long stat_nnz;     // their nonzeros
    unsigned long long stat_vars;    // distinct bound records read per round
    unsigned long long stat_written; // accepted bound changes
    unsigned long long stat_kept_rows;  // queued heavy rows tested from their accumulators
    unsigned long long stat_kept_nnz;   // nonzeros of those rows left unread (no candidates)
    unsigned long long stat_apply_entries;  // changed-list entries the update kernel took
    unsigned long long stat_apply_colent;   // column entries it walked for accepted changes
    unsigned long long stat_apply_corr;     // heavy-row accumulator corrections it made
    // scan rounds of one vector (see Params::scan_ok)
    uint32_t scan[2];                // the round of this parity scans every row
    uint32_t scan_go;                // a bound moved in the last scan-seeding bound update
    uint32_t pad2_;
    unsigned long long scan_rows[NSTRIPE], scan_nnz[NSTRIPE];  // rows a scan round processed
    // incremental heavy-row activities (see Params::inc)
    uint32_t hbuild[2];              // the round of this parity rebuilds them from the bounds
    uint32_t hcand[2];               // heavy chunk tasks that need candidates (heads decided)
    // distinct rows per round over all slots, and their nonzeros (byte
    // accounting of batches: a row read for several vectors counts once)
    unsigned long long stat_urows, stat_unnz;
};

// The leading fields of Ctl for the round in progress (its parity's queue
// lengths and chunk counts), read by the round kernels in one go: both
// parities are loaded and selected without indexing.
struct CtlHead {
    uint32_t round, done;
    uint32_t qcount[NBIN];
    uint32_t hchunks;
    uint32_t scan;
    uint32_t hbuild;
    uint32_t hcand;
};

// Keeps control loads ahead of the first branch on them, so that they are
// issued together rather than one memory round trip after another.
__device__ __forceinline__ void ctl_loaded(uint32_t a, uint32_t b, uint32_t c) {
    asm volatile("" ::"s"(a), "s"(b), "s"(c));
}

__device__ __forceinline__ CtlHead ctl_head(const Ctl *C) {
    CtlHead H;
    H.round = C->round;
    H.done = C->done;
    const bool odd = (H.round & 1u) != 0;
#pragma unroll
    for (int b = 0; b < NBIN; ++b) {
        const uint32_t q0 = C->qcount[0][b], q1 = C->qcount[1][b];
        H.qcount[b] = odd ? q1 : q0;
    }
    const uint32_t h0 = C->hchunks[0], h1 = C->hchunks[1];
    H.hchunks = odd ? h1 : h0;
    const uint32_t sc0 = C->scan[0], sc1 = C->scan[1];
    H.scan = odd ? sc1 : sc0;
    const uint32_t hb0 = C->hbuild[0], hb1 = C->hbuild[1];
    H.hbuild = odd ? hb1 : hb0;
    const uint32_t hc0 = C->hcand[0], hc1 = C->hcand[1];
    H.hcand = odd ? hc1 : hc0;
    return H;
}

struct Params {
    DInst I;                     // the instance when there is one
    const DInst *insts;          // per-instance table when slots mix instances
    int32_t multi;
    double feastol, inttol, tau;
    int32_t heavy_chunk;         // nonzeros per heavy chunk
    int32_t force_exact;
    int32_t nslots;
    int32_t sn;                  // variables per slot (stride of the per-variable arrays)
    int32_t snw, srw;            // 32-bit words per slot of the variable / row bitmaps
    double2 *bnd;                // [nslots][sn]
    longlong2 *cand;             // [nslots][sn] (lower key, upper key)
    uint32_t *vflag;             // [nslots][snw]
    uint32_t *rflag;             // [nslots][srw]
    SlotInfo *info;              // [nslots]
    uint64_t *q[2][NBIN];        // task queues (slot << 32 | row)
    int4 *hrec[2];               // heavy chunks: (slot, row, chunk index, chunks of the row)
    Acc *hpart;                  // [chunks][2] partial (min, max) states
    double *hrng;                // [chunks] partial widths (slack filter)
    uint64_t *chg;               // (slot << 32 | var) entries of the round, nstripe lists
    int32_t nstripe;             // 1, or NSTRIPE for an engine of one slot
    int64_t chg_stride;          // entries per stripe
    Ctl *ctl;
    uint32_t *touched;           // [nslots][snw] bound records read this round
                                 // (only when counting them)
    uint32_t *useen;             // [srw] rows read this round by any slot (only
                                 // when counting; one instance)
    // jobs: bounds are an overlay on the instance's base; a slot's own
    // record of var i is valid only where its dirty bit is set
    int32_t overlay;
    uint32_t *filt;              // [nslots][FILT_WORDS] hashed summary of the dirty bits
    uint32_t *dirty;             // [nslots][snw]
    int32_t *dlist;              // [nslots][sn]
    int32_t *dcount;             // [nslots]
    // Scan rounds (one plain vector): when a bound update changes many
    // variables, the next round does not queue rows through the columns;
    // instead the row kernel walks every row and processes those holding a
    // variable of the changed bitmap.  The set of rows is the same.
    int32_t scan_ok;             // the engine runs one plain vector
    uint32_t scan_min;           // changed entries from which the next round scans
    uint32_t *cbits;             // [2][snw] variables changed by the update feeding parity p
    const int32_t *allrows;      // every row, grouped by bin
    int64_t allstart[NBIN + 1];  // bin offsets in allrows
    const int4 *allhrec;         // chunk records of every heavy row
    int32_t allhchunks;
    uint32_t *hhit;              // [m] heavy row holds a changed variable (scan rounds)
    // Incremental heavy rows (one plain vector, or a cold start of up to
    // INC_SLOTS): the exact finite parts of each heavy row's min and max
    // activity live in carry-save fixed-point accumulators that every
    // accepted bound change corrects (its old term out, its new term in,
    // both exact), so a queued heavy row is tested without reading its
    // nonzeros.  The first round, and the round after an update of at least
    // inc_max changed entries (a scan-seeding one included), rebuild them
    // from the bounds instead.
    int32_t inc;                 // enabled
    int32_t nheavy;              // heavy rows
    int32_t inc_slots;           // slots with accumulators (the vectors of the call)
    long long *hacc;             // [slot][nheavy][2][HL] limbs (min side, max side)
    int32_t *hinf;               // [slot][nheavy][2] infinite contributions
    unsigned long long *hwid;    // [slot][nheavy] slack-filter width bound (bits of a double >= 0)
    double2 *hact;               // [slot][nheavy] the round's rounded (min, max) finite parts
    int4 *hcrec[2];              // chunk tasks of heavy rows whose head found candidates needed
    uint32_t inc_max;            // changed entries from which the next round rebuilds
    uint32_t inc_period;         // a rebuild at least every inc_period rounds, so that no
                                 // carry-save limb can reach 2^62 (see propagate_slots)
    // Incremental heavy rows of job slots (overlays on their instance's
    // base): a slot's limbs and infinite counts hold only the corrections of
    // its own bound changes, so a heavy row's activity is the base row's
    // exact sum (the instance's hblimb, hbinf) plus them, and the base width
    // bounds its width (a job's bounds lie inside the base).  Admission
    // corrects for the job's first bounds, the update kernel for every later
    // change, and a retired slot clears the rows of its changed variables.
    // Never rebuilt.
    int32_t inc_base;
};

// Instance of slot s (MULTI: slots mix instances; otherwise the kernel
// argument, uniform across the grid).
template <bool MULTI>
__device__ __forceinline__ DInst inst_of(const Params &P, int s) {
    if constexpr (MULTI) return P.insts[P.info[s].inst];
    else return P.I;
}

__device__ __forceinline__ uint32_t fhash(int i) { return ((uint32_t)i * 2654435761u) >> 17; }

// Bound records of one slot.  Outside jobs a slot owns a dense vector; a
// job reads the base except where its dirty bit is set (the small hashed
// filter answers "certainly clean" for almost every variable from cache).
struct BView {
    const double2 *own, *base;
    const uint32_t *filt, *dirty;
    int overlay;
    __device__ __forceinline__ double2 operator[](int i) const {
        if (!overlay) return own[i];
        double2 b = base[i];
        uint32_t h = fhash(i);
        if ((filt[h >> 5] >> (h & 31)) & 1u) {
            if ((dirty[i >> 5] >> (i & 31)) & 1u) b = own[i];
        }
        return b;
    }
};

__device__ __forceinline__ BView bview(const Params &P, int s, const double2 *base) {
    BView v;
    v.own = P.bnd + (size_t)s * P.sn;
    v.base = base;
    v.filt = P.filt + (size_t)s * FILT_WORDS;
    v.dirty = P.dirty + (size_t)s * P.snw;
    v.overlay = P.overlay;
    return v;
}

// Ordered 64-bit key of a double: signed integer order equals double order.
__device__ __forceinline__ long long dkey(double x) {
    long long b = __double_as_longlong(x);
    return b < 0 ? (b ^ 0x7fffffffffffffffll) : b;
}
__device__ __forceinline__ double dunkey(long long k) {
    return __longlong_as_double(k < 0 ? (k ^ 0x7fffffffffffffffll) : k);
}

__device__ __forceinline__ int light_group(int b) { return b >= 6 ? 64 : (1 << b); }

__host__ __device__ __forceinline__ int row_bin(int64_t len, int64_t heavy_threshold) {
    if (len > heavy_threshold) return BIN_HEAVY;
    if (len > 1024) return BIN_BLOCK;
    int b = 0;
    while ((1ll << b) < len) ++b;
    return b;
}

// ------------------------------------------------------------------------
// Threshold tests (shared by the candidate scatter and the apply step).
// ------------------------------------------------------------------------
__device__ __forceinline__ bool take_upper(bool is_int, double c, double old, double tau) {
    if (is_int) return c < old;
    if (isinf(old)) return c < old && !isinf(c);
    return c < old - tau * fmax(1.0, fabs(old));
}
__device__ __forceinline__ bool take_lower(bool is_int, double c, double old, double tau) {
    if (is_int) return c > old;
    if (isinf(old)) return c > old && !isinf(c);
    return c > old + tau * fmax(1.0, fabs(old));
}

struct RowAct {
    double minfin, maxfin;
    int nmin, nmax;
    double lo, hi;
    double rng;  // largest nonzero width of the row (slack filter)
};

// Slack filter.  The width of a nonzero bounds from above how much slack
// its row must have before no candidate of the row can move the
// variable's bounds: |a| times (domain + 1 + 2^-50 max|bound|), enlarged
// by 2^-40.  With every contribution finite and slack S = side - activity
// at least the width, the candidate of the Section 2.1 formula is, after
// its three roundings (each below 2^-53 relative), still at least one unit
// beyond the opposite bound: neither the threshold test nor integer
// rounding can accept it.  An infinite bound gives an infinite width.
__device__ __forceinline__ double nz_width(double a, double lb, double ub) {
    double d = ub - lb;
    d = d + 1.0;
    d = d + fmax(fabs(lb), fabs(ub)) * 0x1p-50;
    return (fabs(a) * d) * (1.0 + 0x1p-40);
}

// True when no candidate of the row can be taken: on each side the side is
// infinite, at least two contributions are infinite (no candidate exists),
// or all are finite and the slack reaches the row's width.  The slacks are
// the same floating-point differences the candidate formula starts from.
__device__ __forceinline__ bool row_quiet(const RowAct &R) {
    const double INF = __builtin_inf();
    const bool fin = R.rng < INF;
    const bool qhi = R.hi == INF || R.nmin >= 2 || (R.nmin == 0 && fin && R.hi - R.minfin >= R.rng);
    const bool qlo = R.lo == -INF || R.nmax >= 2 || (R.nmax == 0 && fin && R.maxfin - R.lo >= R.rng);
    return qhi && qlo;
}

// Maximum over aligned groups of G lanes (order-free).
template <int G>
__device__ __forceinline__ double group_max(double x) {
#pragma unroll
    for (int w = 1; w < G; w <<= 1) x = fmax(x, __shfl_xor(x, w, 64));
    return x;
}

// Bound candidates of one nonzero (Section 2.1, second display, and its
// mirror for the lower side).  cl/cu = -inf/+inf when absent.
__device__ __forceinline__ void nz_candidates(const RowAct &R, double a, double lb, double ub,
                                              bool is_int, double inttol, double &cl, double &cu) {
    const double INF = __builtin_inf();
    cl = -INF;
    cu = INF;
    if (R.hi < INF) {
        double bown = a > 0.0 ? lb : ub;
        bool own_inf = isinf(bown);
        bool have = false;
        double v = 0.0;
        if (!own_inf && R.nmin == 0) {
            double r = R.hi - R.minfin;
            double t = a * bown;
            v = r + t;
            have = true;
        } else if (own_inf && R.nmin == 1) {
            v = R.hi - R.minfin;
            have = true;
        }
        if (have) {
            double c = v / a;
            if (a > 0.0) cu = is_int ? floor(c + inttol) : c;
            else cl = is_int ? ceil(c - inttol) : c;
        }
    }
    if (R.lo > -INF) {
        double bown = a > 0.0 ? ub : lb;
        bool own_inf = isinf(bown);
        bool have = false;
        double v = 0.0;
        if (!own_inf && R.nmax == 0) {
            double r = R.lo - R.maxfin;
            double t = a * bown;
            v = r + t;
            have = true;
        } else if (own_inf && R.nmax == 1) {
            v = R.lo - R.maxfin;
            have = true;
        }
        if (have) {
            double c = v / a;
            if (a > 0.0) cl = is_int ? ceil(c - inttol) : c;
            else cu = is_int ? floor(c + inttol) : c;
        }
    }
}

// ------------------------------------------------------------------------
// Wave-aggregated appends (one atomic per wave and destination).
// Must be reached by every lane of the wave.
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    uint32_t lo = (uint32_t)mask, hi = (uint32_t)(mask >> 32);
    return __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
}

__device__ __forceinline__ void wave_push(uint64_t *q, uint32_t *counter, bool want, uint64_t v) {
    uint64_t mask = __ballot(want);
    if (mask == 0) return;
    int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (__lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (want) q[base + lane_rank(mask)] = v;
}

// Mark var i of slot s as having a candidate this round; first marker
// appends (s, i) to the round's changed list.
__device__ __forceinline__ void mark_var(const Params &P, bool want, int s, int i) {
    bool first = false;
    if (want) {
        uint32_t bit = 1u << (i & 31);
        uint32_t old = atomicOr(&P.vflag[(size_t)s * P.snw + (i >> 5)], bit);
        first = (old & bit) == 0;
    }
    const int st = blockIdx.x & (P.nstripe - 1);
    wave_push(P.chg + (size_t)st * P.chg_stride, &P.ctl->nchanged[st], first,
              ((uint64_t)(uint32_t)s << 32) | (uint32_t)i);
}

// Scatter the significant candidates of one nonzero.  Returns whether the
// variable needs marking.
__device__ __forceinline__ bool scatter(const Params &P, int s, int i, double cl, double cu,
                                        double lb, double ub, bool is_int) {
    bool any = false;
    longlong2 *cp = &P.cand[(size_t)s * P.sn + i];
    if (take_lower(is_int, cl, lb, P.tau)) {
        atomicMax(&cp->x, dkey(canon0(cl)));
        any = true;
    }
    if (take_upper(is_int, cu, ub, P.tau)) {
        atomicMin(&cp->y, dkey(canon0(cu)));
        any = true;
    }
    return any;
}

// Distinct rows read in this round over all slots (accounting mode only):
// the matrix term of a batch counts a row once per round.
__device__ __forceinline__ void count_row(const Params &P, int k, int64_t len) {
    if (!P.useen) return;
    uint32_t bit = 1u << (k & 31);
    uint32_t old = atomicOr(&P.useen[k >> 5], bit);
    if ((old & bit) == 0) {
        atomicAdd(&P.ctl->stat_urows, 1ull);
        atomicAdd(&P.ctl->stat_unnz, (unsigned long long)len);
    }
}

// Distinct bound records read in this round (accounting mode only).
__device__ __forceinline__ void count_read(const Params &P, int s, int i) {
    if (!P.touched) return;
    uint32_t bit = 1u << (i & 31);
    uint32_t old = atomicOr(&P.touched[(size_t)s * P.snw + (i >> 5)], bit);
    if ((old & bit) == 0) atomicAdd(&P.ctl->stat_vars, 1ull);
}

// Terms of one nonzero into the two accumulators.
__device__ __forceinline__ void add_terms(Acc &mn, Acc &mx, double a, double lb, double ub) {
    double bmin = a > 0.0 ? lb : ub;
    double bmax = a > 0.0 ? ub : lb;
    if (isinf(bmin)) mn.ninf += 1;
    else acc_add(mn, a * bmin);
    if (isinf(bmax)) mx.ninf += 1;
    else acc_add(mx, a * bmax);
}

// Exact activity of one side of a row over [p0, p1) by one lane.  Kept out
// of line so its accumulator lives in scratch memory and does not raise the
// register count of the kernels that may call it.
__device__ __noinline__ double exact_side(const DInst &I, const BView bnd, int64_t p0, int64_t p1,
                                          bool maxside) {
    SuperAcc S;
    sa_zero(S);
    for (int64_t p = p0; p < p1; ++p) {
        double a = I.val[p];
        double2 b = bnd[I.col[p]];
        double bb = (a > 0.0) != maxside ? b.x : b.y;
        if (!isinf(bb)) sa_add(S, a * bb);
    }
    return canon0(sa_round(S));
}

// Incremental heavy rows keep carry-save accumulators (bp_carry.h); these
// are the atomic adds into them.
constexpr int INC_SLOTS = 16;  // vectors of one call that keep incremental heavy rows
static_assert(CARRY_WORDS == SA_WORDS, "carry-save and exact accumulators differ in width");

__device__ __forceinline__ void inc_add(long long *L, double x, bool negate) {
    if (x == 0.0) return;
    int d0;
    long long q0, q1, q2;
    carry_pieces(x, negate, d0, q0, q1, q2);
    if (q0) atomicAdd((unsigned long long *)&L[d0], (unsigned long long)q0);
    if (q1) atomicAdd((unsigned long long *)&L[d0 + 1], (unsigned long long)q1);
    if (q2) atomicAdd((unsigned long long *)&L[d0 + 2], (unsigned long long)q2);
}

// Wave form (reached by every lane): the pieces of the lanes whose first
// limb is the same are summed across the wave first, so each distinct limb
// position costs three atomics by one lane instead of one per lane.
__device__ __forceinline__ void inc_add_wave(long long *L, double x, bool act) {
    int d0 = 0;
    long long q0 = 0, q1 = 0, q2 = 0;
    act = act && x != 0.0;
    if (act) carry_pieces(x, false, d0, q0, q1, q2);
    uint64_t pend = __ballot(act);
    while (pend) {
        const int leader = __ffsll((long long)pend) - 1;
        const int d = __shfl(d0, leader, 64);
        const bool mine = act && d0 == d;
        long long s0 = mine ? q0 : 0, s1 = mine ? q1 : 0, s2 = mine ? q2 : 0;
#pragma unroll
        for (int w = 1; w < 64; w <<= 1) {
            s0 += __shfl_xor(s0, w, 64);
            s1 += __shfl_xor(s1, w, 64);
            s2 += __shfl_xor(s2, w, 64);
        }
        if (__lane_id() == leader) {
            if (s0) atomicAdd((unsigned long long *)&L[d], (unsigned long long)s0);
            if (s1) atomicAdd((unsigned long long *)&L[d + 1], (unsigned long long)s1);
            if (s2) atomicAdd((unsigned long long *)&L[d + 2], (unsigned long long)s2);
        }
        pend &= ~__ballot(mine);
        act = act && !mine;
    }
}

// A bound change of one contribution: the term at the old bound out, the
// term at the new one in (an infinite bound is counted instead).
__device__ __forceinline__ void inc_move(long long *L, int32_t *ninf, double a, double bo, double bn) {
    if (bo == bn) return;
    if (isinf(bo)) atomicSub(ninf, 1);
    else inc_add(L, a * bo, true);
    if (isinf(bn)) atomicAdd(ninf, 1);
    else inc_add(L, a * bn, false);
}

__device__ __forceinline__ bool row_bad(const RowAct &R, double feastol) {
    if (R.nmin == 0 && R.minfin > R.hi + feastol) return true;
    if (R.nmax == 0 && R.maxfin < R.lo - feastol) return true;
    return false;
}

__device__ __forceinline__ void report_bad_row(const Params &P, int s, int k) {
    atomicMin(&P.info[s].row_bad_min, k);
    atomicAdd(&P.info[s].row_bad_count, 1);
}

__device__ __forceinline__ void clear_rflag(const Params &P, int s, int k) {
    uint32_t bit = 1u << (k & 31);
    atomicAnd(&P.rflag[(size_t)s * P.srw + (k >> 5)], ~bit);
}

// Scan rounds: does variable i hold a change of the update feeding par?
__device__ __forceinline__ bool scan_hit(const Params &P, int par, int i) {
    return (P.cbits[(size_t)par * P.snw + (i >> 5)] >> (i & 31)) & 1u;
}

// Rows and nonzeros a workgroup processed in a scan round, added once per
// workgroup to its stripe of the round's totals.  Reached by the whole
// workgroup.
__device__ void scan_count_flush(const Params &P, unsigned long long rows, unsigned long long nnz) {
    __shared__ unsigned long long sr[WG / 64], sz[WG / 64];
#pragma unroll
    for (int w = 1; w < 64; w <<= 1) {
        rows += __shfl_xor(rows, w, 64);
        nnz += __shfl_xor(nnz, w, 64);
    }
    if (__lane_id() == 0) {
        sr[threadIdx.x >> 6] = rows;
        sz[threadIdx.x >> 6] = nnz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long r = 0, z = 0;
        for (int j = 0; j < WG / 64; ++j) {
            r += sr[j];
            z += sz[j];
        }
        const int st = blockIdx.x & (NSTRIPE - 1);
        if (r) {
            atomicAdd(&P.ctl->scan_rows[st], r);
            atomicAdd(&P.ctl->scan_nnz[st], z);
        }
    }
}

// ------------------------------------------------------------------------
// Light rows: G lanes per row, len <= G (bins 0..6) or one wave per row
// with several nonzeros per lane (bins 7..10).  In a scan round the rows
// come from the list of every row (rows32) and a row holding no changed
// variable is skipped; the processed rows are counted in sc_rows/sc_nnz.
// ------------------------------------------------------------------------
template <bool MULTI, int G>
__device__ void light_rows(const Params &P, const uint64_t *q, uint32_t count, uint32_t unit,
                           const int32_t *rows32, int par, unsigned long long &sc_rows,
                           unsigned long long &sc_nnz) {
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const int per_wave = 64 / G;
    uint32_t t = (unit * (WG / 64) + wave) * per_wave + lane / G;
    const int gl = lane & (G - 1);
    bool valid = t < count;
    int s = 0, k = 0;
    bool live = false;
    int64_t p0 = 0, p1 = 0;
    double2 sd = make_double2(0.0, 0.0);
    DInst I = P.I;
    if (valid) {
        if (rows32) {
            k = rows32[t];
        } else {
            uint64_t task = q[t];
            s = (int)(task >> 32);
            k = (int)(uint32_t)task;
        }
        I = inst_of<MULTI>(P, s);
        // independent loads, issued together
        int32_t state = P.info[s].state;
        p0 = I.row_ptr[k];
        p1 = I.row_ptr[k + 1];
        sd = I.side[k];
        live = state == SLOT_ACTIVE;
        if (gl == 0 && !rows32) clear_rflag(P, s, k);
    }
    if (rows32) {
        // scan round: keep the row only if one of its variables changed
        bool mine = false;
        const int it_hit = G < 64 ? 1 : (int)((p1 - p0 + 63) / 64);
        for (int it = 0; it < it_hit; ++it) {
            const int64_t p = p0 + gl + (int64_t)it * G;
            if (live && p < p1) mine = mine || scan_hit(P, par, I.col[p]);
        }
        const uint64_t hm = __ballot(mine);
        const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1)) << ((lane / G) * G);
        live = live && (hm & gmask) != 0;
        if (live && gl == 0) {
            sc_rows += 1;
            sc_nnz += (unsigned long long)(p1 - p0);
        }
    }
    if (live && gl == 0) count_row(P, k, p1 - p0);
    if (!live) p1 = p0;
    const BView bnd = bview(P, s, I.base);
    Acc mn, mx;
    acc_zero(mn);
    acc_zero(mx);
    // Trip count is uniform across the wave: bins 0..6 have len <= G (one
    // pass); bins 7..10 have one row per wave.
    int first_i = 0;
    double first_a = 0.0;
    double2 first_b = make_double2(0.0, 0.0);
    uint8_t first_t = 0;
    double wmax = 0.0;
    const int64_t len = p1 - p0;
    const int iters = G < 64 ? 1 : (int)((len + 63) / 64);
    for (int it = 0; it < iters; ++it) {
        int64_t p = p0 + gl + (int64_t)it * G;
        if (p < p1) {
            int i = I.col[p];
            double a = I.val[p];
            double2 b = bnd[i];
            uint8_t vt = I.vtype[i];
            add_terms(mn, mx, a, b.x, b.y);
            wmax = fmax(wmax, nz_width(a, b.x, b.y));
            count_read(P, s, i);
            if (it == 0) {
                first_i = i;
                first_a = a;
                first_b = b;
                first_t = vt;
            }
        }
    }
    acc_group_reduce<G>(mn);
    acc_group_reduce<G>(mx);
    RowAct R;
    R.minfin = 0.0;
    R.maxfin = 0.0;
    R.lo = 0.0;
    R.hi = 0.0;
    R.nmin = mn.ninf;
    R.nmax = mx.ninf;
    R.rng = group_max<G>(wmax);
    bool ok_min = !P.force_exact && acc_certify(mn, R.minfin);
    bool ok_max = !P.force_exact && acc_certify(mx, R.maxfin);
    if (live && gl == 0) {
        if (!ok_min) R.minfin = exact_side(I, bnd, p0, p1, false);
        if (!ok_max) R.maxfin = exact_side(I, bnd, p0, p1, true);
    }
    {
        // The group's first lane holds the exact values; every lane of the
        // wave takes part in the shuffles.
        int src = (lane / G) * G;
        double e0 = __shfl(R.minfin, src, 64);
        double e1 = __shfl(R.maxfin, src, 64);
        if (!ok_min) R.minfin = e0;
        if (!ok_max) R.maxfin = e1;
    }
    bool bad = false, quiet = false;
    if (live) {
        R.lo = sd.x;
        R.hi = sd.y;
        bad = row_bad(R, P.feastol);
        if (bad && gl == 0) report_bad_row(P, s, k);
        quiet = !bad && row_quiet(R);
    }
    for (int it = 0; it < iters; ++it) {
        int64_t p = p0 + gl + (int64_t)it * G;
        bool has = live && !bad && !quiet && p < p1;
        int i = 0;
        bool need = false;
        if (has) {
            double a;
            double2 b;
            bool is_int;
            if (it == 0) {
                i = first_i;
                a = first_a;
                b = first_b;
                is_int = first_t != 0;
            } else {
                i = I.col[p];
                a = I.val[p];
                b = bnd[i];
                is_int = I.vtype[i] != 0;
            }
            double cl, cu;
            nz_candidates(R, a, b.x, b.y, is_int, P.inttol, cl, cu);
            need = scatter(P, s, i, cl, cu, b.x, b.y, is_int);
        }
        mark_var(P, need, s, i);
    }
}

// ------------------------------------------------------------------------
// Workgroup reduction helpers (256 lanes = 4 waves).
// ------------------------------------------------------------------------
struct WgScratch {
    double s[2][4], c[2][4], e[2][4];
    int n[2][4];
    double w[4];
    double act[2];
    int flag;
};

// Workgroup reduction of the two accumulators and of the width maximum;
// every lane ends with the same values.
__device__ inline void wg_reduce(Acc &mn, Acc &mx, double &wmax, WgScratch &W) {
    acc_group_reduce<64>(mn);
    acc_group_reduce<64>(mx);
    wmax = group_max<64>(wmax);
    const int wave = threadIdx.x >> 6;
    if (__lane_id() == 0) {
        W.s[0][wave] = mn.s; W.c[0][wave] = mn.c; W.e[0][wave] = mn.e; W.n[0][wave] = mn.ninf;
        W.s[1][wave] = mx.s; W.c[1][wave] = mx.c; W.e[1][wave] = mx.e; W.n[1][wave] = mx.ninf;
        W.w[wave] = wmax;
    }
    __syncthreads();
    wmax = W.w[0];
    for (int w = 1; w < WG / 64; ++w) wmax = fmax(wmax, W.w[w]);
    // Every lane combines the four wave states in wave order.
    Acc A[2];
    for (int side = 0; side < 2; ++side) {
        A[side].s = W.s[side][0]; A[side].c = W.c[side][0]; A[side].e = W.e[side][0];
        A[side].ninf = W.n[side][0];
        for (int w = 1; w < WG / 64; ++w)
            acc_merge(A[side], W.s[side][w], W.c[side][w], W.e[side][w], W.n[side][w]);
    }
    mn = A[0];
    mx = A[1];
    __syncthreads();
}

// Block rows: one workgroup per row (1024 < len <= heavy threshold).
template <bool MULTI>
__device__ void block_row(const Params &P, const uint64_t *q, uint32_t t, WgScratch &W,
                          const int32_t *rows32, int par, unsigned long long &sc_rows,
                          unsigned long long &sc_nnz) {
    int s = 0, k = 0;
    if (rows32) {
        k = rows32[t];
    } else {
        uint64_t task = q[t];
        s = (int)(task >> 32);
        k = (int)(uint32_t)task;
    }
    bool live = P.info[s].state == SLOT_ACTIVE;
    if (threadIdx.x == 0 && !rows32) clear_rflag(P, s, k);
    if (!live) return;  // workgroup-uniform
    const DInst I = inst_of<MULTI>(P, s);
    int64_t p0 = I.row_ptr[k], p1 = I.row_ptr[k + 1];
    if (rows32) {
        // scan round: keep the row only if one of its variables changed
        bool mine = false;
        for (int64_t p = p0 + threadIdx.x; p < p1; p += WG) mine = mine || scan_hit(P, par, I.col[p]);
        if (!__syncthreads_or(mine)) return;  // workgroup-uniform
        if (threadIdx.x == 0) {
            sc_rows += 1;
            sc_nnz += (unsigned long long)(p1 - p0);
        }
    }
    if (threadIdx.x == 0) count_row(P, k, p1 - p0);
    const BView bnd = bview(P, s, I.base);
    Acc mn, mx;
    acc_zero(mn);
    acc_zero(mx);
    double wmax = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += WG) {
        double2 b = bnd[I.col[p]];
        double a = I.val[p];
        add_terms(mn, mx, a, b.x, b.y);
        wmax = fmax(wmax, nz_width(a, b.x, b.y));
        count_read(P, s, I.col[p]);
    }
    wg_reduce(mn, mx, wmax, W);
    RowAct R;
    R.nmin = mn.ninf;
    R.nmax = mx.ninf;
    R.rng = wmax;
    bool ok_min = !P.force_exact && acc_certify(mn, R.minfin);
    bool ok_max = !P.force_exact && acc_certify(mx, R.maxfin);
    if (!(ok_min && ok_max)) {
        if (threadIdx.x == 0) {
            W.act[0] = ok_min ? R.minfin : exact_side(I, bnd, p0, p1, false);
            W.act[1] = ok_max ? R.maxfin : exact_side(I, bnd, p0, p1, true);
        }
        __syncthreads();
        R.minfin = W.act[0];
        R.maxfin = W.act[1];
        __syncthreads();
    }
    double2 sd = I.side[k];
    R.lo = sd.x;
    R.hi = sd.y;
    if (row_bad(R, P.feastol)) {
        if (threadIdx.x == 0) report_bad_row(P, s, k);
        return;
    }
    if (row_quiet(R)) return;  // workgroup-uniform
    const int64_t len = p1 - p0;
    const int iters = (int)((len + WG - 1) / WG);
    for (int it = 0; it < iters; ++it) {
        int64_t p = p0 + threadIdx.x + (int64_t)it * WG;
        bool need = false;
        int i = 0;
        if (p < p1) {
            i = I.col[p];
            double a = I.val[p];
            double2 b = bnd[i];
            bool is_int = I.vtype[i] != 0;
            double cl, cu;
            nz_candidates(R, a, b.x, b.y, is_int, P.inttol, cl, cu);
            need = scatter(P, s, i, cl, cu, b.x, b.y, is_int);
        }
        mark_var(P, need, s, i);
    }
}

// Heavy chunk, activity part: the partial states of one chunk of a heavy
// row.  The chunks of a row are contiguous; the candidate kernel of the
// same round combines them (the kernel boundary makes them visible).
template <bool MULTI>
__device__ void heavy_chunk_activity(const Params &P, int par, uint32_t u, WgScratch &W,
                                     bool scan) {
    const int4 rec = scan ? P.allhrec[u] : P.hrec[par][u];
    const int s = rec.x, k = rec.y, c = rec.z;
    const bool live = P.info[s].state == SLOT_ACTIVE;
    if (c == 0 && threadIdx.x == 0 && !scan) clear_rflag(P, s, k);
    if (!live) return;  // workgroup-uniform
    const DInst I = inst_of<MULTI>(P, s);
    const int64_t r0 = I.row_ptr[k], r1 = I.row_ptr[k + 1];
    int64_t p0 = r0 + (int64_t)c * P.heavy_chunk;
    int64_t p1 = min(r1, p0 + (int64_t)P.heavy_chunk);
    if (c == 0 && threadIdx.x == 0 && !scan) count_row(P, k, r1 - r0);
    const BView bnd = bview(P, s, I.base);
    Acc mn, mx;
    acc_zero(mn);
    acc_zero(mx);
    double wmax = 0.0;
    bool mine = false;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += WG) {
        const int i = I.col[p];
        double2 b = bnd[i];
        double a = I.val[p];
        add_terms(mn, mx, a, b.x, b.y);
        wmax = fmax(wmax, nz_width(a, b.x, b.y));
        count_read(P, s, i);
        if (scan) mine = mine || scan_hit(P, par, i);
    }
    // scan round: the row is processed if any of its chunks holds a change
    if (scan && __syncthreads_or(mine) && threadIdx.x == 0) atomicOr(&P.hhit[k], 1u);
    wg_reduce(mn, mx, wmax, W);
    if (threadIdx.x == 0) {
        P.hpart[2 * (size_t)u] = mn;
        P.hpart[2 * (size_t)u + 1] = mx;
        P.hrng[u] = wmax;
    }
}

// Heavy chunk, rebuild of the incremental accumulators (one plain vector):
// the chunk's exact terms at the current bounds are summed into workgroup
// limbs and added to the row's accumulators (zeroed by the previous round's
// end), with the infinite counts and the largest nonzero width.  Every heavy
// row takes part, queued or not.  In a scan round the chunk also marks its
// row when it holds a changed variable.
__device__ void inc_build_chunk(const Params &P, int par, uint32_t u, bool scan) {
    __shared__ long long L[2 * HL];
    __shared__ int32_t ninf[2];
    __shared__ unsigned long long wbits;
    const uint32_t na = (uint32_t)P.allhchunks;
    const int s = (int)(u / na);  // every slot rebuilds every heavy chunk
    const int4 rec = P.allhrec[u % na];
    const int k = rec.y, c = rec.z;
    if (P.info[s].state != SLOT_ACTIVE) return;  // workgroup-uniform
    for (int j = threadIdx.x; j < 2 * HL; j += WG) L[j] = 0;
    if (threadIdx.x == 0) {
        ninf[0] = 0;
        ninf[1] = 0;
        wbits = 0ull;
    }
    __syncthreads();
    const DInst &I = P.I;
    const int64_t r0 = I.row_ptr[k], r1 = I.row_ptr[k + 1];
    const int64_t p0 = r0 + (int64_t)c * P.heavy_chunk;
    const int64_t p1 = min(r1, p0 + (int64_t)P.heavy_chunk);
    const BView bnd = bview(P, s, I.base);
    int nmin = 0, nmax = 0;
    double wmax = 0.0;
    bool mine = false;
    const int iters = (int)((p1 - p0 + WG - 1) / WG);  // uniform: whole waves add together
    for (int it = 0; it < iters; ++it) {
        const int64_t p = p0 + threadIdx.x + (int64_t)it * WG;
        const bool in = p < p1;
        double tmin = 0.0, tmax = 0.0;
        if (in) {
            const int i = I.col[p];
            const double2 b = bnd[i];
            const double a = I.val[p];
            const double bmin = a > 0.0 ? b.x : b.y;
            const double bmax = a > 0.0 ? b.y : b.x;
            if (isinf(bmin)) nmin += 1;
            else tmin = a * bmin;
            if (isinf(bmax)) nmax += 1;
            else tmax = a * bmax;
            wmax = fmax(wmax, nz_width(a, b.x, b.y));
            count_read(P, s, i);
            if (scan) mine = mine || scan_hit(P, par, i);
        }
        inc_add_wave(L, tmin, in);
        inc_add_wave(L + HL, tmax, in);
    }
    if (nmin) atomicAdd(&ninf[0], nmin);
    if (nmax) atomicAdd(&ninf[1], nmax);
    if (wmax > 0.0) atomicMax(&wbits, (unsigned long long)__double_as_longlong(wmax));
    if (scan && __syncthreads_or(mine) && threadIdx.x == 0) atomicOr(&P.hhit[k], 1u);
    __syncthreads();
    const size_t hs = (size_t)s * P.nheavy + P.I.hidx[k];
    long long *G = P.hacc + hs * 2 * HL;
    for (int j = threadIdx.x; j < 2 * HL; j += WG)
        if (L[j]) atomicAdd((unsigned long long *)&G[j], (unsigned long long)L[j]);
    if (threadIdx.x == 0) {
        if (ninf[0]) atomicAdd(&P.hinf[2 * hs], ninf[0]);
        if (ninf[1]) atomicAdd(&P.hinf[2 * hs + 1], ninf[1]);
        if (wbits) atomicMax(&P.hwid[hs], wbits);
    }
}

// The rounded finite parts of heavy row h (accumulators hs) by the whole
// workgroup: limbs staged in LDS (plus the base row's limbs blimb for job
// slots), one lane per side rounds them.
__device__ double2 inc_row_activity(const Params &P, size_t hs, const long long *blimb) {
    __shared__ long long L[2 * HL];
    __shared__ double act[2];
    __shared__ int range[4];  // lowest and highest nonzero limb of each side
    if (threadIdx.x < 4) range[threadIdx.x] = (threadIdx.x & 1) ? -1 : HL;
    __syncthreads();
    for (int j = threadIdx.x; j < 2 * HL; j += WG) {
        long long v = P.hacc[hs * 2 * HL + j];
        if (blimb) v += blimb[j];
        L[j] = v;
        if (v) {
            const int side = j >= HL ? 2 : 0, d = j >= HL ? j - HL : j;
            atomicMin(&range[side], d);
            atomicMax(&range[side + 1], d);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) act[0] = carry_round(L, range[0], range[1]);
    if (threadIdx.x == 64) act[1] = carry_round(L + HL, range[2], range[3]);
    __syncthreads();
    const double2 r = make_double2(act[0], act[1]);
    __syncthreads();  // L and act are reused by the next task
    return r;
}

// Infinite counts and slack-filter width of heavy row h (accumulators hs):
// for job slots the base row's counts plus the slot's corrections, and the
// base width.
__device__ __forceinline__ void inc_counts(const Params &P, const DInst &I, size_t hs, int h, RowAct &R) {
    R.nmin = P.hinf[2 * hs];
    R.nmax = P.hinf[2 * hs + 1];
    if (P.inc_base) {
        R.nmin += I.hbinf[2 * h];
        R.nmax += I.hbinf[2 * h + 1];
        R.rng = I.hbwid[h];
    } else {
        R.rng = __longlong_as_double((long long)P.hwid[hs]);
    }
}

// Heavy row head (round without a rebuild): chunk 0 of each queued heavy
// row rounds the row's accumulators once for all its chunks.
// It also tests the row: an infeasible row is reported, a quiet one ends
// here, and only the chunks of the others become candidate tasks for the
// heavy kernel, so a round whose heavy rows are all quiet leaves it idle.
template <bool MULTI>
__device__ void inc_head(const Params &P, int par, uint32_t u) {
    const int4 rec = P.hrec[par][u];
    const int s = rec.x, k = rec.y, c = rec.z, nch = rec.w;
    if (c != 0) return;  // workgroup-uniform
    if (threadIdx.x == 0) clear_rflag(P, s, k);
    if (P.info[s].state != SLOT_ACTIVE) return;  // workgroup-uniform
    const DInst I = inst_of<MULTI>(P, s);
    const int h = I.hidx[k];
    const size_t hs = (size_t)s * P.nheavy + h;
    const double2 a = inc_row_activity(P, hs, P.inc_base ? I.hblimb + (size_t)h * 2 * HL : nullptr);
    __shared__ RowAct RS;
    __shared__ int todo;
    if (threadIdx.x == 0) {
        P.hact[hs] = a;
        const double2 sd = I.side[k];
        RowAct R;
        R.minfin = a.x;
        R.maxfin = a.y;
        inc_counts(P, I, hs, h, R);
        R.lo = sd.x;
        R.hi = sd.y;
        const bool bad = row_bad(R, P.feastol), quiet = !bad && row_quiet(R);
        if (bad) report_bad_row(P, s, k);
        if (P.touched) {  // byte accounting: tested from the accumulators
            atomicAdd(&P.ctl->stat_kept_rows, 1ull);
            if (bad || quiet)
                atomicAdd(&P.ctl->stat_kept_nnz, (unsigned long long)(I.row_ptr[k + 1] - I.row_ptr[k]));
        }
        todo = 0;
        if (!bad && !quiet) {
            if (P.inc_base) {
                // job slots: the head computes the candidates itself
                RS = R;
                todo = 1;
            } else {
                const uint32_t at = atomicAdd(&P.ctl->hcand[par], (uint32_t)nch);
                for (int j = 0; j < nch; ++j) P.hcrec[par][at + j] = make_int4(s, k, j, nch);
            }
        }
    }
    if (!P.inc_base) return;  // uniform
    __syncthreads();
    if (todo) {
        // Job slots never rebuild their accumulators, so a round's heavy
        // rows are decided here and the heavy kernel is not launched: the
        // workgroup walks the whole row for the slot's candidates.
        const RowAct R = RS;
        const int64_t r0 = I.row_ptr[k], r1 = I.row_ptr[k + 1];
        if (threadIdx.x == 0) count_row(P, k, r1 - r0);
        const BView bnd = bview(P, s, I.base);
        const int iters = (int)((r1 - r0 + WG - 1) / WG);
        for (int it = 0; it < iters; ++it) {
            const int64_t p = r0 + threadIdx.x + (int64_t)it * WG;
            bool need = false;
            int i = 0;
            if (p < r1) {
                i = I.col[p];
                const double av = I.val[p];
                const double2 b = bnd[i];
                const bool is_int = I.vtype[i] != 0;
                double cl, cu;
                nz_candidates(R, av, b.x, b.y, is_int, P.inttol, cl, cu);
                need = scatter(P, s, i, cl, cu, b.x, b.y, is_int);
            }
            mark_var(P, need, s, i);
        }
    }
    __syncthreads();  // RS and todo are reused by the next task
}

// Heavy chunk, candidate part.  Every wave combines the row's partials
// (lane l takes chunks l, l+64, ... in order, then a butterfly), certifies
// the sums and tests the row; the chunk's nonzeros then give candidates.
template <bool MULTI>
__device__ void heavy_chunk_candidates(const Params &P, int par, uint32_t u, bool scan,
                                       bool rebuild, bool decided) {
    // decided: a task of a row its head already tested (not infeasible, not
    // quiet), from the head's list
    const int4 rec = decided ? P.hcrec[par][u] : (scan ? P.allhrec[u] : P.hrec[par][u]);
    const int s = rec.x, k = rec.y, c = rec.z, nch = rec.w;
    // With incremental heavy rows a rebuild round does not walk the queued
    // chunks in the row kernel: the queue flag of the row is cleared here,
    // for draining slots too, so no flag outlives its round.
    if (P.inc && !decided && c == 0 && threadIdx.x == 0 && !scan) clear_rflag(P, s, k);
    if (P.info[s].state != SLOT_ACTIVE) return;  // workgroup-uniform
    const DInst I = inst_of<MULTI>(P, s);
    if (scan) {
        // scan round: rows without a changed variable are not processed
        if (!P.hhit[k]) return;  // workgroup-uniform
        if (c == 0 && threadIdx.x == 0) {
            const int st = blockIdx.x & (NSTRIPE - 1);
            atomicAdd(&P.ctl->scan_rows[st], 1ull);
            atomicAdd(&P.ctl->scan_nnz[st], (unsigned long long)(I.row_ptr[k + 1] - I.row_ptr[k]));
        }
    }
    const int lane = __lane_id();
    const int64_t r0 = I.row_ptr[k], r1 = I.row_ptr[k + 1];
    const double2 sd = I.side[k];
    const BView bnd = bview(P, s, I.base);
    RowAct R;
    R.minfin = 0.0;
    R.maxfin = 0.0;
    R.lo = sd.x;
    R.hi = sd.y;
    if (P.inc) {
        // incremental accumulators: exact sums rounded once, by the row's
        // head in the row kernel, or here in a rebuild round (the row
        // kernel built them); the stored width bounds the current one
        // (bounds only shrink)
        const int h = I.hidx[k];
        const size_t hs = (size_t)s * P.nheavy + h;
        inc_counts(P, I, hs, h, R);
        const double2 a = rebuild ? inc_row_activity(P, hs, nullptr) : P.hact[hs];
        R.minfin = a.x;
        R.maxfin = a.y;
    } else {
        const uint32_t u0 = u - (uint32_t)c;
        Acc A, B;
        acc_zero(A);
        acc_zero(B);
        double wmax = 0.0;
        for (int j = lane; j < nch; j += 64) {
            Acc a = P.hpart[2 * (size_t)(u0 + j)], b = P.hpart[2 * (size_t)(u0 + j) + 1];
            acc_merge(A, a.s, a.c, a.e, a.ninf);
            acc_merge(B, b.s, b.c, b.e, b.ninf);
            wmax = fmax(wmax, P.hrng[u0 + j]);
        }
        acc_group_reduce<64>(A);
        acc_group_reduce<64>(B);
        R.nmin = A.ninf;
        R.nmax = B.ninf;
        R.rng = group_max<64>(wmax);
        bool ok_min = !P.force_exact && acc_certify(A, R.minfin);
        bool ok_max = !P.force_exact && acc_certify(B, R.maxfin);
        if (lane == 0) {
            if (!ok_min) R.minfin = exact_side(I, bnd, r0, r1, false);
            if (!ok_max) R.maxfin = exact_side(I, bnd, r0, r1, true);
        }
    }
    R.minfin = __shfl(R.minfin, 0, 64);
    R.maxfin = __shfl(R.maxfin, 0, 64);
    int64_t p0 = r0 + (int64_t)c * P.heavy_chunk;
    int64_t p1 = min(r1, p0 + (int64_t)P.heavy_chunk);
    const bool bad = !decided && row_bad(R, P.feastol);
    const bool quiet = !decided && !bad && row_quiet(R);  // uniform
    if (P.touched && P.inc && !rebuild && !decided && threadIdx.x == 0) {
        // byte accounting: the row was tested from its accumulators, and
        // without candidates its nonzeros are not read at all
        if (c == 0) atomicAdd(&P.ctl->stat_kept_rows, 1ull);
        if (bad || quiet) atomicAdd(&P.ctl->stat_kept_nnz, (unsigned long long)(p1 - p0));
    }
    if (bad) {
        if (c == 0 && threadIdx.x == 0) report_bad_row(P, s, k);
        return;
    }
    if (quiet) return;
    if (decided && c == 0 && threadIdx.x == 0) count_row(P, k, r1 - r0);  // read for its candidates
    const int iters = (int)((p1 - p0 + WG - 1) / WG);
    for (int it = 0; it < iters; ++it) {
        int64_t p = p0 + threadIdx.x + (int64_t)it * WG;
        bool need = false;
        int i = 0;
        if (p < p1) {
            i = I.col[p];
            double a = I.val[p];
            double2 b = bnd[i];
            bool is_int = I.vtype[i] != 0;
            double cl, cu;
            nz_candidates(R, a, b.x, b.y, is_int, P.inttol, cl, cu);
            need = scatter(P, s, i, cl, cu, b.x, b.y, is_int);
        }
        mark_var(P, need, s, i);
    }
}

__device__ inline uint32_t light_units(uint32_t count, int b) {
    uint32_t G = (uint32_t)light_group(b);
    return (uint32_t)(((uint64_t)count * G + WG - 1) / WG);
}

template <bool MULTI>
#ifndef BP_ROWS_WAVES
#define BP_ROWS_WAVES 4  // waves per SIMD the row kernel's register budget targets
#endif
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(BP_ROWS_WAVES))) k_rows(Params P) {
    __shared__ WgScratch W;
    // The round's counters of both parities are read together (one memory
    // round trip) and selected afterwards; a finished run has no units.
    const CtlHead H = ctl_head(P.ctl);
    const int par = H.round & 1;
    // A scan round walks every row (the instance's bin lists) instead of the
    // queues.
    const bool scan = P.scan_ok && H.scan;
    uint32_t qc[NBIN];
#pragma unroll
    for (int b = 0; b < NBIN; ++b)
        qc[b] = scan ? (uint32_t)(P.allstart[b + 1] - P.allstart[b]) : H.qcount[b];
    // Heavy chunks: partial states of the queued chunks, or, with
    // incremental accumulators, every chunk in a rebuild round and the
    // queued row heads (one record per row) otherwise.
    const uint32_t C_hchunks = P.inc ? (H.hbuild ? (uint32_t)P.allhchunks * (uint32_t)P.inc_slots : H.hchunks)
                                     : (scan ? (uint32_t)P.allhchunks : H.hchunks);
    unsigned long long sc_rows = 0, sc_nnz = 0;
    // Work units: heavy chunks, block rows, then light bins 10..0.
    uint32_t start[NBIN + 1];
    start[0] = 0;
    start[1] = C_hchunks;
    start[2] = start[1] + qc[BIN_BLOCK];
    for (int j = 0; j < NLIGHT; ++j) {
        int b = NLIGHT - 1 - j;
        start[3 + j] = start[2 + j] + light_units(qc[b], b);
    }
    const uint32_t total = H.done ? 0u : start[2 + NLIGHT];
    for (uint32_t u = blockIdx.x; u < total; u += gridDim.x) {
        if (u < start[1]) {
            if (P.inc && H.hbuild) inc_build_chunk(P, par, u, scan);
            else if (P.inc) inc_head<MULTI>(P, par, u);
            else heavy_chunk_activity<MULTI>(P, par, u, W, scan);
        } else if (u < start[2]) {
            block_row<MULTI>(P, P.q[par][BIN_BLOCK], u - start[1], W,
                             scan ? P.allrows + P.allstart[BIN_BLOCK] : nullptr, par, sc_rows, sc_nnz);
        } else {
            // bin of unit u by constant-index selects (start[] stays in
            // registers; a dynamic index would place it in scratch memory)
            int j = 0;
            uint32_t ubase = start[2], cnt = qc[NLIGHT - 1];
#pragma unroll
            for (int t = 0; t < NLIGHT - 1; ++t) {
                const bool past = u >= start[3 + t];
                j += past ? 1 : 0;
                ubase = past ? start[3 + t] : ubase;
                cnt = past ? qc[NLIGHT - 2 - t] : cnt;
            }
            int b = NLIGHT - 1 - j;
            uint32_t lu = u - ubase;
            const uint64_t *q = P.q[par][b];
            const int32_t *r32 = scan ? P.allrows + P.allstart[b] : nullptr;
            switch (b) {
                case 0: light_rows<MULTI, 1>(P, q, cnt, lu, r32, par, sc_rows, sc_nnz); break;
                case 1: light_rows<MULTI, 2>(P, q, cnt, lu, r32, par, sc_rows, sc_nnz); break;
                case 2: light_rows<MULTI, 4>(P, q, cnt, lu, r32, par, sc_rows, sc_nnz); break;
                case 3: light_rows<MULTI, 8>(P, q, cnt, lu, r32, par, sc_rows, sc_nnz); break;
                case 4: light_rows<MULTI, 16>(P, q, cnt, lu, r32, par, sc_rows, sc_nnz); break;
                case 5: light_rows<MULTI, 32>(P, q, cnt, lu, r32, par, sc_rows, sc_nnz); break;
                default: light_rows<MULTI, 64>(P, q, cnt, lu, r32, par, sc_rows, sc_nnz); break;
            }
        }
        __syncthreads();
    }
    if (scan) scan_count_flush(P, sc_rows, sc_nnz);
}

template <bool MULTI>
__global__ void __launch_bounds__(WG) k_heavy(Params P) {
    const CtlHead H = ctl_head(P.ctl);
    const int par = H.round & 1;
    const bool scan = P.scan_ok && H.scan;
    // with incremental heavy rows, a round without a rebuild takes only the
    // chunks whose row head asked for candidates
    const bool decided = P.inc && !H.hbuild;
    const uint32_t nh = decided ? H.hcand : (scan ? (uint32_t)P.allhchunks : H.hchunks);
    const uint32_t total = H.done ? 0u : nh;
    for (uint32_t u = blockIdx.x; u < total; u += gridDim.x)
        heavy_chunk_candidates<MULTI>(P, par, u, scan, P.inc && H.hbuild, decided);
}

// ------------------------------------------------------------------------
// Queueing rows for the next round.
// ------------------------------------------------------------------------
// Add newly queued rows to their slots' pending counters: one atomic pair
// per wave when every queuing lane belongs to the same slot (always the
// case for a single bound vector), one per lane otherwise.
__device__ __forceinline__ void count_pending(const Params &P, bool first, int s, int64_t len) {
    uint64_t mask = __ballot(first);
    if (mask == 0) return;
    int leader = __ffsll((long long)mask) - 1;
    int s0 = __shfl(s, leader, 64);
    if (__all(!first || s == s0)) {
        unsigned long long tot = first ? (unsigned long long)len : 0ull;
#pragma unroll
        for (int w = 1; w < 64; w <<= 1) tot += __shfl_xor(tot, w, 64);
        if (__lane_id() == leader) {
            atomicAdd(&P.info[s0].pending_rows, (int32_t)__popcll(mask));
            atomicAdd(&P.info[s0].pending_nnz, tot);
        }
    } else if (first) {
        atomicAdd(&P.info[s].pending_rows, 1);
        atomicAdd(&P.info[s].pending_nnz, (unsigned long long)len);
    }
}

// Append the (slot, row) tasks of the lanes with first == true to their bin
// queues of parity par: one ballot per bin, then one atomic per non-empty
// bin issued by lanes 0..BIN_HEAVY-1 in parallel; heavy rows become chunk
// records.  With heads_only (incremental heavy rows, next round without an
// accumulator rebuild) a heavy row queues only its chunk 0: that round
// tests the row from its accumulators in the head task, and the head lists
// the row's chunks as candidate tasks itself when it needs them.  Reached
// by every lane of the wave.
__device__ __forceinline__ void append_rows(const Params &P, int par, bool first, int s, int k,
                                            int bin, int64_t len, bool heads_only = false) {
    if (!__any(first)) return;
    const int lane = __lane_id();
    if (first && bin == BIN_HEAVY) {
        const int nch = (int)((len + P.heavy_chunk - 1) / P.heavy_chunk);
        const int nrec = heads_only ? 1 : nch;
        uint32_t cb = atomicAdd(&P.ctl->hchunks[par], (uint32_t)nrec);
        for (int c = 0; c < nrec; ++c) P.hrec[par][cb + c] = make_int4(s, k, c, nch);
    }
    const bool lt = first && bin != BIN_HEAVY;
    uint32_t cnt = 0;
    uint64_t mine = 0;
#pragma unroll
    for (int b = 0; b < BIN_HEAVY; ++b) {
        uint64_t mb = __ballot(lt && bin == b);
        if (lane == b) cnt = (uint32_t)__popcll(mb);
        if (lt && bin == b) mine = mb;
    }
    uint32_t base = 0;
    if (lane < BIN_HEAVY && cnt) base = atomicAdd(&P.ctl->qcount[par][lane], cnt);
    uint32_t mybase = __shfl(base, lt ? bin : 0, 64);
    if (lt) P.q[par][bin][mybase + lane_rank(mine)] = ((uint64_t)(uint32_t)s << 32) | (uint32_t)k;
}

// Queue, for the round of parity par, the rows of the column [c0, c0+len)
// of the variable held by each lane with want == true (at most one per
// lane; lanes may hold different slots and instances).  The column entries
// of the whole wave are walked 64 at a time.  A row is queued once per
// slot: the first lane to set its bit in the slot's row bitmap appends it.
// With count == false the slot counters are left alone and the wave totals
// (rows, nonzeros) are returned instead.  With incremental heavy rows, the
// lane's bound change (old bl/bu, new nl/nu) also corrects the accumulators
// of every heavy row of its column.  Reached by every lane of the wave.
template <bool MULTI>
__device__ void enqueue_columns(const Params &P, int par, bool want, int s, long long c0,
                                uint32_t len, bool count = true, uint32_t *rows_out = nullptr,
                                unsigned long long *nnz_out = nullptr, bool correct = false,
                                double bl = 0.0, double bu = 0.0, double nl = 0.0,
                                double nu = 0.0) {
    uint32_t tot_rows = 0;
    unsigned long long tot_nnz = 0, tot_corr = 0;
    const int lane = __lane_id();
    if (!want) {
        c0 = 0;
        len = 0;
    }
    uint32_t incl = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    const uint32_t tot = __shfl(incl, 63, 64);
    for (uint32_t off = 0; off < tot; off += 64) {
        const uint32_t j = off + lane;
        const bool has = j < tot;
        // owner lane: the smallest o with incl[o] > j (six halvings of 64)
        int lo = 0, hi = 63;
#pragma unroll
        for (int step = 0; step < 6; ++step) {
            int mid = (lo + hi) >> 1;
            uint32_t v = __shfl(incl, mid, 64);
            if (v > j) hi = mid;
            else lo = mid + 1;
        }
        const uint32_t oincl = __shfl(incl, lo, 64);
        const uint32_t olen = __shfl(len, lo, 64);
        const long long oc0 = __shfl(c0, lo, 64);
        const int os = __shfl(s, lo, 64);
        int k = 0;
        int bin = 0;
        int64_t rlen = 0;
        bool first = false;
        const double obl = __shfl(bl, lo, 64), obu = __shfl(bu, lo, 64);
        const double onl = __shfl(nl, lo, 64), onu = __shfl(nu, lo, 64);
        if (has) {
            const DInst I = inst_of<MULTI>(P, os);
            const long long e = oc0 + (long long)(j - (oincl - olen));
            k = I.col_row[e];
            uint32_t bit = 1u << (k & 31);
            uint32_t *wp = &P.rflag[(size_t)os * P.srw + (k >> 5)];
            // Independent loads issued together.  Rows shared by many changed
            // variables (dense rows) are mostly seen set already: the relaxed
            // load spares their atomics.
            uint32_t cur = __hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bin = I.rbin[k];
            int64_t rp0 = I.row_ptr[k], rp1 = I.row_ptr[k + 1];
            if ((cur & bit) == 0) first = (atomicOr(wp, bit) & bit) == 0;
            rlen = rp1 - rp0;
            if (correct && bin == BIN_HEAVY) {
                tot_corr += 1;
                const double a = I.cval[e];
                const size_t hs = (size_t)os * P.nheavy + I.hidx[k];
                long long *Lh = P.hacc + hs * 2 * HL;
                inc_move(Lh, &P.hinf[2 * hs], a, a > 0.0 ? obl : obu, a > 0.0 ? onl : onu);
                inc_move(Lh + HL, &P.hinf[2 * hs + 1], a, a > 0.0 ? obu : obl, a > 0.0 ? onu : onl);
            }
        }
        if (count) {
            count_pending(P, first, os, first ? rlen : 0);
        } else {
            unsigned long long x = first ? (unsigned long long)rlen : 0ull;
#pragma unroll
            for (int w = 1; w < 64; w <<= 1) x += __shfl_xor(x, w, 64);
            tot_nnz += x;
            tot_rows += (uint32_t)__popcll(__ballot(first));
        }
        append_rows(P, par, first, os, k, bin, rlen, correct);
    }
    if (rows_out) *rows_out = tot_rows;
    if (nnz_out) *nnz_out = tot_nnz;
    if (P.touched && correct) {  // byte accounting only
#pragma unroll
        for (int w = 1; w < 64; w <<= 1) tot_corr += __shfl_xor(tot_corr, w, 64);
        if (lane == 0 && tot_corr) atomicAdd(&P.ctl->stat_apply_corr, tot_corr);
    }
}

// Dirty tracking for jobs: first change of var i in slot s.
__device__ __forceinline__ void mark_dirty(const Params &P, int s, int i) {
    uint32_t bit = 1u << (i & 31);
    uint32_t old = atomicOr(&P.dirty[(size_t)s * P.snw + (i >> 5)], bit);
    uint32_t h = fhash(i);
    atomicOr(&P.filt[(size_t)s * FILT_WORDS + (h >> 5)], 1u << (h & 31));
    if ((old & bit) == 0) {
        int d = atomicAdd(&P.dcount[s], 1);
        P.dlist[(size_t)s * P.sn + d] = i;
    }
}

// Round end for every slot: outcome, counters, next round (one workgroup).
// Job engines, at the round end (the one workgroup of k_end, after its slot
// pass; each thread reads back the slots it wrote): the slots that are free
// now get the next jobs in slot order, and the finished ones their staging
// offsets and completion-ring positions, by workgroup prefix sums.  The
// retire kernel then needs no atomics on these shared counters, which every
// one of its workgroups would otherwise hit at once.
__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
    return (uint32_t)__popcll(mask & ((1ull << __lane_id()) - 1ull));
}

template <int NT>
__device__ void assign_claims(const Params &P, uint32_t next0, uint32_t total) {
    Ctl *C = P.ctl;
    __shared__ uint32_t w_free[NT / 64], w_fin[NT / 64];
    __shared__ unsigned long long w_cnt[NT / 64];
    __shared__ unsigned long long b_stage;
    __shared__ uint32_t b_free, b_fin, b_ring;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        b_free = 0;
        b_fin = 0;
        b_stage = C->stage_count;
        b_ring = C->done_jobs;
    }
    __syncthreads();
    const uint32_t avail = next0 < total ? total - next0 : 0u;
    for (int c0 = 0; c0 < P.nslots; c0 += NT) {
        const int s = c0 + threadIdx.x;
        bool fr = false, fn = false;
        unsigned long long cnt = 0;
        if (s < P.nslots) {
            const SlotInfo &S = P.info[s];
            fr = S.state == SLOT_FREE;
            fn = S.retire != 0;
            if (fn && S.status != 1)
                cnt = (unsigned long long)__hip_atomic_load(&P.dcount[s], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint64_t mf = __ballot(fr), mn = __ballot(fn);
        unsigned long long inc = cnt;  // inclusive prefix of the staged counts in the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned long long y = __shfl_up(inc, d, 64);
            if (lane >= d) inc += y;
        }
        if (lane == 63) {
            w_free[wave] = (uint32_t)__popcll(mf);
            w_fin[wave] = (uint32_t)__popcll(mn);
            w_cnt[wave] = inc;
        }
        __syncthreads();
        uint32_t rf = b_free + lane_prefix(mf), rn = b_fin + lane_prefix(mn);
        unsigned long long off = b_stage + inc - cnt;
        for (int w = 0; w < wave; ++w) {
            rf += w_free[w];
            rn += w_fin[w];
            off += w_cnt[w];
        }
        if (s < P.nslots) {
            SlotInfo &S = P.info[s];
            if (fr) S.claim = rf < avail ? (int32_t)(next0 + rf) : CLAIM_NONE;
            if (fn) {
                S.stage_off = off;
                S.ring_pos = b_ring + rn;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 0; w < NT / 64; ++w) {
                b_free += w_free[w];
                b_fin += w_fin[w];
                b_stage += w_cnt[w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        C->next_job = next0 + min(b_free, avail);
        C->stage_count = b_stage;
        C->done_jobs = b_ring + b_fin;
        C->claims = 1u;
    }
}

// NT threads: END_WG for job engines, whose many slots the one workgroup
// walks every round; WG otherwise.
constexpr int END_WG = 1024;
template <int NT>
__global__ void __launch_bounds__(NT) k_end(Params P) {
    Ctl *C = P.ctl;
    // Control fields and this thread's first slot record read together,
    // before the early exit.
    const uint32_t c_done = C->done, c_round = C->round, c_max_rounds = C->max_rounds;
    const uint32_t c_next_job = C->next_job, c_total_jobs = C->total_jobs;
    const uint32_t c_scan_go = C->scan_go;
    const uint32_t c_hb0 = C->hbuild[0], c_hb1 = C->hbuild[1];
    const int s_first = threadIdx.x;
    SlotInfo first;
    if (s_first < P.nslots) first = P.info[s_first];
    else first.state = SLOT_FREE;
    ctl_loaded(c_done, c_round, c_max_rounds);
    ctl_loaded(c_next_job, c_total_jobs, c_done);
    asm volatile("" ::"v"(first.state));
    if (c_done) return;
    const int par = c_round & 1;
    // A scan round counted its processed rows itself (they were not queued);
    // a scan-seeding update marks pending work with scan_go.
    unsigned long long sc_rows = 0, sc_nnz = 0;
    if (P.scan_ok) {
#pragma unroll
        for (int st = 0; st < NSTRIPE; ++st) {
            sc_rows += C->scan_rows[st];
            sc_nnz += C->scan_nnz[st];
        }
    }
    __shared__ uint32_t s_active, s_finished;
    if (threadIdx.x == 0) {
        s_active = 0;
        s_finished = 0;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < P.nslots; s += NT) {
        SlotInfo &S = P.info[s];
        const SlotInfo V = s == s_first ? first : S;  // values at the round end
        if (V.state == SLOT_DRAINING) {
            S.state = SLOT_FREE;
            continue;
        }
        if (V.state != SLOT_ACTIVE) continue;
        // nonzeros of this round's scanned rows (one vector: slot 0)
        const unsigned long long nnz0 = V.nnz + (s == 0 ? sc_nnz : 0ull);
        if (nnz0 != V.nnz) S.nnz = nnz0;
        const int32_t pending = V.pending_rows + (s == 0 && c_scan_go ? 1 : 0);
        bool fin = true;
        bool drain = false;
        if (V.row_bad_count > 0) {
            S.status = 1;
            drain = V.pending_rows > 0;
        } else if (V.var_bad_min != NONE) {
            S.status = 1;
            drain = V.pending_rows > 0;
        } else if (pending == 0) {
            S.status = 0;
        } else if ((uint32_t)V.rounds >= c_max_rounds) {
            S.status = 2;
            drain = true;
        } else {
            fin = false;
            S.rounds = V.rounds + 1;
            S.nnz = nnz0 + V.pending_nnz;
            atomicAdd(&C->stat_rows, (unsigned long long)V.pending_rows);
            atomicAdd(&C->stat_nnz, V.pending_nnz);
            S.pending_rows = 0;
            S.pending_nnz = 0;
            S.row_bad_min = NONE;
            S.row_bad_count = 0;
            S.var_bad_min = NONE;
            atomicAdd(&s_active, 1u);
        }
        if (fin) {
            S.state = drain ? SLOT_DRAINING : SLOT_FREE;
            S.retire = 1;
            atomicAdd(&s_finished, 1u);
            if (drain) atomicAdd(&s_active, 1u);  // still has queued tasks
        }
    }
    if (c_total_jobs > 0) assign_claims<NT>(P, c_next_job, c_total_jobs);
    if (P.touched) {
        size_t words = (size_t)P.nslots * P.snw;
        for (size_t w = threadIdx.x; w < words; w += NT) P.touched[w] = 0u;
    }
    if (P.useen)
        for (size_t w = threadIdx.x; w < (size_t)P.srw; w += NT) P.useen[w] = 0u;
    // the next round rebuilds the heavy-row accumulators: start from zero
    if (P.inc && (par ? c_hb0 : c_hb1)) {
        const size_t nh = (size_t)P.inc_slots * P.nheavy;
        for (size_t w = threadIdx.x; w < nh * 2 * HL; w += NT) P.hacc[w] = 0;
        for (size_t w = threadIdx.x; w < 2 * nh; w += NT) P.hinf[w] = 0;
        for (size_t w = threadIdx.x; w < nh; w += NT) P.hwid[w] = 0ull;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int b = 0; b < NBIN; ++b) C->qcount[par][b] = 0;
        C->hchunks[par] = 0;
        C->hcand[par] = 0;
        for (int st = 0; st < NSTRIPE; ++st) C->nchanged[st] = 0;
        if (P.scan_ok) {
            if (sc_rows) {
                atomicAdd(&C->stat_rows, sc_rows);
                atomicAdd(&C->stat_nnz, sc_nnz);
            }
            for (int st = 0; st < NSTRIPE; ++st) {
                C->scan_rows[st] = 0;
                C->scan_nnz[st] = 0;
            }
            C->scan[par] = 0;
            C->scan_go = 0;
        }
        if (P.inc) C->hbuild[par] = 0;
        C->active = s_active;
        C->finished = s_finished;
        C->round = c_round + 1;
        if (s_active == 0 && c_next_job >= c_total_jobs) C->done = 1;
    }
}

constexpr int APPLY_V = 16;  // changed variables per wave and step in k_apply

template <bool MULTI>
__global__ void __launch_bounds__(WG) k_apply(Params P) {
    Ctl *C = P.ctl;
    // Control fields and the stripe lengths, read together.
    const uint32_t c_round = C->round, c_done = C->done;
    const uint32_t c_scan0 = C->scan[0], c_scan1 = C->scan[1];
    uint32_t pre[NSTRIPE + 1];
    pre[0] = 0;
#pragma unroll
    for (int st = 0; st < NSTRIPE; ++st) pre[st + 1] = pre[st] + C->nchanged[st];
    ctl_loaded(c_round, c_done, pre[NSTRIPE]);
    ctl_loaded(c_scan0, c_scan1, c_done);
    const int par = c_round & 1;
    const int npar = par ^ 1;
    const uint32_t total = c_done ? 0u : pre[NSTRIPE];
    // Scan rounds (one plain vector): this round's changed bitmap and heavy
    // hits are cleared once the round's row kernels have read them; a large
    // update makes the next round scan every row instead of queueing rows.
    const bool scan_now = P.scan_ok && (par ? c_scan1 : c_scan0) && !c_done;
    const bool scan_next = P.scan_ok && total >= P.scan_min;
    // many changes: the next round rebuilds the heavy-row accumulators
    // rather than taking that many corrections
    const bool periodic = P.inc_period != 0u && (c_round + 1u) % P.inc_period == 0u;
    const bool rebuild_next = P.inc && (scan_next || total >= P.inc_max || periodic);
    if (scan_now) {
        const size_t g = (size_t)blockIdx.x * WG + threadIdx.x, G = (size_t)gridDim.x * WG;
        for (size_t w = g; w < (size_t)P.snw; w += G) P.cbits[(size_t)par * P.snw + w] = 0u;
        for (size_t u = g; u < (size_t)P.allhchunks; u += G) P.hhit[P.allhrec[u].y] = 0u;
    }
    const double INF = __builtin_inf();
    const int lane = __lane_id();
    const uint32_t nwaves = gridDim.x * (WG / 64);
    const uint32_t gw = blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    // One bound vector: the wave adds its accepted changes and queued rows
    // to running totals, and the workgroup adds them to the counters once.
    const bool single = P.nslots == 1;
    uint32_t w_rows = 0;
    unsigned long long w_nnz = 0, w_written = 0;
    // Wave-uniform trip count: whole waves reach the aggregated appends.
    for (uint32_t e0 = gw * APPLY_V; e0 < total; e0 += nwaves * APPLY_V) {
        uint32_t e = e0 + lane;
        bool has = lane < APPLY_V && e < total;
        int s = 0, i = 0;
        bool go = false;
        long long c0 = 0;
        uint32_t clen = 0;
        double ol = 0.0, ou = 0.0, wl = 0.0, wu = 0.0;  // old and written bounds
        if (has) {
            int st = 0;
#pragma unroll
            for (int j = 1; j < NSTRIPE; ++j) st += e >= pre[j] ? 1 : 0;
            uint64_t ent = P.chg[(size_t)st * P.chg_stride + (e - pre[st])];
            s = (int)(ent >> 32);
            i = (int)(uint32_t)ent;
            const DInst I = inst_of<MULTI>(P, s);
            c0 = I.col_ptr[i];
            clen = (uint32_t)(I.col_ptr[i + 1] - c0);
            longlong2 *cp = &P.cand[(size_t)s * P.sn + i];
            long long kl = cp->x, ku = cp->y;
            cp->x = dkey(-INF);
            cp->y = dkey(INF);
            P.vflag[(size_t)s * P.snw + (i >> 5)] = 0u;  // whole word: every var in it is handled this round
            SlotInfo &S = P.info[s];
            if (S.row_bad_count == 0) {
                double2 *bp = &P.bnd[(size_t)s * P.sn + i];
                double2 b = bview(P, s, I.base)[i];
                bool is_int = I.vtype[i] != 0;
                double L = dunkey(kl), U = dunkey(ku);
                double nl = b.x, nu = b.y;
                bool ch = false;
                if (take_upper(is_int, U, b.y, P.tau)) { nu = canon0(U); ch = true; }
                if (take_lower(is_int, L, b.x, P.tau)) { nl = canon0(L); ch = true; }
                if (ch && nl > nu) {
                    if (is_int || nl - nu > P.feastol) atomicMin(&S.var_bad_min, i);
                    else nl = nu;
                }
                if (ch) {
                    *bp = make_double2(nl, nu);
                    go = true;
                    if (P.overlay) mark_dirty(P, s, i);
                    ol = b.x;
                    ou = b.y;
                    wl = nl;
                    wu = nu;
                }
            }
        }
        uint64_t wm = __ballot(go);
        if (P.touched) {  // byte accounting only
            unsigned long long ce = go ? (unsigned long long)clen : 0ull;
#pragma unroll
            for (int w = 1; w < 64; w <<= 1) ce += __shfl_xor(ce, w, 64);
            const unsigned long long ne = (unsigned long long)__popcll(__ballot(has));
            if (lane == 0) {
                atomicAdd(&C->stat_apply_entries, ne);
                if (!scan_next && ce) atomicAdd(&C->stat_apply_colent, ce);
            }
        }
        if (scan_next) {
            // the next round scans every row for these variables
            w_written += (unsigned long long)__popcll(wm);
            if (go) atomicOr(&P.cbits[(size_t)npar * P.snw + (i >> 5)], 1u << (i & 31));
        } else if (single) {
            w_written += (unsigned long long)__popcll(wm);
            uint32_t r = 0;
            unsigned long long z = 0;
            enqueue_columns<MULTI>(P, npar, go, s, c0, clen, false, &r, &z, P.inc && !rebuild_next, ol, ou,
                                   wl, wu);
            w_rows += r;
            w_nnz += z;
        } else {
            if (wm && lane == __ffsll((long long)wm) - 1)
                atomicAdd(&C->stat_written, (unsigned long long)__popcll(wm));
            enqueue_columns<MULTI>(P, npar, go, s, c0, clen, true, nullptr, nullptr, P.inc && !rebuild_next,
                                   ol, ou, wl, wu);
        }
    }
    // many changes: the next round rebuilds the heavy-row accumulators
    if (rebuild_next && blockIdx.x == 0 && threadIdx.x == 0) C->hbuild[npar] = 1u;
    if (single) {
        __shared__ unsigned long long a_rows[WG / 64], a_nnz[WG / 64], a_written[WG / 64];
        const int wave = threadIdx.x >> 6;
        if (lane == 0) {
            a_rows[wave] = w_rows;
            a_nnz[wave] = w_nnz;
            a_written[wave] = w_written;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long r = 0, z = 0, w = 0;
            for (int j = 0; j < WG / 64; ++j) {
                r += a_rows[j];
                z += a_nnz[j];
                w += a_written[j];
            }
            if (r) {
                atomicAdd(&P.info[0].pending_rows, (int32_t)r);
                atomicAdd(&P.info[0].pending_nnz, z);
            }
            if (w) atomicAdd(&C->stat_written, w);
            if (scan_next && w) C->scan_go = 1u;
            if (scan_next && blockIdx.x == 0) C->scan[npar] = 1u;
        }
    }
}

// ------------------------------------------------------------------------
// Jobs (the paper's Section 2.2 probing, and serving requests).  A job is
// either a probe (fix binary a at value b) or a fixing job (apply the bound
// fixings [a, a+b) of the fix list and propagate).  Jobs are admitted in
// order into free slots at round boundaries; their bounds are an overlay
// on the instance's base.
// ------------------------------------------------------------------------
enum : int32_t { JOB_PROBE = 0, JOB_FIX = 1 };

// The restriction a probe job applies to integer variable j with base
// bounds [l, u] (Section 2.2, probing cache), side h in {0, 1}: a binary
// (base inside [0, 1]) is fixed to h; a boxed integer takes the half below
// or at and above (l + u) / 2, [l, ceil((l + u)/2) - 1] or
// [ceil((l + u)/2), u]; an integer bounded below only takes x = l or
// x >= l + 1, one bounded above only x <= u - 1 or x = u.  The result is
// intersected with [l, u] by the caller.  False for a variable with no
// finite bound (never admitted: the entry points reject it).
__device__ __forceinline__ bool probe_restriction(double l, double u, int h, double &lo, double &hi) {
    const double INF = __builtin_inf();
    if (l >= 0.0 && u <= 1.0) {
        lo = hi = (double)h;
    } else if (l > -INF && u < INF) {
        const double mid_up = ceil((l + u) / 2.0);
        lo = h ? mid_up : l;
        hi = h ? u : mid_up - 1.0;
    } else if (l > -INF) {
        lo = h ? l + 1.0 : l;
        hi = h ? u : l;
    } else if (u < INF) {
        lo = h ? u : l;
        hi = h ? u : u - 1.0;
    } else {
        return false;
    }
    return true;
}

struct Job {
    int32_t inst, kind, a, b;
};

struct JobIO {
    const Job *jobs;         // [total]
    const int32_t *fix_var;  // fixings of JOB_FIX jobs
    const double2 *fix_box;
    int8_t *status;          // [total]
    int32_t *rounds;
    int64_t *nnz;
    int32_t *n_bad_rows;     // infeasibility evidence (may be null)
    int32_t *bad_row;
    int32_t *bad_var;
    int64_t *stage_off;      // [total] start of the job's staged list
    int64_t *stage_cnt;      // [total] its length
    int32_t *stage_var;      // [stage_cap] lists, ascending within a job
    double *stage_lb, *stage_ub;
    int64_t stage_cap;
    uint32_t *done_ring;     // finished job ids in completion order (may be null)
};

constexpr int SORT_MAX = 4096;  // lists up to this length are sorted in LDS

struct RetireScratch {
    int32_t key[SORT_MAX];
    uint32_t wsum[WG];
    uint32_t total;
    long long off;
    int32_t job, flag, badv;
    uint32_t rows;
    unsigned long long nnz;
    // the claimed job: its descriptor and, for a probe, the variable's base
    // bounds and column range
    Job jd;
    double2 pb;
    long long pc0, pc1;
};

// Write a job's outcome and reserve its staged list: at the offset and
// ring position the round end assigned (pre), or by atomics.
__device__ void write_job(const Params &P, const JobIO &IO, int p, int status, int rounds,
                          unsigned long long nnz, int nbad, int badrow, int badvar, int cnt,
                          RetireScratch &R, const SlotInfo *pre = nullptr) {
    if (threadIdx.x == 0) {
        IO.status[p] = (int8_t)status;
        IO.rounds[p] = rounds;
        IO.nnz[p] = (int64_t)nnz;
        if (IO.n_bad_rows) {
            IO.n_bad_rows[p] = nbad;
            IO.bad_row[p] = badrow;
            IO.bad_var[p] = badvar;
        }
        const unsigned long long off =
            pre ? pre->stage_off : atomicAdd(&P.ctl->stage_count, (unsigned long long)cnt);
        IO.stage_off[p] = (int64_t)off;
        IO.stage_cnt[p] = cnt;
        R.off = (long long)off;
        if (IO.done_ring) {
            const uint32_t d = pre ? pre->ring_pos : atomicAdd(&P.ctl->done_jobs, 1u);
            IO.done_ring[d] = (uint32_t)p;
        }
    }
    __syncthreads();
}

// Stage the dirty variables of slot s (with their bounds) in ascending order
// at R.off: bitonic sort in LDS for short lists, an ordered scan of the
// dirty bitmap for long ones.
__device__ void stage_sorted(const Params &P, const JobIO &IO, int s, const DInst &I, int cnt,
                             RetireScratch &R) {
    const long long off = R.off;
    if (off + cnt > IO.stage_cap) return;  // counted only; the call reports the size
    const BView bnd = bview(P, s, I.base);
    if (cnt <= SORT_MAX) {
        int npow = 1;
        while (npow < cnt) npow <<= 1;
        for (int t = threadIdx.x; t < npow; t += WG)
            R.key[t] = t < cnt ? P.dlist[(size_t)s * P.sn + t] : 0x7fffffff;
        __syncthreads();
        for (int size = 2; size <= npow; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = threadIdx.x; t < npow; t += WG) {
                    int u = t ^ stride;
                    if (u > t) {
                        bool up = (t & size) == 0;
                        int a = R.key[t], b = R.key[u];
                        if ((a > b) == up) {
                            R.key[t] = b;
                            R.key[u] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int t = threadIdx.x; t < cnt; t += WG) {
            int i = R.key[t];
            double2 b = bnd[i];
            IO.stage_var[off + t] = i;
            IO.stage_lb[off + t] = b.x;
            IO.stage_ub[off + t] = b.y;
        }
        __syncthreads();
    } else {
        const uint32_t *dw = P.dirty + (size_t)s * P.snw;
        const int nw = (I.n + 31) / 32;
        long long run = 0;
        for (int w0 = 0; w0 < nw; w0 += WG) {
            int w = w0 + threadIdx.x;
            uint32_t bits = w < nw ? dw[w] : 0u;
            R.wsum[threadIdx.x] = (uint32_t)__popc(bits);
            __syncthreads();
            if (threadIdx.x == 0) {  // exclusive prefix of the popcounts
                uint32_t acc = 0;
                for (int t = 0; t < WG; ++t) {
                    uint32_t x = R.wsum[t];
                    R.wsum[t] = acc;
                    acc += x;
                }
                R.total = acc;
            }
            __syncthreads();
            long long pos = run + R.wsum[threadIdx.x];
            while (bits) {
                int b = __ffs(bits) - 1;
                bits &= bits - 1;
                int i = w * 32 + b;
                double2 bb = bnd[i];
                IO.stage_var[off + pos] = i;
                IO.stage_lb[off + pos] = bb.x;
                IO.stage_ub[off + pos] = bb.y;
                ++pos;
            }
            run += R.total;
            __syncthreads();
        }
    }
}

// With incremental heavy rows over the base: clear the corrections of
// every heavy row holding one of slot s's cnt dirty variables (a row's
// corrections come only from bound changes of its own variables, all of
// which are dirty).  Each wave takes a variable and walks its column 64
// entries at a time, marking the column's heavy rows in an LDS bitmap;
// the workgroup then clears the marked rows together, so that the clears
// of a slot's rows are in flight at once.  (Instances of more heavy rows
// than the bitmap holds clear each row as its column walk finds it.)  The
// clears are atomics like the next job's corrections, and their results
// are waited for: they are done when the caller's next barrier is.
constexpr int CLEAR_MAP = 64;  // bitmap words (one per lane of a wave)
static_assert(CLEAR_MAP == 64 && SORT_MAX >= CLEAR_MAP * 33, "clear bitmap and row list fit the sort keys");
__device__ void clear_heavy(const Params &P, const DInst &I, int s, int cnt, RetireScratch &R) {
    if (!(P.inc && P.inc_base)) return;  // uniform
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const int w0 = wave, nw = WG / 64;
    unsigned long long junk = 0;
    if (cnt < P.nheavy && P.nheavy <= CLEAR_MAP * 32) {  // uniform
        uint32_t *map = (uint32_t *)R.key;
        int32_t *list = R.key + CLEAR_MAP;
        if (threadIdx.x < CLEAR_MAP) map[threadIdx.x] = 0u;
        __syncthreads();
        for (int t = wave; t < cnt; t += nw) {
            const int i = P.dlist[(size_t)s * P.sn + t];
            const int64_t c0 = I.col_ptr[i], c1 = I.col_ptr[i + 1];
            for (int64_t e = c0 + lane; e < c1; e += 64) {
                const int h = I.hidx[I.col_row[e]];
                if (h >= 0) atomicOr(&map[h >> 5], 1u << (h & 31));
            }
        }
        __syncthreads();
        if (wave == 0) {  // the marked rows, in order, by a prefix of the words' popcounts
            const uint32_t w = map[lane];
            const int c = __popc(w);
            int x = c;
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(x, d, 64);
                if (lane >= d) x += y;
            }
            int pos = x - c;
            for (uint32_t b = w; b; b &= b - 1) list[pos++] = lane * 32 + __ffs(b) - 1;
            if (lane == 63) R.total = (uint32_t)x;
        }
        __syncthreads();
        const int per = 2 * HL + 2;  // limbs of both sides, then the two infinite counts
        const int items = (int)R.total * per;
        for (int u = threadIdx.x; u < items; u += WG) {
            const int q = u / per, j = u - q * per;
            const size_t hs = (size_t)s * P.nheavy + list[q];
            if (j < 2 * HL) junk |= atomicExch((unsigned long long *)(P.hacc + hs * 2 * HL) + j, 0ull);
            else junk |= (unsigned long long)(uint32_t)atomicExch(&P.hinf[2 * hs + (j - 2 * HL)], 0);
        }
        asm volatile("" ::"v"(junk));
        return;
    }
    if (cnt >= P.nheavy) {
        // a long list (a fixing job): every heavy row of the slot instead
        const size_t n = (size_t)P.nheavy * 2 * HL, t0 = (size_t)w0 * 64 + lane, step = (size_t)nw * 64;
        unsigned long long *L = (unsigned long long *)(P.hacc + (size_t)s * n);
        for (size_t j = t0; j < n; j += step) junk |= atomicExch(&L[j], 0ull);
        for (size_t j = t0; j < 2 * (size_t)P.nheavy; j += step)
            junk |= (unsigned long long)(uint32_t)atomicExch(&P.hinf[(size_t)s * 2 * P.nheavy + j], 0);
        cnt = 0;
    }
    for (int t = w0; t < cnt; t += nw) {
        const int i = P.dlist[(size_t)s * P.sn + t];
        const int64_t c0 = I.col_ptr[i], c1 = I.col_ptr[i + 1];
        for (int64_t e0 = c0; e0 < c1; e0 += 64) {
            const int64_t e = e0 + lane;
            const int h = e < c1 ? I.hidx[I.col_row[e]] : -1;
            uint64_t hm = __ballot(h >= 0);
            while (hm) {
                const int q = __ffsll((long long)hm) - 1;
                hm &= hm - 1;
                const size_t hs = (size_t)s * P.nheavy + __shfl(h, q, 64);
                unsigned long long *L = (unsigned long long *)(P.hacc + hs * 2 * HL);
                for (int j = lane; j < 2 * HL; j += 64) junk |= atomicExch(&L[j], 0ull);
                if (lane < 2) junk |= (unsigned long long)(uint32_t)atomicExch(&P.hinf[2 * hs + lane], 0);
            }
        }
    }
    asm volatile("" ::"v"(junk));
}

// Forget the dirty variables of slot s (instance I): it reads the base
// again, and its heavy-row corrections are cleared.  (Clearing them in two
// waves while the others write the job's results was timed slower.)  R's
// sort keys are free here and serve the clear.
__device__ void restore_slot(const Params &P, const DInst &I, int s, int cnt, RetireScratch &R) {
    uint32_t *dw = P.dirty + (size_t)s * P.snw;
    uint32_t *fw = P.filt + (size_t)s * FILT_WORDS;
    for (int t = threadIdx.x; t < cnt; t += WG) {
        int i = P.dlist[(size_t)s * P.sn + t];
        // every set bit of these words belongs to this list
        dw[i >> 5] = 0u;
        fw[fhash(i) >> 5] = 0u;
    }
    clear_heavy(P, I, s, cnt, R);
    __syncthreads();
    if (threadIdx.x == 0) P.dcount[s] = 0;
    __syncthreads();
}

__device__ __forceinline__ int dcount_now(const Params &P, int s) {
    return (int)__hip_atomic_load(&P.dcount[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Claim the next job (by thread 64, the second wave, so that the round
// trips overlap the first wave's work) and read what its admission needs
// first: the descriptor and, for a probe, the variable's base bounds and
// column range.  Visible to the workgroup after its next barrier.
template <bool MULTI>
__device__ __forceinline__ void claim_job(const Params &P, const JobIO &IO, RetireScratch &R,
                                          const SlotInfo *pre = nullptr) {
    if (threadIdx.x != 64) return;
    uint32_t p;
    if (pre) p = pre->claim == CLAIM_NONE ? 0xffffffffu : (uint32_t)pre->claim;  // assigned at the round end
    else p = atomicAdd(&P.ctl->next_job, 1u);
    R.job = (int)p;
    if (p >= P.ctl->total_jobs) return;
    const Job J = IO.jobs[p];
    R.jd = J;
    if (J.kind == JOB_PROBE) {
        DInst I;
        if constexpr (MULTI) I = P.insts[J.inst];
        else I = P.I;
        R.pb = I.base[J.a];
        R.pc0 = I.col_ptr[J.a];
        R.pc1 = I.col_ptr[J.a + 1];
    }
}

// The first dirty variable of a clean slot (every free slot is clean): no
// returning atomics are needed to find out that it is new.
__device__ __forceinline__ void mark_dirty_first(const Params &P, int s, int i) {
    atomicOr(&P.dirty[(size_t)s * P.snw + (i >> 5)], 1u << (i & 31));
    const uint32_t h = fhash(i);
    atomicOr(&P.filt[(size_t)s * FILT_WORDS + (h >> 5)], 1u << (h & 31));
    P.dlist[(size_t)s * P.sn] = i;
    P.dcount[s] = 1;
}

// Set up the claimed job p (its descriptor and first reads in R) in the
// free slot s.  Returns true if the slot now runs it; false if the job
// finished at admission (its results are written).
template <bool MULTI>
__device__ bool admit_job(const Params &P, const JobIO &IO, int s, int p, int par,
                          RetireScratch &R) {
    SlotInfo &S = P.info[s];
    const Job J = R.jd;
    DInst I;
    if constexpr (MULTI) I = P.insts[J.inst];
    else I = P.I;
    double2 pbox = make_double2(0.0, 0.0);  // a probe's box, within the base
    if (J.kind == JOB_PROBE) {
        const int j = J.a;
        const double2 b = R.pb;
        double lo = 0.0, hi = 0.0;
        probe_restriction(b.x, b.y, J.b, lo, hi);
        pbox = make_double2(canon0(fmax(lo, b.x)), canon0(fmin(hi, b.y)));
        if (pbox.x > pbox.y) {  // the restriction leaves nothing of the base box
            write_job(P, IO, p, 1, 0, 0ull, 0, -1, j, 0, R);
            return false;
        }
        if (pbox.x == b.x && pbox.y == b.y) {  // the base already lies in it
            write_job(P, IO, p, 0, 0, 0ull, 0, -1, -1, 0, R);
            return false;
        }
    }
    if (threadIdx.x == 0) {
        S.status = 0;
        S.rounds = 0;
        S.row_bad_min = NONE;
        S.row_bad_count = 0;
        S.var_bad_min = NONE;
        S.pending_rows = 0;
        S.pending_nnz = 0;
        S.nnz = 0;
        S.job = p;
        S.retire = 0;
        S.inst = J.inst;
        R.badv = NONE;
        R.rows = 0;
        R.nnz = 0;
    }
    __syncthreads();
    // Apply the job's bounds (each changed variable becomes dirty).
    if (J.kind == JOB_PROBE) {
        if (threadIdx.x == 0) {
            P.bnd[(size_t)s * P.sn + J.a] = pbox;
            mark_dirty_first(P, s, J.a);
        }
    } else {
        for (int f = J.a + threadIdx.x; f < J.a + J.b; f += WG) {
            const int i = IO.fix_var[f];
            const double2 fb = IO.fix_box[f];
            const double2 b = I.base[i];
            double nl = canon0(fmax(b.x, fb.x)), nu = canon0(fmin(b.y, fb.y));
            double slack = I.vtype[i] ? 0.0 : P.feastol;
            if (nl > nu + slack) atomicMin(&R.badv, i);
            if (nl != b.x || nu != b.y) {
                P.bnd[(size_t)s * P.sn + i] = make_double2(nl, nu);
                mark_dirty(P, s, i);
            }
        }
    }
    __syncthreads();
    const bool probe = J.kind == JOB_PROBE;
    const int nd = probe ? 1 : dcount_now(P, s);
    if (R.badv != NONE) {  // a crossed box before the first round
        write_job(P, IO, p, 1, 0, 0ull, 0, -1, R.badv, 0, R);
        restore_slot(P, I, s, nd, R);
        return false;
    }
    // The first round holds the rows of the changed variables; with
    // incremental heavy rows their changes from the base bounds are the
    // slot's first corrections.
    const int wave = threadIdx.x >> 6;
    for (int d0 = wave * 64; d0 < nd; d0 += WG) {
        int d = d0 + __lane_id();
        bool want = d < nd;
        long long c0 = 0;
        uint32_t len = 0;
        double2 ob = make_double2(0.0, 0.0), nb = make_double2(0.0, 0.0);
        if (want && probe) {  // the probed variable, read at the claim
            c0 = R.pc0;
            len = (uint32_t)(R.pc1 - R.pc0);
            ob = R.pb;
            nb = pbox;
        } else if (want) {
            int i = P.dlist[(size_t)s * P.sn + d];
            c0 = I.col_ptr[i];
            len = (uint32_t)(I.col_ptr[i + 1] - c0);
            if (P.inc) {
                ob = I.base[i];
                nb = P.bnd[(size_t)s * P.sn + i];
            }
        }
        uint32_t rows = 0;
        unsigned long long nnz = 0;
        enqueue_columns<MULTI>(P, par, want, s, c0, len, false, &rows, &nnz, P.inc != 0, ob.x, ob.y,
                               nb.x, nb.y);
        if (__lane_id() == 0) {
            atomicAdd(&R.rows, rows);
            atomicAdd(&R.nnz, nnz);
        }
    }
    __syncthreads();
    if (R.rows > 0) {
        if (threadIdx.x == 0) {
            S.rounds = 1;
            S.nnz = R.nnz;
            S.state = SLOT_ACTIVE;
            atomicAdd(&P.ctl->stat_rows, (unsigned long long)R.rows);
            atomicAdd(&P.ctl->stat_nnz, R.nnz);
        }
        __syncthreads();
        return true;
    }
    // Changed variables in no row: nothing to propagate; the list is the
    // changed variables themselves.
    write_job(P, IO, p, 0, 0, 0ull, 0, -1, -1, nd, R);
    stage_sorted(P, IO, s, I, nd, R);
    restore_slot(P, I, s, nd, R);
    return false;
}

// One workgroup per slot: write the results of a slot that finished at the
// last round end, restore it, then admit the next jobs into free slots.
template <bool MULTI>
__global__ void __launch_bounds__(WG) k_retire(Params P, JobIO IO) {
    __shared__ RetireScratch R;
    Ctl *C = P.ctl;
    const int par = C->round & 1;
    for (int s = blockIdx.x; s < P.nslots; s += gridDim.x) {
        SlotInfo &S = P.info[s];
        // A slot that is free after this step (retired without draining, or
        // idle) claims its next job before retiring the last one.
        const bool admits = S.state == SLOT_FREE;
        const SlotInfo *pre = C->claims ? &S : nullptr;
        if (admits) claim_job<MULTI>(P, IO, R, pre);
        if (S.retire) {
            const int p = S.job;
            const int status = S.status;
            const int dcnt = dcount_now(P, s);
            const int cnt = status == 1 ? 0 : dcnt;
            DInst I;
            if constexpr (MULTI) I = P.insts[S.inst];
            else I = P.I;
            int nbad = 0, brow = -1, bvar = -1;
            if (status == 1) {
                if (S.row_bad_count > 0) {
                    nbad = S.row_bad_count;
                    brow = S.row_bad_min;
                } else {
                    bvar = S.var_bad_min;
                }
            }
            write_job(P, IO, p, status, S.rounds, S.nnz, nbad, brow, bvar, cnt, R, pre);
            if (cnt > 0) stage_sorted(P, IO, s, I, cnt, R);
            restore_slot(P, I, s, dcnt, R);
            if (threadIdx.x == 0) S.retire = 0;
            __syncthreads();
        }
        if (!admits) continue;
        // Admit jobs until one needs rounds or none is left.  A claim past
        // the end of the list takes no job; the counter may then exceed the
        // list length, and a host that appends jobs first lowers it back to
        // the old length (no kernel runs meanwhile).
        __syncthreads();
        for (;;) {
            const uint32_t p = (uint32_t)R.job;
            __syncthreads();
            if (p >= C->total_jobs) break;
            if (admit_job<MULTI>(P, IO, s, (int)p, par, R)) break;
            claim_job<MULTI>(P, IO, R);
            __syncthreads();
        }
        __syncthreads();
    }
}

// off[p+1] = off[p] + count[p] over np jobs (one workgroup).
__global__ void __launch_bounds__(WG) k_job_offsets(const int64_t *cnt, int64_t *off, int64_t np) {
    __shared__ long long part[WG];
    __shared__ long long carry;
    if (threadIdx.x == 0) {
        carry = 0;
        off[0] = 0;
    }
    __syncthreads();
    for (int64_t b0 = 0; b0 < np; b0 += WG) {
        int64_t p = b0 + threadIdx.x;
        long long x = p < np ? cnt[p] : 0;
        part[threadIdx.x] = x;
        __syncthreads();
        for (int d = 1; d < WG; d <<= 1) {
            long long y = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += y;
            __syncthreads();
        }
        if (p < np) off[p + 1] = carry + part[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == WG - 1) carry += part[WG - 1];
        __syncthreads();
    }
}

// Copy every job's staged list to its place in the caller's arrays.
__global__ void k_job_gather(const JobIO IO, const int64_t *off, int64_t np, int32_t *ovar,
                             double *olb, double *oub) {
    for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
        int64_t src = IO.stage_off[p], dst = off[p], c = IO.stage_cnt[p];
        for (int64_t t = threadIdx.x; t < c; t += blockDim.x) {
            ovar[dst + t] = IO.stage_var[src + t];
            olb[dst + t] = IO.stage_lb[src + t];
            oub[dst + t] = IO.stage_ub[src + t];
        }
    }
}

// Probe jobs 2t + v: binary vars[t] at value v.
__global__ void k_make_probe_jobs(const int32_t *vars, int32_t k, Job *jobs) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < 2 * k; p += gridDim.x * blockDim.x) {
        Job J;
        J.inst = 0;
        J.kind = JOB_PROBE;
        J.a = vars[p >> 1];
        J.b = p & 1;
        jobs[p] = J;
    }
}

}  // namespace bp
