/*
 * bp.h -- C ABI of the MI355X bound-propagation library (libbp.so).
 *
 * The library propagates variable bounds through the rows of a sparse MILP
 * constraint matrix (the paper's Section 2.1, "Bound Propagation") and
 * probes binary variables at 0 and at 1 to fill a probing cache (Section
 * 2.2, "Probing Cache").  Every compute step runs in HIP kernels written
 * for gfx950; no C++ type, exception or torch type crosses this boundary.
 *
 * Problem.  Rows k = 0..m-1 read  lo_k <= sum_i a_ki x_i <= hi_k  (either
 * side may be infinite; the paper's form  sum a z <= g  is lo = -inf).
 * Variables i = 0..n-1 carry bounds [lb_i, ub_i] (either may be infinite)
 * and a type: 0 continuous, 1 integer (binaries are integers in [0, 1]).
 *
 * Propagation semantics (what every entry point computes).  Rounds are
 * round-synchronous: each round reads the bounds as they were when it
 * started.  Round r processes the rows that hold a variable whose bounds
 * changed in round r-1 (all rows in the first round of a cold start;
 * Section 1 names this "propagation on changed constraints").  For each such
 * row the minimum and maximum activities (Section 2.1, first display, and
 * its mirror) are the correctly rounded exact sums of the rounded finite
 * terms fl(a*b), with infinite contributions counted.  A row whose minimum
 * activity exceeds hi + feastol, or whose maximum activity is below
 * lo - feastol, with no infinite contribution, is infeasible.  Each nonzero
 * yields bound candidates (Section 2.1, second display, and its mirror):
 * v = fl(fl(side - activity) + fl(a*b_own)) (or fl(side - activity) when
 * the variable's own contribution is the single infinite one), c = fl(v/a);
 * integer variables take floor(c + inttol) for upper and ceil(c - inttol)
 * for lower candidates.  A variable takes the tightest candidate of each
 * side if it passes the threshold (Section 2.1, closing sentence): any
 * strict improvement for integers; for continuous variables an old
 * infinite bound, or a move larger than tau * max(1, |old|).  Crossed
 * bounds are infeasible for integers and for continuous variables crossed
 * by more than feastol; otherwise lb is set to ub.  -0.0 is stored as +0.0.
 * The loop stops when a round changes nothing (BP_OK), when a row or a
 * variable is infeasible (BP_INFEASIBLE, at the end of the detecting round),
 * or after max_rounds rounds with work left (BP_ROUND_LIMIT).
 *
 * Memory.  bp_load takes host arrays and copies them; the caller may free
 * them on return.  All other entry points take device pointers (for example
 * torch tensors' data_ptr()) for bounds, variable lists and outputs, and
 * host pointers for result structs.  Each call runs on the given HIP stream
 * (NULL: the null stream) and returns once its results are complete.
 *
 * Threads.  An instance is not thread-safe; distinct instances may be used
 * from distinct threads on distinct streams.
 *
 * Errors.  Negative return codes are errors; outputs are then untouched
 * except where stated.  bp_last_error() returns a thread-local message.
 */
#ifndef BP_H
#define BP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Outcomes (>= 0) and errors (< 0). */
#define BP_OK 0
#define BP_INFEASIBLE 1
#define BP_ROUND_LIMIT 2
#define BP_EINVAL (-1)     /* malformed input: NaN, lo > hi, unsorted or duplicate
                              columns, explicit zero, index out of range, CSC not
                              the transpose, probe variable not an integer with a
                              finite base bound */
#define BP_ENOMEM (-2)     /* device or host allocation failed */
#define BP_EDEVICE (-3)    /* a HIP call failed */
#define BP_ECAPACITY (-4)  /* an output buffer is too small (see bp_probe_out) */
#define BP_ESTATE (-5)     /* bp_probe before a feasible base exists */
#define BP_ECANCELED (-6)  /* bp_server_results of a request that was cancelled */

/* Flags (bp_options.flags). */
#define BP_FLAG_FORCE_EXACT 1u  /* compute every activity on the exact slow path
                                   (a check of that path; results are identical) */
#define BP_FLAG_TIME_KERNELS 2u /* time the activity kernel with HIP events; read
                                   the totals with bp_kernel_stats */
#define BP_FLAG_HOST_ROUNDS 4u  /* drive rounds from the host one at a time
                                   instead of device-resident graphs of rounds */
#define BP_FLAG_COUNT_VARS 8u   /* count the distinct bound records each round
                                   gathers (bp_stats.vars_read); slower, for
                                   byte accounting only */
#define BP_FLAG_BATCH_SLOTS 16u /* run bp_propagate_batch on the slot engine
                                   (one slot per vector) whatever the batch
                                   size; results are identical */
#define BP_FLAG_LV_DENSE 64u    /* bp_propagate_batch (one vector per lane): keep
                                   every vector's records whole even when the
                                   instance has a base (no overlay on it);
                                   results are identical */
#define BP_FLAG_FULL_ROWS 32u   /* bp_propagate: recompute every queued heavy
                                   row from its nonzeros each round instead of
                                   keeping its exact activities up to date
                                   through the bound changes; results are
                                   identical */

/* A sparse matrix in compressed form: CSR (ptr over m rows, idx = column
 * indices ascending in each row) or CSC (ptr over n columns, idx = row
 * indices ascending in each column).  ptr has length (CSR: m, CSC: n) + 1,
 * ptr[0] = 0 and the last entry = nnz; idx and val have length nnz. */
typedef struct {
    int64_t m, n, nnz;
    const int64_t *ptr;
    const int32_t *idx;
    const double *val;
} bp_sparse;

typedef struct {
    double feastol;      /* absolute feasibility tolerance, default 1e-6 */
    double inttol;       /* integer rounding tolerance, default 1e-6 */
    double tau;          /* continuous threshold, default 1e-3 */
    int32_t max_rounds;  /* default 1000 */
    uint32_t flags;      /* BP_FLAG_* */
    int32_t heavy_threshold; /* rows longer than this are split across
                                workgroups; default 8192 (0: default) */
    int32_t rounds_per_launch; /* rounds per captured graph; default 16.  A
                                  bp_probe call after the instance's first
                                  uses the smallest power of two from 8 up
                                  that covered the last call's rounds, when
                                  that is fewer */
    int32_t probe_slots; /* bound vectors in flight during bp_probe; default 512 */
    int32_t heavy_chunk; /* nonzeros per workgroup of a heavy row; default 1024,
                            rounded up to a multiple of 256 */
    int32_t repair_calls;    /* bp_round: repair procedures per rounding on a
                                marked path; default 0 (no repair) */
    int32_t repair_attempts; /* bp_round: attempts per repair; default 8 (0: default) */
    int32_t repair_shifts;   /* bp_round: shifts per attempt; default 64 (0: default) */
    int32_t lv_grid;         /* bp_propagate_batch, one vector per lane: workgroups
                                per round kernel over all vector groups; default
                                2048 (0: default) */
} bp_options;

typedef struct {
    int32_t status;            /* BP_OK, BP_INFEASIBLE or BP_ROUND_LIMIT */
    int32_t rounds;            /* rounds with a non-empty row worklist */
    int64_t nnz_propagated;    /* sum over rounds of the nonzeros of their rows */
    int32_t n_infeasible_rows; /* infeasible rows in the detecting round */
    int32_t infeasible_var;    /* smallest crossed variable, or -1 */
    int64_t infeasible_row;    /* smallest infeasible row, or -1 (rows take
                                  precedence over variables) */
} bp_result;

/* Outputs of bp_probe, all caller-owned DEVICE buffers except the two
 * int64 fields.  Probe p = 2t + v is vars[t] fixed to v (double probing,
 * Section 2.2).  Its implied list holds every variable whose (lb, ub)
 * differs from the base, the probed variable included, ascending by
 * variable; it is empty for infeasible probes and for a probe whose value
 * the base already fixes. */
typedef struct {
    /* status/rounds/nnz may be NULL when k == 0; off always has 2k+1 entries */
    int8_t *status;    /* [2k] BP_OK / BP_INFEASIBLE / BP_ROUND_LIMIT */
    int32_t *rounds;   /* [2k] */
    int64_t *nnz;      /* [2k] nnz propagated */
    int64_t *off;      /* [2k+1] list offsets */
    int32_t *var;      /* [cap] */
    double *lb;        /* [cap] */
    double *ub;        /* [cap] */
    int64_t cap;       /* capacity of var/lb/ub (in) */
    int64_t required;  /* total implied entries (out; set also on BP_ECAPACITY) */
} bp_probe_out;

typedef struct bp_instance bp_instance;

/* Counters since load or the last reset.  ms and launches cover the
 * activity kernel (k_rows) and apply_ms the bound-update kernel (k_apply)
 * when BP_FLAG_TIME_KERNELS is set; vars_read, the kept-row counts and the
 * apply_* counts need BP_FLAG_COUNT_VARS; the other fields are kept always. */
typedef struct {
    double ms;            /* summed HIP-event time of the activity kernel */
    int64_t launches;     /* activity-kernel launches timed */
    int64_t rows;         /* row tasks processed (sum over rounds of |R_r|) */
    int64_t nnz;          /* nonzeros of those rows */
    int64_t vars_read;    /* distinct (vector, variable) bound records read per
                             round, summed over rounds */
    int64_t vars_written; /* bound records written (accepted changes) */
    int64_t rows_kept;    /* queued heavy rows of a single vector tested from
                             their incremental accumulators (BP_FLAG_COUNT_VARS) */
    int64_t nnz_kept;     /* nonzeros of those rows never read in their round
                             (no candidates were needed; BP_FLAG_COUNT_VARS) */
    double apply_ms;        /* summed HIP-event time of the bound-update kernel */
    int64_t apply_entries;  /* changed-list entries it took */
    int64_t apply_colent;   /* column entries it walked for accepted changes */
    int64_t apply_corr;     /* heavy-row accumulator corrections it made */
    int64_t rows_union;     /* distinct rows read per round over all vectors of
                               a call, summed over rounds (BP_FLAG_COUNT_VARS;
                               bp_propagate, bp_propagate_batch on the slot
                               engine and bp_probe; scan rounds not counted) */
    int64_t nnz_union;      /* nonzeros of those rows */
    int64_t lv_corr_chunks; /* long-row chunk tasks of the one-vector-per-lane
                               batch engine summed as the chunk's sums at the
                               base bounds plus each vector's corrections */
} bp_stats;

/* Fill *opt with the defaults. */
void bp_options_default(bp_options *opt);

/* Load an instance (host arrays; copied to the device).
 *   csr      the constraint matrix by rows (required)
 *   csc      the same matrix by columns, or NULL to build it; if given it is
 *            checked to be the transpose of csr (BP_EINVAL otherwise)
 *   row_lo, row_hi  [m] sides (+-inf allowed, lo <= hi, lo != +inf, hi != -inf)
 *   vartype  [n] 0 continuous, 1 integer
 *   opt      options, or NULL for the defaults
 *   stream   HIP stream (hipStream_t) for the uploads
 *   out      receives the instance handle
 * The matrix is validated: columns ascending and distinct in each row,
 * indices in range, coefficients finite and nonzero (BP_EINVAL).  Rows and
 * columns are binned by length (the paper's Section 2.1 load-balancing
 * paragraph). */
int bp_load(const bp_sparse *csr, const bp_sparse *csc, const double *row_lo,
            const double *row_hi, const uint8_t *vartype, const bp_options *opt,
            void *stream, bp_instance **out);

/* Propagate one bound vector to its fixed point.
 *   lb, ub     DEVICE [n], read and overwritten with the result
 *   changed    DEVICE [n_changed] variable ids whose bounds the caller changed
 *              since a fixed point; NULL (with any n_changed) for a cold start
 *              in which the first round holds every row
 *   res        HOST, receives the outcome
 * Returns res->status, or an error.  After BP_OK the result becomes the
 * instance's base for bp_probe.  After BP_INFEASIBLE the bounds hold the
 * state at the end of the detecting round. */
int bp_propagate(bp_instance *h, double *lb, double *ub, const int32_t *changed,
                 int64_t n_changed, bp_result *res, void *stream);

/* Propagate B independent bound vectors together (bulk rounding candidates).
 *   lb, ub       DEVICE [B*n], vector b at offset b*n, read and overwritten
 *   changed_ptr  DEVICE [B+1] offsets into changed_idx, or NULL: cold start
 *                for every vector
 *   changed_idx  DEVICE variable ids
 *   res          HOST [B]
 * Returns BP_OK when the call ran (per-vector outcomes are in res) or an
 * error.  Does not change the base.  The bounds of a vector whose outcome
 * is BP_INFEASIBLE are unspecified (with 16 or more vectors they keep the
 * input).  Batches of 16 or more vectors run one vector per lane (bounds
 * stored [variable][vector] in device memory the instance keeps; about
 * 40 B per variable and vector); BP_FLAG_BATCH_SLOTS keeps the slot
 * engine.  When the instance has a base (a BP_OK bp_propagate, which may
 * be a warm start with an empty change list from any box), the lanes read
 * each vector as an overlay on it: only the records that differ from the
 * base are stored and read per vector, which suits vectors that are the
 * base with a few changes (bulk rounding); BP_FLAG_LV_DENSE turns this
 * off.  Results are the same either way. */
int bp_propagate_batch(bp_instance *h, int32_t B, double *lb, double *ub,
                       const int64_t *changed_ptr, const int32_t *changed_idx,
                       bp_result *res, void *stream);

/* Double probing (the paper's Section 2.2 probing cache): every integer
 * variable vars[t] (DEVICE [k]) is restricted in two ways and propagated
 * from the base; probe 2t+h is restriction h.  With base bounds [l, u]:
 *   - a binary (base inside [0, 1]): x = 0 (h = 0) and x = 1 (h = 1);
 *   - a boxed integer: x < (l+u)/2, i.e. [l, ceil((l+u)/2) - 1], and
 *     x >= (l+u)/2, i.e. [ceil((l+u)/2), u];
 *   - only l finite: x = l and x >= l + 1;
 *   - only u finite: x <= u - 1 and x = u.
 * A restriction that leaves nothing of [l, u] is BP_INFEASIBLE before any
 * round; one that contains [l, u] is BP_OK with no rounds and no list.
 * Returns BP_OK, BP_ESTATE without a base, BP_EINVAL if a variable is not
 * an integer with a finite base bound, or BP_ECAPACITY (out->required set,
 * other outputs unspecified). */
int bp_probe(bp_instance *h, const int32_t *vars, int32_t k, bp_probe_out *out,
             void *stream);

/* Probe-priority and implied-slack scores of every variable j at the
 * bounds DEVICE lb/ub [n] (any bounds: the instance's own, a base, ...).
 * Row activities are those of propagation (correctly rounded sums of the
 * finite terms a*b, counts of the infinite ones).  With d = a*b_max -
 * a*b_min the amount by which moving j between its bounds moves row k's
 * extreme activities (b_min/b_max: the bound giving j's smallest/largest
 * contribution), and the slacks hi_k - minfin_k and maxfin_k - lo_k of the
 * finite sides without infinite terms:
 *   nviol[j]       rows whose d exceeds a slack by more than feastol
 *                  (Section 2.2: the violations revealed by flipping j's
 *                  contribution), counted only when j's coefficients have
 *                  both signs and both its bounds are finite; else 0;
 *   maxviol[j]     the largest such excess (0 if none);
 *   minunit[j]     the smallest slack / |a| over j's row sides (Section 2.2,
 *                  third criterion; +inf if none);
 *   slack_score[j] S_j = correctly rounded sum of (a / slack)^2 over the
 *                  same sides (Section 2.3, implied-slack sort; +inf if a
 *                  slack is zero, 0 if no side).
 * Each value is computed with a fixed operation order (no fused multiply-
 * add), so results are reproducible bit for bit.  Outputs are DEVICE [n],
 * caller-owned; any may be NULL.  Returns BP_OK, or BP_EINVAL for a null
 * argument or a NaN bound (outputs untouched). */
typedef struct {
    int32_t *nviol;
    double *maxviol;
    double *minunit;
    double *slack_score;
} bp_scores_out;

int bp_scores(bp_instance *h, const double *lb, const double *ub, bp_scores_out *out,
              void *stream);

/* bp_scores for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and results as bp_scores, bit for bit; the call allocates
 * nothing: its work buffers (packed bounds, 16 B per variable; row
 * activities, 16 B per row; the partial sums of the rows longer than 1024
 * nonzeros; each part rounded up to 256 B, plus 256 B) live in a static
 * device array of BP_SCORES_NOALLOC_MAX_BYTES that every device running the
 * library holds until the process ends.  An instance needing more returns
 * BP_EINVAL (outputs untouched).  All calls on one device share that array:
 * calls that overlap on one device (distinct streams or threads) race, and
 * the caller must order them.  The first call on a device also looks up the
 * array's device address (no allocation).  The instance's other entry
 * points are unaffected. */
#define BP_SCORES_NOALLOC_MAX_BYTES (64ll << 20)

int bp_scores_noalloc(bp_instance *h, const double *lb, const double *ub, bp_scores_out *out,
                      void *stream);

/* Probe order (Section 2.2): the DEVICE variable ids vars [k] sorted by
 * more violated rows first (nviol), then the larger maxviol, then the
 * smaller minunit, then the smaller id -- scores at DEVICE lb/ub [n] as
 * bp_scores computes them -- into DEVICE order [k] (caller-owned; ids may
 * repeat).  Returns BP_OK, or BP_EINVAL for k < 0, an id outside [0, n), a
 * null argument or a NaN bound (order untouched). */
int bp_probe_order(bp_instance *h, const double *lb, const double *ub, const int32_t *vars,
                   int32_t k, int32_t *order, void *stream);

/* Probing cache of binaries for bp_round: bp_probe's output for the DEVICE
 * variable ids vars [k], each a binary of the box the cache was computed
 * around (probe 2t + v fixed vars[t] to v); status [2k], off [2k + 1] and
 * the implied lists var / lb / ub [off[2k]] as bp_probe_out holds them.
 * The box given to bp_round must lie inside the cache's box. */
typedef struct {
    const int32_t *vars;
    int32_t k;
    const int8_t *status;
    const int64_t *off;
    const int32_t *var;
    const double *lb, *ub;
} bp_cache;

typedef struct {
    int32_t status;       /* BP_OK, or BP_INFEASIBLE for a path marked infeasible */
    int32_t bulks;        /* propagation steps with more than one variable */
    int32_t singles;      /* steps with one variable (recovery mode, last 36) */
    int32_t recoveries;   /* times recovery mode was entered */
    int32_t fixed;        /* integer variables fixed at the end */
    int32_t iterations;   /* steps in all */
    int64_t nnz_propagated; /* over every propagation of both bulks and of
                               the repairs */
    int32_t repairs;      /* repair procedures run (opt.repair_calls at most) */
    int32_t repaired;     /* of them, the ones that succeeded */
} bp_round_result;

/* Bound-propagation rounding (the paper's Algorithm 1 with Section 2.3,
 * without the LP polish): every integer variable of
 * the box DEVICE lb/ub [n] with lb < ub is fixed towards the fractional
 * point DEVICE x [n], a bulk at a time, each bulk propagated.
 *   - order: interval width 1, then 2, then wider; then the distance of x
 *     (clamped into the box) to the nearest integer; then index;
 *   - bulk size: with R variables unfixed, 1 in recovery mode or when
 *     R <= 36, else ceil(sqrt(R)); a bulk of more than one first re-sorts the
 *     unfixed variables by the implied-slack score S (bp_scores at the
 *     current box) descending, stably;
 *   - two candidate values per member, h = 0 and 1, from the caller's draws
 *     DEVICE draws [2n] in [0, 1) (draws[2j + h]): with x clamped into the
 *     box and f = x - floor(x), random rounding (up when the draw is below
 *     f) for 0.25 < f < 0.75, else the nearest integer;
 *   - with a cache: a member whose cached probe for its value is infeasible
 *     is dropped, then one whose value lies outside the box implied by the
 *     other members' cached lists; the kept members' fixings and cached
 *     implications start the bulk (warm start);
 *   - both bulks propagate as one bp_propagate_batch; the first not
 *     infeasible one is accepted (a bulk keeping no member fails); when both
 *     fail, recovery mode (one variable per bulk) is entered, or, if already
 *     in it, the path is marked infeasible and from then on a failed bulk's
 *     members are fixed to their first values without propagation;
 *   - with opt.repair_calls > 0 (instance options): while the path is
 *     marked, each step ends with bp_repair of the current box, with the
 *     box the call started from as the original box and the attempt and
 *     shift limits opt.repair_attempts / opt.repair_shifts, until a repair
 *     succeeds (its box replaces the current one and the mark is cleared)
 *     or repair_calls repairs have run (Algorithm 1's Run-Repair-Procedure).
 * lb/ub hold the final box on return (every such integer variable fixed).
 * The result is the same bit for bit as the plain sequential procedure.
 * Returns BP_OK (res set), or BP_EINVAL for a null argument, NaN in x or the
 * box, a draw outside [0, 1) or a cached id out of range (lb/ub untouched). */
int bp_round(bp_instance *h, double *lb, double *ub, const double *x, const double *draws,
             const bp_cache *cache, bp_round_result *res, void *stream);

/* Repair procedure (the paper's Section 2.3, repair passage; Algorithm 1's
 * Run-Repair-Procedure).  Given a box DEVICE lb/ub [n] whose fixed integer
 * variables (lb == ub) form a tentative assignment F, and the original box
 * DEVICE lb0/ub0 [n] containing it, search new values for F:
 *   - violation of row k at a box: with the activities of propagation,
 *     fl(minfin - hi) when no minimum term is infinite and minfin >
 *     fl(hi + feastol); fl(lo - maxfin) when no maximum term is infinite and
 *     maxfin < fl(lo - feastol); else 0;
 *   - a shift takes the most violated row (largest violation, then smallest
 *     index); each F variable j of it with value v and coefficient a gets
 *     r = fl(-e / a) (hi side) or fl(e / a) (lo side) and the move d of
 *     magnitude max(1, ceil(|r| - inttol)) with the sign of r, limited to
 *     lb0 - v <= d <= ub0 - v (an infinite original bound sets no limit);
 *     d = 0: no candidate.  Its score is the correctly rounded sum, over
 *     j's rows, of the change of the row's violation when j's terms
 *     fl(c*v) become fl(c*(v + d)) in fl(fl(act - fl(c*v)) + fl(c*(v+d)));
 *     the lowest score (then the smallest j) is applied when negative, else
 *     the repair fails (reason 1);
 *   - an attempt shifts until no row is violated (more than max_shifts
 *     shifts: failure, reason 2), then propagates (cold) the original box
 *     with F's current values.  A result that is not infeasible ends the
 *     repair: lb/ub become it.  An infeasible one detected in round d ends
 *     the repair after max_attempts such propagations (reason 3), else the
 *     next attempt starts from the state of the same propagation after
 *     d - 1 rounds.
 * The variables outside F never shift: their bounds are what propagation
 * from F implies.  A failed repair leaves lb/ub as given.  The result is
 * the same bit for bit as the plain sequential procedure.
 * Returns BP_OK (res set: status BP_OK if repaired, BP_INFEASIBLE if not;
 * reason 0 when repaired), or BP_EINVAL for a null argument, a NaN, lb0 >
 * ub0, a box outside the original box, max_shifts < 0 or max_attempts < 1
 * (lb/ub untouched). */
typedef struct {
    int32_t status;   /* BP_OK (repaired) or BP_INFEASIBLE */
    int32_t attempts; /* propagations from the original box */
    int32_t shifts;   /* shifts applied */
    int32_t reason;   /* 0 repaired, 1 no shift lowers the violation, 2 shift
                         limit, 3 attempt limit */
    int64_t nnz_propagated; /* over the repair's propagations */
} bp_repair_result;

int bp_repair(bp_instance *h, double *lb, double *ub, const double *lb0, const double *ub0,
              int32_t max_shifts, int32_t max_attempts, bp_repair_result *res, void *stream);

/* Schedule chosen by bp_autotune. */
typedef struct {
    int32_t heavy_threshold;   /* rows longer than this split across workgroups */
    int32_t heavy_chunk;       /* nonzeros per workgroup of a heavy row */
    int32_t rounds_per_launch; /* rounds per captured graph */
    int32_t probe_slots;       /* bound vectors in flight while probing */
    double ms;                 /* time of the chosen schedule on the workload */
    int32_t trials;            /* schedules timed (0: taken from the cache) */
    int32_t from_cache;
    int32_t lv_grid;           /* bp_autotune_batch: lane-engine workgroups per round
                                  kernel (0: not tuned) */
} bp_tuning;

/* Autotuner: time candidate schedules (heavy-row threshold and chunk size,
 * rounds per graph; and probe slots when vars != NULL) on the caller's own
 * workload -- a cold bp_propagate from DEVICE lb/ub [n] (left unchanged),
 * then, if k > 0, bp_probe of DEVICE vars [k] from the resulting base -- and
 * keep the fastest in the instance's options.  Every schedule computes the
 * same results; only time differs.  With cache_path != NULL the choice is
 * read from / appended to that text file, keyed by the device architecture
 * and a signature of the instance (sizes and row-length bins).  The base is
 * left at the cold propagation's result. */
int bp_autotune(bp_instance *h, const double *lb, const double *ub, const int32_t *vars,
                int32_t k, const char *cache_path, bp_tuning *out, void *stream);

/* Autotuner of batched propagation: time bp_propagate_batch of the caller's
 * own batch (B vectors DEVICE lb/ub [B*n] with changed_ptr/changed_idx as
 * bp_propagate_batch takes them; left unchanged: each trial starts from a
 * copy) over the schedules of the engine that runs it -- for 16 or more
 * vectors the lane engine's workgroups per round kernel (lv_grid) and the
 * rounds per captured graph -- and keep the fastest in the instance's
 * options.  Every schedule gives the same results (checked per vector on
 * every trial).  With cache_path != NULL the choice is read from / appended
 * to that text file, keyed by the device architecture, the instance
 * signature and the batch size.  Returns BP_OK, or an error of the batch
 * call. */
int bp_autotune_batch(bp_instance *h, int32_t B, const double *lb, const double *ub,
                      const int64_t *changed_ptr, const int32_t *changed_idx, const char *cache_path,
                      bp_tuning *out, void *stream);

/* Copy the base bounds into DEVICE lb/ub [n].  BP_ESTATE without a base. */
int bp_get_base(bp_instance *h, double *lb, double *ub, void *stream);

/* Counters and kernel timing since load or the last reset (see bp_stats). */
int bp_kernel_stats(bp_instance *h, bp_stats *out, int reset);

/* Device bytes held by the instance (matrix copies and work buffers). */
int64_t bp_device_bytes(const bp_instance *h);

void bp_free(bp_instance *h);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of propagate and probe requests over several
 * resident instances (the batching and serving pattern around the paper's
 * Section 2.1 propagation and Section 2.2 probing).  Every request becomes
 * jobs (one per propagate request, two per probed binary); jobs of all
 * requests and instances advance round-synchronously in the same launches,
 * each in a slot of a fixed pool whose size is set by a device-memory
 * budget.  A slot that finishes is refilled with the next queued job at the
 * next round boundary, so requests that arrive while others run join the
 * work already on the device.  Each job's result equals what bp_propagate
 * (from the instance's base with the request's bounds applied) or bp_probe
 * would return for it alone.
 * ------------------------------------------------------------------------- */
#define BP_REQ_PROBE 0      /* probe `count` integer variables as bp_probe does */
#define BP_REQ_PROPAGATE 1  /* intersect `count` variables' bounds with
                               [lb, ub] and propagate from the base */

typedef struct bp_server bp_server;

typedef struct {
    int32_t instance;      /* index into the instances given to bp_server_create */
    int32_t kind;          /* BP_REQ_PROBE or BP_REQ_PROPAGATE */
    int32_t count;         /* binaries (probe) or bound changes (propagate) */
    int32_t reserved;
    const int32_t *vars;   /* HOST [count]; distinct variables */
    const double *lb;      /* HOST [count] new bounds (propagate only) */
    const double *ub;
} bp_request;

typedef struct {
    int64_t id;            /* as returned by bp_server_submit */
    int32_t instance, kind;
    int32_t jobs;          /* 1 (propagate) or 2*count (probe) */
    int32_t flags;         /* BP_COMPLETION_CANCELLED or 0 */
    double submit_us;      /* host clock, microseconds since bp_server_create */
    double done_us;        /* when the server observed the last job finish */
} bp_completion;

#define BP_COMPLETION_CANCELLED 1  /* taken out of the queue before it ran */

/* Create a server over `count` loaded instances, each with a base (a
 * feasible bp_propagate was run on it; BP_ESTATE otherwise).  Instances are
 * grouped into at most four classes by their number of variables (a class
 * spans a factor of r = max(8, (n_max / n_min)^(1/3.5)) from its smallest
 * instance), and each class gets a pool of slots sized for its own largest
 * instance (variables, rows, row bins and heavy chunks), so a request holds
 * a slot of its class's footprint.  `budget_bytes` of device memory are
 * shared out from the pool with the smallest slots up, each taking at most
 * its fair share of what is left and at most opt->probe_slots slots (opt
 * NULL: the first instance's options).  If that leaves a pool fewer than
 * min(16, probe_slots) slots, all instances share one pool of slots sized
 * for the largest.  Pools run side by side on streams of their own (the
 * first on `stream`).  Each pool's request queue and result staging (about
 * 1.2 GB: 2^21 jobs, 2^24 fixings, 2^25 staged implications) are allocated
 * beside the budget.  The instances must outlive the server, or their
 * eviction (bp_server_evict). */
int bp_server_create(bp_instance *const *instances, int32_t count, const bp_options *opt,
                     int64_t budget_bytes, void *stream, bp_server **out);

/* Serve one more loaded instance (with a base; BP_ESTATE otherwise) under
 * the next free index (*index; an evicted instance's index is reused), in
 * the pool with the smallest slots that hold it.  BP_ECAPACITY if no pool's
 * slots, sized at creation, hold it (more variables, rows, row-bin tasks or
 * heavy chunks than a pool's largest instance then) or the table of 4096
 * instances is full; BP_EINVAL for a different heavy chunk size or an
 * instance already served. */
int bp_server_add_instance(bp_server *sv, bp_instance *instance, int32_t *index);

/* Stop serving instance `index`: later requests for it get BP_EINVAL, and
 * its owner may free it.  BP_ESTATE while it has requests that are neither
 * finished nor cancelled; BP_EINVAL for an index not served. */
int bp_server_evict(bp_server *sv, int32_t index);

/* Queue a request (arrays are copied).  BP_EINVAL for a bad instance index,
 * kind, variable, a repeated variable, or a probe variable that is not a
 * binary of the base. */
int bp_server_submit(bp_server *sv, const bp_request *req, int64_t *id);

/* Move queued requests to the device, run up to `rounds` rounds, and
 * collect the requests that finished.  *busy receives the number of
 * requests submitted and not yet finished. */
int bp_server_run(bp_server *sv, int32_t rounds, int32_t *busy);

/* Cancel a request that still waits in the host queue: requests submitted
 * while the device job list is full, or not yet moved to the device by a
 * bp_server_run.  It finishes at once: bp_server_poll reports it with
 * flags = BP_COMPLETION_CANCELLED, and bp_server_results returns
 * BP_ECANCELED.  BP_ESTATE if its jobs are already on the device or it has
 * finished (those run to the end); BP_EINVAL for an unknown id. */
int bp_server_cancel(bp_server *sv, int64_t id);

/* Queue timeout: cancel, as bp_server_cancel does, every request that has
 * waited in the host queue for more than max_wait_us microseconds since its
 * bp_server_submit.  *n (if not NULL) receives the number cancelled. */
int bp_server_expire(bp_server *sv, double max_wait_us, int32_t *n);

/* Finished requests since the last poll, in completion order (at most max;
 * *n receives the number written). */
int bp_server_poll(bp_server *sv, bp_completion *out, int32_t max, int32_t *n);

/* Results of a finished request, into HOST arrays of `jobs` entries (status,
 * rounds, nnz, n_bad_rows, bad_row, bad_var; any may be NULL) and its
 * implication lists: off [jobs+1], var/lb/ub [cap] (job j's list is
 * [off[j], off[j+1]), ascending by variable).  BP_ECAPACITY with *required
 * set if cap is too small; BP_ESTATE if the request has not finished. */
int bp_server_results(bp_server *sv, int64_t id, int8_t *status, int32_t *rounds, int64_t *nnz,
                      int32_t *n_bad_rows, int32_t *bad_row, int32_t *bad_var, int64_t *off,
                      int32_t *var, double *lb, double *ub, int64_t cap, int64_t *required);

/* Slots over all pools, and the device bytes of a slot sized for every
 * served instance (the slot of a one-pool server: a budget of k times it
 * gives such a server k slots). */
int bp_server_info(const bp_server *sv, int32_t *slots, int64_t *bytes_per_slot);

/* The server's pools: *npools receives their number (if not NULL); for
 * 0 <= pool < npools, its slots, device bytes per slot and the number of
 * instances it serves (outputs may be NULL).  BP_EINVAL for another pool
 * index when an output other than npools is asked for. */
int bp_server_pool_info(const bp_server *sv, int32_t pool, int32_t *npools, int32_t *slots,
                        int64_t *bytes_per_slot, int32_t *instances);

void bp_server_destroy(bp_server *sv);

/* Thread-local description of the last error ("" if none). */
const char *bp_last_error(void);

/* Failure injection, for tests of the error paths: from this call on, the
 * k-th device allocation the library makes (in any entry point, on any
 * thread) fails with BP_ENOMEM as if the device were out of memory, and the
 * injection then disarms itself; k = 0 disarms it.  A call that fails this
 * way returns BP_ENOMEM and leaks nothing: an instance or server under
 * construction is destroyed, and an existing instance may lose its work
 * buffers, which its next call allocates again.  Outputs are untouched as
 * for any error, except that bp_round, whose repairs allocate their buffers
 * on first use, may leave lb/ub at a later step's box.  BP_EINVAL for
 * k < 0. */
int bp_debug_fail_alloc(int64_t k);

#ifdef __cplusplus
}
#endif

#endif /* BP_H */
