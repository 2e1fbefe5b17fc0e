/*
 * bp_oracle.c -- plain, slow, single-threaded CPU oracle for bound
 * propagation and probing.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity reference for the GPU
 * library.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or helper with
 * the GPU path, and the GPU path never calls it.
 *
 * What it computes (the paper's Section 2.1 "Bound Propagation" and
 * Section 2.2 "Probing Cache"):
 *
 *   rows      lo_k <= sum_i a_ki x_i <= hi_k      (the paper's  a.z <= g  is
 *             the case lo = -inf; a finite lo is the mirrored row)
 *   activity  L_min^k = sum_{a>0} a l_i + sum_{a<0} a u_i   (Section 2.1,
 *             first display) and its mirror L_max^k
 *   bounds    u_i <- min_k (g_k - L_min^k + a_ki l_i) / a_ki  over a_ki > 0,
 *             l_i <- max_k (g_k - L_min^k + a_ki u_i) / a_ki  over a_ki < 0
 *             (Section 2.1, second display), and the mirrored forms for lo
 *   rounds    the two steps repeat while some update passes a threshold
 *             (Section 2.1, closing sentence of the bound formulas)
 *   probing   a binary fixed to 0 and to 1, each propagated from the same
 *             base (Section 2.2), the implications being the bounds that
 *             differ from the base
 *   rounding  bulk fix-and-propagate of the integer variables towards a
 *             fractional point (Algorithm 1 and Section 2.3, without the LP
 *             polish)
 *   repair    bound shifts that remove row violations one row at a time,
 *             then propagation of the fixed variables from the original
 *             bounds (Section 2.3, the repair passage; Algorithm 1's
 *             Run-Repair-Procedure)
 *   scores    the probe priority (Section 2.2: rows violated when a
 *             variable's contribution flips between its bounds, the largest
 *             violation, the smallest unit slack) and the implied-slack score
 *             S = sum of (a / slack)^2 (Section 2.3)
 *
 * Readings where the paper is silent (each one is also listed with the
 * design notes):
 *   - rounds are round-synchronous (Jacobi): every row of a round sees the
 *     bounds as they were when the round started;
 *   - activities are the correctly rounded exact sum of the rounded terms
 *     fl(a*b) over the finite contributions; infinite contributions are
 *     counted, and a candidate uses the residual activity only when at most
 *     the variable's own contribution is infinite;
 *   - candidate op order: v = fl(fl(side - act) + fl(a*b_own)), c = fl(v/a);
 *     integer variables round c up/down with tolerance inttol;
 *   - threshold: integer variables accept any strict improvement;
 *     continuous ones accept an old infinite bound, else an improvement
 *     larger than tau * max(1, |old bound|);
 *   - feasibility tolerance feastol (absolute) for the row test and for a
 *     crossing of continuous bounds (Section 3 uses 1e-6 absolute);
 *   - propagation after a call's first round only revisits rows holding a
 *     variable whose bounds changed in the previous round (Section 1,
 *     "propagation on changed constraints");
 *   - -0.0 is stored as +0.0.
 *
 * Two modes give the same results: DEFINITION recomputes every row and every
 * variable in every round; WORKLIST only the rows of the changed variables.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_INFEASIBLE 1
#define ORC_ROUND_LIMIT 2
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ECAPACITY (-4)

#define ORC_MODE_WORKLIST 0
#define ORC_MODE_DEFINITION 1

typedef struct {
    int64_t m, n, nnz;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
    const double *lo, *hi;
    const uint8_t *vtype; /* 0 continuous, 1 integer */
} orc_instance;

typedef struct {
    double feastol, inttol, tau;
    int32_t max_rounds;
} orc_options;

typedef struct {
    int32_t status, rounds;
    int64_t nnz_propagated;
    int32_t n_infeasible_rows;
    int64_t infeasible_row;
    int32_t infeasible_var;
} orc_result;

/* ------------------------------------------------------------------------ */
/* Correctly rounded sum of doubles.                                         */
/*                                                                           */
/* Shewchuk's adaptive-precision summation (Shewchuk 1997, "Adaptive        */
/* Precision Floating-Point Arithmetic and Fast Robust Geometric            */
/* Predicates"): the running sum is kept as a list of non-overlapping       */
/* partials of increasing magnitude whose exact sum equals the exact sum of */
/* the inputs so far.  Each input is merged with two-sum steps.  The final  */
/* value adds the partials from the largest down and fixes the one case     */
/* where that rounding could be off: a remainder of exactly half an ulp,    */
/* resolved by the sign of the next partial.  Inputs must be finite.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *p;
    int64_t len, cap;
    double stack[64];
} orc_partials;

static void partials_init(orc_partials *s) {
    s->p = s->stack;
    s->len = 0;
    s->cap = 64;
}

static void partials_free(orc_partials *s) {
    if (s->p != s->stack) free(s->p);
}

static int partials_push(orc_partials *s, double v) {
    if (s->len == s->cap) {
        int64_t nc = s->cap * 2;
        double *np_ = (double *)malloc((size_t)nc * sizeof(double));
        if (!np_) return -1;
        memcpy(np_, s->p, (size_t)s->len * sizeof(double));
        if (s->p != s->stack) free(s->p);
        s->p = np_;
        s->cap = nc;
    }
    s->p[s->len++] = v;
    return 0;
}

static int partials_add(orc_partials *s, double x) {
    int64_t keep = 0;
    for (int64_t j = 0; j < s->len; ++j) {
        double y = s->p[j];
        if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
        double hi = x + y;
        double lo = y - (hi - x); /* exact error of hi, since |x| >= |y| */
        if (lo != 0.0) s->p[keep++] = lo;
        x = hi;
    }
    s->len = keep;
    return partials_push(s, x);
}

static double partials_round(const orc_partials *s) {
    int64_t k = s->len;
    if (k == 0) return 0.0;
    double hi = s->p[--k];
    double lo = 0.0;
    while (k > 0) {
        double x = hi;
        double y = s->p[--k];
        hi = x + y;
        double yr = hi - x;
        lo = y - yr;
        if (lo != 0.0) break;
    }
    /* hi + lo is exact here and lo is at most half an ulp of hi.  If lo is
     * exactly half an ulp and the next lower partial has the same sign, the
     * true sum lies beyond the halfway point: round away from hi. */
    if (k > 0 && ((lo < 0.0 && s->p[k - 1] < 0.0) || (lo > 0.0 && s->p[k - 1] > 0.0))) {
        double y = lo * 2.0;
        double x = hi + y;
        double yr = x - hi;
        if (y == yr) hi = x;
    }
    return hi;
}

double orc_exact_sum(const double *x, int64_t n) {
    orc_partials s;
    partials_init(&s);
    for (int64_t i = 0; i < n; ++i) {
        if (partials_add(&s, x[i]) != 0) { partials_free(&s); return NAN; }
    }
    double r = partials_round(&s);
    partials_free(&s);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Propagation.                                                             */
/* ------------------------------------------------------------------------ */
static double canon(double x) { return x == 0.0 ? 0.0 : x; }

typedef struct {
    double minfin, maxfin;
    int64_t ninf_min, ninf_max;
} orc_activity;

/* Row activity (Section 2.1, first display, and its mirror).  Terms are the
 * rounded products a*l (a > 0) or a*u (a < 0) for the minimum; the maximum
 * swaps l and u.  Infinite contributions are counted, not summed. */
static int row_activity(const orc_instance *I, int64_t k, const double *lb, const double *ub,
                        double *buf_min, double *buf_max, orc_activity *act) {
    int64_t a0 = I->row_ptr[k], a1 = I->row_ptr[k + 1];
    int64_t nmin = 0, nmax = 0;
    act->ninf_min = 0;
    act->ninf_max = 0;
    for (int64_t p = a0; p < a1; ++p) {
        int32_t i = I->col[p];
        double a = I->val[p];
        double bmin = a > 0.0 ? lb[i] : ub[i];
        double bmax = a > 0.0 ? ub[i] : lb[i];
        if (isinf(bmin)) act->ninf_min += 1; else buf_min[nmin++] = a * bmin;
        if (isinf(bmax)) act->ninf_max += 1; else buf_max[nmax++] = a * bmax;
    }
    act->minfin = canon(orc_exact_sum(buf_min, nmin));
    act->maxfin = canon(orc_exact_sum(buf_max, nmax));
    if (isnan(act->minfin) || isnan(act->maxfin)) return ORC_ENOMEM;
    return 0;
}

static int row_infeasible(const orc_instance *I, int64_t k, const orc_activity *act,
                          const orc_options *o) {
    if (act->ninf_min == 0 && act->minfin > I->hi[k] + o->feastol) return 1;
    if (act->ninf_max == 0 && act->maxfin < I->lo[k] - o->feastol) return 1;
    return 0;
}

/* Candidates of one nonzero (Section 2.1, second display, with its mirror
 * for lo).  Writes an upper candidate into *cu / a lower one into *cl when
 * present (they start at +inf / -inf). */
static void nonzero_candidates(const orc_instance *I, int64_t k, double a, int32_t i,
                               const orc_activity *act, const double *lb, const double *ub,
                               const orc_options *o, double *cl, double *cu) {
    int is_int = I->vtype[i] != 0;
    double hi = I->hi[k], lo = I->lo[k];
    if (!isinf(hi)) {
        double bown = a > 0.0 ? lb[i] : ub[i];
        int own_inf = isinf(bown);
        int have = 0;
        double v = 0.0;
        if (!own_inf && act->ninf_min == 0) {
            double r = hi - act->minfin;
            double t = a * bown;
            v = r + t;
            have = 1;
        } else if (own_inf && act->ninf_min == 1) {
            v = hi - act->minfin;
            have = 1;
        }
        if (have) {
            double c = v / a;
            if (a > 0.0) { /* upper bound candidate */
                if (is_int) c = floor(c + o->inttol);
                if (c < *cu) *cu = c;
            } else {       /* lower bound candidate */
                if (is_int) c = ceil(c - o->inttol);
                if (c > *cl) *cl = c;
            }
        }
    }
    if (!isinf(lo)) {
        double bown = a > 0.0 ? ub[i] : lb[i];
        int own_inf = isinf(bown);
        int have = 0;
        double v = 0.0;
        if (!own_inf && act->ninf_max == 0) {
            double r = lo - act->maxfin;
            double t = a * bown;
            v = r + t;
            have = 1;
        } else if (own_inf && act->ninf_max == 1) {
            v = lo - act->maxfin;
            have = 1;
        }
        if (have) {
            double c = v / a;
            if (a > 0.0) { /* lower bound candidate */
                if (is_int) c = ceil(c - o->inttol);
                if (c > *cl) *cl = c;
            } else {       /* upper bound candidate */
                if (is_int) c = floor(c + o->inttol);
                if (c < *cu) *cu = c;
            }
        }
    }
}

/* Threshold test (the paper only says "a threshold"; reading above). */
static int accept_upper(int is_int, double cand, double old, const orc_options *o) {
    if (is_int) return cand < old;
    if (isinf(old)) return !isinf(cand) && cand < old;
    return cand < old - o->tau * fmax(1.0, fabs(old));
}

static int accept_lower(int is_int, double cand, double old, const orc_options *o) {
    if (is_int) return cand > old;
    if (isinf(old)) return !isinf(cand) && cand > old;
    return cand > old + o->tau * fmax(1.0, fabs(old));
}

typedef struct {
    int64_t *col_ptr; /* CSC built here, independently of the GPU path */
    int32_t *col_row;
    double *buf_min, *buf_max;
    double *cl, *cu;
    int32_t *touched;   /* vars with a candidate this round */
    uint8_t *tmark;
    int32_t *rows, *next_rows; /* worklists */
    uint8_t *rmark;
    int32_t *changed;   /* S_r */
    double *nlb, *nub;  /* staged new bounds (definition mode) */
} orc_work;

static void work_free(orc_work *w) {
    free(w->col_ptr); free(w->col_row); free(w->buf_min); free(w->buf_max);
    free(w->cl); free(w->cu); free(w->touched); free(w->tmark);
    free(w->rows); free(w->next_rows); free(w->rmark); free(w->changed);
    free(w->nlb); free(w->nub);
    memset(w, 0, sizeof(*w));
}

static int work_init(const orc_instance *I, orc_work *w) {
    memset(w, 0, sizeof(*w));
    int64_t m = I->m, n = I->n, nnz = I->nnz;
    int64_t maxlen = 0;
    for (int64_t k = 0; k < m; ++k) {
        int64_t L = I->row_ptr[k + 1] - I->row_ptr[k];
        if (L > maxlen) maxlen = L;
    }
    w->col_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    w->col_row = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    w->buf_min = (double *)malloc((size_t)(maxlen > 0 ? maxlen : 1) * sizeof(double));
    w->buf_max = (double *)malloc((size_t)(maxlen > 0 ? maxlen : 1) * sizeof(double));
    w->cl = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    w->cu = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    w->touched = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    w->tmark = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    w->rows = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    w->next_rows = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    w->rmark = (uint8_t *)calloc((size_t)(m > 0 ? m : 1), 1);
    w->changed = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    w->nlb = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    w->nub = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!w->col_ptr || !w->col_row || !w->buf_min || !w->buf_max || !w->cl || !w->cu ||
        !w->touched || !w->tmark || !w->rows || !w->next_rows || !w->rmark || !w->changed ||
        !w->nlb || !w->nub) {
        work_free(w);
        return ORC_ENOMEM;
    }
    for (int64_t p = 0; p < nnz; ++p) w->col_ptr[I->col[p] + 1] += 1;
    for (int64_t i = 0; i < n; ++i) w->col_ptr[i + 1] += w->col_ptr[i];
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!fill) { work_free(w); return ORC_ENOMEM; }
    memcpy(fill, w->col_ptr, (size_t)n * sizeof(int64_t));
    for (int64_t k = 0; k < m; ++k)
        for (int64_t p = I->row_ptr[k]; p < I->row_ptr[k + 1]; ++p)
            w->col_row[fill[I->col[p]]++] = (int32_t)k;
    free(fill);
    for (int64_t i = 0; i < n; ++i) { w->cl[i] = -INFINITY; w->cu[i] = INFINITY; }
    return 0;
}

/* Validation of the instance and of a bound vector (malformed input is an
 * error, not a propagation outcome). */
int orc_validate(const orc_instance *I) {
    if (I->m < 0 || I->n < 0 || I->nnz < 0) return ORC_EINVAL;
    if (I->m >= INT32_MAX || I->n >= INT32_MAX) return ORC_EINVAL;
    if (I->row_ptr[0] != 0 || I->row_ptr[I->m] != I->nnz) return ORC_EINVAL;
    for (int64_t k = 0; k < I->m; ++k) {
        if (I->row_ptr[k + 1] < I->row_ptr[k]) return ORC_EINVAL;
        if (isnan(I->lo[k]) || isnan(I->hi[k]) || I->lo[k] > I->hi[k]) return ORC_EINVAL;
        if (I->lo[k] == INFINITY || I->hi[k] == -INFINITY) return ORC_EINVAL;
        for (int64_t p = I->row_ptr[k]; p < I->row_ptr[k + 1]; ++p) {
            if (I->col[p] < 0 || I->col[p] >= I->n) return ORC_EINVAL;
            if (p > I->row_ptr[k] && I->col[p] <= I->col[p - 1]) return ORC_EINVAL;
            if (!(I->val[p] != 0.0) || isinf(I->val[p])) return ORC_EINVAL; /* also NaN */
        }
    }
    for (int64_t i = 0; i < I->n; ++i)
        if (I->vtype[i] > 1) return ORC_EINVAL;
    return 0;
}

static void add_row(const orc_instance *I, orc_work *w, int64_t k, int64_t *cnt) {
    (void)I;
    if (!w->rmark[k]) { w->rmark[k] = 1; w->next_rows[(*cnt)++] = (int32_t)k; }
}

/* PROPAGATE.  lb/ub (length n) are read and written in place.  changed ==
 * NULL with n_changed < 0 is a cold start (every row in the first round);
 * otherwise the first round holds the rows of the listed variables. */
int orc_propagate(const orc_instance *I, double *lb, double *ub, const int32_t *changed,
                  int64_t n_changed, const orc_options *o, int mode, orc_result *res) {
    res->status = ORC_OK;
    res->rounds = 0;
    res->nnz_propagated = 0;
    res->n_infeasible_rows = 0;
    res->infeasible_row = -1;
    res->infeasible_var = -1;
    const int64_t m = I->m, n = I->n;
    /* Step 0: an empty box before any round. */
    for (int64_t i = 0; i < n; ++i) {
        if (isnan(lb[i]) || isnan(ub[i])) return ORC_EINVAL;
        double slack = I->vtype[i] ? 0.0 : o->feastol;
        if (lb[i] > ub[i] + slack) {
            res->status = ORC_INFEASIBLE;
            res->infeasible_var = (int32_t)i;
            return ORC_INFEASIBLE;
        }
    }
    if (changed != NULL && n_changed == 0) return ORC_OK;
    orc_work w;
    int rc = work_init(I, &w);
    if (rc) return rc;
    for (int64_t i = 0; i < n; ++i) { lb[i] = canon(lb[i]); ub[i] = canon(ub[i]); }

    /* First worklist. */
    int64_t nrows = 0;
    if (changed == NULL) {
        for (int64_t k = 0; k < m; ++k) w.next_rows[nrows++] = (int32_t)k;
    } else {
        for (int64_t t = 0; t < n_changed; ++t) {
            int32_t i = changed[t];
            if (i < 0 || i >= n) { work_free(&w); return ORC_EINVAL; }
            for (int64_t p = w.col_ptr[i]; p < w.col_ptr[i + 1]; ++p) add_row(I, &w, w.col_row[p], &nrows);
        }
    }

    orc_activity *acts = NULL;
    if (mode == ORC_MODE_DEFINITION) {
        acts = (orc_activity *)malloc((size_t)(m > 0 ? m : 1) * sizeof(orc_activity));
        if (!acts) { work_free(&w); return ORC_ENOMEM; }
    }

    int status = ORC_OK;
    for (;;) {
        /* Step 1: the round's worklist R_r. */
        if (nrows == 0) break;
        if (res->rounds >= o->max_rounds) { status = ORC_ROUND_LIMIT; break; }
        { int32_t *t = w.rows; w.rows = w.next_rows; w.next_rows = t; }
        int64_t cur = nrows;
        for (int64_t t = 0; t < cur; ++t) w.rmark[w.rows[t]] = 0;
        res->rounds += 1;
        for (int64_t t = 0; t < cur; ++t) {
            int64_t k = w.rows[t];
            res->nnz_propagated += I->row_ptr[k + 1] - I->row_ptr[k];
        }

        int64_t ntouched = 0;
        int64_t bad_row = -1, n_bad = 0;
        if (mode == ORC_MODE_WORKLIST) {
            /* Steps 2-4 over R_r only. */
            for (int64_t t = 0; t < cur; ++t) {
                int64_t k = w.rows[t];
                orc_activity act;
                if ((rc = row_activity(I, k, lb, ub, w.buf_min, w.buf_max, &act))) goto fail;
                if (row_infeasible(I, k, &act, o)) {
                    n_bad += 1;
                    if (bad_row < 0 || k < bad_row) bad_row = k;
                    continue;
                }
                if (n_bad) continue; /* the round ends infeasible; skip candidates */
                for (int64_t p = I->row_ptr[k]; p < I->row_ptr[k + 1]; ++p) {
                    int32_t i = I->col[p];
                    nonzero_candidates(I, k, I->val[p], i, &act, lb, ub, o, &w.cl[i], &w.cu[i]);
                    if (!w.tmark[i]) { w.tmark[i] = 1; w.touched[ntouched++] = i; }
                }
            }
        } else {
            /* Definition: every row's activity, every row's candidates. */
            for (int64_t k = 0; k < m; ++k) {
                if ((rc = row_activity(I, k, lb, ub, w.buf_min, w.buf_max, &acts[k]))) goto fail;
                if (row_infeasible(I, k, &acts[k], o)) {
                    n_bad += 1;
                    if (bad_row < 0 || k < bad_row) bad_row = k;
                }
            }
            if (!n_bad) {
                for (int64_t k = 0; k < m; ++k)
                    for (int64_t p = I->row_ptr[k]; p < I->row_ptr[k + 1]; ++p)
                        nonzero_candidates(I, k, I->val[p], I->col[p], &acts[k], lb, ub, o,
                                           &w.cl[I->col[p]], &w.cu[I->col[p]]);
                for (int64_t i = 0; i < n; ++i) w.touched[ntouched++] = (int32_t)i;
            }
        }
        if (n_bad) {
            /* Step 3: the round ends with the row evidence. */
            res->status = ORC_INFEASIBLE;
            res->infeasible_row = bad_row;
            res->n_infeasible_rows = (int32_t)n_bad;
            status = ORC_INFEASIBLE;
            for (int64_t t = 0; t < ntouched; ++t) {
                int32_t i = w.touched[t];
                w.cl[i] = -INFINITY; w.cu[i] = INFINITY; w.tmark[i] = 0;
            }
            break;
        }

        /* Step 5: acceptance against the round-start bounds (staged). */
        int64_t nchg = 0;
        int32_t bad_var = -1;
        for (int64_t t = 0; t < ntouched; ++t) {
            int32_t i = w.touched[t];
            int is_int = I->vtype[i] != 0;
            double L = w.cl[i], U = w.cu[i];
            double nl = lb[i], nu = ub[i];
            int ch = 0;
            if (accept_upper(is_int, U, ub[i], o)) { nu = canon(U); ch = 1; }
            if (accept_lower(is_int, L, lb[i], o)) { nl = canon(L); ch = 1; }
            /* Step 6: crossing. */
            if (ch && nl > nu) {
                if (is_int || nl - nu > o->feastol) {
                    if (bad_var < 0 || i < bad_var) bad_var = i;
                } else {
                    nl = nu;
                }
            }
            w.nlb[i] = nl;
            w.nub[i] = nu;
            if (ch) w.changed[nchg++] = i;
            w.cl[i] = -INFINITY; w.cu[i] = INFINITY; w.tmark[i] = 0;
        }
        /* Step 7: commit all at once. */
        for (int64_t t = 0; t < nchg; ++t) {
            int32_t i = w.changed[t];
            lb[i] = w.nlb[i];
            ub[i] = w.nub[i];
        }
        if (bad_var >= 0) {
            res->status = ORC_INFEASIBLE;
            res->infeasible_var = bad_var;
            status = ORC_INFEASIBLE;
            break;
        }
        /* Next worklist: rows holding a changed variable. */
        nrows = 0;
        for (int64_t t = 0; t < nchg; ++t) {
            int32_t i = w.changed[t];
            for (int64_t p = w.col_ptr[i]; p < w.col_ptr[i + 1]; ++p) add_row(I, &w, w.col_row[p], &nrows);
        }
    }
    res->status = status;
    free(acts);
    work_free(&w);
    return status;
fail:
    free(acts);
    work_free(&w);
    return rc;
}

/* The box of probe h (0 or 1) of integer variable j with base bounds
 * [l, u] (Section 2.2, probing cache):
 *   - base inside [0, 1] (a binary): x = h;
 *   - both bounds finite: x < (l + u) / 2, i.e. [l, ceil((l + u) / 2) - 1],
 *     and x >= (l + u) / 2, i.e. [ceil((l + u) / 2), u];
 *   - only l finite: x = l, and x >= l + 1;
 *   - only u finite (the mirror case): x <= u - 1, and x = u.
 * Returns 0, or -1 for a variable with no finite bound. */
int orc_probe_box(double l, double u, int h, double *nl, double *nu) {
    const double INF = HUGE_VAL;
    if (l >= 0.0 && u <= 1.0) {
        *nl = (double)h;
        *nu = (double)h;
    } else if (l > -INF && u < INF) {
        double c = ceil((l + u) / 2.0);
        if (h == 0) { *nl = l; *nu = c - 1.0; }
        else { *nl = c; *nu = u; }
    } else if (l > -INF) {
        if (h == 0) { *nl = l; *nu = l; }
        else { *nl = l + 1.0; *nu = u; }
    } else if (u < INF) {
        if (h == 0) { *nl = l; *nu = u - 1.0; }
        else { *nl = u; *nu = u; }
    } else {
        return -1;
    }
    return 0;
}

/* PROBE (Section 2.2): for each listed integer variable j and h in {0, 1},
 * propagate from the base (lb, ub) with j restricted to the box of probe h
 * (orc_probe_box) intersected with its base bounds.  Probe p = 2t + h.  An
 * empty box is infeasible before any round; a box equal to the base bounds
 * changes nothing.  Implied list of a feasible (or round-limited) probe:
 * every variable whose bounds differ from the base, ascending.  Infeasible
 * probes list nothing.  Returns ORC_ECAPACITY (with *required set) if cap
 * is too small. */
int orc_probe(const orc_instance *I, const double *base_lb, const double *base_ub,
              const int32_t *vars, int32_t k, const orc_options *o, int mode,
              int8_t *status, int32_t *rounds, int64_t *nnz, int32_t *n_infeasible_rows,
              int64_t *off, int32_t *ivar, double *ilb, double *iub, int64_t cap,
              int64_t *required) {
    const int64_t n = I->n;
    double *lb = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *ub = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!lb || !ub) { free(lb); free(ub); return ORC_ENOMEM; }
    int64_t total = 0;
    off[0] = 0;
    int rc_all = 0;
    for (int32_t t = 0; t < k; ++t) {
        int32_t j = vars[t];
        double box[2][2];
        if (j < 0 || j >= n || I->vtype[j] == 0 ||
            orc_probe_box(base_lb[j], base_ub[j], 0, &box[0][0], &box[0][1]) != 0) {
            free(lb); free(ub);
            return ORC_EINVAL;
        }
        orc_probe_box(base_lb[j], base_ub[j], 1, &box[1][0], &box[1][1]);
        for (int h = 0; h < 2; ++h) {
            int64_t p = 2 * (int64_t)t + h;
            /* the box intersected with the base bounds */
            double nl = box[h][0] > base_lb[j] ? box[h][0] : base_lb[j];
            double nu = box[h][1] < base_ub[j] ? box[h][1] : base_ub[j];
            int same = nl == base_lb[j] && nu == base_ub[j];
            orc_result r;
            memset(&r, 0, sizeof(r));
            r.infeasible_row = -1;
            r.infeasible_var = -1;
            if (nl > nu) {
                r.status = ORC_INFEASIBLE;
                r.infeasible_var = j;
            } else if (same) {
                r.status = ORC_OK;
            } else {
                memcpy(lb, base_lb, (size_t)n * sizeof(double));
                memcpy(ub, base_ub, (size_t)n * sizeof(double));
                lb[j] = nl;
                ub[j] = nu;
                int rc = orc_propagate(I, lb, ub, &j, 1, o, mode, &r);
                if (rc < 0) { free(lb); free(ub); return rc; }
            }
            status[p] = (int8_t)r.status;
            rounds[p] = r.rounds;
            nnz[p] = r.nnz_propagated;
            if (n_infeasible_rows) n_infeasible_rows[p] = r.n_infeasible_rows;
            int64_t cnt = 0;
            if (r.status != ORC_INFEASIBLE && !same) {
                for (int64_t i = 0; i < n; ++i) {
                    if (lb[i] != base_lb[i] || ub[i] != base_ub[i]) {
                        if (total + cnt < cap) {
                            ivar[total + cnt] = (int32_t)i;
                            ilb[total + cnt] = lb[i];
                            iub[total + cnt] = ub[i];
                        }
                        cnt += 1;
                    }
                }
            }
            total += cnt;
            off[p + 1] = total;
        }
    }
    free(lb);
    free(ub);
    if (required) *required = total;
    if (total > cap) rc_all = ORC_ECAPACITY;
    return rc_all;
}

/* ------------------------------------------------------------------------ */
/* Probe priority and implied-slack scores.                                 */
/* ------------------------------------------------------------------------ */
/* SCORES at the bounds (lb, ub), for every variable j (Section 2.2, the
 * three prioritisation criteria of the probing cache; Section 2.3, the unit
 * slack consumption s = a / slack and S_j = sum of s^2).  Row activities are
 * those of the propagation (correctly rounded sums of the finite terms and
 * counts of the infinite ones).  For each nonzero (k, j, a):
 *
 *   flipped contribution (criteria 1 and 2), only when j's column holds
 *   coefficients of both signs and both bounds of j are finite:
 *     d = fl(fl(a*b_max) - fl(a*b_min)), b_min/b_max the bound giving j's
 *         minimum/maximum contribution (lb/ub for a > 0, ub/lb for a < 0):
 *         by how much moving j from one to the other raises the row's
 *         minimum activity and lowers its maximum activity;
 *     hi side (hi_k finite, no infinite minimum term): e = fl(d - fl(hi_k -
 *         minfin_k)); lo side (lo_k finite, no infinite maximum term):
 *         e = fl(d - fl(maxfin_k - lo_k));
 *     the row is violated when some side has e > feastol; its violation is
 *     the largest such e.  nviol_j counts the violated rows of j and
 *     maxviol_j is their largest violation (0 when there is none);
 *
 *   unit slack (criterion 3 and the implied-slack sort), for each finite
 *   side of row k without infinite terms on that side:
 *     slack = fl(hi_k - minfin_k) or fl(maxfin_k - lo_k);
 *     s = fl(a / slack), term fl(s*s); S_j is the correctly rounded sum of
 *     the terms of j (+inf when some term is infinite, i.e. a zero slack;
 *     0 without terms); minunit_j is the smallest fl(slack / |a|) (+inf
 *     without terms).
 *
 * Any output pointer may be NULL. */
int orc_scores(const orc_instance *I, const double *lb, const double *ub, const orc_options *o,
               int32_t *nviol, double *maxviol, double *minunit, double *slack_score) {
    const int64_t m = I->m, n = I->n, nnz = I->nnz;
    const double INF = HUGE_VAL;
    int rc = 0;
    double *bmin = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    double *bmax = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    orc_activity *act = (orc_activity *)malloc((size_t)(m > 0 ? m : 1) * sizeof(orc_activity));
    int64_t *tcount = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int8_t *sign = (int8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *nv = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    double *mv = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *mu = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int8_t *sinf = (int8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    double *terms = NULL;
    int64_t *tfill = NULL;
    if (!bmin || !bmax || !act || !tcount || !sign || !nv || !mv || !mu || !sinf) {
        rc = ORC_ENOMEM;
        goto done;
    }
    for (int64_t k = 0; k < m; ++k)
        if ((rc = row_activity(I, k, lb, ub, bmin, bmax, &act[k])) != 0) goto done;
    /* which variables have coefficients of both signs */
    for (int64_t p = 0; p < nnz; ++p) sign[I->col[p]] |= I->val[p] > 0.0 ? 1 : 2;
    for (int64_t j = 0; j < n; ++j) mu[j] = INF;
    /* count the unit-slack terms of each variable, then collect them */
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t k = 0; k < m; ++k) {
            const orc_activity *A = &act[k];
            const int hi_ok = I->hi[k] < INF && A->ninf_min == 0;
            const int lo_ok = I->lo[k] > -INF && A->ninf_max == 0;
            const double slack_hi = hi_ok ? I->hi[k] - A->minfin : 0.0;
            const double slack_lo = lo_ok ? A->maxfin - I->lo[k] : 0.0;
            for (int64_t p = I->row_ptr[k]; p < I->row_ptr[k + 1]; ++p) {
                const int32_t j = I->col[p];
                const double a = I->val[p];
                if (pass == 0) {
                    tcount[j + 1] += hi_ok + lo_ok;
                    /* flipped contribution */
                    if (sign[j] == 3 && !isinf(lb[j]) && !isinf(ub[j])) {
                        const double b_min = a > 0.0 ? lb[j] : ub[j];
                        const double b_max = a > 0.0 ? ub[j] : lb[j];
                        const double d = a * b_max - a * b_min;
                        int viol = 0;
                        double worst = 0.0;
                        if (hi_ok) {
                            double e = d - slack_hi;
                            if (e > o->feastol) { viol = 1; worst = e; }
                        }
                        if (lo_ok) {
                            double e = d - slack_lo;
                            if (e > o->feastol && (!viol || e > worst)) { viol = 1; worst = e; }
                        }
                        if (viol) {
                            nv[j] += 1;
                            if (worst > mv[j]) mv[j] = worst;
                        }
                    }
                    /* smallest unit slack */
                    if (hi_ok) {
                        double u = slack_hi / fabs(a);
                        if (u < mu[j]) mu[j] = u;
                    }
                    if (lo_ok) {
                        double u = slack_lo / fabs(a);
                        if (u < mu[j]) mu[j] = u;
                    }
                } else {
                    for (int side = 0; side < 2; ++side) {
                        if (side == 0 ? !hi_ok : !lo_ok) continue;
                        double s = a / (side == 0 ? slack_hi : slack_lo);
                        double t = s * s;
                        if (isinf(t)) sinf[j] = 1;
                        else terms[tfill[j]++] = t;
                    }
                }
            }
        }
        if (pass == 0) {
            for (int64_t j = 0; j < n; ++j) tcount[j + 1] += tcount[j];
            terms = (double *)malloc((size_t)(tcount[n] > 0 ? tcount[n] : 1) * sizeof(double));
            tfill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
            if (!terms || !tfill) { rc = ORC_ENOMEM; goto done; }
            for (int64_t j = 0; j < n; ++j) tfill[j] = tcount[j];
        }
    }
    for (int64_t j = 0; j < n; ++j) {
        if (nviol) nviol[j] = nv[j];
        if (maxviol) maxviol[j] = canon(mv[j]);
        if (minunit) minunit[j] = canon(mu[j]);
        if (slack_score) {
            if (sinf[j]) slack_score[j] = INF;
            else slack_score[j] = canon(orc_exact_sum(terms + tcount[j], tfill[j] - tcount[j]));
        }
    }
done:
    free(bmin); free(bmax); free(act); free(tcount); free(sign); free(nv); free(mv); free(mu);
    free(sinf); free(terms); free(tfill);
    return rc;
}

/* Probe order (Section 2.2): the listed variables sorted by more violated
 * rows first, then the larger maximum violation, then the smaller minimum
 * unit slack, then the smaller index. */
typedef struct {
    int32_t var, nviol;
    double maxviol, minunit;
} orc_prio;

static int prio_cmp(const void *x, const void *y) {
    const orc_prio *a = (const orc_prio *)x, *b = (const orc_prio *)y;
    if (a->nviol != b->nviol) return a->nviol > b->nviol ? -1 : 1;
    if (a->maxviol != b->maxviol) return a->maxviol > b->maxviol ? -1 : 1;
    if (a->minunit != b->minunit) return a->minunit < b->minunit ? -1 : 1;
    if (a->var != b->var) return a->var < b->var ? -1 : 1;
    return 0;
}

int orc_probe_order(const orc_instance *I, const double *lb, const double *ub,
                    const orc_options *o, const int32_t *vars, int32_t k, int32_t *order) {
    const int64_t n = I->n;
    for (int32_t t = 0; t < k; ++t)
        if (vars[t] < 0 || vars[t] >= n) return ORC_EINVAL;
    int32_t *nv = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    double *mv = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *mu = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    orc_prio *P = (orc_prio *)malloc((size_t)(k > 0 ? k : 1) * sizeof(orc_prio));
    int rc = ORC_ENOMEM;
    if (nv && mv && mu && P) rc = orc_scores(I, lb, ub, o, nv, mv, mu, NULL);
    if (rc == 0) {
        for (int32_t t = 0; t < k; ++t) {
            int32_t j = vars[t];
            P[t].var = j;
            P[t].nviol = nv[j];
            P[t].maxviol = mv[j];
            P[t].minunit = mu[j];
        }
        qsort(P, (size_t)k, sizeof(orc_prio), prio_cmp);
        for (int32_t t = 0; t < k; ++t) order[t] = P[t].var;
    }
    free(nv); free(mv); free(mu); free(P);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Repair procedure.                                                        */
/* ------------------------------------------------------------------------ */
/* REPAIR (Section 2.3, the repair passage; Algorithm 1 calls it as
 * Run-Repair-Procedure).  The paper gives the outline: remove the violation
 * of a row by shifting the bounds of one of its variables, a variable at a
 * time, with a shift computed for every variable of the row that would make
 * the row feasible; then propagate the fixed variables from the original
 * bounds; repeat until that propagation is feasible or a limit is reached.
 * Readings (the paper leaves them open):
 *
 *   fixed     F = the integer variables with lb == ub in the given box: the
 *             repair searches values for them ("given fixed variables"); the
 *             other variables' bounds are what propagation from F implies,
 *             so they are not shifted, and only F's values carry into the
 *             propagation from the original box (lb0, ub0), which must
 *             contain the given box;
 *   violation of row k at a box: with the propagation's activities, the
 *             hi side is violated when no minimum term is infinite and
 *             minfin > fl(hi + feastol), by e = fl(minfin - hi); the lo side
 *             when no maximum term is infinite and maxfin < fl(lo - feastol),
 *             by e = fl(lo - maxfin) (at most one side can be); else e = 0;
 *   row       the most violated row (largest e, then smallest index);
 *   shift     of a variable j of F with value v and coefficient a in that
 *             row: v moves by d (both bounds of j).  The hi side needs
 *             a*d <= -e: r = fl(-e / a); the lo side needs a*d >= e:
 *             r = fl(e / a); |d| = max(1, ceil(|r| - inttol)) with the sign
 *             of r, so that the row's violation goes (up to inttol) in one
 *             shift.  The value stays inside the original box: d >=
 *             lb0 - v when shifting down, d <= ub0 - v when shifting up (an
 *             infinite original bound sets no limit); j is no candidate
 *             when d = 0;
 *   score     of candidate j: the change of the total violation, the
 *             correctly rounded sum over j's rows r of fl(e_r' - e_r), where
 *             e_r' is r's violation with j's terms replaced: minfin' =
 *             fl(fl(minfin - fl(c*v)) + fl(c*v')) for the coefficient c of
 *             j in r and v' = v + d, and the same for maxfin;
 *   choice    the candidate with the lowest score, then the smallest index,
 *             applied when its score is negative; its rows' activities are
 *             then recomputed exactly.  No candidate with a negative score:
 *             the repair fails;
 *   attempt   shifts until no row is violated (at most max_shifts in one
 *             attempt, else the repair fails); then F's current values are
 *             fixed in a copy of the original box and propagated cold.  A
 *             propagation that is not infeasible ends the repair: the box
 *             becomes its result.  One infeasible in round d ends the repair
 *             after max_attempts (>= 1) such propagations; otherwise the next
 *             attempt starts from the state of the same propagation after
 *             d - 1 rounds, where the row conflicts that stopped it show as
 *             violations.
 *
 * lb/ub are replaced by the repaired box, or left as given when the repair
 * fails.  res: status ORC_OK (repaired) or ORC_INFEASIBLE (failed), the
 * attempts (propagations from the original box), the shifts applied, the
 * reason a failed repair stopped (1: no candidate lowers the violation,
 * 2: shift limit, 3: attempt limit) and the nonzeros propagated. */
typedef struct {
    int32_t status, attempts, shifts, reason;
    int64_t nnz_propagated;
} orc_repair_result;

static double row_violation(const orc_instance *I, int64_t k, double minfin, double maxfin,
                            int64_t ninf_min, int64_t ninf_max, const orc_options *o) {
    if (ninf_min == 0 && !isinf(I->hi[k]) && minfin > I->hi[k] + o->feastol)
        return minfin - I->hi[k];
    if (ninf_max == 0 && !isinf(I->lo[k]) && maxfin < I->lo[k] - o->feastol)
        return I->lo[k] - maxfin;
    return 0.0;
}

/* The shifted value of a fixed integer variable (value v, coefficient a)
 * for a violation e of the hi side (hi_side = 1) or the lo side, inside
 * [l0, u0]; returns 0 when it cannot move. */
static int repair_shift(double a, double e, int hi_side, double v, double l0, double u0,
                        const orc_options *o, double *nv) {
    double r = hi_side ? (-e) / a : e / a;
    double mag = ceil(fabs(r) - o->inttol);
    if (mag < 1.0) mag = 1.0;
    double d = r < 0.0 ? -mag : mag;
    if (d < 0.0 && !isinf(l0) && d < l0 - v) d = l0 - v;
    if (d > 0.0 && !isinf(u0) && d > u0 - v) d = u0 - v;
    if (d == 0.0) return 0;
    *nv = canon(v + d);
    return 1;
}

int orc_repair(const orc_instance *I, double *lb, double *ub, const double *lb0, const double *ub0,
               int32_t max_shifts, int32_t max_attempts, const orc_options *o,
               orc_repair_result *res) {
    const int64_t m = I->m, n = I->n, nnz = I->nnz;
    memset(res, 0, sizeof(*res));
    res->status = ORC_INFEASIBLE;
    for (int64_t j = 0; j < n; ++j) {
        if (isnan(lb[j]) || isnan(ub[j]) || isnan(lb0[j]) || isnan(ub0[j])) return ORC_EINVAL;
        if (lb[j] < lb0[j] || ub[j] > ub0[j] || lb0[j] > ub0[j]) return ORC_EINVAL;
    }
    if (max_shifts < 0 || max_attempts < 1) return ORC_EINVAL;
    int rc = 0;
    const size_t N1 = (size_t)(n > 0 ? n : 1), M1 = (size_t)(m > 0 ? m : 1);
    const size_t Z1 = (size_t)(nnz > 0 ? nnz : 1);
    double *cl = (double *)malloc(N1 * sizeof(double));
    double *cu = (double *)malloc(N1 * sizeof(double));
    double *pl = (double *)malloc(N1 * sizeof(double));
    double *pu = (double *)malloc(N1 * sizeof(double));
    int8_t *fixed = (int8_t *)malloc(N1);
    orc_activity *act = (orc_activity *)malloc(M1 * sizeof(orc_activity));
    double *bmin = (double *)malloc(Z1 * sizeof(double));
    double *bmax = (double *)malloc(Z1 * sizeof(double));
    double *diffs = (double *)malloc(M1 * sizeof(double));
    int64_t *cptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *crow = (int32_t *)malloc(Z1 * sizeof(int32_t));
    double *cval = (double *)malloc(Z1 * sizeof(double));
    int64_t *cfill = (int64_t *)malloc(N1 * sizeof(int64_t));
    if (!cl || !cu || !pl || !pu || !fixed || !act || !bmin || !bmax || !diffs || !cptr || !crow ||
        !cval || !cfill) {
        rc = ORC_ENOMEM;
        goto done;
    }
    /* columns (row indices ascending) */
    for (int64_t p = 0; p < nnz; ++p) cptr[I->col[p] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) cptr[j + 1] += cptr[j];
    for (int64_t j = 0; j < n; ++j) cfill[j] = cptr[j];
    for (int64_t k = 0; k < m; ++k)
        for (int64_t p = I->row_ptr[k]; p < I->row_ptr[k + 1]; ++p) {
            int64_t e = cfill[I->col[p]]++;
            crow[e] = (int32_t)k;
            cval[e] = I->val[p];
        }
    memcpy(cl, lb, (size_t)n * sizeof(double));
    memcpy(cu, ub, (size_t)n * sizeof(double));
    for (int64_t j = 0; j < n; ++j) fixed[j] = I->vtype[j] && lb[j] == ub[j];
    for (;;) {
        /* shifts */
        for (int64_t k = 0; k < m; ++k)
            if ((rc = row_activity(I, k, cl, cu, bmin, bmax, &act[k])) != 0) goto done;
        int32_t shifts = 0;
        for (;;) {
            int64_t kb = -1;
            double eb = 0.0;
            for (int64_t k = 0; k < m; ++k) {
                double e = row_violation(I, k, act[k].minfin, act[k].maxfin, act[k].ninf_min,
                                         act[k].ninf_max, o);
                if (e > eb) { eb = e; kb = k; }
            }
            if (kb < 0) break;
            if (shifts >= max_shifts) { res->reason = 2; goto done; }
            const int hi_side = act[kb].ninf_min == 0 && !isinf(I->hi[kb]) &&
                                act[kb].minfin > I->hi[kb] + o->feastol;
            int32_t jb = -1;
            double sb = 0.0, vbest = 0.0;
            for (int64_t p = I->row_ptr[kb]; p < I->row_ptr[kb + 1]; ++p) {
                const int32_t j = I->col[p];
                double nv;
                if (!fixed[j] || !repair_shift(I->val[p], eb, hi_side, cl[j], lb0[j], ub0[j], o, &nv))
                    continue;
                int64_t nd = 0;
                for (int64_t q = cptr[j]; q < cptr[j + 1]; ++q) {
                    const int64_t r = crow[q];
                    const double c = cval[q];
                    const orc_activity *A = &act[r];
                    const double mn = canon((A->minfin - c * cl[j]) + c * nv);
                    const double mx = canon((A->maxfin - c * cl[j]) + c * nv);
                    double e0 = row_violation(I, r, A->minfin, A->maxfin, A->ninf_min, A->ninf_max, o);
                    double e1 = row_violation(I, r, mn, mx, A->ninf_min, A->ninf_max, o);
                    diffs[nd++] = e1 - e0;
                }
                double score = canon(orc_exact_sum(diffs, nd));
                if (jb < 0 || score < sb) { jb = j; sb = score; vbest = nv; }
            }
            if (jb < 0 || !(sb < 0.0)) { res->reason = 1; goto done; }
            cl[jb] = vbest;
            cu[jb] = vbest;
            shifts += 1;
            res->shifts += 1;
            for (int64_t q = cptr[jb]; q < cptr[jb + 1]; ++q)
                if ((rc = row_activity(I, crow[q], cl, cu, bmin, bmax, &act[crow[q]])) != 0) goto done;
        }
        /* propagation of the fixed variables from the original box */
        memcpy(pl, lb0, (size_t)n * sizeof(double));
        memcpy(pu, ub0, (size_t)n * sizeof(double));
        for (int64_t j = 0; j < n; ++j)
            if (fixed[j]) { pl[j] = cl[j]; pu[j] = cl[j]; }
        memcpy(cl, pl, (size_t)n * sizeof(double));
        memcpy(cu, pu, (size_t)n * sizeof(double));
        orc_result pr;
        int prc = orc_propagate(I, pl, pu, NULL, -1, o, ORC_MODE_WORKLIST, &pr);
        if (prc < 0) { rc = prc; goto done; }
        res->attempts += 1;
        res->nnz_propagated += pr.nnz_propagated;
        if (pr.status != ORC_INFEASIBLE) {
            memcpy(lb, pl, (size_t)n * sizeof(double));
            memcpy(ub, pu, (size_t)n * sizeof(double));
            res->status = ORC_OK;
            res->reason = 0;
            goto done;
        }
        if (res->attempts >= max_attempts) { res->reason = 3; goto done; }
        if (pr.rounds > 1) {
            /* the same propagation stopped before its detecting round */
            orc_options o2 = *o;
            o2.max_rounds = pr.rounds - 1;
            orc_result pr2;
            prc = orc_propagate(I, cl, cu, NULL, -1, &o2, ORC_MODE_WORKLIST, &pr2);
            if (prc < 0) { rc = prc; goto done; }
            res->nnz_propagated += pr2.nnz_propagated;
        }
    }
done:
    free(cl); free(cu); free(pl); free(pu); free(fixed); free(act); free(bmin); free(bmax);
    free(diffs); free(cptr); free(crow); free(cval); free(cfill);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Bound-propagation rounding (bulk fix-and-propagate).                     */
/* ------------------------------------------------------------------------ */
/* ROUND (the paper's Algorithm 1 and Section 2.3, without the repair
 * procedure and the LP polish): fix every integer variable of the box
 * (lb, ub) to a value drawn from the fractional point x, a bulk of
 * variables at a time, propagating after each bulk.
 *
 *   unset     the integer variables with lb < ub at the start, sorted by
 *             interval class (width 1, width 2, other), then by the distance
 *             of x (clamped into the box) to the nearest integer, then index;
 *   bulk      R unfixed variables left: 1 in recovery mode or when R <= 36,
 *             else ceil(sqrt(R)).  A bulk larger than one first re-sorts the
 *             unfixed variables by the implied-slack score S (orc_scores at
 *             the current box) descending, stably;
 *   values    two candidate values per member, h = 0 and 1, from the draw
 *             u = draws[2j + h]: with x clamped into the current box and
 *             f = x - floor(x), random rounding (up when u < f) for
 *             0.25 < f < 0.75, else the nearest integer (f < 0.5 down);
 *   cache     (optional probing cache of binaries: probe 2t + v fixes
 *             cache_vars[t] to v) a member whose cached probe for its value
 *             is infeasible is dropped; then a member whose value lies
 *             outside the box implied by the cached lists of the remaining
 *             members is dropped; the kept members' fixings and cached
 *             implications form the warm start of the bulk;
 *   propagate each of the two bulks from the current box with its fixings
 *             and implications applied, the changed list holding the kept
 *             members and the implied variables; a bulk that keeps no
 *             member counts as failed;
 *   accept    the first bulk that is not infeasible replaces the box and
 *             ends recovery mode;
 *   recover   when both fail: enter recovery mode (one variable per bulk)
 *             unless already in it or the path is marked infeasible, else
 *             mark the path infeasible; on a marked path a failed bulk's
 *             members are fixed to their first values without propagation
 *             and recovery mode ends;
 *   repair    (optional, limits rp) while the path is marked infeasible,
 *             each step ends with the repair procedure (orc_repair) on the
 *             current box, with the box the rounding started from as the
 *             original box, until one succeeds (its box replaces the
 *             current one and the mark is cleared) or rp->calls repairs
 *             have run; after that the marked path continues without
 *             repair (Algorithm 1; Section 2.3, the repair passage).
 *
 * lb/ub (length n) are read and written in place.  draws has 2n entries in
 * [0, 1).  res: status (ORC_OK, or ORC_INFEASIBLE for a marked path), then
 * bulks, singles (propagation steps with more than one / one variable),
 * recoveries, the number of variables fixed, nnz propagated (repairs'
 * propagations included), repairs run and repairs that succeeded. */
typedef struct {
    int32_t status, bulks, singles, recoveries, fixed, iterations;
    int64_t nnz_propagated;
    int32_t repairs, repaired;
} orc_round_result;

/* Repair inside the rounding: at most `calls` repair procedures per
 * rounding, each with the attempt and shift limits of orc_repair. */
typedef struct {
    int32_t calls, attempts, shifts;
} orc_repair_limits;

typedef struct {
    int32_t var, cls;
    double frac, key;
    int64_t pos;
} orc_rkey;

static int rkey_initial(const void *x, const void *y) {
    const orc_rkey *a = (const orc_rkey *)x, *b = (const orc_rkey *)y;
    if (a->cls != b->cls) return a->cls < b->cls ? -1 : 1;
    if (a->frac != b->frac) return a->frac < b->frac ? -1 : 1;
    return a->var < b->var ? -1 : (a->var > b->var ? 1 : 0);
}

static int rkey_slack(const void *x, const void *y) {
    const orc_rkey *a = (const orc_rkey *)x, *b = (const orc_rkey *)y;
    if (a->key != b->key) return a->key > b->key ? -1 : 1;
    return a->pos < b->pos ? -1 : (a->pos > b->pos ? 1 : 0);
}

static double clampd(double v, double l, double u) { return v < l ? l : (v > u ? u : v); }

/* Candidate value of variable j for draw u in the box [l, u_]. */
static double round_value(double x, double l, double hi, double u) {
    double xc = clampd(x, l, hi);
    double fl = floor(xc);
    double f = xc - fl;
    double v;
    if (f > 0.25 && f < 0.75) v = u < f ? fl + 1.0 : fl;
    else v = f < 0.5 ? fl : fl + 1.0;
    return clampd(v, l, hi);
}

int orc_round(const orc_instance *I, double *lb, double *ub, const double *x, const double *draws,
              int32_t k, const int32_t *cache_vars, const int8_t *cstatus, const int64_t *coff,
              const int32_t *cvar, const double *clb, const double *cub, const orc_options *o,
              const orc_repair_limits *rp, orc_round_result *res) {
    const int64_t n = I->n;
    memset(res, 0, sizeof(*res));
    for (int64_t j = 0; j < n; ++j)
        if (isnan(x[j]) || isnan(lb[j]) || isnan(ub[j])) return ORC_EINVAL;
    for (int64_t j = 0; j < 2 * n; ++j)
        if (!(draws[j] >= 0.0 && draws[j] < 1.0)) return ORC_EINVAL;
    int rc = 0;
    int64_t *cpos = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    orc_rkey *keys = (orc_rkey *)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_rkey));
    int32_t *order = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    double *S = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *vl[2], *vu[2], *val[2], *box_l, *box_u;
    int32_t *chg = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int8_t *keep = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
    vl[0] = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    vl[1] = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    vu[0] = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    vu[1] = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    val[0] = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    val[1] = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    box_l = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    box_u = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *start_l = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *start_u = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!cpos || !keys || !order || !S || !chg || !keep || !vl[0] || !vl[1] || !vu[0] || !vu[1] ||
        !val[0] || !val[1] || !box_l || !box_u || !start_l || !start_u) {
        rc = ORC_ENOMEM;
        goto done;
    }
    memcpy(start_l, lb, (size_t)n * sizeof(double));
    memcpy(start_u, ub, (size_t)n * sizeof(double));
    /* cache lookup: cpos[j] = t of the cached binary j, or -1 */
    for (int64_t j = 0; j < n; ++j) cpos[j] = -1;
    for (int32_t t = 0; t < k; ++t) {
        if (cache_vars[t] < 0 || cache_vars[t] >= n) { rc = ORC_EINVAL; goto done; }
        cpos[cache_vars[t]] = t;
    }
    /* initial order */
    int64_t nu = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (!I->vtype[j] || !(lb[j] < ub[j])) continue;
        double w = ub[j] - lb[j];
        double xc = clampd(x[j], lb[j], ub[j]);
        double f = xc - floor(xc);
        keys[nu].var = (int32_t)j;
        keys[nu].cls = w == 1.0 ? 0 : (w == 2.0 ? 1 : 2);
        keys[nu].frac = f < 1.0 - f ? f : 1.0 - f;
        nu += 1;
    }
    qsort(keys, (size_t)nu, sizeof(orc_rkey), rkey_initial);
    for (int64_t t = 0; t < nu; ++t) order[t] = keys[t].var;
    int recovery = 0, infeasible = 0;
    const int64_t cap_iter = 2 * nu + 16;
    for (;;) {
        /* the unfixed variables, in order */
        int64_t R = 0;
        for (int64_t t = 0; t < nu; ++t)
            if (lb[order[t]] < ub[order[t]]) order[R++] = order[t];
        nu = R;
        if (R == 0) break;
        if (res->iterations >= cap_iter) { rc = ORC_EINVAL; goto done; } /* cannot happen */
        res->iterations += 1;
        int64_t bulk = (recovery || R <= 36) ? 1 : (int64_t)ceil(sqrt((double)R));
        if (bulk > 1) {
            if ((rc = orc_scores(I, lb, ub, o, NULL, NULL, NULL, S)) != 0) goto done;
            for (int64_t t = 0; t < R; ++t) {
                keys[t].var = order[t];
                keys[t].key = S[order[t]];
                keys[t].pos = t;
            }
            qsort(keys, (size_t)R, sizeof(orc_rkey), rkey_slack);
            for (int64_t t = 0; t < R; ++t) order[t] = keys[t].var;
        }
        if (bulk > R) bulk = R;
        int ok[2] = {0, 0};
        orc_result pr[2];
        for (int h = 0; h < 2; ++h) {
            /* values */
            for (int64_t t = 0; t < bulk; ++t) {
                int32_t j = order[t];
                val[h][t] = round_value(x[j], lb[j], ub[j], draws[2 * (int64_t)j + h]);
                keep[t] = 1;
            }
            /* cache: infeasible cached values, then values outside the box
             * implied by the other members' cached lists */
            for (int64_t t = 0; t < bulk; ++t) {
                int32_t j = order[t];
                int64_t c = cpos[j];
                double v = val[h][t];
                if (c >= 0 && (v == 0.0 || v == 1.0) && cstatus[2 * c + (int64_t)v] == ORC_INFEASIBLE)
                    keep[t] = 0;
            }
            memcpy(box_l, lb, (size_t)n * sizeof(double));
            memcpy(box_u, ub, (size_t)n * sizeof(double));
            for (int64_t t = 0; t < bulk; ++t) {
                int64_t c = cpos[order[t]];
                double v = val[h][t];
                if (!keep[t] || c < 0 || !(v == 0.0 || v == 1.0)) continue;
                int64_t p = 2 * c + (int64_t)v;
                for (int64_t e = coff[p]; e < coff[p + 1]; ++e) {
                    if (clb[e] > box_l[cvar[e]]) box_l[cvar[e]] = clb[e];
                    if (cub[e] < box_u[cvar[e]]) box_u[cvar[e]] = cub[e];
                }
            }
            for (int64_t t = 0; t < bulk; ++t) {
                int32_t j = order[t];
                if (keep[t] && !(box_l[j] <= val[h][t] && val[h][t] <= box_u[j])) keep[t] = 0;
            }
            /* warm start: kept fixings and their cached implications; the
             * changed list is every variable whose box moved */
            memcpy(vl[h], lb, (size_t)n * sizeof(double));
            memcpy(vu[h], ub, (size_t)n * sizeof(double));
            int64_t nc = 0, kept = 0;
            for (int64_t t = 0; t < bulk; ++t) {
                if (!keep[t]) continue;
                int32_t j = order[t];
                double v = val[h][t];
                kept += 1;
                int64_t c = cpos[j];
                if (c >= 0 && (v == 0.0 || v == 1.0)) {
                    int64_t p = 2 * c + (int64_t)v;
                    for (int64_t e = coff[p]; e < coff[p + 1]; ++e) {
                        int32_t i = cvar[e];
                        if (clb[e] > vl[h][i]) vl[h][i] = clb[e];
                        if (cub[e] < vu[h][i]) vu[h][i] = cub[e];
                    }
                }
            }
            for (int64_t t = 0; t < bulk; ++t) {
                if (!keep[t]) continue;
                vl[h][order[t]] = val[h][t];
                vu[h][order[t]] = val[h][t];
            }
            for (int64_t i = 0; i < n; ++i)
                if (vl[h][i] != lb[i] || vu[h][i] != ub[i]) chg[nc++] = (int32_t)i;
            memset(&pr[h], 0, sizeof(pr[h]));
            if (kept == 0) {
                pr[h].status = ORC_INFEASIBLE;
                continue;
            }
            int prc = orc_propagate(I, vl[h], vu[h], chg, nc, o, ORC_MODE_WORKLIST, &pr[h]);
            if (prc < 0) { rc = prc; goto done; }
            res->nnz_propagated += pr[h].nnz_propagated;
            ok[h] = pr[h].status != ORC_INFEASIBLE;
        }
        if (bulk > 1) res->bulks += 1;
        else res->singles += 1;
        if (ok[0] || ok[1]) {
            int h = ok[0] ? 0 : 1;
            memcpy(lb, vl[h], (size_t)n * sizeof(double));
            memcpy(ub, vu[h], (size_t)n * sizeof(double));
            recovery = 0;
        } else {
            if (!recovery && !infeasible) {
                recovery = 1;
                res->recoveries += 1;
            } else {
                infeasible = 1;
            }
            if (infeasible) {
                for (int64_t t = 0; t < bulk; ++t) {
                    int32_t j = order[t];
                    lb[j] = val[0][t];
                    ub[j] = val[0][t];
                }
                recovery = 0;
            }
        }
        if (infeasible && rp && res->repairs < rp->calls) {
            orc_repair_result rr;
            int rrc = orc_repair(I, lb, ub, start_l, start_u, rp->shifts, rp->attempts, o, &rr);
            if (rrc < 0) { rc = rrc; goto done; }
            res->repairs += 1;
            res->nnz_propagated += rr.nnz_propagated;
            if (rr.status == ORC_OK) {
                res->repaired += 1;
                infeasible = 0;
            }
        }
    }
    res->status = infeasible ? ORC_INFEASIBLE : ORC_OK;
done:
    if (rc == 0) {
        int64_t fixed = 0;
        for (int64_t j = 0; j < n; ++j) fixed += I->vtype[j] && lb[j] == ub[j];
        res->fixed = (int32_t)fixed;
    }
    free(cpos); free(keys); free(order); free(S); free(chg); free(keep);
    free(vl[0]); free(vl[1]); free(vu[0]); free(vu[1]); free(val[0]); free(val[1]);
    free(box_l); free(box_u); free(start_l); free(start_u);
    return rc;
}
