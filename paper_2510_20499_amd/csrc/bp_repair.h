// bp_repair.h -- the repair procedure (kernels and host side of bp_repair,
// and the repair step of bp_round).  Included by bp_engine.hip after the
// scores, whose row pass provides the exact row activities.
//
// The paper's Section 2.3 (repair passage) and Algorithm 1's
// Run-Repair-Procedure: remove a row's violation by shifting the bounds of
// one variable of the row, a variable at a time, with a shift computed for
// every variable of the row; then propagate the fixed variables from the
// original bounds; repeat until that propagation is feasible or a limit is
// reached.  Readings (fixed by the include/bp.h comment of bp_repair):
// only the fixed integer variables F of the given box shift; the most
// violated row first; an integer shift of max(1, ceil(|r| - inttol)) units
// inside the original box; each candidate scored by the exact change of the
// total violation over its column; a failed propagation restarts from its
// own state one round before the detecting round.
//
// Per shift: the row pass (exact activities of every row, certified sums
// with the exact fallback), the violation of every row and its arg max
// (two passes of atomics), one lane per candidate of the chosen row walking
// its column, a one-workgroup arg min, and the update of one variable.  The
// host reads two small records per shift.  Repairs are rare (a marked
// rounding path), so the loop favours simplicity over launch count.
#pragma once

namespace bp {

// Control record of one repair shift (host-read).
struct RpCtl {
    unsigned long long ebits;  // bits of the largest row violation (a double >= 0)
    int32_t row;               // the most violated row, smallest index among equals
    int32_t bad;               // input check
    int32_t valid, var;        // best candidate: exists, variable
    double score, value;       // its score and new value
};

struct RpCand {
    double score, value;
    int32_t var, valid;
};

// Violation of a row at its activities: the excess over hi (no infinite
// minimum term) or below lo (no infinite maximum term) beyond feastol, else
// 0.  At most one side can be violated.
__device__ __forceinline__ double rp_violation(double2 sd, double minfin, double maxfin, int nmin,
                                               int nmax, double feastol) {
    const double INF = __builtin_inf();
    if (nmin == 0 && sd.y < INF && minfin > sd.y + feastol) return minfin - sd.y;
    if (nmax == 0 && sd.x > -INF && maxfin < sd.x - feastol) return sd.x - maxfin;
    return 0.0;
}

// New value of a fixed integer variable (value v, coefficient a) against a
// violation e of the hi side (hi_side) or the lo side, inside [l0, u0];
// false when it cannot move.
__device__ __forceinline__ bool rp_shift(double a, double e, bool hi_side, double v, double l0,
                                         double u0, double inttol, double &nv) {
    const double r = hi_side ? (-e) / a : e / a;
    double mag = ceil(fabs(r) - inttol);
    if (mag < 1.0) mag = 1.0;
    double d = r < 0.0 ? -mag : mag;
    if (d < 0.0 && !isinf(l0) && d < l0 - v) d = l0 - v;
    if (d > 0.0 && !isinf(u0) && d > u0 - v) d = u0 - v;
    if (d == 0.0) return false;
    nv = canon0(v + d);
    return true;
}

// Change of column entry q's row violation when the variable moves v -> nv.
__device__ __forceinline__ double rp_diff(const DInst &I, const double *cval, const RowSums *S,
                                          int64_t q, double v, double nv, double feastol) {
    const int r = I.col_row[q];
    const double c = cval[q];
    const RowSums A = S[r];
    const double2 sd = I.side[r];
    const double mn = canon0((A.minfin - c * v) + c * nv);
    const double mx = canon0((A.maxfin - c * v) + c * nv);
    const double e0 = rp_violation(sd, A.minfin, A.maxfin, A.nmin, A.nmax, feastol);
    const double e1 = rp_violation(sd, mn, mx, A.nmin, A.nmax, feastol);
    return e1 - e0;
}

// Exact sum of a candidate's changes (slow path of its certified sum).
__device__ __noinline__ double rp_exact_score(const DInst &I, const double *cval, const RowSums *S,
                                              int64_t j, double v, double nv, double feastol) {
    SuperAcc A;
    sa_zero(A);
    for (int64_t q = I.col_ptr[j]; q < I.col_ptr[j + 1]; ++q) sa_add(A, rp_diff(I, cval, S, q, v, nv, feastol));
    return canon0(sa_round(A));
}

__global__ void k_rp_check(const double *lb, const double *ub, const double *lb0, const double *ub0,
                           int64_t n, int32_t *bad) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double l = lb[j], u = ub[j], l0 = lb0[j], u0 = ub0[j];
        if (isnan(l) || isnan(u) || isnan(l0) || isnan(u0) || l < l0 || u > u0 || l0 > u0)
            atomicOr(bad, 1);
    }
}

__global__ void k_rp_fixed(const uint8_t *vtype, const double *lb, const double *ub, int64_t n,
                           uint8_t *fixed) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        fixed[j] = (vtype[j] && lb[j] == ub[j]) ? 1 : 0;
}

__global__ void k_rp_reset(RpCtl *c) {
    if (threadIdx.x == 0) {
        c->ebits = 0ull;
        c->row = 0x7fffffff;
        c->bad = 0;
        c->valid = 0;
        c->var = -1;
        c->score = 0.0;
        c->value = 0.0;
    }
}

// Largest violation over all rows (wave maxima, one atomic per wave).
__global__ void k_rp_viol_max(DInst I, const RowSums *S, double feastol, RpCtl *c) {
    unsigned long long best = 0ull;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.m;
         k += (int64_t)gridDim.x * blockDim.x) {
        const RowSums A = S[k];
        const double e = rp_violation(I.side[k], A.minfin, A.maxfin, A.nmin, A.nmax, feastol);
        const unsigned long long b = (unsigned long long)__double_as_longlong(e);
        if (b > best) best = b;
    }
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const unsigned long long o = __shfl_xor(best, w, 64);
        if (o > best) best = o;
    }
    if (__lane_id() == 0 && best) atomicMax(&c->ebits, best);
}

// Smallest row holding the largest violation.
__global__ void k_rp_viol_row(DInst I, const RowSums *S, double feastol, RpCtl *c) {
    const unsigned long long top = c->ebits;
    if (!top) return;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.m;
         k += (int64_t)gridDim.x * blockDim.x) {
        const RowSums A = S[k];
        const double e = rp_violation(I.side[k], A.minfin, A.maxfin, A.nmin, A.nmax, feastol);
        if ((unsigned long long)__double_as_longlong(e) == top) atomicMin(&c->row, (int)k);
    }
}

// One lane per nonzero of the chosen row: the shift of its variable (when
// fixed) and the certified sum of the changes over the variable's column.
__global__ void k_rp_cand(DInst I, const double *cval, const RowSums *S, const double2 *box,
                          const uint8_t *fixed, const double *lb0, const double *ub0, const RpCtl *c,
                          double feastol, double inttol, RpCand *cand) {
    const int kb = c->row;
    const int64_t p0 = I.row_ptr[kb], L = I.row_ptr[kb + 1] - p0;
    const RowSums R = S[kb];
    const double2 sd = I.side[kb];
    const double e = __longlong_as_double((long long)c->ebits);
    const bool hi_side = R.nmin == 0 && sd.y < __builtin_inf() && R.minfin > sd.y + feastol;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < L;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = I.col[p0 + t];
        RpCand out;
        out.var = j;
        out.valid = 0;
        out.score = 0.0;
        out.value = 0.0;
        double nv = 0.0;
        const double v = box[j].x;
        if (fixed[j] && rp_shift(I.val[p0 + t], e, hi_side, v, lb0[j], ub0[j], inttol, nv)) {
            Acc A;
            acc_zero(A);
            for (int64_t q = I.col_ptr[j]; q < I.col_ptr[j + 1]; ++q) acc_add(A, rp_diff(I, cval, S, q, v, nv, feastol));
            double sc = 0.0;
            if (!acc_certify(A, sc)) sc = rp_exact_score(I, cval, S, j, v, nv, feastol);
            out.valid = 1;
            out.score = canon0(sc);
            out.value = nv;
        }
        cand[t] = out;
    }
}

// Lowest score, then the smaller position in the row (= smaller variable,
// columns ascend in a row); one workgroup of RP_BEST threads.
constexpr int RP_BEST = 1024;

__global__ void __launch_bounds__(RP_BEST) k_rp_best(const RpCand *cand, int64_t L, RpCtl *c) {
    __shared__ double ss[RP_BEST];
    __shared__ long long st[RP_BEST];
    double bs = 0.0;
    long long bt = -1;
    for (int64_t t = threadIdx.x; t < L; t += RP_BEST) {
        const RpCand x = cand[t];
        if (x.valid && (bt < 0 || x.score < bs)) {
            bs = x.score;
            bt = t;
        }
    }
    ss[threadIdx.x] = bs;
    st[threadIdx.x] = bt;
    __syncthreads();
    for (int w = RP_BEST / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double os = ss[threadIdx.x + w];
            const long long ot = st[threadIdx.x + w];
            const long long mt = st[threadIdx.x];
            if (ot >= 0 && (mt < 0 || os < ss[threadIdx.x] || (os == ss[threadIdx.x] && ot < mt))) {
                ss[threadIdx.x] = os;
                st[threadIdx.x] = ot;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && st[0] >= 0) {
        const RpCand x = cand[st[0]];
        c->valid = 1;
        c->var = x.var;
        c->score = x.score;
        c->value = x.value;
    }
}

__global__ void k_rp_apply(const RpCtl *c, double2 *box) {
    if (threadIdx.x == 0 && c->valid) box[c->var] = make_double2(c->value, c->value);
}

// The original box with F's current values: the start of a propagation
// from the original bounds.
__global__ void k_rp_fixbox(const double2 *box, const uint8_t *fixed, const double *lb0,
                            const double *ub0, int64_t n, double *pl, double *pu) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (fixed[j]) {
            const double v = box[j].x;
            pl[j] = v;
            pu[j] = v;
        } else {
            pl[j] = lb0[j];
            pu[j] = ub0[j];
        }
    }
}

}  // namespace bp
