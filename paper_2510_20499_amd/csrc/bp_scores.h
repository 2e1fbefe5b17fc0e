// bp_scores.h -- probe priority and implied-slack scores (kernels and host
// side of bp_scores / bp_probe_order).  Included by bp_engine.hip after the
// instance and its helpers.
//
// The paper's Section 2.2 ranks the variables to probe by three criteria in
// lexicographic order: the number of rows a variable violates when its
// contribution flips from one bound to the other (only for variables whose
// coefficients have both signs), the largest such violation, and the
// smallest unit slack; Section 2.3 defines the unit slack consumption
// s = a / slack of a variable in a row and the implied-slack score
// S = sum of s^2 over the rows of the variable.
//
// Two passes over the instance at the given bounds:
//   rows  exact activities of every row (the same correctly rounded sums and
//         infinite counts as propagation), light rows by the row bins of the
//         instance (G lanes per row), longer rows by chunks of SC_CHUNK
//         nonzeros whose partial sums a wave per row merges;
//   vars  one lane per variable walks its column (CSC values, built once per
//         instance) and computes its four scores; the sum of s^2 is certified
//         like the activities and falls back to the exact accumulator.
// The probe order sorts (nviol desc, maxviol desc, minunit asc, index asc)
// keys with a bitonic network in global memory.
#pragma once

namespace bp {

constexpr int SC_CHUNK = 4096;  // nonzeros per partial sum of a row longer than 1024

struct ScRowAct {
    double minfin, maxfin;
    int32_t nmin, nmax;
};

__device__ __forceinline__ BView sc_view(const double2 *bnd) {
    BView v;
    v.own = bnd;
    v.base = bnd;
    v.filt = nullptr;
    v.dirty = nullptr;
    v.overlay = 0;
    return v;
}

// Activities of the rows rows[0..count) of one light bin, G lanes per row
// (G == 64: one row per wave, several nonzeros per lane).
template <int G>
__global__ void __launch_bounds__(WG) k_sc_light(DInst I, const double2 *bnd, const int32_t *rows,
                                                 int64_t count, ScRowAct *act) {
    const int lane = __lane_id();
    const int gl = lane & (G - 1);
    const int64_t per_wave = 64 / G;
    const int64_t nwaves = (int64_t)gridDim.x * (WG / 64);
    const BView view = sc_view(bnd);
    // Wave-uniform trip count: the group reductions shuffle across the wave.
    for (int64_t w = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6); w * per_wave < count;
         w += nwaves) {
        const int64_t t = w * per_wave + lane / G;
        const bool valid = t < count;
        int k = 0;
        int64_t p0 = 0, p1 = 0;
        if (valid) {
            k = rows[t];
            p0 = I.row_ptr[k];
            p1 = I.row_ptr[k + 1];
        }
        Acc mn, mx;
        acc_zero(mn);
        acc_zero(mx);
        const int iters = G < 64 ? 1 : (int)((p1 - p0 + 63) / 64);
        for (int it = 0; it < iters; ++it) {
            const int64_t p = p0 + gl + (int64_t)it * G;
            if (p < p1) {
                const double a = I.val[p];
                const double2 b = bnd[I.col[p]];
                add_terms(mn, mx, a, b.x, b.y);
            }
        }
        acc_group_reduce<G>(mn);
        acc_group_reduce<G>(mx);
        double vmin = 0.0, vmax = 0.0;
        const bool okmin = acc_certify(mn, vmin);
        const bool okmax = acc_certify(mx, vmax);
        if (valid && gl == 0) {
            if (!okmin) vmin = exact_side(I, view, p0, p1, false);
            if (!okmax) vmax = exact_side(I, view, p0, p1, true);
            ScRowAct r;
            r.minfin = vmin;
            r.maxfin = vmax;
            r.nmin = mn.ninf;
            r.nmax = mx.ninf;
            act[k] = r;
        }
    }
}

// Partial sums of the chunks of the long rows: chunk u is (row, chunk
// index, chunks of the row, -); one workgroup per chunk.
__global__ void __launch_bounds__(WG) k_sc_chunks(DInst I, const double2 *bnd, const int4 *chunks,
                                                  int64_t nchunks, Acc *part) {
    __shared__ WgScratch W;
    for (int64_t u = blockIdx.x; u < nchunks; u += gridDim.x) {
        const int4 rec = chunks[u];
        const int64_t r0 = I.row_ptr[rec.x], r1 = I.row_ptr[rec.x + 1];
        const int64_t p0 = r0 + (int64_t)rec.y * SC_CHUNK;
        const int64_t p1 = min(r1, p0 + (int64_t)SC_CHUNK);
        Acc mn, mx;
        acc_zero(mn);
        acc_zero(mx);
        double wmax = 0.0;
        for (int64_t p = p0 + threadIdx.x; p < p1; p += WG) {
            const double2 b = bnd[I.col[p]];
            add_terms(mn, mx, I.val[p], b.x, b.y);
        }
        wg_reduce(mn, mx, wmax, W);
        if (threadIdx.x == 0) {
            part[2 * u] = mn;
            part[2 * u + 1] = mx;
        }
    }
}

// One wave per long row: its chunk partials merged in chunk order (lane l
// takes chunks l, l + 64, ...), certified, else the exact accumulator.
__global__ void __launch_bounds__(WG) k_sc_combine(DInst I, const double2 *bnd, const int32_t *rows,
                                                   const int64_t *first, int64_t nrows,
                                                   const Acc *part, ScRowAct *act) {
    const int lane = __lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (WG / 64);
    const BView view = sc_view(bnd);
    for (int64_t w = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6); w < nrows; w += nwaves) {
        const int k = rows[w];
        const int64_t c0 = first[w], nch = first[w + 1] - c0;
        Acc A, B;
        acc_zero(A);
        acc_zero(B);
        for (int64_t j = lane; j < nch; j += 64) {
            const Acc a = part[2 * (c0 + j)], b = part[2 * (c0 + j) + 1];
            acc_merge(A, a.s, a.c, a.e, a.ninf);
            acc_merge(B, b.s, b.c, b.e, b.ninf);
        }
        acc_group_reduce<64>(A);
        acc_group_reduce<64>(B);
        double vmin = 0.0, vmax = 0.0;
        const bool okmin = acc_certify(A, vmin);
        const bool okmax = acc_certify(B, vmax);
        if (lane == 0) {
            const int64_t p0 = I.row_ptr[k], p1 = I.row_ptr[k + 1];
            if (!okmin) vmin = exact_side(I, view, p0, p1, false);
            if (!okmax) vmax = exact_side(I, view, p0, p1, true);
            ScRowAct r;
            r.minfin = vmin;
            r.maxfin = vmax;
            r.nmin = A.ninf;
            r.nmax = B.ninf;
            act[k] = r;
        }
    }
}

// CSC values: entry p of column j is row k = col_row[p]; its coefficient is
// found by binary search of j in row k (column indices ascend in a row).
__global__ void k_sc_cval(DInst I, double *cval) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < I.n;
         j += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t p = I.col_ptr[j]; p < I.col_ptr[j + 1]; ++p) {
            const int k = I.col_row[p];
            int64_t lo = I.row_ptr[k], hi = I.row_ptr[k + 1] - 1;
            while (lo < hi) {
                const int64_t mid = lo + ((hi - lo) >> 1);
                if (I.col[mid] < j) lo = mid + 1;
                else hi = mid;
            }
            cval[p] = I.val[lo];
        }
    }
}

// The two finite sides of row k usable for slack (no infinite term on that
// side) and their slacks hi - minfin and maxfin - lo.
struct ScSides {
    bool hi_ok, lo_ok;
    double slack_hi, slack_lo;
};

__device__ __forceinline__ ScSides sc_sides(const ScRowAct &R, double2 sd) {
    ScSides S;
    S.hi_ok = sd.y < __builtin_inf() && R.nmin == 0;
    S.lo_ok = sd.x > -__builtin_inf() && R.nmax == 0;
    S.slack_hi = S.hi_ok ? sd.y - R.minfin : 0.0;
    S.slack_lo = S.lo_ok ? R.maxfin - sd.x : 0.0;
    return S;
}

// Exact sum of the finite (a / slack)^2 terms of variable j (slow path).
__device__ __noinline__ double sc_exact_score(const DInst &I, const double *cval,
                                              const ScRowAct *act, int64_t j) {
    SuperAcc S;
    sa_zero(S);
    for (int64_t p = I.col_ptr[j]; p < I.col_ptr[j + 1]; ++p) {
        const int k = I.col_row[p];
        const double a = cval[p];
        const ScSides sd = sc_sides(act[k], I.side[k]);
        for (int side = 0; side < 2; ++side) {
            if (side == 0 ? !sd.hi_ok : !sd.lo_ok) continue;
            const double s = a / (side == 0 ? sd.slack_hi : sd.slack_lo);
            const double t = s * s;
            if (!isinf(t)) sa_add(S, t);
        }
    }
    return canon0(sa_round(S));
}

// Scores of every variable, one lane per variable (any output may be null).
__global__ void __launch_bounds__(WG) k_sc_vars(DInst I, const double2 *bnd, const double *cval,
                                                const ScRowAct *act, double feastol, int32_t *nviol,
                                                double *maxviol, double *minunit, double *sscore) {
    const double INF = __builtin_inf();
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < I.n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double2 b = bnd[j];
        const bool finite = !isinf(b.x) && !isinf(b.y);
        bool pos = false, neg = false, sinf = false;
        int32_t nv = 0;
        double mv = 0.0, mu = INF;
        Acc A;
        acc_zero(A);
        for (int64_t p = I.col_ptr[j]; p < I.col_ptr[j + 1]; ++p) {
            const int k = I.col_row[p];
            const double a = cval[p];
            const ScSides sd = sc_sides(act[k], I.side[k]);
            pos = pos || a > 0.0;
            neg = neg || a < 0.0;
            if (finite) {
                // flipped contribution: how far moving j between its bounds
                // pushes the row's extreme activities
                const double bmin = a > 0.0 ? b.x : b.y;
                const double bmax = a > 0.0 ? b.y : b.x;
                const double d = a * bmax - a * bmin;
                bool viol = false;
                double worst = 0.0;
                if (sd.hi_ok) {
                    const double e = d - sd.slack_hi;
                    if (e > feastol) {
                        viol = true;
                        worst = e;
                    }
                }
                if (sd.lo_ok) {
                    const double e = d - sd.slack_lo;
                    if (e > feastol && (!viol || e > worst)) {
                        viol = true;
                        worst = e;
                    }
                }
                if (viol) {
                    nv += 1;
                    if (worst > mv) mv = worst;
                }
            }
            for (int side = 0; side < 2; ++side) {
                if (side == 0 ? !sd.hi_ok : !sd.lo_ok) continue;
                const double slack = side == 0 ? sd.slack_hi : sd.slack_lo;
                const double u = slack / fabs(a);
                if (u < mu) mu = u;
                const double s = a / slack;
                const double t = s * s;
                if (isinf(t)) sinf = true;
                else acc_add(A, t);
            }
        }
        if (!(pos && neg)) {
            nv = 0;
            mv = 0.0;
        }
        if (nviol) nviol[j] = nv;
        if (maxviol) maxviol[j] = canon0(mv);
        if (minunit) minunit[j] = canon0(mu);
        if (sscore) {
            double v = 0.0;
            if (sinf) v = INF;
            else if (!acc_certify(A, v)) v = sc_exact_score(I, cval, act, j);
            sscore[j] = canon0(v);
        }
    }
}

__global__ void k_sc_nan(const double2 *bnd, int64_t n, int32_t *bad) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double2 b = bnd[j];
        if (isnan(b.x) || isnan(b.y)) atomicOr(bad, 1);
    }
}

// Probe order keys: more violated rows, larger violation, smaller unit
// slack, smaller index first.  Padding keys (nviol = -1) go last.
struct ScKey {
    int32_t nviol, var;
    double maxviol, minunit;
};

__device__ __forceinline__ bool sc_before(const ScKey &a, const ScKey &b) {
    if (a.nviol != b.nviol) return a.nviol > b.nviol;
    if (a.maxviol != b.maxviol) return a.maxviol > b.maxviol;
    if (a.minunit != b.minunit) return a.minunit < b.minunit;
    return a.var < b.var;
}

__global__ void k_sc_keys(const int32_t *vars, int64_t k, int64_t kpad, const int32_t *nv,
                          const double *mv, const double *mu, ScKey *keys) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < kpad;
         t += (int64_t)gridDim.x * blockDim.x) {
        ScKey K;
        if (t < k) {
            const int32_t j = vars[t];
            K.nviol = nv[j];
            K.var = j;
            K.maxviol = mv[j];
            K.minunit = mu[j];
        } else {
            K.nviol = -1;
            K.var = NONE;
            K.maxviol = 0.0;
            K.minunit = 0.0;
        }
        keys[t] = K;
    }
}

// One compare-exchange step of the bitonic network over kpad (a power of
// two) keys: blocks of `size` sorted alternately up and down, partners at
// distance `stride`.
__global__ void k_sc_bitonic(ScKey *keys, int64_t kpad, int64_t size, int64_t stride) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < kpad;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = i ^ stride;
        if (l <= i) continue;
        const bool up = (i & size) == 0;
        const ScKey A = keys[i], B = keys[l];
        const bool swap = up ? sc_before(B, A) : sc_before(A, B);
        if (swap) {
            keys[i] = B;
            keys[l] = A;
        }
    }
}

__global__ void k_sc_order_out(const ScKey *keys, int64_t k, int32_t *order) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < k;
         t += (int64_t)gridDim.x * blockDim.x)
        order[t] = keys[t].var;
}

}  // namespace bp
