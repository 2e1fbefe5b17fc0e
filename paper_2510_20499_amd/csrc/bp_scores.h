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
//         nonzeros whose partial sums a wave per row merges; each row keeps
//         only its two slacks (16 B, +inf for a side that has none);
//   vars  one lane per variable walks its column (the instance's CSC
//         coefficients) four entries at a time and computes its four scores; the
//         sum of s^2 is certified like the activities and falls back to the
//         exact accumulator.
// The probe order sorts (nviol desc, maxviol desc, minunit asc, index asc)
// keys with a bitonic network in global memory.
#pragma once

namespace bp {

constexpr int SC_CHUNK = 4096;  // nonzeros per partial sum of a row longer than 1024

// Slacks of row k from its exact activities: (hi - minfin, maxfin - lo), +inf
// for a side that is infinite or has an infinite term.  A usable side's
// slack can only be +inf when its activity overflowed; it then adds nothing
// to any score (zero term, infinite unit slack, no violation), exactly as
// a side without slack.
__device__ __forceinline__ double2 sc_slacks(double2 sd, double minfin, double maxfin, int nmin,
                                             int nmax) {
    const double INF = __builtin_inf();
    const bool hi_ok = sd.y < INF && nmin == 0;
    const bool lo_ok = sd.x > -INF && nmax == 0;
    double sh = hi_ok ? sd.y - minfin : INF;
    double sl = lo_ok ? maxfin - sd.x : INF;
    return make_double2(sh, sl);
}

// Exact activities of a row (the repair procedure needs them whole, not
// only as slacks): finite parts and infinite-term counts.
struct RowSums {
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

// Activities of one unit (256 / G rows) of the rows rows[0..count) of a
// light bin, G lanes per row (G == 64: one row per wave, several nonzeros
// per lane); the row's slacks are stored.  Reached by whole waves.
template <int G>
__device__ void sc_light_unit(const DInst &I, const double2 *bnd, const int32_t *rows,
                              int64_t count, int64_t unit, double2 *slk, RowSums *full) {
    const int lane = __lane_id();
    const int gl = lane & (G - 1);
    const int64_t per_wave = 64 / G;
    const int64_t t = (unit * (WG / 64) + (threadIdx.x >> 6)) * per_wave + lane / G;
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
        const BView view = sc_view(bnd);
        if (!okmin) vmin = exact_side(I, view, p0, p1, false);
        if (!okmax) vmax = exact_side(I, view, p0, p1, true);
        slk[k] = sc_slacks(I.side[k], vmin, vmax, mn.ninf, mx.ninf);
        if (full) full[k] = RowSums{canon0(vmin), canon0(vmax), mn.ninf, mx.ninf};
    }
}

// Partial sums of chunk u of the long rows (chunk record: row, chunk index,
// chunks of the row); one workgroup.
__device__ void sc_chunk_unit(const DInst &I, const double2 *bnd, const int4 *chunks, int64_t u,
                              Acc *part, WgScratch &W) {
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

// Work of the row pass: the chunks of the long rows first (one unit each),
// then the light bins 10..0 (256 / G rows per unit).
struct ScRowsWork {
    const int4 *chunks;
    int64_t nchunks;
    const int32_t *rows[NLIGHT];  // rows of light bin b
    int64_t count[NLIGHT];
    int64_t start[NLIGHT + 2];    // unit offsets: [0] chunks, [1 + j] bin 10 - j
};

__global__ void __launch_bounds__(WG) k_sc_rows(DInst I, const double2 *bnd, ScRowsWork R,
                                                Acc *part, double2 *slk, RowSums *full) {
    __shared__ WgScratch W;
    const int64_t total = R.start[NLIGHT + 1];
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        if (u < R.start[1]) {
            sc_chunk_unit(I, bnd, R.chunks, u, part, W);
            continue;
        }
        int j = 0;
        while (u >= R.start[2 + j]) ++j;
        const int b = NLIGHT - 1 - j;
        const int64_t lu = u - R.start[1 + j];
        switch (b) {
            case 0: sc_light_unit<1>(I, bnd, R.rows[0], R.count[0], lu, slk, full); break;
            case 1: sc_light_unit<2>(I, bnd, R.rows[1], R.count[1], lu, slk, full); break;
            case 2: sc_light_unit<4>(I, bnd, R.rows[2], R.count[2], lu, slk, full); break;
            case 3: sc_light_unit<8>(I, bnd, R.rows[3], R.count[3], lu, slk, full); break;
            case 4: sc_light_unit<16>(I, bnd, R.rows[4], R.count[4], lu, slk, full); break;
            case 5: sc_light_unit<32>(I, bnd, R.rows[5], R.count[5], lu, slk, full); break;
            default: sc_light_unit<64>(I, bnd, R.rows[b], R.count[b], lu, slk, full); break;
        }
    }
}

// One wave per long row: its chunk partials merged in chunk order (lane l
// takes chunks l, l + 64, ...), certified, else the exact accumulator.
__global__ void __launch_bounds__(WG) k_sc_combine(DInst I, const double2 *bnd, const int32_t *rows,
                                                   const int64_t *first, int64_t nrows,
                                                   const Acc *part, double2 *slk, RowSums *full) {
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
            slk[k] = sc_slacks(I.side[k], vmin, vmax, A.ninf, B.ninf);
            if (full) full[k] = RowSums{canon0(vmin), canon0(vmax), A.ninf, B.ninf};
        }
    }
}

// The terms of one column entry (coefficient a, row slacks sl) into the
// running scores of its variable.
struct ScVar {
    bool pos, neg, sinf;
    int32_t nv;
    double mv, mu;
    Acc A;
};

__device__ __forceinline__ void sc_entry(ScVar &V, double a, double2 sl, bool finite, double bmin_lo,
                                         double bmin_hi, double feastol) {
    const double INF = __builtin_inf();
    const bool hi_ok = sl.x < INF, lo_ok = sl.y < INF;
    V.pos = V.pos || a > 0.0;
    V.neg = V.neg || a < 0.0;
    if (finite) {
        // flipped contribution: how far moving the variable between its
        // bounds pushes the row's extreme activities
        const double bmin = a > 0.0 ? bmin_lo : bmin_hi;
        const double bmax = a > 0.0 ? bmin_hi : bmin_lo;
        const double d = a * bmax - a * bmin;
        bool viol = false;
        double worst = 0.0;
        if (hi_ok) {
            const double e = d - sl.x;
            if (e > feastol) {
                viol = true;
                worst = e;
            }
        }
        if (lo_ok) {
            const double e = d - sl.y;
            if (e > feastol && (!viol || e > worst)) {
                viol = true;
                worst = e;
            }
        }
        if (viol) {
            V.nv += 1;
            if (worst > V.mv) V.mv = worst;
        }
    }
    for (int side = 0; side < 2; ++side) {
        if (side == 0 ? !hi_ok : !lo_ok) continue;
        const double slack = side == 0 ? sl.x : sl.y;
        const double u = slack / fabs(a);
        if (u < V.mu) V.mu = u;
        const double s = a / slack;
        const double t = s * s;
        if (isinf(t)) V.sinf = true;
        else acc_add(V.A, t);
    }
}

// Exact sum of the finite (a / slack)^2 terms of variable j (slow path).
__device__ __noinline__ double sc_exact_score(const DInst &I, const double *cval,
                                              const double2 *slk, int64_t j) {
    const double INF = __builtin_inf();
    SuperAcc S;
    sa_zero(S);
    for (int64_t p = I.col_ptr[j]; p < I.col_ptr[j + 1]; ++p) {
        const double a = cval[p];
        const double2 sl = slk[I.col_row[p]];
        for (int side = 0; side < 2; ++side) {
            const double slack = side == 0 ? sl.x : sl.y;
            if (!(slack < INF)) continue;
            const double s = a / slack;
            const double t = s * s;
            if (!isinf(t)) sa_add(S, t);
        }
    }
    return canon0(sa_round(S));
}

constexpr int SC_UNROLL = 4;  // column entries whose loads a lane issues together

// Scores of every variable, one lane per variable (any output may be null).
__global__ void __launch_bounds__(WG) k_sc_vars(DInst I, const double2 *bnd, const double *cval,
                                                const double2 *slk, double feastol, int32_t *nviol,
                                                double *maxviol, double *minunit, double *sscore) {
    const double INF = __builtin_inf();
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < I.n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double2 b = bnd[j];
        const bool finite = !isinf(b.x) && !isinf(b.y);
        ScVar V;
        V.pos = V.neg = V.sinf = false;
        V.nv = 0;
        V.mv = 0.0;
        V.mu = INF;
        acc_zero(V.A);
        const int64_t c0 = I.col_ptr[j], c1 = I.col_ptr[j + 1];
        for (int64_t p = c0; p < c1; p += SC_UNROLL) {
            int k[SC_UNROLL];
            double a[SC_UNROLL];
            double2 sl[SC_UNROLL];
#pragma unroll
            for (int q = 0; q < SC_UNROLL; ++q) {
                if (p + q < c1) {
                    k[q] = I.col_row[p + q];
                    a[q] = cval[p + q];
                }
            }
#pragma unroll
            for (int q = 0; q < SC_UNROLL; ++q)
                if (p + q < c1) sl[q] = slk[k[q]];
#pragma unroll
            for (int q = 0; q < SC_UNROLL; ++q)
                if (p + q < c1) sc_entry(V, a[q], sl[q], finite, b.x, b.y, feastol);
        }
        if (!(V.pos && V.neg)) {
            V.nv = 0;
            V.mv = 0.0;
        }
        if (nviol) nviol[j] = V.nv;
        if (maxviol) maxviol[j] = canon0(V.mv);
        if (minunit) minunit[j] = canon0(V.mu);
        if (sscore) {
            double v = 0.0;
            if (V.sinf) v = INF;
            else if (!acc_certify(V.A, v)) v = sc_exact_score(I, cval, slk, j);
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

// The same network inside LDS for the steps whose partners lie in one tile
// of SC_TILE keys: sizes size_lo..size_hi, the first of them starting at
// `stride0`, every later one at size / 2.  Directions come from the global
// index, so tiles of one block of the network agree.
constexpr int SC_TILE = 1024;
constexpr int SC_TILE_THREADS = SC_TILE / 2;  // one compare-exchange per thread and step

__global__ void __launch_bounds__(SC_TILE_THREADS) k_sc_bitonic_tile(ScKey *keys, int64_t kpad,
                                                                     int64_t size_lo, int64_t size_hi,
                                                                     int64_t stride0) {
    __shared__ ScKey T[SC_TILE];
    const int64_t tile = kpad < SC_TILE ? kpad : SC_TILE;
    for (int64_t base = (int64_t)blockIdx.x * tile; base < kpad; base += (int64_t)gridDim.x * tile) {
        for (int64_t t = threadIdx.x; t < tile; t += SC_TILE_THREADS) T[t] = keys[base + t];
        for (int64_t size = size_lo; size <= size_hi; size <<= 1) {
            for (int64_t stride = size == size_lo ? stride0 : size >> 1; stride > 0; stride >>= 1) {
                __syncthreads();
                for (int64_t q = threadIdx.x; q < tile / 2; q += SC_TILE_THREADS) {
                    const int64_t i = 2 * stride * (q / stride) + (q % stride);
                    const int64_t l = i + stride;
                    const bool up = ((base + i) & size) == 0;
                    const ScKey A = T[i], B = T[l];
                    if (up ? sc_before(B, A) : sc_before(A, B)) {
                        T[i] = B;
                        T[l] = A;
                    }
                }
            }
        }
        __syncthreads();
        for (int64_t t = threadIdx.x; t < tile; t += SC_TILE_THREADS) keys[base + t] = T[t];
        __syncthreads();
    }
}

__global__ void k_sc_order_out(const ScKey *keys, int64_t k, int32_t *order) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < k;
         t += (int64_t)gridDim.x * blockDim.x)
        order[t] = keys[t].var;
}

}  // namespace bp
