// bp_round.h -- bound-propagation rounding (bulk fix-and-propagate): the
// device steps of bp_round and its host loop.  Included by bp_engine.hip
// after the scores (bp_scores.h, bp_scores_run.h).
//
// The paper's Algorithm 1 (PROPAGATION-ROUND) with Section 2.3, without the
// repair procedure and the LP polish: the integer variables of a box are
// fixed towards a fractional point x a bulk at a time, and every bulk is
// propagated.  The host runs the loop (bulk sizes, acceptance, recovery);
// every per-variable step runs on the device:
//   - the unfixed list is kept in order by stable compactions (block counts,
//     a one-workgroup scan of the counts, block-local scans);
//   - the initial order and the implied-slack re-sort use the bitonic key
//     sort of the probe order, with the position as the last key (stable);
//   - S comes from the scores kernels at the current box;
//   - candidate values, the probing-cache conflict tests and the warm starts
//     of the two bulks are one lane per member / cache entry, with the same
//     order-preserving 64-bit keys and integer min/max atomics as the
//     propagation's candidates;
//   - the two bulks run as one bp_propagate_batch of two vectors.
#pragma once

namespace bp {

constexpr int CMP_BLOCK = 1024;  // elements per block of the stable compaction

// Number of flagged elements in each block of CMP_BLOCK.
__global__ void __launch_bounds__(WG) k_cmp_count(const uint8_t *flags, int64_t N, int32_t *bcnt) {
    __shared__ int32_t s;
    for (int64_t b = blockIdx.x; b * CMP_BLOCK < N; b += gridDim.x) {
        if (threadIdx.x == 0) s = 0;
        __syncthreads();
        int32_t c = 0;
        for (int64_t i = b * CMP_BLOCK + threadIdx.x; i < min(N, (b + 1) * CMP_BLOCK); i += WG)
            c += flags[i] ? 1 : 0;
        atomicAdd(&s, c);
        __syncthreads();
        if (threadIdx.x == 0) bcnt[b] = s;
        __syncthreads();
    }
}

// Exclusive scan of the block counts by one workgroup; total in *total.
__global__ void __launch_bounds__(WG) k_cmp_scan(int32_t *bcnt, int64_t nb, int64_t *total) {
    __shared__ int64_t part[WG];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += WG) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nb ? bcnt[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < WG; d <<= 1) {
            const int64_t y = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nb) bcnt[i] = (int32_t)(carry + part[threadIdx.x] - v);
        __syncthreads();
        if (threadIdx.x == WG - 1) carry += part[WG - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// out[offset of block + rank in block] = values ? values[i] : i for every
// flagged i, in order.
__global__ void __launch_bounds__(WG) k_cmp_write(const uint8_t *flags, const int32_t *values,
                                                  int64_t N, const int32_t *boff, int32_t *out) {
    __shared__ int32_t part[WG];
    constexpr int PER = CMP_BLOCK / WG;
    for (int64_t b = blockIdx.x; b * CMP_BLOCK < N; b += gridDim.x) {
        // thread t takes elements [t*PER, t*PER + PER) of the block
        const int64_t i0 = b * CMP_BLOCK + (int64_t)threadIdx.x * PER;
        int32_t c = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) c += (i0 + q < N && flags[i0 + q]) ? 1 : 0;
        part[threadIdx.x] = c;
        __syncthreads();
        for (int d = 1; d < WG; d <<= 1) {
            const int32_t y = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += y;
            __syncthreads();
        }
        int32_t pos = boff[b] + part[threadIdx.x] - c;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int64_t i = i0 + q;
            if (i < N && flags[i]) out[pos++] = values ? values[i] : (int32_t)i;
        }
        __syncthreads();
    }
}

// Flags: integer variables with lb < ub.
__global__ void k_rd_flag_start(const uint8_t *vtype, const double *lb, const double *ub, int64_t n,
                                uint8_t *flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = (vtype[i] != 0 && lb[i] < ub[i]) ? 1 : 0;
}

// Flags: entries of the order list that are still unfixed.
__global__ void k_rd_flag_unfixed(const int32_t *order, int64_t R, const double *lb, const double *ub,
                                  uint8_t *flags) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < R;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = order[t];
        flags[t] = lb[j] < ub[j] ? 1 : 0;
    }
}

// Initial order keys: interval class (width 1, width 2, other), distance of
// x (clamped into the box) to the nearest integer, index.
__global__ void k_rd_initial_keys(const int32_t *vars, int64_t R, int64_t kpad, const double *x,
                                  const double *lb, const double *ub, ScKey *keys) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < kpad;
         t += (int64_t)gridDim.x * blockDim.x) {
        ScKey K;
        if (t < R) {
            const int32_t j = vars[t];
            const double l = lb[j], u = ub[j];
            const double w = u - l;
            const double xc = fmin(fmax(x[j], l), u);
            const double f = xc - floor(xc);
            const double frac = f < 1.0 - f ? f : 1.0 - f;
            K.nviol = w == 1.0 ? 2 : (w == 2.0 ? 1 : 0);  // descending: width 1 first
            K.var = j;
            K.maxviol = -frac;  // descending: nearest to an integer first
            K.minunit = 0.0;
        } else {
            K.nviol = -1;
            K.var = NONE;
            K.maxviol = 0.0;
            K.minunit = 0.0;
        }
        keys[t] = K;
    }
}

// Implied-slack keys: S descending, then the current position.
__global__ void k_rd_slack_keys(const int32_t *order, int64_t R, int64_t kpad, const double *S,
                                ScKey *keys) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < kpad;
         t += (int64_t)gridDim.x * blockDim.x) {
        ScKey K;
        if (t < R) {
            K.nviol = 0;
            K.var = (int32_t)t;
            K.maxviol = S[order[t]];
            K.minunit = 0.0;
        } else {
            K.nviol = -1;
            K.var = NONE;
            K.maxviol = 0.0;
            K.minunit = 0.0;
        }
        keys[t] = K;
    }
}

// out[t] = keys[t].var (sorted variables) or src[keys[t].var] (permuted
// positions).
__global__ void k_rd_from_keys(const ScKey *keys, int64_t R, const int32_t *src, int32_t *out) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < R;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = src ? src[keys[t].var] : keys[t].var;
}

// Candidate value of a variable for draw u in the box [l, hi]: with x
// clamped into the box and f = x - floor(x), random rounding (up when
// u < f) for 0.25 < f < 0.75, else the nearest integer.
__device__ __forceinline__ double rd_value(double x, double l, double hi, double u) {
    const double xc = x < l ? l : (x > hi ? hi : x);
    const double fl = floor(xc);
    const double f = xc - fl;
    double v;
    if (f > 0.25 && f < 0.75) v = u < f ? fl + 1.0 : fl;
    else v = f < 0.5 ? fl : fl + 1.0;
    return v < l ? l : (v > hi ? hi : v);
}

// Probing cache of binaries: probe 2t + v fixed vars[t] to v.
struct RdCache {
    int32_t k;
    const int32_t *pos;    // [n] t of a cached variable, -1
    const int8_t *status;  // [2k]
    const int64_t *off;    // [2k + 1]
    const int32_t *var;
    const double *lb, *ub;
};

__device__ __forceinline__ int64_t rd_probe(const RdCache &C, int32_t j, double v) {
    if (C.k == 0) return -1;
    const int32_t t = C.pos[j];
    if (t < 0 || !(v == 0.0 || v == 1.0)) return -1;
    return 2 * (int64_t)t + (int64_t)v;
}

// Per member t and bulk h: the value, kept unless its cached probe is
// infeasible; the member map mpos[j] = t; the members' boxes reset to the
// current bounds.  mbox[h][t] holds order-preserving keys.
__global__ void k_rd_values(const int32_t *order, int64_t bulk, const double *x, const double *draws,
                            const double *lb, const double *ub, RdCache C, double *val,
                            uint8_t *keep, int32_t *mpos, longlong2 *mbox) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < bulk;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = order[t];
        mpos[j] = (int32_t)t;
        for (int h = 0; h < 2; ++h) {
            const double v = rd_value(x[j], lb[j], ub[j], draws[2 * (int64_t)j + h]);
            val[h * bulk + t] = v;
            const int64_t p = rd_probe(C, j, v);
            keep[h * bulk + t] = (p >= 0 && C.status[p] == 1) ? 0 : 1;
            mbox[h * bulk + t] = make_longlong2(dkey(lb[j]), dkey(ub[j]));
        }
    }
}

// The cached lists of the kept members narrow the boxes of the members they
// mention (one lane per member and bulk, walking its list).
__global__ void k_rd_member_boxes(const int32_t *order, int64_t bulk, RdCache C, const double *val,
                                  const uint8_t *keep, const int32_t *mpos, longlong2 *mbox) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < 2 * bulk;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int h = (int)(g / bulk);
        const int64_t t = g - h * bulk;
        if (!keep[g]) continue;
        const int64_t p = rd_probe(C, order[t], val[g]);
        if (p < 0) continue;
        for (int64_t e = C.off[p]; e < C.off[p + 1]; ++e) {
            const int32_t i = C.var[e];
            const int32_t ti = mpos[i];
            if (ti < 0) continue;
            longlong2 *b = &mbox[h * bulk + ti];
            atomicMax(&b->x, dkey(C.lb[e]));
            atomicMin(&b->y, dkey(C.ub[e]));
        }
    }
}

// A member whose value lies outside its narrowed box is dropped; the member
// map is cleared; kept members are counted per bulk.
__global__ void k_rd_member_check(const int32_t *order, int64_t bulk, const double *val,
                                  uint8_t *keep, int32_t *mpos, const longlong2 *mbox,
                                  int32_t *kept) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < bulk;
         t += (int64_t)gridDim.x * blockDim.x) {
        for (int h = 0; h < 2; ++h) {
            const int64_t g = h * bulk + t;
            const double v = val[g];
            const longlong2 b = mbox[g];
            if (keep[g] && !(dunkey(b.x) <= v && v <= dunkey(b.y))) keep[g] = 0;
            if (keep[g]) atomicAdd(&kept[h], 1);
        }
        mpos[order[t]] = -1;
    }
}

// Warm starts: both vectors start as the current box (as keys).
__global__ void k_rd_warm_init(const double *lb, const double *ub, int64_t n, longlong2 *vk) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const longlong2 k = make_longlong2(dkey(lb[i]), dkey(ub[i]));
        vk[i] = k;
        vk[n + i] = k;
    }
}

// The kept members' cached implications into the warm starts.
__global__ void k_rd_warm_implied(const int32_t *order, int64_t bulk, RdCache C, const double *val,
                                  const uint8_t *keep, int64_t n, longlong2 *vk) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < 2 * bulk;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int h = (int)(g / bulk);
        const int64_t t = g - h * bulk;
        if (!keep[g]) continue;
        const int64_t p = rd_probe(C, order[t], val[g]);
        if (p < 0) continue;
        for (int64_t e = C.off[p]; e < C.off[p + 1]; ++e) {
            longlong2 *b = &vk[h * n + C.var[e]];
            atomicMax(&b->x, dkey(C.lb[e]));
            atomicMin(&b->y, dkey(C.ub[e]));
        }
    }
}

// The kept members' fixings (after every implication).
__global__ void k_rd_warm_fix(const int32_t *order, int64_t bulk, const double *val,
                              const uint8_t *keep, int64_t n, longlong2 *vk) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < 2 * bulk;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int h = (int)(g / bulk);
        const int64_t t = g - h * bulk;
        if (!keep[g]) continue;
        const long long k = dkey(val[g]);
        vk[h * n + order[t]] = make_longlong2(k, k);
    }
}

// Warm starts out as bound vectors [2][n]; flags of the variables whose box
// moved (vector h at [h * n + i]).
__global__ void k_rd_warm_out(const longlong2 *vk, const double *lb, const double *ub, int64_t n,
                              double *vl, double *vu, uint8_t *flags) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < 2 * n;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g < n ? g : g - n;
        const longlong2 k = vk[g];
        const double l = dunkey(k.x), u = dunkey(k.y);
        vl[g] = l;
        vu[g] = u;
        flags[g] = (l != lb[i] || u != ub[i]) ? 1 : 0;
    }
}

// On a path marked infeasible: the members fixed to their first values.
__global__ void k_rd_fix_first(const int32_t *order, int64_t bulk, const double *val, double *lb,
                               double *ub) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < bulk;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = order[t];
        lb[j] = val[t];
        ub[j] = val[t];
    }
}

// Input checks: NaN in x or the box, a draw outside [0, 1), a cached
// variable out of range.
__global__ void k_rd_check(const double *x, const double *draws, const double *lb, const double *ub,
                           int64_t n, const int32_t *cvars, int32_t k, const int64_t *coff,
                           int32_t *bad) {
    const int64_t N = max(2 * n, 2 * (int64_t)k + 1);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < 2 * n && !(draws[i] >= 0.0 && draws[i] < 1.0)) atomicOr(bad, 1);
        if (i < n && (isnan(x[i]) || isnan(lb[i]) || isnan(ub[i]))) atomicOr(bad, 1);
        if (i < k && (cvars[i] < 0 || cvars[i] >= n)) atomicOr(bad, 1);
        // cache offsets: start at 0, never decrease
        if (k > 0 && i == 0 && coff[0] != 0) atomicOr(bad, 1);
        if (k > 0 && i < 2 * (int64_t)k && coff[i + 1] < coff[i]) atomicOr(bad, 1);
    }
}

// Cache lookup: the last listed position of each cached variable.
__global__ void k_rd_cache_pos(const int32_t *cvars, int32_t k, int32_t *pos) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < k;
         t += (int64_t)gridDim.x * blockDim.x)
        atomicMax(&pos[cvars[t]], (int32_t)t);
}

// Flags: integer variables fixed (lb == ub).
__global__ void k_rd_flag_fixed(const uint8_t *vtype, const double *lb, const double *ub, int64_t n,
                                uint8_t *flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = (vtype[i] != 0 && lb[i] == ub[i]) ? 1 : 0;
}

}  // namespace bp
