// bp_sum.h -- order-independent row activities on gfx950.
//
// A row activity (the paper's Section 2.1, first display) is defined here as
// the correctly rounded exact sum of the rounded terms fl(a*b).  That value
// does not depend on the order of summation, so every schedule (one lane,
// a sub-wave, a workgroup, several workgroups) returns the same bits.
//
// Fast path: each lane keeps (s, c, e, ninf).  Adding a term x uses two
// error-free two-sums: s + x = s' + t exactly, c + t = c' + f exactly, and
// only |f| is dropped into the bound e.  Merging two states works the same
// way.  At the end the exact sum lies within e*(1+2^-20) of s + c, and the
// result fl(s + c) is certified when s + c is exact (e == 0) or when it is
// further than that bound from the rounding boundaries around fl(s + c).
//
// Slow path (uncertified rows only): one lane adds the row's terms into a
// 2176-bit two's-complement fixed-point accumulator with unit 2^-1074 (the
// smallest subnormal), which holds any sum of up to 2^31 doubles exactly,
// and rounds it to nearest-even once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bp {

struct Acc {
    double s, c, e;
    int ninf;
};

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &t) {
    s = a + b;
    double bb = s - a;
    t = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void acc_zero(Acc &A) {
    A.s = 0.0;
    A.c = 0.0;
    A.e = 0.0;
    A.ninf = 0;
}

__device__ __forceinline__ void acc_add(Acc &A, double x) {
    double s, t, c, f;
    two_sum(A.s, x, s, t);
    two_sum(A.c, t, c, f);
    A.s = s;
    A.c = c;
    A.e += fabs(f);
}

__device__ __forceinline__ void acc_merge(Acc &A, double bs, double bc, double be, int bn) {
    double s, t, c1, f1, c, f2;
    two_sum(A.s, bs, s, t);
    two_sum(A.c, bc, c1, f1);
    two_sum(c1, t, c, f2);
    A.s = s;
    A.c = c;
    A.e = ((A.e + be) + fabs(f1)) + fabs(f2);
    A.ninf += bn;
}

// Butterfly reduction across groups of G lanes (G a power of two <= 64).
// Every lane of a group ends with the same state.
template <int G>
__device__ __forceinline__ void acc_group_reduce(Acc &A) {
#pragma unroll
    for (int w = 1; w < G; w <<= 1) {
        double bs = __shfl_xor(A.s, w, 64);
        double bc = __shfl_xor(A.c, w, 64);
        double be = __shfl_xor(A.e, w, 64);
        int bn = __shfl_xor(A.ninf, w, 64);
        // Merge in lane order so both partners compute identical bits.
        bool lower = (__lane_id() & w) == 0;
        Acc X;
        if (lower) {
            X = A;
            acc_merge(X, bs, bc, be, bn);
        } else {
            X.s = bs; X.c = bc; X.e = be; X.ninf = bn;
            acc_merge(X, A.s, A.c, A.e, A.ninf);
        }
        A = X;
    }
}

__device__ __forceinline__ double canon0(double x) { return x == 0.0 ? 0.0 : x; }

// Certified rounding of the fast-path state; false if the state cannot
// decide the correctly rounded value.
__device__ __forceinline__ bool acc_certify(const Acc &A, double &out) {
    double r, d;
    two_sum(A.s, A.c, r, d);
    if (A.e == 0.0) {
        out = canon0(r);
        return true;
    }
    double ar = fabs(r);
    if (!(ar < __builtin_inf())) return false;
    uint64_t b = (uint64_t)__double_as_longlong(ar);
    double up = __longlong_as_double((long long)(b + 1)) - ar;
    double dn = b == 0 ? up : ar - __longlong_as_double((long long)(b - 1));
    double h = 0.5 * fmin(up, dn);
    double margin = (fabs(d) + A.e * (1.0 + 0x1p-20)) * (1.0 + 0x1p-50);
    if (margin < h) {
        out = canon0(r);
        return true;
    }
    return false;
}

// ------------------------------------------------------------------------
// Exact fixed-point accumulator (slow path).
// ------------------------------------------------------------------------
constexpr int SA_WORDS = 34;

struct SuperAcc {
    uint64_t w[SA_WORDS];
};

__device__ __noinline__ void sa_zero(SuperAcc &S) {
#pragma unroll 1
    for (int i = 0; i < SA_WORDS; ++i) S.w[i] = 0;
}

__device__ __noinline__ void sa_add(SuperAcc &S, double x) {
    if (x == 0.0) return;
    uint64_t b = (uint64_t)__double_as_longlong(x);
    bool neg = (b >> 63) != 0;
    uint64_t be = (b >> 52) & 0x7FF;
    uint64_t mant = b & ((1ull << 52) - 1);
    int pos;
    if (be == 0) {
        pos = 0;
    } else {
        mant |= (1ull << 52);
        pos = (int)be - 1;
    }
    int wi = pos >> 6, sh = pos & 63;
    uint64_t lo = mant << sh;
    uint64_t hi = sh ? (mant >> (64 - sh)) : 0;
    if (!neg) {
        uint64_t o = S.w[wi];
        S.w[wi] = o + lo;
        uint64_t carry = S.w[wi] < o ? 1 : 0;
        int j = wi + 1;
        uint64_t add = hi;
        while (j < SA_WORDS && (add | carry)) {
            uint64_t o2 = S.w[j];
            uint64_t t = o2 + add;
            uint64_t c1 = t < o2 ? 1 : 0;
            uint64_t t2 = t + carry;
            uint64_t c2 = t2 < t ? 1 : 0;
            S.w[j] = t2;
            carry = c1 | c2;
            add = 0;
            ++j;
        }
    } else {
        uint64_t o = S.w[wi];
        S.w[wi] = o - lo;
        uint64_t borrow = o < lo ? 1 : 0;
        int j = wi + 1;
        uint64_t sub = hi;
        while (j < SA_WORDS && (sub | borrow)) {
            uint64_t o2 = S.w[j];
            uint64_t t = o2 - sub;
            uint64_t b1 = o2 < sub ? 1 : 0;
            uint64_t t2 = t - borrow;
            uint64_t b2 = t < borrow ? 1 : 0;
            S.w[j] = t2;
            borrow = b1 | b2;
            sub = 0;
            ++j;
        }
    }
}

__device__ inline bool sa_is_zero(const SuperAcc &S) {
    uint64_t x = 0;
#pragma unroll 1
    for (int i = 0; i < SA_WORDS; ++i) x |= S.w[i];
    return x == 0;
}

// Bits [lo, lo+cnt) of the magnitude (cnt <= 64), lo may be negative.
__device__ inline uint64_t sa_bits(const SuperAcc &S, int lo, int cnt) {
    uint64_t r = 0;
    for (int k = 0; k < cnt; ++k) {
        int p = lo + k;
        if (p < 0) continue;
        uint64_t bit = (S.w[p >> 6] >> (p & 63)) & 1ull;
        r |= bit << k;
    }
    return r;
}

__device__ inline bool sa_any_below(const SuperAcc &S, int lim) {
    if (lim <= 0) return false;
    int full = lim >> 6;
    for (int i = 0; i < full; ++i)
        if (S.w[i]) return true;
    int rem = lim & 63;
    if (rem && (S.w[full] & ((1ull << rem) - 1))) return true;
    return false;
}

// Correctly rounded value of the accumulator.  Destroys the state: a
// negative accumulator is negated in place.
__device__ __noinline__ double sa_round(SuperAcc &S) {
    bool neg = (S.w[SA_WORDS - 1] >> 63) != 0;
    if (neg) {  // magnitude = two's complement negation
        uint64_t carry = 1;
        for (int i = 0; i < SA_WORDS; ++i) {
            uint64_t v = ~S.w[i];
            uint64_t t = v + carry;
            carry = (t < v) ? 1 : 0;
            S.w[i] = t;
        }
    }
    int top = -1;
    for (int i = SA_WORDS - 1; i >= 0; --i) {
        if (S.w[i]) {
            top = i * 64 + 63 - __clzll((long long)S.w[i]);
            break;
        }
    }
    if (top < 0) return 0.0;
    double mag;
    if (top <= 52) {
        mag = ldexp((double)S.w[0], -1074);
    } else {
        uint64_t M = sa_bits(S, top - 52, 53);
        uint64_t guard = sa_bits(S, top - 53, 1);
        bool sticky = sa_any_below(S, top - 53);
        int e = top - 52 - 1074;
        if (guard && (sticky || (M & 1ull))) {
            M += 1;
            if (M == (1ull << 53)) {
                M >>= 1;
                e += 1;
            }
        }
        if (e > 971) mag = __builtin_inf();
        else mag = ldexp((double)M, e);
    }
    return neg ? -mag : mag;
}

}  // namespace bp
