// bp_carry.h -- carry-save form of the exact fixed-point accumulator used by
// the incremental heavy-row activities (part of bp_engine.hip's translation
// unit; also compiled for the host by a CPU test of the rounding).
//
// The exact accumulator is a 2176-bit two's complement integer in units of
// 2^-1074, wide enough for any sum of doubles.  Its carry-save form holds it
// as HL signed 64-bit limbs, limb j counting multiples of 2^(32 j - 1074).  A
// double is placed where the exact accumulator places it (its integer
// mantissa at bit `pos`) and split into three 32-bit pieces for consecutive
// limbs, so concurrent integer atomics build the exact sum in any order; one
// rounding at the end gives the correctly rounded sum.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

namespace bp {

constexpr int CARRY_WORDS = 34;          // 64-bit words of the 2176-bit accumulator
constexpr int HL = 2 * CARRY_WORDS;      // 32-bit limbs

// The three signed pieces of +-x and the limb of the first one (x finite and
// nonzero; an infinite product lands where the exact accumulator puts it).
__host__ __device__ inline void carry_pieces(double x, bool negate, int &d0, long long &q0, long long &q1,
                                             long long &q2) {
    uint64_t b;
    memcpy(&b, &x, sizeof(b));
    const bool neg = ((b >> 63) != 0) != negate;
    const uint64_t be = (b >> 52) & 0x7FF;
    uint64_t mant = b & ((1ull << 52) - 1);
    int pos = 0;
    if (be != 0) {
        mant |= 1ull << 52;
        pos = (int)be - 1;
    }
    d0 = pos >> 5;
    const int sh = pos & 31;
    const uint64_t lo = mant << sh;
    const uint64_t hi = sh ? (mant >> (64 - sh)) : 0ull;
    q0 = (long long)(lo & 0xffffffffull);
    q1 = (long long)(lo >> 32);
    q2 = (long long)hi;
    if (neg) {
        q0 = -q0;
        q1 = -q1;
        q2 = -q2;
    }
}

// Correctly rounded value of carry-save limbs (destroys them).  Only limbs
// [lo, hi] are nonzero (lo > hi: none): limbs below lo stay zero, and since
// every limb is below 2^62 in magnitude the carries settle within two limbs
// above hi, where the sign is read.  Carries are propagated digit by digit;
// a negative sum is negated; the 53 bits below the leading one, the next
// (guard) bit and whether any lower bit is set then give the
// round-to-nearest-even result, the value the exact accumulator rounds to.
// +0.0 for a zero sum.
__host__ __device__ inline double carry_round(long long *L, int lo, int hi) {
    if (lo > hi) return 0.0;
    const int last = hi + 2 < HL - 1 ? hi + 2 : HL - 1;
    long long carry = 0;
    for (int j = lo; j <= last; ++j) {
        const long long t = L[j] + carry;
        L[j] = t & 0xffffffffll;
        carry = t >> 32;
    }
    const bool neg = carry < 0;
    if (neg) {  // magnitude: the two's complement negation of the digits
        long long borrow = 0;
        for (int j = lo; j <= last; ++j) {
            const long long t = -L[j] - borrow;
            L[j] = t & 0xffffffffll;
            borrow = t < 0 ? 1 : 0;
        }
    }
    int T = last;
    while (T >= lo && L[T] == 0) --T;
    if (T < lo) return 0.0;
    const uint64_t dT = (uint64_t)L[T];
    const uint64_t d1 = T >= 1 ? (uint64_t)L[T - 1] : 0ull;
    const uint64_t d2 = T >= 2 ? (uint64_t)L[T - 2] : 0ull;
    const int b = 31 - __builtin_clz((unsigned)dT);  // leading bit within digit T
    const int top = 32 * T + b;                      // in units of 2^-1074
    double mag;
    if (top <= 52) {  // below 2^53 units: exact (digits 0 and 1 only)
        mag = ldexp((double)(T == 1 ? (dT << 32) | d1 : dT), -1074);
    } else {
        const uint64_t win = (d1 << 32) | d2;  // the two digits below digit T
        uint64_t M = (dT << (52 - b)) | (win >> (b + 12));
        const uint64_t guard = (win >> (b + 11)) & 1ull;
        bool sticky = (win & ((1ull << (b + 11)) - 1ull)) != 0ull;
        for (int j = T - 3; j >= lo && !sticky; --j) sticky = L[j] != 0;
        int e = top - 52 - 1074;
        if (guard && (sticky || (M & 1ull))) {
            M += 1;
            if (M == (1ull << 53)) {
                M >>= 1;
                e += 1;
            }
        }
        mag = e > 971 ? __builtin_inf() : ldexp((double)M, e);
    }
    const double r = neg ? -mag : mag;
    return r == 0.0 ? 0.0 : r;
}

}  // namespace bp
