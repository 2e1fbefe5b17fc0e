"""The carry-save accumulator of the incremental heavy-row activities
(paper_2510_20499_amd/csrc/bp_carry.h), compiled for the host: sums of
doubles placed piece by piece into its limbs -- added, and added then taken
out again, in shuffled order -- must round to the correctly rounded exact
sum, which Python computes with rationals.  Covers cancellation, subnormal
terms, ties and sums that overflow."""
import math
import os
import random
import shutil
import struct
import subprocess
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_20499_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HARNESS = r"""
#include "bp_carry.h"
#include <cstdio>
#include <cstring>
// stdin: cases of "n" then n lines "bits sign" (sign 1: take the term out);
// stdout: the rounded sum's bits per case.
int main() {
    int n;
    while (scanf("%d", &n) == 1) {
        long long L[bp::HL];
        memset(L, 0, sizeof(L));
        for (int i = 0; i < n; ++i) {
            unsigned long long bits;
            int neg;
            if (scanf("%llx %d", &bits, &neg) != 2) return 2;
            double x;
            memcpy(&x, &bits, 8);
            if (x == 0.0) continue;
            int d;
            long long q0, q1, q2;
            bp::carry_pieces(x, neg != 0, d, q0, q1, q2);
            L[d] += q0;
            L[d + 1] += q1;
            L[d + 2] += q2;
        }
        int lo = bp::HL, hi = -1;
        for (int j = 0; j < bp::HL; ++j)
            if (L[j]) {
                if (j < lo) lo = j;
                hi = j;
            }
        double r = bp::carry_round(L, lo, hi);
        unsigned long long rb;
        memcpy(&rb, &r, 8);
        printf("%016llx\n", rb);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("carry")
    src = d / "harness.cpp"
    src.write_text(HARNESS)
    exe = d / "harness"
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-ffp-contract=off",
                    "-I" + CSRC, str(src), "-o", str(exe)], check=True, capture_output=True)
    return str(exe)


def _bits(x):
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def _exact(terms):
    """Correctly rounded value of the exact sum (inf on overflow)."""
    s = sum((Fraction(x) * (-1 if neg else 1) for x, neg in terms), Fraction(0))
    if s == 0:
        return 0.0
    try:
        return float(s)
    except OverflowError:
        return math.inf if s > 0 else -math.inf


def _cases(seed, count):
    rng = random.Random(seed)
    out = []
    for t in range(count):
        mode = t % 6
        n = rng.randint(1, 40)
        xs = []
        for i in range(n):
            if mode == 0:
                e = rng.randint(-1000, 1000)
            elif mode == 1:
                e = rng.randint(-30, 30)
            elif mode == 2:
                e = rng.randint(-1074, 0)
            elif mode == 3:
                e = rng.randint(0, 8)
            elif mode == 4:
                e = rng.randint(1000, 1023)
            else:
                e = rng.randint(-60, 60)
            x = math.ldexp(rng.uniform(-1.0, 1.0), e)
            if mode in (1, 3, 5) and xs and rng.random() < 0.35:
                x = -xs[rng.randrange(len(xs))]  # cancellation
            if mode == 5 and rng.random() < 0.2:
                x = math.ldexp(1.0, rng.randint(-60, 60))  # powers of two: ties
            xs.append(x)
        terms = [(x, False) for x in xs]
        # terms added and taken out again leave the sum unchanged
        for _ in range(rng.randint(0, 4)):
            y = math.ldexp(rng.uniform(-1.0, 1.0), rng.randint(-200, 200))
            terms += [(y, False), (y, True)]
        rng.shuffle(terms)
        out.append(terms)
    # fixed cases: a zero sum, the smallest subnormal, a tie to even, overflow
    out.append([(1.0, False), (1.0, True)])
    out.append([(math.ldexp(1.0, -1074), False)])
    out.append([(1.0, False), (math.ldexp(1.0, -53), False)])
    out.append([(1.0, False), (math.ldexp(1.0, -53), False), (math.ldexp(1.0, -105), False)])
    out.append([(1.7976931348623157e308, False), (1.7976931348623157e308, False)])
    out.append([(-1.7976931348623157e308, False), (-1.7976931348623157e308, False)])
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_carry_save_sums_round_like_exact_sums(harness, seed):
    cases = _cases(seed, 3000)
    lines = []
    for terms in cases:
        lines.append(str(len(terms)))
        lines += ["%016x %d" % (_bits(x), 1 if neg else 0) for x, neg in terms]
    out = subprocess.run([harness], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split()
    assert len(out) == len(cases)
    bad = [(i, out[i], "%016x" % _bits(_exact(t))) for i, t in enumerate(cases)
           if int(out[i], 16) != _bits(_exact(t))]
    assert not bad, bad[:5]
