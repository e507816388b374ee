"""The kernels form every quotient by a projected depth p2 from one
correctly rounded reciprocal y = RN(1/p2): q = RN(a y), rem = fma(-p2, q, a),
result = fma(rem, y, q), which by Markstein's theorem equals the correctly
rounded a / p2.  This CPU check runs the same float32 sequence (C, libm's
fmaf, no contraction) over every significand of the divisor against IEEE
division, with dividends of both signs, so the bit-exact key maps do not
rest on the GPU tests alone.

The reciprocal itself comes from the hardware estimate (documented within
one ulp of 1/p2) and one Newton step y0 + y0 (1 - p2 y0) in fused
multiply-adds, with the low bit set where the significand of p2 is all ones.
The second test runs that step from every float within one ulp of 1/p2, for
every significand of three binades, and requires RN(1/p2) every time."""
import os
import subprocess

import pytest

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (uint32_t)st; }
int main(void) {
    unsigned long long bad = 0, n = 0;
    for (uint32_t mb = 0; mb < (1u << 23); ++mb) {
        /* divisors over [1, 2) and, scaled, the range of projected depths */
        const float b = u2f(((127u + (mb & 7u) - 3u) << 23) | mb);
        volatile float one = 1.0f;
        const float y = one / b;
        for (int k = 0; k < 6; ++k) {
            /* dividends: image coordinates times depth, up to ~2^20 */
            float a = u2f(((118u + rnd() % 24u) << 23) | (rnd() & 0x7FFFFFu));
            if (k & 1) a = -a;
            const float q = a * y;
            const float rem = fmaf(-b, q, a);
            const float got = fmaf(rem, y, q);
            volatile float want = a / b;
            ++n;
            if (f2u(got) != f2u(want)) ++bad;
        }
    }
    printf("%llu %llu\n", n, bad);
    return bad != 0;
}
"""


def test_quotient_from_reciprocal_is_correctly_rounded(tmp_path):
    c = tmp_path / "q.c"
    c.write_text(SRC)
    exe = tmp_path / "q"
    try:
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", str(c), "-o", str(exe), "-lm"],
                       check=True, capture_output=True)
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"no C compiler: {e}")
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    n, bad = map(int, res.stdout.split())
    assert n == 6 * (1 << 23) and bad == 0


RCP_SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
int main(void) {
    unsigned long long n = 0, bad = 0;
    for (int e = -8; e <= 8; e += 8)
        for (uint32_t m = 0; m < (1u << 23); ++m) {
            const float b = u2f(((uint32_t)(127 + e) << 23) | m);
            volatile float one = 1.0f;
            const float want = one / b;
            const long double exact = 1.0L / (long double)b;
            const long double ulp = ldexpl(1.0L, ilogbl(exact) - 23);
            for (int d = -2; d <= 2; ++d) {
                const float y0 = u2f(f2u(want) + (uint32_t)d);
                if (fabsl((long double)y0 - exact) > ulp) continue;   /* the estimate's bound */
                const float y1 = fmaf(fmaf(-b, y0, 1.0f), y0, y0);
                const uint32_t ones = ((f2u(b) & 0x7FFFFFu) + 1u) >> 23;
                const float y = u2f(f2u(y1) | ones);
                ++n;
                if (f2u(y) != f2u(want)) ++bad;
            }
        }
    printf("%llu %llu\n", n, bad);
    return bad != 0;
}
"""


def test_reciprocal_from_estimate_is_correctly_rounded(tmp_path):
    c = tmp_path / "r.c"
    c.write_text(RCP_SRC)
    exe = tmp_path / "r"
    try:
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", str(c), "-o", str(exe), "-lm"],
                       check=True, capture_output=True)
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"no C compiler: {e}")
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    n, bad = map(int, res.stdout.split())
    assert n >= 3 * (1 << 23) and bad == 0
