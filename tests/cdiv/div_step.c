/* Checks, on the host, the division the tile sweep uses for a centroid:
 * for an integer count d in [1, 127] and y = 1/d correctly rounded,
 *     q = a*y;  r = fma(-q, d, a);  step = fma(r, y, q)
 * equals a/d correctly rounded whenever |a| >= 128 x the smallest normal
 * number (the kernel divides below that), in double and in float.  a runs
 * over random bit patterns of every exponent and over values whose quotient
 * sits next to a rounding boundary.  Prints: values checked with the step,
 * mismatches among them (0 expected), and mismatches below the bound (the
 * reason for the bound: subnormal quotients can be exact midpoints). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint64_t next(void)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main(int argc, char** argv)
{
    const long n = argc > 1 ? atol(argv[1]) : 200000;
    long stepped = 0, bad = 0, below_bad = 0;
    for (int d = 1; d <= 127; ++d) {
        const double yd = 1.0 / (double)d, dd = (double)d;
        const float yf = 1.0f / (float)d, df = (float)d;
        for (long k = 0; k < n; ++k) {
            double a;
            if (k % 4 == 3) {
                /* quotients beside midpoints: a = d * m + a few ulps */
                const double m = (double)(next() >> 11) * 0x1p-53 + 1.0;
                a = ldexp(dd * m + (double)((int)(next() % 5) - 2) * 0x1p-52, (int)(next() % 200) - 100);
            } else {
                uint64_t u = next();
                u &= ~(0x7FFull << 52);
                u |= (next() % 2046) << 52;   /* every finite exponent; subnormals when 0 */
                memcpy(&a, &u, 8);
                if (fabs(a) >= 0x1p1000) a = ldexp(a, -100);
            }
            {
                const double q = a * yd, r = fma(-q, dd, a), got = fma(r, yd, q), want = a / dd;
                const int differ = memcmp(&got, &want, 8) != 0;
                if (fabs(a) >= 0x1p-1015) { ++stepped; bad += differ; }
                else below_bad += differ;
            }
            const float af = (float)a;
            if (isfinite(af)) {
                const float qf = af * yf, rf = fmaf(-qf, df, af), gf = fmaf(rf, yf, qf), wf = af / df;
                const int differ = memcmp(&gf, &wf, 4) != 0;
                if (fabsf(af) >= 0x1p-119f) { ++stepped; bad += differ; }
                else below_bad += differ;
            }
        }
    }
    printf("%ld %ld %ld\n", stepped, bad, below_bad);
    return 0;
}
