/* Host check of the division used by the red-black relaxation kernels for
 * diagonals held over many passes: with y = RN(1/d) (one correctly rounded
 * division per cell) the quotient is formed as q0 = RN(a y),
 * r = -RN(q0 d - a) (exact under a fused multiply-add), q = RN(q0 + r y).
 * By Markstein's theorem q equals RN(a / d) outside the subnormal range; this
 * program compares both bit for bit on random pairs in FP64 and FP32: small
 * integer diagonals (the finest level's 1..12), multiples of 1/8, random
 * values over wide ranges, signed and zero numerators.  Prints the mismatch
 * counts and exits non-zero if any. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint64_t nx(void) {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
}
static double mant64(void) { /* [1, 2) */
    uint64_t b = 0x3FF0000000000000ull | (nx() >> 12);
    double v;
    memcpy(&v, &b, 8);
    return v;
}
static float mant32(void) {
    uint32_t b = 0x3F800000u | (uint32_t)(nx() >> 41);
    float v;
    memcpy(&v, &b, 4);
    return v;
}

static long check64(long n) {
    long bad = 0;
    for (long i = 0; i < n; i++) {
        double d;
        switch (nx() % 4) {
            case 0: d = (double)(1 + nx() % 12); break;
            case 1: d = (double)(1 + nx() % 96) * 0.125; break;
            case 2: d = ldexp(mant64(), (int)(nx() % 8)); break;
            default: d = ldexp(mant64(), (int)(nx() % 40) - 20); break;
        }
        double a = ldexp(mant64(), (int)(nx() % 200) - 100) * ((nx() & 1) ? -1.0 : 1.0);
        if ((nx() & 255) == 0) a = (nx() & 1) ? -0.0 : 0.0;
        const double y = 1.0 / d;
        const double q0 = a * y;
        const double r = -fma(q0, d, -a);
        const double q = fma(r, y, q0);
        const double ref = a / d;
        if (memcmp(&q, &ref, sizeof q) != 0) bad++;
    }
    return bad;
}

static long check32(long n) {
    long bad = 0;
    for (long i = 0; i < n; i++) {
        float d;
        switch (nx() % 4) {
            case 0: d = (float)(1 + nx() % 12); break;
            case 1: d = (float)(1 + nx() % 96) * 0.125f; break;
            case 2: d = ldexpf(mant32(), (int)(nx() % 8)); break;
            default: d = ldexpf(mant32(), (int)(nx() % 30) - 15); break;
        }
        float a = ldexpf(mant32(), (int)(nx() % 80) - 40) * ((nx() & 1) ? -1.0f : 1.0f);
        if ((nx() & 255) == 0) a = (nx() & 1) ? -0.0f : 0.0f;
        const float y = 1.0f / d;
        const float q0 = a * y;
        const float r = -fmaf(q0, d, -a);
        const float q = fmaf(r, y, q0);
        const float ref = a / d;
        if (memcmp(&q, &ref, sizeof q) != 0) bad++;
    }
    return bad;
}

int main(int argc, char **argv) {
    const long n = argc > 1 ? atol(argv[1]) : 2000000;
    const long b64 = check64(n), b32 = check32(n);
    printf("pairs %ld fp64 mismatches %ld fp32 mismatches %ld\n", n, b64, b32);
    return (b64 || b32) ? 1 : 0;
}
