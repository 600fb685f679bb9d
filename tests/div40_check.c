/* Check of the division used by the natural-cubic prediction on the GPU:
 * x / 40 as q0 = x * RN(1/40), r = fma(-q0, 40, x), q = fma(r, RN(1/40), q0)
 * (Brisebarre, Muller and Raina, IEEE Trans. Computers 53(8), 2004).
 * The claim: q equals the correctly rounded x / 40 (bit for bit) for every
 * float with 2^-123 <= |x| < inf.  The kernels take the plain division for
 * every other input.
 *
 *   div40_check          sampled: every exponent, 2^15 mantissas each, plus
 *                        the whole binade at the range limit
 *   div40_check --all    all 2^32 inputs
 *
 * Prints "violations N" (inputs inside the claimed range where q differs)
 * and "outside M" (mismatches below the range, which must be nonzero, or the
 * range limit is not the tight one).  Exit status 1 if N > 0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

static float from_bits(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t to_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

static unsigned long long violations, outside;

static void check(uint32_t u) {
    const float x = from_bits(u);
    if (isnan(x)) return;
    const volatile float d = 40.0f;
    const float ref = x / d;
    const float c = 0.025f;
    const float q0 = x * c;
    const float r = fmaf(-q0, 40.0f, x);
    const float q = fmaf(r, c, q0);
    if (to_bits(q) == to_bits(ref)) return;
    if (fabsf(x) >= 0x1p-123f && fabsf(x) < INFINITY) ++violations;
    else ++outside;
}

int main(int argc, char** argv) {
    if (argc > 1 && strcmp(argv[1], "--all") == 0) {
        for (uint64_t u = 0; u < (1ull << 32); ++u) check((uint32_t)u);
    } else {
        for (uint32_t sign = 0; sign < 2; ++sign)
            for (uint32_t e = 0; e < 256; ++e)
                for (uint32_t m = 0; m < (1u << 23); m += 1u << 8)
                    check(sign << 31 | e << 23 | m);
        /* the binades on both sides of the limit, in full */
        for (uint32_t e = 3; e <= 4; ++e)
            for (uint32_t m = 0; m < (1u << 23); ++m) check(e << 23 | m);
    }
    printf("violations %llu\noutside %llu\n", violations, outside);
    return violations != 0;
}
