/* The oracle's C core under the host sanitizers (AddressSanitizer and
 * UndefinedBehaviorSanitizer, built by tests/test_native_sanitizers.py):
 * plan, compress (global and windowed), decompress, histogram, length-
 * limited Huffman lengths and canonical codes on small fields of many
 * shapes, with every buffer sized exactly, and the reconstruction checked
 * against the bound.  Exit status 0 when every check holds. */
#include "szo.c"

#include <stdio.h>

static uint64_t rng = 88172645463325252ull;
static uint64_t next(void) { rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17; return rng; }
static double unif(void) { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }

static int one(uint32_t ndim, const uint64_t *n, double eb, int mode, int spl, uint32_t R)
{
    szo_params p;
    szo_config cfg;
    uint64_t N = 1, na, nout = 0, i;
    float *x, *anch, *recon, *oval, *out;
    uint16_t *codes;
    uint32_t *oidx, *h, *code, d;
    uint8_t *len, *cls;
    double tol;
    int rc, bad = 0;
    memset(&p, 0, sizeof p);
    p.ndim = ndim;
    p.S = ndim == 3 ? 8 : 16;
    for (d = 0; d < ndim; ++d) {
        p.n[d] = n[d];
        p.w[d] = d == 0 ? 4 * p.S : p.S;
        p.interp[d] = spl;
        p.order[d] = -1;
        N *= n[d];
    }
    p.R = R;
    p.eb_mode = mode;
    p.eb = eb;
    x = (float *)malloc(N * sizeof(float));
    for (i = 0; i < N; ++i) x[i] = (float)(10.0 * sin(0.01 * (double)i) + unif());
    rc = szo_plan(x, &p, &cfg);
    if (rc) { printf("plan rc %d\n", rc); free(x); return 1; }
    na = szo_num_anchors(&p);
    anch = (float *)malloc((na ? na : 1) * sizeof(float));
    codes = (uint16_t *)malloc(N * sizeof(uint16_t));
    recon = (float *)malloc(N * sizeof(float));
    oidx = (uint32_t *)malloc(N * sizeof(uint32_t));
    oval = (float *)malloc(N * sizeof(float));
    cls = (uint8_t *)malloc(N);
    out = (float *)malloc(N * sizeof(float));
    rc = szo_compress(x, &p, &cfg, anch, codes, recon, oidx, oval, &nout, cls);
    if (rc) { printf("compress rc %d\n", rc); bad = 1; }
    if (!rc) rc = szo_decompress(&p, &cfg, anch, codes, oidx, oval, nout, out);
    if (rc) { printf("decompress rc %d\n", rc); bad = 1; }
    tol = cfg.e;
    for (i = 0; !bad && i < N; ++i)
        if (out[i] != recon[i] || fabs((double)out[i] - (double)x[i]) > tol) {
            printf("point %llu: %g vs %g (recon %g, bound %g)\n", (unsigned long long)i,
                   (double)out[i], (double)x[i], (double)recon[i], tol);
            bad = 1;
        }
    if (!bad) {
        rc = szo_compress_windowed(x, &p, &cfg, codes, recon);
        if (rc) { printf("windowed rc %d\n", rc); bad = 1; }
    }
    h = (uint32_t *)calloc(2 * R, sizeof(uint32_t));
    len = (uint8_t *)malloc(2 * R);
    code = (uint32_t *)malloc(2 * R * sizeof(uint32_t));
    szo_histogram(codes, N, 2 * R, h);
    if (szo_huffman_lengths(h, 2 * R, 24, len) < 0) { printf("huffman failed\n"); bad = 1; }
    else szo_canonical_codes(len, 2 * R, code);
    free(x); free(anch); free(codes); free(recon); free(oidx); free(oval); free(cls); free(out);
    free(h); free(len); free(code);
    return bad;
}

int main(void)
{
    int fails = 0, cases = 0, t;
    for (t = 0; t < 40; ++t) {
        uint32_t ndim = 2 + (uint32_t)(next() % 2), d;
        uint64_t n[3];
        static const double ebs[] = {1e-1, 1e-2, 1e-3, 1e-5, 0.0};
        static const uint32_t Rs[] = {2, 3, 16, 512, 1024};
        for (d = 0; d < ndim; ++d) n[d] = 1 + next() % (ndim == 3 ? 40 : 150);
        fails += one(ndim, n, ebs[next() % 5], (int)(next() % 2), (int)(next() % 4), Rs[next() % 5]);
        ++cases;
    }
    printf("%d cases, %d failed\n", cases, fails);
    return fails != 0;
}
