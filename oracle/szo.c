/*
 * szo.c -- plain, slow, scalar CPU oracle of the G-Interp error-bounded
 * compressor (cuSZ-i, arXiv 2312.05492).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with the
 * HIP implementation: every step below is written from the paper.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fPIC -shared
 *   (no -march, no FMA contraction, IEEE denormals) so that every FP32
 *   operation is one correctly rounded IEEE operation in the order written.
 *
 * Contents and the passage each part follows:
 *   szo_alpha            Eq. 1 (Sec. V-C.2, error-bound reduction factor)
 *   szo_plan             Sec. V-C.1 data profiling (value range, sampled
 *                        cubic-spline tests) and Sec. V-C.2 auto-tuning
 *                        (alpha, cubic per dimension, dimension order);
 *                        Sec. V-B.2 level-wise error bounds
 *   szo_stencil          Sec. V-B.1 spline formulas (linear, quadratic,
 *                        cubic not-a-knot, cubic natural)
 *   szo_compress         Sec. V-A (anchors on a stride-S lattice, levels
 *                        S/2..1, dimensions one after another), Sec. V-B.1
 *                        (stencil by available neighbours), Sec. III-A
 *                        (closed-loop quantisation, |q| >= R -> outlier),
 *                        Sec. V-D (windows of 4 basic blocks bound the
 *                        neighbour search)
 *   szo_compress_windowed  the same result computed window by window
 *                        (a second formulation, for an internal check)
 *   szo_decompress       Sec. V-B.1 (decompression replays the predictions)
 *   szo_histogram        Sec. VI-A (quant-code histogram)
 *   szo_huffman_lengths  Sec. VI-A (Huffman codebook built on the host)
 *   szo_canonical_codes, szo_encode, szo_decode
 *                        Sec. III-A / VI-A (coarse-grained chunked Huffman)
 *
 * Where the paper is silent the readings are the ones listed in the design
 * notes (quantiser rounding, outlier payload, level numbering, window rule,
 * profiling sample positions, codebook tie-breaks, bit order).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <float.h>

/* SZO_PLANT > 0 compiles one deliberate mistake into a separate test build
 * (never the oracle's own library), so that tests can show the pins catch it:
 * 1 NAK outer taps with the wrong sign, 2 natural cubic with its outer term
 * dropped, 3 left quadratic reading x[n+3] for x[n-3], 4 quantiser truncating
 * instead of rounding, 5 bound rounded to nearest instead of down, 6 level
 * bounds shifted by one level, 7 canonical codes counting the wrong length,
 * 8 profiling keeping the cubic with the larger error, 9 smoothest dimension
 * first, 10 x[n+3] unavailable at the window's last point, 11 each code's
 * bits written least significant first, 12 Eq. 1 falling instead of rising
 * between 1e-3 and 1e-2, 13 relative bound scaled by the maximum instead of
 * the range. */
#ifndef SZO_PLANT
#define SZO_PLANT 0
#endif

#define SZO_OK 0
#define SZO_ERR_ARG (-1)
#define SZO_ERR_NONFINITE (-2)
#define SZO_ERR_OOM (-3)
#define SZO_ERR_CORRUPT (-5)

#define SZO_LIN 0
#define SZO_NAK 1
#define SZO_NAT 2
#define SZO_AUTO 3

/* stencil classes recorded for the spline map of Fig. spline-on-2D-slice */
#define SZO_CLS_NONE 0
#define SZO_CLS_ANCHOR 1
#define SZO_CLS_ONE 2      /* one neighbour: previous point */
#define SZO_CLS_LINEAR 3
#define SZO_CLS_QUAD 4
#define SZO_CLS_CUBIC 5

#define SZO_MAX_LEVELS 16

typedef struct {
    uint32_t ndim;      /* 1, 2 or 3 */
    uint32_t S;         /* anchor stride (power of two) */
    uint64_t n[3];      /* n[0] = x (fastest) .. n[ndim-1] slowest */
    uint32_t w[3];      /* window extent per dimension (multiple of S) */
    uint32_t R;         /* quant-code radius: codes 1..2R-1, 0 = outlier */
    int32_t eb_mode;    /* 0 absolute, 1 value-range relative */
    int32_t pad0;
    double eb;
    int32_t interp[3];  /* SZO_LIN/NAK/NAT/AUTO per dimension */
    int32_t order[3];   /* order[k] = dimension of the k-th pass; -1 = auto */
    double alpha;       /* <= 0: Eq. 1 */
} szo_params;

typedef struct {
    float vmin, vmax;
    double range;
    double eps;          /* value-range relative bound used in Eq. 1 */
    double e_abs;        /* absolute bound in FP64 */
    float e;             /* largest float <= e_abs */
    int32_t levels;      /* L = log2(S) */
    double alpha;
    float el[SZO_MAX_LEVELS];    /* e_l for l = 1..L at index l-1 */
    float ebx2[SZO_MAX_LEVELS];  /* 2*e_l */
    float inv[SZO_MAX_LEVELS];   /* 1/(2*e_l) */
    int32_t spline[3];   /* per dimension: SZO_LIN/NAK/NAT */
    int32_t order[3];
    double prof[3][3];   /* profiled L1 errors [dim][LIN,NAK,NAT] */
    int32_t profiled;
    int32_t pad1;
} szo_config;

/* ------------------------------------------------------------------ */
/* Eq. 1: alpha = A(eps), piecewise linear in the relative bound.      */
double szo_alpha(double eps)
{
    if (eps >= 1e-1) return 2.0;
    if (eps >= 1e-2) return 1.75 + 0.25 * (eps - 1e-2) / (1e-1 - 1e-2);
    if (eps >= 1e-3) return 1.5 + (SZO_PLANT == 12 ? -0.25 : 0.25) * (eps - 1e-3) / (1e-2 - 1e-3);
    if (eps >= 1e-4) return 1.25 + 0.25 * (eps - 1e-4) / (1e-3 - 1e-4);
    if (eps >= 1e-5) return 1.0 + 0.25 * (eps - 1e-5) / (1e-4 - 1e-5);
    return 1.0;
}

/* largest float that is <= v (v >= 0): the bound never grows in FP32 */
float szo_round_down(double v)
{
    float f;
    if (!(v > 0.0)) return 0.0f;
    if (v >= (double)FLT_MAX) return FLT_MAX;
    f = (float)v;
    if ((double)f > v && SZO_PLANT != 5) f = nextafterf(f, 0.0f);
    return f;
}

/* ------------------------------------------------------------------ */
/* Sec. V-B.1: the four splines.  kind selects the formula; a = x[n-3],
 * b = x[n-1], c = x[n+1], d = x[n+3].  Evaluated in FP32 exactly as
 * written, each operation rounded, no contraction. */
#define SZO_ST_ONE 0
#define SZO_ST_LINEAR 1
#define SZO_ST_QUAD_LEFT 2   /* uses x[n-3], x[n-1], x[n+1] */
#define SZO_ST_QUAD_RIGHT 3  /* uses x[n-1], x[n+1], x[n+3] */
#define SZO_ST_NAK 4
#define SZO_ST_NAT 5

float szo_stencil(int kind, float a, float b, float c, float d)
{
    switch (kind) {
    case SZO_ST_ONE:        return b;
    case SZO_ST_LINEAR:     return (b + c) * 0.5f;
    case SZO_ST_QUAD_LEFT:  return ((6.0f * b + 3.0f * c) - (SZO_PLANT == 3 ? d : a)) * 0.125f;
    case SZO_ST_QUAD_RIGHT: return ((3.0f * b + 6.0f * c) - d) * 0.125f;
    case SZO_ST_NAK:
        if (SZO_PLANT == 1) return (9.0f * (b + c) + (a + d)) * 0.0625f;
        return (9.0f * (b + c) - (a + d)) * 0.0625f;
    case SZO_ST_NAT:
        if (SZO_PLANT == 2) return (23.0f * (b + c)) / 40.0f;
        return (23.0f * (b + c) - 3.0f * (a + d)) / 40.0f;
    }
    return 0.0f;
}

static uint64_t lin(const uint64_t *n, uint64_t x, uint64_t y, uint64_t z)
{
    return x + n[0] * (y + n[1] * z);
}

static int is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

static int check_params(const szo_params *p)
{
    uint32_t d;
    if (p->ndim < 1 || p->ndim > 3) return SZO_ERR_ARG;
    if (!is_pow2(p->S) || p->S < 2) return SZO_ERR_ARG;
    if (p->R < 2 || p->R > 32768) return SZO_ERR_ARG;
    if (!(p->eb >= 0.0) || !isfinite(p->eb)) return SZO_ERR_ARG;
    for (d = 0; d < p->ndim; ++d) {
        if (p->n[d] == 0) return SZO_ERR_ARG;
        if (p->w[d] == 0 || p->w[d] % p->S) return SZO_ERR_ARG;
        if (p->interp[d] < 0 || p->interp[d] > 3) return SZO_ERR_ARG;
    }
    if (p->order[0] >= 0) {
        int seen[3] = {0, 0, 0};
        for (d = 0; d < p->ndim; ++d) {
            if (p->order[d] < 0 || p->order[d] >= (int)p->ndim) return SZO_ERR_ARG;
            if (seen[p->order[d]]++) return SZO_ERR_ARG;
        }
    }
    return SZO_OK;
}

/* three coordinates with unused dimensions set to extent 1 */
static void dims3(const szo_params *p, uint64_t *n)
{
    n[0] = p->n[0];
    n[1] = p->ndim >= 2 ? p->n[1] : 1;
    n[2] = p->ndim == 3 ? p->n[2] : 1;
}

/* ------------------------------------------------------------------ */
/* Sec. V-C.1 profiling and Sec. V-C.2 auto-tuning, Sec. V-B.2 level eb. */
static uint64_t sample_pos(uint64_t nd, int t)
{
    uint64_t v = ((uint64_t)(2 * t + 1) * nd) / 8;
    if (nd >= 7) {
        if (v < 3) v = 3;
        if (v > nd - 4) v = nd - 4;
    }
    return v;
}

int szo_plan(const float *x, const szo_params *p, szo_config *cfg)
{
    uint64_t n[3], N, i;
    uint32_t d, k;
    int rc = check_params(p), need_prof = 0;
    float vmin, vmax;
    if (rc) return rc;
    memset(cfg, 0, sizeof(*cfg));
    dims3(p, n);
    N = n[0] * n[1] * n[2];

    /* value range (exact FP32 comparisons); non-finite input rejected */
    vmin = x[0];
    vmax = x[0];
    for (i = 0; i < N; ++i) {
        if (!isfinite(x[i])) return SZO_ERR_NONFINITE;
        if (x[i] < vmin) vmin = x[i];
        if (x[i] > vmax) vmax = x[i];
    }
    cfg->vmin = vmin + 0.0f;   /* -0 and +0 are the same value */
    cfg->vmax = vmax + 0.0f;
    cfg->range = (double)cfg->vmax - (double)cfg->vmin;

    /* absolute and relative bound: one divided by the range is the other */
    if (p->eb_mode == 1) {
        cfg->eps = p->eb;
        cfg->e_abs = p->eb * (SZO_PLANT == 13 ? (double)cfg->vmax : cfg->range);
    } else {
        cfg->e_abs = p->eb;
        if (cfg->range > 0.0) cfg->eps = p->eb / cfg->range;
        else cfg->eps = p->eb > 0.0 ? INFINITY : 0.0;
    }
    cfg->e = szo_round_down(cfg->e_abs);
    cfg->alpha = p->alpha > 0.0 ? p->alpha : szo_alpha(cfg->eps);

    /* level-wise bound e_l = e / alpha^(l-1); l = 1 is stride 1 */
    cfg->levels = 0;
    for (k = p->S; k > 1; k >>= 1) cfg->levels++;
    {
        double apow = SZO_PLANT == 6 ? cfg->alpha : 1.0;
        int l;
        for (l = 1; l <= cfg->levels; ++l) {
            cfg->el[l - 1] = szo_round_down(cfg->e_abs / apow);
            cfg->ebx2[l - 1] = 2.0f * cfg->el[l - 1];
            cfg->inv[l - 1] = 1.0f / cfg->ebx2[l - 1];
            apow = apow * cfg->alpha;
        }
    }

    for (d = 0; d < p->ndim; ++d)
        if (p->interp[d] == SZO_AUTO) need_prof = 1;
    if (p->order[0] < 0) need_prof = 1;

    if (need_prof) {
        /* uniformly spaced 4^D sub-grid; each sample runs the cubic
         * splines (and linear) along every dimension on original values */
        uint64_t pos[3][4];
        int tz, ty, tx, nt[3];
        cfg->profiled = 1;
        for (d = 0; d < 3; ++d) {
            int t;
            nt[d] = (d < p->ndim) ? 4 : 1;
            for (t = 0; t < 4; ++t) pos[d][t] = d < p->ndim ? sample_pos(n[d], t) : 0;
        }
        for (tz = 0; tz < nt[2]; ++tz)
            for (ty = 0; ty < nt[1]; ++ty)
                for (tx = 0; tx < nt[0]; ++tx) {
                    uint64_t c[3];
                    c[0] = pos[0][tx];
                    c[1] = pos[1][ty];
                    c[2] = pos[2][tz];
                    for (d = 0; d < p->ndim; ++d) {
                        uint64_t cm3[3], cm1[3], cp1[3], cp3[3];
                        float a, b, cc, dd, v;
                        if (n[d] < 7) continue;
                        memcpy(cm3, c, sizeof c); memcpy(cm1, c, sizeof c);
                        memcpy(cp1, c, sizeof c); memcpy(cp3, c, sizeof c);
                        cm3[d] -= 3; cm1[d] -= 1; cp1[d] += 1; cp3[d] += 3;
                        a = x[lin(n, cm3[0], cm3[1], cm3[2])];
                        b = x[lin(n, cm1[0], cm1[1], cm1[2])];
                        cc = x[lin(n, cp1[0], cp1[1], cp1[2])];
                        dd = x[lin(n, cp3[0], cp3[1], cp3[2])];
                        v = x[lin(n, c[0], c[1], c[2])];
                        cfg->prof[d][0] += fabs((double)v - (double)szo_stencil(SZO_ST_LINEAR, a, b, cc, dd));
                        cfg->prof[d][1] += fabs((double)v - (double)szo_stencil(SZO_ST_NAK, a, b, cc, dd));
                        cfg->prof[d][2] += fabs((double)v - (double)szo_stencil(SZO_ST_NAT, a, b, cc, dd));
                    }
                }
    }

    /* per dimension: the cubic with the lower profiled error (ties: NAK) */
    {
        double score[3] = {0, 0, 0};
        for (d = 0; d < p->ndim; ++d) {
            int s = p->interp[d];
            if (s == SZO_AUTO)
                s = (SZO_PLANT == 8 ? cfg->prof[d][2] > cfg->prof[d][1]
                                    : cfg->prof[d][2] < cfg->prof[d][1]) ? SZO_NAT : SZO_NAK;
            cfg->spline[d] = s;
            score[d] = cfg->prof[d][s == SZO_LIN ? 0 : (s == SZO_NAK ? 1 : 2)];
        }
        if (p->order[0] >= 0) {
            for (d = 0; d < p->ndim; ++d) cfg->order[d] = p->order[d];
        } else {
            /* least smooth (largest error) first; ties: slower dim first.
             * plain selection: repeatedly take the best remaining dim */
            int used[3] = {0, 0, 0};
            for (k = 0; k < p->ndim; ++k) {
                int best = -1;
                int dd;
                for (dd = (int)p->ndim - 1; dd >= 0; --dd) {
                    if (used[dd]) continue;
                    if (best < 0 || (SZO_PLANT == 9 ? score[dd] < score[best]
                                                    : score[dd] > score[best])) best = dd;
                }
                used[best] = 1;
                cfg->order[k] = best;
            }
        }
    }
    return SZO_OK;
}

/* ------------------------------------------------------------------ */
/* Prediction of point c along dimension d at stride s (Sec. V-B.1), with
 * neighbours restricted to the window interval of c along d (Sec. V-D).
 * r is the array of reconstructed values.  Returns the prediction and
 * writes the stencil class. */
static float predict(const float *r, const uint64_t *n, const uint64_t *c, int d,
                     uint64_t s, uint64_t wd, int spline, int *cls)
{
    uint64_t lo = (c[d] / wd) * wd;
    uint64_t hi = lo + wd < n[d] - 1 ? lo + wd : n[d] - 1;
    int has_m3 = c[d] >= lo + 3 * s;
    int has_p1 = c[d] + s <= hi;
    int has_p3 = SZO_PLANT == 10 ? c[d] + 3 * s < hi : c[d] + 3 * s <= hi;
    uint64_t cc[3];
    uint64_t step;
    float a = 0.0f, b, cp = 0.0f, dp = 0.0f;

    step = (d == 0) ? 1 : (d == 1 ? n[0] : n[0] * n[1]);
    memcpy(cc, c, sizeof cc);
    {
        uint64_t i = lin(n, cc[0], cc[1], cc[2]);
        b = r[i - s * step];
        if (has_m3) a = r[i - 3 * s * step];
        if (has_p1) cp = r[i + s * step];
        if (has_p3) dp = r[i + 3 * s * step];
    }
    if (!has_p1) {
        *cls = SZO_CLS_ONE;
        return szo_stencil(SZO_ST_ONE, a, b, cp, dp);
    }
    if (spline == SZO_LIN || (!has_m3 && !has_p3)) {
        *cls = SZO_CLS_LINEAR;
        return szo_stencil(SZO_ST_LINEAR, a, b, cp, dp);
    }
    if (has_m3 && !has_p3) {
        *cls = SZO_CLS_QUAD;
        return szo_stencil(SZO_ST_QUAD_LEFT, a, b, cp, dp);
    }
    if (!has_m3 && has_p3) {
        *cls = SZO_CLS_QUAD;
        return szo_stencil(SZO_ST_QUAD_RIGHT, a, b, cp, dp);
    }
    *cls = SZO_CLS_CUBIC;
    return szo_stencil(spline == SZO_NAT ? SZO_ST_NAT : SZO_ST_NAK, a, b, cp, dp);
}

/* Sec. III-A closed-loop quantisation of one point.  Returns 1 for an
 * outlier.  q_out receives the quant-code q (not yet offset by R) and
 * xr_out the value the decompressor will reproduce. */
static int quantize(float xv, float p, float el, float ebx2, float inv, int32_t R,
                    int32_t *q_out, float *xr_out)
{
    float diff = xv - p;
    float qf, t, xr;
    int32_t q;
    if (el == 0.0f) {
        /* only exact predictions; the decompressor rebuilds p + 0 * 2e_l,
         * which is +0 where p is -0, so that is the value kept here */
        if (diff == 0.0f) { *q_out = 0; *xr_out = p + 0.0f * ebx2; return 0; }
        return 1;
    }
    qf = diff * inv;
    if (!(fabsf(qf) < (float)R)) return 1;
    q = SZO_PLANT == 4 ? (int32_t)qf : (int32_t)rintf(qf);   /* round half to even */
    if (q >= R || q <= -R) return 1;
    t = (float)q * ebx2;
    xr = p + t;
    if (!(fabs((double)xv - (double)xr) <= (double)el)) return 1;
    *q_out = q;
    *xr_out = xr;
    return 0;
}

/* the set of points visited by pass (s, k): along d = order[k] the odd
 * multiples of s; along dims already done at this level multiples of s;
 * along dims still to come multiples of 2s. */
static void pass_grid(const szo_config *cfg, int ndim, int k, uint64_t s,
                      uint64_t *start, uint64_t *step)
{
    int j;
    start[0] = start[1] = start[2] = 0;
    step[0] = step[1] = step[2] = 1;
    for (j = 0; j < ndim; ++j) {
        int dj = cfg->order[j];
        if (j < k) { start[dj] = 0; step[dj] = s; }
        else if (j == k) { start[dj] = s; step[dj] = 2 * s; }
        else { start[dj] = 0; step[dj] = 2 * s; }
    }
}

static int count_anchors(const szo_params *p, const uint64_t *n, uint64_t *na)
{
    uint32_t d;
    uint64_t tot = 1;
    for (d = 0; d < 3; ++d) {
        na[d] = d < p->ndim ? (n[d] + p->S - 1) / p->S : 1;
        tot *= na[d];
    }
    return (int)(tot > 0);
}

uint64_t szo_num_anchors(const szo_params *p)
{
    uint64_t n[3], na[3];
    dims3(p, n);
    count_anchors(p, n, na);
    return na[0] * na[1] * na[2];
}

/* Global formulation of the traversal (Sec. V-A): the whole field, pass by
 * pass.  Outputs: anchors (C-order lattice), codes (q + R; 0 = outlier; R at
 * anchors), recon (the reconstruction), outliers (index ascending,
 * original value), optional stencil class per point. */
int szo_compress(const float *x, const szo_params *p, const szo_config *cfg,
                 float *anchors, uint16_t *codes, float *recon,
                 uint32_t *oidx, float *oval, uint64_t *n_out, uint8_t *cls)
{
    uint64_t n[3], na[3], N, i, ax, ay, az;
    int rc = check_params(p);
    int lvl, k;
    uint8_t *is_out;
    const int32_t R = (int32_t)p->R;
    if (rc) return rc;
    dims3(p, n);
    N = n[0] * n[1] * n[2];
    if (N >= 0xFFFFFFFFull) return SZO_ERR_ARG;
    count_anchors(p, n, na);
    is_out = (uint8_t *)calloc(N, 1);
    if (!is_out) return SZO_ERR_OOM;
    memcpy(recon, x, N * sizeof(float));
    for (i = 0; i < N; ++i) codes[i] = 0;
    if (cls) memset(cls, SZO_CLS_NONE, N);

    /* anchors: every lattice point, stored losslessly */
    for (az = 0; az < na[2]; ++az)
        for (ay = 0; ay < na[1]; ++ay)
            for (ax = 0; ax < na[0]; ++ax) {
                uint64_t gi = lin(n, ax * p->S, ay * p->S, az * p->S);
                anchors[ax + na[0] * (ay + na[1] * az)] = x[gi];
                codes[gi] = (uint16_t)R;
                if (cls) cls[gi] = SZO_CLS_ANCHOR;
            }

    /* levels from stride S/2 down to 1, dimensions in the chosen order */
    for (lvl = cfg->levels; lvl >= 1; --lvl) {
        uint64_t s = (uint64_t)1 << (lvl - 1);
        for (k = 0; k < (int)p->ndim; ++k) {
            int d = cfg->order[k];
            uint64_t start[3], step[3], c[3];
            pass_grid(cfg, (int)p->ndim, k, s, start, step);
            for (c[2] = start[2]; c[2] < n[2]; c[2] += step[2])
                for (c[1] = start[1]; c[1] < n[1]; c[1] += step[1])
                    for (c[0] = start[0]; c[0] < n[0]; c[0] += step[0]) {
                        int cl;
                        int32_t q = 0;
                        float xr = 0.0f;
                        uint64_t gi = lin(n, c[0], c[1], c[2]);
                        float pr = predict(recon, n, c, d, s, p->w[d], cfg->spline[d], &cl);
                        if (cls) cls[gi] = (uint8_t)cl;
                        if (quantize(x[gi], pr, cfg->el[lvl - 1], cfg->ebx2[lvl - 1],
                                     cfg->inv[lvl - 1], R, &q, &xr)) {
                            codes[gi] = 0;
                            recon[gi] = x[gi];
                            is_out[gi] = 1;
                        } else {
                            codes[gi] = (uint16_t)(q + R);
                            recon[gi] = xr;
                        }
                    }
        }
    }

    /* outliers in ascending linear index (stream compaction) */
    {
        uint64_t m = 0;
        for (i = 0; i < N; ++i)
            if (is_out[i]) {
                oidx[m] = (uint32_t)i;
                oval[m] = x[i];
                ++m;
            }
        *n_out = m;
    }
    free(is_out);
    return SZO_OK;
}

/* Window-by-window formulation of the same result: each window copies its
 * block (its own points plus the far faces it borrows, clipped to the
 * field) and runs all passes on the block alone, then keeps the points it
 * owns.  Equality with szo_compress shows that windows are independent. */
int szo_compress_windowed(const float *x, const szo_params *p, const szo_config *cfg,
                          uint16_t *codes, float *recon)
{
    uint64_t n[3], nw[3], wi[3];
    uint32_t d;
    int rc = check_params(p);
    const int32_t R = (int32_t)p->R;
    float *blk, *bx;
    uint16_t *bq;
    uint64_t w3[3], bmax;
    if (rc) return rc;
    dims3(p, n);
    for (d = 0; d < 3; ++d) {
        w3[d] = d < p->ndim ? p->w[d] : 1;
        nw[d] = (n[d] + w3[d] - 1) / w3[d];
    }
    bmax = (w3[0] + 1) * (w3[1] + 1) * (w3[2] + 1);
    blk = (float *)malloc(bmax * sizeof(float));
    bx = (float *)malloc(bmax * sizeof(float));
    bq = (uint16_t *)malloc(bmax * sizeof(uint16_t));
    if (!blk || !bx || !bq) { free(blk); free(bx); free(bq); return SZO_ERR_OOM; }

    for (wi[2] = 0; wi[2] < nw[2]; ++wi[2])
        for (wi[1] = 0; wi[1] < nw[1]; ++wi[1])
            for (wi[0] = 0; wi[0] < nw[0]; ++wi[0]) {
                uint64_t lo[3], ext[3], c[3], bn[3];
                int lvl, k;
                for (d = 0; d < 3; ++d) {
                    uint64_t hi;
                    lo[d] = wi[d] * w3[d];
                    hi = d < p->ndim ? (lo[d] + w3[d] < n[d] - 1 ? lo[d] + w3[d] : n[d] - 1) : 0;
                    ext[d] = hi - lo[d] + 1;
                    bn[d] = ext[d];
                }
                for (c[2] = 0; c[2] < ext[2]; ++c[2])
                    for (c[1] = 0; c[1] < ext[1]; ++c[1])
                        for (c[0] = 0; c[0] < ext[0]; ++c[0]) {
                            uint64_t bi = lin(bn, c[0], c[1], c[2]);
                            blk[bi] = x[lin(n, lo[0] + c[0], lo[1] + c[1], lo[2] + c[2])];
                            bx[bi] = blk[bi];
                            bq[bi] = 0;
                            if (c[0] % p->S == 0 && c[1] % p->S == 0 && c[2] % p->S == 0)
                                bq[bi] = (uint16_t)R;
                        }
                /* in block coordinates the window interval along d is the
                 * whole block extent, so the block acts as a small field
                 * whose window equals its extent */
                for (lvl = cfg->levels; lvl >= 1; --lvl) {
                    uint64_t s = (uint64_t)1 << (lvl - 1);
                    for (k = 0; k < (int)p->ndim; ++k) {
                        int dd = cfg->order[k];
                        uint64_t start[3], step[3];
                        pass_grid(cfg, (int)p->ndim, k, s, start, step);
                        for (c[2] = start[2]; c[2] < ext[2]; c[2] += step[2])
                            for (c[1] = start[1]; c[1] < ext[1]; c[1] += step[1])
                                for (c[0] = start[0]; c[0] < ext[0]; c[0] += step[0]) {
                                    int cl;
                                    int32_t q = 0;
                                    float xr = 0.0f;
                                    uint64_t bi = lin(bn, c[0], c[1], c[2]);
                                    float pr = predict(blk, bn, c, dd, s, ext[dd] + 1,
                                                       cfg->spline[dd], &cl);
                                    if (quantize(bx[bi], pr, cfg->el[lvl - 1], cfg->ebx2[lvl - 1],
                                                 cfg->inv[lvl - 1], R, &q, &xr)) {
                                        bq[bi] = 0;
                                        blk[bi] = bx[bi];
                                    } else {
                                        bq[bi] = (uint16_t)(q + R);
                                        blk[bi] = xr;
                                    }
                                }
                    }
                }
                /* keep the owned points: all but the borrowed far faces */
                for (c[2] = 0; c[2] < ext[2]; ++c[2])
                    for (c[1] = 0; c[1] < ext[1]; ++c[1])
                        for (c[0] = 0; c[0] < ext[0]; ++c[0]) {
                            uint64_t bi = lin(bn, c[0], c[1], c[2]);
                            if (c[0] >= w3[0] || c[1] >= w3[1] || c[2] >= w3[2]) continue;
                            codes[lin(n, lo[0] + c[0], lo[1] + c[1], lo[2] + c[2])] = bq[bi];
                            recon[lin(n, lo[0] + c[0], lo[1] + c[1], lo[2] + c[2])] = blk[bi];
                        }
            }
    free(blk);
    free(bx);
    free(bq);
    return SZO_OK;
}

/* Decompression replays the predictions (Sec. V-B.1): anchors copied,
 * outliers restored, every other point = prediction + q * 2 e_l, with the
 * prediction, product and sum evaluated exactly as in compression. */
int szo_decompress(const szo_params *p, const szo_config *cfg, const float *anchors,
                   const uint16_t *codes, const uint32_t *oidx, const float *oval,
                   uint64_t n_out, float *out)
{
    uint64_t n[3], na[3], N, i, ax, ay, az;
    int rc = check_params(p);
    int lvl, k;
    const int32_t R = (int32_t)p->R;
    if (rc) return rc;
    dims3(p, n);
    N = n[0] * n[1] * n[2];
    count_anchors(p, n, na);
    for (i = 0; i < N; ++i) out[i] = 0.0f;
    for (i = 0; i < n_out; ++i) {
        if (oidx[i] >= N) return SZO_ERR_CORRUPT;
        out[oidx[i]] = oval[i];
    }
    for (az = 0; az < na[2]; ++az)
        for (ay = 0; ay < na[1]; ++ay)
            for (ax = 0; ax < na[0]; ++ax)
                out[lin(n, ax * p->S, ay * p->S, az * p->S)] = anchors[ax + na[0] * (ay + na[1] * az)];
    for (lvl = cfg->levels; lvl >= 1; --lvl) {
        uint64_t s = (uint64_t)1 << (lvl - 1);
        for (k = 0; k < (int)p->ndim; ++k) {
            int d = cfg->order[k];
            uint64_t start[3], step[3], c[3];
            pass_grid(cfg, (int)p->ndim, k, s, start, step);
            for (c[2] = start[2]; c[2] < n[2]; c[2] += step[2])
                for (c[1] = start[1]; c[1] < n[1]; c[1] += step[1])
                    for (c[0] = start[0]; c[0] < n[0]; c[0] += step[0]) {
                        int cl;
                        uint64_t gi = lin(n, c[0], c[1], c[2]);
                        float pr = predict(out, n, c, d, s, p->w[d], cfg->spline[d], &cl);
                        if (codes[gi] != 0) {
                            float t = (float)((int32_t)codes[gi] - R) * cfg->ebx2[lvl - 1];
                            out[gi] = pr + t;
                        }
                    }
        }
    }
    return SZO_OK;
}

/* ------------------------------------------------------------------ */
/* Sec. VI-A: histogram of the quant-codes over all points. */
void szo_histogram(const uint16_t *codes, uint64_t n, uint32_t nsym, uint32_t *h)
{
    uint64_t i;
    memset(h, 0, nsym * sizeof(uint32_t));
    for (i = 0; i < n; ++i)
        if (codes[i] < nsym) h[codes[i]]++;
}

/* Length-limited Huffman code lengths (Sec. VI-A codebook on the host) by
 * package-merge (Larmore and Hirschberg).  Deterministic reading:
 *  - leaves = symbols with h > 0, ordered by (weight, symbol);
 *  - each round packages consecutive pairs of the previous list (an odd
 *    last item is dropped) and merges the packages into the leaves, a leaf
 *    going first when weights are equal;
 *  - after Lmax - 1 rounds the first 2m - 2 items are selected, and a
 *    symbol's length is the number of times its leaf occurs in them.
 * One symbol present: length 1.  Returns the number of symbols coded. */
typedef struct { uint64_t w; int32_t leaf; } szo_item;

int szo_huffman_lengths(const uint32_t *h, uint32_t nsym, uint32_t Lmax, uint8_t *len)
{
    uint32_t m = 0, s, i, j;
    szo_item *leaves, **lists;
    uint32_t *lsize;
    int level;
    memset(len, 0, nsym);
    for (s = 0; s < nsym; ++s) if (h[s]) ++m;
    if (m == 0) return 0;
    if (m == 1) {
        for (s = 0; s < nsym; ++s) if (h[s]) len[s] = 1;
        return 1;
    }
    if (Lmax < 1 || Lmax > 31 || ((uint64_t)1 << Lmax) < m) return SZO_ERR_ARG;
    leaves = (szo_item *)malloc(m * sizeof(szo_item));
    lists = (szo_item **)calloc(Lmax, sizeof(szo_item *));
    lsize = (uint32_t *)calloc(Lmax, sizeof(uint32_t));
    if (!leaves || !lists || !lsize) return SZO_ERR_OOM;
    /* leaves sorted by (weight, symbol): insertion sort, plainly */
    j = 0;
    for (s = 0; s < nsym; ++s) {
        if (!h[s]) continue;
        i = j;
        while (i > 0 && leaves[i - 1].w > h[s]) { leaves[i] = leaves[i - 1]; --i; }
        leaves[i].w = h[s];
        leaves[i].leaf = (int32_t)s;
        ++j;
    }
    lists[0] = (szo_item *)malloc(m * sizeof(szo_item));
    memcpy(lists[0], leaves, m * sizeof(szo_item));
    lsize[0] = m;
    for (level = 1; level < (int)Lmax; ++level) {
        uint32_t np = lsize[level - 1] / 2, a = 0, b = 0, o = 0;
        szo_item *pk = (szo_item *)malloc((np ? np : 1) * sizeof(szo_item));
        lists[level] = (szo_item *)malloc((m + np) * sizeof(szo_item));
        for (i = 0; i < np; ++i) {
            pk[i].w = lists[level - 1][2 * i].w + lists[level - 1][2 * i + 1].w;
            pk[i].leaf = -1;
        }
        while (a < m || b < np) {
            if (b >= np || (a < m && leaves[a].w <= pk[b].w)) lists[level][o++] = leaves[a++];
            else lists[level][o++] = pk[b++];
        }
        lsize[level] = o;
        free(pk);
    }
    /* count leaf occurrences in the selected prefix, level by level */
    {
        uint32_t take = 2 * m - 2;
        for (level = (int)Lmax - 1; level >= 0; --level) {
            uint32_t packages = 0;
            for (i = 0; i < take && i < lsize[level]; ++i) {
                if (lists[level][i].leaf >= 0) len[lists[level][i].leaf]++;
                else packages++;
            }
            take = 2 * packages;
        }
    }
    for (level = 0; level < (int)Lmax; ++level) free(lists[level]);
    free(lists);
    free(lsize);
    free(leaves);
    return (int)m;
}

/* Canonical code assignment (as in DEFLATE): shorter codes first, equal
 * lengths in symbol order, consecutive integers. */
void szo_canonical_codes(const uint8_t *len, uint32_t nsym, uint32_t *code)
{
    uint32_t bl_count[33], next_code[33], s, b, c = 0;
    memset(bl_count, 0, sizeof bl_count);
    for (s = 0; s < nsym; ++s) bl_count[len[s]]++;
    bl_count[0] = 0;
    for (b = 1; b <= 32; ++b) {
        c = (c + bl_count[SZO_PLANT == 7 ? b : b - 1]) << 1;
        next_code[b] = c;
    }
    for (s = 0; s < nsym; ++s) {
        code[s] = 0;
        if (len[s]) code[s] = next_code[len[s]]++;
    }
}

/* Chunked encode: chunk j holds symbols [jC, min((j+1)C, n)); its
 * codewords are concatenated most-significant bit first from bit 31 of its
 * first word and zero-padded to a word.  chunk_bits[j] = its bit count.
 * Chunks follow each other word-aligned.  Returns the word count, or
 * (uint64_t)-1 when a symbol has no code. */
uint64_t szo_encode(const uint16_t *sym, uint64_t n, const uint8_t *len, const uint32_t *code,
                    uint32_t C, uint16_t *chunk_bits, uint32_t *words)
{
    uint64_t nchunks = (n + C - 1) / C, j, wpos = 0;
    for (j = 0; j < nchunks; ++j) {
        uint64_t i, end = (j + 1) * C < n ? (j + 1) * C : n;
        uint64_t bits = 0;
        uint32_t cur = 0;
        int filled = 0;   /* bits used in cur */
        for (i = j * C; i < end; ++i) {
            int L = len[sym[i]], b;
            if (L == 0) return (uint64_t)-1;
            for (b = L - 1; b >= 0; --b) {
                uint32_t bit = (code[sym[i]] >> (SZO_PLANT == 11 ? L - 1 - b : b)) & 1u;
                cur |= bit << (31 - filled);
                ++filled;
                ++bits;
                if (filled == 32) { words[wpos++] = cur; cur = 0; filled = 0; }
            }
        }
        if (filled) words[wpos++] = cur;
        chunk_bits[j] = (uint16_t)bits;
    }
    return wpos;
}

/* Canonical decode, one bit at a time.  Returns 0 or SZO_ERR_CORRUPT. */
int szo_decode(const uint32_t *words, uint64_t n_words, const uint16_t *chunk_bits, uint64_t n,
               uint32_t C, const uint8_t *len, uint32_t nsym, uint16_t *sym)
{
    uint32_t first[33], count[33], offset[33], b, s;
    uint16_t *sorted;
    uint64_t nchunks = (n + C - 1) / C, j, wpos = 0;
    uint32_t code_next = 0, k = 0;
    memset(count, 0, sizeof count);
    for (s = 0; s < nsym; ++s) if (len[s]) count[len[s]]++;
    sorted = (uint16_t *)malloc((nsym ? nsym : 1) * sizeof(uint16_t));
    if (!sorted) return SZO_ERR_OOM;
    for (b = 1; b <= 32; ++b) {
        code_next = (code_next + (b > 1 ? count[b - 1] : 0)) << 1;
        first[b] = code_next;
        offset[b] = k;
        for (s = 0; s < nsym; ++s) if (len[s] == b) sorted[k++] = (uint16_t)s;
    }
    for (j = 0; j < nchunks; ++j) {
        uint64_t i, end = (j + 1) * C < n ? (j + 1) * C : n;
        uint64_t bitpos = 0, cb = chunk_bits[j];
        uint64_t nw = (cb + 31) / 32;
        if (wpos + nw > n_words) { free(sorted); return SZO_ERR_CORRUPT; }
        for (i = j * C; i < end; ++i) {
            uint32_t c = 0;
            int found = 0;
            for (b = 1; b <= 32 && !found; ++b) {
                uint32_t bit;
                if (bitpos >= cb) { free(sorted); return SZO_ERR_CORRUPT; }
                bit = (words[wpos + bitpos / 32] >> (31 - bitpos % 32)) & 1u;
                ++bitpos;
                c = (c << 1) | bit;
                if (count[b] && c >= first[b] && c - first[b] < count[b]) {
                    sym[i] = sorted[offset[b] + (c - first[b])];
                    found = 1;
                }
            }
            if (!found) { free(sorted); return SZO_ERR_CORRUPT; }
        }
        if (bitpos != cb) { free(sorted); return SZO_ERR_CORRUPT; }
        wpos += nw;
    }
    free(sorted);
    return SZO_OK;
}
