// kernels.hip -- gfx950 kernels of libszi (G-Interp compressor, cuSZ-i,
// arXiv 2312.05492).  Built with -ffp-contract=off: every FP32 expression of
// the predictor and quantiser is evaluated as written, one rounding per
// operation, so that results are reproducible bit for bit.
#include <float.h>
#include <math.h>

#include "szi_internal.h"

namespace szi {

// ------------------------------------------------------------- helpers
__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
// exclusive prefix sum across the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total) {
    const int lane = threadIdx.x & 63;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, 63);
    return x - v;
}

// Division by a small divisor m (< kMagicN) of dividends t < 2^16 through a
// multiply-high by ceil(2^32 / m); exact because t * m < 2^32.  The
// multipliers come from a constant table, so no divide runs on the GPU.
constexpr int kMagicN = 2048;
struct MagicTable {
    uint32_t v[kMagicN];
    constexpr MagicTable() : v() {
        for (int m = 0; m < kMagicN; ++m) v[m] = m > 1 ? 0xFFFFFFFFu / (uint32_t)m + 1u : 0u;
    }
};
__constant__ MagicTable kMagic = MagicTable();

struct FastDiv {
    uint32_t m, mg;
    __device__ __forceinline__ void set(uint32_t mm) {
        m = mm;
        mg = kMagic.v[mm];
    }
    __device__ __forceinline__ uint32_t div(uint32_t t) const { return m > 1 ? __umulhi(t, mg) : t; }
};

__device__ __forceinline__ bool finite_bits(float v) {
    return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u;
}

// ------------------------------------------------------- value range
// Partial min / max / non-finite counts: kRangeBlocks blocks per field.
__global__ __launch_bounds__(256) void k_range(const FieldDesc* __restrict__ F, float* pmin,
                                               float* pmax, uint32_t* pbad) {
    const FieldDesc& f = F[blockIdx.y];
    const float* in = f.in;
    const uint64_t n = f.npts;
    float mn = INFINITY, mx = -INFINITY;
    uint32_t bad = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t head = 0;
    if ((reinterpret_cast<uintptr_t>(in) & 15) == 0) {
        const float4* in4 = reinterpret_cast<const float4*>(in);
        const uint64_t n4 = n / 4;
        uint64_t i = tid;
        for (; i + 3 * stride < n4; i += 4 * stride) {
            float4 a = in4[i], b = in4[i + stride], c = in4[i + 2 * stride], d = in4[i + 3 * stride];
            float vv[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w,
                            c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                mn = fminf(mn, vv[k]);
                mx = fmaxf(mx, vv[k]);
                bad += finite_bits(vv[k]) ? 0u : 1u;
            }
        }
        for (; i < n4; i += stride) {
            float4 a = in4[i];
            float vv[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                mn = fminf(mn, vv[k]);
                mx = fmaxf(mx, vv[k]);
                bad += finite_bits(vv[k]) ? 0u : 1u;
            }
        }
        head = n4 * 4;
    }
    for (uint64_t i = head + tid; i < n; i += stride) {
        float v = in[i];
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
        bad += finite_bits(v) ? 0u : 1u;
    }
    __shared__ float smn[4], smx[4];
    __shared__ uint32_t sbad[4];
    mn = wave_min(mn);
    mx = wave_max(mx);
    bad = wave_sum(bad);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smn[w] = mn;
        smx[w] = mx;
        sbad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            mn = fminf(mn, smn[k]);
            mx = fmaxf(mx, smx[k]);
            bad += sbad[k];
        }
        const uint64_t o = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
        pmin[o] = mn;
        pmax[o] = mx;
        pbad[o] = bad;
    }
}

// ------------------------------------------------------- spline formulas
// Sec. V-B.1.  a = x[n-3s], b = x[n-s], c = x[n+s], d = x[n+3s] along the
// pass dimension; availability decides the spline.
enum { SPL_LIN = 0, SPL_NAK = 1, SPL_NAT = 2, SPL_AUTO = 3 };

__device__ __forceinline__ float spline_predict(int spl, bool m3, bool p1, bool p3, float a,
                                                float b, float c, float d) {
    if (!p1) return b;
    if (spl == SPL_LIN || (!m3 && !p3)) return (b + c) * 0.5f;
    if (m3 && !p3) return ((6.0f * b + 3.0f * c) - a) * 0.125f;
    if (!m3 && p3) return ((3.0f * b + 6.0f * c) - d) * 0.125f;
    if (spl == SPL_NAT) return (23.0f * (b + c) - 3.0f * (a + d)) / 40.0f;
    return (9.0f * (b + c) - (a + d)) * 0.0625f;
}

// ------------------------------------------------------- profiling
// Sec. V-C.1: a uniform 4^D sub-grid of samples; at each, the linear and
// both cubic splines along every dimension on original values (stride 1);
// L1 errors accumulated in FP64 in ascending sample order.
__device__ __forceinline__ int sample_pos(int nd, int t) {
    int v = (int)(((int64_t)(2 * t + 1) * nd) / 8);
    if (nd >= 7) {
        v = v < 3 ? 3 : v;
        v = v > nd - 4 ? nd - 4 : v;
    }
    return v;
}

__global__ __launch_bounds__(64) void k_profile(const FieldDesc* __restrict__ F, FieldPlan* P) {
    const FieldDesc& f = F[blockIdx.x];
    __shared__ double err[64][3][3];
    const int t = threadIdx.x;
    const int D = f.ndim;
    const int ns = D == 3 ? 64 : 16;
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 3; ++k) err[t][d][k] = 0.0;
    if (f.need_prof && t < ns) {
        int c[3];
        c[0] = sample_pos(f.n[0], t & 3);
        c[1] = sample_pos(f.n[1], (t >> 2) & 3);
        c[2] = D == 3 ? sample_pos(f.n[2], t >> 4) : 0;
        const int64_t st[3] = {1, f.n[0], (int64_t)f.n[0] * f.n[1]};
        const int64_t gi = c[0] + st[1] * c[1] + st[2] * c[2];
        const float x = f.in[gi];
        for (int d = 0; d < D; ++d) {
            if (f.n[d] < 7) continue;
            const float a = f.in[gi - 3 * st[d]], b = f.in[gi - st[d]];
            const float cc = f.in[gi + st[d]], dd = f.in[gi + 3 * st[d]];
            const float pl = (b + cc) * 0.5f;
            const float pk = (9.0f * (b + cc) - (a + dd)) * 0.0625f;
            const float pn = (23.0f * (b + cc) - 3.0f * (a + dd)) / 40.0f;
            err[t][d][0] = fabs((double)x - (double)pl);
            err[t][d][1] = fabs((double)x - (double)pk);
            err[t][d][2] = fabs((double)x - (double)pn);
        }
    }
    __syncthreads();
    if (t == 0) {
        double s[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (f.need_prof)
            for (int k = 0; k < ns; ++k)
                for (int d = 0; d < D; ++d)
                    if (f.n[d] >= 7)
                        for (int e = 0; e < 3; ++e) s[d][e] = s[d][e] + err[k][d][e];
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e < 3; ++e) P[blockIdx.x].prof[d][e] = s[d][e];
    }
}

// ------------------------------------------------------- plan
// Sec. V-C.1 (absolute/relative bound from the range), Eq. 1 (alpha),
// Sec. V-B.2 (level bounds), Sec. V-C.2 (spline per dimension, order).
__device__ double eq1_alpha(double eps) {
    if (eps >= 1e-1) return 2.0;
    if (eps >= 1e-2) return 1.75 + 0.25 * (eps - 1e-2) / (1e-1 - 1e-2);
    if (eps >= 1e-3) return 1.5 + 0.25 * (eps - 1e-3) / (1e-2 - 1e-3);
    if (eps >= 1e-4) return 1.25 + 0.25 * (eps - 1e-4) / (1e-3 - 1e-4);
    if (eps >= 1e-5) return 1.0 + 0.25 * (eps - 1e-5) / (1e-4 - 1e-5);
    return 1.0;
}

// largest float not above v (v >= 0)
__device__ float floor_to_f32(double v) {
    if (!(v > 0.0)) return 0.0f;
    if (v >= (double)FLT_MAX) return FLT_MAX;
    float f = (float)v;
    if ((double)f > v) f = __uint_as_float(__float_as_uint(f) - 1u);
    return f;
}

__global__ __launch_bounds__(256) void k_plan(const FieldDesc* __restrict__ F, FieldPlan* P,
                                              const float* pmin, const float* pmax,
                                              const uint32_t* pbad) {
    const FieldDesc& f = F[blockIdx.x];
    FieldPlan& p = P[blockIdx.x];
    float mn = INFINITY, mx = -INFINITY;
    uint32_t bad = 0;
    for (int i = threadIdx.x; i < kRangeBlocks; i += blockDim.x) {
        const uint64_t o = (uint64_t)blockIdx.x * kRangeBlocks + i;
        mn = fminf(mn, pmin[o]);
        mx = fmaxf(mx, pmax[o]);
        bad += pbad[o];
    }
    __shared__ float smn[4], smx[4];
    __shared__ uint32_t sbad[4];
    mn = wave_min(mn);
    mx = wave_max(mx);
    bad = wave_sum(bad);
    if ((threadIdx.x & 63) == 0) {
        smn[threadIdx.x >> 6] = mn;
        smx[threadIdx.x >> 6] = mx;
        sbad[threadIdx.x >> 6] = bad;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int k = 1; k < 4; ++k) {
        mn = fminf(mn, smn[k]);
        mx = fmaxf(mx, smx[k]);
        bad += sbad[k];
    }
    p.vmin = mn + 0.0f;
    p.vmax = mx + 0.0f;
    p.nonfinite = bad;
    p.status = bad ? -2 : 0;
    p.range = (double)p.vmax - (double)p.vmin;
    if (f.eb_mode == 1) {
        p.eps = f.eb;
        p.e_abs = f.eb * p.range;
    } else {
        p.e_abs = f.eb;
        p.eps = p.range > 0.0 ? f.eb / p.range : (f.eb > 0.0 ? INFINITY : 0.0);
    }
    p.e = floor_to_f32(p.e_abs);
    p.alpha = f.alpha_req > 0.0 ? f.alpha_req : eq1_alpha(p.eps);
    p.levels = f.L;
    double apow = 1.0;
    for (int l = 0; l < kMaxLevels; ++l) {
        if (l < f.L) {
            p.el[l] = floor_to_f32(p.e_abs / apow);
            p.ebx2[l] = 2.0f * p.el[l];
            p.inv[l] = 1.0f / p.ebx2[l];
            apow = apow * p.alpha;
        } else {
            p.el[l] = 0.0f;
            p.ebx2[l] = 0.0f;
            p.inv[l] = 0.0f;
        }
    }
    const int D = f.ndim;
    double score[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        int s = d < D ? f.interp[d] : SPL_LIN;
        if (s == SPL_AUTO) s = p.prof[d][2] < p.prof[d][1] ? SPL_NAT : SPL_NAK;
        p.spline[d] = s;
        score[d] = p.prof[d][s];
    }
    if (f.order_req[0] >= 0) {
        for (int k = 0; k < 3; ++k) p.order[k] = k < D ? f.order_req[k] : -1;
    } else {
        // least smooth first; a strictly larger error wins, else the slower
        bool used[3] = {false, false, false};
        for (int k = 0; k < 3; ++k) {
            if (k >= D) {
                p.order[k] = -1;
                continue;
            }
            int best = -1;
            for (int d = D - 1; d >= 0; --d) {
                if (used[d]) continue;
                if (best < 0 || score[d] > score[best]) best = d;
            }
            used[best] = true;
            p.order[k] = best;
        }
    }
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------- interpolation
// One window per iteration of a persistent workgroup.  The window owns the
// points [lo, lo + W) of each dimension; its block adds the far faces
// (lo + W), whose points are computed identically by both windows sharing
// them (neighbours are searched inside the point's own window interval
// along the pass dimension only), so windows are independent (Sec. V-A/D).
// Levels run from stride S/2 to 1; at each level one pass per dimension in
// the planned order, separated by workgroup barriers.

// Points of pass (level lvl, k-th dimension in the order): along the pass
// dimension the odd multiples of s, along dimensions already passed at
// this level the multiples of s, along those still to come the multiples
// of 2s (s = 2^(lvl-1)).
struct PassGrid {
    int st0, st1, st2;   // first coordinate
    int sh0, sh1, sh2;   // log2 of the step
    int m0, m1, m2;      // counts
    uint32_t total;
    FastDiv d0, d01;
};

// position of dimension j in the order (order holds ND distinct dims)
__device__ __forceinline__ int order_pos(int o0, int o1, int j) {
    return o0 == j ? 0 : (o1 == j ? 1 : 2);
}

__device__ __forceinline__ void pass_axis(int kj, int k, int lvl, int ext, int& st, int& sh,
                                          int& m) {
    st = kj == k ? (1 << (lvl - 1)) : 0;
    sh = kj < k ? lvl - 1 : lvl;
    m = ext > st ? ((ext - 1 - st) >> sh) + 1 : 0;
}

__device__ __forceinline__ void pass_grid(PassGrid& g, int o0, int o1, int ND, int k, int lvl,
                                          int e0, int e1, int e2) {
    pass_axis(order_pos(o0, o1, 0), k, lvl, e0, g.st0, g.sh0, g.m0);
    pass_axis(order_pos(o0, o1, 1), k, lvl, e1, g.st1, g.sh1, g.m1);
    if (ND == 3) {
        pass_axis(order_pos(o0, o1, 2), k, lvl, e2, g.st2, g.sh2, g.m2);
    } else {
        g.st2 = 0;
        g.sh2 = 0;
        g.m2 = 1;
    }
    g.total = (uint32_t)(g.m0 * g.m1 * g.m2);
    g.d0.set((uint32_t)g.m0);
    g.d01.set((uint32_t)(g.m0 * g.m1));
}

template <int ND, int W0, int W1, int W2>
struct Geom {
    static constexpr int B0 = W0 + 1;
    static constexpr int B1 = W1 + 1;
    static constexpr int B2 = ND == 3 ? W2 + 1 : 1;
    static constexpr int BN = B0 * B1 * B2;
};

struct WinInfo {
    int lo[3], ext[3], own[3];
};

__device__ __forceinline__ void window_info(const FieldDesc& f, uint64_t w, int W0, int W1,
                                            int W2, WinInfo& wi) {
    const int Wd[3] = {W0, W1, W2};
    const uint32_t nw0 = (uint32_t)f.nwin[0], nw1 = (uint32_t)f.nwin[1];
    const uint32_t wz = (uint32_t)(w / ((uint64_t)nw0 * nw1));
    const uint32_t r = (uint32_t)(w - (uint64_t)wz * nw0 * nw1);
    const uint32_t wy = r / nw0;
    const uint32_t wx = r - wy * nw0;
    const uint32_t widx[3] = {wx, wy, wz};
    for (int d = 0; d < 3; ++d) {
        if (d < f.ndim) {
            wi.lo[d] = (int)widx[d] * Wd[d];
            const int span = f.n[d] - 1 - wi.lo[d];
            wi.ext[d] = (span < Wd[d] ? span : Wd[d]) + 1;
            wi.own[d] = wi.ext[d] < Wd[d] ? wi.ext[d] : Wd[d];
        } else {
            wi.lo[d] = 0;
            wi.ext[d] = 1;
            wi.own[d] = 1;
        }
    }
}

template <int ND, int W0, int W1, int W2>
__global__ __launch_bounds__(kThreads) void k_compress(const FieldDesc* __restrict__ F,
                                                       const FieldPlan* __restrict__ P,
                                                       const uint64_t* __restrict__ item_off,
                                                       int nfields, uint64_t nitems) {
    using G = Geom<ND, W0, W1, W2>;
    __shared__ float v[G::BN];
    __shared__ uint16_t q[G::BN + 1];
    extern __shared__ uint32_t hist[];
    const int tid = threadIdx.x;
    int f = 0, cur = -1;
    uint32_t cntR = 0;

    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        while (it >= item_off[f + 1]) ++f;
        if (f != cur) {
            if (cur >= 0) {
                // flush the previous field's histogram
                const uint32_t s = wave_sum(cntR);
                cntR = 0;
                if ((tid & 63) == 0 && s) atomicAdd(&hist[F[cur].R], s);
                __syncthreads();
                for (int b = tid; b < 2 * F[cur].R; b += kThreads)
                    if (hist[b]) atomicAdd(&F[cur].hist[b], hist[b]);
                __syncthreads();
            }
            cur = f;
            for (int b = tid; b < 2 * F[cur].R; b += kThreads) hist[b] = 0;
            __syncthreads();
        }
        const FieldDesc& fd = F[f];
        const FieldPlan& pl = P[f];
        WinInfo wi;
        window_info(fd, it - item_off[f], W0, W1, W2, wi);
        const int R = fd.R;
        const int n0 = fd.n[0];
        const uint64_t n01 = (uint64_t)fd.n[0] * fd.n[1];

        // load the block (own points and borrowed far faces)
        {
            FastDiv e0, e01;
            e0.set((uint32_t)wi.ext[0]);
            e01.set((uint32_t)(wi.ext[0] * wi.ext[1]));
            const uint32_t tot = (uint32_t)(wi.ext[0] * wi.ext[1] * wi.ext[2]);
            const float* base = fd.in + wi.lo[0] + (uint64_t)wi.lo[1] * n0 + wi.lo[2] * n01;
            for (uint32_t t = tid; t < tot; t += kThreads) {
                const uint32_t c2 = e01.div(t);
                const uint32_t r = t - c2 * e01.m;
                const uint32_t c1 = e0.div(r);
                const uint32_t c0 = r - c1 * e0.m;
                v[c0 + G::B0 * (c1 + G::B1 * c2)] = base[c0 + (uint64_t)c1 * n0 + c2 * n01];
            }
        }
        __syncthreads();

        const int o0 = pl.order[0], o1 = pl.order[1], o2 = pl.order[2];
        for (int lvl = fd.L; lvl >= 1; --lvl) {
            const int s = 1 << (lvl - 1);
            const float el = pl.el[lvl - 1], ebx2 = pl.ebx2[lvl - 1], inv = pl.inv[lvl - 1];
            const double eld = (double)el;
            for (int k = 0; k < ND; ++k) {
                const int d = k == 0 ? o0 : (k == 1 ? o1 : o2);
                const int spl = d == 0 ? pl.spline[0] : (d == 1 ? pl.spline[1] : pl.spline[2]);
                PassGrid g;
                pass_grid(g, o0, o1, ND, k, lvl, wi.ext[0], wi.ext[1], wi.ext[2]);
                const int sd = d == 0 ? 1 : (d == 1 ? G::B0 : G::B0 * G::B1);
                const int ed = d == 0 ? wi.ext[0] : (d == 1 ? wi.ext[1] : wi.ext[2]);
                for (uint32_t t = tid; t < g.total; t += kThreads) {
                    const uint32_t i2 = g.d01.div(t);
                    const uint32_t r = t - i2 * g.d01.m;
                    const uint32_t i1 = g.d0.div(r);
                    const uint32_t i0 = r - i1 * g.d0.m;
                    const int c0 = g.st0 + ((int)i0 << g.sh0);
                    const int c1 = g.st1 + ((int)i1 << g.sh1);
                    const int c2 = g.st2 + ((int)i2 << g.sh2);
                    const int li = c0 + G::B0 * (c1 + G::B1 * c2);
                    const int cd = d == 0 ? c0 : (d == 1 ? c1 : c2);
                    const bool p1 = cd + s <= ed - 1;
                    const bool m3 = cd >= 3 * s;
                    const bool p3 = cd + 3 * s <= ed - 1;
                    const float b = v[li - s * sd];
                    const float cc = p1 ? v[li + s * sd] : 0.0f;
                    const float a = m3 ? v[li - 3 * s * sd] : 0.0f;
                    const float dd = p3 ? v[li + 3 * s * sd] : 0.0f;
                    const float p = spline_predict(spl, m3, p1, p3, a, b, cc, dd);
                    const float x = v[li];
                    // Sec. III-A: quantise the residual with bin 2 e_l; the
                    // adjusted prediction replaces the value
                    const float diff = x - p;
                    bool outl;
                    int qi = 0;
                    float xr = p;
                    if (el == 0.0f) {
                        outl = !(diff == 0.0f);
                    } else {
                        const float qf = diff * inv;
                        outl = !(fabsf(qf) < (float)R);
                        if (!outl) {
                            qi = (int)rintf(qf);
                            outl = qi >= R || qi <= -R;
                        }
                        if (!outl) {
                            const float tq = (float)qi * ebx2;
                            xr = p + tq;
                            outl = !(fabs((double)x - (double)xr) <= eld);
                        }
                    }
                    v[li] = outl ? x : xr;
                    q[li] = outl ? (uint16_t)0 : (uint16_t)(qi + R);
                }
                __syncthreads();
            }
        }

        // write the owned codes and anchors; histogram of owned codes
        {
            FastDiv o0, o01;
            o0.set((uint32_t)wi.own[0]);
            o01.set((uint32_t)(wi.own[0] * wi.own[1]));
            const uint32_t tot = (uint32_t)(wi.own[0] * wi.own[1] * wi.own[2]);
            const uint64_t gbase = wi.lo[0] + (uint64_t)wi.lo[1] * n0 + wi.lo[2] * n01;
            const int smask = fd.S - 1;
            for (uint32_t t = tid; t < tot; t += kThreads) {
                const uint32_t c2 = o01.div(t);
                const uint32_t r = t - c2 * o01.m;
                const uint32_t c1 = o0.div(r);
                const uint32_t c0 = r - c1 * o0.m;
                const int li = c0 + G::B0 * (c1 + G::B1 * c2);
                const bool anchor = ((c0 | c1 | c2) & smask) == 0;
                const uint16_t code = anchor ? (uint16_t)R : q[li];
                fd.codes[gbase + c0 + (uint64_t)c1 * n0 + c2 * n01] = code;
                if (anchor) {
                    const int a0 = (wi.lo[0] + c0) / fd.S, a1 = (wi.lo[1] + c1) / fd.S;
                    const int a2 = (wi.lo[2] + c2) / fd.S;
                    fd.anchors[a0 + (uint64_t)fd.na[0] * (a1 + (uint64_t)fd.na[1] * a2)] = v[li];
                }
                if (code == (uint16_t)R)
                    ++cntR;
                else
                    atomicAdd(&hist[code], 1u);
            }
        }
        __syncthreads();
    }
    if (cur >= 0) {
        const uint32_t s = wave_sum(cntR);
        if ((tid & 63) == 0 && s) atomicAdd(&hist[F[cur].R], s);
        __syncthreads();
        for (int b = tid; b < 2 * F[cur].R; b += kThreads)
            if (hist[b]) atomicAdd(&F[cur].hist[b], hist[b]);
    }
}

template <int ND, int W0, int W1, int W2>
__global__ __launch_bounds__(kThreads) void k_decompress(const FieldDesc* __restrict__ F,
                                                         const FieldPlan* __restrict__ P,
                                                         const uint64_t* __restrict__ item_off,
                                                         int nfields, uint64_t nitems) {
    using G = Geom<ND, W0, W1, W2>;
    __shared__ float v[G::BN];
    __shared__ uint16_t q[G::BN + 1];
    const int tid = threadIdx.x;
    int f = 0;
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        while (it >= item_off[f + 1]) ++f;
        const FieldDesc& fd = F[f];
        const FieldPlan& pl = P[f];
        WinInfo wi;
        window_info(fd, it - item_off[f], W0, W1, W2, wi);
        const int R = fd.R;
        const int n0 = fd.n[0];
        const uint64_t n01 = (uint64_t)fd.n[0] * fd.n[1];
        const int smask = fd.S - 1;
        {
            FastDiv e0, e01;
            e0.set((uint32_t)wi.ext[0]);
            e01.set((uint32_t)(wi.ext[0] * wi.ext[1]));
            const uint32_t tot = (uint32_t)(wi.ext[0] * wi.ext[1] * wi.ext[2]);
            const uint64_t gbase = wi.lo[0] + (uint64_t)wi.lo[1] * n0 + wi.lo[2] * n01;
            for (uint32_t t = tid; t < tot; t += kThreads) {
                const uint32_t c2 = e01.div(t);
                const uint32_t r = t - c2 * e01.m;
                const uint32_t c1 = e0.div(r);
                const uint32_t c0 = r - c1 * e0.m;
                const int li = c0 + G::B0 * (c1 + G::B1 * c2);
                const uint64_t g = gbase + c0 + (uint64_t)c1 * n0 + c2 * n01;
                const uint16_t code = fd.codes[g];
                q[li] = code;
                if (((c0 | c1 | c2) & smask) == 0) {
                    const int a0 = (wi.lo[0] + c0) / fd.S, a1 = (wi.lo[1] + c1) / fd.S;
                    const int a2 = (wi.lo[2] + c2) / fd.S;
                    v[li] = fd.anchors[a0 + (uint64_t)fd.na[0] * (a1 + (uint64_t)fd.na[1] * a2)];
                } else if (code == 0) {
                    v[li] = fd.out[g];   // outlier value scattered beforehand
                }
            }
        }
        __syncthreads();
        const int o0 = pl.order[0], o1 = pl.order[1], o2 = pl.order[2];
        for (int lvl = fd.L; lvl >= 1; --lvl) {
            const int s = 1 << (lvl - 1);
            const float ebx2 = pl.ebx2[lvl - 1];
            for (int k = 0; k < ND; ++k) {
                const int d = k == 0 ? o0 : (k == 1 ? o1 : o2);
                const int spl = d == 0 ? pl.spline[0] : (d == 1 ? pl.spline[1] : pl.spline[2]);
                PassGrid g;
                pass_grid(g, o0, o1, ND, k, lvl, wi.ext[0], wi.ext[1], wi.ext[2]);
                const int sd = d == 0 ? 1 : (d == 1 ? G::B0 : G::B0 * G::B1);
                const int ed = d == 0 ? wi.ext[0] : (d == 1 ? wi.ext[1] : wi.ext[2]);
                for (uint32_t t = tid; t < g.total; t += kThreads) {
                    const uint32_t i2 = g.d01.div(t);
                    const uint32_t r = t - i2 * g.d01.m;
                    const uint32_t i1 = g.d0.div(r);
                    const uint32_t i0 = r - i1 * g.d0.m;
                    const int c0 = g.st0 + ((int)i0 << g.sh0);
                    const int c1 = g.st1 + ((int)i1 << g.sh1);
                    const int c2 = g.st2 + ((int)i2 << g.sh2);
                    const int li = c0 + G::B0 * (c1 + G::B1 * c2);
                    const int code = q[li];
                    if (code == 0) continue;
                    const int cd = d == 0 ? c0 : (d == 1 ? c1 : c2);
                    const bool p1 = cd + s <= ed - 1;
                    const bool m3 = cd >= 3 * s;
                    const bool p3 = cd + 3 * s <= ed - 1;
                    const float b = v[li - s * sd];
                    const float cc = p1 ? v[li + s * sd] : 0.0f;
                    const float a = m3 ? v[li - 3 * s * sd] : 0.0f;
                    const float dd = p3 ? v[li + 3 * s * sd] : 0.0f;
                    const float p = spline_predict(spl, m3, p1, p3, a, b, cc, dd);
                    const float tq = (float)(code - R) * ebx2;
                    v[li] = p + tq;
                }
                __syncthreads();
            }
        }
        {
            FastDiv o0, o01;
            o0.set((uint32_t)wi.own[0]);
            o01.set((uint32_t)(wi.own[0] * wi.own[1]));
            const uint32_t tot = (uint32_t)(wi.own[0] * wi.own[1] * wi.own[2]);
            const uint64_t gbase = wi.lo[0] + (uint64_t)wi.lo[1] * n0 + wi.lo[2] * n01;
            for (uint32_t t = tid; t < tot; t += kThreads) {
                const uint32_t c2 = o01.div(t);
                const uint32_t r = t - c2 * o01.m;
                const uint32_t c1 = o0.div(r);
                const uint32_t c0 = r - c1 * o0.m;
                fd.out[gbase + c0 + (uint64_t)c1 * n0 + c2 * n01] = v[c0 + G::B0 * (c1 + G::B1 * c2)];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------- Huffman
// Chunked coarse-grained Huffman (Sec. VI-A).  A workgroup of 4 waves
// handles kChunksPerBlock consecutive chunks of one field; each wave encodes
// one chunk at a time with C/64 consecutive symbols per lane.
constexpr int kChunksPerBlock = 16;

__device__ __forceinline__ int block_field(const uint64_t* __restrict__ boff, int nfields,
                                           uint64_t b) {
    int lo = 0, hi = nfields - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_huff_stats(const FieldDesc* __restrict__ F, int nfields,
                                                    const uint64_t* __restrict__ boff,
                                                    uint32_t* cwords, uint32_t* couts) {
    extern __shared__ uint32_t cb[];
    const int f = block_field(boff, nfields, blockIdx.x);
    const FieldDesc& fd = F[f];
    const int nsym = 2 * fd.R;
    for (int s = threadIdx.x; s < nsym; s += blockDim.x) cb[s] = fd.cbook[s];
    __syncthreads();
    const uint64_t first = (blockIdx.x - boff[f]) * kChunksPerBlock;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int C = fd.chunk;
    const int per = C >> 6;
    for (int j = wave; j < kChunksPerBlock; j += 4) {
        const uint64_t ch = first + j;
        if (ch >= fd.nchunks) break;   // no barrier in this loop
        const uint64_t s0 = ch * C + (uint64_t)lane * per;
        uint32_t bits = 0, zeros = 0;
        for (int k = 0; k < per; ++k) {
            const uint64_t i = s0 + k;
            if (i < fd.npts) {
                const uint16_t sym = fd.codes[i];
                bits += cb[sym] >> 24;
                zeros += sym == 0 ? 1u : 0u;
            }
        }
        bits = wave_sum(bits);
        zeros = wave_sum(zeros);
        if (lane == 0) {
            fd.chunk_bits[ch] = (uint16_t)bits;
            cwords[fd.chunk_base + ch] = (bits + 31) >> 5;
            if (couts) couts[fd.chunk_base + ch] = zeros;
        }
    }
}

// Exclusive scan of one or two u32 arrays into u64 offsets with a single
// workgroup: each thread sums a contiguous run, the runs are scanned, then
// each thread writes its run.  totals[0..1] receive the sums.
__global__ __launch_bounds__(1024) void k_scan_pairs(const uint32_t* __restrict__ a,
                                                     const uint32_t* __restrict__ b, uint64_t n,
                                                     uint64_t* aoff, uint64_t* boff,
                                                     uint64_t* totals) {
    const int t = threadIdx.x;
    const uint64_t per = (n + 1023) / 1024;
    const uint64_t beg = t * per, end = beg + per < n ? beg + per : n;
    uint64_t sa = 0, sb = 0;
    for (uint64_t i = beg; i < end; ++i) {
        sa += a[i];
        if (b) sb += b[i];
    }
    __shared__ uint64_t xa[1024], xb[1024];
    xa[t] = sa;
    xb[t] = sb;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint64_t ya = t >= o ? xa[t - o] : 0, yb = t >= o ? xb[t - o] : 0;
        __syncthreads();
        xa[t] += ya;
        xb[t] += yb;
        __syncthreads();
    }
    uint64_t ra = xa[t] - sa, rb = xb[t] - sb;
    for (uint64_t i = beg; i < end; ++i) {
        aoff[i] = ra;
        ra += a[i];
        if (b) {
            boff[i] = rb;
            rb += b[i];
        }
    }
    if (t == 1023) {
        totals[0] = xa[1023];
        totals[1] = xb[1023];
    }
}

__global__ __launch_bounds__(256) void k_huff_encode(const FieldDesc* __restrict__ F, int nfields,
                                                     const uint64_t* __restrict__ boff,
                                                     const uint64_t* __restrict__ word_off,
                                                     const uint64_t* __restrict__ out_off,
                                                     int max_chunk_words) {
    extern __shared__ uint32_t smem[];
    const int f = block_field(boff, nfields, blockIdx.x);
    const FieldDesc& fd = F[f];
    const int nsym = 2 * fd.R;
    uint32_t* cb = smem;
    for (int s = threadIdx.x; s < nsym; s += blockDim.x) cb[s] = fd.cbook[s];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t* wbuf = smem + nsym + wave * max_chunk_words;
    __syncthreads();
    const uint64_t first = (blockIdx.x - boff[f]) * kChunksPerBlock;
    const int C = fd.chunk;
    const int per = C >> 6;
    // offsets of this field's first chunk, so the field's sections start at 0
    const uint64_t wbase = word_off[fd.chunk_base], obase = out_off[fd.chunk_base];
    // every wave runs the same number of iterations: the barriers below
    // are workgroup-wide
    for (int j0 = 0; j0 < kChunksPerBlock; j0 += 4) {
        const uint64_t ch = first + j0 + wave;
        const bool live = ch < fd.nchunks;
        const uint64_t s0 = ch * C + (uint64_t)lane * per;
        uint32_t bits = 0, zeros = 0;
        for (int k = 0; live && k < per; ++k) {
            const uint64_t i = s0 + k;
            if (i < fd.npts) {
                const uint16_t sym = fd.codes[i];
                bits += cb[sym] >> 24;
                zeros += sym == 0 ? 1u : 0u;
            }
        }
        uint32_t tb, tz;
        const uint32_t boffl = wave_excl_scan(bits, &tb);
        const uint32_t zoffl = wave_excl_scan(zeros, &tz);
        const int nw = live ? (int)((tb + 31) >> 5) : 0;
        for (int k = lane; k < nw; k += 64) wbuf[k] = 0;
        __syncthreads();
        uint32_t pos = boffl;
        uint32_t zo = zoffl;
        const uint64_t ow = live ? word_off[fd.chunk_base + ch] - wbase : 0;
        const uint64_t oo = live ? out_off[fd.chunk_base + ch] - obase : 0;
        for (int k = 0; live && k < per; ++k) {
            const uint64_t i = s0 + k;
            if (i >= fd.npts) break;
            const uint16_t sym = fd.codes[i];
            const uint32_t e = cb[sym];
            const uint32_t len = e >> 24, cw = e & 0xFFFFFFu;
            // codeword bits [pos, pos + len) MSB first
            const uint32_t wi = pos >> 5, bo = pos & 31;
            const uint64_t sh = (uint64_t)cw << (64 - len - bo);   // in a 64-bit window
            atomicOr(&wbuf[wi], (uint32_t)(sh >> 32));
            if (bo + len > 32) atomicOr(&wbuf[wi + 1], (uint32_t)sh);
            pos += len;
            if (sym == 0) {
                if (oo + zo < fd.n_outliers) {   // the histogram sized the list
                    fd.outlier_idx[oo + zo] = (uint32_t)i;
                    fd.outlier_val[oo + zo] = fd.in[i];
                }
                ++zo;
            }
        }
        __syncthreads();
        for (int k = lane; k < nw; k += 64)
            if (ow + k < fd.words_cap) fd.words[ow + k] = wbuf[k];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_chunk_words(const FieldDesc* __restrict__ F, int nfields,
                                                     const uint64_t* __restrict__ coff,
                                                     uint32_t* cwords, uint64_t total) {
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (uint64_t)gridDim.x * blockDim.x) {
        const int f = block_field(coff, nfields, c);
        cwords[c] = ((uint32_t)F[f].chunk_bits[c - coff[f]] + 31u) >> 5;
    }
}

// one thread decodes one chunk; canonical decode with a 2^kLutBits table
// for short codes and first-code search for longer ones
__global__ __launch_bounds__(256) void k_huff_decode(const FieldDesc* __restrict__ F, int nfields,
                                                     const uint64_t* __restrict__ boff,
                                                     const uint64_t* __restrict__ word_off,
                                                     int nsym_max) {
    extern __shared__ uint32_t tab[];
    const int f = block_field(boff, nfields, blockIdx.x);
    const FieldDesc& fd = F[f];
    const int nsym = 2 * fd.R;
    const int ntab = dtab_words(nsym);
    for (int k = threadIdx.x; k < ntab; k += blockDim.x) tab[k] = fd.dtab[k];
    __syncthreads();
    const uint64_t ch = (blockIdx.x - boff[f]) * 256 + threadIdx.x;
    if (ch >= fd.nchunks) return;
    const uint64_t wbase = word_off[fd.chunk_base];
    const uint64_t w0 = word_off[fd.chunk_base + ch] - wbase;
    const uint32_t cbits = fd.chunk_bits[ch];
    const uint64_t wend = w0 + ((cbits + 31) >> 5);
    const uint32_t* words = fd.words;
    const int C = fd.chunk;
    const uint64_t s0 = ch * C;
    const uint64_t s1 = s0 + C < fd.npts ? s0 + C : fd.npts;
    uint64_t buf = 0;   // next bits, most significant first
    int nb = 0;
    uint64_t wp = w0;
    for (uint64_t i = s0; i < s1; ++i) {
        if (nb <= 32) {
            const uint32_t wv = wp < wend ? words[wp] : 0u;
            ++wp;
            buf |= (uint64_t)wv << (32 - nb);
            nb += 32;
        }
        const uint32_t e = tab[buf >> (64 - kLutBits)];
        uint32_t len = e >> 16, sym = e & 0xFFFFu;
        if (len == 0) {
            for (int l = kLutBits + 1; l <= kLmax; ++l) {
                const uint32_t code = (uint32_t)(buf >> (64 - l));
                const uint32_t rel = code - tab[kDtFirst + l];
                if (rel < tab[kDtCount + l]) {
                    sym = tab[kDtSorted + tab[kDtOffset + l] + rel];
                    len = l;
                    break;
                }
            }
            if (len == 0) len = 1;   // corrupt stream: consume a bit and go on
        }
        fd.codes[i] = (uint16_t)sym;
        buf <<= len;
        nb -= (int)len;
    }
}

__global__ __launch_bounds__(256) void k_scatter_outliers(const FieldDesc* __restrict__ F) {
    const FieldDesc& fd = F[blockIdx.y];
    const uint64_t n = fd.npts;
    const uint64_t no = fd.n_outliers;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < no;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t idx = fd.outlier_idx[k];
        if (idx < n) fd.out[idx] = fd.outlier_val[k];
    }
}

// ------------------------------------------------------- launchers
hipError_t launch_range(const FieldDesc* d_fields, int nfields, float* d_part_min,
                        float* d_part_max, uint32_t* d_part_bad, hipStream_t st) {
    hipLaunchKernelGGL(k_range, dim3(kRangeBlocks, nfields), dim3(256), 0, st, d_fields,
                       d_part_min, d_part_max, d_part_bad);
    return hipGetLastError();
}

hipError_t launch_profile(const FieldDesc* d_fields, FieldPlan* d_plans, int nfields,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_profile, dim3(nfields), dim3(64), 0, st, d_fields, d_plans);
    return hipGetLastError();
}

hipError_t launch_plan(const FieldDesc* d_fields, FieldPlan* d_plans, int nfields,
                       const float* d_part_min, const float* d_part_max,
                       const uint32_t* d_part_bad, hipStream_t st) {
    hipLaunchKernelGGL(k_plan, dim3(nfields), dim3(256), 0, st, d_fields, d_plans, d_part_min,
                       d_part_max, d_part_bad);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_compress(int ndim, const FieldDesc* d_fields, const FieldPlan* d_plans,
                           int nfields, const uint64_t* d_item_off, uint64_t nitems, int grid,
                           int max_R, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    if ((uint64_t)grid > nitems) grid = (int)nitems;
    const size_t lds = (size_t)2 * max_R * sizeof(uint32_t);
    if (ndim == 3)
        hipLaunchKernelGGL((k_compress<3, 32, 8, 8>), dim3(grid), dim3(kThreads), lds, st,
                           d_fields, d_plans, d_item_off, nfields, nitems);
    else
        hipLaunchKernelGGL((k_compress<2, 64, 16, 1>), dim3(grid), dim3(kThreads), lds, st,
                           d_fields, d_plans, d_item_off, nfields, nitems);
    return hipGetLastError();
}

hipError_t launch_decompress(int ndim, const FieldDesc* d_fields, const FieldPlan* d_plans,
                             int nfields, const uint64_t* d_item_off, uint64_t nitems, int grid,
                             hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    if ((uint64_t)grid > nitems) grid = (int)nitems;
    if (ndim == 3)
        hipLaunchKernelGGL((k_decompress<3, 32, 8, 8>), dim3(grid), dim3(kThreads), 0, st,
                           d_fields, d_plans, d_item_off, nfields, nitems);
    else
        hipLaunchKernelGGL((k_decompress<2, 64, 16, 1>), dim3(grid), dim3(kThreads), 0, st,
                           d_fields, d_plans, d_item_off, nfields, nitems);
    return hipGetLastError();
}

// d_chunk_off here is the prefix of BLOCKS per field (kChunksPerBlock chunks each)
hipError_t launch_huff_stats(const FieldDesc* d_fields, int nfields, const uint64_t* d_block_off,
                             uint64_t nblocks, uint32_t* d_cwords, uint32_t* d_couts,
                             int max_nsym, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_huff_stats, dim3((unsigned)nblocks), dim3(256),
                       (size_t)max_nsym * sizeof(uint32_t), st, d_fields, nfields, d_block_off,
                       d_cwords, d_couts);
    return hipGetLastError();
}

hipError_t launch_scan_pairs(const uint32_t* d_a, const uint32_t* d_b, uint64_t n,
                             const uint64_t* /*d_seg_start*/, int /*nseg*/, uint64_t* d_aoff,
                             uint64_t* d_boff, uint64_t* d_totals, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_pairs, dim3(1), dim3(1024), 0, st, d_a, d_b, n, d_aoff, d_boff,
                       d_totals);
    return hipGetLastError();
}

hipError_t launch_huff_encode(const FieldDesc* d_fields, int nfields, const uint64_t* d_block_off,
                              uint64_t nblocks, const uint64_t* d_word_off,
                              const uint64_t* d_out_off, int max_nsym, int max_chunk,
                              hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const int mcw = (max_chunk * kLmax + 31) / 32 + 1;
    const size_t lds = ((size_t)max_nsym + 4 * (size_t)mcw) * sizeof(uint32_t);
    hipLaunchKernelGGL(k_huff_encode, dim3((unsigned)nblocks), dim3(256), lds, st, d_fields,
                       nfields, d_block_off, d_word_off, d_out_off, mcw);
    return hipGetLastError();
}

hipError_t launch_scan_words(const FieldDesc* d_fields, int nfields, const uint64_t* d_chunk_off,
                             uint64_t nchunks_total, uint32_t* d_tmp, uint64_t* d_word_off,
                             hipStream_t st) {
    if (nchunks_total == 0) return hipSuccess;
    uint64_t blocks = (nchunks_total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_chunk_words, dim3((unsigned)blocks), dim3(256), 0, st, d_fields, nfields,
                       d_chunk_off, d_tmp, nchunks_total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // totals land past the end of the offsets array
    hipLaunchKernelGGL(k_scan_pairs, dim3(1), dim3(1024), 0, st, d_tmp, (const uint32_t*)nullptr,
                       nchunks_total, d_word_off, (uint64_t*)nullptr, d_word_off + nchunks_total);
    return hipGetLastError();
}

// d_chunk_off: prefix of DECODE blocks (256 chunks each) per field
hipError_t launch_huff_decode(const FieldDesc* d_fields, int nfields, const uint64_t* d_block_off,
                              uint64_t nblocks, const uint64_t* d_word_off, int max_nsym,
                              hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const size_t lds = (size_t)dtab_words(max_nsym) * sizeof(uint32_t);
    hipLaunchKernelGGL(k_huff_decode, dim3((unsigned)nblocks), dim3(256), lds, st, d_fields,
                       nfields, d_block_off, d_word_off, max_nsym);
    return hipGetLastError();
}

hipError_t launch_scatter_outliers(const FieldDesc* d_fields, int nfields, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_outliers, dim3(256, nfields), dim3(256), 0, st, d_fields);
    return hipGetLastError();
}

}  // namespace szi
