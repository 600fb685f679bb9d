// k_interp.hip -- the G-Interp predictor-quantiser (compression) and its
// replay (decompression) on gfx950 (Sec. V-A, V-B, V-D; Sec. III-A).
//
// One window per iteration of a persistent workgroup of 4 wave64.  A window
// owns the points [lo, lo + W) of each dimension; its block adds the far
// faces (lo + W).  Neighbours are searched inside the point's own window
// interval along the pass dimension only, so the faces shared by two windows
// are computed identically by both and windows are independent.  Levels run
// from stride S/2 to 1; at each level one pass per dimension in the planned
// order, separated by workgroup barriers.  The block lives in LDS; a pass
// reads neighbours and replaces values in place (points of one pass never
// neighbour each other along the pass dimension).
//
// Arithmetic: every FP32 expression is evaluated in the order written, one
// rounding per operation (the library is built with -ffp-contract=off).
#include "dev_common.h"

namespace szi {

constexpr int kLoadBatch = 11;  // global loads in flight per thread while staging a block

template <int ND, int W0, int W1, int W2>
struct Geom {
    static constexpr int B0 = W0 + 1;
    static constexpr int B1 = W1 + 1;
    static constexpr int B2 = ND == 3 ? W2 + 1 : 1;
    static constexpr int BN = B0 * B1 * B2;
    static constexpr int O2 = ND == 3 ? W2 : 1;
    static constexpr int OWN = W0 * W1 * O2;
    static constexpr int PER = (BN + kThreads - 1) / kThreads;   // block points per thread
};

struct WinInfo {
    int lo0, lo1, lo2;
    int e0, e1, e2;      // block extents (own points + far face where present)
    int o0, o1, o2;      // owned extents
    bool full;
    uint32_t gbase;      // linear index of the window origin
};

template <int ND, int W0, int W1, int W2>
__device__ __forceinline__ void window_info(const FieldDesc& f, uint64_t w, WinInfo& wi) {
    const uint32_t nw0 = (uint32_t)f.nwin[0], nw1 = (uint32_t)f.nwin[1];
    const uint32_t wz = (uint32_t)(w / ((uint64_t)nw0 * nw1));
    const uint32_t r = (uint32_t)(w - (uint64_t)wz * nw0 * nw1);
    const uint32_t wy = r / nw0;
    const uint32_t wx = r - wy * nw0;
    wi.lo0 = (int)wx * W0;
    wi.lo1 = (int)wy * W1;
    wi.lo2 = ND == 3 ? (int)wz * W2 : 0;
    const int s0 = f.n[0] - 1 - wi.lo0, s1 = f.n[1] - 1 - wi.lo1;
    const int s2 = ND == 3 ? f.n[2] - 1 - wi.lo2 : 0;
    wi.e0 = (s0 < W0 ? s0 : W0) + 1;
    wi.e1 = (s1 < W1 ? s1 : W1) + 1;
    wi.e2 = ND == 3 ? (s2 < W2 ? s2 : W2) + 1 : 1;
    wi.o0 = wi.e0 < W0 ? wi.e0 : W0;
    wi.o1 = wi.e1 < W1 ? wi.e1 : W1;
    wi.o2 = ND == 3 ? (wi.e2 < W2 ? wi.e2 : W2) : 1;
    wi.full = wi.e0 == W0 + 1 && wi.e1 == W1 + 1 && (ND == 2 || wi.e2 == W2 + 1);
    wi.gbase = (uint32_t)wi.lo0 + (uint32_t)wi.lo1 * (uint32_t)f.n[0] +
               (uint32_t)wi.lo2 * (uint32_t)f.n[0] * (uint32_t)f.n[1];
}

// The thread index, made opaque to the optimiser: per-thread offsets that
// only depend on it would otherwise be hoisted out of the window loop and
// held in registers for the whole kernel.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Points of pass (level lvl, k-th dimension of the order): along the pass
// dimension the odd multiples of s, along dimensions already passed at this
// level the multiples of s, along those still to come the multiples of 2s
// (s = 2^(lvl-1)).
struct PassGrid {
    int st0, st1, st2;
    int sh0, sh1, sh2;
    int m0, m1, m2;
    uint32_t total;
    FastDiv d0, d01;
};

__device__ __forceinline__ int order_pos(int o0, int o1, int j) {
    return o0 == j ? 0 : (o1 == j ? 1 : 2);
}

__device__ __forceinline__ void pass_axis(int kj, int k, int lvl, int ext, int& st, int& sh,
                                          int& m) {
    st = kj == k ? (1 << (lvl - 1)) : 0;
    sh = kj < k ? lvl - 1 : lvl;
    m = ext > st ? ((ext - 1 - st) >> sh) + 1 : 0;
}

template <int ND>
__device__ __forceinline__ void pass_grid(PassGrid& g, int o0, int o1, int k, int lvl, int e0,
                                          int e1, int e2) {
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

// Sec. V-B.1 splines by neighbour availability.  b is always present; a,
// c, d are read from clamped addresses (their own point when absent) and
// then ignored.  spl is uniform across the pass.
__device__ __forceinline__ float predict(int spl, bool m3, bool p1, bool p3, float a, float b,
                                         float c, float d) {
    const float sbc = b + c;
    float p = sbc * 0.5f;                          // linear
    if (spl != SPL_LIN) {
        // quadratic: (-1/8, 6/8, 3/8) on (a, b, c) or (3/8, 6/8, -1/8) on (b, c, d)
        const float wb = m3 ? 6.0f : 3.0f, wc = m3 ? 3.0f : 6.0f;
        const float e = m3 ? a : d;
        const float pq = ((wb * b + wc * c) - e) * 0.125f;
        const float sad = a + d;
        float pc;
        if (spl == SPL_NAT)
            pc = (23.0f * sbc - 3.0f * sad) / 40.0f;   // natural cubic
        else
            pc = (9.0f * sbc - sad) * 0.0625f;         // not-a-knot cubic
        p = (m3 && p3) ? pc : ((m3 || p3) ? pq : p);
    }
    return p1 ? p : b;                             // one neighbour: x[n-1]
}

// One point of a pass: the prediction along the pass dimension, then
// either the closed-loop quantisation (compression) or the replay.
template <bool COMP>
__device__ __forceinline__ void point(float* v, uint16_t* q, int li, bool m3, bool p1, bool p3,
                                      int s1, int s3, int spl, float el, float ebx2, float inv,
                                      float Rf, double eld, int R) {
    const float b = v[li - s1];
    const float c = v[p1 ? li + s1 : li];
    const float a = v[m3 ? li - s3 : li];
    const float dd = v[p3 ? li + s3 : li];
    const float p = predict(spl, m3, p1, p3, a, b, c, dd);
    if (COMP) {
        const float x = v[li];
        const float diff = x - p;
        bool outl;
        float qr = 0.0f;
        float xr = p;
        if (el == 0.0f) {   // uniform: keep exact predictions only
            outl = !(diff == 0.0f);
        } else {
            const float qf = diff * inv;
            qr = rintf(qf);                            // round half to even
            // |rint(qf)| < R is equivalent to |qf| < R and |q| < R (R is an
            // integer); NaN and Inf fail it
            outl = !(fabsf(qr) < Rf);
            xr = p + qr * ebx2;                        // qr is an exact small integer
            outl = outl || !(fabs((double)x - (double)xr) <= eld);
        }
        v[li] = outl ? x : xr;
        q[li] = outl ? (uint16_t)0 : (uint16_t)((int)qr + R);
    } else {
        const int code = q[li];
        if (code != 0) v[li] = p + (float)(code - R) * ebx2;
    }
}

// pass over the points of one (level, dimension) of a partial window
template <int ND, class G, bool COMP>
__device__ __forceinline__ void run_pass(float* v, uint16_t* q, const PassGrid& g, int d, int s,
                                         int ed, int spl, float el, float ebx2, float inv,
                                         int R) {
    const int sd = d == 0 ? 1 : (d == 1 ? G::B0 : G::B0 * G::B1);
    const int s1 = s * sd, s3 = 3 * s * sd;
    const float Rf = (float)R;
    const double eld = (double)el;
    for (uint32_t t = opaque_tid(); t < g.total; t += kThreads) {
        const uint32_t i2 = g.d01.div(t);
        const uint32_t r = t - i2 * g.d01.m;
        const uint32_t i1 = g.d0.div(r);
        const uint32_t i0 = r - i1 * g.d0.m;
        const int c0 = g.st0 + ((int)i0 << g.sh0);
        const int c1 = g.st1 + ((int)i1 << g.sh1);
        const int c2 = g.st2 + ((int)i2 << g.sh2);
        const int li = c0 + G::B0 * (c1 + G::B1 * c2);
        const int cd = d == 0 ? c0 : (d == 1 ? c1 : c2);
        point<COMP>(v, q, li, cd >= 3 * s, cd + s < ed, cd + 3 * s < ed, s1, s3, spl, el, ebx2,
                    inv, Rf, eld, R);
    }
}

// pass over the points of one (level, dimension) of a full window, listed
// in the pass table (LDS)
template <int ND, class G, bool COMP>
__device__ __forceinline__ void run_pass_tab(float* v, uint16_t* q, const uint16_t* ptab,
                                             uint32_t off, uint32_t cnt, uint32_t ncub, int d,
                                             int s, int spl, float el, float ebx2, float inv,
                                             int R) {
    const int sd = d == 0 ? 1 : (d == 1 ? G::B0 : G::B0 * G::B1);
    const int s1 = s * sd, s3 = 3 * s * sd;
    const float Rf = (float)R;
    const double eld = (double)el;
    for (uint32_t t = opaque_tid(); t < cnt; t += kThreads) {
        const uint32_t e = ptab[off + t];
        if (t < ncub)   // all four neighbours: the cubic stencil, no selects
            point<COMP>(v, q, (int)(e & 0xFFFu), true, true, true, s1, s3, spl, el, ebx2, inv, Rf,
                        eld, R);
        else
            point<COMP>(v, q, (int)(e & 0xFFFu), (e >> 12) & 1u, true, (e >> 13) & 1u, s1, s3,
                        spl, el, ebx2, inv, Rf, eld, R);
    }
}

// extents are passed as separate scalars: selecting a struct member by a
// runtime dimension index would make the compiler address it in memory
// Per-pass parameters of a field, kept in LDS so that a pass reads them with
// one LDS access instead of dependent global loads of the plan.
struct PassParam {
    int32_t d, s, spl, sd;     // pass dimension, stride, spline, LDS stride along d
    float el, ebx2, inv;       // level bound, 2*e_l, 1/(2*e_l)
    int32_t lvl;
};

template <int ND, class G, bool COMP, bool FULL>
__device__ __forceinline__ void run_levels(float* v, uint16_t* q, const uint16_t* ptab,
                                           const uint32_t* pmeta, const PassParam* pp,
                                           int o0, int o1, int L, int R, int e0, int e1, int e2) {
    const int npass = ND * L;
    for (int pass = 0; pass < npass; ++pass) {
        const PassParam r = pp[pass];
        if (FULL) {
            run_pass_tab<ND, G, COMP>(v, q, ptab, pmeta[pass], pmeta[kMaxPasses + pass],
                                      pmeta[2 * kMaxPasses + pass], r.d, r.s, r.spl, r.el, r.ebx2,
                                      r.inv, R);
        } else {
            const int ed = r.d == 0 ? e0 : (r.d == 1 ? e1 : e2);
            PassGrid g;
            pass_grid<ND>(g, o0, o1, pass % ND, r.lvl, e0, e1, e2);
            run_pass<ND, G, COMP>(v, q, g, r.d, r.s, ed, r.spl, r.el, r.ebx2, r.inv, R);
        }
        __syncthreads();
    }
}

template <int ND, class G>
__device__ __forceinline__ void load_pass_params(PassParam* pp, const FieldPlan& pl, int L) {
    const int npass = ND * L;
    const int p = threadIdx.x;
    if (p < npass) {
        const int lvl = L - p / ND, k = p % ND;
        const int d = pl.order[k];
        PassParam r;
        r.d = d;
        r.s = 1 << (lvl - 1);
        r.spl = pl.spline[d];
        r.sd = d == 0 ? 1 : (d == 1 ? G::B0 : G::B0 * G::B1);
        r.el = pl.el[lvl - 1];
        r.ebx2 = pl.ebx2[lvl - 1];
        r.inv = pl.inv[lvl - 1];
        r.lvl = lvl;
        pp[p] = r;
    }
}

// copy the pass table of the field's order into LDS (after a barrier)
template <int ND, class G>
__device__ __forceinline__ void load_pass_table(uint16_t* ptab, uint32_t* pmeta,
                                                const uint16_t* __restrict__ gtab,
                                                const PassMeta* __restrict__ gmeta,
                                                const FieldPlan& pl) {
    const int id = ND == 3 ? 2 * pl.order[0] + (pl.order[1] > pl.order[2] ? 1 : 0) : pl.order[0];
    const PassMeta& m = gmeta[id];
    if (threadIdx.x < kMaxPasses) {
        pmeta[threadIdx.x] = m.off[threadIdx.x] - m.off[0];
        pmeta[kMaxPasses + threadIdx.x] = m.cnt[threadIdx.x];
        pmeta[2 * kMaxPasses + threadIdx.x] = m.ncub[threadIdx.x];
    }
    uint32_t total = 0;
    for (int p = 0; p < ND * (ND == 3 ? 3 : 4); ++p) total += m.cnt[p];
    const SZI_G uint16_t* src = gp(gtab) + m.off[0];
    // rare path (once per field): keep it from holding many registers
#pragma unroll 1
    for (uint32_t t = threadIdx.x; t < total; t += kThreads) ptab[t] = src[t];
}

// block point t -> block coordinates, for a full window (constant extents)
// or a partial one (runtime extents)
template <class G, bool FULL>
__device__ __forceinline__ void block_coord(uint32_t t, const FastDiv& e0, const FastDiv& e01,
                                            uint32_t& c0, uint32_t& c1, uint32_t& c2) {
    if (FULL) {
        c2 = t / (G::B0 * G::B1);
        const uint32_t r = t - c2 * (G::B0 * G::B1);
        c1 = r / G::B0;
        c0 = r - c1 * G::B0;
    } else {
        c2 = e01.div(t);
        const uint32_t r = t - c2 * e01.m;
        c1 = e0.div(r);
        c0 = r - c1 * e0.m;
    }
}

template <int ND, int W0, int W1, int W2, bool FULL>
__device__ __forceinline__ void compress_window(float* v, uint16_t* q, uint32_t* hist,
                                                uint32_t& cntR, const uint16_t* ptab,
                                                const uint32_t* pmeta, const PassParam* pp,
                                                const FieldDesc& fd,
                                                const FieldPlan& pl, const WinInfo& wi) {
    using G = Geom<ND, W0, W1, W2>;
    const int tid = opaque_tid();
    const uint32_t n0 = (uint32_t)fd.n[0];
    const uint32_t n01 = n0 * (uint32_t)fd.n[1];
    const SZI_G float* base = gp(fd.in) + wi.gbase;
    // load: every load of the block in flight before the first LDS store
    {
        FastDiv e0, e01;
        e0.set((uint32_t)wi.e0);
        e01.set((uint32_t)(wi.e0 * wi.e1));
        const uint32_t tot = FULL ? (uint32_t)G::BN : (uint32_t)(wi.e0 * wi.e1 * wi.e2);
        // batches of kLoadBatch loads in flight per thread
        for (int k0 = 0; k0 < G::PER; k0 += kLoadBatch) {
            float val[kLoadBatch];
            int li[kLoadBatch];
#pragma unroll
            for (int k = 0; k < kLoadBatch; ++k) {
                const uint32_t t = tid + (k0 + k) * kThreads;
                li[k] = -1;
                if (t < tot) {
                    uint32_t c0, c1, c2;
                    block_coord<G, FULL>(t, e0, e01, c0, c1, c2);
                    li[k] = (int)(c0 + G::B0 * (c1 + G::B1 * c2));
                    val[k] = base[c0 + c1 * n0 + c2 * n01];
                }
            }
#pragma unroll
            for (int k = 0; k < kLoadBatch; ++k)
                if (li[k] >= 0) v[li[k]] = val[k];
        }
    }
    __syncthreads();
    run_levels<ND, G, true, FULL>(v, q, ptab, pmeta, pp, pl.order[0], pl.order[1], fd.L, fd.R,
                                  wi.e0, wi.e1, wi.e2);
    // owned codes (anchors carry R), anchors, histogram
    const int R = fd.R;
    const int smask = fd.S - 1;
    const int shS = __builtin_ctz((unsigned)fd.S);
    if (FULL && (n0 & 1) == 0) {
        // pairs of x-neighbours: one 32-bit store per two codes
        constexpr int HX = W0 / 2;
        constexpr int NP = HX * W1 * G::O2;
        for (int t = tid; t < NP; t += kThreads) {
            const int px = t % HX, row = t / HX;
            const int c1 = row % W1, c2 = row / W1;
            const int c0 = 2 * px;
            const int li = c0 + G::B0 * (c1 + G::B1 * c2);
            const bool arow = ((c1 | c2) & smask) == 0;
            const bool a0 = arow && (c0 & smask) == 0;   // c0 + 1 is odd: never an anchor
            const uint32_t qa = a0 ? (uint32_t)R : q[li];
            const uint32_t qb = q[li + 1];
            const uint32_t g = wi.gbase + c0 + c1 * n0 + c2 * n01;
            *reinterpret_cast<SZI_G uint32_t*>(gp(fd.codes) + g) = qa | (qb << 16);
            if (a0) {
                const uint32_t ax = (uint32_t)(wi.lo0 + c0) >> shS;
                const uint32_t ay = (uint32_t)(wi.lo1 + c1) >> shS;
                const uint32_t az = (uint32_t)(wi.lo2 + c2) >> shS;
                gp(fd.anchors)[ax + (uint32_t)fd.na[0] * (ay + (uint32_t)fd.na[1] * az)] = v[li];
            }
            if (qa == (uint32_t)R) ++cntR; else atomicAdd(&hist[qa], 1u);
            if (qb == (uint32_t)R) ++cntR; else atomicAdd(&hist[qb], 1u);
        }
    } else {
        FastDiv o0, o01;
        o0.set((uint32_t)wi.o0);
        o01.set((uint32_t)(wi.o0 * wi.o1));
        const uint32_t tot = (uint32_t)(wi.o0 * wi.o1 * wi.o2);
        for (uint32_t t = tid; t < tot; t += kThreads) {
            const uint32_t c2 = o01.div(t);
            const uint32_t r = t - c2 * o01.m;
            const uint32_t c1 = o0.div(r);
            const uint32_t c0 = r - c1 * o0.m;
            const int li = c0 + G::B0 * (c1 + G::B1 * c2);
            const bool anchor = ((c0 | c1 | c2) & smask) == 0;
            const uint32_t code = anchor ? (uint32_t)R : q[li];
            gp(fd.codes)[wi.gbase + c0 + c1 * n0 + c2 * n01] = (uint16_t)code;
            if (anchor) {
                const uint32_t ax = (uint32_t)(wi.lo0 + c0) >> shS;
                const uint32_t ay = (uint32_t)(wi.lo1 + c1) >> shS;
                const uint32_t az = (uint32_t)(wi.lo2 + c2) >> shS;
                gp(fd.anchors)[ax + (uint32_t)fd.na[0] * (ay + (uint32_t)fd.na[1] * az)] = v[li];
            }
            if (code == (uint32_t)R) ++cntR; else atomicAdd(&hist[code], 1u);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void flush_hist(uint32_t* hist, uint32_t& cntR, const FieldDesc& fd) {
    const uint32_t s = wave_sum(cntR);
    cntR = 0;
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(&hist[fd.R], s);
    __syncthreads();
#pragma unroll 1
    for (int b = threadIdx.x; b < 2 * fd.R; b += kThreads)
        if (hist[b]) gatomic_add(gp(fd.hist) + b, hist[b]);
    __syncthreads();
}

template <int ND, int W0, int W1, int W2>
__global__ __launch_bounds__(kThreads) void k_compress(const FieldDesc* __restrict__ F,
                                                       const FieldPlan* __restrict__ P,
                                                       const uint64_t* __restrict__ item_off,
                                                       int nfields, uint64_t nitems,
                                                       const uint16_t* __restrict__ gtab,
                                                       const PassMeta* __restrict__ gmeta) {
    using G = Geom<ND, W0, W1, W2>;
    __shared__ float v[G::BN];
    __shared__ uint16_t q[G::BN + 1];
    __shared__ uint16_t ptab[G::BN + 1];
    __shared__ uint32_t pmeta[3 * kMaxPasses];
    __shared__ PassParam pp[kMaxPasses];
    extern __shared__ uint32_t hist[];
    int f = 0, cur = -1;
    uint32_t cntR = 0;   // thread-private count of the centre code (Sec. VI-A, top-1 cache)
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        while (it >= item_off[f + 1]) ++f;
        if (f != cur) {
            if (cur >= 0) flush_hist(hist, cntR, F[cur]);
            cur = f;
#pragma unroll 1
            for (int b = threadIdx.x; b < 2 * F[cur].R; b += kThreads) hist[b] = 0;
            load_pass_table<ND, G>(ptab, pmeta, gtab, gmeta, P[f]);
            load_pass_params<ND, G>(pp, P[f], F[f].L);
            __syncthreads();
        }
        const FieldDesc& fd = F[f];
        const FieldPlan& pl = P[f];
        WinInfo wi;
        window_info<ND, W0, W1, W2>(fd, it - item_off[f], wi);
        if (wi.full)
            compress_window<ND, W0, W1, W2, true>(v, q, hist, cntR, ptab, pmeta, pp, fd, pl, wi);
        else
            compress_window<ND, W0, W1, W2, false>(v, q, hist, cntR, ptab, pmeta, pp, fd, pl, wi);
    }
    if (cur >= 0) flush_hist(hist, cntR, F[cur]);
}

template <int ND, int W0, int W1, int W2, bool FULL>
__device__ __forceinline__ void decompress_window(float* v, uint16_t* q, const uint16_t* ptab,
                                                  const uint32_t* pmeta, const PassParam* pp,
                                                  const FieldDesc& fd,
                                                  const FieldPlan& pl, const WinInfo& wi) {
    using G = Geom<ND, W0, W1, W2>;
    const int tid = opaque_tid();
    const uint32_t n0 = (uint32_t)fd.n[0];
    const uint32_t n01 = n0 * (uint32_t)fd.n[1];
    const int smask = fd.S - 1;
    const int shS = __builtin_ctz((unsigned)fd.S);
    {
        FastDiv e0, e01;
        e0.set((uint32_t)wi.e0);
        e01.set((uint32_t)(wi.e0 * wi.e1));
        const uint32_t tot = FULL ? (uint32_t)G::BN : (uint32_t)(wi.e0 * wi.e1 * wi.e2);
        for (int k0 = 0; k0 < G::PER; k0 += kLoadBatch) {
            uint32_t code[kLoadBatch], gi[kLoadBatch];
            int li[kLoadBatch];
            uint32_t ai[kLoadBatch];   // anchor index + 1, or 0
#pragma unroll
            for (int k = 0; k < kLoadBatch; ++k) {
                const uint32_t t = tid + (k0 + k) * kThreads;
                li[k] = -1;
                if (t < tot) {
                    uint32_t c0, c1, c2;
                    block_coord<G, FULL>(t, e0, e01, c0, c1, c2);
                    li[k] = (int)(c0 + G::B0 * (c1 + G::B1 * c2));
                    gi[k] = wi.gbase + c0 + c1 * n0 + c2 * n01;
                    code[k] = gp(fd.codes)[gi[k]];
                    ai[k] = 0;
                    if (((c0 | c1 | c2) & smask) == 0) {
                        const uint32_t ax = (uint32_t)(wi.lo0 + c0) >> shS;
                        const uint32_t ay = (uint32_t)(wi.lo1 + c1) >> shS;
                        const uint32_t az = (uint32_t)(wi.lo2 + c2) >> shS;
                        ai[k] = 1 + ax + (uint32_t)fd.na[0] * (ay + (uint32_t)fd.na[1] * az);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < kLoadBatch; ++k) {
                if (li[k] < 0) continue;
                q[li[k]] = (uint16_t)code[k];
                if (ai[k])
                    v[li[k]] = gp(fd.anchors)[ai[k] - 1];
                else if (code[k] == 0)
                    v[li[k]] = gp(fd.out)[gi[k]];   // outlier, scattered before the replay
            }
        }
    }
    __syncthreads();
    run_levels<ND, G, false, FULL>(v, q, ptab, pmeta, pp, pl.order[0], pl.order[1], fd.L, fd.R,
                                   wi.e0, wi.e1, wi.e2);
    if (FULL && (n0 & 1) == 0) {
        constexpr int HX = W0 / 2;
        constexpr int NP = HX * W1 * G::O2;
        for (int t = tid; t < NP; t += kThreads) {
            const int px = t % HX, row = t / HX;
            const int c1 = row % W1, c2 = row / W1;
            const int c0 = 2 * px;
            const int li = c0 + G::B0 * (c1 + G::B1 * c2);
            typedef float vf2 __attribute__((ext_vector_type(2)));
            vf2 o;
            o.x = v[li];
            o.y = v[li + 1];
            *reinterpret_cast<SZI_G vf2*>(gp(fd.out) + wi.gbase + c0 + c1 * n0 + c2 * n01) = o;
        }
    } else {
        FastDiv o0, o01;
        o0.set((uint32_t)wi.o0);
        o01.set((uint32_t)(wi.o0 * wi.o1));
        const uint32_t tot = (uint32_t)(wi.o0 * wi.o1 * wi.o2);
        for (uint32_t t = tid; t < tot; t += kThreads) {
            const uint32_t c2 = o01.div(t);
            const uint32_t r = t - c2 * o01.m;
            const uint32_t c1 = o0.div(r);
            const uint32_t c0 = r - c1 * o0.m;
            gp(fd.out)[wi.gbase + c0 + c1 * n0 + c2 * n01] = v[c0 + G::B0 * (c1 + G::B1 * c2)];
        }
    }
    __syncthreads();
}

template <int ND, int W0, int W1, int W2>
__global__ __launch_bounds__(kThreads) void k_decompress(const FieldDesc* __restrict__ F,
                                                         const FieldPlan* __restrict__ P,
                                                         const uint64_t* __restrict__ item_off,
                                                         int nfields, uint64_t nitems,
                                                         const uint16_t* __restrict__ gtab,
                                                         const PassMeta* __restrict__ gmeta) {
    using G = Geom<ND, W0, W1, W2>;
    __shared__ float v[G::BN];
    __shared__ uint16_t q[G::BN + 1];
    __shared__ uint16_t ptab[G::BN + 1];
    __shared__ uint32_t pmeta[3 * kMaxPasses];
    __shared__ PassParam pp[kMaxPasses];
    int f = 0, cur = -1;
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        while (it >= item_off[f + 1]) ++f;
        if (f != cur) {
            cur = f;
            load_pass_table<ND, G>(ptab, pmeta, gtab, gmeta, P[f]);
            load_pass_params<ND, G>(pp, P[f], F[f].L);
            __syncthreads();
        }
        const FieldDesc& fd = F[f];
        WinInfo wi;
        window_info<ND, W0, W1, W2>(fd, it - item_off[f], wi);
        if (wi.full)
            decompress_window<ND, W0, W1, W2, true>(v, q, ptab, pmeta, pp, fd, P[f], wi);
        else
            decompress_window<ND, W0, W1, W2, false>(v, q, ptab, pmeta, pp, fd, P[f], wi);
    }
}

// ------------------------------------------------------- launchers
// The persistent grid is the number of workgroups resident at once
// (occupancy from the runtime x compute units) unless per_cu overrides it.
template <class K>
static int resident_grid(K kernel, size_t lds, int num_cus, int per_cu) {
    if (per_cu > 0) return num_cus * per_cu;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kThreads, lds) != hipSuccess ||
        occ < 1) {
        (void)hipGetLastError();
        occ = 4;
    }
    return num_cus * occ;
}

hipError_t launch_compress(int ndim, const FieldDesc* d_fields, const FieldPlan* d_plans,
                           int nfields, const uint64_t* d_item_off, uint64_t nitems,
                           const uint16_t* d_ptab, const PassMeta* d_pmeta, int num_cus,
                           int per_cu, int max_R, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    const size_t lds = (size_t)2 * max_R * sizeof(uint32_t);
    if (ndim == 3) {
        auto k = k_compress<3, 32, 8, 8>;
        uint64_t grid = (uint64_t)resident_grid(k, lds, num_cus, per_cu);
        if (grid > nitems) grid = nitems;
        hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kThreads), lds, st, d_fields, d_plans,
                           d_item_off, nfields, nitems, d_ptab, d_pmeta);
    } else {
        auto k = k_compress<2, 64, 16, 1>;
        uint64_t grid = (uint64_t)resident_grid(k, lds, num_cus, per_cu);
        if (grid > nitems) grid = nitems;
        hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kThreads), lds, st, d_fields, d_plans,
                           d_item_off, nfields, nitems, d_ptab, d_pmeta);
    }
    return hipGetLastError();
}

hipError_t launch_decompress(int ndim, const FieldDesc* d_fields, const FieldPlan* d_plans,
                             int nfields, const uint64_t* d_item_off, uint64_t nitems,
                             const uint16_t* d_ptab, const PassMeta* d_pmeta, int num_cus,
                             int per_cu, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    if (ndim == 3) {
        auto k = k_decompress<3, 32, 8, 8>;
        uint64_t grid = (uint64_t)resident_grid(k, 0, num_cus, per_cu);
        if (grid > nitems) grid = nitems;
        hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kThreads), 0, st, d_fields, d_plans,
                           d_item_off, nfields, nitems, d_ptab, d_pmeta);
    } else {
        auto k = k_decompress<2, 64, 16, 1>;
        uint64_t grid = (uint64_t)resident_grid(k, 0, num_cus, per_cu);
        if (grid > nitems) grid = nitems;
        hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kThreads), 0, st, d_fields, d_plans,
                           d_item_off, nfields, nitems, d_ptab, d_pmeta);
    }
    return hipGetLastError();
}

}  // namespace szi
