// k_interp.hip -- the G-Interp predictor-quantiser (compression) and its
// replay (decompression) on gfx950 (Sec. V-A, V-B, V-D; Sec. III-A).
//
// One wave64 per window, kWaves windows per workgroup.  A window owns the
// points [lo, lo + W) of each dimension; its block adds the far faces
// (lo + W), which the next window owns.  Neighbours are searched inside the
// point's own window interval along the pass dimension only, so a face point
// is computed identically by both windows that hold it and windows are
// independent.  A wave stages its block in LDS, runs the passes (levels from
// stride S/2 down to 1, one pass per dimension in the planned order) without
// any workgroup barrier, and writes out the points it owns.  The block of
// the wave's next window is loaded into registers while the current one is
// processed.
//
// A pass along dimension d at stride s works on lines: block points that
// share every coordinate but d.  The targets of a line are its odd multiples
// of s, its knowns the even ones.  A lane takes K consecutive targets of one
// line, reads the K + 3 knowns around them once, and predicts all K; every
// LDS offset along the line is a compile-time constant.
//
// Arithmetic: every FP32 expression is evaluated in the order written, one
// rounding per operation (the library is built with -ffp-contract=off).
#include "dev_common.h"

#include <map>
#include <mutex>

namespace szi {

constexpr int kWaves = kWinPerGroup;    // windows in flight per workgroup, one per wave
static_assert(kWaves * 64 == kThreads, "one wave per window of a group");
constexpr int kPad = 8;                 // guard floats on both sides of a block in LDS
constexpr int kXcds = 8;                // L2 domains; workgroup i runs on domain i % kXcds

template <int ND>
constexpr int vlen() { return kPad + Geo<ND>::BN + kPad; }

// The window a wave works on.  Every member is wave-uniform.
struct Win {
    uint64_t gbase;          // linear index of the window origin
    uint32_t n0, n01;        // field strides
    int lo0, lo1, lo2;       // origin
    int e0, e1, e2;          // block extents (owned points + far face where present)
    uint32_t op;             // owned extents o0 | o1 << 8 | o2 << 16 (each at most 64)
    bool full;
    __device__ int own(int d) const { return (int)((op >> (8 * d)) & 255u); }
};

template <int ND>
__device__ __forceinline__ Win make_win(const FieldDesc& f, uint32_t w) {
    using G = Geo<ND>;
    Win wi;
    const uint32_t nw0 = (uint32_t)f.nwin[0];
    const uint32_t nw01 = nw0 * (uint32_t)f.nwin[1];
    const uint32_t wz = w / nw01;
    const uint32_t r = w - wz * nw01;
    const uint32_t wy = r / nw0;
    const uint32_t wx = r - wy * nw0;
    wi.n0 = (uint32_t)f.n[0];
    wi.n01 = wi.n0 * (uint32_t)f.n[1];
    wi.lo0 = (int)wx * G::W0;
    wi.lo1 = (int)wy * G::W1;
    wi.lo2 = ND == 3 ? (int)wz * G::W2 : 0;
    const int s0 = f.n[0] - 1 - wi.lo0, s1 = f.n[1] - 1 - wi.lo1;
    const int s2 = ND == 3 ? f.n[2] - 1 - wi.lo2 : 0;
    wi.e0 = (s0 < G::W0 ? s0 : G::W0) + 1;
    wi.e1 = (s1 < G::W1 ? s1 : G::W1) + 1;
    wi.e2 = ND == 3 ? (s2 < G::W2 ? s2 : G::W2) + 1 : 1;
    const int o0 = wi.e0 < G::W0 ? wi.e0 : G::W0;
    const int o1 = wi.e1 < G::W1 ? wi.e1 : G::W1;
    const int o2 = ND == 3 ? (wi.e2 < G::W2 ? wi.e2 : G::W2) : 1;
    static_assert(G::W0 < 256 && G::W1 < 256 && G::W2 < 256, "owned extents fit 8 bits");
    wi.op = (uint32_t)o0 | ((uint32_t)o1 << 8) | ((uint32_t)o2 << 16);
    wi.full = wi.e0 == G::B0 && wi.e1 == G::B1 && (ND == 2 || wi.e2 == G::B2);
    wi.gbase = (uint64_t)wi.lo0 + (uint64_t)wi.lo1 * wi.n0 + (uint64_t)wi.lo2 * wi.n01;
    return wi;
}

// byte offset from a window origin: the 64-bit base stays in scalar
// registers and the per-lane part is a 32-bit offset (the host bounds the
// span of a window below 4 GiB)
template <class T>
__device__ __forceinline__ const SZI_G T* at(const SZI_G T* base, uint32_t off) {
    return (const SZI_G T*)((const SZI_G char*)base + (off * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ SZI_G T* at(SZI_G T* base, uint32_t off) {
    return (SZI_G T*)((SZI_G char*)base + (off * (uint32_t)sizeof(T)));
}

// ------------------------------------------------------------ block staging
// Slots of the block load, NPRE per lane; slot k of a lane is a (global
// offset from the window origin, LDS index) pair and whether the lane holds
// a point of the block there (of its in-extent part, for partial windows).
// 3D: slots 0-35 hold rows (y, z) and (y, z + 4) of planes 0-7 (lanes 0-31
// and 32-63, x = lane % 32), slots 36-40 rows (y, 8) and (y + 5, 8), slots
// 41-42 the x = 32 column (row = lane and lane + 64).  2D: slots 0-16 rows
// y (x = lane), slot 17 the x = 64 column (row = lane).
template <int ND>
struct LaneMap;

template <>
struct LaneMap<3> {
    uint32_t x, hi;
    uint32_t gA, gB, gC0, gC1;   // per-lane global offsets
    int yc0, zc0, yc1, zc1;      // column rows
    __device__ __forceinline__ void init(uint32_t lane, uint32_t n0, uint32_t n01) {
        x = lane & 31u;
        hi = lane >> 5;
        gA = x + hi * 4u * n01;
        gB = x + hi * 5u * n0;
        yc0 = (int)(lane % 9u);
        zc0 = (int)(lane / 9u);
        yc1 = (int)((lane + 64u) % 9u);
        zc1 = (int)((lane + 64u) / 9u);
        gC0 = 32u + (uint32_t)yc0 * n0 + (uint32_t)zc0 * n01;
        gC1 = 32u + (uint32_t)yc1 * n0 + (uint32_t)zc1 * n01;
    }
    template <bool FULL>
    __device__ __forceinline__ bool slot(int k, const Win& wi, uint32_t& g, int& l) const {
        if (k < 36) {
            const int zl = k / 9, y = k % 9;
            g = (uint32_t)y * wi.n0 + (uint32_t)zl * wi.n01 + gA;
            l = zl * 297 + y * 33 + (int)x + (int)hi * (4 * 297);
            return FULL || ((int)x < wi.e0 && y < wi.e1 && zl + 4 * (int)hi < wi.e2);
        } else if (k < 41) {
            const int p = k - 36;
            g = (uint32_t)p * wi.n0 + 8u * wi.n01 + gB;
            l = 8 * 297 + p * 33 + (int)x + (int)hi * (5 * 33);
            const bool exists = p + 5 * (int)hi <= 8;
            return exists && (FULL || ((int)x < wi.e0 && p + 5 * (int)hi < wi.e1 && 8 < wi.e2));
        } else {
            const bool c1 = k == 42;
            const int r = (int)(x + 32u * hi) + (c1 ? 64 : 0);
            g = c1 ? gC1 : gC0;
            l = 32 + 33 * r;
            const int y = c1 ? yc1 : yc0, z = c1 ? zc1 : zc0;
            return r < 81 && (FULL || (32 < wi.e0 && y < wi.e1 && z < wi.e2));
        }
    }
};

template <>
struct LaneMap<2> {
    uint32_t x;
    uint32_t gC;
    __device__ __forceinline__ void init(uint32_t lane, uint32_t n0, uint32_t) {
        x = lane;
        gC = 64u + lane * n0;
    }
    template <bool FULL>
    __device__ __forceinline__ bool slot(int k, const Win& wi, uint32_t& g, int& l) const {
        if (k < 17) {
            g = (uint32_t)k * wi.n0 + x;
            l = k * 65 + (int)x;
            return FULL || ((int)x < wi.e0 && k < wi.e1);
        }
        g = gC;
        l = 64 + 65 * (int)x;
        return x < 17u && (FULL || (64 < wi.e0 && (int)x < wi.e1));
    }
};

// 16-byte staging of a whole FP32 block whose rows are 16-byte aligned
// (n[0] a multiple of 4): lane = (quad q of x, row).  3D: slots 0-8 hold
// planes z = 0-8 at rows y = lane / 8, slot 9 rows y = 8 of planes lane / 8,
// slot 10 row (8, 8); then the x = 32 column in two scalar slots.  2D: slots
// 0-4 rows 4k + lane / 16, then the x = 64 column.  NQ quads and NC column
// values per lane, the quads first in the register array.
template <int ND>
struct QuadMap;

template <>
struct QuadMap<3> {
    static constexpr int NQ = 11, NC = 2, N = 4 * NQ + NC;
    uint32_t gq, gy8, gc0, gc1;   // per-lane global offsets
    int lq, ly8;                  // per-lane LDS offsets
    bool c1v;
    __device__ __forceinline__ void init(uint32_t lane, uint32_t n0, uint32_t n01) {
        const uint32_t q = lane & 7u, r = lane >> 3;
        gq = 4u * q + r * n0;
        lq = 4 * (int)q + 33 * (int)r;
        gy8 = 4u * q + 8u * n0 + r * n01;
        ly8 = 4 * (int)q + 8 * 33 + 297 * (int)r;
        gc0 = 32u + (lane % 9u) * n0 + (lane / 9u) * n01;
        gc1 = 32u + ((lane + 64u) % 9u) * n0 + ((lane + 64u) / 9u) * n01;
        c1v = lane + 64u < 81u;
    }
    // quad slot k: global offset and LDS index of its first value
    __device__ __forceinline__ bool quad(int k, uint32_t lane, uint32_t n01, uint32_t& g,
                                         int& l) const {
        if (k < 9) {
            g = gq + (uint32_t)k * n01;
            l = lq + 297 * k;
            return true;
        }
        if (k == 9) {
            g = gy8;
            l = ly8;
            return true;
        }
        g = gy8 + 8u * n01 - (lane >> 3) * n01;   // row (8, 8)
        l = 4 * (int)(lane & 7u) + 8 * 33 + 8 * 297;
        return lane < 8u;
    }
    __device__ __forceinline__ bool col(int k, uint32_t lane, uint32_t& g, int& l) const {
        g = k == 0 ? gc0 : gc1;
        l = 32 + 33 * ((int)lane + 64 * k);
        return k == 0 || c1v;
    }
};

template <>
struct QuadMap<2> {
    static constexpr int NQ = 5, NC = 1, N = 4 * NQ + NC;
    uint32_t gq, gc0, n0;
    int lq;
    uint32_t r;
    __device__ __forceinline__ void init(uint32_t lane, uint32_t nn0, uint32_t) {
        const uint32_t q = lane & 15u;
        r = lane >> 4;
        n0 = nn0;
        gq = 4u * q + r * nn0;
        lq = 4 * (int)q + 65 * (int)r;
        gc0 = 64u + lane * nn0;
    }
    __device__ __forceinline__ bool quad(int k, uint32_t lane, uint32_t, uint32_t& g,
                                         int& l) const {
        g = gq + (uint32_t)(4 * k) * n0;
        l = lq + 65 * 4 * k;
        return 4 * k + (int)r < 17;
    }
    __device__ __forceinline__ bool col(int, uint32_t lane, uint32_t& g, int& l) const {
        g = gc0;
        l = 64 + 65 * (int)lane;
        return lane < 17u;
    }
};

template <int ND>
__device__ __forceinline__ void load_quads(float* pre, const SZI_G float* wb, const QuadMap<ND>& qm,
                                           uint32_t lane, uint32_t n01) {
    using Q = QuadMap<ND>;
#pragma unroll
    for (int k = 0; k < Q::NQ; ++k) {
        uint32_t g;
        int l;
        vf4 t = {0.0f, 0.0f, 0.0f, 0.0f};
        if (qm.quad(k, lane, n01, g, l)) t = *at((const SZI_G vf4*)wb, g >> 2);
        pre[4 * k] = t.x;
        pre[4 * k + 1] = t.y;
        pre[4 * k + 2] = t.z;
        pre[4 * k + 3] = t.w;
    }
#pragma unroll
    for (int k = 0; k < Q::NC; ++k) {
        uint32_t g;
        int l;
        float t = 0.0f;
        if (qm.col(k, lane, g, l)) t = *at(wb, g);
        pre[4 * Q::NQ + k] = t;
    }
}

template <int ND>
__device__ __forceinline__ void commit_quads(float* v, const float* pre, const QuadMap<ND>& qm,
                                             uint32_t lane, uint32_t n01) {
    using Q = QuadMap<ND>;
#pragma unroll
    for (int k = 0; k < Q::NQ; ++k) {
        uint32_t g;
        int l;
        if (qm.quad(k, lane, n01, g, l)) {
            v[l] = pre[4 * k];
            v[l + 1] = pre[4 * k + 1];
            v[l + 2] = pre[4 * k + 2];
            v[l + 3] = pre[4 * k + 3];
        }
    }
#pragma unroll
    for (int k = 0; k < Q::NC; ++k) {
        uint32_t g;
        int l;
        if (qm.col(k, lane, g, l)) v[l] = pre[4 * Q::NQ + k];
    }
}

// Slots a lane does not load keep the value fill.
template <int ND, bool FULL, class T, class U>
__device__ __forceinline__ void load_block(U* pre, const SZI_G T* wb, const LaneMap<ND>& lm,
                                           const Win& wi, U fill) {
#pragma unroll
    for (int k = 0; k < Geo<ND>::NPRE; ++k) {
        uint32_t g;
        int l;
        U t = fill;
        if (lm.template slot<FULL>(k, wi, g, l)) t = (U)*at(wb, g);
        pre[k] = t;
    }
}

template <int ND, bool FULL, class T, class U>
__device__ __forceinline__ void commit_block(T* dst, const U* pre, const LaneMap<ND>& lm,
                                             const Win& wi) {
#pragma unroll
    for (int k = 0; k < Geo<ND>::NPRE; ++k) {
        uint32_t g;
        int l;
        if (lm.template slot<FULL>(k, wi, g, l)) dst[l] = (T)pre[k];
    }
}

// anchors of the block (Sec. V-A: stored losslessly), one per lane
template <int ND>
__device__ __forceinline__ bool anchor_slot(uint32_t lane, const FieldDesc& f, const Win& wi,
                                            uint32_t& gi, int& li) {
    using G = Geo<ND>;
    constexpr int S = 1 << G::SHS;
    const int ax = (int)(lane % 5u);
    const int ay = ND == 3 ? (int)((lane / 5u) & 1u) : (int)(lane / 5u);
    const int az = ND == 3 ? (int)(lane / 10u) : 0;
    li = ax * S + ay * S * G::SY + az * S * G::SZ;
    gi = (uint32_t)((wi.lo0 >> G::SHS) + ax) +
         (uint32_t)f.na[0] * ((uint32_t)((wi.lo1 >> G::SHS) + ay) +
                              (uint32_t)f.na[1] * (uint32_t)((wi.lo2 >> G::SHS) + az));
    return lane < (uint32_t)G::NANCH && ax * S < wi.e0 && ay * S < wi.e1 && az * S < wi.e2;
}

// ------------------------------------------------------------------ passes
// Division by 40 in the natural cubic, as a multiply by RN(1/40) followed
// by one fused multiply-add correction (Brisebarre, Muller and Raina,
// "Accelerating correctly rounded floating-point division when the divisor
// is known in advance", IEEE Trans. Computers 53(8), 2004).  Checked
// exhaustively over all FP32 inputs: equal to the correctly rounded x / 40
// for 2^-123 <= |x| < inf.  Smaller numerators (zeros included) take the
// division.  An infinite numerator gives NaN instead of an infinity; both
// make the point an outlier (the quantiser's range test fails on either),
// so compression and replay are unchanged.
__device__ __forceinline__ float div40_fast(float x) {
    const float c = 0.025f;
    const float q0 = x * c;
    const float r = fmaf(-q0, 40.0f, x);
    return fmaf(r, c, q0);
}

// Sec. V-B.1 splines by neighbour availability (a = x[-3s], b = x[-s],
// c = x[+s], d = x[+3s]); with one neighbour the value of x[-s].  num
// receives the natural cubic's numerator where that cubic gives the
// prediction, else 1 (a value the fast division handles).  The stencil is
// picked by selects, not branches: where the flags are compile-time
// constants only the chosen formula remains, elsewhere the wave computes
// the candidates and keeps one per lane.
template <int SPL>
__device__ __forceinline__ float predict(bool m3, bool p1, bool p3, float a, float b, float c,
                                         float d, float& num) {
    const float sbc = b + c;
    float p = sbc * 0.5f;   // linear
    num = 1.0f;
    if (SPL != SPL_LIN) {
        const float ql = ((6.0f * b + 3.0f * c) - a) * 0.125f;   // quadratic on a, b, c
        const float qr = ((3.0f * b + 6.0f * c) - d) * 0.125f;   // quadratic on b, c, d
        float cu;
        if (SPL == SPL_NAT) {
            const float n = 23.0f * sbc - 3.0f * (a + d);       // natural cubic, / 40
            cu = div40_fast(n);
            num = m3 && p3 && p1 ? n : 1.0f;
        } else {
            cu = (9.0f * sbc - (a + d)) * 0.0625f;              // not-a-knot cubic
        }
        p = m3 ? (p3 ? cu : ql) : (p3 ? qr : p);
    }
    return p1 ? p : b;
}

// LDS values of one task: K targets of one line (segment seg, starting at
// LDS index base), the K + 3 knowns around them and the targets' original
// values (compression) or quant-codes (decompression).
template <int K>
struct Task {
    int base;       // LDS index of the segment start
    uint32_t gl;    // its global offset from the window origin
    uint32_t seg;
    bool own;       // the line lies in the window's owned part
    float kn[K + 3];
    float xt[K];
    uint32_t ct[K];
};

// Where a pass leaves its results besides the block: compression stores
// the quant-code of every owned target in the codes array and counts it in
// the histogram; the replay finds outliers' values in the output array.
struct PassOut {
    SZI_G uint16_t* cb;       // the window's codes (compression)
    const SZI_G float* ob;    // the window's output values (replay)
    uint32_t* hist;           // LDS histogram (compression)
};

// One pass: dimension D, stride s = 1 << SH, spline SPL.  FULL: the window
// interval along D is the whole block, so the stencil flags are constants.
// Tasks are software-pipelined: the LDS reads of a lane's next task are
// issued before the current one is computed.  Within a pass no task reads a
// point another task writes (targets never neighbour each other along D and
// knowns are not written), so the reordering is safe.
//
// The block holds a value at every known point.  In the replay a point not
// yet reconstructed holds its quant-code instead (as the bits of the
// float), which the pass reading it as a target replaces by the value.
template <int ND, int D, int SH, int SPL, bool COMP, bool FULL>
__device__ __forceinline__ void pass_lines(float* v, uint32_t lane, const PassDesc& pd,
                                           const Win& wi, int ed, int R, const PassOut& po,
                                           uint32_t& cntR) {
    using G = Geo<ND>;
    constexpr int s = 1 << SH;
    constexpr int W = D == 0 ? G::W0 : (D == 1 ? G::W1 : G::W2);
    constexpr int SD = D == 0 ? 1 : (D == 1 ? G::SY : G::SZ);
    constexpr int T = W / (2 * s);   // targets per line
    // targets per task: x-lines take 4 (fewer live registers: the 2D
    // four-wave variant fits 128 VGPRs without spills; against 8, interp
    // and replay are 18 % faster on 2D fields and 7-9 % on 3D ones)
    constexpr int KMAX = D == 0 ? 4 : 8;
    constexpr int K = T > KMAX ? KMAX : T;
    constexpr int NSEG = T / K;
    static_assert(NSEG == 1 || D == 0, "lines split into segments run along x only");
    static_assert(NSEG == 1 || 2 * s <= kPad, "guard band narrower than the stencil");
    const uint32_t ntask = pd.nlines * (uint32_t)NSEG;
    const uint32_t ne = pd.ne, magic = pd.magic;
    const int le = pd.le, lf = pd.lf;
    const float ebx2 = pd.ebx2, inv = pd.inv, Rf = (float)R;
    const float el = pd.el;
    const uint32_t ge = pd.ge, gf = pd.gf;
    const uint32_t gsd = D == 0 ? 1u : (D == 1 ? wi.n0 : wi.n01);   // global stride along D
    // owned lines: i0 << she below the owned extent along de, i1 << shg
    // below the one along dg (the extents come out of the packed word by
    // the descriptor's bit offsets: four scalar operations a count)
    const int own0 = (int)((((wi.op >> pd.obe) & 255u) + (uint32_t)pd.rne) >> pd.she);
    const int own1 = ND == 2 ? 1 : (int)((((wi.op >> pd.obg) & 255u) + (uint32_t)pd.rng) >> pd.shg);

    auto fetch = [&](uint32_t t, Task<K>& tk) {
        tk.seg = NSEG > 1 ? (t & (uint32_t)(NSEG - 1)) : 0u;
        const uint32_t ln = NSEG > 1 ? t / (uint32_t)NSEG : t;
        const uint32_t i1 = __umulhi(ln, magic);   // ln / ne (ne >= 2, ln < 2^16)
        const uint32_t i0 = ln - i1 * ne;
        tk.base = (int)i0 * le + (int)i1 * lf + (int)tk.seg * (2 * K * s) * SD;
        tk.gl = i0 * ge + i1 * gf + tk.seg * (uint32_t)(2 * K * s) * gsd;
        if (COMP) tk.own = (int)i0 < own0 && (int)i1 < own1;
        // knowns at (2i - 2) s from the segment start; whole lines read only
        // the ones inside the block, split lines all of them (the guard band
        // and the neighbouring line absorb the ends; the flags drop them)
#pragma unroll
        for (int i = 0; i < K + 3; ++i) {
            const int pos = (2 * i - 2) * s;
            tk.kn[i] = (NSEG > 1 || (pos >= 0 && pos <= W)) ? v[tk.base + pos * SD] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int li = tk.base + (2 * j + 1) * s * SD;
            if (COMP)
                tk.xt[j] = v[li];
            else
                tk.ct[j] = __float_as_uint(v[li]);
        }
    };

    auto compute = [&](const Task<K>& tk) {
        const int p0 = (int)tk.seg * (2 * K * s);   // segment start along D
        float pr[K], nm[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int pos = (2 * j + 1) * s;   // target position in the segment
            const bool m3 = NSEG > 1 ? (j >= 1 || tk.seg > 0u) : (j >= 1);
            bool p3 = NSEG > 1 ? (j <= K - 2 || tk.seg < (uint32_t)(NSEG - 1))
                               : ((2 * j + 4) * s <= W);
            bool p1 = true;
            if (!FULL) {   // the window interval ends at ed - 1
                p1 = p0 + pos + s <= ed - 1;
                p3 = p0 + pos + 3 * s <= ed - 1;
            }
            pr[j] = predict<SPL>(m3, p1, p3, tk.kn[j], tk.kn[j + 1], tk.kn[j + 2], tk.kn[j + 3],
                                 nm[j]);
        }
        if (SPL == SPL_NAT) {   // numerators below the fast division's range: rare
            bool need = false;
#pragma unroll
            for (int j = 0; j < K; ++j) need = need || !(fabsf(nm[j]) >= 0x1p-123f);
            if (wave_any(need)) {
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if (!(fabsf(nm[j]) >= 0x1p-123f)) pr[j] = nm[j] / 40.0f;
            }
        }
        float* vb = v + tk.base;
        if (COMP) {
            float qr[K], xr[K], vv[K];
            uint32_t cd[K];
            bool need = false;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                // closed-loop quantisation against e_l (Sec. III-A): with
                // e_l = 0, inv = 0 gives q = 0 and xr = p + 0, so only exact
                // predictions pass the bound test below
                const float p = pr[j], xv = tk.xt[j];
                qr[j] = rintf((xv - p) * inv);   // round half to even
                xr[j] = p + qr[j] * ebx2;        // (float)(int)q == q in range
                // |rint(qf)| < R holds iff |qf| < R and |q| < R; NaN fails it.
                // The FP64 bound test |x - xr| <= e_l is decided in FP32
                // where the rounded difference is below e_l (then so is the
                // exact one), in FP64 otherwise (below).
                const bool inr = fabsf(qr[j]) < Rf;
                const bool good = inr && fabsf(xv - xr[j]) < el;
                vv[j] = good ? xr[j] : xv;
                cd[j] = good ? (uint32_t)((int)qr[j] + R) : 0u;
                need = need || (good != inr);
            }
            if (wave_any(need)) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const float xv = tk.xt[j];
                    if (fabsf(qr[j]) < Rf && !(fabsf(xv - xr[j]) < el) &&
                        fabs((double)xv - (double)xr[j]) <= (double)el) {
                        vv[j] = xr[j];
                        cd[j] = (uint32_t)((int)qr[j] + R);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j) vb[(2 * j + 1) * s * SD] = vv[j];
            // owned targets' quant-codes: the window interval along D ends
            // at ed - 1
            if (tk.own) {
                SZI_G char* cbb = (SZI_G char*)po.cb + (uint64_t)(2u * tk.gl);
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const int pos = (2 * j + 1) * s;
                    if (FULL || p0 + pos < ed) {
                        if (D == 0) *(SZI_G uint16_t*)(cbb + 2 * pos) = (uint16_t)cd[j];
                        else *(SZI_G uint16_t*)(cbb + (uint64_t)(2u * (uint32_t)pos * gsd)) = (uint16_t)cd[j];
                    }
                }
            }
            // histogram without branches: every target adds one; the centre
            // code and targets the window does not own go to a bin of the
            // lane's own past the 2R symbols (no two lanes share an
            // address), and the count of the latter is taken off the centre
            // bin when the histogram is flushed
            const uint32_t rb = (uint32_t)(2 * R) + lane;
            if (FULL) cntR += (uint32_t)(K * __popcll(wave_ballot(!tk.own)));
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int pos = (2 * j + 1) * s;
                const bool ot = tk.own && (FULL || p0 + pos < ed);
                if (!FULL) cntR += (uint32_t)__popcll(wave_ballot(!ot));
                const uint32_t bin = ot && cd[j] != (uint32_t)R ? cd[j] : rb;
                atomicAdd(&po.hist[bin], 1u);
            }
        } else {
            bool out = false;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const uint32_t code = tk.ct[j];
                pr[j] = pr[j] + (float)((int)code - R) * ebx2;
                out = out || code == 0u;
            }
            // code 0: an outlier, whose value the scatter step put in the
            // output array (points outside the field hold a code no point
            // takes, so the load stays inside it); rare, so one uniform test
            if (wave_any(out)) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const int pos = (2 * j + 1) * s;
                    if (tk.ct[j] == 0u) pr[j] = *at(po.ob, tk.gl + (uint32_t)pos * gsd);
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j) vb[(2 * j + 1) * s * SD] = pr[j];
        }
    };

    // two task slots in turn, so that no values are copied between them
    uint32_t t = lane;
    if (t >= ntask) return;
    Task<K> ta, tb;
    fetch(t, ta);
#pragma unroll 1
    while (true) {
        t += 64;
        bool more = t < ntask;
        if (more) fetch(t, tb);
        compute(ta);
        if (!more) break;
        t += 64;
        more = t < ntask;
        if (more) fetch(t, ta);
        compute(tb);
        if (!more) break;
    }
}

template <int ND, int D, int SH, bool COMP>
__device__ __forceinline__ void run_pass(float* v, uint32_t lane, const PassDesc& pd, const Win& wi,
                                         int R, const PassOut& po, uint32_t& cntR) {
    using G = Geo<ND>;
    constexpr int W = D == 0 ? G::W0 : (D == 1 ? G::W1 : G::W2);
    const int ed = D == 0 ? wi.e0 : (D == 1 ? wi.e1 : wi.e2);
    // the stencil flags depend on the extent along D only
    if (ed == W + 1) {
        if (pd.spl == SPL_LIN)
            pass_lines<ND, D, SH, SPL_LIN, COMP, true>(v, lane, pd, wi, ed, R, po, cntR);
        else if (pd.spl == SPL_NAT)
            pass_lines<ND, D, SH, SPL_NAT, COMP, true>(v, lane, pd, wi, ed, R, po, cntR);
        else
            pass_lines<ND, D, SH, SPL_NAK, COMP, true>(v, lane, pd, wi, ed, R, po, cntR);
    } else {
        if (pd.spl == SPL_LIN)
            pass_lines<ND, D, SH, SPL_LIN, COMP, false>(v, lane, pd, wi, ed, R, po, cntR);
        else if (pd.spl == SPL_NAT)
            pass_lines<ND, D, SH, SPL_NAT, COMP, false>(v, lane, pd, wi, ed, R, po, cntR);
        else
            pass_lines<ND, D, SH, SPL_NAK, COMP, false>(v, lane, pd, wi, ed, R, po, cntR);
    }
}

// A wave's own LDS accesses execute in program order; this keeps the
// compiler from moving them across a pass boundary.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The passes of one level (stride 1 << SH), in the planned order.
template <int ND, int SH, bool COMP>
__device__ __forceinline__ void run_level(float* v, uint32_t lane, const FieldPlan& pl, int R,
                                          const Win& wi, const PassOut& po, uint32_t& cntR) {
    constexpr int L = ND == 3 ? 3 : 4;
#pragma unroll 1
    for (int k = 0; k < ND; ++k) {
        const PassDesc pd = pl.pass[(L - 1 - SH) * ND + k];
        if (pd.d == 0) run_pass<ND, 0, SH, COMP>(v, lane, pd, wi, R, po, cntR);
        else if (ND == 2 || pd.d == 1) run_pass<ND, 1, SH, COMP>(v, lane, pd, wi, R, po, cntR);
        else if constexpr (ND == 3) run_pass<ND, 2, SH, COMP>(v, lane, pd, wi, R, po, cntR);
        wave_sync();
    }
}

template <int ND, bool COMP>
__device__ __forceinline__ void run_levels(float* v, uint32_t lane, const FieldPlan& pl, int R,
                                           const Win& wi, const PassOut& po, uint32_t& cntR) {
    if constexpr (ND == 2) run_level<ND, 3, COMP>(v, lane, pl, R, wi, po, cntR);
    run_level<ND, 2, COMP>(v, lane, pl, R, wi, po, cntR);
    run_level<ND, 1, COMP>(v, lane, pl, R, wi, po, cntR);
    run_level<ND, 0, COMP>(v, lane, pl, R, wi, po, cntR);
}

// ---------------------------------------------------------------- write-out
// Rows of the owned part are covered in slots of RPS rows; a slot's rows
// lie in one plane.  Lane = (sub, x-group).
template <int ND, int PER_ROW>
struct OutMap {
    using G = Geo<ND>;
    static constexpr int RPS = 64 / PER_ROW;
    static constexpr int NS = G::W1 * (ND == 3 ? G::W2 : 1) / RPS;
    static constexpr int y0(int k) { return (k * RPS) % G::W1; }
    static constexpr int z0(int k) { return (k * RPS) / G::W1; }
};

// Owned anchors: x = 0, S, 2S, 3S of row 0.  Their values go to the anchor
// array (Sec. V-A: stored losslessly); their quant-code is R (counted in
// the histogram like every owned code, Sec. VI-A).  The passes store the
// codes of all other owned points.
template <int ND>
__device__ __forceinline__ void write_anchors(const float* v, uint32_t lane, const FieldDesc& f,
                                              const Win& wi, uint32_t* hist) {
    using G = Geo<ND>;
    constexpr int S = 1 << G::SHS;
    if (lane < (uint32_t)(G::W0 / S) && (int)lane * S < wi.own(0)) {
        const uint32_t ai = (uint32_t)(wi.lo0 >> G::SHS) + lane +
                            (uint32_t)f.na[0] * ((uint32_t)(wi.lo1 >> G::SHS) +
                                                 (uint32_t)f.na[1] * (uint32_t)(wi.lo2 >> G::SHS));
        gp(f.anchors)[ai] = v[(int)lane * S];
        *at(gp(f.codes) + wi.gbase, lane * (uint32_t)S) = (uint16_t)f.R;
        atomicAdd(&hist[2 * f.R + lane], 1u);   // the lane's centre-code bin
    }
}

// Owned reconstructed values.
template <int ND, bool FULL>
__device__ __forceinline__ void write_values(const float* v, uint32_t lane, const FieldDesc& f,
                                             const Win& wi) {
    using G = Geo<ND>;
    using M = OutMap<ND, G::W0 / 4>;    // x-quads
    SZI_G float* ob = gp(f.out) + wi.gbase;
    const uint32_t sub = lane / (uint32_t)(G::W0 / 4);
    const int x = 4 * (int)(lane % (uint32_t)(G::W0 / 4));
    const int lq = x + (int)sub * G::SY;
    const uint32_t gq = (uint32_t)x + sub * wi.n0;
    if (FULL && (wi.n0 & 3u) == 0u && ((uintptr_t)f.out & 15u) == 0u) {
#pragma unroll
        for (int k = 0; k < M::NS; ++k) {
            const int l = lq + M::y0(k) * G::SY + M::z0(k) * G::SZ;
            vf4 o;
            o.x = v[l];
            o.y = v[l + 1];
            o.z = v[l + 2];
            o.w = v[l + 3];
            const uint32_t g = gq + (uint32_t)M::y0(k) * wi.n0 + (uint32_t)M::z0(k) * wi.n01;
            *at((SZI_G vf4*)ob, g >> 2) = o;
        }
    } else {
#pragma unroll 1
        for (int k = 0; k < M::NS; ++k) {
            const int y = M::y0(k) + (int)sub, z = M::z0(k);
            if (y >= wi.own(1) || z >= wi.own(2)) continue;
            const int l = x + y * G::SY + z * G::SZ;
            const uint32_t g = (uint32_t)x + (uint32_t)y * wi.n0 + (uint32_t)z * wi.n01;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (x + i < wi.own(0)) *at(ob, g + (uint32_t)i) = v[l + i];
        }
    }
}

// ------------------------------------------------------------ group order
// Work is handed out in groups of kWaves windows of one field (the host
// pads each field to whole groups).  Workgroups on one L2 domain take one
// contiguous eighth of the groups, so that windows sharing faces are
// processed close in time on the same L2: in round k its S workgroups take
// the k-th run of S groups, workgroup j the group (j + k) mod S of the run.
// The rotation, and that of the wave slots within a group every kWaves
// rounds, spread windows of one kind (the field's far boundary along x
// always falls in the same slot of every fourth group) over all waves.  A
// fixed group and slot per workgroup and wave sent all of them to a
// quarter of the workgroups, one wave each, which finished a fifth later
// than the rest.
struct GroupSeq {
    uint64_t lo, end;   // the L2 domain's groups
    uint32_t S, j, k;   // workgroups in the domain, this one's index, round
    uint64_t g;         // the round's group (increasing; past end: done)
    __device__ __forceinline__ void set() { g = lo + (uint64_t)k * S + (j + k) % S; }
    __device__ __forceinline__ bool ok() const { return g < end; }
    __device__ __forceinline__ void next() {
        ++k;
        set();
    }
    // the window slot of a wave in the round's group
    __device__ __forceinline__ uint32_t slot(int wave) const {
        return ((uint32_t)wave + k / (uint32_t)kWaves) % (uint32_t)kWaves;
    }
    // Issue priority of the round.  A SIMD issues from its oldest wave
    // first, so with equal work the workgroups dispatched first on a CU
    // finish first and the last ones run on alone.  Dispatch fills the
    // domain's 32 CUs one workgroup each before it places second ones, so
    // the T = S / 32 workgroups that share a CU are j, j + 32, .. of the
    // domain; with priority (k + j / 32) mod T they hold the highest
    // priority in turn, one round each.
    __device__ __forceinline__ void set_priority() const {
        constexpr uint32_t kCusPerDomain = 32;   // 256 CUs in 8 L2 domains
        uint32_t T = S / kCusPerDomain;
        T = T < 1u ? 1u : (T > 4u ? 4u : T);
        const uint32_t p = (k + j / kCusPerDomain) % T;
        if (p == 0u) __builtin_amdgcn_s_setprio(0);
        else if (p == 1u) __builtin_amdgcn_s_setprio(1);
        else if (p == 2u) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(3);
    }
};
__device__ __forceinline__ GroupSeq group_seq(uint64_t ngroups) {
    const uint32_t G = gridDim.x, b = blockIdx.x;
    GroupSeq s;
    if (G >= (uint32_t)kXcds && G % (uint32_t)kXcds == 0u) {
        const uint64_t chunk = (ngroups + kXcds - 1) / kXcds;
        s.lo = (uint64_t)(b % (uint32_t)kXcds) * chunk;
        s.end = s.lo + chunk < ngroups ? s.lo + chunk : ngroups;
        s.S = G / (uint32_t)kXcds;
        s.j = b / (uint32_t)kXcds;
    } else {
        s.lo = 0;
        s.end = ngroups;
        s.S = G;
        s.j = b;
    }
    s.k = 0;
    s.set();
    return s;
}

// --------------------------------------------------------------- kernels
// LDS histogram of a workgroup: the 2R symbols, then one bin per lane that
// collects the centre code and the targets a window does not own; nown
// (wave-uniform) counts the latter.  The flush folds the lane bins into
// the centre bin (modulo 2^32, so the subtraction may wrap on the way).
__device__ __forceinline__ void clear_hist(uint32_t* hist, int R) {
#pragma unroll 1
    for (int b = threadIdx.x; b < 2 * R + 64; b += kThreads) hist[b] = 0;
}
__device__ __forceinline__ void flush_hist(uint32_t* hist, uint32_t& nown, const FieldDesc& fd) {
    if ((threadIdx.x & 63) == 0 && nown) atomicAdd(&hist[fd.R], 0u - nown);
    nown = 0;
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t c = wave_sum(hist[2 * fd.R + threadIdx.x]);
        if (threadIdx.x == 0) atomicAdd(&hist[fd.R], c);
    }
    __syncthreads();
#pragma unroll 1
    for (int b = threadIdx.x; b < 2 * fd.R; b += kThreads)
        if (hist[b]) gatomic_add(gp(fd.hist) + b, hist[b]);
    __syncthreads();
}

// WPE waves per SIMD: the register budget that leaves (3: 168 VGPRs, 4:
// 128) is what a kernel variant is compiled for.  With the block alone in
// LDS (and the histogram of compression), three workgroups of four 3D
// windows fit a CU; 2D blocks are small enough for four.
#define SZI_WINDOW_KERNEL \
    __global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(WPE)))

template <int ND, int WPE>
SZI_WINDOW_KERNEL void k_compress(const FieldDesc* __restrict__ F, const FieldPlan* __restrict__ P,
                                  const uint64_t* __restrict__ goff, uint64_t ngroups) {
    using G = Geo<ND>;
    __shared__ float vbuf[kWaves][vlen<ND>()];
    extern __shared__ uint32_t hist[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    float* v = vbuf[wave] + kPad;
    GroupSeq gs = group_seq(ngroups);
    if (!gs.ok()) return;
    int f = 0;
    // block of the next window: 16-byte quads where the window lies in the
    // field and its rows are aligned, else one value per slot
    constexpr int NPQ = QuadMap<ND>::N > G::NPRE ? QuadMap<ND>::N : G::NPRE;
    float pre[NPQ];
    LaneMap<ND> lm;
    QuadMap<ND> qm;
    Win wn;
    bool valid, quads = false;
    // window of group g for this wave, and the start of its block load
    auto fetch = [&]() {
        while (gs.g >= goff[f + 1]) ++f;
        const uint32_t w = (uint32_t)(gs.g - goff[f]) * kWaves + gs.slot(wave);
        valid = w < (uint32_t)(F[f].nwin[0] * F[f].nwin[1] * F[f].nwin[2]);
        if (valid) {
            wn = make_win<ND>(F[f], w);
            const SZI_G float* wb = gp(F[f].in) + wn.gbase;
            quads = wn.full && (wn.n0 & 3u) == 0u && ((uintptr_t)F[f].in & 15u) == 0u;
            if (quads) {
                qm.init(lane, wn.n0, wn.n01);
                load_quads<ND>(pre, wb, qm, lane, wn.n01);
            } else {
                lm.init(lane, wn.n0, wn.n01);
                if (wn.full) load_block<ND, true>(pre, wb, lm, wn, 0.0f);
                else load_block<ND, false>(pre, wb, lm, wn, 0.0f);
            }
        }
    };
    fetch();
    int hf = -1;         // field whose histogram the workgroup accumulates
    uint32_t cntR = 0;   // targets counted in the lane bins that the windows do not own
    while (true) {
        const int fc = f;
        const Win wc = wn;
        const bool vc = valid, qc = quads;
        if (fc != hf) {   // uniform over the workgroup: groups never span fields
            if (hf >= 0) flush_hist(hist, cntR, F[hf]);
            clear_hist(hist, F[fc].R);
            __syncthreads();
            hf = fc;
        }
        if (vc) {
            if (qc) commit_quads<ND>(v, pre, qm, lane, wc.n01);
            else if (wc.full) commit_block<ND, true>(v, pre, lm, wc);
            else commit_block<ND, false>(v, pre, lm, wc);
        }
        gs.next();
        gs.set_priority();
        const bool more = gs.ok();
        if (more) fetch();   // in flight during the passes below
        if (vc) {
            wave_sync();
            const FieldDesc& fd = F[fc];
            const PassOut po{gp(fd.codes) + wc.gbase, nullptr, hist};
            run_levels<ND, true>(v, lane, P[fc], fd.R, wc, po, cntR);
            write_anchors<ND>(v, lane, fd, wc, hist);
            wave_sync();
        }
        if (!more) break;
    }
    flush_hist(hist, cntR, F[hf]);
}

template <int ND, int WPE>
SZI_WINDOW_KERNEL void k_decompress(const FieldDesc* __restrict__ F,
                                    const FieldPlan* __restrict__ P,
                                    const uint64_t* __restrict__ goff, uint64_t ngroups) {
    using G = Geo<ND>;
    __shared__ float vbuf[kWaves][vlen<ND>()];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    float* v = vbuf[wave] + kPad;
    GroupSeq gs = group_seq(ngroups);
    if (!gs.ok()) return;
    int f = 0;
    // codes of the next window's block; block points outside the field
    // hold a value no code takes
    constexpr uint32_t kNone = 0xFFFFFFFFu;
    uint32_t pre[G::NPRE];
    float apre = 0.0f;   // one anchor per lane
    LaneMap<ND> lm;
    Win wn;
    bool valid;
    auto fetch = [&]() {
        while (gs.g >= goff[f + 1]) ++f;
        const uint32_t w = (uint32_t)(gs.g - goff[f]) * kWaves + gs.slot(wave);
        valid = w < (uint32_t)(F[f].nwin[0] * F[f].nwin[1] * F[f].nwin[2]);
        if (valid) {
            wn = make_win<ND>(F[f], w);
            lm.init(lane, wn.n0, wn.n01);
            const SZI_G uint16_t* cb = gp(F[f].codes) + wn.gbase;
            if (wn.full) load_block<ND, true>(pre, cb, lm, wn, kNone);
            else load_block<ND, false>(pre, cb, lm, wn, kNone);
            uint32_t ga;
            int la;
            if (anchor_slot<ND>(lane, F[f], wn, ga, la)) apre = gp(F[f].anchors)[ga];
        }
    };
    fetch();
    uint32_t unused = 0;
    while (true) {
        const int fc = f;
        const Win wc = wn;
        const bool vc = valid;
        if (vc) {
            // every point of the block takes its code (as float bits), those
            // outside the field the value kNone; the anchors then their values
#pragma unroll
            for (int k = 0; k < G::NPRE; ++k) {
                uint32_t gg;
                int l;
                if (lm.template slot<true>(k, wc, gg, l)) v[l] = __uint_as_float(pre[k]);
            }
            uint32_t ga;
            int la;
            if (anchor_slot<ND>(lane, F[fc], wc, ga, la)) v[la] = apre;
        }
        gs.next();
        gs.set_priority();
        const bool more = gs.ok();
        if (more) fetch();   // in flight during the passes below
        if (vc) {
            wave_sync();
            const FieldDesc& fd = F[fc];
            const PassOut po{nullptr, gp((const float*)fd.out) + wc.gbase, nullptr};
            run_levels<ND, false>(v, lane, P[fc], fd.R, wc, po, unused);
            if (wc.full) write_values<ND, true>(v, lane, fd, wc);
            else write_values<ND, false>(v, lane, fd, wc);
            wave_sync();
        }
        if (!more) break;
    }
}

// ------------------------------------------------------------ 1D fields
// Sec. V-A in one dimension: anchors every kS1 = 512 points, nine levels
// (strides 256 .. 1), one pass per level.  A window is four chunks, 2048
// points, plus the far anchor, as the 3D and 2D windows span four chunks
// along x; one wave per window, its block in LDS, one target per lane at a
// time.  The stencils, the quantiser and the histogram are those of the
// window passes above.
constexpr int kS1 = 512, kL1 = 9, kW1 = 4 * kS1;
constexpr int kV1 = kW1 + 4;   // LDS floats per wave: the block of kW1 + 1

struct Win1 {
    uint64_t lo;   // first point
    int e;         // block extent: owned points, and the far anchor where present
    int o;         // owned extent
};

__device__ __forceinline__ Win1 make_win1(const FieldDesc& f, uint32_t w) {
    Win1 wi;
    wi.lo = (uint64_t)w * (uint64_t)kW1;
    const uint64_t left = f.npts - 1 - wi.lo;
    wi.e = (int)(left < (uint64_t)kW1 ? left : (uint64_t)kW1) + 1;
    wi.o = wi.e < kW1 ? wi.e : kW1;
    return wi;
}

// One level at stride s: the targets at odd multiples of s in the window.
// Compression stores each owned target's quant-code at cb and counts it;
// the replay takes an outlier's value from ob.
template <int SPL, bool COMP>
__device__ __forceinline__ void level1(float* v, uint32_t lane, int s, const Win1& wi, float el,
                                       float ebx2, float inv, int R, SZI_G uint16_t* cb,
                                       const SZI_G float* ob, uint32_t* hist, uint32_t& cntR) {
    const int nt = kW1 / (2 * s);
    const float Rf = (float)R;
    const int last = wi.e - 1;   // the window interval ends here
#pragma unroll 1
    for (int t = (int)lane; t < nt; t += 64) {
        const int p = (2 * t + 1) * s;
        const bool act = p <= last;
        const bool m3 = p >= 3 * s;
        const bool p1 = p + s <= last;
        const bool p3 = p + 3 * s <= last;
        const float a = m3 ? v[p - 3 * s] : 0.0f;
        const float b = v[p - s];
        const float c = p1 ? v[p + s] : 0.0f;
        const float d = p3 ? v[p + 3 * s] : 0.0f;
        float num;
        float pr = predict<SPL>(m3, p1, p3, a, b, c, d, num);
        if (SPL == SPL_NAT) {   // numerators below the fast division's range: rare
            const bool small = !(fabsf(num) >= 0x1p-123f);
            if (wave_any(small) && small) pr = num / 40.0f;
        }
        if (COMP) {
            const float xv = v[p];
            const float q = rintf((xv - pr) * inv);
            const float xr = pr + q * ebx2;
            const bool inr = fabsf(q) < Rf;
            const bool good = inr && fabsf(xv - xr) < el;
            float vv = good ? xr : xv;
            uint32_t cd = good ? (uint32_t)((int)q + R) : 0u;
            if (wave_any(act && good != inr)) {   // the FP64 bound test where FP32 cannot decide
                if (inr && !(fabsf(xv - xr) < el) && fabs((double)xv - (double)xr) <= (double)el) {
                    vv = xr;
                    cd = (uint32_t)((int)q + R);
                }
            }
            const bool own = act && p < wi.o;
            if (act) {
                v[p] = vv;
                if (own) cb[p] = (uint16_t)cd;
                const uint32_t bin = own && cd != (uint32_t)R ? cd : (uint32_t)(2 * R) + lane;
                atomicAdd(&hist[bin], 1u);
            }
            cntR += (uint32_t)__popcll(wave_ballot(act && !own));
        } else if (act) {
            const uint32_t code = __float_as_uint(v[p]);
            // code 0: an outlier, whose value the scatter step put in the output
            v[p] = code == 0u ? ob[p] : pr + (float)((int)code - R) * ebx2;
        }
    }
}

template <bool COMP>
__device__ __forceinline__ void levels1(float* v, uint32_t lane, const FieldPlan& pl, const Win1& wi,
                                        int R, SZI_G uint16_t* cb, const SZI_G float* ob,
                                        uint32_t* hist, uint32_t& cntR) {
#pragma unroll 1
    for (int l = kL1; l >= 1; --l) {
        const int s = 1 << (l - 1);
        const float el = pl.el[l - 1], ebx2 = pl.ebx2[l - 1];
        const float inv = el == 0.0f ? 0.0f : pl.inv[l - 1];
        if (pl.spline[0] == SPL_LIN) level1<SPL_LIN, COMP>(v, lane, s, wi, el, ebx2, inv, R, cb, ob, hist, cntR);
        else if (pl.spline[0] == SPL_NAK) level1<SPL_NAK, COMP>(v, lane, s, wi, el, ebx2, inv, R, cb, ob, hist, cntR);
        else level1<SPL_NAT, COMP>(v, lane, s, wi, el, ebx2, inv, R, cb, ob, hist, cntR);
        wave_sync();
    }
}

__global__ __launch_bounds__(kThreads) void k_compress1d(const FieldDesc* __restrict__ F,
                                                         const FieldPlan* __restrict__ P,
                                                         const uint64_t* __restrict__ goff,
                                                         uint64_t ngroups) {
    __shared__ float vbuf[kWaves][kV1];
    extern __shared__ uint32_t hist[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    float* v = vbuf[wave];
    int f = 0, hf = -1;
    uint32_t cntR = 0;
#pragma unroll 1
    for (GroupSeq gs = group_seq(ngroups); gs.ok(); gs.next()) {
        while (gs.g >= goff[f + 1]) ++f;
        if (f != hf) {   // uniform over the workgroup: groups never span fields
            if (hf >= 0) flush_hist(hist, cntR, F[hf]);
            clear_hist(hist, F[f].R);
            __syncthreads();
            hf = f;
        }
        const FieldDesc& fd = F[f];
        const uint32_t w = (uint32_t)(gs.g - goff[f]) * kWaves + gs.slot(wave);
        if (w >= (uint32_t)fd.nwin[0]) continue;
        const Win1 wi = make_win1(fd, w);
        const SZI_G float* in = gp(fd.in) + wi.lo;
#pragma unroll 4
        for (int i = (int)lane; i < wi.e; i += 64) v[i] = in[i];
        wave_sync();
        SZI_G uint16_t* cb = gp(fd.codes) + wi.lo;
        levels1<true>(v, lane, P[f], wi, fd.R, cb, nullptr, hist, cntR);
        // owned anchors: their values losslessly, quant-code R, counted
        if (lane < (uint32_t)(kW1 / kS1) && (int)lane * kS1 < wi.o) {
            gp(fd.anchors)[wi.lo / kS1 + lane] = v[lane * kS1];
            cb[lane * kS1] = (uint16_t)fd.R;
            atomicAdd(&hist[2 * fd.R + lane], 1u);
        }
        wave_sync();
    }
    if (hf >= 0) flush_hist(hist, cntR, F[hf]);
}

__global__ __launch_bounds__(kThreads) void k_decompress1d(const FieldDesc* __restrict__ F,
                                                           const FieldPlan* __restrict__ P,
                                                           const uint64_t* __restrict__ goff,
                                                           uint64_t ngroups) {
    __shared__ float vbuf[kWaves][kV1];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    float* v = vbuf[wave];
    int f = 0;
    uint32_t unused = 0;
#pragma unroll 1
    for (GroupSeq gs = group_seq(ngroups); gs.ok(); gs.next()) {
        while (gs.g >= goff[f + 1]) ++f;
        const FieldDesc& fd = F[f];
        const uint32_t w = (uint32_t)(gs.g - goff[f]) * kWaves + gs.slot(wave);
        if (w >= (uint32_t)fd.nwin[0]) continue;
        const Win1 wi = make_win1(fd, w);
        // every point takes its code (as float bits), the anchors their values
        const SZI_G uint16_t* cb = gp(fd.codes) + wi.lo;
#pragma unroll 4
        for (int i = (int)lane; i < wi.e; i += 64) v[i] = __uint_as_float((uint32_t)cb[i]);
        wave_sync();
        if (lane <= (uint32_t)(kW1 / kS1) && (int)lane * kS1 < wi.e)
            v[lane * kS1] = gp(fd.anchors)[wi.lo / kS1 + lane];
        wave_sync();
        SZI_G float* ob = gp(fd.out) + wi.lo;
        levels1<false>(v, lane, P[f], wi, fd.R, nullptr, ob, nullptr, unused);
#pragma unroll 4
        for (int i = (int)lane; i < wi.o; i += 64) ob[i] = v[i];
        wave_sync();
    }
}

// ------------------------------------------------------------ any window
// Fields whose anchor stride or window is not the default one (Sec. V-A and
// V-D leave both open: the window trades prediction accuracy at its faces
// against parallelism) run a generic pair of kernels with the geometry read
// from the field descriptor: one wave per window, its block (window + far
// faces) in LDS, each pass's targets one per lane at a time.  The passes,
// stencils, quantiser and histogram are those above.
struct WinG {
    uint64_t gbase;
    uint32_t n0, n01;
    int lo[3], e[3], o[3];   // origin, block extent, owned extent per dimension
    int B0, B01;             // LDS strides
};

__device__ __forceinline__ WinG make_wing(const FieldDesc& f, uint32_t w) {
    WinG wi;
    const uint32_t nw0 = (uint32_t)f.nwin[0], nw01 = nw0 * (uint32_t)f.nwin[1];
    const uint32_t wz = w / nw01, r = w - wz * nw01, wy = r / nw0, wx = r - wy * nw0;
    const uint32_t wc[3] = {wx, wy, wz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        wi.lo[k] = (int)wc[k] * f.w[k];
        const int sk = f.n[k] - 1 - wi.lo[k];
        wi.e[k] = (sk < f.w[k] ? sk : f.w[k]) + 1;
        wi.o[k] = wi.e[k] < f.w[k] ? wi.e[k] : f.w[k];
    }
    wi.n0 = (uint32_t)f.n[0];
    wi.n01 = wi.n0 * (uint32_t)f.n[1];
    wi.B0 = f.ndim >= 1 ? f.w[0] + 1 : 1;
    wi.B01 = wi.B0 * (f.ndim >= 2 ? f.w[1] + 1 : 1);
    wi.gbase = (uint64_t)wi.lo[0] + (uint64_t)wi.lo[1] * wi.n0 + (uint64_t)wi.lo[2] * wi.n01;
    return wi;
}

// a point's block coordinates from its number among m0 x m1 x m2 grid
// points with the given spacing and offset per dimension
struct Grid3 {
    FastDiv f0, f1;
    int step[3], off[3];
    __device__ __forceinline__ void at(uint32_t t, int* c) const {
        const uint32_t t1 = f0.div(t), i0 = t - t1 * f0.m;
        const uint32_t i2 = f1.div(t1), i1 = t1 - i2 * f1.m;
        c[0] = off[0] + (int)i0 * step[0];
        c[1] = off[1] + (int)i1 * step[1];
        c[2] = off[2] + (int)i2 * step[2];
    }
};

// One pass of the generic kernels: dimension d at stride s; the other
// dimensions at multiples of s where this level has passed them, of 2 s
// where not (Sec. V-A).
template <int SPL, bool COMP>
__device__ __forceinline__ void pass_gen(float* v, uint32_t lane, const FieldDesc& fd, const WinG& wi,
                                         int d, int s, const bool* passed, float el, float ebx2,
                                         float inv, SZI_G uint16_t* cb, const SZI_G float* ob,
                                         uint32_t* hist, uint32_t& cntR) {
    const int R = fd.R;
    Grid3 gr;
    uint32_t m[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int lim = wi.e[j] - 1;
        if (j == d) {
            gr.step[j] = 2 * s;
            gr.off[j] = s;
            m[j] = lim >= s ? (uint32_t)((lim - s) / (2 * s) + 1) : 0u;
        } else {
            gr.step[j] = passed[j] ? s : 2 * s;
            gr.off[j] = 0;
            m[j] = (uint32_t)(lim / gr.step[j] + 1);
        }
    }
    gr.f0.set(m[0]);
    gr.f1.set(m[1]);
    const uint32_t nt = m[0] * m[1] * m[2];
    const int lim = wi.e[d] - 1;
    const int sd = d == 0 ? 1 : (d == 1 ? wi.B0 : wi.B01);
    const float Rf = (float)R;
#pragma unroll 1
    for (uint32_t t = lane; t < nt; t += 64) {
        int c[3];
        gr.at(t, c);
        const int li = c[0] + c[1] * wi.B0 + c[2] * wi.B01;
        const int cd = c[d];
        const bool m3 = cd >= 3 * s;
        const bool p1 = cd + s <= lim;
        const bool p3 = cd + 3 * s <= lim;
        const float a = m3 ? v[li - 3 * s * sd] : 0.0f;
        const float b = v[li - s * sd];
        const float cc = p1 ? v[li + s * sd] : 0.0f;
        const float dd = p3 ? v[li + 3 * s * sd] : 0.0f;
        float num;
        float pr = predict<SPL>(m3, p1, p3, a, b, cc, dd, num);
        if (SPL == SPL_NAT) {
            const bool small = !(fabsf(num) >= 0x1p-123f);
            if (wave_any(small) && small) pr = num / 40.0f;
        }
        const uint64_t g = (uint64_t)c[0] + (uint64_t)c[1] * wi.n0 + (uint64_t)c[2] * wi.n01;
        if (COMP) {
            const float xv = v[li];
            const float q = rintf((xv - pr) * inv);
            const float xr = pr + q * ebx2;
            const bool inr = fabsf(q) < Rf;
            const bool good = inr && fabsf(xv - xr) < el;
            float vv = good ? xr : xv;
            uint32_t code = good ? (uint32_t)((int)q + R) : 0u;
            if (wave_any(good != inr)) {   // the FP64 bound test where FP32 cannot decide
                if (inr && !(fabsf(xv - xr) < el) && fabs((double)xv - (double)xr) <= (double)el) {
                    vv = xr;
                    code = (uint32_t)((int)q + R);
                }
            }
            v[li] = vv;
            const bool own = c[0] < wi.o[0] && c[1] < wi.o[1] && c[2] < wi.o[2];
            if (own) cb[g] = (uint16_t)code;
            const uint32_t bin = own && code != (uint32_t)R ? code : (uint32_t)(2 * R) + lane;
            atomicAdd(&hist[bin], 1u);
            cntR += (uint32_t)__popcll(wave_ballot(!own));
        } else {
            const uint32_t code = __float_as_uint(v[li]);
            // code 0: an outlier, whose value the scatter step put in the output
            v[li] = code == 0u ? ob[g] : pr + (float)((int)code - R) * ebx2;
        }
    }
}

template <bool COMP>
__device__ __forceinline__ void levels_gen(float* v, uint32_t lane, const FieldDesc& fd,
                                           const FieldPlan& pl, const WinG& wi, SZI_G uint16_t* cb,
                                           const SZI_G float* ob, uint32_t* hist, uint32_t& cntR) {
#pragma unroll 1
    for (int l = fd.L; l >= 1; --l) {
        const int s = 1 << (l - 1);
        const float el = pl.el[l - 1], ebx2 = pl.ebx2[l - 1];
        const float inv = el == 0.0f ? 0.0f : pl.inv[l - 1];
        bool passed[3] = {false, false, false};
#pragma unroll 1
        for (int k = 0; k < fd.ndim; ++k) {
            const int d = pl.order[k];
            const int spl = pl.spline[d];
            if (spl == SPL_LIN)
                pass_gen<SPL_LIN, COMP>(v, lane, fd, wi, d, s, passed, el, ebx2, inv, cb, ob, hist, cntR);
            else if (spl == SPL_NAK)
                pass_gen<SPL_NAK, COMP>(v, lane, fd, wi, d, s, passed, el, ebx2, inv, cb, ob, hist, cntR);
            else
                pass_gen<SPL_NAT, COMP>(v, lane, fd, wi, d, s, passed, el, ebx2, inv, cb, ob, hist, cntR);
            passed[d] = true;
            wave_sync();
        }
    }
}

// the block's points (a grid of step 1), or its anchor points (step S) up
// to an extent per dimension
__device__ __forceinline__ Grid3 block_grid(const int* ext, int step, uint32_t& n) {
    Grid3 gr;
    uint32_t m[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        gr.step[j] = step;
        gr.off[j] = 0;
        m[j] = (uint32_t)((ext[j] - 1) / step + 1);
    }
    gr.f0.set(m[0]);
    gr.f1.set(m[1]);
    n = m[0] * m[1] * m[2];
    return gr;
}

__device__ __forceinline__ uint32_t anchor_index(const FieldDesc& fd, const WinG& wi, const int* c) {
    return (uint32_t)((wi.lo[0] + c[0]) / fd.S) +
           (uint32_t)fd.na[0] * ((uint32_t)((wi.lo[1] + c[1]) / fd.S) +
                                 (uint32_t)fd.na[1] * (uint32_t)((wi.lo[2] + c[2]) / fd.S));
}

__global__ __launch_bounds__(kThreads) void k_compress_gen(const FieldDesc* __restrict__ F,
                                                           const FieldPlan* __restrict__ P,
                                                           const uint64_t* __restrict__ goff,
                                                           uint64_t ngroups) {
    __shared__ float vbuf[kWaves][kGenMaxBlock];
    extern __shared__ uint32_t hist[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    float* v = vbuf[wave];
    int f = 0, hf = -1;
    uint32_t cntR = 0;
#pragma unroll 1
    for (GroupSeq gs = group_seq(ngroups); gs.ok(); gs.next()) {
        while (gs.g >= goff[f + 1]) ++f;
        if (f != hf) {   // uniform over the workgroup: groups never span fields
            if (hf >= 0) flush_hist(hist, cntR, F[hf]);
            clear_hist(hist, F[f].R);
            __syncthreads();
            hf = f;
        }
        const FieldDesc& fd = F[f];
        const uint32_t w = (uint32_t)(gs.g - goff[f]) * kWaves + gs.slot(wave);
        if (w >= (uint32_t)(fd.nwin[0] * fd.nwin[1] * fd.nwin[2])) continue;
        const WinG wi = make_wing(fd, w);
        const SZI_G float* in = gp(fd.in) + wi.gbase;
        uint32_t nb;
        const Grid3 bg = block_grid(wi.e, 1, nb);
#pragma unroll 1
        for (uint32_t t = lane; t < nb; t += 64) {
            int c[3];
            bg.at(t, c);
            v[c[0] + c[1] * wi.B0 + c[2] * wi.B01] =
                in[(uint64_t)c[0] + (uint64_t)c[1] * wi.n0 + (uint64_t)c[2] * wi.n01];
        }
        wave_sync();
        SZI_G uint16_t* cb = gp(fd.codes) + wi.gbase;
        levels_gen<true>(v, lane, fd, P[f], wi, cb, nullptr, hist, cntR);
        // owned anchors: their values losslessly, quant-code R, counted
        uint32_t na;
        const Grid3 ag = block_grid(wi.o, fd.S, na);
#pragma unroll 1
        for (uint32_t t = lane; t < na; t += 64) {
            int c[3];
            ag.at(t, c);
            gp(fd.anchors)[anchor_index(fd, wi, c)] = v[c[0] + c[1] * wi.B0 + c[2] * wi.B01];
            cb[(uint64_t)c[0] + (uint64_t)c[1] * wi.n0 + (uint64_t)c[2] * wi.n01] = (uint16_t)fd.R;
            atomicAdd(&hist[2 * fd.R + lane], 1u);
        }
        wave_sync();
    }
    if (hf >= 0) flush_hist(hist, cntR, F[hf]);
}

__global__ __launch_bounds__(kThreads) void k_decompress_gen(const FieldDesc* __restrict__ F,
                                                             const FieldPlan* __restrict__ P,
                                                             const uint64_t* __restrict__ goff,
                                                             uint64_t ngroups) {
    __shared__ float vbuf[kWaves][kGenMaxBlock];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    float* v = vbuf[wave];
    int f = 0;
    uint32_t unused = 0;
#pragma unroll 1
    for (GroupSeq gs = group_seq(ngroups); gs.ok(); gs.next()) {
        while (gs.g >= goff[f + 1]) ++f;
        const FieldDesc& fd = F[f];
        const uint32_t w = (uint32_t)(gs.g - goff[f]) * kWaves + gs.slot(wave);
        if (w >= (uint32_t)(fd.nwin[0] * fd.nwin[1] * fd.nwin[2])) continue;
        const WinG wi = make_wing(fd, w);
        // every point takes its code (as float bits), the anchors their values
        const SZI_G uint16_t* cb = gp(fd.codes) + wi.gbase;
        uint32_t nb;
        const Grid3 bg = block_grid(wi.e, 1, nb);
#pragma unroll 1
        for (uint32_t t = lane; t < nb; t += 64) {
            int c[3];
            bg.at(t, c);
            v[c[0] + c[1] * wi.B0 + c[2] * wi.B01] = __uint_as_float(
                (uint32_t)cb[(uint64_t)c[0] + (uint64_t)c[1] * wi.n0 + (uint64_t)c[2] * wi.n01]);
        }
        wave_sync();
        uint32_t na;
        const Grid3 ag = block_grid(wi.e, fd.S, na);
#pragma unroll 1
        for (uint32_t t = lane; t < na; t += 64) {
            int c[3];
            ag.at(t, c);
            v[c[0] + c[1] * wi.B0 + c[2] * wi.B01] = gp(fd.anchors)[anchor_index(fd, wi, c)];
        }
        wave_sync();
        SZI_G float* ob = gp(fd.out) + wi.gbase;
        levels_gen<false>(v, lane, fd, P[f], wi, nullptr, ob, nullptr, unused);
        uint32_t no;
        const Grid3 og = block_grid(wi.o, 1, no);
#pragma unroll 1
        for (uint32_t t = lane; t < no; t += 64) {
            int c[3];
            og.at(t, c);
            ob[(uint64_t)c[0] + (uint64_t)c[1] * wi.n0 + (uint64_t)c[2] * wi.n01] =
                v[c[0] + c[1] * wi.B0 + c[2] * wi.B01];
        }
        wave_sync();
    }
}

// ------------------------------------------------------- launchers
// The persistent grid is the number of workgroups resident at once
// (occupancy from the runtime x compute units) unless per_cu overrides it,
// rounded to whole L2 domains.
// occupancy of a kernel at an LDS size, asked of the runtime once per process
template <class K>
static int resident_per_cu(K kernel, size_t lds) {
    static std::mutex mu;
    static std::map<std::pair<const void*, size_t>, int> known;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), lds);
    auto it = known.find(key);
    if (it != known.end()) return it->second;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kThreads, lds) != hipSuccess ||
        occ < 1) {
        (void)hipGetLastError();
        occ = 2;
    }
    known[key] = occ;
    return occ;
}

template <class K>
static uint64_t resident_grid(K kernel, size_t lds, int num_cus, int per_cu, uint64_t ngroups) {
    const int occ = per_cu > 0 ? per_cu : resident_per_cu(kernel, lds);
    uint64_t grid = (uint64_t)num_cus * (uint64_t)occ;
    if (grid > ngroups) grid = ngroups;
    if (grid > (uint64_t)kXcds) grid -= grid % kXcds;
    return grid;
}

hipError_t launch_compress(int ndim, const FieldDesc* d_fields, const FieldPlan* d_plans,
                           const uint64_t* d_goff, uint64_t ngroups, int num_cus,
                           LaunchShape shape, int max_R, hipStream_t st) {
    if (ngroups == 0) return hipSuccess;
    const size_t lds = (size_t)(2 * max_R + 64) * sizeof(uint32_t);
    auto go = [&](auto k) {
        const uint64_t grid = resident_grid(k, lds, num_cus, shape.per_cu, ngroups);
        hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kThreads), lds, st, d_fields, d_plans,
                           d_goff, ngroups);
    };
    if (ndim == 3) go(k_compress<3, 3>);
    else if (ndim == 1) go(k_compress1d);
    else if (shape.variant == 1) go(k_compress<2, 4>);
    else go(k_compress<2, 3>);
    return hipGetLastError();
}

hipError_t launch_compress_gen(const FieldDesc* d_fields, const FieldPlan* d_plans,
                               const uint64_t* d_goff, uint64_t ngroups, int num_cus, int max_R,
                               hipStream_t st) {
    if (ngroups == 0) return hipSuccess;
    const size_t lds = (size_t)(2 * max_R + 64) * sizeof(uint32_t);
    const uint64_t grid = resident_grid(k_compress_gen, lds, num_cus, 0, ngroups);
    hipLaunchKernelGGL(k_compress_gen, dim3((unsigned)grid), dim3(kThreads), lds, st, d_fields,
                       d_plans, d_goff, ngroups);
    return hipGetLastError();
}

hipError_t launch_decompress_gen(const FieldDesc* d_fields, const FieldPlan* d_plans,
                                 const uint64_t* d_goff, uint64_t ngroups, int num_cus,
                                 hipStream_t st) {
    if (ngroups == 0) return hipSuccess;
    const uint64_t grid = resident_grid(k_decompress_gen, 0, num_cus, 0, ngroups);
    hipLaunchKernelGGL(k_decompress_gen, dim3((unsigned)grid), dim3(kThreads), 0, st, d_fields,
                       d_plans, d_goff, ngroups);
    return hipGetLastError();
}

hipError_t launch_decompress(int ndim, const FieldDesc* d_fields, const FieldPlan* d_plans,
                             const uint64_t* d_goff, uint64_t ngroups, int num_cus,
                             LaunchShape shape, hipStream_t st) {
    if (ngroups == 0) return hipSuccess;
    auto go = [&](auto k) {
        const uint64_t grid = resident_grid(k, 0, num_cus, shape.per_cu, ngroups);
        hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kThreads), 0, st, d_fields, d_plans,
                           d_goff, ngroups);
    };
    if (ndim == 3) go(k_decompress<3, 3>);
    else if (ndim == 1) go(k_decompress1d);
    else if (shape.variant == 1) go(k_decompress<2, 4>);
    else go(k_decompress<2, 3>);
    return hipGetLastError();
}

}  // namespace szi
