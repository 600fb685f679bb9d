// k_plan.hip -- value range, sampled spline profiling and the FP64 plan
// (Sec. V-C.1, Eq. 1, Sec. V-B.2, Sec. V-C.2) on gfx950.
#include "dev_common.h"

namespace szi {

// ------------------------------------------------------- value range
// Partial min / max / non-finite counts: kRangeBlocks blocks per field; the
// extra block x = 0 of each field runs its profiling (first, so that its
// serial work overlaps the streaming blocks).
__device__ void profile_field(const FieldDesc& f, FieldPlan& P);

__global__ __launch_bounds__(256) void k_range(const FieldDesc* __restrict__ F, float* pmin,
                                               float* pmax, uint32_t* pbad, FieldPlan* P) {
    const FieldDesc& f = F[blockIdx.y];
    if (blockIdx.x == 0) {
        profile_field(f, P[blockIdx.y]);
        return;
    }
    const uint32_t blk = blockIdx.x - 1;
    const SZI_G float* in = gp(f.in);
    const uint64_t n = f.npts;
    float mn = INFINITY, mx = -INFINITY;
    uint32_t bad = 0;
    const uint64_t stride = (uint64_t)kRangeBlocks * blockDim.x;
    uint64_t tid = (uint64_t)blk * blockDim.x + threadIdx.x;
    auto take = [&](float v) {
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
        bad += finite_bits(v) ? 0u : 1u;
    };
    // the values before the first 16-byte boundary one by one (a field's
    // values are 4-byte aligned), the aligned interior as quads, the rest
    // one by one
    const uint64_t lead0 = ((16u - (uint32_t)(reinterpret_cast<uintptr_t>(in) & 15u)) & 15u) / 4u;
    const uint64_t lead = lead0 < n ? lead0 : n;
    if (blk == 0 && threadIdx.x < lead) take(in[threadIdx.x]);
    uint64_t head = lead;
    {
        const SZI_G vf4* in4 = reinterpret_cast<const SZI_G vf4*>(in + lead);
        const uint64_t n4 = (n - lead) / 4;
        // a contiguous slice of quads per block, eight rows of 256 quads in
        // flight (each round reads 32 KB in a row; a grid-stride pattern, the
        // eight loads of a lane 8 MB apart, ran at 5.0 TB/s against 6.4)
        const uint64_t per = ((n4 + kRangeBlocks - 1) / kRangeBlocks + 255) / 256 * 256;
        const uint64_t beg = (uint64_t)blk * per, end = beg + per < n4 ? beg + per : n4;
        uint64_t i = beg + threadIdx.x;
        for (; i + 7 * 256 < end; i += 8 * 256) {
            vf4 a[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = __builtin_nontemporal_load(in4 + i + k * 256);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                take(a[k].x);
                take(a[k].y);
                take(a[k].z);
                take(a[k].w);
            }
        }
        for (; i < end; i += 256) {
            const vf4 a = in4[i];
            take(a.x);
            take(a.y);
            take(a.z);
            take(a.w);
        }
        head = lead + n4 * 4;
    }
    for (uint64_t i = head + tid; i < n; i += stride) take(in[i]);   // at most 3 values
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
        const uint64_t o = (uint64_t)blockIdx.y * kRangeBlocks + blk;
        pmin[o] = mn;
        pmax[o] = mx;
        pbad[o] = bad;
    }
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

// Sec. V-C.1 profiling of one field by threads 0-63 of a workgroup.
__device__ void profile_field(const FieldDesc& f, FieldPlan& P) {
    __shared__ double err[64][3][3];
    const int t = threadIdx.x;
    if (t >= 64) return;
    const int D = f.ndim;
    const int ns = D == 3 ? 64 : (D == 2 ? 16 : 4);   // 4^D samples
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 3; ++k) err[t][d][k] = 0.0;
    if (f.need_prof && t < ns) {
        int c[3];
        c[0] = sample_pos(f.n[0], t & 3);
        c[1] = sample_pos(f.n[1], (t >> 2) & 3);
        c[2] = D == 3 ? sample_pos(f.n[2], t >> 4) : 0;
        const int64_t st[3] = {1, f.n[0], (int64_t)f.n[0] * f.n[1]};
        const int64_t gi = c[0] + st[1] * c[1] + st[2] * c[2];
        const SZI_G float* in = gp(f.in);
        const float x = in[gi];
        for (int d = 0; d < D; ++d) {
            if (f.n[d] < 7) continue;
            const float a = in[gi - 3 * st[d]], b = in[gi - st[d]];
            const float cc = in[gi + st[d]], dd = in[gi + 3 * st[d]];
            const float pl = (b + cc) * 0.5f;
            const float pk = (9.0f * (b + cc) - (a + dd)) * 0.0625f;
            const float pn = (23.0f * (b + cc) - 3.0f * (a + dd)) / 40.0f;
            err[t][d][0] = fabs((double)x - (double)pl);
            err[t][d][1] = fabs((double)x - (double)pk);
            err[t][d][2] = fabs((double)x - (double)pn);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();   // one wave: threads 0-63
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // one thread per (dimension, spline) adds that error over the samples in
    // ascending order (the order a single thread adding them all would take)
    if (t < 9) {
        const int d = t / 3, e = t % 3;
        double s = 0.0;
        if (f.need_prof && d < D && f.n[d] >= 7) {
#pragma unroll 8
            for (int k = 0; k < ns; ++k) s = s + err[k][d][e];
        }
        P.prof[d][e] = s;
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

// The passes of a window in execution order, from the plan's order, splines
// and level bounds.  Along the pass dimension d the odd multiples of s;
// along dimensions already passed at this level the multiples of s, along
// those still to come the multiples of 2s (Sec. V-A).  The window kernels
// run the default anchor stride only, so the level count is a constant and
// every input sits in registers: the plan in global memory is only written.
struct PlanIn {
    int order[3], spline[3];
    float el[kMaxLevels], ebx2[kMaxLevels], inv[kMaxLevels];
};

// Pass np of the execution order (level L - np / ND, its np % ND-th pass);
// the descriptors past the last pass are cleared.  Passes are independent:
// one thread each, or a loop.
template <int ND>
__device__ void make_pass(FieldPlan& p, const PlanIn& in, uint32_t n0, uint32_t n01, int np) {
    using G = Geo<ND>;
    constexpr int L = G::SHS;
    if (np >= L * ND) {
        if (np < kMaxPasses) p.pass[np] = PassDesc{};
        return;
    }
    const int W[3] = {G::W0, G::W1, G::W2};
    const int ST[3] = {1, G::SY, G::SZ};
    const uint32_t GS[3] = {1u, n0, n01};
    int pos[3] = {0, 0, 0};   // place of each dimension in the order
#pragma unroll
    for (int k = 0; k < ND; ++k)
#pragma unroll
        for (int j = 0; j < ND; ++j)
            if (in.order[k] == j) pos[j] = k;
    {
        const int lvl = L - np / ND, k = np % ND;
        {
            PassDesc q{};
            const int d = in.order[k];
            // the other dimensions, ascending
            const int e = d == 0 ? 1 : 0;
            const int g = ND == 2 ? -1 : (d == 2 ? 1 : 2);
            // lines sit at multiples of s along dimensions this level has
            // already passed over, of 2 s along the others
            auto shift = [&](int j) { return pos[j] < k ? lvl - 1 : lvl; };
            const int she = shift(e);
            q.d = d;
            q.spl = in.spline[d];
            q.sh = lvl - 1;
            q.ne = (uint32_t)((W[e] >> she) + 1);
            q.le = ST[e] << she;
            q.de = e;
            q.she = she;
            q.ge = GS[e] << she;
            q.obe = 8u * (uint32_t)e;
            q.rne = (1 << she) - 1;
            if (g >= 0) {
                const int shg = shift(g);
                q.nlines = q.ne * (uint32_t)((W[g] >> shg) + 1);
                q.lf = ST[g] << shg;
                q.dg = g;
                q.shg = shg;
                q.gf = GS[g] << shg;
                q.obg = 8u * (uint32_t)g;
                q.rng = (1 << shg) - 1;
            } else {
                q.nlines = q.ne;
                q.lf = 0;
                q.dg = e;
                q.shg = 0;
                q.gf = 0;
            }
            q.magic = kMagic.v[q.ne];
            q.el = in.el[lvl - 1];
            q.ebx2 = in.ebx2[lvl - 1];
            q.inv = q.el == 0.0f ? 0.0f : in.inv[lvl - 1];
            p.pass[np] = q;
        }
    }
}

__device__ void make_pass(const FieldDesc& f, FieldPlan& p, const PlanIn& in, int np) {
    const uint32_t n0 = (uint32_t)f.n[0], n01 = n0 * (uint32_t)f.n[1];
    if (f.ndim == 3) make_pass<3>(p, in, n0, n01, np);
    else if (f.ndim == 2) make_pass<2>(p, in, n0, n01, np);
    // 1D: the line kernels take the level bounds and the spline directly
}


// Decompression prologue, one workgroup of kDecBlockChunks threads per
// Huffman decode block: the block's word count (the decoder's offsets come
// from these sums), a share of the field's outlier values scattered into
// the output (where the replay reads them), and, in the field's first
// block, the pass descriptors of the plan the header carried.
__global__ __launch_bounds__(kDecBlockChunks) void k_dec_prep(const FieldDesc* __restrict__ F,
                                                             FieldPlan* P, int nfields,
                                                             const uint64_t* __restrict__ boff,
                                                             uint32_t* bsum) {
    const int f = block_field(boff, nfields, blockIdx.x);
    const FieldDesc& fd = F[f];
    const uint64_t b = blockIdx.x - boff[f], nb = boff[f + 1] - boff[f];
    const uint64_t ch = b * kDecBlockChunks + threadIdx.x;
    uint32_t w = ch < fd.nchunks ? ((uint32_t)gp(fd.chunk_bits)[ch] + 31u) >> 5 : 0u;
    w = wave_sum(w);
    __shared__ uint32_t s[kDecBlockChunks / 64];
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = w;
    for (uint64_t k = b * kDecBlockChunks + threadIdx.x; k < fd.n_outliers;
         k += nb * kDecBlockChunks) {
        const uint32_t idx = gp(fd.outlier_idx)[k];
        if (idx < fd.npts) gp(fd.out)[idx] = gp(fd.outlier_val)[k];
    }
    if (b == 0 && threadIdx.x < kMaxPasses) {   // one pass descriptor per thread
        const FieldPlan& p = P[f];
        PlanIn in;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            in.order[k] = p.order[k];
            in.spline[k] = p.spline[k];
        }
#pragma unroll
        for (int l = 0; l < kMaxLevels; ++l) {
            in.el[l] = p.el[l];
            in.ebx2[l] = p.ebx2[l];
            in.inv[l] = p.inv[l];
        }
        make_pass(fd, P[f], in, (int)threadIdx.x);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int k = 0; k < kDecBlockChunks / 64; ++k) a += s[k];
        bsum[blockIdx.x] = a;
    }
}

__global__ __launch_bounds__(256) void k_plan(const FieldDesc* __restrict__ F, FieldPlan* P,
                                              const float* pmin, const float* pmax,
                                              const uint32_t* pbad) {
    // a copy of the field record: the plan's stores below then cannot make
    // the compiler load its members again (one wait each)
    const FieldDesc f = F[blockIdx.x];
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
    // the histogram the interpolation accumulates starts at zero
    for (int b = threadIdx.x; b < 2 * f.R; b += blockDim.x) gp(f.hist)[b] = 0u;
    __syncthreads();
    // thread 0: the range, the bound, alpha, the splines and the order; then
    // one thread per level for the level bounds and one per pass for the
    // pass descriptors (the same arithmetic, each value computed once)
    __shared__ PlanIn s_in;
    __shared__ double s_eabs, s_alpha;
    if (threadIdx.x == 0) {
        // the profiling's errors (k_range), read before the plan is written
        double prof[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 3; ++e) prof[d][e] = p.prof[d][e];
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
        s_eabs = p.e_abs;
        s_alpha = p.alpha;
        PlanIn& in = s_in;
        const int D = f.ndim;
        double score[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int s = d < D ? f.interp[d] : SPL_LIN;
            if (s == SPL_AUTO) s = prof[d][2] < prof[d][1] ? SPL_NAT : SPL_NAK;
            in.spline[d] = s;
            p.spline[d] = s;
            score[d] = prof[d][s];
        }
        if (f.order_req[0] >= 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) in.order[k] = k < D ? f.order_req[k] : -1;
        } else {
            // least smooth first; a strictly larger error wins, else the slower
            bool used[3] = {false, false, false};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (k >= D) {
                    in.order[k] = -1;
                    continue;
                }
                int best = -1;
#pragma unroll
                for (int d = 2; d >= 0; --d) {
                    if (d >= D || used[d]) continue;
                    if (best < 0 || score[d] > score[best]) best = d;
                }
                used[best] = true;
                in.order[k] = best;
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) p.order[k] = in.order[k];
    }
    __syncthreads();
    // level l: e_l = e / alpha^l rounded down to FP32, alpha^l as l products
    // in order from 1 (as one loop over the levels forms it)
    if (threadIdx.x < kMaxLevels) {
        const int l = (int)threadIdx.x;
        float el = 0.0f, ebx2 = 0.0f, inv = 0.0f;
        if (l < f.L) {
            double apow = 1.0;
            for (int i = 0; i < l; ++i) apow = apow * s_alpha;
            el = floor_to_f32(s_eabs / apow);
            ebx2 = 2.0f * el;
            inv = 1.0f / ebx2;
        }
        s_in.el[l] = el;
        s_in.ebx2[l] = ebx2;
        s_in.inv[l] = inv;
        p.el[l] = el;
        p.ebx2[l] = ebx2;
        p.inv[l] = inv;
    }
    __syncthreads();
    if (threadIdx.x < kMaxPasses) make_pass(f, p, s_in, (int)threadIdx.x);
}

// zero the histogram of every field (one y-row of workgroups per field)
__global__ void k_zero_hist(const FieldDesc* __restrict__ F) {
    const FieldDesc& f = F[blockIdx.y];
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < 2 * f.R; b += gridDim.x * blockDim.x)
        gp(f.hist)[b] = 0u;
}

// one workgroup per field: its histogram to dst + f * stride
__global__ void k_gather_hist(const FieldDesc* __restrict__ F, uint32_t* dst, uint32_t stride) {
    const FieldDesc& f = F[blockIdx.x];
    for (int b = threadIdx.x; b < 2 * f.R; b += blockDim.x)
        dst[(uint64_t)blockIdx.x * stride + b] = gp(f.hist)[b];
}

// one workgroup per field: its code lengths (padded to 16 bytes), codebook
// and decode tables, staged together at src + tab_src, to the block that
// holds them (the padded lengths end where cbook starts)
__global__ void k_scatter_tables(const FieldDesc* __restrict__ F, const uint8_t* __restrict__ src) {
    const FieldDesc& f = F[blockIdx.x];
    const int nsym = 2 * f.R;
    const uint32_t lenw = (uint32_t)((nsym + 15) & ~15) / 4;
    const uint32_t words = lenw + (uint32_t)nsym + (uint32_t)dtab_words(nsym);
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src + f.tab_src);
    uint32_t* d = const_cast<uint32_t*>(f.cbook) - lenw;
    for (uint32_t k = threadIdx.x; k < words; k += blockDim.x) gp(d)[k] = gp(s)[k];
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------- launchers
hipError_t launch_range(const FieldDesc* d_fields, FieldPlan* d_plans, int nfields,
                        float* d_part_min, float* d_part_max, uint32_t* d_part_bad,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_range, dim3(kRangeBlocks + 1, nfields), dim3(256), 0, st, d_fields,
                       d_part_min, d_part_max, d_part_bad, d_plans);
    return hipGetLastError();
}

hipError_t launch_plan(const FieldDesc* d_fields, FieldPlan* d_plans, int nfields,
                       const float* d_part_min, const float* d_part_max,
                       const uint32_t* d_part_bad, hipStream_t st) {
    hipLaunchKernelGGL(k_plan, dim3(nfields), dim3(256), 0, st, d_fields, d_plans, d_part_min,
                       d_part_max, d_part_bad);
    return hipGetLastError();
}

hipError_t launch_zero_hist(const FieldDesc* d_fields, int nfields, hipStream_t st) {
    if (nfields <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_hist, dim3(4, (unsigned)nfields), dim3(256), 0, st, d_fields);
    return hipGetLastError();
}

hipError_t launch_dec_prep(const FieldDesc* d_fields, FieldPlan* d_plans, int nfields,
                           const uint64_t* d_dboff, uint64_t nblocks, uint32_t* d_bsum,
                           hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dec_prep, dim3((unsigned)nblocks), dim3(kDecBlockChunks), 0, st, d_fields,
                       d_plans, nfields, d_dboff, d_bsum);
    return hipGetLastError();
}

hipError_t launch_gather_hist(const FieldDesc* d_fields, int nfields, uint32_t* dst,
                              uint32_t stride, hipStream_t st) {
    if (nfields <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_hist, dim3((unsigned)nfields), dim3(256), 0, st, d_fields, dst, stride);
    return hipGetLastError();
}

hipError_t launch_scatter_tables(const FieldDesc* d_fields, int nfields, const uint8_t* src,
                                 hipStream_t st) {
    if (nfields <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_tables, dim3((unsigned)nfields), dim3(256), 0, st, d_fields, src);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace szi
