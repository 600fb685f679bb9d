// dev_common.h -- device helpers shared by libszi's gfx950 kernels.
#pragma once

#include <float.h>
#include <math.h>

#include "szi_internal.h"

namespace szi {

// Pointers read from a descriptor are generic to the compiler, which then
// emits flat memory instructions: 64-bit VGPR addresses, and each access
// also counts against the LDS wait counter.  Casting them to the global
// address space gives global_* instructions with a scalar base.
#define SZI_G __attribute__((address_space(1)))
// for lambdas in kernels: their bodies must not become calls
#define SZI_INLINE __attribute__((always_inline))
template <class T>
__device__ __forceinline__ SZI_G T* gp(T* p) {
    return (SZI_G T*)p;
}
template <class T>
__device__ __forceinline__ const SZI_G T* gp(const T* p) {
    return (const SZI_G T*)p;
}
// builtin vectors for wide global loads (no constructors, so they load
// through address-space-qualified pointers)
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef uint32_t vu4 __attribute__((ext_vector_type(4)));
typedef uint32_t vu2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void gatomic_add(SZI_G uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// lane masks straight from a condition (no 0/1 value in a vector register)
__device__ __forceinline__ bool wave_any(bool c) { return __builtin_amdgcn_ballot_w64(c) != 0; }
__device__ __forceinline__ uint64_t wave_ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }

// ------------------------------------------------------------- helpers
__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
// Inclusive prefix sum across the 64 lanes of a wave (all lanes active)
// with DPP lane moves: shifts by 1, 2, 4 and 8 within each row of 16 lanes,
// then the last lane of each row added to the next row (row_bcast:15 into
// rows 1 and 3) and lane 31 added to rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    constexpr int kRowShr = 0x110, kBcast15 = 0x142, kBcast31 = 0x143;
    const int x = (int)v;
    int s = x + __builtin_amdgcn_update_dpp(0, x, kRowShr + 1, 0xF, 0xF, false);
    s += __builtin_amdgcn_update_dpp(0, s, kRowShr + 2, 0xF, 0xF, false);
    s += __builtin_amdgcn_update_dpp(0, s, kRowShr + 4, 0xF, 0xF, false);
    s += __builtin_amdgcn_update_dpp(0, s, kRowShr + 8, 0xF, 0xF, false);
    s += __builtin_amdgcn_update_dpp(0, s, kBcast15, 0xA, 0xF, false);
    s += __builtin_amdgcn_update_dpp(0, s, kBcast31, 0xC, 0xF, false);
    return (uint32_t)s;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}
// exclusive prefix sum across the 64 lanes of a wave (all lanes active)
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total) {
    const uint32_t x = wave_incl_scan(v);
    *total = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
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
static __constant__ MagicTable kMagic = MagicTable();

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

// Window geometry of the interpolation kernels (Sec. V-D): the window a
// wave owns, its block (window + far faces) and the block's LDS strides.
template <int ND>
struct Geo;
template <>
struct Geo<3> {
    static constexpr int W0 = 32, W1 = 8, W2 = 8;   // window
    static constexpr int B0 = 33, B1 = 9, B2 = 9;   // block (window + far faces)
    static constexpr int SY = 33, SZ = 297;         // LDS strides
    static constexpr int BN = B0 * B1 * B2;
    static constexpr int SHS = 3;                   // log2 of the anchor stride
    static constexpr int NPRE = 43;                 // block values per lane
    static constexpr int NANCH = 20;                // anchors in a block
};
template <>
struct Geo<2> {
    static constexpr int W0 = 64, W1 = 16, W2 = 1;
    static constexpr int B0 = 65, B1 = 17, B2 = 1;
    static constexpr int SY = 65, SZ = 0;
    static constexpr int BN = B0 * B1;
    static constexpr int SHS = 4;
    static constexpr int NPRE = 18;
    static constexpr int NANCH = 10;
};
// spline kinds per dimension (include/szi.h sz_interp)
enum { SPL_LIN = 0, SPL_NAK = 1, SPL_NAT = 2, SPL_AUTO = 3 };

// field of a block index given prefix offsets boff[0..nfields]
__device__ __forceinline__ int block_field(const uint64_t* __restrict__ boff, int nfields,
                                           uint64_t b) {
    int lo = 0, hi = nfields - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace szi
