// k_huff.hip -- chunked Huffman encode/decode with fused outlier compaction
// (Sec. VI-A) on gfx950.
//
// Encode: kEncChunks consecutive chunks of one field per workgroup (4 wave64,
// one chunk per wave at a time, C/64 consecutive symbols per lane).
//   k_huff_stats   bit count and outlier count of every chunk; sums per
//                  workgroup block
//   k_scan_blocks  exclusive scan of the block sums (one workgroup)
//   k_huff_encode  chunk offsets = block offset + in-block prefix; packs the
//                  codewords MSB-first through LDS and writes the outliers
//                  (index, original value) in ascending index order
// Decode: kDecChunks chunks per decode block, kSubParts lanes per chunk from
// the bit offsets of its parts that the encoder records (one lane per chunk
// without them).
//   k_dec_prep     (k_plan.hip) word count of every decode block
//   k_huff_decode  sum of the field's earlier block sums and an in-block
//                  scan, then a table-driven canonical decode from a
//                  two-word register window fed by a per-lane LDS word
//                  ring; 64 symbols per lane stored at once
#include "dev_common.h"

namespace szi {

constexpr int kEncChunks = 32;
constexpr int kDecChunks = 256;
static_assert(kEncChunks == kEncBlockChunks && kDecChunks == kDecBlockChunks,
              "the host sizes the Huffman grids with the same chunk counts");

// symbols [s0, s0 + per) of the code array (all inside the field)
template <int PER>
__device__ __forceinline__ void load_syms(const SZI_G uint16_t* __restrict__ codes, uint64_t s0,
                                          uint32_t* sym) {
    if (PER >= 8) {
        const SZI_G vu4* p = reinterpret_cast<const SZI_G vu4*>(codes + s0);
#pragma unroll
        for (int k = 0; k < PER / 8; ++k) {
            const vu4 w = p[k];
            const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                sym[8 * k + 2 * j] = ww[j] & 0xFFFFu;
                sym[8 * k + 2 * j + 1] = ww[j] >> 16;
            }
        }
    } else {
        const vu2 w = *reinterpret_cast<const SZI_G vu2*>(codes + s0);
        sym[0] = w.x & 0xFFFFu;
        sym[1] = w.x >> 16;
        sym[2] = w.y & 0xFFFFu;
        sym[3] = w.y >> 16;
    }
}

template <int PER>
__device__ __forceinline__ void lane_syms(const FieldDesc& fd, uint64_t ch, int lane,
                                          uint32_t* sym, int& nsym_lane) {
    const uint64_t s0 = ch * (uint64_t)(PER * 64) + (uint64_t)lane * PER;
    if (s0 + PER <= fd.npts) {
        load_syms<PER>(gp(fd.codes), s0, sym);
        nsym_lane = PER;
    } else {
        nsym_lane = s0 < fd.npts ? (int)(fd.npts - s0) : 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) sym[k] = k < nsym_lane ? gp(fd.codes)[s0 + k] : 0u;
    }
}

template <int PER>
__global__ __launch_bounds__(256) void k_huff_stats(const FieldDesc* __restrict__ F, int nfields,
                                                    const uint64_t* __restrict__ boff,
                                                    uint32_t* cwords, uint32_t* couts,
                                                    uint32_t* bw, uint32_t* bo) {
    extern __shared__ uint32_t cb[];
    __shared__ uint32_t sw[kEncChunks], so[kEncChunks];
    const int f = block_field(boff, nfields, blockIdx.x);
    const FieldDesc& fd = F[f];
    const int nsym = 2 * fd.R;
    // the field's non-zero word count, which its encode blocks add to
    if (threadIdx.x == 0 && blockIdx.x == boff[f] && fd.nzw) *gp(fd.nzw) = 0ull;
    for (int s = threadIdx.x; s < nsym; s += blockDim.x) cb[s] = gp(fd.cbook)[s];
    __syncthreads();
    const uint64_t first = (blockIdx.x - boff[f]) * kEncChunks;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = wave; j < kEncChunks; j += 4) {
        const uint64_t ch = first + j;
        uint32_t words = 0, zeros = 0;
        if (ch < fd.nchunks) {   // uniform across the wave
            uint32_t sym[PER];
            int ns;
            lane_syms<PER>(fd, ch, lane, sym, ns);
            // bits (< 2^16 per chunk) and outliers (<= 2048) summed as one
            // word: outliers in the high half
            static_assert(PER * 64 * kLmax < 65536, "chunk bits fit 16 bits");
            uint32_t bz = 0;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const bool live = k < ns;
                bz += live ? (cb[sym[k]] >> 24) + (sym[k] == 0 ? 0x10000u : 0u) : 0u;
            }
            bz = wave_sum(bz);
            const uint32_t bits = bz & 0xFFFFu;
            zeros = bz >> 16;
            words = (bits + 31) >> 5;
            if (lane == 0) {
                gp(fd.chunk_bits)[ch] = (uint16_t)bits;
                cwords[fd.chunk_base + ch] = words;
                couts[fd.chunk_base + ch] = zeros;
            }
        }
        if (lane == 0) {
            sw[j] = words;
            so[j] = zeros;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int j = 0; j < kEncChunks; ++j) {
            a += sw[j];
            b += so[j];
        }
        bw[blockIdx.x] = a;
        bo[blockIdx.x] = b;
    }
}

// Exclusive scan of up to two u32 arrays of length n into u64 offsets; one
// workgroup of 1024 threads, a contiguous run per thread: run sums, wave
// scans, the 16 wave totals through LDS (one barrier), then the run's
// offsets.  off[n] receives the total.  LONG = false takes runs of at
// most kRun (n <= 16384) in registers; LONG = true, longer runs kRun
// elements a round (the launchers choose by n).
template <bool LONG>
__global__ __launch_bounds__(1024) void k_scan_blocks(const uint32_t* __restrict__ a,
                                                      const uint32_t* __restrict__ b, uint64_t n,
                                                      uint64_t* aoff, uint64_t* boff) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint64_t per = (n + 1023) / 1024;
    const uint64_t beg = (uint64_t)t * per < n ? (uint64_t)t * per : n;
    const uint64_t end = beg + per < n ? beg + per : n;
    // runs of up to kRun elements sit in registers, all loads issued at once
    constexpr int kRun = 16;
    const bool regs = !LONG && per <= (uint64_t)kRun;   // LONG: runs of more than kRun
    uint32_t va[kRun], vb[kRun];
    uint64_t sa = 0, sb = 0;
    if (regs) {
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const uint64_t i = beg + k;
            va[k] = i < end ? a[i] : 0u;
            vb[k] = (b && i < end) ? b[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            sa += va[k];
            sb += vb[k];
        }
    } else if (LONG) {
        // longer runs (the LONG instance): kRun elements a round, their
        // loads issued together
        for (uint64_t i0 = beg; i0 < end; i0 += kRun) {
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const uint64_t i = i0 + k;
                va[k] = i < end ? a[i] : 0u;
                vb[k] = (b && i < end) ? b[i] : 0u;
            }
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                sa += va[k];
                sb += vb[k];
            }
        }
    }
    uint64_t xa = sa, xb = sb;   // inclusive scans over the wave's lanes
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t ya = __shfl_up(xa, o), yb = __shfl_up(xb, o);
        if (lane >= o) {
            xa += ya;
            xb += yb;
        }
    }
    __shared__ uint64_t wa[16], wb[16];
    if (lane == 63) {
        wa[wave] = xa;
        wb[wave] = xb;
    }
    __syncthreads();
    for (int k = 0; k < wave; ++k) {
        xa += wa[k];
        xb += wb[k];
    }
    uint64_t ra = xa - sa, rb = xb - sb;
    if (regs) {
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const uint64_t i = beg + k;
            if (i < end) {
                aoff[i] = ra;
                if (b) boff[i] = rb;
            }
            ra += va[k];
            rb += vb[k];
        }
    } else if (LONG) {
        for (uint64_t i0 = beg; i0 < end; i0 += kRun) {
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const uint64_t i = i0 + k;
                va[k] = i < end ? a[i] : 0u;
                vb[k] = (b && i < end) ? b[i] : 0u;
            }
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const uint64_t i = i0 + k;
                if (i < end) {
                    aoff[i] = ra;
                    if (b) boff[i] = rb;
                }
                ra += va[k];
                rb += vb[k];
            }
        }
    }
    if (t == 1023) {
        aoff[n] = xa;
        if (b) boff[n] = xb;
    }
}

// Orders the LDS accesses of one wave around this point (a wave's LDS
// instructions execute in issue order, so only the compiler needs holding).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// LDS words of one wave's chunk buffer: the longest chunk, one word for the
// low part of its last code (zero when that code ends in its first word),
// and one for the symbols past a chunk's end (a zero code at the chunk's
// last bit, whose two ORs of zeros then land one word further).
__host__ __device__ constexpr int enc_chunk_words(int chunk) { return (chunk * kLmax + 31) / 32 + 2; }

// One wave per chunk, PER consecutive symbols per lane: the wave scans the
// lanes' bit counts, ORs every code MSB first into the chunk's words in LDS
// and copies them out contiguously.  The waves of a workgroup share only
// the code book, so they synchronise among their own lanes.  (Packing a
// lane's codes in registers with plain stores for the words it owns, and
// loading the next chunk ahead, were both slower.)
template <int PER>
__global__ __launch_bounds__(256) void k_huff_encode(const FieldDesc* __restrict__ F, int nfields,
                                                     const uint64_t* __restrict__ boff,
                                                     const uint32_t* __restrict__ cwords,
                                                     const uint32_t* __restrict__ couts,
                                                     const uint64_t* __restrict__ bwoff,
                                                     const uint64_t* __restrict__ booff,
                                                     uint32_t* __restrict__ bnz) {
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t wnz[4];
    constexpr int C = PER * 64;
    constexpr int MCW = enc_chunk_words(C);
    const int f = block_field(boff, nfields, blockIdx.x);
    const FieldDesc& fd = F[f];
    const int nsym = 2 * fd.R;
    uint32_t* cb = smem;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t* wbuf = smem + nsym + wave * MCW;
    for (int s = threadIdx.x; s < nsym; s += blockDim.x) cb[s] = gp(fd.cbook)[s];
    const uint64_t blk_local = blockIdx.x - boff[f];
    const uint64_t first = blk_local * kEncChunks;
    // this field's sections start at 0: subtract the offsets of its first block
    const uint64_t wbase = bwoff[boff[f]], obase = booff[boff[f]];
    const uint64_t bw0 = bwoff[blockIdx.x] - wbase, bo0 = booff[blockIdx.x] - obase;
    // in-block exclusive prefix of the chunk word and outlier counts
    uint32_t cw = 0, co = 0;
    if (lane < kEncChunks && first + lane < fd.nchunks) {
        cw = cwords[fd.chunk_base + first + lane];
        co = couts[fd.chunk_base + first + lane];
    }
    uint32_t tw, to;
    const uint32_t pw = wave_excl_scan(cw, &tw);
    const uint32_t po = wave_excl_scan(co, &to);
    __syncthreads();   // the code book is in LDS
    uint32_t nz = 0;   // non-zero words written, for the zero-word elision of the blob
    for (int j = wave; j < kEncChunks; j += 4) {
        const uint64_t ch = first + j;
        if (ch >= fd.nchunks) break;   // uniform across the wave
        uint32_t sym[PER];
        int ns = 0;
        lane_syms<PER>(fd, ch, lane, sym, ns);
        // bits (< 2^16 per chunk) in the low half, outliers in the high half:
        // one scan gives both offsets
        static_assert(PER * 64 * kLmax < 65536, "chunk bits fit 16 bits");
        uint32_t e[PER];
        uint32_t bz = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const bool on = k < ns;
            e[k] = on ? cb[sym[k]] : 0u;
            bz += (e[k] >> 24) + ((on && sym[k] == 0) ? 0x10000u : 0u);
        }
        uint32_t tbz;
        const uint32_t pbz = wave_excl_scan(bz, &tbz);
        const uint32_t pos = pbz & 0xFFFFu, tb = tbz & 0xFFFFu;
        const uint32_t nw = (tb + 31) >> 5;
        for (uint32_t k = lane; k < nw; k += 64) wbuf[k] = 0;
        wave_lds_sync();
        {
            // every symbol ORs both words its code may touch, without
            // branches: the second takes the code's low part, zero when the
            // code ends in the first; a symbol past the chunk's end has the
            // zero entry (length 0, no bits) and ORs zeros
            uint32_t p = pos;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const uint32_t len = e[k] >> 24;
                const uint32_t wi = p >> 5, bo = p & 31;
                const uint64_t sh = (uint64_t)(e[k] & 0xFFFFFFu) << ((64u - len - bo) & 63u);   // MSB first
                atomicOr(&wbuf[wi], (uint32_t)(sh >> 32));
                atomicOr(&wbuf[wi + 1], (uint32_t)sh);
                p += len;
            }
        }
        if (tbz >> 16) {   // uniform: outliers in this chunk
            uint32_t zo = pbz >> 16;
            const uint64_t oo = bo0 + (uint32_t)__builtin_amdgcn_readlane((int)po, j);
            const uint64_t s0 = ch * (uint64_t)C + (uint64_t)lane * PER;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                if (k < ns && sym[k] == 0) {
                    if (oo + zo < fd.n_outliers) {   // the histogram sized the list
                        gp(fd.outlier_idx)[oo + zo] = (uint32_t)(s0 + k);
                        gp(fd.outlier_val)[oo + zo] = gp(fd.in)[s0 + k];
                    }
                    ++zo;
                }
            }
        }
        wave_lds_sync();
        const uint64_t ow = bw0 + (uint32_t)__builtin_amdgcn_readlane((int)pw, j);   // j is uniform
        for (uint32_t k = lane; k < nw; k += 64) {
            const uint32_t w = wbuf[k];
            nz += w != 0u;
            if (ow + k < fd.words_cap) gp(fd.words)[ow + k] = w;
        }
        if (fd.sub) {
            // the decoder's starting bits of the chunk's eighths (symbol
            // 8 k PER starts lane 8 k), as one 16-byte store: 0, b1 .. b7
            static_assert(kSubParts == 8, "eight parts: lanes 8, 16, .., 56");
            uint32_t b[8];
            b[0] = 0u;
#pragma unroll
            for (int k = 1; k < 8; ++k) b[k] = (uint32_t)__builtin_amdgcn_readlane((int)pos, 8 * k);
            if (lane == 0)
                *reinterpret_cast<SZI_G vu4*>(gp(fd.sub) + (uint64_t)kSubParts * ch) =
                    vu4{b[0] | (b[1] << 16), b[2] | (b[3] << 16), b[4] | (b[5] << 16), b[6] | (b[7] << 16)};
        }
        wave_lds_sync();
    }
    // one count per block, and one atomic per block for the field's total
    nz = wave_sum(nz);
    if (lane == 0) wnz[wave] = nz;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = wnz[0] + wnz[1] + wnz[2] + wnz[3];
        bnz[blockIdx.x] = t;
        if (fd.nzw) atomicAdd(fd.nzw, (unsigned long long)t);
    }
}

// One lane decodes one chunk: canonical decode with a 2^kLutBits table of
// u16 entries for short codes; a longer code's length comes from comparing
// the next bits with the per-length limits, without a loop or a
// data-dependent branch.  The next bits are a 32-bit window taken with one
// funnel shift from two words held in registers, w0:w1, at bit o of w0
// (1 <= o <= 32, so w1 is always whole and the window always has 32 valid
// bits; a lookup needs at most kLmax = 24).  When o passes 32 the words move
// up by one, w1 taking the next word, which every step has already read from
// the lane's ring, off the critical path of the table lookups.  The ring is
// 32 words per lane in LDS: once per group of 8 symbols every lane requests
// its next 8 words from global memory (two 16-byte loads, if the ring has
// room) and commits them to the ring one group later, so global loads sit at
// fixed points and their latency is covered by a group of decoding.  A group
// consumes at most 6 words and the ring always holds at least 7 ahead of the
// window.  Symbols leave 64 at a time per lane in eight back-to-back 16-byte
// stores.
//
// With Q = kSubParts (8) lanes per chunk, each lane decodes an eighth of
// the chunk's symbols from the bit offset the encoder recorded for it
// (fd.sub: eight per chunk, the first 0, kept with a compressed result):
// eight times the independent chains, each an eighth as long (against four
// lanes a chunk, 1 % faster at rel 1e-3, 5 % at 1e-4 and 38 % on a 64^3
// field).  A workgroup then covers an eighth of a decode block (kDecChunks
// chunks, whose word counts the prologue summed).  A field without offsets
// (an uploaded blob) is decoded by the first lane of each chunk.
constexpr int kRing = 32;   // ring words per lane (power of 2)

template <int Q>
__global__ __launch_bounds__(kDecChunks) void k_huff_decode(const FieldDesc* __restrict__ F,
                                                            int nfields,
                                                            const uint64_t* __restrict__ boff,
                                                            const uint32_t* __restrict__ bsum) {
    // the rings and the look-up table at fixed LDS addresses (a look-up's
    // address is then its index and an offset, with no base to add); the
    // limits, bases and sorted symbols, sized by the radius, after them
    __shared__ __align__(16) uint32_t rings[kDecChunks * kRing];
    __shared__ __align__(16) uint32_t lut32[kDtLimit];   // 2^kLutBits u16 entries
    __shared__ uint32_t scan[kDecChunks / 64];
    __shared__ uint64_t pre[kDecChunks / 64];
    extern __shared__ uint32_t tab_hi[];   // decode-table words kDtLimit .. dtab_words(nsym)
    static_assert(Q == 1 || Q == kSubParts, "one lane or kSubParts per chunk");
    constexpr int CPW = kDecChunks / Q;   // chunks per workgroup
    const uint64_t pblk = blockIdx.x / Q;   // the decode block
    const uint32_t part = blockIdx.x % Q;   // the workgroup's share of it
    const int f = block_field(boff, nfields, pblk);
    const FieldDesc& fd = F[f];
    const int nsym = 2 * fd.R;
    const int ntab = dtab_words(nsym);
    const uint16_t* lut = reinterpret_cast<const uint16_t*>(lut32);
    const int tid = threadIdx.x;
    {
        // the look-up table 16 bytes at a time, its four loads per lane in
        // flight together (word by word where the tables do not start on 16
        // bytes: odd radius), then the rest word by word
        const SZI_G uint32_t* src = gp(fd.dtab);
        static_assert(kDtLimit % (4 * kDecChunks) == 0, "whole rounds of 16-byte copies");
        if (((uintptr_t)fd.dtab & 15u) == 0u) {
            const SZI_G vu4* s4 = reinterpret_cast<const SZI_G vu4*>(src);
            vu4* d4 = reinterpret_cast<vu4*>(lut32);
            vu4 v[kDtLimit / (4 * kDecChunks)];
#pragma unroll
            for (int j = 0; j < kDtLimit / (4 * kDecChunks); ++j) v[j] = s4[tid + j * kDecChunks];
#pragma unroll
            for (int j = 0; j < kDtLimit / (4 * kDecChunks); ++j) d4[tid + j * kDecChunks] = v[j];
        } else {
            for (int k = tid; k < kDtLimit; k += kDecChunks) lut32[k] = src[k];
        }
        for (int k = kDtLimit + tid; k < ntab; k += kDecChunks) tab_hi[k - kDtLimit] = src[k];
    }
    // length limits of the codes longer than the LUT, in scalar registers
    uint32_t lim[kLmax - kLutBits - 1];
#pragma unroll
    for (int l = kLutBits + 1; l < kLmax; ++l)
        lim[l - kLutBits - 1] = __builtin_amdgcn_readfirstlane(gp(fd.dtab)[kDtLimit + l]);
    const uint32_t q = (uint32_t)tid % Q;   // the lane's part of its chunk
    const uint64_t bfirst = (pblk - boff[f]) * kDecChunks;   // the decode block's first chunk
    const uint64_t ch = bfirst + part * CPW + (uint64_t)tid / Q;
    const bool live = ch < fd.nchunks;
    const uint32_t cbits = live ? (uint32_t)gp(fd.chunk_bits)[ch] : 0u;
    const uint32_t nw = (cbits + 31) >> 5;
    // words of the field's earlier blocks (the sum of their word counts),
    // of this block's chunks before the workgroup's, and the workgroup's
    // exclusive scan of its chunks' word counts (each chunk counted once,
    // by its first lane)
    uint64_t pb = 0;
    for (uint64_t i = boff[f] + (uint64_t)tid; i < pblk; i += kDecChunks) pb += bsum[i];
    if (Q > 1)
        for (uint32_t k = (uint32_t)tid; k < part * CPW; k += kDecChunks)
            if (bfirst + k < fd.nchunks) pb += ((uint32_t)gp(fd.chunk_bits)[bfirst + k] + 31u) >> 5;
    for (int o = 32; o > 0; o >>= 1) pb += __shfl_xor(pb, o);
    uint32_t tot;
    const uint32_t wx = wave_excl_scan(q == 0 ? nw : 0u, &tot) - (q == 0 ? 0u : nw);
    if ((tid & 63) == 0) {
        scan[tid >> 6] = tot;
        pre[tid >> 6] = pb;
    }
    __syncthreads();
    uint64_t before = 0;
    for (int k = 0; k < kDecChunks / 64; ++k) before += pre[k];
    for (int k = 0; k < (tid >> 6); ++k) before += scan[k];
    const int C = fd.chunk;
    const bool split = Q > 1 && fd.sub != nullptr;   // the field has sub-chunk offsets
    const int SC = split ? C / Q : C;                // symbols per lane
    const uint64_t s0 = ch * (uint64_t)C + (uint64_t)(split ? q * (uint32_t)SC : 0u);
    int cnt = !live || (!split && q != 0) || s0 >= fd.npts ? 0
              : (s0 + SC <= fd.npts ? SC : (int)(fd.npts - s0));
    const uint32_t bo = split ? (uint32_t)gp(fd.sub)[(uint64_t)Q * ch + q] : 0u;   // entry 0 is 0
    if (bo > cbits) cnt = 0;   // a corrupt offset: nothing to decode from it
    if (cnt == 0) return;
    const uint64_t w0abs = before + wx + (bo >> 5);   // the lane's first word
    const uint32_t b0 = bo & 31u;                     // and bit in it
    // word indices count from the 4-aligned word at or below the lane's
    // first; requests stop after the word that holds the lane's last bit
    // (where the next part starts, else the chunk's end; the ring may
    // then hold stale words past it, which only fill a look-up's unused
    // low bits) and never pass the field's words (the array has kWordPad
    // words of slack, so the 8-word loads of the last request stay inside
    // it).  Stopping at the lane's own end saves a twentieth of decode time.
    const uint64_t wbase = w0abs & ~(uint64_t)3;
    const SZI_G uint32_t* words = gp(fd.words) + wbase;
    const uint32_t be0 = split && q + 1 < (uint32_t)Q ? (uint32_t)gp(fd.sub)[(uint64_t)Q * ch + q + 1] : cbits;
    const uint32_t be = be0 < bo || be0 > cbits ? cbits : be0;   // a corrupt offset: the chunk's end
    const uint64_t wlim0 = before + wx + ((be + 31u) >> 5);
    const uint64_t wlim = wlim0 < fd.words_cap ? wlim0 : fd.words_cap;
    const uint64_t wleft = wlim > wbase ? wlim - wbase : 0;
    const uint32_t wcap = wleft < (1u << 30) ? (uint32_t)wleft : (1u << 30);
    // the lane's ring: word i at ring[(i ^ sw) % kRing], the 16-byte groups
    // permuted per lane so that lanes at the same position hit different banks
    uint32_t* ring = rings + tid * kRing;
    const uint32_t sw = ((uint32_t)tid & (kRing / 4 - 1)) << 2;
    auto slot = [&](uint32_t i) SZI_INLINE { return (i ^ sw) & (uint32_t)(kRing - 1); };
    auto put = [&](uint32_t at, vu4 a, vu4 b) SZI_INLINE {   // words [at, at + 8) into the ring
        *reinterpret_cast<vu4*>(ring + slot(at)) = a;
        *reinterpret_cast<vu4*>(ring + slot(at + 4u)) = b;
    };
    uint32_t wr = 0;                              // next word to request
    uint32_t rd = (uint32_t)(w0abs - wbase);      // next word to read from the ring
    // prime the ring with 16 words
    {
        vu4 a = {0u, 0u, 0u, 0u}, b = a, c = a, d = a;
        if (wcap > 0) {
            a = *reinterpret_cast<const SZI_G vu4*>(words);
            b = *reinterpret_cast<const SZI_G vu4*>(words + 4);
        }
        if (wcap > 8) {
            c = *reinterpret_cast<const SZI_G vu4*>(words + 8);
            d = *reinterpret_cast<const SZI_G vu4*>(words + 12);
        }
        put(0u, a, b);
        put(8u, c, d);
        wr = 16;
    }
    // the window starts at bit b0 of the first word: the top of w1 (o = 32,
    // held as nego = -o) or bit b0 of w0
    uint32_t w0 = 0u, w1;
    int32_t nego;
    if (b0 == 0u) {
        w1 = ring[slot(rd)];
        ++rd;
        nego = -32;
    } else {
        w0 = ring[slot(rd)];
        w1 = ring[slot(rd + 1u)];
        rd += 2;
        nego = -(int32_t)b0;
    }
    uint32_t nxw = ring[slot(rd)];   // the ring word the next move takes
    auto decode_one = [&]() SZI_INLINE -> uint32_t {
        // bits [o, o + 32) of w0:w1 (the shift amount is 32 - o, taken mod 32)
        const uint32_t x = __builtin_amdgcn_alignbit(w0, w1, (uint32_t)nego);
        const uint32_t e = lut[x >> (32 - kLutBits)];
        uint32_t len = e >> kLutSymBits, sym = e & ((1u << kLutSymBits) - 1u);
        if (wave_any(len == 0)) {
            // longer than the table: the length is one more than the number
            // of length limits at or below the next kLmax bits (canonical
            // codes grow with their length), then one look-up
            const uint32_t w = x >> (32 - kLmax);
            uint32_t ln = kLutBits + 1;
#pragma unroll
            for (int l = kLutBits + 1; l < kLmax; ++l) ln += w >= lim[l - kLutBits - 1] ? 1u : 0u;
            const uint32_t i = tab_hi[kDtBase - kDtLimit + ln] + (w >> (kLmax - ln));
            const uint32_t sl = tab_hi[kDtSorted - kDtLimit + (i < (uint32_t)nsym ? i : 0u)];   // a corrupt stream stays inside
            const bool lng = len == 0;
            sym = lng ? sl : sym;
            len = lng ? ln : len;
        }
        // o += len; past 32 the words move up by one (len <= kLmax < 32)
        nego -= (int32_t)len;
        const bool t = nego < -32;
        w0 = t ? w1 : w0;
        w1 = t ? nxw : w1;
        nego += t ? 32 : 0;
        rd += t ? 1u : 0u;
        nxw = ring[slot(rd)];
        return sym;
    };
    SZI_G uint16_t* out = gp(fd.codes) + s0;   // s0: a multiple of 64 symbols
    const bool vec = ((uintptr_t)fd.codes & 15u) == 0u;   // s0 and k are multiples of 8
    // a group: commit the previous request, maybe request 8 more words,
    // then decode up to 8 symbols
    bool pend = false;
    uint32_t pat = 0;
    vu4 la = {0u, 0u, 0u, 0u}, lb = la;
    auto refill = [&]() SZI_INLINE {
        if (pend) put(pat, la, lb);
        // the ring holds [rd, wr) and a request adds 8; the prefetched word
        // at rd is not overwritten because the ring keeps kRing - 8 >= 7
        pend = wr < wcap && wr + 8 - rd <= (uint32_t)kRing;
        if (pend) {
            pat = wr;
            la = *reinterpret_cast<const SZI_G vu4*>(words + wr);
            lb = *reinterpret_cast<const SZI_G vu4*>(words + wr + 4);
            wr += 8;
        }
    };
    auto group8 = [&]() SZI_INLINE -> vu4 {
        refill();
        vu4 pk;
        uint32_t lo, hi;
        lo = decode_one();
        hi = decode_one();
        pk.x = lo | (hi << 16);
        lo = decode_one();
        hi = decode_one();
        pk.y = lo | (hi << 16);
        lo = decode_one();
        hi = decode_one();
        pk.z = lo | (hi << 16);
        lo = decode_one();
        hi = decode_one();
        pk.w = lo | (hi << 16);
        return pk;
    };
    int k = 0;
    // 64 symbols of a lane leave as eight back-to-back 16-byte stores, so
    // that a lane writes a whole 128-byte cache line at once (half lines
    // written far apart in time cost 15 % more decode time)
    if (vec) {
#pragma unroll 1
        for (; k + 64 <= cnt; k += 64) {
            vu4 p[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) p[j] = group8();
            SZI_G vu4* o = reinterpret_cast<SZI_G vu4*>(out + k);
#pragma unroll
            for (int j = 0; j < 8; ++j) o[j] = p[j];
        }
    }
#pragma unroll 1
    while (k < cnt) {
        refill();
        const int e = k + 8 < cnt ? k + 8 : cnt;
#pragma unroll 1
        for (; k < e; ++k) out[k] = (uint16_t)decode_one();
    }
}

// ------------------------------------------------------- zero-word elision
// The de-redundancy step after Huffman coding (taking the place of the
// closed pass of Sec. VI-B): the words section becomes a bitmap of the
// non-zero words (bit k % 32 of bitmap word k / 32 for word k) followed by
// those words in order.  Work is split into tiles of tw words (8192, or 2048
// for calls with few words), one wave per tile: a count pass, an exclusive
// scan of the tile counts over all fields (k_scan_blocks), and a write pass.  The restore (upload of an
// elided blob) runs the same tiling backwards: counts of set bits, scan,
// then each tile's words in place.
static_assert(kElideTileWords % 2048 == 0 && kElideTileSmall % 2048 == 0,
              "a tile is whole rounds of 32 ballots of 64 words");

__device__ __forceinline__ uint64_t elide_words(const ElideField& e) {
    return e.wbeg ? *e.wend - *e.wbeg : e.nw;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// restore = 0: non-zero words per tile of the words; 1: set bits per tile
// of the bitmap (the tile's 64 bitmap words)
template <int RESTORE>
__global__ __launch_bounds__(256) void k_elide_count(const ElideField* __restrict__ E, int nf,
                                                     const uint64_t* __restrict__ toff,
                                                     uint64_t ntiles, uint64_t tw, uint32_t* cnt) {
    // the wave's tile, uniform (so the field record and its pointers sit in
    // scalar registers, loaded once, not again before every word)
    const uint64_t tile = (uint64_t)blockIdx.x * 4 + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    if (tile >= ntiles) return;
    const int f = block_field(toff, nf, tile);
    const ElideField& e = E[f];
    const uint64_t nw = elide_words(e);
    const uint64_t w0 = (tile - toff[f]) * tw;
    const int rounds = (int)(tw / 2048);
    uint32_t n = 0;
    if (!RESTORE && e.nzw && (nw + 31) / 32 + *gp(e.nzw) >= nw) {
        // the field keeps its words: nothing to count
    } else if (RESTORE) {
        const uint64_t nbm = (nw + 31) / 32;
        const SZI_G uint32_t* sec = gp(e.sec);
        for (int j = 0; j < rounds; ++j) {
            const uint64_t b = w0 / 32 + (uint64_t)j * 64 + lane;
            n += (uint32_t)__popc(b < nbm ? sec[b] : 0u);
        }
        for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o);
    } else {
        // 32 loads in flight a round: unconditional loads at indices held
        // inside the words (a predicated load would be waited for at once),
        // the words past the end then taken as zero
        const SZI_G uint32_t* words = gp(e.words);
        const uint64_t last = nw > 0 ? nw - 1 : 0;
        for (int r = 0; r < rounds && nw > 0; ++r) {
            uint32_t w[32];
#pragma unroll
            for (int it = 0; it < 32; ++it) {
                const uint64_t i = w0 + (uint64_t)(r * 32 + it) * 64 + lane;
                w[it] = words[i < nw ? i : last];
            }
#pragma unroll
            for (int it = 0; it < 32; ++it) {
                const uint64_t i = w0 + (uint64_t)(r * 32 + it) * 64 + lane;
                w[it] = i < nw ? w[it] : 0u;
            }
#pragma unroll
            for (int it = 0; it < 32; ++it)
                n += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(w[it] != 0u));
        }
    }
    if (lane == 0) cnt[tile] = n;
}

// elision: bitmap words and non-zero words of a tile into e.sec, if the
// field's section is shorter than its words (else nothing is written)
__global__ __launch_bounds__(256) void k_elide_write(const ElideField* __restrict__ E, int nf,
                                                     const uint64_t* __restrict__ toff,
                                                     uint64_t ntiles, uint64_t tw,
                                                     const uint64_t* __restrict__ off) {
    // the wave's tile, uniform (so the field record and its pointers sit in
    // scalar registers, loaded once, not again before every word)
    const uint64_t tile = (uint64_t)blockIdx.x * 4 + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    if (tile >= ntiles) return;
    const int f = block_field(toff, nf, tile);
    const ElideField& e = E[f];
    const uint64_t nw = elide_words(e), nbm = (nw + 31) / 32;
    const uint64_t first = off[toff[f]];
    const uint64_t nz = e.nzw ? (uint64_t)*gp(e.nzw) : off[toff[f + 1]] - first;
    if (nbm + nz >= nw) return;
    const uint64_t w0 = (tile - toff[f]) * tw;
    if (w0 >= nw) return;
    uint64_t at = nbm + (off[tile] - first);
    SZI_G uint32_t* sec = gp(e.sec);
    const SZI_G uint32_t* words = gp(e.words);
    // rounds of 32 rows of 64 words, each round's loads in flight together
    for (int r = 0; r < (int)(tw / 2048); ++r) {
        uint32_t wv[32];
#pragma unroll
        for (int it = 0; it < 32; ++it) {
            const uint64_t i = w0 + (uint64_t)(r * 32 + it) * 64 + lane;
            wv[it] = i < nw ? words[i] : 0u;
        }
#pragma unroll
        for (int it = 0; it < 32; ++it) {
            const uint64_t i0 = w0 + (uint64_t)(r * 32 + it) * 64;
            const uint32_t w = wv[it];
            const uint64_t m = __builtin_amdgcn_ballot_w64(w != 0u);
            if (lane < 2 && i0 + 32 * lane < nw) sec[i0 / 32 + lane] = (uint32_t)(m >> (32 * lane));
            if (w) sec[at + lanes_below(m)] = w;
            at += (uint64_t)__popcll(m);
        }
    }
}

// restore: the words of a tile from the bitmap and the non-zero words
__global__ __launch_bounds__(256) void k_restore_write(const ElideField* __restrict__ E, int nf,
                                                       const uint64_t* __restrict__ toff,
                                                       uint64_t ntiles, uint64_t tw,
                                                       const uint64_t* __restrict__ off) {
    // the wave's tile, uniform (so the field record and its pointers sit in
    // scalar registers, loaded once, not again before every word)
    const uint64_t tile = (uint64_t)blockIdx.x * 4 + (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    if (tile >= ntiles) return;
    const int f = block_field(toff, nf, tile);
    const ElideField& e = E[f];
    const uint64_t nw = elide_words(e), nbm = (nw + 31) / 32;
    const uint64_t w0 = (tile - toff[f]) * tw;
    if (w0 >= nw) return;
    uint64_t at = nbm + (off[tile] - off[toff[f]]);
    const SZI_G uint32_t* sec = gp(e.sec);
#pragma unroll 4
    for (int it = 0; it < (int)(tw / 64); ++it) {
        const uint64_t i0 = w0 + (uint64_t)it * 64, i = i0 + lane;
        const uint32_t lo = i0 / 32 < nbm ? sec[i0 / 32] : 0u;
        const uint32_t hi = i0 / 32 + 1 < nbm ? sec[i0 / 32 + 1] : 0u;
        const uint64_t m = (uint64_t)lo | (uint64_t)hi << 32;
        const bool set = (m >> lane) & 1u;
        if (i < nw) gp(e.words)[i] = set ? sec[at + lanes_below(m)] : 0u;
        at += (uint64_t)__popcll(m);
    }
}

// ------------------------------------------------------- launchers
hipError_t launch_elide(const ElideField* d_e, int nf, const uint64_t* d_toff, uint64_t ntiles,
                        uint64_t tw, uint32_t* d_cnt, uint64_t* d_off, int restore, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    if (tw == 0 || tw % 2048 != 0) return hipErrorInvalidValue;
    const dim3 g((unsigned)((ntiles + 3) / 4)), b(256);
    if (restore) hipLaunchKernelGGL(k_elide_count<1>, g, b, 0, st, d_e, nf, d_toff, ntiles, tw, d_cnt);
    else hipLaunchKernelGGL(k_elide_count<0>, g, b, 0, st, d_e, nf, d_toff, ntiles, tw, d_cnt);
    if (ntiles > 16 * 1024)
        hipLaunchKernelGGL(k_scan_blocks<true>, dim3(1), dim3(1024), 0, st, d_cnt,
                           (const uint32_t*)nullptr, ntiles, d_off, (uint64_t*)nullptr);
    else
        hipLaunchKernelGGL(k_scan_blocks<false>, dim3(1), dim3(1024), 0, st, d_cnt,
                           (const uint32_t*)nullptr, ntiles, d_off, (uint64_t*)nullptr);
    if (restore) hipLaunchKernelGGL(k_restore_write, g, b, 0, st, d_e, nf, d_toff, ntiles, tw, d_off);
    else hipLaunchKernelGGL(k_elide_write, g, b, 0, st, d_e, nf, d_toff, ntiles, tw, d_off);
    return hipGetLastError();
}

hipError_t launch_huff_stats(const FieldDesc* d_fields, int nfields, const uint64_t* d_boff,
                             uint64_t nblocks, int chunk, uint32_t* d_cwords, uint32_t* d_couts,
                             uint32_t* d_bw, uint32_t* d_bo, int max_nsym, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const size_t lds = (size_t)max_nsym * sizeof(uint32_t);
    const dim3 g((unsigned)nblocks), b(256);
    switch (chunk) {
    case 256: hipLaunchKernelGGL(k_huff_stats<4>, g, b, lds, st, d_fields, nfields, d_boff, d_cwords, d_couts, d_bw, d_bo); break;
    case 512: hipLaunchKernelGGL(k_huff_stats<8>, g, b, lds, st, d_fields, nfields, d_boff, d_cwords, d_couts, d_bw, d_bo); break;
    case 1024: hipLaunchKernelGGL(k_huff_stats<16>, g, b, lds, st, d_fields, nfields, d_boff, d_cwords, d_couts, d_bw, d_bo); break;
    case 2048: hipLaunchKernelGGL(k_huff_stats<32>, g, b, lds, st, d_fields, nfields, d_boff, d_cwords, d_couts, d_bw, d_bo); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scan_blocks(const uint32_t* d_a, const uint32_t* d_b, uint64_t n,
                              uint64_t* d_aoff, uint64_t* d_boff, hipStream_t st) {
    if (n > 16 * 1024)
        hipLaunchKernelGGL(k_scan_blocks<true>, dim3(1), dim3(1024), 0, st, d_a, d_b, n, d_aoff, d_boff);
    else
        hipLaunchKernelGGL(k_scan_blocks<false>, dim3(1), dim3(1024), 0, st, d_a, d_b, n, d_aoff, d_boff);
    return hipGetLastError();
}

hipError_t launch_huff_encode(const FieldDesc* d_fields, int nfields, const uint64_t* d_boff,
                              uint64_t nblocks, int chunk, const uint32_t* d_cwords,
                              const uint32_t* d_couts, const uint64_t* d_bwoff,
                              const uint64_t* d_booff, uint32_t* d_bnz, int max_nsym,
                              hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const int mcw = enc_chunk_words(chunk);
    const size_t lds = ((size_t)max_nsym + 4 * (size_t)mcw) * sizeof(uint32_t);
    const dim3 g((unsigned)nblocks), b(256);
    switch (chunk) {
    case 256: hipLaunchKernelGGL(k_huff_encode<4>, g, b, lds, st, d_fields, nfields, d_boff, d_cwords, d_couts, d_bwoff, d_booff, d_bnz); break;
    case 512: hipLaunchKernelGGL(k_huff_encode<8>, g, b, lds, st, d_fields, nfields, d_boff, d_cwords, d_couts, d_bwoff, d_booff, d_bnz); break;
    case 1024: hipLaunchKernelGGL(k_huff_encode<16>, g, b, lds, st, d_fields, nfields, d_boff, d_cwords, d_couts, d_bwoff, d_booff, d_bnz); break;
    case 2048: hipLaunchKernelGGL(k_huff_encode<32>, g, b, lds, st, d_fields, nfields, d_boff, d_cwords, d_couts, d_bwoff, d_booff, d_bnz); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


hipError_t launch_huff_decode(const FieldDesc* d_fields, int nfields, const uint64_t* d_dboff,
                              uint64_t nblocks, const uint32_t* d_bsum, int max_nsym, int split,
                              hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    const size_t lds = (size_t)(dtab_words(max_nsym) - kDtLimit) *
                       sizeof(uint32_t);
    if (split)
        hipLaunchKernelGGL(k_huff_decode<kSubParts>, dim3((unsigned)(kSubParts * nblocks)), dim3(kDecChunks), lds, st,
                           d_fields, nfields, d_dboff, d_bsum);
    else
        hipLaunchKernelGGL(k_huff_decode<1>, dim3((unsigned)nblocks), dim3(kDecChunks), lds, st,
                           d_fields, nfields, d_dboff, d_bsum);
    return hipGetLastError();
}


}  // namespace szi
