// szi_internal.h -- structures shared by libszi's host code and its gfx950
// kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "szi_limits.h"

namespace szi {

constexpr int kLutBits = 13;       // decode look-up table width (bits)
constexpr int kRangeBlocks = 2048; // partial min/max blocks per field
constexpr int kThreads = 256;      // threads per interpolation workgroup
constexpr int kEncBlockChunks = 32;   // Huffman chunks per encode workgroup
constexpr int kDecBlockChunks = 256;  // Huffman chunks per decode workgroup
constexpr int kWordPad = 8;        // allocated u32 past the end of every Huffman word array

// Static description of one field, written by the host before launch.
// Decode lanes per Huffman chunk: the encoder records where each of a
// chunk's kSubParts equal parts starts, and one lane decodes each part.
constexpr int kSubParts = 8;

struct FieldDesc {
    int32_t ndim;
    int32_t n[3];          // n[0] fastest; unused dims 1
    int32_t w[3];          // window; unused dims 1
    int32_t nwin[3];       // windows per dimension
    int32_t na[3];         // anchors per dimension
    int32_t S, L, R;
    int32_t eb_mode;
    int32_t need_prof;
    int32_t interp[3];     // requested splines (AUTO allowed)
    int32_t order_req[3];  // requested order; order_req[0] < 0 = auto
    int32_t chunk;         // Huffman chunk
    double eb;
    double alpha_req;
    uint64_t npts;
    uint64_t chunk_base;   // first chunk of this field in a batch
    uint64_t tab_src;      // its code tables' offset in a batch's staged table region
    uint64_t nchunks;
    uint64_t n_outliers;
    uint64_t words_cap;    // capacity of words (encode)
    const float* in;       // compress input
    float* out;            // decompress output
    uint16_t* codes;
    float* anchors;
    uint32_t* hist;        // 2R bins
    // Huffman encode/decode
    const uint32_t* cbook; // per symbol: len << 24 | codeword
    uint32_t* words;
    uint16_t* chunk_bits;
    uint32_t* outlier_idx;
    float* outlier_val;
    const uint32_t* dtab;  // decode tables (see DecodeTables layout)
    unsigned long long* nzw;  // compress: the field's non-zero words (stats clears, encode adds)
    uint16_t* sub;         // per chunk kSubParts bit offsets: 0, then where its 2nd .. last eighth starts (or null)
};

// One pass of the interpolation (Sec. V-A: levels from stride S/2 to 1, one
// pass per dimension in the planned order), as the window kernels run it:
// the points of the pass lie on nlines lines along dimension d, line
// i0 + ne * i1 starting at LDS index i0 * le + i1 * lf of the block.
constexpr int kMaxPasses = 12;
// Lines of a pass are numbered i0 + ne * i1 over the two other dimensions
// e < g (i1 = 0 in 2D); line (i0, i1) lies at coordinate i0 << she along e
// and i1 << shg along g, at LDS offset i0 le + i1 lf and global offset
// i0 ge + i1 gf from the window origin.
struct PassDesc {
    int32_t d, spl, sh;        // dimension, spline, log2 of the stride
    uint32_t nlines, ne;
    uint32_t magic;            // multiply-high constant for division by ne
    int32_t le, lf;
    float el, ebx2, inv;       // level bound, 2 e_l, 1 / (2 e_l) (0 when e_l = 0)
    int32_t de, dg;            // the other dimensions (dg = de in 2D)
    int32_t she, shg;          // log2 of the line spacing along de and dg
    uint32_t ge, gf;
    uint32_t obe, obg;         // bit offsets of the owned extents along de and dg in a
                               // window's packed extents (8 bits a dimension)
    int32_t rne, rng;          // (1 << she) - 1 and (1 << shg) - 1
};

// Per-field plan computed on the device from the range and the profile.
struct FieldPlan {
    float vmin, vmax;
    uint32_t nonfinite;
    int32_t status;        // 0 ok, -2 non-finite input
    double range, eps, e_abs;
    float e;
    int32_t levels;
    double alpha;
    float el[kMaxLevels];
    float ebx2[kMaxLevels];
    float inv[kMaxLevels];
    int32_t spline[3];
    int32_t order[3];
    double prof[3][3];     // [dim][linear, NAK, natural] L1 errors
    PassDesc pass[kMaxPasses];   // derived from order, spline and e_l
};

// Windows are handed to the interpolation kernels in groups of this many,
// one per wave of a workgroup; each field is padded to whole groups.
constexpr int kWinPerGroup = 4;

// Decode tables, one u32 array per field:
//   LUT, 1<<kLutBits u16 entries in (1<<kLutBits)/2 words: len << 11 | symbol
//                      for the codes of at most kLutBits bits (symbols < 2048;
//                      len 0 = longer code)
//   limit[kLmax+1]     limit[l]: the codes of length <= l, left-justified to
//                      kLmax bits, lie below it ((first + count) << (kLmax - l))
//   base[kLmax+1]      base[l]: position of length l among the sorted
//                      symbols minus the first code of length l
//   sorted symbols (nsym entries, by (length, symbol))
constexpr int kLutSymBits = 11;
constexpr int kDtLimit = (1 << kLutBits) / 2;
constexpr int kDtBase = kDtLimit + kLmax + 1;
constexpr int kDtSorted = kDtBase + kLmax + 1;
static_assert(2 * kMaxRadius <= (1 << kLutSymBits) && kLutBits < (1 << (16 - kLutSymBits)),
              "LUT entries hold a symbol and a length in 16 bits");
__host__ __device__ inline int dtab_words(int nsym) { return kDtSorted + nsym; }

// ---- launchers (k_plan.hip, k_interp.hip, k_huff.hip) ----
// range partials and, in one extra block per field, the profiling (Sec. V-C.1)
hipError_t launch_range(const FieldDesc* d_fields, FieldPlan* d_plans, int nfields,
                        float* d_part_min, float* d_part_max, uint32_t* d_part_bad,
                        hipStream_t st);
hipError_t launch_plan(const FieldDesc* d_fields, FieldPlan* d_plans, int nfields,
                       const float* d_part_min, const float* d_part_max,
                       const uint32_t* d_part_bad, hipStream_t st);
hipError_t launch_zero_hist(const FieldDesc* d_fields, int nfields, hipStream_t st);
// decompression prologue: block word counts, outlier scatter, pass descriptors
hipError_t launch_dec_prep(const FieldDesc* d_fields, FieldPlan* d_plans, int nfields,
                           const uint64_t* d_dboff, uint64_t nblocks, uint32_t* d_bsum,
                           hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);
// batches: every field's histogram into dst + f * stride, and every field's
// code tables from the staged region src (at tab_src) to its table block
// (the 16-byte-padded lengths before cbook)
hipError_t launch_gather_hist(const FieldDesc* d_fields, int nfields, uint32_t* dst,
                              uint32_t stride, hipStream_t st);
hipError_t launch_scatter_tables(const FieldDesc* d_fields, int nfields, const uint8_t* src,
                                 hipStream_t st);
// Launch shape of a window kernel; every shape gives the same results.
// variant 0: compiled for three waves per SIMD (168 VGPRs); variant 1: for
// four (128 VGPRs; 2D only, whose smaller blocks leave LDS for 16 windows
// per CU).  per_cu: persistent workgroups per CU, 0 = resident capacity.
struct LaunchShape {
    int variant = 0;
    int per_cu = 0;
};
constexpr int kShapeVariants = 2;
hipError_t launch_compress(int ndim, const FieldDesc* d_fields, const FieldPlan* d_plans,
                           const uint64_t* d_goff, uint64_t ngroups, int num_cus,
                           LaunchShape shape, int max_R, hipStream_t st);
// Fields of any anchor stride and window (block points <= kGenMaxBlock):
// the generic window kernels, geometry from the descriptors.
hipError_t launch_compress_gen(const FieldDesc* d_fields, const FieldPlan* d_plans,
                               const uint64_t* d_goff, uint64_t ngroups, int num_cus, int max_R,
                               hipStream_t st);
hipError_t launch_decompress_gen(const FieldDesc* d_fields, const FieldPlan* d_plans,
                                 const uint64_t* d_goff, uint64_t ngroups, int num_cus,
                                 hipStream_t st);
hipError_t launch_decompress(int ndim, const FieldDesc* d_fields, const FieldPlan* d_plans,
                             const uint64_t* d_goff, uint64_t ngroups, int num_cus,
                             LaunchShape shape, hipStream_t st);
hipError_t launch_huff_stats(const FieldDesc* d_fields, int nfields, const uint64_t* d_boff,
                             uint64_t nblocks, int chunk, uint32_t* d_cwords, uint32_t* d_couts,
                             uint32_t* d_bw, uint32_t* d_bo, int max_nsym, hipStream_t st);
hipError_t launch_scan_blocks(const uint32_t* d_a, const uint32_t* d_b, uint64_t n,
                              uint64_t* d_aoff, uint64_t* d_boff, hipStream_t st);
// d_bnz: per encode block, the number of non-zero words it wrote (each
// block also adds it to its field's *nzw, where nzw is set)
hipError_t launch_huff_encode(const FieldDesc* d_fields, int nfields, const uint64_t* d_boff,
                              uint64_t nblocks, int chunk, const uint32_t* d_cwords,
                              const uint32_t* d_couts, const uint64_t* d_bwoff,
                              const uint64_t* d_booff, uint32_t* d_bnz, int max_nsym,
                              hipStream_t st);
// Zero-word elision of one field's Huffman words: words (the field's word
// array), sec (the elided section: bitmap words, then the non-zero words;
// capacity (n_words + 31) / 32 + n_words), and the word count, either n or
// read on the device as *wend - *wbeg (the field's block word offsets).
// nzw, when set, is the field's count of non-zero words from the encoder:
// a field that does not elide is then skipped without reading its words.
struct ElideField {
    uint32_t* words;
    uint32_t* sec;
    const uint64_t* wbeg;
    const uint64_t* wend;
    const unsigned long long* nzw;
    uint64_t nw;
};
// Elision tiles: 8192 words, or 2048 where the call has few words (then
// four times the waves share them, each with one round of loads instead of
// four); the tile size only splits the work, the section is the same.
constexpr uint64_t kElideTileWords = 8192;
constexpr uint64_t kElideTileSmall = 2048;
inline uint64_t elide_tile_words(uint64_t words) {
    return words < (uint64_t)1024 * kElideTileSmall ? kElideTileSmall : kElideTileWords;
}
// restore = 0: elide words into sec where that is shorter; 1: restore words
// from sec.  Fields own the tiles [toff[f], toff[f + 1]) of tw words (a
// multiple of 2048); cnt and off (u32[ntiles], u64[ntiles + 1]) are scratch.
hipError_t launch_elide(const ElideField* d_e, int nf, const uint64_t* d_toff, uint64_t ntiles,
                        uint64_t tw, uint32_t* d_cnt, uint64_t* d_off, int restore, hipStream_t st);
// d_bsum: the word count of every decode block (launch_dec_prep)
// split: every field has sub-chunk offsets (kSubParts lanes per chunk)
hipError_t launch_huff_decode(const FieldDesc* d_fields, int nfields, const uint64_t* d_dboff,
                              uint64_t nblocks, const uint32_t* d_bsum, int max_nsym, int split,
                              hipStream_t st);

// ---- the entry point that allocates nothing (noalloc.hip) ----
// Workspace of sz_decompress_noalloc: a static device array of this many
// bytes per GPU, holding the decoded quant-codes (2 bytes per point) and the
// call's descriptors; fields of up to kNoAllocMaxPoints points.
constexpr uint64_t kNoAllocMaxPoints = 1ull << 25;
constexpr uint64_t kNoAllocScratchBytes = 2 * kNoAllocMaxPoints + (1ull << 20);
// the device address of this GPU's workspace; called with device current
hipError_t noalloc_scratch(int device, void** ptr);
// up to kStageWordsMax u32 written to dst by a kernel that takes them as
// its argument
constexpr int kStageWordsMax = 896;
struct StageWords {
    uint32_t n;
    uint32_t w[kStageWordsMax];
};
hipError_t launch_stage_words(uint32_t* dst, const StageWords& a, hipStream_t st);

}  // namespace szi
