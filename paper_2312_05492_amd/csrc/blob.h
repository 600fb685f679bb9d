// blob.h -- the blob's byte layout (include/szi.h documents it) and its
// validation, as host code without HIP, so that it builds and runs by
// itself (the sanitizer tests build it with the host compiler).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "szi.h"
#include "szi_limits.h"

namespace szi {

// A field's geometry as the kernels take it: dimensions (n[0] fastest),
// anchor stride S, levels L, window, windows and anchors per dimension,
// quantiser radius R and Huffman chunk.
struct Geometry {
    int ndim, n[3], S, L, w[3], nwin[3], na[3], R, chunk;
    uint64_t npts, nanch, nwin_total, nchunks;
    bool generic;   // not the default stride and window: the generic window kernels
};

// The geometry of a field with these dimensions and parameters, or
// SZ_ERR_INVALID_ARG / SZ_ERR_UNSUPPORTED with the reason in *err.
sz_status check_geometry(const sz_dims* d, const sz_params* p, Geometry& g, std::string* err);

// little-endian fields at byte offsets
void put32(uint8_t* h, uint64_t off, uint32_t v);
void put64(uint8_t* h, uint64_t off, uint64_t v);
void putf(uint8_t* h, uint64_t off, float v);
void putd(uint8_t* h, uint64_t off, double v);
uint32_t get32(const uint8_t* h, uint64_t off);
uint64_t get64(const uint8_t* h, uint64_t off);
float getf(const uint8_t* h, uint64_t off);
double getd(const uint8_t* h, uint64_t off);
inline uint64_t pad8(uint64_t b) { return (b + 7) & ~(uint64_t)7; }

// CRC-32 (IEEE 802.3, reflected, as zlib's crc32)
uint32_t crc32_update(uint32_t crc, const uint8_t* p, size_t n);

// code lengths of nsym symbols: every length <= kLmax, at least one code,
// Kraft sum <= 1
bool kraft_ok(const uint8_t* len, int nsym);

// Zero-word elision of the words section (the blob's de-redundancy step
// after Huffman coding): a bitmap, bit k % 32 of bitmap word k / 32 set for
// a non-zero word k, then the non-zero words in order; used when shorter.
constexpr uint32_t kFlagWordsElided = 1;
inline uint64_t elided_words(uint64_t n_words, uint64_t nzw) { return (n_words + 31) / 32 + nzw; }

// bytes of a blob with these section sizes (each section padded to 8 bytes)
uint64_t blob_bytes(uint64_t n_anchors, int R, uint64_t n_chunks, uint64_t words_bytes,
                    uint64_t n_outliers);

// Everything a blob says, checked: the header, its CRC and sizes, every
// section's CRC and zero padding, the words (the elided form's bitmap and
// kept words), chunk bit counts that account for exactly the stored words,
// outlier indices inside the field, code lengths that form a prefix code,
// splines and a processing order.
struct BlobInfo {
    sz_dims dims;
    sz_params params;
    Geometry geo;
    uint64_t n_anchors, n_chunks, n_words, n_outliers;
    bool elided;
    uint64_t wsec;     // words of the words section as stored
    uint64_t nzw;      // non-zero words
    uint64_t off[6];   // section offsets: anchors, lengths, chunk bits, words, outlier idx, val
    uint64_t secb[6];  // section bytes without padding
    double alpha;
    float vmin, vmax, e;
    float el[16];
    int32_t spline[3], order[3];
};

// SZ_OK, or SZ_ERR_CORRUPT / SZ_ERR_UNSUPPORTED with the reason in *err.
// Reads no byte outside [b, b + bytes).
sz_status parse_blob(const uint8_t* b, uint64_t bytes, BlobInfo* out, std::string* err);

}  // namespace szi
