// blob.cpp -- the blob's byte layout and its validation (host code, no HIP).
#include "blob.h"

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

namespace szi {

namespace {

sz_status bad(std::string* err, sz_status s, const char* fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (err) *err = buf;
    return s;
}

}  // namespace

sz_status check_geometry(const sz_dims* d, const sz_params* p, Geometry& g, std::string* err) {
    if (!d || !p) return bad(err, SZ_ERR_INVALID_ARG, "null dims or params");
    if (d->ndim < 1 || d->ndim > 3)
        return bad(err, SZ_ERR_UNSUPPORTED, "ndim %u (1, 2 and 3 are supported)", d->ndim);
    g.ndim = (int)d->ndim;
    uint64_t npts = 1;
    for (int k = 0; k < 3; ++k) {
        if (k < g.ndim) {
            if (d->n[k] == 0 || d->n[k] >= (1ull << 31))
                return bad(err, SZ_ERR_INVALID_ARG, "n[%d] = %llu", k, (unsigned long long)d->n[k]);
            g.n[k] = (int)d->n[k];
            npts *= d->n[k];
            if (npts >= 0xFFFFFFFFull)
                return bad(err, SZ_ERR_INVALID_ARG, "field of more than 2^32 - 2 points");
        } else {
            g.n[k] = 1;
        }
    }
    g.npts = npts;
    if (p->eb_mode != SZ_EB_ABS && p->eb_mode != SZ_EB_REL)
        return bad(err, SZ_ERR_INVALID_ARG, "eb_mode %d", p->eb_mode);
    if (!(p->eb >= 0.0) || p->eb > 1e300) return bad(err, SZ_ERR_INVALID_ARG, "error bound %g", p->eb);
    if (!(p->alpha <= 1e300)) return bad(err, SZ_ERR_INVALID_ARG, "alpha %g", p->alpha);
    if (p->alpha > 0.0 && p->alpha < 1.0) return bad(err, SZ_ERR_INVALID_ARG, "alpha %g < 1", p->alpha);
    for (int k = 0; k < g.ndim; ++k)
        if (p->interp[k] < 0 || p->interp[k] > 3)
            return bad(err, SZ_ERR_INVALID_ARG, "interp[%d] = %d", k, p->interp[k]);
    if (p->order[0] >= 0) {
        int seen = 0;
        for (int k = 0; k < g.ndim; ++k) {
            if (p->order[k] < 0 || p->order[k] >= g.ndim || (seen >> p->order[k]) & 1)
                return bad(err, SZ_ERR_INVALID_ARG, "order is not a permutation");
            seen |= 1 << p->order[k];
        }
    }
    const uint32_t R = p->radius ? p->radius : 512;
    if (R < 2 || R > (uint32_t)kMaxRadius)
        return bad(err, SZ_ERR_UNSUPPORTED, "radius %u (2..%d supported)", R, kMaxRadius);
    g.R = (int)R;
    const uint32_t chunk = p->huff_chunk ? p->huff_chunk : 1024;
    if (chunk != 256 && chunk != 512 && chunk != 1024 && chunk != 2048)
        return bad(err, SZ_ERR_UNSUPPORTED, "Huffman chunk %u", chunk);
    g.chunk = (int)chunk;
    // Sec. V-A: chunks of 8^3, 16^2 or 512 points by default; a window spans
    // four chunks along x and one along the other dimensions.  Other strides
    // (powers of two, at most kMaxLevels levels) and windows (multiples of
    // the stride) run the generic window kernels.
    const int Sdef = g.ndim == 3 ? 8 : (g.ndim == 2 ? 16 : 512);
    const uint32_t S = p->anchor_stride ? p->anchor_stride : (uint32_t)Sdef;
    if (S < 2 || (S & (S - 1)) || S > (1u << kMaxLevels))
        return bad(err, SZ_ERR_UNSUPPORTED, "anchor stride %u (powers of two 2..%d)", S, 1 << kMaxLevels);
    int L = 0;
    while ((1u << L) < S) ++L;
    g.S = (int)S;
    g.L = L;
    g.generic = (int)S != Sdef;
    const int wdef[3] = {4 * (int)S, g.ndim >= 2 ? (int)S : 1, g.ndim == 3 ? (int)S : 1};
    int wk[3] = {1, 1, 1};
    uint64_t block = 1;
    for (int k = 0; k < g.ndim; ++k) {
        const uint32_t w = p->window[k] ? p->window[k] : (uint32_t)wdef[k];
        if (w % S || w > (uint32_t)kGenMaxExtent * 4)
            return bad(err, SZ_ERR_UNSUPPORTED, "window[%d] = %u (a multiple of the stride %u)", k, w, S);
        wk[k] = (int)w;
        block *= (uint64_t)w + 1;
        if ((int)w != (k == 0 ? 4 * Sdef : Sdef)) g.generic = true;
    }
    if (g.generic) {
        for (int k = 0; k < g.ndim; ++k)
            if (wk[k] > kGenMaxExtent)
                return bad(err, SZ_ERR_UNSUPPORTED, "window[%d] = %d (other windows: at most %d)", k,
                           wk[k], kGenMaxExtent);
        if (block > (uint64_t)kGenMaxBlock)
            return bad(err, SZ_ERR_UNSUPPORTED, "window block of %llu points (other windows: at most %d)",
                       (unsigned long long)block, kGenMaxBlock);
    }
    g.nwin_total = 1;
    g.nanch = 1;
    for (int k = 0; k < 3; ++k) {
        g.w[k] = wk[k];
        g.nwin[k] = (g.n[k] + g.w[k] - 1) / g.w[k];
        g.na[k] = k < g.ndim ? (g.n[k] + (int)S - 1) / (int)S : 1;
        g.nwin_total *= (uint64_t)g.nwin[k];
        g.nanch *= (uint64_t)g.na[k];
    }
    // the window kernels address a block by 32-bit byte offsets from its
    // origin and number windows with 32-bit integers
    const uint64_t span = (uint64_t)g.w[0] + (g.ndim >= 2 ? (uint64_t)g.w[1] * (uint64_t)g.n[0] : 0) +
                          (g.ndim == 3 ? (uint64_t)g.w[2] * (uint64_t)g.n[0] * (uint64_t)g.n[1] : 0);
    if ((!g.generic && span * sizeof(float) >= (1ull << 32)) || g.nwin_total >= (1ull << 31))
        return bad(err, SZ_ERR_UNSUPPORTED, "field planes too large (window span %llu points)",
                   (unsigned long long)span);
    g.nchunks = (npts + (uint64_t)g.chunk - 1) / (uint64_t)g.chunk;
    return SZ_OK;
}

void put32(uint8_t* h, uint64_t off, uint32_t v) { std::memcpy(h + off, &v, 4); }
void put64(uint8_t* h, uint64_t off, uint64_t v) { std::memcpy(h + off, &v, 8); }
void putf(uint8_t* h, uint64_t off, float v) { std::memcpy(h + off, &v, 4); }
void putd(uint8_t* h, uint64_t off, double v) { std::memcpy(h + off, &v, 8); }
uint32_t get32(const uint8_t* h, uint64_t off) { uint32_t v; std::memcpy(&v, h + off, 4); return v; }
uint64_t get64(const uint8_t* h, uint64_t off) { uint64_t v; std::memcpy(&v, h + off, 8); return v; }
float getf(const uint8_t* h, uint64_t off) { float v; std::memcpy(&v, h + off, 4); return v; }
double getd(const uint8_t* h, uint64_t off) { double v; std::memcpy(&v, h + off, 8); return v; }

uint32_t crc32_update(uint32_t crc, const uint8_t* p, size_t n) {
    static uint32_t table[256];
    static std::once_flag once;
    std::call_once(once, [] {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
            table[i] = c;
        }
    });
    crc = ~crc;
    for (size_t i = 0; i < n; ++i) crc = table[(crc ^ p[i]) & 0xFF] ^ (crc >> 8);
    return ~crc;
}

bool kraft_ok(const uint8_t* len, int nsym) {
    uint64_t sum = 0;
    int present = 0;
    for (int s = 0; s < nsym; ++s) {
        if (!len[s]) continue;
        if (len[s] > kLmax) return false;
        sum += (uint64_t)1 << (kLmax - len[s]);
        ++present;
    }
    return present > 0 && sum <= ((uint64_t)1 << kLmax);
}

uint64_t blob_bytes(uint64_t n_anchors, int R, uint64_t n_chunks, uint64_t words_bytes,
                    uint64_t n_outliers) {
    return 256 + pad8(n_anchors * 4) + pad8((uint64_t)2 * (uint64_t)R) + pad8(n_chunks * 2) +
           pad8(words_bytes) + pad8(n_outliers * 4) + pad8(n_outliers * 4);
}

}  // namespace szi

extern "C" void sz_params_default(sz_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->eb_mode = SZ_EB_REL;
    p->eb = 1e-3;
    for (int k = 0; k < 3; ++k) {
        p->interp[k] = SZ_INTERP_CUBIC_AUTO;
        p->order[k] = -1;
    }
    p->alpha = 0.0;
    p->radius = 512;
    p->huff_chunk = 1024;
}

namespace szi {

sz_status parse_blob(const uint8_t* b, uint64_t bytes, BlobInfo* out, std::string* err) {
    if (!b || !out) return bad(err, SZ_ERR_INVALID_ARG, "null argument");
    BlobInfo& o = *out;
    std::memset(&o, 0, sizeof o);
    if (bytes < 256) return bad(err, SZ_ERR_CORRUPT, "blob shorter than its header");
    if (std::memcmp(b, "SZI1", 4)) return bad(err, SZ_ERR_CORRUPT, "bad magic");
    if (crc32_update(0, b, 252) != get32(b, 252)) return bad(err, SZ_ERR_CORRUPT, "header CRC mismatch");
    if (get32(b, 4) != 1) return bad(err, SZ_ERR_UNSUPPORTED, "blob version %u", get32(b, 4));
    sz_dims& d = o.dims;
    d.ndim = get32(b, 8);
    for (int k = 0; k < 3; ++k) d.n[k] = get64(b, 16 + 8 * k);
    sz_params& p = o.params;
    sz_params_default(&p);
    p.radius = get32(b, 52);
    p.huff_chunk = get32(b, 60);
    p.eb_mode = (int32_t)get32(b, 64);
    p.eb = getd(b, 72);
    p.anchor_stride = get32(b, 12);
    for (int k = 0; k < 3 && k < (int)d.ndim; ++k) p.window[k] = get32(b, 40 + 4 * k);
    Geometry& g = o.geo;
    std::string why;
    sz_status s = check_geometry(&d, &p, g, &why);
    if (s) return bad(err, s == SZ_ERR_INVALID_ARG ? SZ_ERR_CORRUPT : s, "header: %s", why.c_str());
    if (get32(b, 56) != (uint32_t)kLmax || get32(b, 68) != (uint32_t)g.L)
        return bad(err, SZ_ERR_CORRUPT, "header: length limit or level count");
    o.n_anchors = get64(b, 192);
    o.n_chunks = get64(b, 200);
    o.n_words = get64(b, 208);
    o.n_outliers = get64(b, 216);
    if (o.n_anchors != g.nanch || o.n_chunks != g.nchunks || o.n_outliers > g.npts ||
        o.n_words > (g.npts * kLmax) / 32 + g.nchunks + 1)
        return bad(err, SZ_ERR_CORRUPT, "header: section sizes");
    const int nsym = 2 * g.R;
    const uint32_t flags = get32(b, 124);
    if ((flags & ~kFlagWordsElided) || get32(b, 248))
        return bad(err, SZ_ERR_CORRUPT, "reserved header words are not zero");
    o.elided = (flags & kFlagWordsElided) != 0;
    // an elided words section: its bitmap tells how many words follow
    o.wsec = o.n_words;
    const uint64_t nbm = (o.n_words + 31) / 32;
    if (o.elided) {
        const uint64_t at = 256 + pad8(o.n_anchors * 4) + pad8((uint64_t)nsym) + pad8(o.n_chunks * 2);
        if (at + 4 * nbm > bytes) return bad(err, SZ_ERR_CORRUPT, "blob length %llu", (unsigned long long)bytes);
        for (uint64_t j = 0; j < nbm; ++j) o.nzw += (uint64_t)__builtin_popcount(get32(b + at, 4 * j));
        o.wsec = nbm + o.nzw;
        if (o.wsec >= o.n_words) return bad(err, SZ_ERR_CORRUPT, "elided words are not shorter");
    }
    if (blob_bytes(o.n_anchors, g.R, o.n_chunks, 4 * o.wsec, o.n_outliers) != bytes)
        return bad(err, SZ_ERR_CORRUPT, "blob length %llu", (unsigned long long)bytes);
    const uint64_t secb[6] = {o.n_anchors * 4, (uint64_t)nsym, o.n_chunks * 2,
                              o.wsec * 4, o.n_outliers * 4, o.n_outliers * 4};
    uint64_t pos = 256;
    for (int k = 0; k < 6; ++k) {
        o.off[k] = pos;
        o.secb[k] = secb[k];
        if (crc32_update(0, b + pos, secb[k]) != get32(b, 224 + 4 * k))
            return bad(err, SZ_ERR_CORRUPT, "section %d CRC mismatch", k);
        for (uint64_t q = pos + secb[k]; q < pos + pad8(secb[k]); ++q)
            if (b[q]) return bad(err, SZ_ERR_CORRUPT, "section %d padding is not zero", k);
        pos += pad8(secb[k]);
    }
    const uint8_t* ws = b + o.off[3];
    if (o.elided) {
        // no bit past the words and no zero among the words kept
        if (o.n_words % 32 && (get32(ws, 4 * (nbm - 1)) >> (o.n_words % 32)))
            return bad(err, SZ_ERR_CORRUPT, "elided words: bit past the end");
        for (uint64_t j = nbm; j < o.wsec; ++j)
            if (get32(ws, 4 * j) == 0u)
                return bad(err, SZ_ERR_CORRUPT, "elided words: a zero word among the kept ones");
    } else {
        for (uint64_t j = 0; j < o.n_words; ++j) o.nzw += get32(ws, 4 * j) != 0u;
    }
    // the chunk bit counts must account for exactly the stored words, and
    // outlier indices must lie inside the field
    uint64_t words = 0;
    for (uint64_t j = 0; j < o.n_chunks; ++j) {
        uint16_t cbits;
        std::memcpy(&cbits, b + o.off[2] + 2 * j, 2);
        words += (cbits + 31u) / 32u;
    }
    if (words != o.n_words) return bad(err, SZ_ERR_CORRUPT, "chunk sizes do not match the words");
    for (uint64_t j = 0; j < o.n_outliers; ++j)
        if (get32(b + o.off[4], 4 * j) >= g.npts)
            return bad(err, SZ_ERR_CORRUPT, "outlier index outside the field");
    if (!kraft_ok(b + o.off[1], nsym))
        return bad(err, SZ_ERR_CORRUPT, "code lengths do not form a prefix code");
    o.alpha = getd(b, 80);
    o.vmin = getf(b, 88);
    o.vmax = getf(b, 92);
    o.e = getf(b, 96);
    for (int l = 0; l < 16; ++l) o.el[l] = l < g.L ? getf(b, 128 + 4 * l) : 0.0f;
    int seen = 0;
    for (int k = 0; k < 3; ++k) {
        o.spline[k] = (int32_t)get32(b, 100 + 4 * k);
        o.order[k] = (int32_t)get32(b, 112 + 4 * k);
        if (k < g.ndim) {
            if (o.spline[k] < 0 || o.spline[k] > 2 || o.order[k] < 0 || o.order[k] >= g.ndim ||
                ((seen >> o.order[k]) & 1))
                return bad(err, SZ_ERR_CORRUPT, "header: spline or order");
            seen |= 1 << o.order[k];
        }
    }
    return SZ_OK;
}

}  // namespace szi
