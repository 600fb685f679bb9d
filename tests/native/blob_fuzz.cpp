// The blob validation under the host sanitizers (built by
// tests/test_native_sanitizers.py): each blob named on the command line must
// parse; every truncation and every single-bit flip must be refused; header
// fields and section contents set to extreme values, with their CRCs made
// valid again, must be refused or accepted without reading outside the blob.
// Every buffer handed to the parser is a heap block of exactly the blob's
// length.  Exit status 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "blob.h"

using namespace szi;

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint64_t next() {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return rng;
}

static int parse_copy(const std::vector<uint8_t>& v, uint64_t len, BlobInfo* bi) {
    uint8_t* p = new uint8_t[len ? len : 1];
    std::memcpy(p, v.data(), len);
    std::string err;
    const int rc = parse_blob(p, len, bi, &err);
    delete[] p;
    return rc;
}

// the header CRC (and, for a section k >= 0, that section's CRC) made valid
static void fix_crcs(std::vector<uint8_t>& v, const BlobInfo& bi, int k) {
    if (k >= 0) put32(v.data(), 224 + 4 * k, crc32_update(0, v.data() + bi.off[k], bi.secb[k]));
    put32(v.data(), 252, crc32_update(0, v.data(), 252));
}

int main(int argc, char** argv) {
    int fails = 0;
    long checks = 0;
    for (int a = 1; a < argc; ++a) {
        FILE* f = std::fopen(argv[a], "rb");
        if (!f) { std::printf("cannot open %s\n", argv[a]); return 2; }
        std::vector<uint8_t> blob;
        int ch;
        while ((ch = std::fgetc(f)) != EOF) blob.push_back((uint8_t)ch);
        std::fclose(f);
        BlobInfo bi;
        if (parse_copy(blob, blob.size(), &bi) != SZ_OK) {
            std::printf("%s: the blob itself is refused\n", argv[a]);
            ++fails;
            continue;
        }
        const uint64_t n = blob.size();
        // truncations
        for (uint64_t len = 0; len < n; len += (len < 300 ? 1 : 1 + n / 97)) {
            BlobInfo t;
            ++checks;
            if (parse_copy(blob, len, &t) == SZ_OK) { std::printf("accepted %llu of %llu bytes\n",
                (unsigned long long)len, (unsigned long long)n); ++fails; }
        }
        // single-bit flips: every bit of the header, then samples of the rest
        std::vector<uint64_t> bits;
        for (uint64_t b = 0; b < 256 * 8; ++b) bits.push_back(b);
        for (int s = 0; s < 3000; ++s) bits.push_back(next() % (n * 8));
        for (uint64_t b : bits) {
            std::vector<uint8_t> v = blob;
            v[b / 8] ^= (uint8_t)(1u << (b % 8));
            BlobInfo t;
            ++checks;
            if (parse_copy(v, n, &t) == SZ_OK) { std::printf("accepted a flip of bit %llu\n",
                (unsigned long long)b); ++fails; }
        }
        // header words set to extreme values with the header CRC fixed
        const uint32_t vals32[] = {0u, 1u, 2u, 3u, 7u, 31u, 255u, 0x7FFFFFFFu, 0x80000000u, 0xFFFFFFFFu};
        for (uint64_t off = 4; off < 252; off += 4)
            for (uint32_t val : vals32) {
                std::vector<uint8_t> v = blob;
                put32(v.data(), off, val);
                fix_crcs(v, bi, -1);
                BlobInfo t;
                ++checks;
                (void)parse_copy(v, n, &t);   // refused or accepted, read inside the blob
            }
        const uint64_t vals64[] = {0ull, 1ull, 1ull << 31, 1ull << 32, 1ull << 40, ~0ull, ~0ull / 3};
        for (uint64_t off = 16; off < 40; off += 8)
            for (uint64_t val : vals64) {
                std::vector<uint8_t> v = blob;
                put64(v.data(), off, val);
                fix_crcs(v, bi, -1);
                BlobInfo t;
                ++checks;
                (void)parse_copy(v, n, &t);
            }
        for (uint64_t off = 192; off < 224; off += 8)
            for (uint64_t val : vals64) {
                std::vector<uint8_t> v = blob;
                put64(v.data(), off, val);
                fix_crcs(v, bi, -1);
                BlobInfo t;
                ++checks;
                if (parse_copy(v, n, &t) == SZ_OK && val != get64(blob.data(), off)) {
                    std::printf("accepted section count %llu at %llu\n", (unsigned long long)val,
                                (unsigned long long)off);
                    ++fails;
                }
            }
        // section contents that break the stream's rules, CRCs fixed
        for (int rep = 0; rep < 200; ++rep) {
            std::vector<uint8_t> v = blob;
            const int kind = (int)(next() % 4);
            int sec = -1;
            bool must_refuse = false;
            if (kind == 0 && bi.n_chunks) {          // a chunk's bit count changed
                sec = 2;
                const uint64_t j = next() % bi.n_chunks;
                uint16_t cb;
                std::memcpy(&cb, v.data() + bi.off[2] + 2 * j, 2);
                const uint16_t nb = (uint16_t)(cb + 32 + 32 * (next() % 100));
                std::memcpy(v.data() + bi.off[2] + 2 * j, &nb, 2);
                must_refuse = ((nb + 31u) / 32u) != ((cb + 31u) / 32u);
            } else if (kind == 1 && bi.n_outliers) {  // an outlier index outside the field
                sec = 4;
                const uint64_t j = next() % bi.n_outliers;
                put32(v.data() + bi.off[4], 4 * j, (uint32_t)(bi.geo.npts + next() % 1000));
                must_refuse = true;
            } else if (kind == 2) {                   // a code length beyond the limit
                sec = 1;
                v[bi.off[1] + next() % bi.secb[1]] = (uint8_t)(25 + next() % 200);
                must_refuse = true;
            } else if (kind == 3) {                   // random bytes anywhere in the words
                sec = 3;
                if (!bi.secb[3]) continue;
                v[bi.off[3] + next() % bi.secb[3]] ^= (uint8_t)(1 + next() % 255);
            } else {
                continue;
            }
            fix_crcs(v, bi, sec);
            BlobInfo t;
            ++checks;
            if (parse_copy(v, n, &t) == SZ_OK && must_refuse) {
                std::printf("accepted a section %d edit of kind %d\n", sec, kind);
                ++fails;
            }
        }
        std::printf("%s: %llu bytes, ok\n", argv[a], (unsigned long long)n);
    }
    std::printf("%ld checks, %d failed\n", checks, fails);
    return fails != 0;
}
