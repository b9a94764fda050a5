/*
 * Plain CPU rANS coder for compressed time frames -- TEST INFRASTRUCTURE ONLY.
 *
 * Section 4 of arXiv:2411.02206 puts the track-model decoding right after the
 * entropy decoding of the compressed time frame (the ANS coding of the
 * paper's introduction; its table lists "TPC Entropy Decoding" as a step of
 * its own).  The paper does not give the coded format, so this project
 * defines one, written here plainly so that the GPU decoder can be checked
 * against it:
 *
 *   - every array of a compressed frame (the 19 arrays of tmd_frame_in, in
 *     that order) is split into byte planes: plane p of an array of w-byte
 *     little-endian elements holds byte p of every element (39 planes: 15
 *     bytes per track, 10 per attached cluster, 4 per bin, 10 per unattached
 *     cluster);
 *   - each plane is coded with a static model: symbol frequencies f[0..255]
 *     summing to 2^12, stored with the plane;
 *   - the plane's symbols are cut into chunks of 64 x 512 symbols, and symbol
 *     i of a chunk belongs to interleaved stream i mod 64;
 *   - each stream is range-variant ANS (rANS, Duda's asymmetric numeral
 *     systems) with a 32-bit state kept in [2^23, 2^31) and byte-wise
 *     renormalisation: to code symbol s (start c_s, frequency f_s) the coder
 *     first emits the low byte of x while x >= 2^19 f_s, then sets
 *     x = (x / f_s) 2^12 + x mod f_s + c_s; symbols are coded last to first,
 *     and the final state is written in front of the stream's bytes, so the
 *     decoder reads forward: x = the first 4 bytes (little endian); per
 *     symbol s = the symbol whose range [c_s, c_s + f_s) holds x mod 2^12,
 *     x = f_s (x >> 12) + (x mod 2^12) - c_s, then while x < 2^23 it shifts
 *     in the next byte.
 *
 * Layout (little endian): a 64-byte header -- magic "TMDR", version 1,
 * n_tracks, n_attached, n_unattached, 0 -- then the byte offset (u64) of
 * each of the 39 planes, then the planes, each starting on an 8-byte
 * boundary: f[256] (u16), then for every chunk the byte offsets (u32, from
 * the start of the plane's data) of its 64 streams and of the end of its last
 * stream (65 words), then the data.  A plane of n symbols has ceil(n / 32768)
 * chunks; the last one holds n mod 32768 (if not 0) symbols.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define R_PROB_BITS 12
#define R_PROB (1u << R_PROB_BITS)
#define R_LOW (1u << 23)
#define R_LANES 64
#define R_PER_LANE 512
#define R_CHUNK (R_LANES * R_PER_LANE)
#define R_NARR 19
#define R_NPLANE 39
#define R_HDR 64
#define R_NBIN (36 * 152)

/* element width and count class (0: tracks, 1: attached, 2: bins, 3: unattached) of the 19 arrays */
static const int r_width[R_NARR] = {1, 1, 1, 2, 4, 2, 2, 2, 1, 1, 2, 2, 2, 2, 4, 4, 2, 2, 2};
static const int r_kind[R_NARR] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 2, 3, 3, 3, 3};

static uint64_t r_count(int a, uint32_t nT, uint32_t nA, uint32_t nU)
{
    switch (r_kind[a]) {
    case 0: return nT;
    case 1: return nA;
    case 2: return R_NBIN;
    default: return nU;
    }
}

static uint64_t r_align8(uint64_t v) { return (v + 7) & ~(uint64_t)7; }

/* Frequencies summing to 2^12 with every present symbol at least 1: each
 * symbol gets the integer part of its exact share count * 2^12 / n (at least
 * 1); the units still missing go one by one to the symbols with the largest
 * remainders, the units in excess (from symbols raised to 1) are taken one by
 * one from the symbols furthest above their share (ties: the lowest symbol). */
static void r_normalise(const uint64_t *cnt, uint64_t n, uint16_t *f)
{
    memset(f, 0, 256 * sizeof(uint16_t));
    if (n == 0) {
        f[0] = (uint16_t)R_PROB;
        return;
    }
    int64_t sum = 0;
    for (int s = 0; s < 256; s++) {
        if (!cnt[s]) continue;
        uint64_t v = cnt[s] * R_PROB / n;
        f[s] = (uint16_t)(v ? v : 1);
        sum += f[s];
    }
    while (sum != (int64_t)R_PROB) {
        /* excess of symbol s over its share, in units of 1/n: f n - count 2^12 */
        int best = -1;
        int64_t bx = 0;
        for (int s = 0; s < 256; s++) {
            if (!cnt[s]) continue;
            const int64_t ex = (int64_t)f[s] * (int64_t)n - (int64_t)(cnt[s] * R_PROB);
            if (sum < (int64_t)R_PROB) {
                if (best < 0 || ex < bx) { best = s; bx = ex; }
            } else if (f[s] > 1) {
                if (best < 0 || ex > bx) { best = s; bx = ex; }
            }
        }
        if (sum < (int64_t)R_PROB) {
            f[best]++;
            sum++;
        } else {
            f[best]--;
            sum--;
        }
    }
}

/* bytes of the coded frame at most (for the caller's buffer) */
uint64_t oracle_rans_bound(uint32_t nT, uint32_t nA, uint32_t nU)
{
    uint64_t b = R_HDR + 8 * R_NPLANE;
    for (int a = 0; a < R_NARR; a++) {
        uint64_t n = r_count(a, nT, nA, nU);
        uint64_t ch = (n + R_CHUNK - 1) / R_CHUNK;
        /* per plane: table, offsets, 4 state bytes per stream, at most 2 bytes per symbol (f >= 1: a symbol
         * costs at most 12 bits; renormalisation emits whole bytes) */
        b += (uint64_t)r_width[a] * (8 + 512 + 4 * 65 * ch + 4 * R_LANES * ch + 2 * n + 8);
    }
    return b;
}

/* Encode the 19 arrays (arr[a], r_count(a) elements of r_width[a] bytes).
 * Returns the coded size, or 0 if cap is too small. */
uint64_t oracle_rans_encode(const void *const *arr, uint32_t nT, uint32_t nA, uint32_t nU, uint8_t *dst, uint64_t cap)
{
    if (cap < oracle_rans_bound(nT, nA, nU)) return 0;
    memset(dst, 0, R_HDR + 8 * R_NPLANE);
    memcpy(dst, "TMDR", 4);
    uint32_t hdr[5] = {1u, nT, nA, nU, 0u};
    memcpy(dst + 4, hdr, sizeof(hdr));
    uint64_t pos = R_HDR + 8 * R_NPLANE;
    int plane = 0;
    /* scratch: one stream's bytes, written backwards (at most 2 bytes per symbol + 4) */
    uint8_t *tmp = (uint8_t *)malloc(2 * R_PER_LANE + 8);
    uint8_t *sym = NULL;
    for (int a = 0; a < R_NARR; a++) {
        const uint64_t n = r_count(a, nT, nA, nU);
        const int w = r_width[a];
        free(sym);
        sym = (uint8_t *)malloc(n ? n : 1);
        for (int p = 0; p < w; p++, plane++) {
            const uint8_t *src = (const uint8_t *)arr[a];
            for (uint64_t i = 0; i < n; i++) sym[i] = src[i * w + p];
            uint64_t cnt[256];
            memset(cnt, 0, sizeof(cnt));
            for (uint64_t i = 0; i < n; i++) cnt[sym[i]]++;
            uint16_t f[256];
            r_normalise(cnt, n, f);
            uint32_t c[256];
            uint32_t run = 0;
            for (int s = 0; s < 256; s++) {
                c[s] = run;
                run += f[s];
            }
            pos = r_align8(pos);
            memcpy(dst + 8 * plane + R_HDR, &pos, 8);
            memcpy(dst + pos, f, 512);
            const uint64_t nch = (n + R_CHUNK - 1) / R_CHUNK;
            uint8_t *offs = dst + pos + 512;
            uint8_t *data = offs + 4 * 65 * nch;
            uint32_t dpos = 0;
            for (uint64_t ch = 0; ch < nch; ch++) {
                const uint64_t c0 = ch * R_CHUNK;
                const uint64_t len = (n - c0) < R_CHUNK ? (n - c0) : R_CHUNK;
                for (int l = 0; l < R_LANES; l++) {
                    /* symbols c0 + l + 64 j of this chunk, coded last to first */
                    uint8_t *end = tmp + 2 * R_PER_LANE + 8, *ptr = end;
                    uint32_t x = R_LOW;
                    uint64_t k = 0;
                    while ((uint64_t)l + R_LANES * k < len) k++;
                    for (uint64_t j = k; j-- > 0;) {
                        const uint8_t s = sym[c0 + l + R_LANES * j];
                        const uint32_t x_max = ((R_LOW >> R_PROB_BITS) << 8) * f[s];
                        while (x >= x_max) {
                            *--ptr = (uint8_t)(x & 0xFF);
                            x >>= 8;
                        }
                        x = ((x / f[s]) << R_PROB_BITS) + (x % f[s]) + c[s];
                    }
                    ptr -= 4;
                    ptr[0] = (uint8_t)x;
                    ptr[1] = (uint8_t)(x >> 8);
                    ptr[2] = (uint8_t)(x >> 16);
                    ptr[3] = (uint8_t)(x >> 24);
                    memcpy(offs + 4 * (65 * ch + l), &dpos, 4);
                    memcpy(data + dpos, ptr, (size_t)(end - ptr));
                    dpos += (uint32_t)(end - ptr);
                }
                memcpy(offs + 4 * (65 * ch + 64), &dpos, 4);
            }
            pos = (uint64_t)(data - dst) + dpos;
        }
    }
    free(sym);
    free(tmp);
    return pos;
}

/* Decode a coded frame into the 19 arrays (arr[a] sized as for encoding).
 * Returns 0, or -1 if the data is not a well-formed coded frame of this
 * shape. */
int oracle_rans_decode(const uint8_t *src, uint64_t size, uint32_t nT, uint32_t nA, uint32_t nU, void *const *arr)
{
    if (size < R_HDR + 8 * R_NPLANE || memcmp(src, "TMDR", 4) != 0) return -1;
    uint32_t hdr[5];
    memcpy(hdr, src + 4, sizeof(hdr));
    if (hdr[0] != 1u || hdr[1] != nT || hdr[2] != nA || hdr[3] != nU) return -1;
    int plane = 0;
    for (int a = 0; a < R_NARR; a++) {
        const uint64_t n = r_count(a, nT, nA, nU);
        const int w = r_width[a];
        for (int p = 0; p < w; p++, plane++) {
            uint64_t pos;
            memcpy(&pos, src + R_HDR + 8 * plane, 8);
            const uint64_t nch = (n + R_CHUNK - 1) / R_CHUNK;
            if (pos > size || size - pos < 512 + 4 * 65 * nch) return -1;
            uint16_t f[256];
            memcpy(f, src + pos, 512);
            uint32_t c[256], run = 0;
            for (int s = 0; s < 256; s++) {
                c[s] = run;
                run += f[s];
            }
            if (n && run != R_PROB) return -1;
            const uint8_t *offs = src + pos + 512;
            const uint8_t *data = offs + 4 * 65 * nch;
            uint8_t *dst = (uint8_t *)arr[a];
            for (uint64_t ch = 0; ch < nch; ch++) {
                const uint64_t c0 = ch * R_CHUNK;
                const uint64_t len = (n - c0) < R_CHUNK ? (n - c0) : R_CHUNK;
                for (int l = 0; l < R_LANES; l++) {
                    uint32_t o0, o1;
                    memcpy(&o0, offs + 4 * (65 * ch + l), 4);
                    memcpy(&o1, offs + 4 * (65 * ch + l + 1), 4);
                    const uint8_t *ptr = data + o0, *end = data + o1;
                    if (o1 < o0 || o1 - o0 < 4 || (uint64_t)(end - src) > size) return -1;
                    uint32_t x = (uint32_t)ptr[0] | ((uint32_t)ptr[1] << 8) | ((uint32_t)ptr[2] << 16) |
                                 ((uint32_t)ptr[3] << 24);
                    ptr += 4;
                    for (uint64_t j = 0; (uint64_t)l + R_LANES * j < len; j++) {
                        const uint32_t slot = x & (R_PROB - 1);
                        int s = 0;
                        while (!(slot >= c[s] && slot < c[s] + f[s])) s++;
                        x = (uint32_t)f[s] * (x >> R_PROB_BITS) + slot - c[s];
                        while (x < R_LOW) {
                            if (ptr >= end) return -1;
                            x = (x << 8) | *ptr++;
                        }
                        dst[(c0 + l + R_LANES * j) * w + p] = (uint8_t)s;
                    }
                }
            }
        }
    }
    return 0;
}
