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
 *     summing to 2^12 (c_s: the sum of f below s), stored with the plane;
 *   - the plane's symbols are cut into chunks of 64 x 512; symbol i of a
 *     chunk belongs to lane i mod 64, and is the (i div 64)-th symbol, its
 *     "step", of that lane;
 *   - every lane is a range-variant ANS coder (rANS, Duda's asymmetric
 *     numeral systems) with a 32-bit state x kept in [2^16, 2^32) and
 *     renormalisation by 16-bit words; the 64 lanes of a chunk share one
 *     word stream.  Decoding a chunk: x of each lane starts at its stored
 *     final state; step by step, and within a step lane by lane in ascending
 *     order, a lane that has a symbol there takes s = the symbol whose range
 *     [c_s, c_s + f_s) holds x mod 2^12, sets x = f_s (x >> 12) +
 *     (x mod 2^12) - c_s, and if x < 2^16 then x = (x << 16) | the next word
 *     of the stream (at most one per symbol).  At the end every lane's x is
 *     back at 2^16 and every word has been read.  Coding runs the same steps
 *     in reverse (last step first, lanes in descending order, x starting at
 *     2^16): a lane about to code s first emits x mod 2^16 and shifts x right
 *     by 16 if x >= 2^20 f_s, then sets x = (x div f_s) 2^12 + x mod f_s +
 *     c_s; the emitted words, read backwards, are the stream.
 *
 * Layout (little endian): a 64-byte header -- magic "TMDR", version 2,
 * n_tracks, n_attached, n_unattached, 0 -- then the byte offset (u64) of
 * each of the 39 planes, then the planes, each on a 16-byte boundary: f[256]
 * (u16), then nch + 1 offsets (u32) of each chunk's data and of the end of
 * the last chunk, counted from the start of the plane's data, which is the
 * next 16-byte boundary; each chunk's data (on a 16-byte boundary, offsets
 * multiples of 16) is the 64 final states (u32) and the word stream (u16),
 * zero-padded to a multiple of 16 bytes.  A plane of n symbols has
 * ceil(n / 32768) chunks; the last one holds n mod 32768 (if not 0).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define R_PROB_BITS 12
#define R_PROB (1u << R_PROB_BITS)
#define R_LOW (1u << 16)
#define R_LANES 64
#define R_PER_LANE 512
#define R_CHUNK (R_LANES * R_PER_LANE)
#define R_NARR 19
#define R_NPLANE 39
#define R_HDR 64
#define R_VERSION 2u
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

static uint64_t r_align16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

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
    uint64_t b = r_align16(R_HDR + 8 * R_NPLANE);
    for (int a = 0; a < R_NARR; a++) {
        uint64_t n = r_count(a, nT, nA, nU);
        uint64_t ch = (n + R_CHUNK - 1) / R_CHUNK;
        /* per plane: alignment, model, chunk offsets, then per chunk the
         * states, at most one word per symbol, and padding */
        b += (uint64_t)r_width[a] * (16 + 512 + 4 * (ch + 1) + 16 + ch * (4 * R_LANES + 16) + 2 * n);
    }
    return b;
}

static void put32(uint8_t *d, uint32_t v)
{
    for (int q = 0; q < 4; q++) d[q] = (uint8_t)(v >> (8 * q));
}

static uint32_t get32(const uint8_t *d)
{
    return (uint32_t)d[0] | ((uint32_t)d[1] << 8) | ((uint32_t)d[2] << 16) | ((uint32_t)d[3] << 24);
}

/* Encode the 19 arrays (arr[a], r_count(a) elements of r_width[a] bytes).
 * Returns the coded size, or 0 if cap is too small. */
uint64_t oracle_rans_encode(const void *const *arr, uint32_t nT, uint32_t nA, uint32_t nU, uint8_t *dst, uint64_t cap)
{
    if (cap < oracle_rans_bound(nT, nA, nU)) return 0;
    memset(dst, 0, r_align16(R_HDR + 8 * R_NPLANE));
    memcpy(dst, "TMDR", 4);
    const uint32_t hdr[5] = {R_VERSION, nT, nA, nU, 0u};
    for (int q = 0; q < 5; q++) put32(dst + 4 + 4 * q, hdr[q]);
    uint64_t pos = r_align16(R_HDR + 8 * R_NPLANE);
    int plane = 0;
    uint16_t *words = (uint16_t *)malloc(sizeof(uint16_t) * R_CHUNK);  /* one chunk's words, in emission order */
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
            for (uint64_t q = 0; q < 8; q++) dst[R_HDR + 8 * plane + q] = (uint8_t)(pos >> (8 * q));
            for (int s = 0; s < 256; s++) {
                dst[pos + 2 * s] = (uint8_t)f[s];
                dst[pos + 2 * s + 1] = (uint8_t)(f[s] >> 8);
            }
            const uint64_t nch = (n + R_CHUNK - 1) / R_CHUNK;
            uint8_t *offs = dst + pos + 512;
            const uint64_t data0 = r_align16(pos + 512 + 4 * (nch + 1));
            memset(dst + pos + 512, 0, data0 - (pos + 512));
            uint64_t dpos = 0;  /* from data0 */
            for (uint64_t ch = 0; ch < nch; ch++) {
                const uint64_t c0 = ch * R_CHUNK;
                const uint64_t len = (n - c0) < R_CHUNK ? (n - c0) : R_CHUNK;
                const uint64_t steps = (len + R_LANES - 1) / R_LANES;
                uint32_t x[R_LANES];
                for (int l = 0; l < R_LANES; l++) x[l] = R_LOW;
                uint64_t nw = 0;
                for (uint64_t j = steps; j-- > 0;) {
                    for (int l = R_LANES - 1; l >= 0; l--) {
                        const uint64_t i = R_LANES * j + (uint64_t)l;
                        if (i >= len) continue;
                        const uint8_t s = sym[c0 + i];
                        if ((uint64_t)x[l] >= ((uint64_t)(R_LOW >> R_PROB_BITS) << 16) * f[s]) {
                            words[nw++] = (uint16_t)(x[l] & 0xFFFF);
                            x[l] >>= 16;
                        }
                        x[l] = ((x[l] / f[s]) << R_PROB_BITS) + x[l] % f[s] + c[s];
                    }
                }
                put32(offs + 4 * ch, (uint32_t)dpos);
                uint8_t *d = dst + data0 + dpos;
                for (int l = 0; l < R_LANES; l++) put32(d + 4 * l, x[l]);
                for (uint64_t k = 0; k < nw; k++) {  /* the stream is the emitted words read backwards */
                    const uint16_t v = words[nw - 1 - k];
                    d[4 * R_LANES + 2 * k] = (uint8_t)v;
                    d[4 * R_LANES + 2 * k + 1] = (uint8_t)(v >> 8);
                }
                const uint64_t used = 4 * R_LANES + 2 * nw;
                memset(d + used, 0, r_align16(used) - used);
                dpos += r_align16(used);
            }
            put32(offs + 4 * nch, (uint32_t)dpos);
            const uint64_t end = data0 + dpos;
            pos = plane + 1 < R_NPLANE ? r_align16(end) : end;
        }
    }
    free(sym);
    free(words);
    return pos;
}

/* Decode a coded frame into the 19 arrays (arr[a] sized as for encoding).
 * Returns 0, or -1 if the data is not a well-formed coded frame of this
 * shape. */
int oracle_rans_decode(const uint8_t *src, uint64_t size, uint32_t nT, uint32_t nA, uint32_t nU, void *const *arr)
{
    if (size < R_HDR + 8 * R_NPLANE || memcmp(src, "TMDR", 4) != 0) return -1;
    if (get32(src + 4) != R_VERSION || get32(src + 8) != nT || get32(src + 12) != nA || get32(src + 16) != nU)
        return -1;
    int plane = 0;
    for (int a = 0; a < R_NARR; a++) {
        const uint64_t n = r_count(a, nT, nA, nU);
        const int w = r_width[a];
        for (int p = 0; p < w; p++, plane++) {
            uint64_t pos = 0;
            for (int q = 7; q >= 0; q--) pos = (pos << 8) | src[R_HDR + 8 * plane + q];
            const uint64_t nch = (n + R_CHUNK - 1) / R_CHUNK;
            if (pos > size || size - pos < 512 + 4 * (nch + 1)) return -1;
            uint32_t f[256], c[256], run = 0;
            for (int s = 0; s < 256; s++) {
                f[s] = (uint32_t)src[pos + 2 * s] | ((uint32_t)src[pos + 2 * s + 1] << 8);
                c[s] = run;
                run += f[s];
            }
            if (n && run != R_PROB) return -1;
            const uint8_t *offs = src + pos + 512;
            const uint64_t data0 = r_align16(pos + 512 + 4 * (nch + 1));
            uint8_t *dst = (uint8_t *)arr[a];
            for (uint64_t ch = 0; ch < nch; ch++) {
                const uint64_t o0 = get32(offs + 4 * ch), o1 = get32(offs + 4 * ch + 4);
                if (o1 < o0 || o1 - o0 < 4 * R_LANES || data0 + o1 > size) return -1;
                const uint8_t *d = src + data0 + o0;
                const uint64_t nwords = (o1 - o0 - 4 * R_LANES) / 2;
                const uint64_t c0 = ch * R_CHUNK;
                const uint64_t len = (n - c0) < R_CHUNK ? (n - c0) : R_CHUNK;
                const uint64_t steps = (len + R_LANES - 1) / R_LANES;
                uint32_t x[R_LANES];
                for (int l = 0; l < R_LANES; l++) x[l] = get32(d + 4 * l);
                uint64_t k = 0;  /* words read */
                for (uint64_t j = 0; j < steps; j++) {
                    for (int l = 0; l < R_LANES; l++) {
                        const uint64_t i = R_LANES * j + (uint64_t)l;
                        if (i >= len) continue;
                        const uint32_t slot = x[l] & (R_PROB - 1);
                        int s = 0;
                        while (!(slot >= c[s] && slot < c[s] + f[s])) s++;
                        x[l] = f[s] * (x[l] >> R_PROB_BITS) + slot - c[s];
                        if (x[l] < R_LOW) {
                            if (k >= nwords) return -1;
                            const uint32_t v = (uint32_t)d[4 * R_LANES + 2 * k] | ((uint32_t)d[4 * R_LANES + 2 * k + 1] << 8);
                            k++;
                            x[l] = (x[l] << 16) | v;
                        }
                        dst[(c0 + i) * w + p] = (uint8_t)s;
                    }
                }
                /* a well-formed chunk: every state back at its start, every word read (padding < 16 bytes) */
                for (int l = 0; l < R_LANES; l++)
                    if (x[l] != R_LOW) return -1;
                if (o1 - o0 - 4 * R_LANES - 2 * k >= 16) return -1;
            }
        }
    }
    return 0;
}
