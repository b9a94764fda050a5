// libtmd: TPC track-model decoding on AMD MI355X (gfx950).
//
// What is decoded (arXiv:2411.02206, section 4): attached clusters are stored
// as residuals to their track, so each track is propagated through the pad
// rows and the residuals are added (the paper's first kernel: one GPU thread
// per track); unattached clusters are stored as differences to the previous
// cluster of their TPC region, so each region is a running sum (the paper's
// second kernel, one region per thread).  The paper precomputes on the CPU the
// indices into its structure-of-arrays input; here those indices (track start
// offsets, per-(sector,row) offsets, output slots) are computed on the GPU.
//
// The track model (the paper does not define one): state x, y, z, sin(phi)
// (s), tan(lambda) (tgl) and curvature k = q/pT * Bz * 0.00299792458 in the
// local frame of a sector.  Per cluster: optional rotation by d * 20 degrees
// into a neighbouring sector frame, exact helix step in y to the next pad row
// (dy = dx (s0 + s1) / (c0 + c1), s1 = s0 + k dx), chord step in z, rounding of
// the predicted pad and time to 1/32 units, addition of the stored integer
// residuals, and a fixed-gain update that moves the state onto the decoded
// cluster.  Every float32 operation is written out in a fixed order and the
// library is built with -ffp-contract=off and IEEE division / square root, so
// the result is bit-identical to any other implementation of the same
// equations under the same rules.
//
// Pipeline (all frames of a plan in each launch):
//   K1 k_tilesum     sum of track lengths per tile of 256 tracks
//   K2 k_count       track start offsets (scan), per-cluster (sector,row) walk,
//                    per-tile bin histogram
//   K3 k_colscan     per bin, exclusive prefix of the tile histograms
//   K4 k_offsets     per frame, bin offsets of the output and of the
//                    unattached input (flags count mismatches)
//   K5 k_unattached  per bin, running sums of the differences (one wave)
//   K6 k_rank        per tile, stable slot of every attached cluster
//   K7 k_attached    one lane per track: the float32 propagate-and-update
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "tmd.h"

#define NSEC TMD_NSEC
#define NROW TMD_NROW
#define NBIN TMD_NBIN

namespace {

constexpr int kTile = 256;  // tracks per tile: K2, K6, K7 blocks
constexpr int kWave = 64;
constexpr int kTileWaves = kTile / kWave;
constexpr uint32_t kTimeLim = 1u << 24;

// ---------------------------------------------------------------------------
// constant tables (float32, each the nearest float to a double expression)
// ---------------------------------------------------------------------------
struct Geo {
    float x[NROW], pw[NROW], inv_pw[NROW], padoff[NROW], pwq[NROW], ks[NROW], kt[NROW];
    float cosb[18], sinb[18];
    float kb, vdq, inv_vd32, snp_max;
};

void build_geo(float bz, Geo *g)
{
    // 4 pad regions: first row, radius of the region start, row pitch, pad width
    static const int rs[5] = {0, 63, 97, 127, 152};
    static const double xs[4] = {84.85, 134.0, 168.0, 204.0};
    static const double pitch[4] = {0.75, 1.00, 1.20, 1.50};
    static const double padw[4] = {0.416, 0.608, 0.608, 0.608};
    const double pi = 3.14159265358979323846;
    for (int g4 = 0; g4 < 4; g4++) {
        for (int r = rs[g4]; r < rs[g4 + 1]; r++) {
            double xd = xs[g4] + ((double)(r - rs[g4]) + 0.5) * pitch[g4];
            int npads = 2 * (int)floor(xd * tan(pi / 18.0) / padw[g4]);
            g->x[r] = (float)xd;
            g->pw[r] = (float)padw[g4];
            g->inv_pw[r] = (float)(1.0 / padw[g4]);
            g->padoff[r] = (float)(npads / 2);
            g->pwq[r] = g->pw[r] * 0.03125f;
            g->ks[r] = (float)(0.0625 / pitch[g4]);
            g->kt[r] = g->ks[r];
        }
    }
    for (int d = 0; d < 18; d++) {
        // d >= 9: half turn plus (d - 9) steps, so that d = 9 is exactly (-1, 0)
        double ang = (double)(d % 9) * pi / 9.0;
        double sg = d < 9 ? 1.0 : -1.0;
        g->cosb[d] = (float)(sg * cos(ang));
        g->sinb[d] = (float)(sg * sin(ang));
    }
    g->kb = (float)((double)bz * 0.00299792458);
    g->vdq = (float)0.516 * 0.03125f;
    g->inv_vd32 = (float)(32.0 / 0.516);
    g->snp_max = (float)0.999;
}

// ---------------------------------------------------------------------------
// per-frame descriptor (device copy in the plan)
// ---------------------------------------------------------------------------
struct FrameDesc {
    // input
    const uint8_t *ncls, *sec0, *row0;
    const uint16_t *pad0;
    const uint32_t *time0;
    const int16_t *qpt, *snp, *tgl;
    const int8_t *rdiff;
    const uint8_t *sdiff;
    const int16_t *pres, *tres;
    const uint16_t *cqtot, *cqmax;
    const uint32_t *ucount, *utdiff;
    const uint16_t *updiff, *uqtot, *uqmax;
    // output
    uint32_t *roff, *rna, *otime;
    uint16_t *opad, *oqtot, *oqmax;
    // workspace
    uint32_t *start;    // [nT + 1] first cluster of each track
    uint32_t *tilesum;  // [ntile] clusters per tile
    uint32_t *hist;     // [ntile][NBIN] per-tile bin counts, then exclusive prefixes
    uint32_t *uin;      // [NBIN] first unattached input entry of each bin
    uint32_t *ueff;     // [NBIN] unattached clusters decoded per bin
    uint32_t *dest;     // [nA] output slot of each attached cluster
    uint32_t *status;
    uint64_t cap;  // entries of the output cluster arrays; every store is checked against it
    uint32_t nT, nA, nU, ntile, tile0;
    uint32_t pad_[3];
};

// ---------------------------------------------------------------------------
// wave helpers (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t wave_incl_add(uint32_t v)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, (unsigned)d);
        if (lane >= (uint32_t)d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v |= __shfl_xor(v, d);
    return v;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// exclusive scan over a block of kTile threads; returns the block total in *tot
__device__ uint32_t block_excl_add(uint32_t v, uint32_t *tot)
{
    __shared__ uint32_t part[kTileWaves];
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_add(v);
    if (lane == kWave - 1) part[w] = inc;
    __syncthreads();
    uint32_t base = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kTileWaves; i++) {
        uint32_t p = part[i];
        if (i < (int)w) base += p;
        all += p;
    }
    __syncthreads();
    *tot = all;
    return base + inc - v;
}

// ---------------------------------------------------------------------------
// shared pieces of the track walk
// ---------------------------------------------------------------------------
struct HeaderPos {
    int sec, row;
    uint32_t flags;
};

__device__ __forceinline__ HeaderPos header_pos(uint32_t sec0, uint32_t row0)
{
    HeaderPos h;
    h.flags = 0;
    h.sec = (int)sec0;
    h.row = (int)row0;
    if (sec0 >= NSEC) { h.flags |= TMD_F_HDR; h.sec = (int)(sec0 % NSEC); }
    if (row0 >= NROW) { h.flags |= TMD_F_HDR; h.row = NROW - 1; }
    return h;
}

// clusters of a track that lie inside the declared attached stream
__device__ __forceinline__ uint32_t track_len(uint32_t start, uint32_t ncls, uint32_t nA)
{
    if (start >= nA) return 0;
    uint32_t room = nA - start;
    return ncls < room ? ncls : room;
}

__device__ __forceinline__ void step_pos(int &sec, int &row, int rd, uint32_t sd)
{
    if (sd >= 18) sd %= 18;
    if (sd) sec = (sec / 18) * 18 + (sec % 18 + (int)sd) % 18;
    row += rd;
    row = row < 0 ? 0 : (row > NROW - 1 ? NROW - 1 : row);
}

// (sector,row) key of clusters cb + lane of one track, computed by the whole
// wave; (sec, row) is the position before cluster cb and is advanced to the
// position of the last cluster of the chunk.  Lanes >= cnt return 0.
__device__ __forceinline__ uint32_t chunk_keys(const FrameDesc &F, uint32_t c0, uint32_t cb,
                                               uint32_t cnt, int &sec, int &row, bool &monotone)
{
    const uint32_t lane = lane_id();
    const uint32_t j = cb + lane;
    const bool act = lane < cnt;
    int rd = 0;
    uint32_t sd = 0;
    if (act && j > 0) {
        rd = F.rdiff[c0 + j];
        sd = F.sdiff[c0 + j];
        if (sd >= 18) sd %= 18;
    }
    // fast path: prefix sums without clamping
    int prow = row + (int)wave_incl_add((uint32_t)rd);
    uint32_t psec = (uint32_t)(sec % 18) + wave_incl_add(sd);
    bool inrange = !act || (prow >= 0 && prow < NROW);
    int side = sec / 18;
    uint32_t key;
    if (__ballot(!inrange) == 0) {
        int s = side * 18 + (int)(psec % 18);
        key = act ? (uint32_t)(s * NROW + prow) : 0u;
    } else {
        // a row leaves [0, 151] somewhere: walk the chunk in order
        int s = sec, r = row;
        key = 0;
        for (uint32_t i = 0; i < cnt; i++) {
            int rdi = __shfl(rd, (int)i);
            uint32_t sdi = (uint32_t)__shfl((int)sd, (int)i);
            if (cb + i > 0) step_pos(s, r, rdi, sdi);
            if (i == lane) key = (uint32_t)(s * NROW + r);
        }
    }
    // rows strictly monotone inside the chunk (and no clamping) => distinct keys
    uint64_t live = __ballot(act && lane > 0);
    uint64_t up = __ballot(act && lane > 0 && rd > 0);
    uint64_t dn = __ballot(act && lane > 0 && rd < 0);
    monotone = ((up == live) || (dn == live)) && __ballot(!inrange) == 0;
    uint32_t last = readlane(key, (int)(cnt - 1));
    sec = (int)(last / NROW);
    row = (int)(last % NROW);
    return key;
}

// ---------------------------------------------------------------------------
// K1: clusters per tile; also clears the frame's status word
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTile) void k_tilesum(const FrameDesc *__restrict__ fd,
                                                   const uint32_t *__restrict__ tile_frame)
{
    const uint32_t tile = blockIdx.x;
    const FrameDesc &F = fd[tile_frame[tile]];
    const uint32_t lt = tile - F.tile0;
    const uint32_t t = lt * kTile + threadIdx.x;
    uint32_t v = t < F.nT ? F.ncls[t] : 0u;
    uint32_t tot;
    block_excl_add(v, &tot);
    if (threadIdx.x == 0) {
        F.tilesum[lt] = tot;
        if (lt == 0) *F.status = 0u;
    }
}

// ---------------------------------------------------------------------------
// K2: track starts and per-tile histogram of cluster bins
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTile) void k_count(const FrameDesc *__restrict__ fd,
                                                 const uint32_t *__restrict__ tile_frame)
{
    __shared__ uint32_t hist[NBIN];
    const uint32_t tile = blockIdx.x;
    const FrameDesc &F = fd[tile_frame[tile]];
    const uint32_t lt = tile - F.tile0;
    const uint32_t t = lt * kTile + threadIdx.x;

    // clusters of all earlier tiles of the frame
    uint32_t pre = 0;
    for (uint32_t i = threadIdx.x; i < lt; i += kTile) pre += F.tilesum[i];
    uint32_t dummy;
    uint32_t pre_excl = block_excl_add(pre, &dummy);
    (void)pre_excl;
    const uint32_t before = dummy;

    for (uint32_t i = threadIdx.x; i < NBIN; i += kTile) hist[i] = 0;
    const uint32_t nc = t < F.nT ? F.ncls[t] : 0u;
    uint32_t tot;
    const uint32_t start = before + block_excl_add(nc, &tot);  // also syncs
    if (t < F.nT) {
        F.start[t] = start;
        if (t == F.nT - 1) {
            F.start[F.nT] = start + nc;
            if (start + nc != F.nA) atomicOr(F.status, TMD_F_COUNT);
        }
        const uint32_t n = track_len(start, nc, F.nA);
        if (n > 0) {
            HeaderPos h = header_pos(F.sec0[t], F.row0[t]);
            int sec = h.sec, row = h.row;
            atomicAdd(&hist[sec * NROW + row], 1u);
            for (uint32_t j = 1; j < n; j++) {
                step_pos(sec, row, F.rdiff[start + j], F.sdiff[start + j]);
                atomicAdd(&hist[sec * NROW + row], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t *dst = F.hist + (size_t)lt * NBIN;
    for (uint32_t i = threadIdx.x; i < NBIN; i += kTile) dst[i] = hist[i];
}

// ---------------------------------------------------------------------------
// K3: per bin, exclusive prefix over the frame's tiles; totals -> row_nattached
// grid (ceil(NBIN/64), n_frames), block 1024 = 16 waves; lane = bin
// ---------------------------------------------------------------------------
constexpr int kScanWaves = 16;

__global__ __launch_bounds__(kWave * kScanWaves) void k_colscan(const FrameDesc *__restrict__ fd)
{
    __shared__ uint32_t part[kScanWaves][kWave];
    const FrameDesc &F = fd[blockIdx.y];
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    const uint32_t k = blockIdx.x * kWave + lane;
    const uint32_t per = (F.ntile + kScanWaves - 1) / kScanWaves;
    const uint32_t a = w * per;
    const uint32_t b = min(a + per, F.ntile);
    uint32_t sum = 0;
    if (k < NBIN)
        for (uint32_t i = a; i < b; i++) sum += F.hist[(size_t)i * NBIN + k];
    part[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, total = 0;
    for (uint32_t i = 0; i < kScanWaves; i++) {
        uint32_t p = part[i][lane];
        if (i < w) run += p;
        total += p;
    }
    if (k < NBIN) {
        for (uint32_t i = a; i < b; i++) {
            uint32_t *h = F.hist + (size_t)i * NBIN + k;
            uint32_t v = *h;
            *h = run;
            run += v;
        }
        if (w == 0) F.rna[k] = total;
    }
}

// ---------------------------------------------------------------------------
// K4: per frame, output offsets and unattached input offsets
// grid n_frames, block 1024; thread i owns bins [6i, 6i + 6)
// ---------------------------------------------------------------------------
constexpr int kOffThreads = 1024;
constexpr int kOffPer = (NBIN + kOffThreads - 1) / kOffThreads;  // 6

__global__ __launch_bounds__(kOffThreads) void k_offsets(const FrameDesc *__restrict__ fd)
{
    __shared__ unsigned long long part64[kOffThreads / kWave];
    __shared__ uint32_t part32[kOffThreads / kWave];
    const FrameDesc &F = fd[blockIdx.x];
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    const uint32_t b0 = threadIdx.x * kOffPer;

    // unattached input: exclusive prefix of un_count in 64 bits, cut at nU
    unsigned long long cnt[kOffPer];
    unsigned long long own = 0;
    for (int i = 0; i < kOffPer; i++) {
        uint32_t b = b0 + i;
        cnt[i] = b < NBIN ? F.ucount[b] : 0u;
        own += cnt[i];
    }
    // 64-bit wave scan as two 32-bit halves with carry
    unsigned long long inc = own;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        unsigned long long t = __shfl_up(inc, (unsigned)d);
        if (lane >= (uint32_t)d) inc += t;
    }
    if (lane == kWave - 1) part64[w] = inc;
    __syncthreads();
    unsigned long long base = 0, all = 0;
    for (uint32_t i = 0; i < kOffThreads / kWave; i++) {
        if (i < w) base += part64[i];
        all += part64[i];
    }
    unsigned long long us = base + inc - own;
    uint32_t eff[kOffPer];
    uint32_t ownout = 0;
    for (int i = 0; i < kOffPer; i++) {
        uint32_t b = b0 + i;
        uint32_t e = 0;
        if (us < F.nU) {
            unsigned long long room = (unsigned long long)F.nU - us;
            e = cnt[i] < room ? (uint32_t)cnt[i] : (uint32_t)room;
        }
        if (b < NBIN) {
            F.uin[b] = (uint32_t)(us < F.nU ? us : F.nU);
            F.ueff[b] = e;
            eff[i] = e + F.rna[b];
        } else {
            eff[i] = 0;
        }
        ownout += eff[i];
        us += cnt[i];
    }
    if (threadIdx.x == 0 && (all != F.nU || (F.nT == 0 && F.nA != 0))) atomicOr(F.status, TMD_F_COUNT);

    uint32_t inc32 = wave_incl_add(ownout);
    if (lane == kWave - 1) part32[w] = inc32;
    __syncthreads();
    uint32_t base32 = 0;
    for (uint32_t i = 0; i < w; i++) base32 += part32[i];
    uint32_t o = base32 + inc32 - ownout;
    for (int i = 0; i < kOffPer; i++) {
        uint32_t b = b0 + i;
        if (b < NBIN) F.roff[b] = o;
        o += eff[i];
    }
    if (threadIdx.x == kOffThreads - 1) F.roff[NBIN] = o;
}

// ---------------------------------------------------------------------------
// K5: unattached clusters; one wave per (bin, frame)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void k_unattached(const FrameDesc *__restrict__ fd)
{
    const FrameDesc &F = fd[blockIdx.y];
    const uint32_t k = blockIdx.x;
    const uint32_t cnt = F.ueff[k];
    if (cnt == 0) return;
    const uint32_t src = F.uin[k];
    const uint32_t dst = F.roff[k] + F.rna[k];
    const uint32_t lane = lane_id();
    uint32_t ct = 0, cp = 0;
    for (uint32_t i = 0; i < cnt; i += kWave) {
        const uint32_t idx = i + lane;
        const bool act = idx < cnt;
        uint32_t td = act ? F.utdiff[src + idx] : 0u;
        uint32_t pd = act ? (uint32_t)F.updiff[src + idx] : 0u;
        uint32_t st = ct + wave_incl_add(td);
        uint32_t sp = cp + wave_incl_add(pd);
        if (act && dst + idx < F.cap) {
            F.otime[dst + idx] = st;
            F.opad[dst + idx] = (uint16_t)sp;
            F.oqtot[dst + idx] = F.uqtot[src + idx];
            F.oqmax[dst + idx] = F.uqmax[src + idx];
        }
        ct = readlane(st, kWave - 1);
        cp = readlane(sp, kWave - 1);
    }
}

// ---------------------------------------------------------------------------
// K6: stable output slot of every attached cluster.  Within a bin the order is
// the stream order (track, then cluster).  Block = one tile of 256 tracks;
// each wave takes 64 consecutive tracks one at a time, 64 clusters per step.
// LDS: per-wave counters (16 bit: a wave's 64 tracks put at most 64*255
// clusters in one bin, and three waves' prefix stays below 2^16) and the bin
// bases of the tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTile) void k_rank(const FrameDesc *__restrict__ fd,
                                                const uint32_t *__restrict__ tile_frame)
{
    __shared__ uint32_t wcnt32[kTileWaves * NBIN / 2];  // 16-bit counters, packed
    __shared__ uint32_t base[NBIN];
    uint16_t *wcnt = reinterpret_cast<uint16_t *>(wcnt32);
    const uint32_t tile = blockIdx.x;
    const FrameDesc &F = fd[tile_frame[tile]];
    const uint32_t lt = tile - F.tile0;
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;

    for (uint32_t i = threadIdx.x; i < kTileWaves * NBIN / 2; i += kTile) wcnt32[i] = 0;
    __syncthreads();

    const uint32_t t_first = lt * kTile + w * kWave;
    // pass 1: per-wave bin counts
    for (uint32_t tt = 0; tt < kWave; tt++) {
        const uint32_t t = t_first + tt;
        if (t >= F.nT) break;
        const uint32_t c0 = F.start[t];
        const uint32_t n = track_len(c0, F.ncls[t], F.nA);
        if (n == 0) continue;
        HeaderPos h = header_pos(F.sec0[t], F.row0[t]);
        int sec = h.sec, row = h.row;
        for (uint32_t cb = 0; cb < n; cb += kWave) {
            const uint32_t cnt = min(n - cb, (uint32_t)kWave);
            bool mono;
            uint32_t key = chunk_keys(F, c0, cb, cnt, sec, row, mono);
            if (lane < cnt) {
                uint32_t idx = w * NBIN + key;
                atomicAdd(&wcnt32[idx >> 1], 1u << (16 * (idx & 1)));
            }
        }
    }
    __syncthreads();
    // exclusive prefix over the waves; bin base of this tile
    const uint32_t *G = F.hist + (size_t)lt * NBIN;
    for (uint32_t k = threadIdx.x; k < NBIN; k += kTile) {
        uint32_t run = 0;
        for (uint32_t i = 0; i < kTileWaves; i++) {
            uint32_t v = wcnt[i * NBIN + k];
            wcnt[i * NBIN + k] = (uint16_t)run;
            run += v;
        }
        base[k] = F.roff[k] + G[k];
    }
    __syncthreads();
    // pass 2: slots
    for (uint32_t tt = 0; tt < kWave; tt++) {
        const uint32_t t = t_first + tt;
        if (t >= F.nT) break;
        const uint32_t c0 = F.start[t];
        const uint32_t n = track_len(c0, F.ncls[t], F.nA);
        if (n == 0) continue;
        HeaderPos h = header_pos(F.sec0[t], F.row0[t]);
        int sec = h.sec, row = h.row;
        for (uint32_t cb = 0; cb < n; cb += kWave) {
            const uint32_t cnt = min(n - cb, (uint32_t)kWave);
            bool mono;
            uint32_t key = chunk_keys(F, c0, cb, cnt, sec, row, mono);
            const bool act = lane < cnt;
            const uint64_t lt_mask = (1ull << lane) - 1ull;
            uint64_t same;
            if (mono) {
                same = 1ull << lane;
            } else {
                // lanes holding the same key: intersect per-bit ballots
                same = __ballot(act);
#pragma unroll
                for (int bit = 0; bit < 13; bit++) {
                    uint64_t m = __ballot(act && ((key >> bit) & 1u));
                    same &= ((key >> bit) & 1u) ? m : ~m;
                }
            }
            const uint32_t below = (uint32_t)__popcll(same & lt_mask);
            const uint32_t slot_idx = w * NBIN + key;
            uint32_t r = 0;
            if (act) r = wcnt[slot_idx];
            // every lane reads before any lane writes
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0);
            if (act) {
                F.dest[c0 + cb + lane] = base[key] + r + below;
                const bool leader = (same >> lane) == 1ull;  // highest lane of its group
                if (leader) wcnt[slot_idx] = (uint16_t)(r + below + 1);
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// ---------------------------------------------------------------------------
// K7: attached decode, one lane per track
// ---------------------------------------------------------------------------
__device__ __forceinline__ float clamp_snp(float v, float smax, uint32_t &fl)
{
    if (v != v) { fl |= TMD_F_SNP; return 0.0f; }
    if (v > smax) { fl |= TMD_F_SNP; return smax; }
    if (v < -smax) { fl |= TMD_F_SNP; return -smax; }
    return v;
}

__device__ __forceinline__ int32_t sat_i32(float v)
{
    if (v != v) return 0;
    if (v > 1073741824.0f) return 1073741824;
    if (v < -1073741824.0f) return -1073741824;
    return (int32_t)v;
}

__global__ __launch_bounds__(kTile) void k_attached(const FrameDesc *__restrict__ fd,
                                                    const uint32_t *__restrict__ tile_frame,
                                                    const Geo *__restrict__ geo_g)
{
    __shared__ Geo geo;
    {
        const uint32_t *s = reinterpret_cast<const uint32_t *>(geo_g);
        uint32_t *d = reinterpret_cast<uint32_t *>(&geo);
        for (uint32_t i = threadIdx.x; i < sizeof(Geo) / 4; i += kTile) d[i] = s[i];
    }
    __syncthreads();
    const uint32_t tile = blockIdx.x;
    const FrameDesc &F = fd[tile_frame[tile]];
    const uint32_t t = (tile - F.tile0) * kTile + threadIdx.x;
    uint32_t fl = 0;
    if (t < F.nT) {
        const uint32_t ncls = F.ncls[t];
        const uint32_t c0 = F.start[t];
        const uint32_t n = track_len(c0, ncls, F.nA);
        if (ncls == 0) fl |= TMD_F_HDR;
        HeaderPos h = header_pos(F.sec0[t], F.row0[t]);
        fl |= h.flags;
        int sec = h.sec, row = h.row;
        uint32_t t0u = F.time0[t];
        if (t0u >= kTimeLim) { fl |= TMD_F_TIME; t0u = kTimeLim - 1; }
        const int32_t t0 = (int32_t)t0u;
        const uint16_t pad0 = F.pad0[t];
        const float smax = geo.snp_max;
        float x = geo.x[row];
        float y = ((float)pad0 * 0x1p-5f - geo.padoff[row]) * geo.pw[row];
        float z = 0.0f;
        float s = clamp_snp((float)F.snp[t] * 0x1p-15f, smax, fl);
        float tgl = (float)F.tgl[t] * 0x1p-12f;
        const float k = ((float)F.qpt[t] * 0x1p-10f) * geo.kb;
        if (n > 0 && F.dest[c0] < F.cap) {
            uint32_t o = F.dest[c0];
            F.otime[o] = (uint32_t)t0;
            F.opad[o] = pad0;
            F.oqtot[o] = F.cqtot[c0];
            F.oqmax[o] = F.cqmax[c0];
        }
        for (uint32_t j = 1; j < n; j++) {
            const uint32_t c = c0 + j;
            uint32_t d = F.sdiff[c];
            if (d >= 18) { fl |= TMD_F_SEC; d %= 18; }
            if (d != 0) {
                const float ca = geo.cosb[d], sa = geo.sinb[d];
                const float cs = sqrtf((1.0f - s) * (1.0f + s));
                const float xn = (x * ca) + (y * sa);
                const float yn = (y * ca) - (x * sa);
                const float sn = (s * ca) - (cs * sa);
                const float cn = (cs * ca) + (s * sa);
                if (!(cn > 0.0f)) fl |= TMD_F_ROT;
                x = xn;
                y = yn;
                s = clamp_snp(sn, smax, fl);
                sec = (sec / 18) * 18 + (sec % 18 + (int)d) % 18;
            }
            row += F.rdiff[c];
            if (row < 0) { fl |= TMD_F_ROW; row = 0; }
            if (row > NROW - 1) { fl |= TMD_F_ROW; row = NROW - 1; }
            const float xr = geo.x[row];
            const float dx = xr - x;
            const float s1 = clamp_snp(s + (k * dx), smax, fl);
            const float a0 = sqrtf((1.0f - s) * (1.0f + s));
            const float a1 = sqrtf((1.0f - s1) * (1.0f + s1));
            const float dydx = (s + s1) / (a0 + a1);
            y = y + (dx * dydx);
            z = z + (tgl * (dx * sqrtf(1.0f + (dydx * dydx))));
            s = s1;
            x = xr;
            const int32_t P = sat_i32(rintf(((y * geo.inv_pw[row]) + geo.padoff[row]) * 32.0f));
            const int32_t T = sat_i32(rintf(z * geo.inv_vd32));
            const int32_t pres = F.pres[c];
            const int32_t tres = F.tres[c];
            int32_t padq = P + pres;
            if (padq < 0) { fl |= TMD_F_PAD; padq = 0; }
            if (padq > 65535) { fl |= TMD_F_PAD; padq = 65535; }
            int32_t timeq = t0 + T + tres;
            if (timeq < 0) { fl |= TMD_F_TIME; timeq = 0; }
            if (timeq > (int32_t)kTimeLim - 1) { fl |= TMD_F_TIME; timeq = (int32_t)kTimeLim - 1; }
            const uint32_t o = F.dest[c];
            if (o < F.cap) {
                F.otime[o] = (uint32_t)timeq;
                F.opad[o] = (uint16_t)padq;
                F.oqtot[o] = F.cqtot[c];
                F.oqmax[o] = F.cqmax[c];
            }
            const float nuy = (float)pres * geo.pwq[row];
            const float nuz = (float)tres * geo.vdq;
            y = y + nuy;
            z = z + nuz;
            s = clamp_snp(s + (nuy * geo.ks[row]), smax, fl);
            tgl = tgl + (nuz * geo.kt[row]);
        }
    }
    fl = wave_or(fl);
    if (lane_id() == 0 && fl) atomicOr(F.status, fl);
}

// ---------------------------------------------------------------------------
// arithmetic self-test
// ---------------------------------------------------------------------------
__global__ void k_selftest_fp(const float *a, const float *b, float *out, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = a[i], y = b[i];
    out[4 * i + 0] = sqrtf(x);
    out[4 * i + 1] = x / y;
    out[4 * i + 2] = rintf(x);
    out[4 * i + 3] = x * y + x;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
constexpr int kStages = 7;
const char *kStageNames[kStages] = {"tilesum", "count", "colscan", "offsets",
                                    "unattached", "rank", "attached"};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct FrameLayout {
    size_t start, tilesum, hist, uin, ueff, dest;
    uint32_t ntile, tile0;
};

}  // namespace

struct tmd_plan {
    int device = 0;
    uint32_t n_frames = 0;
    uint32_t total_tiles = 0;
    tmd_params params{};
    std::vector<tmd_frame_shape> shapes;
    std::vector<FrameLayout> layout;
    size_t ws_bytes = 0;
    Geo *d_geo = nullptr;
    uint32_t *d_tile_frame = nullptr;
    FrameDesc *d_desc = nullptr;
    uint32_t *d_status = nullptr;
    uint32_t *h_status = nullptr;  // pinned
    FrameDesc *h_desc = nullptr;   // pinned staging
    std::vector<FrameDesc> last_desc;
    bool desc_valid = false;
    hipEvent_t desc_done = nullptr;
    hipEvent_t done = nullptr;
    bool profiling = false;
    std::vector<std::vector<hipEvent_t>> prof_events;
    hipGraphExec_t graph = nullptr;
    hipStream_t graph_stream = nullptr;
    void *graph_ws = nullptr;
};

namespace {

int hip_fail(hipError_t e)
{
    (void)e;
    return TMD_E_HIP;
}

#define HIP_TRY(x)                                 \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return hip_fail(e_); \
    } while (0)

template <class T>
bool aligned(const T *p)
{
    return ((uintptr_t)p % alignof(T)) == 0;
}

int launch_all(tmd_plan_t *P, hipStream_t s, bool record)
{
    std::vector<hipEvent_t> ev;
    if (record) {
        ev.resize(kStages + 1);
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        HIP_TRY(hipEventRecord(ev[0], s));
    }
    int st = 0;
    auto mark = [&]() -> int {
        if (record) {
            if (hipEventRecord(ev[++st], s) != hipSuccess) return TMD_E_HIP;
        }
        return TMD_OK;
    };
    const uint32_t T = P->total_tiles;
    if (T) hipLaunchKernelGGL(k_tilesum, dim3(T), dim3(kTile), 0, s, P->d_desc, P->d_tile_frame);
    if (mark()) return TMD_E_HIP;
    if (T) hipLaunchKernelGGL(k_count, dim3(T), dim3(kTile), 0, s, P->d_desc, P->d_tile_frame);
    if (mark()) return TMD_E_HIP;
    hipLaunchKernelGGL(k_colscan, dim3((NBIN + kWave - 1) / kWave, P->n_frames), dim3(kWave * kScanWaves), 0,
                       s, P->d_desc);
    if (mark()) return TMD_E_HIP;
    hipLaunchKernelGGL(k_offsets, dim3(P->n_frames), dim3(kOffThreads), 0, s, P->d_desc);
    if (mark()) return TMD_E_HIP;
    hipLaunchKernelGGL(k_unattached, dim3(NBIN, P->n_frames), dim3(kWave), 0, s, P->d_desc);
    if (mark()) return TMD_E_HIP;
    if (T) hipLaunchKernelGGL(k_rank, dim3(T), dim3(kTile), 0, s, P->d_desc, P->d_tile_frame);
    if (mark()) return TMD_E_HIP;
    if (T) hipLaunchKernelGGL(k_attached, dim3(T), dim3(kTile), 0, s, P->d_desc, P->d_tile_frame, P->d_geo);
    if (mark()) return TMD_E_HIP;
    HIP_TRY(hipGetLastError());
    if (record) P->prof_events.push_back(ev);
    return TMD_OK;
}

}  // namespace

extern "C" {

const char *tmd_strerror(int code)
{
    switch (code) {
    case TMD_OK: return "ok";
    case TMD_E_ARG: return "invalid argument (null or misaligned pointer, bad size or shape)";
    case TMD_E_CAPACITY: return "output capacity smaller than n_attached + n_unattached";
    case TMD_E_INPUT: return "stream counts disagree with the frame shape (streams were cut)";
    case TMD_E_STREAM: return "the track model clamped values of the stream";
    case TMD_E_HIP: return "HIP runtime error";
    default: return "unknown error";
    }
}

const char *tmd_version(void) { return "tmd 1.0 gfx950"; }

int tmd_tables(float bz, float *dst, int cap)
{
    const int n = 7 * NROW + 2 * 18 + 4;
    if (!dst || cap < n) return -n;
    Geo g;
    build_geo(bz, &g);
    const float *rows[7] = {g.x, g.pw, g.inv_pw, g.padoff, g.pwq, g.ks, g.kt};
    int o = 0;
    for (int a = 0; a < 7; a++)
        for (int r = 0; r < NROW; r++) dst[o++] = rows[a][r];
    for (int d = 0; d < 18; d++) dst[o++] = g.cosb[d];
    for (int d = 0; d < 18; d++) dst[o++] = g.sinb[d];
    dst[o++] = g.kb;
    dst[o++] = g.vdq;
    dst[o++] = g.inv_vd32;
    dst[o++] = g.snp_max;
    return o;
}

void tmd_free(tmd_plan_t *P)
{
    if (!P) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != P->device) (void)hipSetDevice(P->device);
    if (P->done) (void)hipEventSynchronize(P->done);
    for (auto &v : P->prof_events)
        for (auto e : v) (void)hipEventDestroy(e);
    if (P->graph) (void)hipGraphExecDestroy(P->graph);
    if (P->desc_done) (void)hipEventDestroy(P->desc_done);
    if (P->done) (void)hipEventDestroy(P->done);
    if (P->d_geo) (void)hipFree(P->d_geo);
    if (P->d_tile_frame) (void)hipFree(P->d_tile_frame);
    if (P->d_desc) (void)hipFree(P->d_desc);
    if (P->d_status) (void)hipFree(P->d_status);
    if (P->h_status) (void)hipHostFree(P->h_status);
    if (P->h_desc) (void)hipHostFree(P->h_desc);
    if (cur != P->device) (void)hipSetDevice(cur);
    delete P;
}

int tmd_plan(const tmd_frame_shape *shapes, uint32_t n_frames, const tmd_params *p, tmd_plan_t **plan,
             size_t *workspace_bytes)
{
    if (!shapes || !p || !plan || !workspace_bytes || n_frames == 0) return TMD_E_ARG;
    *plan = nullptr;
    for (uint32_t f = 0; f < n_frames; f++)
        if (shapes[f].n_tracks > TMD_MAX_TRACKS) return TMD_E_ARG;
    tmd_plan_t *P = new (std::nothrow) tmd_plan_t();
    if (!P) return TMD_E_HIP;
    P->n_frames = n_frames;
    P->params = *p;
    P->shapes.assign(shapes, shapes + n_frames);
    size_t off = 0;
    uint32_t tiles = 0;
    std::vector<uint32_t> tile_frame;
    for (uint32_t f = 0; f < n_frames; f++) {
        const tmd_frame_shape &S = shapes[f];
        FrameLayout L;
        L.ntile = (S.n_tracks + kTile - 1) / kTile;
        L.tile0 = tiles;
        tiles += L.ntile;
        tile_frame.insert(tile_frame.end(), L.ntile, f);
        L.start = off;   off += align256(4 * ((size_t)S.n_tracks + 1));
        L.tilesum = off; off += align256(4 * (size_t)(L.ntile ? L.ntile : 1));
        L.hist = off;    off += align256(4 * (size_t)L.ntile * NBIN);
        L.uin = off;     off += align256(4 * (size_t)NBIN);
        L.ueff = off;    off += align256(4 * (size_t)NBIN);
        L.dest = off;    off += align256(4 * (size_t)(S.n_attached ? S.n_attached : 1));
        P->layout.push_back(L);
    }
    P->total_tiles = tiles;
    P->ws_bytes = off;
    int rc = TMD_OK;
    do {
        if (hipGetDevice(&P->device) != hipSuccess) { rc = TMD_E_HIP; break; }
        Geo g;
        build_geo(p->bz_tesla, &g);
        if (hipMalloc(&P->d_geo, sizeof(Geo)) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipMemcpy(P->d_geo, &g, sizeof(Geo), hipMemcpyHostToDevice) != hipSuccess) { rc = TMD_E_HIP; break; }
        size_t tf = sizeof(uint32_t) * (tile_frame.empty() ? 1 : tile_frame.size());
        if (hipMalloc(&P->d_tile_frame, tf) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (!tile_frame.empty() &&
            hipMemcpy(P->d_tile_frame, tile_frame.data(), tf, hipMemcpyHostToDevice) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        if (hipMalloc(&P->d_desc, sizeof(FrameDesc) * n_frames) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipMalloc(&P->d_status, sizeof(uint32_t) * n_frames) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipMemset(P->d_status, 0, sizeof(uint32_t) * n_frames) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipHostMalloc((void **)&P->h_status, sizeof(uint32_t) * n_frames, 0) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        memset(P->h_status, 0, sizeof(uint32_t) * n_frames);
        if (hipHostMalloc((void **)&P->h_desc, sizeof(FrameDesc) * n_frames, 0) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        if (hipEventCreateWithFlags(&P->desc_done, hipEventDisableTiming) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipEventCreateWithFlags(&P->done, hipEventDisableTiming) != hipSuccess) { rc = TMD_E_HIP; break; }
    } while (0);
    if (rc != TMD_OK) {
        tmd_free(P);
        return rc;
    }
    *plan = P;
    *workspace_bytes = P->ws_bytes;
    return TMD_OK;
}

int tmd_decode(tmd_plan_t *P, const tmd_frame_in *in, tmd_frame_out *out, void *workspace, void *stream)
{
    if (!P || !in || !out || !workspace) return TMD_E_ARG;
    if ((uintptr_t)workspace % 256) return TMD_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    std::vector<FrameDesc> desc(P->n_frames);
    for (uint32_t f = 0; f < P->n_frames; f++) {
        const tmd_frame_shape &S = P->shapes[f];
        const tmd_frame_in &I = in[f];
        const tmd_frame_out &O = out[f];
        const FrameLayout &L = P->layout[f];
        if (O.capacity < (uint64_t)S.n_attached + S.n_unattached) return TMD_E_CAPACITY;
        // every array that the kernels touch must be present and aligned
        if (S.n_tracks && (!I.trk_ncls || !I.trk_sec0 || !I.trk_row0 || !I.trk_pad0 || !I.trk_time0 ||
                           !I.trk_qpt || !I.trk_snp || !I.trk_tgl))
            return TMD_E_ARG;
        if (S.n_attached && (!I.cls_row_diff || !I.cls_sec_diff || !I.cls_pad_res || !I.cls_time_res ||
                             !I.cls_qtot || !I.cls_qmax))
            return TMD_E_ARG;
        if (!I.un_count) return TMD_E_ARG;
        if (S.n_unattached && (!I.un_time_diff || !I.un_pad_diff || !I.un_qtot || !I.un_qmax))
            return TMD_E_ARG;
        if (!O.row_offset || !O.row_nattached) return TMD_E_ARG;
        if ((S.n_attached || S.n_unattached) && (!O.time || !O.pad || !O.qtot || !O.qmax)) return TMD_E_ARG;
        if (!aligned(I.trk_pad0) || !aligned(I.trk_time0) || !aligned(I.trk_qpt) || !aligned(I.trk_snp) ||
            !aligned(I.trk_tgl) || !aligned(I.cls_pad_res) || !aligned(I.cls_time_res) ||
            !aligned(I.cls_qtot) || !aligned(I.cls_qmax) || !aligned(I.un_count) ||
            !aligned(I.un_time_diff) || !aligned(I.un_pad_diff) || !aligned(I.un_qtot) ||
            !aligned(I.un_qmax) || !aligned(O.row_offset) || !aligned(O.row_nattached) ||
            !aligned(O.time) || !aligned(O.pad) || !aligned(O.qtot) || !aligned(O.qmax))
            return TMD_E_ARG;
        FrameDesc &D = desc[f];
        memset(&D, 0, sizeof(D));
        D.ncls = I.trk_ncls; D.sec0 = I.trk_sec0; D.row0 = I.trk_row0; D.pad0 = I.trk_pad0;
        D.time0 = I.trk_time0; D.qpt = I.trk_qpt; D.snp = I.trk_snp; D.tgl = I.trk_tgl;
        D.rdiff = I.cls_row_diff; D.sdiff = I.cls_sec_diff; D.pres = I.cls_pad_res; D.tres = I.cls_time_res;
        D.cqtot = I.cls_qtot; D.cqmax = I.cls_qmax;
        D.ucount = I.un_count; D.utdiff = I.un_time_diff; D.updiff = I.un_pad_diff;
        D.uqtot = I.un_qtot; D.uqmax = I.un_qmax;
        D.roff = O.row_offset; D.rna = O.row_nattached; D.otime = O.time; D.opad = O.pad;
        D.oqtot = O.qtot; D.oqmax = O.qmax;
        char *ws = (char *)workspace;
        D.start = (uint32_t *)(ws + L.start);
        D.tilesum = (uint32_t *)(ws + L.tilesum);
        D.hist = (uint32_t *)(ws + L.hist);
        D.uin = (uint32_t *)(ws + L.uin);
        D.ueff = (uint32_t *)(ws + L.ueff);
        D.dest = (uint32_t *)(ws + L.dest);
        D.status = P->d_status + f;
        D.cap = O.capacity;
        D.nT = S.n_tracks; D.nA = S.n_attached; D.nU = S.n_unattached;
        D.ntile = L.ntile; D.tile0 = L.tile0;
    }
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != P->device) HIP_TRY(hipSetDevice(P->device));
    int rc = TMD_OK;
    do {
        const size_t dbytes = sizeof(FrameDesc) * P->n_frames;
        if (!P->desc_valid || memcmp(desc.data(), P->last_desc.data(), dbytes) != 0) {
            // the staging buffer may still feed the previous upload
            if (P->desc_valid && hipEventSynchronize(P->desc_done) != hipSuccess) { rc = TMD_E_HIP; break; }
            memcpy(P->h_desc, desc.data(), dbytes);
            if (hipMemcpyAsync(P->d_desc, P->h_desc, dbytes, hipMemcpyHostToDevice, s) != hipSuccess) {
                rc = TMD_E_HIP;
                break;
            }
            if (hipEventRecord(P->desc_done, s) != hipSuccess) { rc = TMD_E_HIP; break; }
            P->last_desc = desc;
            P->desc_valid = true;
        }
        rc = launch_all(P, s, P->profiling);
        if (rc != TMD_OK) break;
        if (hipMemcpyAsync(P->h_status, P->d_status, sizeof(uint32_t) * P->n_frames, hipMemcpyDeviceToHost,
                           s) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        if (hipEventRecord(P->done, s) != hipSuccess) { rc = TMD_E_HIP; break; }
    } while (0);
    if (cur != P->device) (void)hipSetDevice(cur);
    return rc;
}

int tmd_status(tmd_plan_t *P, uint32_t frame, uint32_t *flags)
{
    if (!P || !flags || frame >= P->n_frames) return TMD_E_ARG;
    HIP_TRY(hipEventSynchronize(P->done));
    uint32_t f = P->h_status[frame];
    *flags = f;
    if (f & TMD_F_COUNT) return TMD_E_INPUT;
    if (f) return TMD_E_STREAM;
    return TMD_OK;
}

int tmd_set_profiling(tmd_plan_t *P, int enable)
{
    if (!P) return TMD_E_ARG;
    P->profiling = enable != 0;
    return TMD_OK;
}

int tmd_stage_times(tmd_plan_t *P, double *ms, uint32_t n, uint32_t *calls)
{
    if (!P || (!ms && n)) return TMD_E_ARG;
    std::vector<double> acc(kStages, 0.0);
    for (auto &ev : P->prof_events) {
        HIP_TRY(hipEventSynchronize(ev[kStages]));
        for (int i = 0; i < kStages; i++) {
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
            acc[i] += t;
        }
    }
    if (calls) *calls = (uint32_t)P->prof_events.size();
    for (auto &ev : P->prof_events)
        for (auto e : ev) (void)hipEventDestroy(e);
    P->prof_events.clear();
    for (uint32_t i = 0; i < n && i < (uint32_t)kStages; i++) ms[i] = acc[i];
    return kStages;
}

const char *tmd_stage_name(uint32_t stage) { return stage < (uint32_t)kStages ? kStageNames[stage] : ""; }

int tmd_selftest_fp(const float *a, const float *b, float *out, uint32_t n, void *stream)
{
    if (!a || !b || !out) return TMD_E_ARG;
    if (n == 0) return TMD_OK;
    hipLaunchKernelGGL(k_selftest_fp, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, a, b, out, n);
    HIP_TRY(hipGetLastError());
    return TMD_OK;
}

}  // extern "C"
