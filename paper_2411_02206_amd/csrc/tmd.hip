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
// Pipeline (all frames of a plan in each launch, in this order):
//   K1 k_tilesum     sum of track lengths per tile of 256 tracks; clears the
//                    frames' status words
//   K2 k_count       track start offsets (scan), per-cluster (sector,row) walk,
//                    per-tile bin histogram
//   K3 k_colscan     per bin, exclusive prefix of the tile histograms
//   K4 k_offsets     per frame, bin offsets of the output and of the
//                    unattached input (flags count mismatches)
//   K6 k_rank        per tile, stable slot of every attached cluster
//   K7 k_attached    one lane per track (a few lanes take a second track
//                    after the first): the float32 propagate-and-update
//   K5 k_unattached  per bin, running sums of the differences (one wave)
#include <hip/hip_runtime.h>

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "tmd.h"

#define NSEC TMD_NSEC
#define NROW TMD_NROW
#define NBIN TMD_NBIN

namespace {

constexpr int kTile = 256;  // tracks per tile: K2, K6, K7 blocks
constexpr int kWave = 64;
constexpr int kTileWaves = kTile / kWave;
constexpr int kAttWaves = 1;  // waves per workgroup of the attached decode
constexpr uint32_t kTimeLim = 1u << 24;

// ---------------------------------------------------------------------------
// constant tables (float32, each the nearest float to a double expression)
// ---------------------------------------------------------------------------
struct RowGeo {  // one pad row (32 bytes)
    float x;       // local x of the row (cm)
    float inv_pw;  // 1 / pad width
    float padoff;  // half the number of pads (pad 0 is the -y edge)
    float pwq;     // pad quantum: pad width / 32
    float ks, kt;  // update gains of sin(phi) and tan(lambda): 0.0625 / row pitch
    float pw;      // pad width (cm)
    float unused;
};
static_assert(sizeof(RowGeo) == 32 && offsetof(RowGeo, ks) == 16, "row table layout");

struct Geo {
    RowGeo row[NROW];
    float cosb[18], sinb[18];  // rotation by d * 20 degrees
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
    memset(g, 0, sizeof(*g));
    for (int g4 = 0; g4 < 4; g4++) {
        for (int r = rs[g4]; r < rs[g4 + 1]; r++) {
            double xd = xs[g4] + ((double)(r - rs[g4]) + 0.5) * pitch[g4];
            int npads = 2 * (int)floor(xd * tan(pi / 18.0) / padw[g4]);
            RowGeo &R = g->row[r];
            R.x = (float)xd;
            R.pw = (float)padw[g4];
            R.inv_pw = (float)(1.0 / padw[g4]);
            R.padoff = (float)(npads / 2);
            R.pwq = R.pw * 0.03125f;
            R.ks = (float)(0.0625 / pitch[g4]);
            R.kt = R.ks;
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
// per-frame descriptor.  On the device its pointers are in the global address
// space, so that loads and stores through them are global (not flat) accesses.
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__)
#define GLB __attribute__((address_space(1)))
#else
#define GLB
#endif

// scheduling key of a track: home sector (sector of cluster 0) * 3 + direction
// class (0: rows strictly increasing, 1: strictly decreasing, 2: other).  In
// schedule order (key, index) the tracks of a wave are neighbours in the
// stream, so their clusters on one row fill neighbouring output slots of one
// bin; ordering by anything that separates stream neighbours (such as the rows
// a track spans) scatters the decode's stores.
constexpr int kNKey = NSEC * 3;
constexpr int kHRow = NBIN + kNKey;  // per-tile histogram row: bins, then keys

// per-cluster record written by the rank kernel for the decode kernel (16 B):
// x = output slot, y = pad residual (low 16, signed) | time residual (high 16),
// z = qTot (low 16) | qMax (high 16), w = row (bits 0-7) | rotation (bits
// 8-15: the cluster's sector step modulo 18, the number of 20-degree turns
// from the previous cluster's frame)

// one field list, two views: FrameDesc (device, global pointers) and
// FrameDescHost (host, plain pointers) have the same layout
#define TMD_FRAME_FIELDS(Q)                                                                   \
    /* input */                                                                               \
    const Q uint8_t *ncls, *sec0, *row0;                                                      \
    const Q uint16_t *pad0;                                                                   \
    const Q uint32_t *time0;                                                                  \
    const Q int16_t *qpt, *snp, *tgl;                                                         \
    const Q int8_t *rdiff;                                                                    \
    const Q uint8_t *sdiff;                                                                   \
    const Q int16_t *pres, *tres;                                                             \
    const Q uint16_t *cqtot, *cqmax;                                                          \
    const Q uint32_t *ucount, *utdiff;                                                        \
    const Q uint16_t *updiff, *uqtot, *uqmax;                                                 \
    /* output */                                                                              \
    Q uint32_t *roff, *rna, *otime;                                                           \
    Q uint16_t *opad, *oqtot, *oqmax;                                                         \
    /* workspace */                                                                           \
    Q uint32_t *start;   /* [nT + 1] first cluster of each track */                           \
    Q uint32_t *tilesum; /* [ntile] clusters per tile */                                      \
    Q uint32_t *hist;    /* [ntile][kHRow] per-tile bin/key counts, then exclusive prefixes */ \
    Q uint32_t *uin;     /* [NBIN] first unattached input entry of each bin */                \
    Q uint32_t *ueff;    /* [NBIN] unattached clusters decoded per bin */                     \
    Q uint4 *recs;       /* [nA] (slot, charges, residuals, row|rot), stream order */         \
    Q uint16_t *ckey;    /* [nA] (sector,row) bin of each attached cluster, stream order */    \
    Q uint32_t *keyinfo; /* [kNKey] tracks per scheduling key, [kNKey] key starts */          \
    Q uint16_t *tkey;    /* [nT] scheduling key of each track */                              \
    Q uint32_t *order;   /* [nT] tracks sorted by (key, index): the decode's schedule */      \
    Q uint32_t *status;                                                                       \
    const Q uint32_t *pre_status; /* flags the frame starts with (entropy decoding), or null */ \
    uint64_t cap; /* entries of the output cluster arrays; every store is checked */          \
    uint32_t nT, nA, nU, ntile, tile0;                                                        \
    uint32_t awaves; /* waves of the attached decode */                                       \
    uint32_t un_fused; /* the unattached clusters are decoded with their entropy decoding */  \
    uint32_t pad_;

struct FrameDesc {
    TMD_FRAME_FIELDS(GLB)
};
struct FrameDescHost {
    TMD_FRAME_FIELDS()
};
static_assert(sizeof(FrameDesc) == sizeof(FrameDescHost), "descriptor layouts differ");

// ---------------------------------------------------------------------------
// wave helpers (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    // lanes without a source keep 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xf, false);
}

// inclusive prefix sum over the 64 lanes (DPP row shifts, then row broadcasts)
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t v)
{
    v += dpp<0x111, 0xf>(v);  // row_shr:1
    v += dpp<0x112, 0xf>(v);  // row_shr:2
    v += dpp<0x114, 0xf>(v);  // row_shr:4
    v += dpp<0x118, 0xf>(v);  // row_shr:8
    v += dpp<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v)
{
    return (uint64_t)readlane((uint32_t)v, 0) | ((uint64_t)readlane((uint32_t)(v >> 32), 0) << 32);
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v |= __shfl_xor(v, d);
    return v;
}

// exclusive scan over a block of kTile threads; returns the block total in *tot
template <int NW = kTileWaves>  // waves of the block
__device__ uint32_t block_excl_add(uint32_t v, uint32_t *tot)
{
    __shared__ uint32_t part[NW];
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_add(v);
    if (lane == kWave - 1) part[w] = inc;
    __syncthreads();
    uint32_t base = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        uint32_t p = part[i];
        if (i < (int)w) base += p;
        all += p;
    }
    __syncthreads();
    *tot = all;
    return base + inc - v;
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) round robin by
// workgroup id.  This maps workgroup b to a tile so that each XCD gets one
// contiguous range of tiles: neighbouring tiles, whose stores share cache
// lines, then meet in the same L2.  A bijection for any grid size.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n)
{
    const uint32_t x = b % kXcds, i = b / kXcds;
    const uint32_t q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// Copy n 16-byte vectors from global memory to LDS, all loads of a batch in
// flight before the first LDS write (a load-then-store loop would wait for
// every load in turn).
template <int BATCH, int NT>
__device__ __forceinline__ void copy_to_lds(uint4 *dst, const GLB uint4 *src, uint32_t n)
{
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += BATCH * NT) {
        uint4 v[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; b++) {
            const uint32_t i = i0 + b * NT;
            v[b] = make_uint4(0, 0, 0, 0);
            if (i < n) v[b] = src[i];
        }
#pragma unroll
        for (int b = 0; b < BATCH; b++) {
            const uint32_t i = i0 + b * NT;
            if (i < n) dst[i] = v[b];
        }
    }
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

__device__ __forceinline__ uint32_t key_class(uint32_t key) { return key % 3u; }

__device__ __forceinline__ void step_pos(int &sec, int &row, int rd, uint32_t sd)
{
    if (sd >= 18) sd %= 18;
    if (sd) sec = (sec / 18) * 18 + (sec % 18 + (int)sd) % 18;
    row += rd;
    row = row < 0 ? 0 : (row > NROW - 1 ? NROW - 1 : row);
}

// ---------------------------------------------------------------------------
// K1: clusters per tile (the extra blocks after the tiles clear the status
// word of each frame)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTile) void k_tilesum(const FrameDesc *__restrict__ fd,
                                                   const uint32_t *__restrict__ tile_frame, uint32_t ntiles,
                                                   uint32_t *__restrict__ work)
{
    if (blockIdx.x >= ntiles) {  // one extra block per frame: clear its status word
        if (threadIdx.x == 0) {
            const FrameDesc &G = fd[blockIdx.x - ntiles];
            *G.status = G.pre_status ? *G.pre_status : 0u;
        }
        // (and the first one the attached decode's work counters, if used)
        if (work && blockIdx.x == ntiles && threadIdx.x < kXcds) work[threadIdx.x] = 0u;
        return;
    }
    const uint32_t tile = blockIdx.x;
    const FrameDesc F = fd[tile_frame[tile]];
    const uint32_t lt = tile - F.tile0;
    if (lt >= F.ntile) return;  // a tile of the planned capacity beyond this call's frame
    const uint32_t t = lt * kTile + threadIdx.x;
    const uint32_t v = t < F.nT ? F.ncls[t] : 0u;
    uint32_t tot;
    block_excl_add(v, &tot);
    if (threadIdx.x == 0) F.tilesum[lt] = tot;
}

// ---------------------------------------------------------------------------
// Flat walk of a wave's consecutive tracks (32 in the count kernel).  Their
// decoded clusters form one contiguous range [A, E) of the cluster stream; the
// wave walks it in chunks of 64 clusters (lane = cluster), loading several
// chunks at a time.
// Inside a chunk the rows and sectors are segmented prefix sums: a segment
// starts at a track's first cluster (its header position) or continues the
// previous chunk's last track.  If a row would leave [0, 151] the chunk is
// walked cluster by cluster with the clamps instead.
// ---------------------------------------------------------------------------
struct WaveLds {
    uint8_t hrow[kWave];   // header row of track lane l (clamped)
    uint8_t hsec[kWave];   // header sector of track lane l (wrapped)
    uint8_t hm[kWave];     // per chunk: track lane whose first cluster is at lo + i, or 0xFF
    uint32_t cls[kWave];   // K2: direction bits of track lane l (bit 0 all up, bit 1 all down)
};

__device__ __forceinline__ uint32_t bperm(uint32_t v, uint32_t src_lane)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src_lane * 4u), (int)v);
}

struct WalkState {
    int csec, crow;     // position of the last cluster of the previous chunk
    uint32_t ctrack;    // track lane of the last cluster of the previous chunk
};

// Per-lane track setup; returns the wave's cluster range [A, E).  Lane l < ntr
// holds track tw + l (if < nT): its start, decoded length and header position.
__device__ __forceinline__ void wave_setup(const FrameDesc &F, uint32_t tw, uint32_t ntr, WaveLds &L,
                                           uint32_t start_in, uint32_t &start_l, uint32_t &n_l, uint32_t &A,
                                           uint32_t &E)
{
    const uint32_t lane = lane_id();
    const uint32_t t = tw + lane;
    uint32_t nc = 0;
    start_l = 0xFFFFFFFFu;
    n_l = 0;
    uint8_t r = 0, s = 0;
    if (lane < ntr && t < F.nT) {
        start_l = start_in;
        nc = F.ncls[t];
        n_l = track_len(start_l, nc, F.nA);
        HeaderPos h = header_pos(F.sec0[t], F.row0[t]);
        r = (uint8_t)h.row;
        s = (uint8_t)h.sec;
    }
    L.hrow[lane] = r;
    L.hsec[lane] = s;
    L.cls[lane] = 3u;
    const uint32_t a = readlane(start_l, 0);  // track tw exists whenever the wave runs
    const uint32_t sum = readlane(wave_incl_add(nc), kWave - 1);
    const unsigned long long e = (unsigned long long)a + sum;
    A = a;
    E = (uint32_t)(e < F.nA ? e : F.nA);
    if (A > E) A = E;
}

// Keys of the chunk [lo, lo + 64) ∩ [lo, E).  rd/sd: this lane's raw row and
// sector steps (loaded by the caller).  Returns the (sector,row) key (0 for
// inactive lanes) and, in *tl, the track lane the cluster belongs to.
__device__ __forceinline__ uint32_t walk_chunk(uint32_t lo, uint32_t E, int rd, uint32_t sd, uint32_t start_l,
                                               uint32_t n_l, WaveLds &L, WalkState &ws, uint32_t &fl,
                                               uint32_t &tl, bool &clamped)
{
    const uint32_t lane = lane_id();
    const uint32_t c = lo + lane;
    const bool act = c < E;
    // mark the first cluster of every track starting in this chunk
    L.hm[lane] = 0xFFu;
    __builtin_amdgcn_wave_barrier();
    if (n_l > 0 && start_l >= lo && start_l - lo < (uint32_t)kWave) L.hm[start_l - lo] = (uint8_t)lane;
    __builtin_amdgcn_wave_barrier();
    const uint32_t h = L.hm[lane];
    const bool head = act && h != 0xFFu;
    const bool step = act && !head;
    uint32_t sdm = 0;
    int rdv = 0;
    if (step) {
        rdv = rd;
        sdm = sd;
        if (sdm >= 18) {
            fl |= TMD_F_SEC;
            sdm %= 18;
        }
    }
    // row and sector steps in one inclusive sum: low half row step + 128
    // (0..255), high half sector step (0..17); over 64 lanes neither half
    // carries into the other
    const uint32_t PK = wave_incl_add(step ? (uint32_t)(rdv + 128) | (sdm << 16) : 0u);
    // the segment's head: the last head lane at or below this lane (every lane
    // between it and this one is a step, since inactive lanes come last)
    const uint64_t hm = __ballot(head);
    const uint64_t upto = hm & (lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull));
    const uint32_t hl = upto ? (uint32_t)(kWave - 1) - (uint32_t)__clzll(upto) : 0u;
    const uint32_t PKH = bperm(PK, hl), TH = bperm(h, hl);
    int row, sec;
    if (upto) {
        const int br = L.hrow[TH], bs = L.hsec[TH];
        row = br + ((int)(PK & 0xFFFFu) - (int)(PKH & 0xFFFFu)) - 128 * (int)(lane - hl);
        sec = (bs / 18) * 18 + (int)((uint32_t)(bs % 18) + ((PK >> 16) - (PKH >> 16))) % 18;
        tl = TH;
    } else {
        row = ws.crow + (int)(PK & 0xFFFFu) - 128 * (int)(lane + 1u);
        sec = (ws.csec / 18) * 18 + (int)((uint32_t)(ws.csec % 18) + (PK >> 16)) % 18;
        tl = ws.ctrack;
    }
    clamped = __ballot(act && (row < 0 || row >= NROW)) != 0;
    if (clamped) {
        // walk the chunk in order with the clamps
        fl |= TMD_F_ROW;
        int s = ws.csec, r = ws.crow;
        for (uint32_t i = 0; i < (uint32_t)kWave; i++) {
            if (lo + i >= E) break;
            const uint32_t hi = (uint32_t)__shfl((int)h, (int)i);
            const int rdi = __shfl(rd, (int)i);
            const uint32_t sdi = (uint32_t)__shfl((int)sd, (int)i);
            if (hi != 0xFFu) {
                r = L.hrow[hi];
                s = L.hsec[hi];
            } else {
                step_pos(s, r, rdi, sdi);
            }
            if (i == lane) {
                row = r;
                sec = s;
            }
        }
    }
    const uint32_t key = act ? (uint32_t)(sec * NROW + row) : 0u;
    const uint32_t last = (E - lo) < (uint32_t)kWave ? (E - lo - 1) : (uint32_t)(kWave - 1);
    const uint32_t lk = readlane(key, (int)last);
    ws.csec = (int)(lk / NROW);
    ws.crow = (int)(lk % NROW);
    ws.ctrack = readlane(tl, (int)last);
    return key;
}

// ---------------------------------------------------------------------------
// K2: track starts, per-tile histogram of cluster bins and of scheduling keys
// ---------------------------------------------------------------------------
constexpr int kGroup = 4;  // chunks loaded together by a walk
// the count kernel: 8 waves per tile of 256 tracks, 32 tracks per wave (the
// walk still covers 64 clusters per step; more waves per tile hide more of
// its latency)
constexpr int kCountWaves = 8;
constexpr int kCountTracks = kTile / kCountWaves;
constexpr int kCountThreads = kCountWaves * kWave;

__global__ __launch_bounds__(kCountThreads) void k_count(const FrameDesc *__restrict__ fd,
                                                         const uint32_t *__restrict__ tile_frame)
{
    // the tile's 16-bit bin counters, shared by its waves (256 tracks put at
    // most 256 * 255 < 2^16 clusters in one bin); 17 KB of LDS in all, so
    // that every tile of a frame can be resident at once
    __shared__ uint32_t wcnt32[NBIN / 2];
    __shared__ uint32_t khist[kNKey];
    __shared__ WaveLds wl[kCountWaves];
    const uint16_t *wcnt = reinterpret_cast<const uint16_t *>(wcnt32);
    const uint32_t tile = blockIdx.x;
    const FrameDesc F = fd[tile_frame[tile]];
    const uint32_t lt = tile - F.tile0;
    if (lt >= F.ntile) return;  // a tile of the planned capacity beyond this call's frame
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    // wave w takes tracks [32 w, 32 w + 32) of the tile in lanes 0..31
    const bool tl_ok = lane < (uint32_t)kCountTracks;
    const uint32_t t = lt * kTile + w * kCountTracks + lane;

    // clusters of all earlier tiles of the frame
    uint32_t pre = 0;
    for (uint32_t i = threadIdx.x; i < lt; i += kCountThreads) pre += F.tilesum[i];
    uint32_t before;
    block_excl_add<kCountWaves>(pre, &before);

    for (uint32_t i = threadIdx.x; i < NBIN / 2; i += kCountThreads) wcnt32[i] = 0;
    for (uint32_t i = threadIdx.x; i < kNKey; i += kCountThreads) khist[i] = 0;
    const uint32_t nc = tl_ok && t < F.nT ? F.ncls[t] : 0u;
    uint32_t tot;
    const uint32_t start = before + block_excl_add<kCountWaves>(nc, &tot);  // also syncs
    if (tl_ok && t < F.nT) {
        F.start[t] = start;
        if (t == F.nT - 1) {
            F.start[F.nT] = start + nc;
            if (start + nc != F.nA) atomicOr(F.status, TMD_F_COUNT);
        }
    }
    const uint32_t tw = lt * kTile + w * kCountTracks;
    if (tw < F.nT) {
        WaveLds &L = wl[w];
        uint32_t start_l, n_l, A, E;
        wave_setup(F, tw, kCountTracks, L, start, start_l, n_l, A, E);
        WalkState ws{0, 0, 0};
        uint32_t fl = 0;
        // groups of kGroup chunks; two groups alternate so that the loads of
        // one are in flight while the other is walked.  Loads are
        // unconditional: lanes past E read cluster E - 1, and the walk ignores
        // their steps.
        struct Group {
            int rd[kGroup];
            uint32_t sd[kGroup];
        };
        auto load = [&](uint32_t g, Group &P) {
#pragma unroll
            for (int u = 0; u < kGroup; u++) {
                const uint32_t c = g + u * kWave + lane;
                const uint32_t cc = c < E ? c : E - 1;
                P.rd[u] = (int)F.rdiff[cc];
                P.sd[u] = (uint32_t)F.sdiff[cc];
            }
        };
        auto walk = [&](uint32_t g, const Group &P) {
#pragma unroll
            for (int u = 0; u < kGroup; u++) {
                const uint32_t lo = g + u * kWave;
                if (lo >= E) break;
                uint32_t tl;
                bool clamped;
                const uint32_t key = walk_chunk(lo, E, P.rd[u], P.sd[u], start_l, n_l, L, ws, fl, tl, clamped);
                const uint32_t c = lo + lane;
                const bool act = c < E;
                // direction of this step for the track's class: the bits it
                // clears (1: not all up, 2: not all down)
                uint32_t clr = 0;
                if (act) {
                    F.ckey[c] = (uint16_t)key;
                    atomicAdd(&wcnt32[key >> 1], 1u << (16 * (key & 1)));
                    const bool head = L.hm[lane] != 0xFFu;
                    if (clamped) clr = 3u;
                    else if (!head) clr = (P.rd[u] > 0 ? 0u : 1u) | (P.rd[u] < 0 ? 0u : 2u);
                }
                // one LDS atomic per run of lanes with the same track and bits
                // (row_shr:1 within each row of 16 lanes; row starts count as
                // run starts)
                const uint32_t ptl = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)tl, 0x111, 0xf,
                                                                           0xf, false);
                const uint32_t pclr = (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)clr, 0x111,
                                                                            0xf, 0xf, false);
                if (clr && (ptl != tl || pclr != clr)) atomicAnd(&L.cls[tl], ~clr);
            }
        };
        constexpr uint32_t kStep = kWave * kGroup;
        Group P0, P1;
        if (A < E) load(A, P0);
        for (uint32_t g = A; g < E; g += 2 * kStep) {
            load(g + kStep, P1);
            walk(g, P0);
            if (g + kStep >= E) break;
            load(g + 2 * kStep, P0);
            walk(g + kStep, P1);
        }
        fl = wave_or(fl);
        if (lane == 0 && fl) atomicOr(F.status, fl);
        __builtin_amdgcn_wave_barrier();
        if (tl_ok && tw + lane < F.nT) {
            const uint32_t bits = L.cls[lane];
            const uint32_t cls = n_l <= 1 ? 0u : ((bits & 1u) ? 0u : ((bits & 2u) ? 1u : 2u));
            const uint32_t key = (uint32_t)L.hsec[lane] * 3u + cls;
            F.tkey[tw + lane] = (uint16_t)key;
            atomicAdd(&khist[key], 1u);
        }
    }
    __syncthreads();
    // the tile's row of the histogram: bin counts, then key counts
    GLB uint32_t *dst = F.hist + (size_t)lt * kHRow;
    for (uint32_t k = threadIdx.x; k < NBIN; k += kCountThreads) dst[k] = wcnt[k];
    for (uint32_t i = threadIdx.x; i < kNKey; i += kCountThreads) dst[NBIN + i] = khist[i];
}

// ---------------------------------------------------------------------------
// K3: per histogram column (bin or key), exclusive prefix over the frame's
// tiles; bin totals -> row_nattached, key totals -> keyinfo
// grid (ceil(kHRow/64), n_frames), block 1024 = 16 waves; lane = column
// ---------------------------------------------------------------------------
constexpr int kScanWaves = 16;
constexpr int kColBatch = 8;
constexpr int kColKeep = 64;  // column entries per wave kept in registers (a frame of 64 * 16 tiles)

__global__ __launch_bounds__(kWave * kScanWaves) void k_colscan(const FrameDesc *__restrict__ fd)
{
    __shared__ uint32_t part[kScanWaves][kWave];
    const FrameDesc F = fd[blockIdx.y];
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    const uint32_t k = blockIdx.x * kWave + lane;
    const uint32_t per = (F.ntile + kScanWaves - 1) / kScanWaves;
    const uint32_t a = w * per;
    const uint32_t b = min(a + per, F.ntile);
    // a wave's share of the column: up to kColKeep entries stay in registers
    // between the sum and the prefix (read once); longer shares are read again
    uint32_t keep[kColKeep];
    uint32_t sum = 0;
    if (k < kHRow) {
#pragma unroll
        for (int u = 0; u < kColKeep; u++) {
            keep[u] = a + u < b ? F.hist[(size_t)(a + u) * kHRow + k] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kColKeep; u++) sum += keep[u];
        // loads in batches of kColBatch, so that a batch is in flight together
        for (uint32_t i0 = a + kColKeep; i0 < b; i0 += kColBatch) {
            uint32_t v[kColBatch];
#pragma unroll
            for (int u = 0; u < kColBatch; u++) v[u] = i0 + u < b ? F.hist[(size_t)(i0 + u) * kHRow + k] : 0u;
#pragma unroll
            for (int u = 0; u < kColBatch; u++) sum += v[u];
        }
    }
    part[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, total = 0;
    for (uint32_t i = 0; i < kScanWaves; i++) {
        uint32_t p = part[i][lane];
        if (i < w) run += p;
        total += p;
    }
    if (k < kHRow) {
#pragma unroll
        for (int u = 0; u < kColKeep; u++) {
            if (a + u < b) F.hist[(size_t)(a + u) * kHRow + k] = run;
            run += keep[u];
        }
        for (uint32_t i0 = a + kColKeep; i0 < b; i0 += kColBatch) {
            uint32_t v[kColBatch];
#pragma unroll
            for (int u = 0; u < kColBatch; u++) v[u] = i0 + u < b ? F.hist[(size_t)(i0 + u) * kHRow + k] : 0u;
#pragma unroll
            for (int u = 0; u < kColBatch; u++) {
                if (i0 + u < b) F.hist[(size_t)(i0 + u) * kHRow + k] = run;
                run += v[u];
            }
        }
        if (w == 0) {
            if (k < NBIN) F.rna[k] = total;
            else F.keyinfo[k - NBIN] = total;
        }
    }
}

// ---------------------------------------------------------------------------
// K4: per frame, output offsets, unattached input offsets, key starts
// grid n_frames, block 1024; thread i owns bins [6i, 6i + 6)
// ---------------------------------------------------------------------------
constexpr int kOffThreads = 1024;
constexpr int kOffPer = (NBIN + kOffThreads - 1) / kOffThreads;  // 6
constexpr int kKeyPer = (kNKey + kOffThreads - 1) / kOffThreads;

__global__ __launch_bounds__(kOffThreads) void k_offsets(const FrameDesc *__restrict__ fd)
{
    __shared__ unsigned long long part64[kOffThreads / kWave];
    __shared__ uint32_t part32[kOffThreads / kWave];
    const FrameDesc F = fd[blockIdx.x];
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    const uint32_t b0 = threadIdx.x * kOffPer;

    // every input read up front (one memory round trip): unattached counts,
    // attached counts and tracks per scheduling key, all per bin or key
    unsigned long long cnt[kOffPer];
    uint32_t na[kOffPer];
    unsigned long long own = 0;
    for (int i = 0; i < kOffPer; i++) {
        uint32_t b = b0 + i;
        cnt[i] = b < NBIN ? F.ucount[b] : 0u;
        na[i] = b < NBIN ? F.rna[b] : 0u;
        own += cnt[i];
    }
    uint32_t kc[kKeyPer];
    uint32_t kown = 0;
    for (int i = 0; i < kKeyPer; i++) {
        const uint32_t key = threadIdx.x * kKeyPer + i;
        kc[i] = key < (uint32_t)kNKey ? F.keyinfo[key] : 0u;
        kown += kc[i];
    }

    // unattached input: exclusive prefix of un_count in 64 bits, cut at nU
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
            eff[i] = e + na[i];
        } else {
            eff[i] = 0;
        }
        ownout += eff[i];
        us += cnt[i];
    }
    if (threadIdx.x == 0 && (all != F.nU || (F.nT == 0 && F.nA != 0))) atomicOr(F.status, TMD_F_COUNT);
    // flags of a step before the decode that may have ended after k_tilesum
    // took the frame's starting flags (entropy decoding beside the first
    // kernels)
    if (threadIdx.x == 0 && F.pre_status) atomicOr(F.status, *F.pre_status);

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

    // start of each scheduling key in the decode order
    __syncthreads();  // part32 is reused
    const uint32_t kinc = wave_incl_add(kown);
    if (lane == kWave - 1) part32[w] = kinc;
    __syncthreads();
    uint32_t krun = 0;
    for (uint32_t i = 0; i < w; i++) krun += part32[i];
    krun += kinc - kown;
    for (int i = 0; i < kKeyPer; i++) {
        const uint32_t key = threadIdx.x * kKeyPer + i;
        if (key < (uint32_t)kNKey) F.keyinfo[kNKey + key] = krun;
        krun += kc[i];
    }
}

// ---------------------------------------------------------------------------
// K5: unattached clusters; one wave per (bin, frame).  A lane takes 4
// consecutive clusters of a group of 256 and moves them with one wide access
// per array (16 bytes of time, 8 of each 16-bit field: the address unit
// handles a wave's access at a cost that grows with the instructions more
// than with their width).  Bins start anywhere, so the accesses are not
// aligned to their width (the hardware allows that for global memory).  The
// one lane whose group is cut by the bin's end uses element accesses, so
// nothing outside the bin is read or written.  4 groups (1024 clusters) per
// pass, all their loads in flight together.
// ---------------------------------------------------------------------------
constexpr int kUGroups = 4;

template <class V, class T>
__device__ __forceinline__ V load_wide(const GLB T *p)
{
    V v;
    __builtin_memcpy(&v, (const GLB char *)p, sizeof(V));
    return v;
}

template <class V, class T>
__device__ __forceinline__ void store_wide(GLB T *p, const V &v)
{
    __builtin_memcpy((GLB char *)p, &v, sizeof(V));
}

__global__ __launch_bounds__(kWave) void k_unattached(const FrameDesc *__restrict__ fd)
{
    const FrameDesc F = fd[blockIdx.y];
    if (F.un_fused) return;  // (done by the entropy decoding, k_rans<W, kRansUnPhase>)
    const uint32_t k = blockIdx.x;
    const uint32_t cnt = F.ueff[k];
    if (cnt == 0) return;
    const uint32_t src = F.uin[k];
    const uint32_t dst = F.roff[k] + F.rna[k];
    const uint32_t lane = lane_id();
    // the whole bin lies inside the output (a store past the capacity is never
    // issued; the offsets kernel keeps dst + cnt <= n_attached + n_unattached
    // for consistent streams, and capacity >= that sum)
    const uint32_t room = dst < F.cap ? (uint32_t)min((uint64_t)cnt, F.cap - dst) : 0u;
    uint32_t ct = 0, cp = 0;
    for (uint32_t i = 0; i < cnt; i += kUGroups * 4 * kWave) {
        uint32_t td[kUGroups][4], pd[kUGroups][4], qt[kUGroups][4], qm[kUGroups][4];
#pragma unroll
        for (int u = 0; u < kUGroups; u++) {
            const uint32_t e = i + (uint32_t)u * 4 * kWave + 4 * lane;  // first element of this lane
            if (e + 4 <= cnt) {
                const uint4 t4 = load_wide<uint4>(F.utdiff + src + e);
                const uint2 p4 = load_wide<uint2>(F.updiff + src + e);
                const uint2 a4 = load_wide<uint2>(F.uqtot + src + e);
                const uint2 b4 = load_wide<uint2>(F.uqmax + src + e);
                td[u][0] = t4.x; td[u][1] = t4.y; td[u][2] = t4.z; td[u][3] = t4.w;
                pd[u][0] = p4.x & 0xFFFFu; pd[u][1] = p4.x >> 16; pd[u][2] = p4.y & 0xFFFFu; pd[u][3] = p4.y >> 16;
                qt[u][0] = a4.x & 0xFFFFu; qt[u][1] = a4.x >> 16; qt[u][2] = a4.y & 0xFFFFu; qt[u][3] = a4.y >> 16;
                qm[u][0] = b4.x & 0xFFFFu; qm[u][1] = b4.x >> 16; qm[u][2] = b4.y & 0xFFFFu; qm[u][3] = b4.y >> 16;
            } else {
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const bool act = e + q < cnt;
                    td[u][q] = act ? F.utdiff[src + e + q] : 0u;
                    pd[u][q] = act ? (uint32_t)F.updiff[src + e + q] : 0u;
                    qt[u][q] = act ? (uint32_t)F.uqtot[src + e + q] : 0u;
                    qm[u][q] = act ? (uint32_t)F.uqmax[src + e + q] : 0u;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kUGroups; u++) {
            const uint32_t e = i + (uint32_t)u * 4 * kWave + 4 * lane;
            // running sums: the lane's own four, then the lanes before it
            uint32_t st[4], sp[4];
            st[0] = td[u][0];
            sp[0] = pd[u][0];
#pragma unroll
            for (int q = 1; q < 4; q++) {
                st[q] = st[q - 1] + td[u][q];
                sp[q] = sp[q - 1] + pd[u][q];
            }
            const uint32_t it = wave_incl_add(st[3]), ip = wave_incl_add(sp[3]);
            const uint32_t bt = ct + it - st[3], bp = cp + ip - sp[3];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                st[q] += bt;
                sp[q] += bp;
            }
            if (e + 4 <= room) {
                store_wide(F.otime + dst + e, make_uint4(st[0], st[1], st[2], st[3]));
                store_wide(F.opad + dst + e, make_uint2((sp[0] & 0xFFFFu) | (sp[1] << 16),
                                                        (sp[2] & 0xFFFFu) | (sp[3] << 16)));
                store_wide(F.oqtot + dst + e, make_uint2(qt[u][0] | (qt[u][1] << 16), qt[u][2] | (qt[u][3] << 16)));
                store_wide(F.oqmax + dst + e, make_uint2(qm[u][0] | (qm[u][1] << 16), qm[u][2] | (qm[u][3] << 16)));
            } else {
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    if (e + q < room) {
                        F.otime[dst + e + q] = st[q];
                        F.opad[dst + e + q] = (uint16_t)sp[q];
                        F.oqtot[dst + e + q] = (uint16_t)qt[u][q];
                        F.oqmax[dst + e + q] = (uint16_t)qm[u][q];
                    }
                }
            }
            ct = readlane(it, kWave - 1) + ct;
            cp = readlane(ip, kWave - 1) + cp;
        }
    }
}

// ---------------------------------------------------------------------------
// K6: output slot of every attached cluster, written with the cluster's
// residuals, charges and (sector,row) as one 16-byte record in stream order;
// also places the tile's tracks in the decode schedule.  Within a bin the slot
// order is the stream order (track, then cluster).  Block = one tile of 256
// tracks, whose clusters are one contiguous range of the stream (with the
// bins the count kernel stored).  LDS holds one running slot per bin (bin
// base + tile prefix, advanced by atomic adds): 24 KB, so that every tile of
// a frame can be resident at once.  The range is cut into groups of 256
// clusters, taken by the four waves in turn (group q by wave q % 4).  A
// group's slots are taken in stream order: the wave waits until the tile's
// turn counter reaches q, issues its four chunks' atomic adds (each followed
// by a read-back of the counters), and sets the turn to q + 1.  LDS executes
// one wave's operations in issue order, so the next wave can only see the new
// turn once the atomics are done; no wait is needed in between.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTile) void k_rank(const FrameDesc *__restrict__ fd,
                                                const uint32_t *__restrict__ tile_frame)
{
    __shared__ uint32_t base[NBIN];                // next slot of each bin
    __shared__ uint32_t kcnt[kTileWaves][kNKey];  // tracks per (wave, scheduling key)
    __shared__ uint32_t turn;                      // the group whose slots are taken next
    const uint32_t tile = blockIdx.x;
    const FrameDesc F = fd[tile_frame[tile]];
    const uint32_t lt = tile - F.tile0;
    if (lt >= F.ntile) return;  // a tile of the planned capacity beyond this call's frame
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    const GLB uint32_t *G = F.hist + (size_t)lt * kHRow;
    const uint32_t t = lt * kTile + threadIdx.x;
    static_assert(kNKey <= 128, "schedule keys are matched on 7 bits");

    {
        constexpr int kPer = (NBIN + kTile - 1) / kTile;
        uint32_t ro[kPer], gg[kPer];
#pragma unroll
        for (int b = 0; b < kPer; b++) {
            const uint32_t k = threadIdx.x + b * kTile;
            ro[b] = k < NBIN ? F.roff[k] : 0u;
            gg[b] = k < NBIN ? G[k] : 0u;
        }
#pragma unroll
        for (int b = 0; b < kPer; b++) {
            const uint32_t k = threadIdx.x + b * kTile;
            if (k < NBIN) base[k] = ro[b] + gg[b];
        }
    }
    for (uint32_t i = threadIdx.x; i < kTileWaves * kNKey; i += kTile) (&kcnt[0][0])[i] = 0;
    if (threadIdx.x == 0) turn = 0;
    const bool tv = t < F.nT;
    const uint32_t tk = tv ? (uint32_t)F.tkey[t] : 0u;
    __syncthreads();
    if (tv) atomicAdd(&kcnt[w][tk], 1u);
    // rank among the wave's tracks with the same key (keys < 128: 7 bits)
    uint64_t same = __ballot(tv);
#pragma unroll
    for (int bit = 0; bit < 7; bit++) {
        const uint64_t m = __ballot(tv && ((tk >> bit) & 1u));
        same &= ((tk >> bit) & 1u) ? m : ~m;
    }
    uint32_t local = (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    __syncthreads();

    // decode schedule: tracks sorted by (key, index), stable
    if (tv) {
        for (uint32_t v = 0; v < w; v++) local += kcnt[v][tk];
        F.order[F.keyinfo[kNKey + tk] + G[NBIN + tk] + local] = t;
    }

    // the tile's clusters: [start of its first track, start of the next tile)
    // within nA
    const uint32_t tf = lt * kTile;
    const uint32_t te = tf + kTile < F.nT ? tf + kTile : F.nT;
    const uint32_t A = F.start[tf] < F.nA ? F.start[tf] : F.nA;
    const uint32_t E = F.start[te] < F.nA ? F.start[te] : F.nA;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    // a group of kGroup chunks: its loads, then its ranks and records.  A
    // wave's next group is loaded while the current one is ranked.  Loads are
    // unconditional (lanes past E read cluster E - 1 and ignore it) and raw,
    // so that nothing waits for them until the group is ranked.
    struct Group {
        uint32_t key[kGroup], sd[kGroup], pr[kGroup], tr[kGroup], qt[kGroup], qm[kGroup];
    };
    auto load = [&](uint32_t g, Group &P) {
#pragma unroll
        for (int u = 0; u < kGroup; u++) {
            const uint32_t c = g + u * kWave + lane;
            const uint32_t cc = c < E ? c : E - 1;
            P.key[u] = F.ckey[cc];
            P.sd[u] = F.sdiff[cc];
            P.pr[u] = (uint16_t)F.pres[cc];
            P.tr[u] = (uint16_t)F.tres[cc];
            P.qt[u] = F.cqtot[cc];
            P.qm[u] = F.cqmax[cc];
        }
    };
    auto rank = [&](uint32_t q, uint32_t g, const Group &P) {
        uint32_t k[kGroup], r[kGroup], fin[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; u++) k[u] = P.key[u] < (uint32_t)NBIN ? P.key[u] : 0u;
        // the bins are in registers before the turn is taken (no load is
        // waited for while the turn is held)
        asm volatile("" ::"v"(k[0]), "v"(k[1]), "v"(k[2]), "v"(k[3]));
        static_assert(kGroup == 4, "four chunks per group");
        // wait for this group's turn (bounded: the waves of the block are all
        // resident and every turn is passed on, so the bound is never reached
        // unless something is broken; then the frame is flagged)
        for (uint32_t spin = 0; __hip_atomic_load(&turn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != q;
             spin++) {
            if (spin == (1u << 22)) {
                if (lane == 0) atomicOr(F.status, TMD_F_COUNT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        // slots in stream order: per chunk, one atomic add per lane and a
        // read-back of the counters after it (the returned value is the rank
        // if no other lane of the chunk has the same bin)
#pragma unroll
        for (int u = 0; u < kGroup; u++) {
            r[u] = 0;
            fin[u] = 0;
            const uint32_t c = g + u * kWave + lane;
            if (c < E) r[u] = atomicAdd(&base[k[u]], 1u);
            __builtin_amdgcn_wave_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (c < E) fin[u] = __hip_atomic_load(&base[k[u]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_wave_barrier();
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (lane == 0) __hip_atomic_store(&turn, q + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
        for (int u = 0; u < kGroup; u++) {
            const uint32_t lo = g + u * kWave;
            if (lo >= E) break;
            const uint32_t c = lo + lane;
            const bool act = c < E;
            uint32_t slot = r[u];
            if (__ballot(act && fin[u] - r[u] != 1u)) {
                // some bin occurs more than once in the chunk: rank those
                // lanes in lane (= stream) order
                uint64_t same = __ballot(act);
#pragma unroll
                for (int bit = 0; bit < 13; bit++) {
                    const uint64_t m = __ballot(act && ((k[u] >> bit) & 1u));
                    same &= ((k[u] >> bit) & 1u) ? m : ~m;
                }
                slot = fin[u] - (uint32_t)__popcll(same) + (uint32_t)__popcll(same & lt_mask);
            }
            if (act) {
                const uint32_t rot = P.sd[u] < 18u ? P.sd[u] : P.sd[u] % 18u;
                F.recs[c] = make_uint4(slot, P.qt[u] | (P.qm[u] << 16), P.pr[u] | (P.tr[u] << 16),
                                       (k[u] % NROW) | (rot << 8));
            }
        }
    };
    constexpr uint32_t kStep = kWave * kGroup;
    const uint32_t nq = (E - A + kStep - 1) / kStep;  // groups of the tile
    // Each wave loads two of its groups ahead (its turns come every fourth
    // group, and a turn should not wait for loads).  Loads of groups past the
    // end read cluster E - 1: unconditional, so that waiting for one group
    // never waits for a later one's loads.
    Group P0, P1, P2;
    constexpr uint32_t kW = kTileWaves;
    uint32_t q = w;
    if (q < nq) {
        load(A + q * kStep, P0);
        load(A + (q + kW) * kStep, P1);
        for (;; q += 3 * kW) {
            load(A + (q + 2 * kW) * kStep, P2);
            rank(q, A + q * kStep, P0);
            if (q + kW >= nq) break;
            load(A + (q + 3 * kW) * kStep, P0);
            rank(q + kW, A + (q + kW) * kStep, P1);
            if (q + 2 * kW >= nq) break;
            load(A + (q + 4 * kW) * kStep, P1);
            rank(q + 2 * kW, A + (q + 2 * kW) * kStep, P2);
            if (q + 3 * kW >= nq) break;
        }
    }
}

// ---------------------------------------------------------------------------
// K7: attached decode, one lane per track.  Tracks come in schedule order
// (home sector, direction class, index).  A wave whose tracks all move
// outward (inward) advances row-synchronously: each step processes the lanes
// whose next cluster lies on the lowest (highest) pending row, so the lanes
// of a step write neighbouring slots of the same bin and read the same table
// row.  Other waves advance one cluster per lane per step.  The order of steps
// never changes a result: each track is decoded cluster after cluster either
// way.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float clamp_snp(float v, float smax, uint32_t &fl)
{
    const bool nan = v != v;
    const bool hi = v > smax;
    const bool lo = v < -smax;
    fl |= (nan || hi || lo) ? TMD_F_SNP : 0u;
    float r = hi ? smax : v;
    r = lo ? -smax : r;
    return nan ? 0.0f : r;
}

// The decode loop's forms of the same operations, shorter on this hardware and
// equal bit for bit on the arguments it sees (checked on the device by
// tmd_selftest_math and tmd_selftest_sqrt):
//
// clamp to [-smax, smax] with NaN -> 0; `flag` is set if v was outside or
// NaN.  The median of (v, -smax, smax) is the clamp of every non-NaN v.
__device__ __forceinline__ float clamp_snp_b(float v, float smax, bool &flag)
{
    const float c = __builtin_amdgcn_fmed3f(v, -smax, smax);
    flag |= c != v;  // also for NaN
    return v != v ? 0.0f : c;
}

// rint(v) as int32 clamped to [-2^30, 2^30], NaN -> 0.  v_cvt_i32_f32 turns
// NaN into 0 and saturates values outside int32, so an integer median ends it.
__device__ __forceinline__ int32_t sat_rint(float v)
{
    int32_t i;
    asm("v_cvt_i32_f32 %0, %1" : "=v"(i) : "v"(__builtin_rintf(v)));
    return min(max(i, -(1 << 30)), 1 << 30);
}

// IEEE square root of a positive normal float.  v_sqrt_f32 is within one ulp;
// of its result and the two neighbours, the residuals x - r' * r (one fused
// multiply-add each) pick the correctly rounded one.  This is the correction
// LLVM's AMDGPU back end itself emits for a correctly rounded f32 square root
// (the remainder of each neighbouring float, exact under a fused
// multiply-add, tells on which side of the true root it lies).  Every square root in the
// decode loop has its argument in [2^-9, 2^9]: (1 - s)(1 + s) with |s| <=
// 0.999, and 1 + (dy/dx)^2 with |dy/dx| <= 1.998 / (2 sqrt(0.001999)).
__device__ __forceinline__ float sqrt_pos(float x)
{
    const float r = __builtin_amdgcn_sqrtf(x);
    const float rm = __uint_as_float(__float_as_uint(r) - 1u);
    const float rp = __uint_as_float(__float_as_uint(r) + 1u);
    const float em = __builtin_fmaf(-rm, r, x);
    const float ep = __builtin_fmaf(-rp, r, x);
    const float q = em <= 0.0f ? rm : r;
    return ep > 0.0f ? rp : q;
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp_min_step(uint32_t v)
{
    // lanes (rows) without a source see the identity 0xFFFFFFFF
    return min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, CTRL, ROWMASK, 0xf, false));
}

// minimum over all 64 lanes (inclusive min-scan, then lane 63)
__device__ __forceinline__ uint32_t wave_min(uint32_t v)
{
    v = dpp_min_step<0x111, 0xf>(v);
    v = dpp_min_step<0x112, 0xf>(v);
    v = dpp_min_step<0x114, 0xf>(v);
    v = dpp_min_step<0x118, 0xf>(v);
    v = dpp_min_step<0x142, 0xa>(v);
    v = dpp_min_step<0x143, 0xc>(v);
    return readlane(v, kWave - 1);
}

// maximum over all 64 lanes
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) { return ~wave_min(~v); }

// Record staging: each lane keeps a ring of kRing records of its track in LDS,
// split in two arrays indexed [slot][lane]: rb = (residuals, row | rotation),
// read at every step, and ra = (output slot, charges), read when storing.
// The decode runs in blocks of kBlk steps; at each block boundary the records
// loaded at the previous boundary enter the ring, the block's decoded clusters
// (staged in LDS) are stored, and the next records are loaded.  Between
// boundaries the decode issues no global memory instruction, so no step waits
// for memory: every load and store has a whole block to complete.  A lane
// holds at least kBlk unread records at every boundary (or all that remain),
// enough for the kBlk steps that follow.
//
// Loads are cooperative: the next kBlk records of a track are contiguous, so
// kBlk neighbouring lanes fetch them with one instruction (lane l of load k
// fetches record l % 4 for track lane 16 k + l / 4): 64 contiguous bytes per
// group of four lanes instead of one cache line per lane.
constexpr int kBlk = 4;
constexpr int kRing = 2 * kBlk;
static_assert(kBlk == 4 && kWave == 64, "cooperative loads: 4 records per track, 16 tracks per load");

// per-lane decode state: one track, or two decoded one after the other (the
// second, B, starts at record nA; its initial state waits in the B fields)
struct LaneTrack {
    float x, y, z, s, tgl, k;
    int32_t t0;
    uint32_t pad0, fl, n, c0;
    uint32_t nA, c0B;  // records of the first track (n if there is no second); start of the second
    float xB, yB, sB, tglB, kB;
    int32_t t0B;
    uint32_t pad0B;
};

// records fetched by one cooperative load round, and where they go
struct CoopLoad {
    uint4 v[kBlk];
    uint32_t dst[kBlk];  // ring slot | track lane << 8, or ~0u: nothing to place
};

// Fetch records [L_t, L_t + m_t) of every lane t (L and m: this lane's
// values; m_t <= kBlk).  A lane's records j < nA are those of its first track
// (from c0), the rest those of its second (from c0B).
__device__ __forceinline__ void coop_load(const FrameDesc &F, uint32_t L, uint32_t m, uint32_t c0, uint32_t nA,
                                          uint32_t c0B, CoopLoad &C)
{
    const uint32_t lane = lane_id();
    const uint32_t q = lane & 3u;
    const uint32_t baseA = c0 + L;
    const uint32_t baseB = c0B + L - nA;  // (wraps while L < nA; used only for records >= nA)
    const uint32_t sp = nA > L ? min(nA - L, (uint32_t)kBlk) : 0u;  // of the kBlk, those of the first track
    const uint32_t lm = (L << 8) | (sp << 4) | m;  // L < 2^24, sp, m <= 4
#pragma unroll
    for (int k = 0; k < kBlk; k++) {
        const uint32_t t = 16u * k + (lane >> 2);
        const uint32_t bA = bperm(baseA, t), bB = bperm(baseB, t), lmt = bperm(lm, t);
        const bool ok = q < (lmt & 0xFu);
        const uint32_t a = q < ((lmt >> 4) & 0xFu) ? bA + q : bB + q;
        C.v[k] = F.recs[ok ? a : 0u];
        C.dst[k] = ok ? (((lmt >> 8) + q) % kRing) | (t << 8) : ~0u;
    }
}

__device__ __forceinline__ void coop_place(const CoopLoad &C, uint2 (*ra)[kWave], uint2 (*rb)[kWave])
{
#pragma unroll
    for (int k = 0; k < kBlk; k++) {
        if (C.dst[k] != ~0u) {
            const uint32_t sl = C.dst[k] & 0xFFu, t = C.dst[k] >> 8;
            ra[sl][t] = make_uint2(C.v[k].x, C.v[k].y);
            rb[sl][t] = make_uint2(C.v[k].z, C.v[k].w);
        }
    }
}

// The decode loop of one wave.  MODE 0: rows ascending, 1: descending (both
// row-synchronous), 2: one cluster per lane per step.  In modes 0 and 1 all
// lanes processing a step are on one row, so its table entry is read once per
// wave through the scalar cache.
// a wave-uniform row's table entry through the vector memory path: used when
// the entry requested through the scalar cache one step ahead is not the
// needed one, so that no second scalar load to the same registers is in
// flight (which would make the next request wait for every LDS access)
__device__ __forceinline__ RowGeo row_geo_vmem(const Geo *__restrict__ geo, uint32_t row)
{
    uint32_t r = row;
    asm volatile("" : "+v"(r));  // a per-lane index: a vector load
    const float4 a = *(const GLB float4 *)(&geo->row[r].x);
    const float2 b = *(const GLB float2 *)(&geo->row[r].ks);
    RowGeo R;
    R.x = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(a.x)));
    R.inv_pw = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(a.y)));
    R.padoff = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(a.z)));
    R.pwq = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(a.w)));
    R.ks = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(b.x)));
    R.kt = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(b.y)));
    R.pw = 0.0f;
    return R;
}

template <int MODE>
__device__ __forceinline__ void attached_loop(const FrameDesc &F, const Geo *__restrict__ geo,
                                              uint2 (*ra)[kWave], uint2 (*rb)[kWave], uint2 (*stg)[kWave],
                                              LaneTrack &T)
{
    const uint32_t lane = lane_id();
    // constants in registers (loaded once: the loop's stores could alias them
    // as far as the compiler knows); the rotation table one entry per lane,
    // read with ds_bpermute
    const float smax = geo->snp_max, vdq = geo->vdq, inv_vd32 = geo->inv_vd32;
    const float rcos = lane < 18u ? geo->cosb[lane] : 0.0f, rsin = lane < 18u ? geo->sinb[lane] : 0.0f;
    const uint32_t n = T.n, c0 = T.c0, nA = T.nA, c0B = T.c0B;
    // first records straight into the ring: two rounds of kBlk
    uint32_t L = n < (uint32_t)kRing ? n : (uint32_t)kRing;  // records [0, L) have entered the ring
    {
        CoopLoad C0, C1;
        const uint32_t m0 = n < (uint32_t)kBlk ? n : (uint32_t)kBlk;
        coop_load(F, 0, m0, c0, nA, c0B, C0);
        coop_load(F, kBlk, L - m0, c0, nA, c0B, C1);
        coop_place(C0, ra, rb);
        coop_place(C1, ra, rb);
    }
    CoopLoad nb;  // records [L, L + m), loaded at the last boundary
#pragma unroll
    for (int i = 0; i < kBlk; i++) nb.dst[i] = ~0u;
    uint32_t m = 0;
    uint2 cur = make_uint2(0, 0);  // record j (valid while j < L)
    if (L > 0) cur = rb[0][lane];
    uint32_t j = 0, jb = 0;       // next record; first record of the block
    uint32_t rmask = 0;           // steps of the block at which this lane decoded
    uint32_t vrow = 0xFFFFFFFFu;  // modes 0 and 1: the last row processed
    float x = T.x, y = T.y, z = T.z, s = T.s, tgl = T.tgl;
    float k = T.k;
    int32_t t0 = T.t0;
    uint32_t pad0 = T.pad0;
    // status checks accumulate in registers and are turned into flags once,
    // after the loop: out-of-range pads and times leave high bits in an OR of
    // the raw values; a clamped |sin phi| (or a NaN) leaves |v - clamp(v)| > 0
    // (or NaN) in a sum
    uint32_t pad_or = 0, time_or = 0, rot_bad = 0;
    float snp_dev = 0.0f;
    // modes 0 and 1: the table entry of the row after the last one, requested
    // one step ahead (the step's row is that row unless the wave skips rows)
    uint32_t grow = MODE == 0 ? 0u : (uint32_t)NROW - 1u;
    RowGeo Rn = geo->row[grow];
    // of two consecutive blocks at least one decodes a cluster (a block in
    // which no lane has a record in its ring refills them), so 2 * 64 * 255
    // blocks always suffice
    for (uint32_t blk = 0; blk < 2u * (uint32_t)kWave * 256u; blk++) {
        // (lane masks of compound conditions are ANDs of one-comparison
        // ballots: a ballot of an && costs two more vector instructions)
        for (int st = 0; st < kBlk; st++) {
            const bool live = j < L;
            uint64_t rdy = __ballot(live);
            if (rdy == 0) break;
            bool ready = live;
            RowGeo R;
            if (MODE != 2) {
                // rows 0..151; the descending mode works on 255 - row.  The
                // pending minimum is usually the row after the last one; only
                // if no lane is there is the minimum taken over all lanes
                // (with all lanes active: it reads other lanes).  Lanes with
                // no record left hold v = ~0, which no row matches.
                const uint32_t rr = (cur.y & 0xFFu);
                const uint32_t v = live ? (MODE == 0 ? rr : 255u - rr) : 0xFFFFFFFFu;
                vrow += 1u;
                rdy = __ballot(v == vrow);
                if (rdy == 0) {
                    vrow = wave_min(v);
                    rdy = __ballot(v == vrow);
                }
                ready = v == vrow;
                const uint32_t urow = MODE == 0 ? vrow : 255u - vrow;  // the row of every ready lane
                R = Rn;
                if (urow != grow) R = row_geo_vmem(geo, urow);
            }
            // rotation by d sectors, rare: a wave-uniform branch, the table
            // entry from lane d (read while every lane is active)
            const uint32_t d = (cur.y >> 8) & 0xFFu;  // 0..17
            const bool rot = ready && j > 0 && j != nA && d != 0;
            if ((rdy & __ballot(j > 0) & __ballot(j != nA) & __ballot(d != 0)) != 0) {
                const float ca = __uint_as_float(bperm(__float_as_uint(rcos), d));
                const float sa = __uint_as_float(bperm(__float_as_uint(rsin), d));
                if (rot) {
                    const float cs = sqrt_pos((1.0f - s) * (1.0f + s));
                    const float xn = (x * ca) + (y * sa);
                    const float yn = (y * ca) - (x * sa);
                    const float sn = (s * ca) - (cs * sa);
                    const float cn = (cs * ca) + (s * sa);
                    rot_bad |= (cn > 0.0f) ? 0u : 1u;
                    x = xn;
                    y = yn;
                    const float sc = __builtin_amdgcn_fmed3f(sn, -smax, smax);
                    snp_dev = snp_dev + fabsf(sn - sc);
                    s = sn != sn ? 0.0f : sc;
                }
            }
            if (ready) {
                const uint2 rec = cur;  // x = residuals, y = row | rotation << 8
                uint32_t otime = (uint32_t)t0, opad = pad0;
                if (j > 0 && j != nA) {  // (records 0 and nA: the tracks' header clusters)
                    if (MODE == 2) R = geo->row[rec.y & 0xFFu];
                    const float dx = R.x - x;
                    const float s1r = s + (k * dx);
                    const float s1c = __builtin_amdgcn_fmed3f(s1r, -smax, smax);
                    const float s1 = s1r != s1r ? 0.0f : s1c;
                    const float a0 = sqrt_pos((1.0f - s) * (1.0f + s));
                    const float a1 = sqrt_pos((1.0f - s1) * (1.0f + s1));
                    const float dydx = (s + s1) / (a0 + a1);
                    y = y + (dx * dydx);
                    z = z + (tgl * (dx * sqrt_pos(1.0f + (dydx * dydx))));
                    x = R.x;
                    const int32_t P = sat_rint(((y * R.inv_pw) + R.padoff) * 32.0f);
                    const int32_t Tq = sat_rint(z * inv_vd32);
                    const int32_t pres = (int32_t)(int16_t)(rec.x & 0xFFFFu);
                    const int32_t tres = (int32_t)(int16_t)(rec.x >> 16);
                    const int32_t padq = P + pres;
                    const int32_t timeq = t0 + Tq + tres;
                    pad_or |= (uint32_t)padq;
                    time_or |= (uint32_t)timeq;
                    otime = (uint32_t)min(max(timeq, 0), (int32_t)kTimeLim - 1);
                    opad = (uint32_t)min(max(padq, 0), 65535);
                    const float nuy = (float)pres * R.pwq;
                    const float nuz = (float)tres * vdq;
                    y = y + nuy;
                    z = z + nuz;
                    const float s2r = s1 + (nuy * R.ks);
                    const float s2c = __builtin_amdgcn_fmed3f(s2r, -smax, smax);
                    snp_dev = snp_dev + (fabsf(s1r - s1c) + fabsf(s2r - s2c));
                    s = s2r != s2r ? 0.0f : s2c;
                    tgl = tgl + (nuz * R.kt);
                }
                stg[st][lane] = make_uint2(otime, opad);
                rmask |= 1u << st;
                j++;
                if (j < L) cur = rb[j % kRing][lane];
            }
            // the second track starts (once per lane at most: a wave-uniform
            // branch keeps the copies out of every other step)
            if (__builtin_expect((rdy & __ballot(j == nA) & __ballot(j < n)) != 0, 0)) {
                if (ready && j == nA && j < n) {
                    x = T.xB;
                    y = T.yB;
                    z = 0.0f;
                    s = T.sB;
                    tgl = T.tglB;
                    k = T.kB;
                    t0 = T.t0B;
                    pad0 = T.pad0B;
                }
            }
            if (MODE != 2) {
                const uint32_t g = MODE == 0 ? vrow + 1u : 254u - vrow;
                grow = g < (uint32_t)NROW ? g : (uint32_t)NROW - 1u;
                Rn = geo->row[grow];
            }
        }
        // block boundary.  Records loaded at the last boundary enter the ring:
        // they end below jb + kRing (refill bound below), so their slots are
        // not those of records [jb, L), which hold this block's decoded
        // clusters (stored next) and the unread ones.
        const bool starved = j == L;
        coop_place(nb, ra, rb);
        L += m;
        if (starved && j < L) cur = rb[j % kRing][lane];
        // store the block's clusters step by step: the lanes that decoded at
        // one step share its row, so their slots are neighbours and each
        // store instruction covers a short run of a bin.  Slot and charges
        // come from the ring, time and pad from the staging area.
        uint2 r[kBlk], o[kBlk];
#pragma unroll
        for (int st = 0; st < kBlk; st++) {  // all reads first: one LDS round trip
            const uint32_t idx = jb + (uint32_t)__popc(rmask & ((1u << st) - 1u));
            r[st] = ra[idx % kRing][lane];
            o[st] = stg[st][lane];
        }
#pragma unroll
        for (int st = 0; st < kBlk; st++) {
            if (((rmask >> st) & 1u) && r[st].x < F.cap) {
                F.otime[r[st].x] = o[st].x;
                F.opad[r[st].x] = (uint16_t)o[st].y;
                F.oqtot[r[st].x] = (uint16_t)(r[st].y & 0xFFFFu);
                F.oqmax[r[st].x] = (uint16_t)(r[st].y >> 16);
            }
        }
        rmask = 0;
        jb = j;
        // next records: at most kBlk, and no more than the ring can take
        // without overwriting a record >= j (records [j, L + m) span at most
        // kRing slots), so at the next boundary the ring again holds at least
        // kBlk unread records or all that remain
        m = n - L;
        if (m > (uint32_t)kBlk) m = kBlk;
        const uint32_t room = (uint32_t)kRing - (L - j);
        if (m > room) m = room;
        if (__ballot(j < n) == 0) break;
        coop_load(F, L, m, c0, nA, c0B, nb);
    }
    T.fl |= (snp_dev != 0.0f ? TMD_F_SNP : 0u) | (rot_bad ? TMD_F_ROT : 0u) |
            ((pad_or & 0xFFFF0000u) ? TMD_F_PAD : 0u) | ((time_or & ~(kTimeLim - 1u)) ? TMD_F_TIME : 0u);
}

// initial state of track t (header position, time, pad, angles, curvature)
struct TrackInit {
    float x, y, s, tgl, k;
    int32_t t0;
    uint32_t pad0, fl, n, c0, cls, row;
};

__device__ __forceinline__ void track_init(const FrameDesc &F, const Geo *__restrict__ geo, uint32_t t,
                                           TrackInit &I)
{
    const uint32_t ncls = F.ncls[t];
    I.c0 = F.start[t];
    I.n = track_len(I.c0, ncls, F.nA);
    I.cls = key_class(F.tkey[t]);
    I.fl = ncls == 0 ? TMD_F_HDR : 0u;
    const HeaderPos h = header_pos(F.sec0[t], F.row0[t]);
    I.fl |= h.flags;
    I.row = (uint32_t)h.row;
    uint32_t t0u = F.time0[t];
    if (t0u >= kTimeLim) {
        I.fl |= TMD_F_TIME;
        t0u = kTimeLim - 1;
    }
    I.t0 = (int32_t)t0u;
    I.pad0 = F.pad0[t];
    const RowGeo R = geo->row[h.row];
    I.x = R.x;
    I.y = ((float)I.pad0 * 0x1p-5f - R.padoff) * R.pw;
    I.s = clamp_snp((float)F.snp[t] * 0x1p-15f, geo->snp_max, I.fl);
    I.tgl = (float)F.tgl[t] * 0x1p-12f;
    I.k = ((float)F.qpt[t] * 0x1p-10f) * geo->kb;
}

// The TrackInit of window item `src` (0..127), held by lane src in A (items
// 0..63) or by lane src - 64 in B (items 64..127); src may differ per lane.
__device__ __forceinline__ TrackInit track_init_pull(const TrackInit &A, const TrackInit &B, uint32_t src)
{
    const uint32_t l = src & 63u;
    const bool hi = src >= (uint32_t)kWave;
    auto pick = [&](uint32_t a, uint32_t b) -> uint32_t {
        const uint32_t va = bperm(a, l), vb = bperm(b, l);
        return hi ? vb : va;
    };
    auto pickf = [&](float a, float b) -> float { return __uint_as_float(pick(__float_as_uint(a), __float_as_uint(b))); };
    TrackInit R;
    R.x = pickf(A.x, B.x);
    R.y = pickf(A.y, B.y);
    R.s = pickf(A.s, B.s);
    R.tgl = pickf(A.tgl, B.tgl);
    R.k = pickf(A.k, B.k);
    R.t0 = (int32_t)pick((uint32_t)A.t0, (uint32_t)B.t0);
    R.pad0 = pick(A.pad0, B.pad0);
    R.fl = pick(A.fl, B.fl);
    R.n = pick(A.n, B.n);
    R.c0 = pick(A.c0, B.c0);
    R.cls = pick(A.cls, B.cls);
    R.row = pick(A.row, B.row);
    return R;
}

// Tracks per attached-decode wave: up to two per lane.
constexpr uint32_t kMaxWaveTracks = 2 * kWave;

// Lane assignment of one wave.  The wave takes the tracks at schedule
// positions [b0, b1) of its frame (at most 128).  With more than 64 of them,
// the nx = (b1 - b0) - 64 tracks that start last (in the wave's row order)
// are each decoded after another track of the wave, in the same lane: the
// k-th earliest-starting of them follows the track with the k-th earliest
// end.  Matched this way, a lane's second track starts after its first one
// ends whenever any assignment allows it, so the lane's rows stay in step
// with the wave's (the decode stays correct in any case: a lane's clusters
// are always decoded in order).  Packing tracks of different lengths and
// start rows into the lanes this way raises the lanes' use per wave step.
// `S` is LDS scratch of 320 words.
__device__ __forceinline__ void wave_lanes(const FrameDesc &F, const Geo *__restrict__ geo, uint32_t b0,
                                           uint32_t b1, uint32_t *S, int &mode, LaneTrack &T)
{
    const uint32_t lane = lane_id();
    const uint32_t nt = b1 - b0;
    TrackInit I = {}, J = {};
    if (lane < nt) track_init(F, geo, F.order[b0 + lane], I);
    if (kWave + lane < nt) track_init(F, geo, F.order[b0 + kWave + lane], J);
    // wave mode: 0 rows ascending, 1 rows descending, 2 one cluster per step
    {
        const bool not_asc = (I.n > 0 && I.cls != 0) || (J.n > 0 && J.cls != 0);
        const bool not_dsc = (I.n > 0 && I.cls != 1) || (J.n > 0 && J.cls != 1);
        mode = __ballot(not_asc) == 0 ? 0 : (__ballot(not_dsc) == 0 ? 1 : 2);
    }
    if (nt > (uint32_t)kWave) {
        const uint32_t nx = nt - (uint32_t)kWave;
        // start keys (larger: later in the wave's order), made distinct by the
        // item index; rank 0 = the latest start
        auto start_key = [&](const TrackInit &X) -> uint32_t {
            if (X.n == 0) return 0u;
            return mode == 0 ? X.row + 1u : (mode == 1 ? 256u - X.row : 256u - min(X.n, 255u));
        };
        const uint32_t kI = (start_key(I) << 8) | lane, kJ = (start_key(J) << 8) | (kWave + lane);
        uint32_t *key = S, *ek = S + kMaxWaveTracks, *base_src = ek + kWave, *extra_src = base_src + kWave;
        key[lane] = kI;
        key[kWave + lane] = kJ;
        __syncthreads();
        uint32_t rI = 0, rJ = 0;
        for (uint32_t q = 0; q < nt; q++) {
            const uint32_t v = key[q];
            rI += v > kI ? 1u : 0u;
            rJ += v > kJ ? 1u : 0u;
        }
        // base tracks (rank >= nx) go to lanes 0..63 in rank order; extras
        // (rank < nx) are listed by ascending start (nx - 1 - rank)
        if (lane < nt) {
            if (rI >= nx) base_src[rI - nx] = lane;
            else extra_src[nx - 1 - rI] = lane;
        }
        if (kWave + lane < nt) {
            if (rJ >= nx) base_src[rJ - nx] = kWave + lane;
            else extra_src[nx - 1 - rJ] = kWave + lane;
        }
        __syncthreads();
        const TrackInit B = track_init_pull(I, J, base_src[lane]);
        // end keys of the base tracks; lanes ranked by (end, lane)
        uint32_t end_key = 0;
        if (B.n > 0) {
            if (mode == 2) {
                end_key = B.n;
            } else {
                const uint32_t lr = F.recs[B.c0 + B.n - 1].w & 0xFFu;  // row of the last cluster
                end_key = mode == 0 ? lr + 1u : 256u - lr;
            }
        }
        const uint32_t eI = (end_key << 8) | lane;
        ek[lane] = eI;
        __syncthreads();
        uint32_t er = 0;
        for (uint32_t q = 0; q < (uint32_t)kWave; q++) er += ek[q] < eI ? 1u : 0u;
        const TrackInit X = track_init_pull(I, J, er < nx ? extra_src[er] : 0u);
        __syncthreads();  // the scratch is reused by the decode loop
        I = B;
        if (er < nx) {
            if (I.n == 0) {  // a lane without records: the track becomes its own
                const uint32_t fl0 = I.fl;
                I = X;
                I.fl |= fl0;
            } else {
                T.fl |= X.fl;
                if (X.n > 0) {
                    T.nA = I.n;
                    T.c0B = X.c0;
                    T.n = X.n;  // (added below)
                    T.xB = X.x;
                    T.yB = X.y;
                    T.sB = X.s;
                    T.tglB = X.tgl;
                    T.kB = X.k;
                    T.t0B = X.t0;
                    T.pad0B = X.pad0;
                }
            }
        }
    }
    T.x = I.x;
    T.y = I.y;
    T.s = I.s;
    T.tgl = I.tgl;
    T.k = I.k;
    T.t0 = I.t0;
    T.pad0 = I.pad0;
    T.fl |= I.fl;
    T.c0 = I.c0;
    if (T.n > 0) {  // two tracks: n of the second was set above
        T.n += I.n;
    } else {
        T.n = I.n;
        T.nA = I.n;
    }
}

// Waves: a frame's decode uses F.awaves waves; wave fw takes the tracks at
// schedule positions [fw nT / awaves, (fw + 1) nT / awaves), at most 128 (see
// wave_lanes).  The plan chooses awaves from its tracks-per-wave setting and,
// for a single frame, balances the count over the device's SIMDs.  The grid
// has 4 wave slots per 256-track tile of each frame's planned capacity; slot
// fw of frame f is fw = gw - 4 tile0(f), and slots at or beyond the call's
// awaves return at once.  Slots are dealt to the XCDs in contiguous ranges.
// Persistent mode (work != null): the grid is smaller than the slot count and
// each workgroup takes slot after slot of its XCD's range from that XCD's
// counter in `work` (cleared by the tile-sum kernel of the same call) until
// the range is used up.
__global__ __launch_bounds__(kAttWaves * kWave) void k_attached(const FrameDesc *__restrict__ fd,
                                                               const uint32_t *__restrict__ tile_frame,
                                                               const Geo *__restrict__ geo, uint32_t single,
                                                               uint32_t *__restrict__ work, uint32_t slots)
{
    static_assert(kAttWaves == 1, "one wave per workgroup: the wave index is the workgroup index");
    // LDS holds only the record rings and staging (10 KB per wave); the
    // tables stay in global memory.  One-wave workgroups: the grid's waves
    // are all resident at once, and small workgroups let the dispatcher spread
    // them evenly over the CUs.
    __shared__ uint2 ra[kRing][kWave];  // record rings: (output slot, charges)
    __shared__ uint2 rb[kRing][kWave];  // (residuals, row | rotation << 8)
    __shared__ uint2 stg[kBlk][kWave];  // per step of the block: the decoded (time, pad)
    static_assert(sizeof(stg) >= 320 * sizeof(uint32_t), "lane-assignment scratch lives in the staging area");
    const uint32_t lane = lane_id();
    const uint32_t S = single ? fd[0].awaves : slots;  // wave slots in use
    const uint32_t x = blockIdx.x % kXcds;
    const uint32_t per = S / kXcds, extra = S % kXcds;
    const uint32_t first = x * per + (x < extra ? x : extra), count = per + (x < extra ? 1u : 0u);
    for (uint32_t it = blockIdx.x / kXcds;; ) {
        uint32_t gw;
        if (work) {  // persistent: the next slot of this XCD's range
            uint32_t i = 0;
            if (lane == 0) i = atomicAdd(&work[x], 1u);
            i = __builtin_amdgcn_readfirstlane(i);
            if (i >= count) break;
            gw = first + i;
        } else {  // one slot per workgroup
            if (it >= count) break;
            gw = first + it;
        }
        const FrameDesc F = fd[single ? 0u : tile_frame[gw / kTileWaves]];
        const uint32_t fw = gw - F.tile0 * kTileWaves;  // wave of the frame
        if (fw < F.awaves) {  // (slots beyond this call's frame: nothing to do)
            const uint32_t b0 = (uint32_t)((uint64_t)fw * F.nT / F.awaves);
            const uint32_t b1 = (uint32_t)((uint64_t)(fw + 1) * F.nT / F.awaves);
            int mode = 0;
            LaneTrack T = {};
            wave_lanes(F, geo, b0, b1, reinterpret_cast<uint32_t *>(&stg[0][0]), mode, T);
            if (mode == 0) attached_loop<0>(F, geo, ra, rb, stg, T);
            else if (mode == 1) attached_loop<1>(F, geo, ra, rb, stg, T);
            else attached_loop<2>(F, geo, ra, rb, stg, T);
            const uint32_t fl = wave_or(T.fl);
            if (lane == 0 && fl) atomicOr(F.status, fl);
        }
        if (!work) break;
        __syncthreads();  // the LDS of this item is done before the next one's
    }
}

// ---------------------------------------------------------------------------
// arithmetic self-test
// ---------------------------------------------------------------------------
__global__ void k_selftest_math(const float *a, float smax, uint32_t *out, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = a[i];
    bool f = false;
    const float c = clamp_snp_b(x, smax, f);
    out[4 * i + 0] = __float_as_uint(sqrt_pos(x));
    out[4 * i + 1] = __float_as_uint(c);
    out[4 * i + 2] = f ? 1u : 0u;
    out[4 * i + 3] = (uint32_t)sat_rint(x);
}

// count the floats with bit patterns in [lo, hi) where sqrt_pos differs from
// the IEEE square root
__global__ void k_selftest_sqrt(uint32_t lo, uint32_t hi, uint32_t *count)
{
    uint32_t bad = 0;
    for (uint64_t b = (uint64_t)lo + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < hi;
         b += (uint64_t)gridDim.x * blockDim.x) {
        const float x = __uint_as_float((uint32_t)b);
        bad += __float_as_uint(sqrt_pos(x)) != __float_as_uint(sqrtf(x));
    }
    bad = wave_incl_add(bad);
    if (lane_id() == kWave - 1 && bad) atomicAdd(count, bad);
}

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
// Encoder: the inverse of the decode (section 4: attached clusters are stored
// as residuals to their track's extrapolation, unattached clusters sorted by
// position within their region and stored as differences to the previous
// one).  Input: clusters in physical units (pad and time as doubles, grouped
// by track) and track parameters; output: a compressed frame for tmd_decode.
//
//   E0 k_enc_pack     one lane per cluster: quantise, check the range, pack
//                     the cluster into an 8-byte record
//   E1 k_enc_tracks   one lane per track, over the records: run the same
//                     float32 model as the decode, store packed residuals;
//                     open a new header where the model cannot follow (row
//                     step beyond int8, side change, 255 clusters, a clamp, a
//                     residual beyond int16)
//   E2 k_enc_scan_*   unpack the residuals and copy the charges (one lane per
//                     cluster); header clusters -> header indices (block
//                     sums, prefix)
//   E3 k_enc_headers  header arrays and cluster counts
//   U1 k_enc_un_keys  unattached: quantise, sort keys
//   U2 k_rad_*        stable LSD radix sort by (bin, time, pad), 8 passes of
//                     8 bits; runs of equal keys then sorted by (qTot, qMax),
//                     or, for a run of more than 64, the full 12-pass sort
//   U3 k_enc_un_delta differences to the predecessor within the bin; bin
//                     counts from where the sorted bins begin and end
// ---------------------------------------------------------------------------
struct EncDesc {
    // input
    uint32_t nT, n, nU;
    const GLB uint32_t *first;  // [nT + 1]
    const GLB double *qpt, *tgl;
    const GLB uint8_t *sec, *row;
    const GLB double *pad, *time, *snp;
    const GLB uint16_t *qtot, *qmax;
    const GLB uint8_t *usec, *urow;
    const GLB double *upad, *utime;
    const GLB uint16_t *uqtot, *uqmax;
    // output
    GLB uint8_t *ncls, *sec0, *row0;
    GLB uint16_t *pad0;
    GLB uint32_t *time0;
    GLB int16_t *oqpt, *osnp, *otgl;
    GLB int8_t *rdiff;
    GLB uint8_t *sdiff;
    GLB int16_t *pres, *tres;
    GLB uint16_t *cqtot, *cqmax;
    GLB uint32_t *ucount, *utdiff;
    GLB uint16_t *updiff, *uoqtot, *uoqmax;
    GLB uint32_t *counts;  // [0] headers, [1] splits, [2] input errors
    // workspace
    GLB uint8_t *hn;     // [n] clusters of the header opened at cluster c, else 0
    GLB unsigned long long *rec;  // [n] per cluster: the packed input (k_enc_pack), then the packed
                                  // output of the track walk (k_enc_tracks), in place
    GLB uint32_t *htrk;  // [n] track of the header opened at cluster c
    GLB uint32_t *bsum;  // [ceil(n / 1024) + 1] headers per block of clusters, then their prefix
    GLB unsigned long long *k0, *k1;  // [nU] sort keys (ping-pong)
    GLB uint32_t *v0, *v1;            // [nU] sort payloads (qTot << 16 | qMax)
    GLB uint32_t *rhist;              // [256 * rblocks + 256] radix histograms, digit-major (digit d of
                                      // tile b at d * rblocks + b), then offsets; the digit totals last
    GLB uint32_t *rflag;  // [1] set when a run of equal keys is too long to sort in place
    uint32_t rblocks;
};

constexpr uint32_t kEncErrInput = 1u;  // counts[2]: a cluster outside the codable range
constexpr int kRadTile = 4096;         // radix sort: elements per block (4 waves x 16 chunks of 64)

__device__ __forceinline__ int16_t enc_q16(double v, double scale)
{
    double q = __builtin_rint(v * scale);
    q = q > 32767.0 ? 32767.0 : q;
    q = q < -32767.0 ? -32767.0 : q;
    return (int16_t)q;
}

struct EncState {
    float x, y, z, s, tgl, k;
    int sec, row;
    int32_t t0;
};

__device__ __forceinline__ void enc_init(const Geo *__restrict__ g, EncState &st, int sec0, int row0, uint32_t pad0, uint32_t time0,
                         int16_t qptq, int16_t snpq, int16_t tglq, uint32_t &fl)
{
    if (sec0 >= NSEC) { fl |= TMD_F_HDR; sec0 = sec0 % NSEC; }
    if (row0 >= NROW) { fl |= TMD_F_HDR; row0 = NROW - 1; }
    uint32_t t0 = time0;
    if (t0 >= kTimeLim) { fl |= TMD_F_TIME; t0 = kTimeLim - 1; }
    const RowGeo &R = g->row[row0];
    st.sec = sec0;
    st.row = row0;
    st.t0 = (int32_t)t0;
    st.x = R.x;
    st.y = ((float)pad0 * 0x1p-5f - R.padoff) * R.pw;
    st.z = 0.0f;
    st.s = clamp_snp((float)snpq * 0x1p-15f, g->snp_max, fl);
    st.tgl = (float)tglq * 0x1p-12f;
    st.k = ((float)qptq * 0x1p-10f) * g->kb;
}

// the decode's step (rotation, row step, helix propagation, predicted codes)
__device__ __forceinline__ void enc_predict(const Geo *__restrict__ g, EncState &st, uint32_t sd, int rd, int32_t &P, int32_t &T,
                            uint32_t &fl)
{
    uint32_t d = sd;
    if (d >= 18) { fl |= TMD_F_SEC; d %= 18; }
    if (d != 0) {
        const float ca = g->cosb[d], sa = g->sinb[d];
        const float cs = sqrtf((1.0f - st.s) * (1.0f + st.s));
        const float xn = (st.x * ca) + (st.y * sa);
        const float yn = (st.y * ca) - (st.x * sa);
        const float sn = (st.s * ca) - (cs * sa);
        const float cn = (cs * ca) + (st.s * sa);
        if (!(cn > 0.0f)) fl |= TMD_F_ROT;
        st.x = xn;
        st.y = yn;
        st.s = clamp_snp(sn, g->snp_max, fl);
        st.sec = (st.sec / 18) * 18 + (st.sec % 18 + (int)d) % 18;
    }
    int row = st.row + rd;
    if (row < 0) { fl |= TMD_F_ROW; row = 0; }
    if (row >= NROW) { fl |= TMD_F_ROW; row = NROW - 1; }
    st.row = row;
    const RowGeo &R = g->row[row];
    const float dx = R.x - st.x;
    const float s1 = clamp_snp(st.s + (st.k * dx), g->snp_max, fl);
    const float a0 = sqrtf((1.0f - st.s) * (1.0f + st.s));
    const float a1 = sqrtf((1.0f - s1) * (1.0f + s1));
    const float dydx = (st.s + s1) / (a0 + a1);
    st.y = st.y + (dx * dydx);
    st.z = st.z + (st.tgl * (dx * sqrtf(1.0f + (dydx * dydx))));
    st.s = s1;
    st.x = R.x;
    P = sat_rint(((st.y * R.inv_pw) + R.padoff) * 32.0f);
    T = sat_rint(st.z * g->inv_vd32);
}

__device__ __forceinline__ void enc_update(const Geo *__restrict__ g, EncState &st, int32_t pres, int32_t tres, uint32_t &fl)
{
    const RowGeo &R = g->row[st.row];
    const float nuy = (float)pres * R.pwq;
    const float nuz = (float)tres * g->vdq;
    st.y = st.y + nuy;
    st.z = st.z + nuz;
    st.s = clamp_snp(st.s + (nuy * R.ks), g->snp_max, fl);
    st.tgl = st.tgl + (nuz * R.kt);
}

// Packed records of the track walk.  In: pad code (16 bits), time code (24),
// row (8), sector (8).  Out: row step (8), sector step (8), pad residual
// (16), time residual (16), and bit 48 set where a header opens.
constexpr int kRecTime = 16, kRecRow = 40, kRecSec = 48, kRecOpen = 48;

// E0: one lane per cluster: quantise (rint of 32 x pad and time, in double),
// check the codable range, pack
__global__ __launch_bounds__(256) void k_enc_pack(const EncDesc E)
{
    const uint32_t c = blockIdx.x * 256 + threadIdx.x;
    if (c >= E.n) return;
    const double pq = __builtin_rint(E.pad[c] * 32.0), tq = __builtin_rint(E.time[c] * 32.0);
    unsigned long long r = 0;
    if (pq >= 0.0 && pq <= 65535.0 && tq >= 0.0 && tq < (double)kTimeLim) {
        r = (unsigned long long)(uint32_t)pq | ((unsigned long long)(uint32_t)tq << kRecTime) |
            ((unsigned long long)E.row[c] << kRecRow) | ((unsigned long long)E.sec[c] << kRecSec);
    } else {
        atomicOr(&E.counts[2], kEncErrInput);
    }
    E.rec[c] = r;
}

// E1: one lane per track, over the packed records.  A wave's 64 tracks are
// walked kEncSeg steps at a time: the next kEncSeg records of every lane's
// track are staged in LDS by loads that take 16 consecutive records per 16
// lanes, the lanes step through them there and leave their output records in
// the same slots, and the slots are written back the same way.
constexpr uint32_t kEncSeg = 16;

__global__ __launch_bounds__(256) void k_enc_tracks(const EncDesc E, const Geo *__restrict__ g)
{
    // [wave][lane][slot]; 17 slots per lane keep 16 lanes' reads of one slot
    // on distinct banks
    __shared__ unsigned long long ring[4][kWave][kEncSeg + 1];
    __shared__ uint32_t ta[4][kWave], te[4][kWave];
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    const uint32_t it = blockIdx.x * 256 + threadIdx.x;
    if (it == 0 && (E.first[0] != 0 || E.first[E.nT] != E.n)) atomicOr(&E.counts[2], kEncErrInput);
    uint32_t a = 0, e = 0;
    int16_t qptq = 0, tglq = 0;
    if (it < E.nT) {
        a = E.first[it];
        e = E.first[it + 1];
        if (a > e || e > E.n) {
            atomicOr(&E.counts[2], kEncErrInput);
            a = e = 0;
        }
        qptq = enc_q16(E.qpt[it], 1024.0);
        tglq = enc_q16(E.tgl[it], 4096.0);
    }
    ta[w][lane] = a;
    te[w][lane] = e;
    const uint32_t maxlen = wave_max_u32(e - a);
    uint32_t hdr = a, hcount = 0, splits = 0;
    EncState st = {};
    uint32_t prow = 0, psec = 0;  // the previous cluster's row and sector
    const uint32_t sk = lane % kEncSeg, sq = lane / kEncSeg;
    for (uint32_t j0 = 0; j0 < maxlen; j0 += kEncSeg) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
        for (uint32_t r = 0; r < kWave / 4; r++) {
            const uint32_t sl = 4 * r + sq, cc = ta[w][sl] + j0 + sk;
            if (cc < te[w][sl]) ring[w][sl][sk] = E.rec[cc];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t jj = 0; jj < kEncSeg; jj++) {
            const uint32_t c = a + j0 + jj;
            if (c >= e) break;
            const unsigned long long in = ring[w][lane][jj];
            const uint32_t crow = (uint32_t)(in >> kRecRow) & 0xFFu, csec = (uint32_t)(in >> kRecSec) & 0xFFu;
            const int32_t padq = (int32_t)(in & 0xFFFFu), timeq = (int32_t)((in >> kRecTime) & 0xFFFFFFu);
            bool open_new = c == a;
            int32_t rd = 0, sd = 0, pr = 0, tr = 0;
            if (!open_new) {
                const int drow = (int)crow - (int)prow;
                const bool same_side = (csec / 18) == (psec / 18);
                if (drow < -128 || drow > 127 || !same_side || hcount == 255) {
                    open_new = true;
                } else {
                    rd = drow;
                    sd = ((int)(csec % 18) - (int)(psec % 18) + 18) % 18;
                    EncState trial = st;
                    uint32_t fl = 0;
                    int32_t P, T;
                    enc_predict(g, trial, (uint32_t)sd, rd, P, T, fl);
                    const int64_t p64 = (int64_t)padq - P;
                    const int64_t t64 = (int64_t)timeq - trial.t0 - T;
                    if (fl || p64 < -32768 || p64 > 32767 || t64 < -32768 || t64 > 32767 || trial.sec != (int)csec ||
                        trial.row != (int)crow) {
                        open_new = true;
                    } else {
                        pr = (int32_t)p64;
                        tr = (int32_t)t64;
                        enc_update(g, trial, pr, tr, fl);
                        if (fl) open_new = true;
                        else st = trial;
                    }
                }
            }
            if (open_new) {
                if (c != a) {
                    splits++;
                    E.hn[hdr] = (uint8_t)hcount;
                }
                hdr = c;
                hcount = 1;
                E.htrk[c] = it;
                uint32_t fl = 0;
                enc_init(g, st, (int)csec, (int)crow, (uint32_t)padq, (uint32_t)timeq, qptq,
                         enc_q16(E.snp[c], 32768.0), tglq, fl);
                rd = sd = pr = tr = 0;
            } else {
                hcount++;
            }
            ring[w][lane][jj] = (unsigned long long)(uint8_t)rd | ((unsigned long long)(uint8_t)sd << 8) |
                                ((unsigned long long)(uint16_t)pr << 16) | ((unsigned long long)(uint16_t)tr << 32) |
                                ((unsigned long long)(open_new ? 1u : 0u) << kRecOpen);
            prow = crow;
            psec = csec;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
        for (uint32_t r = 0; r < kWave / 4; r++) {
            const uint32_t sl = 4 * r + sq, cc = ta[w][sl] + j0 + sk;
            if (cc < te[w][sl]) E.rec[cc] = ring[w][sl][sk];
        }
    }
    if (e > a) E.hn[hdr] = (uint8_t)hcount;
    if (splits) atomicAdd(&E.counts[1], splits);
}

// E2: headers per block of 1024 clusters; the track walk's records are
// unpacked into the cluster arrays (hn of a cluster that opens no header set
// to 0) and the charges copied, in cluster order
__global__ __launch_bounds__(256) void k_enc_scan_blocks(const EncDesc E)
{
    uint32_t h = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t c = blockIdx.x * 1024 + q * 256 + threadIdx.x;
        if (c < E.n) {
            const unsigned long long r = E.rec[c];
            const uint32_t open = (uint32_t)(r >> kRecOpen) & 1u;
            h += open;
            if (!open) E.hn[c] = 0;
            E.rdiff[c] = (int8_t)(r & 0xFFu);
            E.sdiff[c] = (uint8_t)((r >> 8) & 0xFFu);
            E.pres[c] = (int16_t)(uint16_t)((r >> 16) & 0xFFFFu);
            E.tres[c] = (int16_t)(uint16_t)((r >> 32) & 0xFFFFu);
            E.cqtot[c] = E.qtot[c];
            E.cqmax[c] = E.qmax[c];
        }
    }
    uint32_t tot;
    block_excl_add(h, &tot);
    if (threadIdx.x == 0) E.bsum[blockIdx.x] = tot;
}

// E2: exclusive prefix of the block counts (one block); the total -> counts[0]
__global__ __launch_bounds__(1024) void k_enc_scan_prefix(const EncDesc E, uint32_t nb)
{
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? E.bsum[b] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_add<16>(v, &tot);
        const uint32_t base = carry;
        if (b < nb) E.bsum[b] = base + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = base + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) E.counts[0] = carry;
}

// E3: header arrays at their indices
__global__ __launch_bounds__(256) void k_enc_headers(const EncDesc E)
{
    const uint32_t c0 = blockIdx.x * 1024 + threadIdx.x * 4;
    uint32_t h[4], cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        h[q] = (c0 + q < E.n) ? E.hn[c0 + q] : 0u;
        cnt += h[q] ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t idx = E.bsum[blockIdx.x] + block_excl_add(cnt, &tot);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (!h[q]) continue;
        const uint32_t c = c0 + q, t = E.htrk[c];
        E.ncls[idx] = (uint8_t)h[q];
        E.sec0[idx] = E.sec[c];
        E.row0[idx] = E.row[c];
        E.pad0[idx] = (uint16_t)__builtin_rint(E.pad[c] * 32.0);
        E.time0[idx] = (uint32_t)__builtin_rint(E.time[c] * 32.0);
        E.oqpt[idx] = enc_q16(E.qpt[t], 1024.0);
        E.osnp[idx] = enc_q16(E.snp[c], 32768.0);
        E.otgl[idx] = enc_q16(E.tgl[t], 4096.0);
        idx++;
    }
}

// U1: quantise unattached clusters, build sort keys
// (bin << 48 | time << 16 | pad) and payloads (qTot << 16 | qMax)
__global__ __launch_bounds__(256) void k_enc_un_keys(const EncDesc E)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= E.nU) return;
    const double pq = __builtin_rint(E.upad[i] * 32.0), tq = __builtin_rint(E.utime[i] * 32.0);
    const uint32_t sec = E.usec[i], row = E.urow[i];
    if (!(pq >= 0.0 && pq <= 65535.0 && tq >= 0.0 && tq <= 4294967295.0) || sec >= NSEC || row >= NROW) {
        atomicOr(&E.counts[2], kEncErrInput);
        E.k0[i] = 0;
        E.v0[i] = 0;
        return;
    }
    const uint64_t bin = sec * NROW + row;
    E.k0[i] = (bin << 48) | ((uint64_t)(uint32_t)tq << 16) | (uint64_t)(uint32_t)pq;
    E.v0[i] = ((uint32_t)E.uqtot[i] << 16) | E.uqmax[i];
}

__global__ __launch_bounds__(256) void k_enc_clear(const EncDesc E)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < NBIN) E.ucount[i] = 0;
    if (i < 3) E.counts[i] = 0;
    if (i == 0) E.rflag[0] = 0;
}

// U2: one pass of a stable LSD radix sort on 8-bit digit `shift` of the key
// (key_pass) or of the payload.  Blocks own tiles of kRadTile elements in
// order; within a tile, wave w owns elements [1024 w, 1024 w + 1024).
// The order wanted is (key, payload).  The key's 8 passes run first; then
// k_rad_fix sorts each run of equal keys by payload (equal keys are rare:
// clusters at one position of one bin).  A run longer than kFixRun sets a flag
// instead, and the full sort follows on the result (4 payload passes, then the
// key's 8): its kernels are always enqueued, as `gated` passes that return at
// once unless the flag is set.
__device__ __forceinline__ uint32_t rad_digit(bool key_pass, unsigned long long k, uint32_t v, uint32_t shift)
{
    return key_pass ? (uint32_t)(k >> shift) & 0xFFu : (v >> shift) & 0xFFu;
}

// (kernel parameters are plain pointers, cast to the global address space
// inside: a qualified parameter type would give the kernel a different symbol
// in the device and host compilations)
__global__ __launch_bounds__(256) void k_rad_hist(const EncDesc E, const unsigned long long *kin_,
                                                  const uint32_t *vin_, uint32_t key_pass, uint32_t shift,
                                                  uint32_t gated)
{
    if (gated && E.rflag[0] == 0) return;
    const GLB unsigned long long *kin = (const GLB unsigned long long *)kin_;
    const GLB uint32_t *vin = (const GLB uint32_t *)vin_;
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kRadTile;
    for (uint32_t q = threadIdx.x; q < (uint32_t)kRadTile; q += 256) {
        const uint32_t i = base + q;
        if (i < E.nU) atomicAdd(&cnt[key_pass ? (uint32_t)(kin[i] >> shift) & 0xFFu : (vin[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    E.rhist[(size_t)threadIdx.x * E.rblocks + blockIdx.x] = cnt[threadIdx.x];
}

// one block per digit d: its counts over the tiles -> their exclusive prefix
// (in place, 256 tiles per round); the digit's total after all histograms.
// The scatter adds the totals of the digits below its own.
__global__ __launch_bounds__(256) void k_rad_offsets(const EncDesc E, uint32_t gated)
{
    if (gated && E.rflag[0] == 0) return;
    const uint32_t d = blockIdx.x, nb = E.rblocks;
    GLB uint32_t *col = E.rhist + (size_t)d * nb;
    uint32_t base = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += 256) {
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? col[b] : 0u;
        uint32_t all;
        const uint32_t ex = block_excl_add(v, &all);
        if (b < nb) col[b] = base + ex;
        base += all;
    }
    if (threadIdx.x == 0) E.rhist[(size_t)256 * nb + d] = base;
}

// The tile is ranked in LDS first: each element's place in the tile sorted
// by digit (stable), then the sorted tile is written out, so that every
// digit's elements go to consecutive addresses.  The tile's elements are read
// once, into registers.
__global__ __launch_bounds__(256) void k_rad_scatter(const EncDesc E, const unsigned long long *kin_,
                                                     const uint32_t *vin_, unsigned long long *kout_,
                                                     uint32_t *vout_, uint32_t key_pass, uint32_t shift,
                                                     uint32_t gated)
{
    if (gated && E.rflag[0] == 0) return;
    const GLB unsigned long long *kin = (const GLB unsigned long long *)kin_;
    const GLB uint32_t *vin = (const GLB uint32_t *)vin_;
    GLB unsigned long long *kout = (GLB unsigned long long *)kout_;
    GLB uint32_t *vout = (GLB uint32_t *)vout_;
    __shared__ uint32_t wcnt[4][256];  // per wave: digit counts, then running places in the sorted tile
    __shared__ uint32_t gdst[256];     // per digit: output index of the sorted tile's place 0
    __shared__ unsigned long long sk[kRadTile];
    __shared__ uint32_t sv[kRadTile];
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    for (uint32_t q = threadIdx.x; q < 4 * 256; q += 256) (&wcnt[0][0])[q] = 0;
    __syncthreads();
    const uint32_t t0 = blockIdx.x * kRadTile, base = t0 + w * 1024;
    unsigned long long kr[16];
    uint32_t vr[16];
#pragma unroll
    for (int ch = 0; ch < 16; ch++) {
        const uint32_t i = base + ch * kWave + lane;
        kr[ch] = 0;
        vr[ch] = 0;
        if (i < E.nU) {
            kr[ch] = kin[i];
            vr[ch] = vin[i];
        }
    }
#pragma unroll
    for (int ch = 0; ch < 16; ch++) {
        const uint32_t i = base + ch * kWave + lane;
        if (i < E.nU) atomicAdd(&wcnt[w][rad_digit(key_pass, kr[ch], vr[ch], shift)], 1u);
    }
    __syncthreads();
    {
        const uint32_t d = threadIdx.x;
        uint32_t c[4], tile = 0;
#pragma unroll
        for (int ww = 0; ww < 4; ww++) {
            c[ww] = wcnt[ww][d];
            tile += c[ww];
        }
        uint32_t all;
        const uint32_t loc = block_excl_add(tile, &all);  // digit d's first place in the sorted tile
        uint32_t run = loc;
#pragma unroll
        for (int ww = 0; ww < 4; ww++) {
            wcnt[ww][d] = run;
            run += c[ww];
        }
        const uint32_t gstart = block_excl_add(E.rhist[(size_t)256 * E.rblocks + d], &all) +
                                E.rhist[(size_t)d * E.rblocks + blockIdx.x];
        gdst[d] = gstart - loc;
    }
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int ch = 0; ch < 16; ch++) {
        const bool act = base + ch * kWave + lane < E.nU;
        const uint32_t dg = act ? rad_digit(key_pass, kr[ch], vr[ch], shift) : 0u;
        uint64_t same = __ballot(act);
#pragma unroll
        for (int bit = 0; bit < 8; bit++) {
            const uint64_t m = __ballot(act && ((dg >> bit) & 1u));
            same &= ((dg >> bit) & 1u) ? m : ~m;
        }
        if (act) {
            const uint32_t pos = wcnt[w][dg] + (uint32_t)__popcll(same & below);
            sk[pos] = kr[ch];
            sv[pos] = vr[ch];
        }
        __builtin_amdgcn_wave_barrier();
        // the last lane of each digit group moves that digit's place on
        if (act && (same & ~below & ~(1ull << lane)) == 0) wcnt[w][dg] += (uint32_t)__popcll(same);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const uint32_t nt = E.nU - t0 < (uint32_t)kRadTile ? E.nU - t0 : (uint32_t)kRadTile;
    for (uint32_t q = threadIdx.x; q < nt; q += 256) {
        const unsigned long long k = sk[q];
        const uint32_t v = sv[q];
        const uint32_t o = gdst[rad_digit(key_pass, k, v, shift)] + q;
        kout[o] = k;
        vout[o] = v;
    }
}

// after the key passes: the lane of the first element of a run of equal keys
// sorts the run's payloads (insertion sort; the keys are all the same), or
// sets the flag if the run is longer than kFixRun
constexpr uint32_t kFixRun = 64;

__global__ __launch_bounds__(256) void k_rad_fix(const EncDesc E, const unsigned long long *ks_, uint32_t *vs_)
{
    const GLB unsigned long long *ks = (const GLB unsigned long long *)ks_;
    GLB uint32_t *vs = (GLB uint32_t *)vs_;
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i + 1 >= E.nU) return;
    const unsigned long long k = ks[i];
    if (ks[i + 1] != k || (i > 0 && ks[i - 1] == k)) return;
    uint32_t j = i + 2;
    while (j < E.nU && j - i <= kFixRun && ks[j] == k) j++;
    if (j - i > kFixRun) {
        E.rflag[0] = 1u;
        return;
    }
    for (uint32_t a = i + 1; a < j; a++) {
        const uint32_t v = vs[a];
        uint32_t b = a;
        while (b > i && vs[b - 1] > v) {
            vs[b] = vs[b - 1];
            b--;
        }
        vs[b] = v;
    }
}

// U3: differences to the predecessor in the same bin (the first against zero);
// a bin's count is the distance from its first element to past its last
__global__ __launch_bounds__(256) void k_enc_un_delta(const EncDesc E, const unsigned long long *ks_,
                                                      const uint32_t *vs_)
{
    const GLB unsigned long long *ks = (const GLB unsigned long long *)ks_;
    const GLB uint32_t *vs = (const GLB uint32_t *)vs_;
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= E.nU) return;
    const unsigned long long k = ks[i];
    const uint32_t bin = (uint32_t)(k >> 48);
    uint32_t pt = 0, pp = 0;
    bool first = true;
    if (i > 0) {
        const unsigned long long kp = ks[i - 1];
        if ((kp >> 48) == bin) {
            pt = (uint32_t)(kp >> 16);
            pp = (uint32_t)kp & 0xFFFFu;
            first = false;
        }
    }
    if (first) atomicSub(&E.ucount[bin], i);
    if (i + 1 == E.nU || (uint32_t)(ks[i + 1] >> 48) != bin) atomicAdd(&E.ucount[bin], i + 1);
    const uint32_t v = vs[i];
    E.utdiff[i] = (uint32_t)(k >> 16) - pt;
    E.updiff[i] = (uint16_t)(((uint32_t)k & 0xFFFFu) - pp);
    E.uoqtot[i] = (uint16_t)(v >> 16);
    E.uoqmax[i] = (uint16_t)(v & 0xFFFFu);
}

// ---------------------------------------------------------------------------
// Entropy-coded frames (the step before the track-model decode; section 4 and
// the paper's introduction: the compressed time frame is ANS-coded).  The
// coded format is this project's, laid out in include/tmd.h: the 19 arrays of
// a frame in 39 byte planes, each plane a static 12-bit model and chunks of
// 64 rANS lanes that share one stream of 16-bit words.
//   k_rans_prep: one block per plane builds its decode tables (the symbol of
//     every 12-bit slot; each symbol's frequency and start) and finds where
//     its chunks' data begins.
//   k_rans<W, 0>: workgroups of kRansWaves waves, one wave per chunk of an
//     array of W-byte elements (the track and attached-cluster arrays and
//     the bin counts, before the track-model decode); the waves of a
//     workgroup take consecutive chunks of one array and share its planes'
//     tables.  Lane l runs lane l
//     of the W planes side by side (W independent state chains), so every
//     step yields whole elements; planes of a single symbol (f = 2^12) need
//     no decoding.  A step's words are consecutive in the chunk's stream
//     (lanes in order), so the stream is read ahead one block of steps early,
//     with one-dword-per-lane loads into an LDS ring per plane; the decoded
//     elements of a block are staged in LDS and written out whole.  Global
//     memory is touched only between blocks.
//   k_rans<W, 1>: the same decoding for the four arrays of unattached
//     clusters, run once the output offsets are known (in place of
//     k_unattached, on a second stream beside k_rank and k_attached): each
//     element goes straight to its output slot, time and pad differences as
//     running sums within their bin.  A chunk's sums start at 0, so
//     k_rans_unfix then adds to a chunk's leading elements the sum of their
//     bin's elements in the chunks before (from a record per chunk).
// ---------------------------------------------------------------------------
constexpr int kRansPlanes = 39, kRansArrays = 19, kRansLanes = 64, kRansPerLane = 512;
constexpr uint32_t kRansChunk = kRansLanes * kRansPerLane;
constexpr uint32_t kRansLow = 1u << 16;
constexpr uint32_t kRansHdr = 64;
constexpr uint32_t kRansVersion = 2;
constexpr uint32_t kRansBad = TMD_F_CODED;
constexpr uint32_t kRansUnit = 128;              // words per read-ahead load (a dword per lane)
constexpr uint32_t kRansTab = 4096 + 4 * 256;    // bytes of a plane's decode tables
constexpr uint32_t kRansWaves = 4;               // waves (chunks) per workgroup of k_rans
// steps per block (a lane's elements per block), and words of a plane's ring,
// for W-byte elements (4-byte ones take shorter blocks and rings: less LDS)
constexpr uint32_t rans_blk(int W) { return W == 4 ? 2 : 4; }
constexpr uint32_t rans_ring(int W) { return W == 4 ? 512 : 1024; }
// (a block reads fewer than kRansLanes blk words; the read-ahead keeps
// 2 kRansLanes blk words ahead and lands whole units)
static_assert(2 * kRansLanes * rans_blk(1) + kRansUnit <= rans_ring(1) &&
                  2 * kRansLanes * rans_blk(2) + kRansUnit <= rans_ring(2) &&
                  2 * kRansLanes * rans_blk(4) + kRansUnit <= rans_ring(4),
              "the ring holds what is read ahead");

__device__ __constant__ const uint8_t kRansWidth[kRansArrays] = {1, 1, 1, 2, 4, 2, 2, 2, 1, 1, 2, 2, 2, 2, 4, 4, 2, 2, 2};
// first plane of each array
__device__ __constant__ const uint8_t kRansPlane0[kRansArrays] = {0,  1,  2,  3,  5,  9,  11, 13, 15, 16,
                                                                  17, 19, 21, 23, 25, 29, 33, 35, 37};

// The arrays of unattached clusters (time and pad differences, charges),
// decoded straight into the output by k_rans<W, kRansUnPhase>
constexpr uint32_t kRansUn0 = 15;
// Work lists (phases) of the entropy decoding: 0, the track and attached
// arrays and the bin counts (before the track-model decode); 1, the
// unattached arrays (into the output, once the decode's offsets are known).
// (Decoding the arrays that only k_rank and k_attached read beside the
// decode's first kernels instead saved nothing: those kernels and the
// entropy decoding both need the vector ALUs.)
constexpr int kRansPhases = 2, kRansUnPhase = 1;
constexpr int rans_phase(int a) { return a >= (int)kRansUn0 ? 1 : 0; }

struct RansDesc {  // (the same layout on the host and the device: 920 bytes)
    const GLB uint8_t *src;       // the coded frame (16-byte aligned)
    uint64_t size;
    GLB uint8_t *dst[kRansArrays];
    uint32_t n[kRansArrays];      // elements of each array
    GLB uint8_t *tabs;            // per plane kRansTab bytes: sym[4096], then f | c << 16 for each symbol
    GLB uint64_t *pinfo;          // per plane: its position, the start of its chunks' data (0: unusable)
    GLB uint32_t *err;            // TMD_F_CODED if the data is not a well-formed coded frame
    GLB uint4 *urec;              // [2][chunks of nU]: time's, then pad's chunk records (k_rans_unfix)
    uint32_t nT, nA, nU;
    // work lists: per phase and width class (1, 2, 4 bytes) the arrays
    uint32_t nw[kRansPhases][3];
    uint32_t warr[kRansPhases][3][12];
    uint32_t witem0[kRansPhases][3][13];  // first work item of each, then the total
};

static_assert(sizeof(RansDesc) == 920, "descriptor layout");

__global__ void k_fill32(uint32_t *p, uint32_t n, uint32_t v)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

__device__ __forceinline__ uint32_t rans_rd32(const GLB uint8_t *s, uint64_t o)
{
    return (uint32_t)s[o] | ((uint32_t)s[o + 1] << 8) | ((uint32_t)s[o + 2] << 16) | ((uint32_t)s[o + 3] << 24);
}

// (the descriptors of all frames of a call: device memory, one per frame)
__global__ __launch_bounds__(256) void k_rans_prep(const RansDesc *descs)
{
    __shared__ uint32_t cend[256];  // c_s + f_s
    __shared__ uint32_t wsum[4];
    const uint32_t p = blockIdx.x % kRansPlanes, t = threadIdx.x;
    const GLB RansDesc *R = (const GLB RansDesc *)descs + blockIdx.x / kRansPlanes;
    uint32_t a = 0;
    while (a + 1 < (uint32_t)kRansArrays && kRansPlane0[a + 1] <= p) a++;
    const uint64_t n = R->n[a];
    const uint64_t nch = (n + kRansChunk - 1) / kRansChunk;
    bool ok = R->size >= kRansHdr + 8 * kRansPlanes;
    if (p == 0 && t == 0) {  // the header: "TMDR", version 2, the frame's shape
        bool hok = ok && R->src[0] == 'T' && R->src[1] == 'M' && R->src[2] == 'D' && R->src[3] == 'R' &&
                   rans_rd32(R->src, 4) == kRansVersion && rans_rd32(R->src, 8) == R->nT &&
                   rans_rd32(R->src, 12) == R->nA && rans_rd32(R->src, 16) == R->nU;
        if (!hok) atomicOr(R->err, kRansBad);
    }
    uint64_t pos = 0;
    if (ok) pos = (uint64_t)rans_rd32(R->src, kRansHdr + 8 * p) | ((uint64_t)rans_rd32(R->src, kRansHdr + 8 * p + 4) << 32);
    ok = ok && pos <= R->size && R->size - pos >= 512 + 4 * (nch + 1);
    const uint32_t f = ok ? (uint32_t)R->src[pos + 2 * t] | ((uint32_t)R->src[pos + 2 * t + 1] << 8) : 0u;
    // exclusive prefix of the frequencies over the block's 4 waves
    const uint32_t inc = wave_incl_add(f);
    if (lane_id() == kWave - 1) wsum[t / kWave] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (uint32_t q = 0; q < 4; q++) {
        base += q < t / kWave ? wsum[q] : 0u;
        tot += wsum[q];
    }
    const uint32_t c = base + inc - f;
    cend[t] = c + f;
    if (n && tot != 4096u) ok = false;
    GLB uint8_t *tab = R->tabs + (uint64_t)p * kRansTab;
    ((GLB uint32_t *)(tab + 4096))[t] = f | (c << 16);
    __syncthreads();
    // the symbol of slots 16t .. 16t + 15: the number of symbols whose range
    // ends at or below the slot
    uint32_t slot = 16 * t, lo = 0, hi = 256;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cend[mid] <= slot) lo = mid + 1;
        else hi = mid;
    }
    uint32_t s = lo, wv[4];
    for (int q = 0; q < 16; q++, slot++) {
        while (s < 255 && cend[s] <= slot) s++;
        if (q % 4 == 0) wv[q / 4] = 0;
        wv[q / 4] |= min(s, 255u) << (8 * (q % 4));  // (256 only in a model that does not sum to 2^12)
    }
    *(GLB uint4 *)(tab + 16 * t) = make_uint4(wv[0], wv[1], wv[2], wv[3]);
    if (t == 0) {
        R->pinfo[2 * p] = pos;
        R->pinfo[2 * p + 1] = ok ? ((pos + 512 + 4 * (nch + 1) + 15) & ~15ull) : 0ull;
        if (!ok && n) atomicOr(R->err, kRansBad);
    }
}

// A wave's chunk, for rans_chunk: where its planes' data and tables are,
// where its elements go, and the bytes of its planes of one symbol.
template <int W>
struct RansChunk {
    using Elem = typename std::conditional<W == 1, uint8_t, typename std::conditional<W == 2, uint16_t, uint32_t>::type>::type;
    const GLB uint8_t *src;
    const GLB uint64_t *pinfo;  // of the array's first plane
    uint32_t ch;
    GLB Elem *dst;              // the chunk's first element
    uint32_t len, steps, cval;
    const uint8_t *sym;         // LDS: sym[plane][4096]
    const uint32_t *fc;         // LDS: fc[plane][256]
    uint32_t *ring;             // LDS: this wave's rings, ring[chain][rans_ring(W) / 2]
    Elem *stage;                // LDS: this wave's stage
    uint32_t *trash;            // LDS: this wave's trash slots
    uint32_t lane;
    GLB uint32_t *err;
    GLB uint32_t *err2;         // a second word to flag (the frame's status), or null
};

// The elements of a block (staged in LDS, step-major) written to the chunk's
// place in its array: B consecutive elements per lane.
template <int W>
__device__ __forceinline__ void rans_store_block(const RansChunk<W> &C, uint32_t j0)
{
    using Elem = typename RansChunk<W>::Elem;
    using Out = typename std::conditional<rans_blk(W) * W == 4, uint32_t, uint2>::type;  // a lane's elements of a block
    constexpr uint32_t B = rans_blk(W);
    static_assert(B * W == 4 || B * W == 8, "4 or 8 bytes per lane and block");
    const uint32_t len = C.len, lane = C.lane;
    const uint32_t nb = len - kRansLanes * j0 < kRansLanes * B ? len - kRansLanes * j0 : kRansLanes * B;
    const Elem *sv = C.stage + B * lane;
    GLB Elem *dv = C.dst + kRansLanes * j0 + B * lane;
    if (B * lane + B <= nb) {
        *(GLB Out *)dv = *(const Out *)sv;
    } else {
        for (uint32_t e = 0; e < B; e++)
            if (B * lane + e < nb) dv[e] = sv[e];
    }
}

// Decode one chunk whose planes pl[0 .. K-1] need decoding (K independent
// state chains per lane).  One step takes one symbol of each chain per lane,
// the chains side by side (table reads of all chains, then their arithmetic,
// then their ring reads).  A lane whose state fell below 2^16 takes the word
// at rd + (the number of such lanes below it); every lane reads the ring and
// masks the word out where it is not needed (no branch, so the chains' reads
// can overlap).  Global memory is touched only between blocks.  At the end of
// each block, emit(j0) takes the block's elements from the stage (element
// 64 (j0 + s) + l of the chunk at stage[64 s + l]).
template <int W, int K, class Emit>
__device__ __forceinline__ void rans_chunk(const RansChunk<W> &C, const uint32_t *pl, Emit &&emit)
{
    using Elem = typename RansChunk<W>::Elem;
    constexpr uint32_t B = rans_blk(W), RING = rans_ring(W), AHEAD = 2 * kRansLanes * B;
    const uint32_t lane = C.lane, len = C.len, steps = C.steps;
    // the plane of chain k (chain k is plane k when every plane is decoded:
    // then the tables' places and the bytes' shifts are constants)
    auto plane = [&](int k) -> uint32_t { return K == W ? (uint32_t)k : pl[k]; };
    // the chains' data: states, word streams
    uint32_t x[K ? K : 1], nwords[K ? K : 1], rd[K ? K : 1], wr[K ? K : 1];
    const GLB uint32_t *wsrc[K ? K : 1];
    const uint8_t *sym[K ? K : 1];
    const uint32_t *fc[K ? K : 1];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const uint64_t pos = readlane64(C.pinfo[2 * plane(k)]), data0 = readlane64(C.pinfo[2 * plane(k) + 1]);
        const uint32_t o0 = readlane(rans_rd32(C.src, pos + 512 + 4ull * C.ch), 0);
        const uint32_t o1 = readlane(rans_rd32(C.src, pos + 512 + 4ull * C.ch + 4), 0);
        wsrc[k] = (const GLB uint32_t *)(C.src + data0 + o0);
        x[k] = wsrc[k][lane];
        wsrc[k] += kRansLanes;
        nwords[k] = (o1 - o0 - 4 * kRansLanes) / 2;
        rd[k] = 0;
        sym[k] = C.sym + 4096 * plane(k);
        fc[k] = C.fc + 256 * plane(k);
    }
    // the first AHEAD words of each stream (a chain's loads in flight together)
#pragma unroll
    for (int k = 0; k < K; k++) {
        constexpr uint32_t U = AHEAD / kRansUnit;
        uint32_t v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            const uint32_t wi = kRansUnit * u + 2 * lane;
            v[u] = wi < nwords[k] ? wsrc[k][wi / 2] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; u++) C.ring[k * (RING / 2) + ((kRansUnit * u + 2 * lane) % RING) / 2] = v[u];
        wr[k] = AHEAD;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    auto step = [&](bool live) -> uint32_t {
        uint32_t slot[K ? K : 1], sy[K ? K : 1], e[K ? K : 1], xn[K ? K : 1], need[K ? K : 1];
        uint64_t msk[K ? K : 1];
#pragma unroll
        for (int k = 0; k < K; k++) {
            slot[k] = x[k] & 4095u;
            sy[k] = sym[k][slot[k]];
        }
#pragma unroll
        for (int k = 0; k < K; k++) e[k] = fc[k][sy[k]];
#pragma unroll
        for (int k = 0; k < K; k++) {
            xn[k] = __umul24(e[k] & 0xFFFFu, x[k] >> 12) + slot[k] - (e[k] >> 16);
            need[k] = live && xn[k] < kRansLow;
            msk[k] = __builtin_amdgcn_ballot_w64(need[k]);
        }
        uint32_t v = C.cval;
#pragma unroll
        for (int k = 0; k < K; k++) {
            // rd + (lanes below this one that take a word), by mbcnt's addend
            const uint32_t wi = __builtin_amdgcn_mbcnt_hi((uint32_t)(msk[k] >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)msk[k], rd[k]));
            const uint32_t w = ((const uint16_t *)(C.ring + k * (RING / 2)))[wi & (RING - 1)];
            // x = need ? x << 16 | w : x, as one select on the ballot's mask
            // (written out, so that the ring read is not moved under a branch)
            const uint32_t xs = (xn[k] << 16) | w;
            uint32_t xr;
            asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(xr) : "v"(xn[k]), "v"(xs), "s"(msk[k]));
            xn[k] = xr;
            rd[k] += (uint32_t)__popcll(msk[k]);
            if (live) x[k] = xn[k];
            v |= sy[k] << (8 * plane(k));
        }
        return v;
    };
    uint32_t over = 0;  // a stream read beyond its words
    for (uint32_t j0 = 0; j0 < steps; j0 += B) {
        // read ahead what the next block may read: up to P units per chain
        // (the units not needed are not loaded, their registers hold 0).  P
        // units always reach rd + AHEAD: the previous block's read-ahead
        // reached its own rd + AHEAD, and a block reads fewer than kRansLanes B
        // words, P units' worth.
        constexpr int P = (int)(kRansLanes * B / kRansUnit);
        static_assert(P >= 1 && P * kRansUnit == kRansLanes * B, "a block's reads are whole units");
        uint32_t pf[K ? K : 1][P], m[K ? K : 1];
#pragma unroll
        for (int k = 0; k < K; k++) {
            m[k] = 0;
#pragma unroll
            for (int u = 0; u < P; u++) {
                const uint32_t u0 = wr[k] + kRansUnit * u;
                const uint32_t wi = u0 + 2 * lane;
                const bool take = u0 < rd[k] + AHEAD && u0 < nwords[k];
                pf[k][u] = take && wi < nwords[k] ? wsrc[k][wi / 2] : 0u;
                m[k] += take;
            }
        }
        if (kRansLanes * (j0 + B) <= len) {  // every lane has a symbol at every step
#pragma unroll
            for (uint32_t s = 0; s < B; s++) C.stage[kRansLanes * s + lane] = (Elem)step(true);
        } else {
            for (uint32_t s = 0; s < B; s++) {
                const uint32_t j = j0 + s;
                if (j >= steps) break;
                C.stage[kRansLanes * s + lane] = (Elem)step(kRansLanes * j + lane < len);
            }
        }
        // end of the block: the read-ahead has arrived, the elements go out.
        // Every register is written (a write under a condition would make the
        // compiler wait for all loads at the next block's start): the units
        // loaded into the ring, the others into the wave's trash slots.
#pragma unroll
        for (int k = 0; k < K; k++) {
#pragma unroll
            for (int u = 0; u < P; u++) {
                uint32_t *d = (uint32_t)u < m[k] ? &C.ring[k * (RING / 2) + ((wr[k] + kRansUnit * u + 2 * lane) % RING) / 2]
                                                 : &C.trash[lane];
                *d = pf[k][u];
            }
            wr[k] += kRansUnit * m[k];
            over |= rd[k] > nwords[k];
        }
        // (the stage and the rings are this wave's own: in-order LDS, no barrier)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        emit(j0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // a well-formed chunk: every state back at its start, every word read
    bool fine = !over;
#pragma unroll
    for (int k = 0; k < K; k++) fine = fine && x[k] == kRansLow && nwords[k] - rd[k] < 8;
    if (__ballot(!fine) && lane == 0) {
        atomicOr(C.err, kRansBad);
        if (C.err2) atomicOr(C.err2, kRansBad);
    }
}

// The fused placement of the unattached arrays (k_rans<W, kRansUnPhase>): a
// wave's chunk holds elements [c0, c0 + len) of one array; element g belongs to the
// last bin b with uin[b] <= g and goes to output slot g + (roff[b] + rna[b] -
// uin[b]) if g < uin[b] + room[b] (room: what k_unattached would store of the
// bin).  Time and pad differences become running sums within the bin; the
// sums of the chunk's leading elements (those of a bin that began in an
// earlier chunk) miss that bin's earlier elements, which k_rans_unfix adds.
// A window of 64 bins' start, shift and end (lane j: bin wb + j) is kept in
// registers; the bin of the current element only moves forward.
struct RansUnBins {
    const GLB uint32_t *uin, *ueff, *roff, *rna;
    uint64_t cap;
    uint32_t wb;              // first bin of the window
    uint32_t wst, wsh, wlim;  // (lane j) bin wb + j: start, slot shift, end of its stored elements

    __device__ __forceinline__ void load(uint32_t b0, uint32_t lane)
    {
        wb = b0;
        const uint32_t b = b0 + lane;
        uint32_t st = 0xFFFFFFFFu, sh = 0, lim = 0;
        if (b < (uint32_t)NBIN) {
            const uint32_t u = uin[b], e = ueff[b], d = roff[b] + rna[b];
            const uint32_t room = d < cap ? (uint32_t)min((uint64_t)e, cap - d) : 0u;
            st = u;
            sh = d - u;
            lim = u + room;
        }
        wst = st;
        wsh = sh;
        wlim = lim;
    }
};

// (witem: for each phase and width class, the first work item of each
// frame, then the total; a work item is kRansWaves consecutive chunks of one
// array of the class.  Phase kRansUnPhase: the unattached arrays, placed into
// the frame's output, fd being the track-model decode's frame descriptors.)
template <int W, int PH>
__global__ __launch_bounds__(kRansLanes * kRansWaves) void k_rans(const RansDesc *descs, const uint32_t *witem,
                                                                  uint32_t nf, const FrameDesc *fd)
{
    constexpr int WI = W == 1 ? 0 : (W == 2 ? 1 : 2);
    constexpr bool UN = PH == kRansUnPhase;
    constexpr uint32_t B = rans_blk(W), RING = rans_ring(W);
    using Elem = typename RansChunk<W>::Elem;
    __shared__ __align__(16) uint8_t sym[W][4096];  // the symbol of every slot
    __shared__ __align__(16) uint32_t fc[W][256];   // f | c << 16 of every symbol
    __shared__ uint32_t ring[kRansWaves][W][RING / 2];  // 2 words per entry
    __shared__ __align__(16) Elem stage[kRansWaves][B * kRansLanes];
    __shared__ uint32_t trash[kRansWaves][kRansLanes];  // where read-ahead units not loaded are written
    const uint32_t wave = threadIdx.x / kRansLanes, lane = lane_id();
    // the frame of this work item: the last one whose first item is at or below it
    const GLB uint32_t *fi = (const GLB uint32_t *)witem + (3 * PH + WI) * (nf + 1);
    uint32_t flo = 0, fhi = nf - 1;
    while (flo < fhi) {
        const uint32_t mid = (flo + fhi + 1) >> 1;
        if (readlane(fi[mid], 0) <= blockIdx.x) flo = mid;
        else fhi = mid - 1;
    }
    const GLB RansDesc *R = (const GLB RansDesc *)descs + flo;
    const uint32_t item = blockIdx.x - readlane(fi[flo], 0);
    // the array and chunks of this item (the descriptor's fields read once,
    // into wave-uniform registers)
    uint32_t a = readlane(R->warr[PH][WI][0], 0), i0 = 0;
    const uint32_t nw = readlane(R->nw[PH][WI], 0);
#pragma unroll
    for (int k = 1; k < 12; k++)
        if ((uint32_t)k < nw && readlane(R->witem0[PH][WI][k], 0) <= item) {
            a = readlane(R->warr[PH][WI][k], 0);
            i0 = readlane(R->witem0[PH][WI][k], 0);
        }
    const GLB uint8_t *const src = (const GLB uint8_t *)readlane64((uint64_t)R->src);
    const uint64_t size = readlane64(R->size);
    const uint32_t n = readlane(R->n[a], 0), p0 = readlane(kRansPlane0[a], 0);
    const uint32_t nch = (n + kRansChunk - 1) / kRansChunk;
    // the planes' tables, shared by the workgroup's waves
    static_assert(kRansTab / 16 <= 2 * kRansLanes * kRansWaves, "2 table loads per thread");
#pragma unroll
    for (int q = 0; q < W; q++) {
        const GLB uint4 *tb = (const GLB uint4 *)(R->tabs + (uint64_t)(p0 + q) * kRansTab);
        uint4 tv[2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const uint32_t i = threadIdx.x + kRansLanes * kRansWaves * k;
            tv[k] = tb[min(i, kRansTab / 16 - 1)];
        }
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const uint32_t i = threadIdx.x + kRansLanes * kRansWaves * k;
            if (i < kRansTab / 16) *(uint4 *)(i < 256 ? (void *)&sym[q][16 * i] : (void *)&fc[q][4 * (i - 256)]) = tv[k];
        }
    }
    __syncthreads();
    // this wave's chunk (no workgroup barrier after this point)
    const uint32_t ch = kRansWaves * (item - i0) + wave;
    if (ch >= nch) return;
    const uint32_t c0 = ch * kRansChunk;
    const uint32_t len = n - c0 < kRansChunk ? n - c0 : kRansChunk;
    const uint32_t steps = (len + kRansLanes - 1) / kRansLanes;
    GLB Elem *dst = UN ? nullptr : (GLB Elem *)readlane64((uint64_t)R->dst[a]) + c0;  // (UN: the output instead)
    uint32_t(*rg)[RING / 2] = ring[wave];
    Elem *stg = stage[wave];
    // the unattached arrays are decoded after k_tilesum took the frame's
    // starting flags from R->err: their flags go to the frame's status too
    GLB uint32_t *status = nullptr;
    if constexpr (UN) status = (GLB uint32_t *)readlane64((uint64_t)((const GLB FrameDesc *)fd)[flo].status);
    // planes of one symbol: its byte, nothing to decode
    uint32_t cst = 0, csym[W];
#pragma unroll
    for (int q = 0; q < W; q++) {
        csym[q] = readlane(sym[q][0], 0);
        if ((readlane(fc[q][csym[q]], 0) & 0xFFFFu) == 4096u) cst |= 1u << q;
    }
    // the W planes' chunk data must be well formed: offsets, sizes, states
    uint32_t x[W];
    bool bad = false;
#pragma unroll
    for (int q = 0; q < W; q++) {
        const uint64_t pos = readlane64(R->pinfo[2 * (p0 + q)]), data0 = readlane64(R->pinfo[2 * (p0 + q) + 1]);
        uint32_t o0 = 0, o1 = 0;
        if (data0) {
            o0 = readlane(rans_rd32(src, pos + 512 + 4ull * ch), 0);
            o1 = readlane(rans_rd32(src, pos + 512 + 4ull * ch + 4), 0);
        }
        const bool qok = data0 && o1 >= o0 && o1 - o0 >= 4 * kRansLanes && (o0 % 16) == 0 &&
                         ((o1 - o0) % 16) == 0 && data0 + o1 <= size;
        bad |= !qok;
        const uint64_t d0 = qok ? data0 + o0 : 0;
        x[q] = qok ? ((const GLB uint32_t *)(src + d0))[lane] : kRansLow;
    }
    // every stored state is in [2^16, 2^32) (this also waits for the states
    // here, not inside the loop)
#pragma unroll
    for (int q = 0; q < W; q++) bad |= __ballot(x[q] < kRansLow) != 0;
    if (bad && lane == 0) {  // not a well-formed chunk: flagged, its elements 0
        atomicOr(R->err, kRansBad);
        if (UN) atomicOr(status, kRansBad);
    }
    if (!UN && bad) {
        for (uint32_t e = lane; e < len; e += kRansLanes) dst[e] = 0;
        return;
    }
    // the planes that need decoding run as K chains; the others only add
    // their byte to every element (a malformed chunk: no chains, elements 0)
    uint32_t cval = 0, K = 0, pl[W];
#pragma unroll
    for (int q = 0; q < W; q++) {
        pl[q] = 0;
        if (((cst >> q) & 1u) && !bad) cval |= csym[q] << (8 * q);
    }
#pragma unroll
    for (int q = 0; q < W; q++)
        if (!((cst >> q) & 1u) && !bad) {
#pragma unroll
            for (int k = 0; k < W; k++) pl[k] = (uint32_t)k == K ? (uint32_t)q : pl[k];
            K++;
        }
    RansChunk<W> C{src, R->pinfo + 2 * p0, ch, dst, len, steps, cval, &sym[0][0], &fc[0][0], &rg[0][0], stg,
                   trash[wave], lane, R->err, status};
    auto run = [&](auto &&emit) {
        switch (K) {
        case 0: rans_chunk<W, 0>(C, pl, emit); break;
        case 1: rans_chunk<W, 1>(C, pl, emit); break;
        case 2: if constexpr (W >= 2) rans_chunk<W, 2>(C, pl, emit); break;
        case 3: if constexpr (W >= 3) rans_chunk<W, 3>(C, pl, emit); break;
        default: if constexpr (W >= 4) rans_chunk<W, 4>(C, pl, emit); break;
        }
    };
    if constexpr (!UN) {
        run([&](uint32_t j0) { rans_store_block<W>(C, j0); });
    } else {
        // the output array, and whether its elements are running sums
        const GLB FrameDesc *F = (const GLB FrameDesc *)fd + flo;
        const uint32_t q = a - kRansUn0;  // 0 time, 1 pad, 2 qtot, 3 qmax
        const bool scan = q < 2;
        GLB uint8_t *out;
        if (W == 4) out = (GLB uint8_t *)readlane64((uint64_t)F->otime);
        else out = (GLB uint8_t *)readlane64(q == 1 ? (uint64_t)F->opad : (q == 2 ? (uint64_t)F->oqtot : (uint64_t)F->oqmax));
        RansUnBins U;
        U.uin = (const GLB uint32_t *)readlane64((uint64_t)F->uin);
        U.ueff = (const GLB uint32_t *)readlane64((uint64_t)F->ueff);
        U.roff = (const GLB uint32_t *)readlane64((uint64_t)F->roff);
        U.rna = (const GLB uint32_t *)readlane64((uint64_t)F->rna);
        U.cap = readlane64(F->cap);
        // the bin of element c0: the last bin whose start is at or below it
        // (starts are non-decreasing, uin[0] = 0): 64 samples 86 bins apart,
        // then the 85 bins after the last sample at or below c0
        const uint32_t lo = 86u * ((uint32_t)__popcll(__ballot(U.uin[86u * lane] <= c0)) - 1u);
        const uint32_t bA = lo + 1 + lane, bB = lo + 65 + lane;
        const bool inA = bA < (uint32_t)NBIN && bA <= lo + 85 && U.uin[min(bA, (uint32_t)NBIN - 1)] <= c0;
        const bool inB = bB < (uint32_t)NBIN && bB <= lo + 85 && U.uin[min(bB, (uint32_t)NBIN - 1)] <= c0;
        uint32_t cb = lo + (uint32_t)__popcll(__ballot(inA)) + (uint32_t)__popcll(__ballot(inB));
        U.load(cb, lane);
        // the current bin cb (of the last element so far): its slot shift,
        // the end of its stored elements, the chunk's sum before its start
        uint32_t sh = readlane(U.wsh, 0), lim = readlane(U.wlim, 0), base = 0;
        const uint32_t sh0 = sh, lim0 = lim;
        uint32_t nstart = readlane(U.wst, 1);          // start of bin cb + 1
        bool head = readlane(U.wst, 0) == c0;           // a bin begins in this chunk
        uint32_t lead = head ? 0u : len;                 // elements before the first such bin
        uint32_t carry = 0;                              // running sum of the chunk's elements
        run([&](uint32_t j0) {
            const uint32_t tb = kRansLanes * j0;  // the block's first element
            const uint32_t nb = len - tb < kRansLanes * B ? len - tb : kRansLanes * B;
            if (nstart > c0 + tb + nb - 1) {
                // no bin begins in this block: every element is in bin cb.
                // A lane takes B consecutive elements, their sums come from one
                // wave scan of the lanes' totals, and they go out as one access
                // (not aligned to its width; the hardware allows that).
                static_assert(B * W == 8, "8 bytes per lane and block");
                const uint32_t e0 = B * lane, g0 = c0 + tb + e0;
                uint32_t v[B];
#pragma unroll
                for (uint32_t e = 0; e < B; e++) v[e] = e0 + e < nb ? (uint32_t)stg[e0 + e] : 0u;
                if (scan) {
#pragma unroll
                    for (uint32_t e = 1; e < B; e++) v[e] += v[e - 1];
                    const uint32_t I = wave_incl_add(v[B - 1]);
                    const uint32_t add = carry + (I - v[B - 1]) - base;
#pragma unroll
                    for (uint32_t e = 0; e < B; e++) v[e] += add;
                    carry += readlane(I, kRansLanes - 1);
                }
                if (e0 + B <= nb && g0 + B <= lim) {
                    uint2 o;
                    if constexpr (W == 4) o = make_uint2(v[0], v[1]);
                    else o = make_uint2((v[0] & 0xFFFFu) | (v[1] << 16), (v[2] & 0xFFFFu) | (v[3] << 16));
                    store_wide((GLB Elem *)out + g0 + sh, o);
                } else {
#pragma unroll
                    for (uint32_t e = 0; e < B; e++)
                        if (e0 + e < nb && g0 + e < lim) ((GLB Elem *)out)[g0 + e + sh] = (Elem)v[e];
                }
                return;
            }
            // a bin begins in this block: step by step, 64 consecutive
            // elements at a time
#pragma unroll
            for (uint32_t s = 0; s < B; s++) {
                const uint32_t t0 = kRansLanes * (j0 + s);
                if (t0 >= len) break;
                const uint32_t t = t0 + lane;
                const bool live = t < len;
                const uint32_t v = live ? (uint32_t)stg[kRansLanes * s + lane] : 0u;
                uint32_t S = v;
                if (scan) {
                    S = carry + wave_incl_add(v);
                    carry = readlane(S, kRansLanes - 1);
                }
                const uint32_t gs = c0 + t0, g = gs + lane;
                const uint32_t gl = c0 + (t0 + kRansLanes - 1 < len ? t0 + kRansLanes - 1 : len - 1);
                // the lane's bin: the current one, or one that begins in this step
                uint32_t lsh = sh, llim = lim, lbase = base;
                while (nstart <= gl) {  // bin cb + 1 begins at lane nstart - gs of this step
                    const uint32_t h = nstart - gs;
                    base = readlane(S, (int)h) - readlane(v, (int)h);
                    cb++;
                    if (!head) {
                        head = true;
                        lead = nstart - c0;
                    }
                    if (cb + 1 - U.wb >= (uint32_t)kRansLanes) U.load(cb, lane);
                    sh = readlane(U.wsh, (int)(cb - U.wb));
                    lim = readlane(U.wlim, (int)(cb - U.wb));
                    const bool sel = g >= nstart;
                    lsh = sel ? sh : lsh;
                    llim = sel ? lim : llim;
                    lbase = sel ? base : lbase;
                    nstart = readlane(U.wst, (int)(cb + 1 - U.wb));
                }
                const uint32_t val = scan ? S - lbase : v;
                if (live && g < llim) {
                    if (W == 4) ((GLB uint32_t *)out)[g + lsh] = val;
                    else ((GLB uint16_t *)out)[g + lsh] = (uint16_t)val;
                }
            }
        });
        if (scan && lane == 0) {
            // the chunk's record: the sum of its last bin's elements, whether
            // a bin begins in it, how many leading elements were stored, and
            // the slot of its first element
            const uint32_t ls = lim0 > c0 ? min(lim0 - c0, lead) : 0u;
            GLB uint4 *rec = (GLB uint4 *)readlane64((uint64_t)R->urec) + (uint64_t)q * nch + ch;
            *rec = make_uint4(carry - base, head ? 1u : 0u, ls, c0 + sh0);
        }
    }
}

// The running sums of the chunks' leading elements: one wave per (chunk,
// array: time or pad, frame).  The sum of their bin's elements in the chunks
// before is the sum of those chunks' last-bin sums, back to the chunk in
// which the bin began.
__global__ __launch_bounds__(kRansLanes) void k_rans_unfix(const RansDesc *descs, const FrameDesc *fd)
{
    const uint32_t ch = blockIdx.x, q = blockIdx.y, lane = lane_id();
    const GLB RansDesc *R = (const GLB RansDesc *)descs + blockIdx.z;
    const uint32_t n = R->n[kRansUn0 + q];
    const uint32_t nch = (n + kRansChunk - 1) / kRansChunk;
    if (ch == 0 || ch >= nch) return;
    const GLB uint4 *rec = R->urec + (uint64_t)q * nch;
    const uint4 me = rec[ch];
    const uint32_t ls = readlane(me.z, 0), d0 = readlane(me.w, 0);
    if (ls == 0) return;
    uint32_t carry = 0;
    for (int32_t c = (int32_t)ch - 1; c >= 0; c -= kRansLanes) {
        const int32_t ci = c - (int32_t)lane;
        uint4 r = make_uint4(0u, 1u, 0u, 0u);
        if (ci >= 0) r = rec[ci];
        const uint64_t hm = __ballot(r.y != 0);
        const uint32_t stop = hm ? (uint32_t)__builtin_ctzll(hm) : (uint32_t)kRansLanes;
        carry += readlane(wave_incl_add(lane <= stop ? r.x : 0u), kRansLanes - 1);
        if (hm) break;
    }
    const GLB FrameDesc *F = (const GLB FrameDesc *)fd + blockIdx.z;
    if (q == 0) {
        GLB uint32_t *o = (GLB uint32_t *)readlane64((uint64_t)F->otime) + d0;
        for (uint32_t i = lane; i < ls; i += kRansLanes) o[i] += carry;
    } else {
        GLB uint16_t *o = (GLB uint16_t *)readlane64((uint64_t)F->opad) + d0;
        for (uint32_t i = lane; i < ls; i += kRansLanes) o[i] = (uint16_t)(o[i] + carry);
    }
}

// ---------------------------------------------------------------------------
// Entropy coding of a frame on the device (the inverse of k_rans, same
// format): per-plane histograms, the 12-bit models, one wave per chunk coding
// its 64 lanes backwards (each step's words go in front of the later steps'
// ones, lanes in order), then a single block placing the planes and a wave
// per chunk packing its states and words into place.
// ---------------------------------------------------------------------------
constexpr uint32_t kRansMeta0 = (64 + 8 * kRansPlanes + 15) & ~15u;  // the header and the plane offsets

struct RansEncDesc {
    const GLB uint8_t *src[kRansArrays];
    uint32_t n[kRansArrays];
    uint32_t item0[kRansPlanes + 1];
    GLB uint32_t *hist;    // [plane][256] symbol counts
    GLB uint16_t *freq;    // [plane][256] the model
    GLB uint16_t *words;   // [item][kRansChunk]: each chunk's words, ending at the end of its area
    GLB uint32_t *states;  // [item][64]: each chunk's final states
    GLB uint32_t *nwords;  // [item]: words of each chunk
    GLB uint64_t *cstart;  // [item]: offset of each chunk's data from its plane's data
    GLB uint64_t *ppos;    // [plane]: position of each plane; [kRansPlanes]: the coded size
    GLB uint8_t *dst;
    GLB uint64_t *size;    // the coded size (the caller's word)
    uint32_t nT, nA, nU;
};

// bytes of a chunk's data: its states and words, padded to 16
__device__ __forceinline__ uint64_t rans_chunk_bytes(uint32_t nw) { return (4ull * kRansLanes + 2ull * nw + 15) & ~15ull; }

// plane p of an item, and the array and byte of that plane
__device__ __forceinline__ void rans_item_plane(const uint32_t *item0, uint32_t item, uint32_t &p, uint32_t &a,
                                                uint32_t &b)
{
    p = 0;
    while (p + 1 < (uint32_t)kRansPlanes && item0[p + 1] <= item) p++;
    a = 0;
    while (a + 1 < (uint32_t)kRansArrays && kRansPlane0[a + 1] <= p) a++;
    b = p - kRansPlane0[a];
}

// symbol counts of one chunk of one plane
__global__ __launch_bounds__(256) void k_renc_hist(const RansEncDesc E)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint32_t p, a, b;
    rans_item_plane(E.item0, blockIdx.x, p, a, b);
    const uint32_t w = kRansWidth[a], n = E.n[a];
    const uint32_t c0 = (blockIdx.x - E.item0[p]) * kRansChunk;
    const uint32_t len = n - c0 < kRansChunk ? n - c0 : kRansChunk;
    const GLB uint8_t *src = E.src[a];
    for (uint32_t i = threadIdx.x; i < len; i += 256) atomicAdd(&h[src[(uint64_t)(c0 + i) * w + b]], 1u);
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&E.hist[256 * p + threadIdx.x], h[threadIdx.x]);
}

// The model of each plane (one wave per plane): frequencies summing to 2^12,
// every symbol that occurs at least 1: first max(1, floor(count 2^12 / n));
// while the sum is short, one more unit to the symbol whose f n - count 2^12
// is smallest; while it is over, one unit less for the symbol with f > 1
// whose f n - count 2^12 is largest (ties: the lowest symbol).  A plane
// without symbols gets f[0] = 2^12.
__global__ __launch_bounds__(64) void k_renc_model(const RansEncDesc E)
{
    const uint32_t p = blockIdx.x, lane = threadIdx.x;
    uint32_t a = 0;
    while (a + 1 < (uint32_t)kRansArrays && kRansPlane0[a + 1] <= p) a++;
    const uint64_t n = E.n[a];
    uint64_t cnt[4];
    int64_t f[4];
    int64_t sum = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        cnt[q] = E.hist[256 * p + 4 * lane + q];
        f[q] = 0;
        if (n && cnt[q]) {
            const uint64_t v = (cnt[q] << 12) / n;
            f[q] = v ? (int64_t)v : 1;
        }
        sum += f[q];
    }
    for (int off = 1; off < kWave; off <<= 1) sum += __shfl_xor(sum, off);
    if (n == 0) {
#pragma unroll
        for (int q = 0; q < 4; q++) f[q] = (lane == 0 && q == 0) ? 4096 : 0;
        sum = 4096;
    }
    while (sum != 4096) {
        const bool up = sum < 4096;
        // this lane's best candidate (its lowest symbol on ties), then the wave's
        int64_t bx = 0;
        int bs = -1;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (!cnt[q] || (!up && f[q] <= 1)) continue;
            const int64_t ex = f[q] * (int64_t)n - (int64_t)(cnt[q] << 12);
            if (bs < 0 || (up ? ex < bx : ex > bx)) {
                bs = 4 * (int)lane + q;
                bx = ex;
            }
        }
        for (int off = 1; off < kWave; off <<= 1) {
            const int64_t ox = __shfl_xor(bx, off);
            const int os = __shfl_xor(bs, off);
            const bool take = os >= 0 && (bs < 0 || (up ? ox < bx : ox > bx) || (ox == bx && os < bs));
            if (take) {
                bx = ox;
                bs = os;
            }
        }
        if (bs >> 2 == (int)lane) {
#pragma unroll
            for (int q = 0; q < 4; q++)
                if ((bs & 3) == q) f[q] += up ? 1 : -1;
        }
        sum += up ? 1 : -1;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) E.freq[256 * p + 4 * lane + q] = (uint16_t)f[q];
}

// one wave per chunk: the 64 lanes code their symbols from the last step to
// the first; a step's words (lanes in order) go in front of the words of the
// steps after it, so the area ends with the stream in reading order
__global__ __launch_bounds__(kRansLanes) void k_renc_code(const RansEncDesc E)
{
    __shared__ uint32_t f[256], c[256];
    const uint32_t lane = lane_id(), item = blockIdx.x;
    uint32_t p, a, b;
    rans_item_plane(E.item0, item, p, a, b);
    uint32_t run = 0;
    uint32_t fl[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        fl[q] = E.freq[256 * p + 4 * lane + q];
        run += fl[q];
    }
    const uint32_t incl = wave_incl_add(run);
    run = incl - run;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        f[4 * lane + q] = fl[q];
        c[4 * lane + q] = run;
        run += fl[q];
    }
    __syncthreads();
    const uint32_t w = kRansWidth[a], n = E.n[a];
    const uint32_t c0 = (item - E.item0[p]) * kRansChunk;
    const uint32_t len = n - c0 < kRansChunk ? n - c0 : kRansChunk;
    const uint32_t steps = (len + kRansLanes - 1) / kRansLanes;
    const GLB uint8_t *src = E.src[a];
    GLB uint16_t *area = E.words + (uint64_t)item * kRansChunk;
    uint32_t wp = kRansChunk;  // start of the words written so far
    uint32_t x = kRansLow;
    for (uint32_t j = steps; j-- > 0;) {
        const uint32_t i = kRansLanes * j + lane;
        const bool live = i < len;
        const uint32_t s = live ? src[(uint64_t)(c0 + i) * w + b] : 0u;
        const uint32_t fs = f[s];
        const bool emit = live && (uint64_t)x >= ((uint64_t)(kRansLow >> 12) << 16) * fs;
        const uint64_t msk = __ballot(emit);
        const uint32_t ne = (uint32_t)__popcll(msk);
        if (emit) {
            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(msk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)msk, 0u));
            area[wp - ne + r] = (uint16_t)x;
            x >>= 16;
        }
        wp -= ne;
        if (live) x = ((x / fs) << 12) + x % fs + c[s];
    }
    E.states[(uint64_t)item * kRansLanes + lane] = x;
    if (lane == 0) E.nwords[item] = kRansChunk - wp;
}

// single block: plane positions, chunk starts, the header, offsets and models
__global__ __launch_bounds__(256) void k_renc_place(const RansEncDesc E)
{
    __shared__ uint64_t part[256];
    const uint32_t t = threadIdx.x;
    uint64_t pos = kRansMeta0;
    for (uint32_t i = 64 + 8 * kRansPlanes + t; i < kRansMeta0; i += 256) E.dst[i] = 0;
    for (uint32_t p = 0; p < (uint32_t)kRansPlanes; p++) {
        const uint32_t i0 = E.item0[p], i1 = E.item0[p + 1], nch = i1 - i0;
        const uint64_t data0 = (pos + 512 + 4ull * (nch + 1) + 15) & ~15ull;
        // the plane's model
        {
            const uint16_t v = E.freq[256 * p + t];
            E.dst[pos + 2 * t] = (uint8_t)v;
            E.dst[pos + 2 * t + 1] = (uint8_t)(v >> 8);
        }
        for (uint64_t q = pos + 512 + 4ull * (nch + 1) + t; q < data0; q += 256) E.dst[q] = 0;
        if (t == 0) {
            E.ppos[p] = pos;
            for (int q = 0; q < 8; q++) E.dst[64 + 8 * p + q] = (uint8_t)(pos >> (8 * q));
        }
        // chunk starts: exclusive prefix of the chunk sizes, 256 at a time
        uint64_t base = 0;
        for (uint32_t i = i0; i < i1; i += 256) {
            const uint64_t v = i + t < i1 ? rans_chunk_bytes(E.nwords[i + t]) : 0;
            part[t] = v;
            __syncthreads();
            for (uint32_t off = 1; off < 256; off <<= 1) {
                const uint64_t o = t >= off ? part[t - off] : 0;
                __syncthreads();
                part[t] += o;
                __syncthreads();
            }
            if (i + t < i1) E.cstart[i + t] = base + part[t] - v;
            base += part[255];
            __syncthreads();
        }
        if (t == 0) {  // the end of the plane's data, after its last chunk's offset
            const uint32_t v = (uint32_t)base;
            for (int q = 0; q < 4; q++) E.dst[pos + 512 + 4ull * nch + q] = (uint8_t)(v >> (8 * q));
        }
        const uint64_t end = data0 + base;
        const uint64_t next = p + 1 < (uint32_t)kRansPlanes ? (end + 15) & ~15ull : end;
        pos = next;  // (the data ends on a 16-byte boundary: no gap)
    }
    if (t < 64) {  // the header: "TMDR", version 2, the shape, zeros
        uint8_t v = 0;
        if (t < 4) v = (uint8_t)"TMDR"[t];
        else if (t < 24) {
            const uint32_t h[5] = {kRansVersion, E.nT, E.nA, E.nU, 0u};
            v = (uint8_t)(h[(t - 4) / 4] >> (8 * ((t - 4) % 4)));
        }
        E.dst[t] = v;
    }
    if (t == 0) {
        E.ppos[kRansPlanes] = pos;
        *E.size = pos;
    }
}

// one wave per chunk: its offset, states and words, then zero padding
__global__ __launch_bounds__(kRansLanes) void k_renc_pack(const RansEncDesc E)
{
    const uint32_t lane = lane_id(), item = blockIdx.x;
    uint32_t p, a, b;
    rans_item_plane(E.item0, item, p, a, b);
    const uint32_t ch = item - E.item0[p], nch = E.item0[p + 1] - E.item0[p];
    const uint64_t pos = E.ppos[p];
    const uint64_t data0 = (pos + 512 + 4ull * (nch + 1) + 15) & ~15ull;
    const uint64_t cs = E.cstart[item];
    const uint32_t nw = E.nwords[item];
    if (lane < 4) E.dst[pos + 512 + 4ull * ch + lane] = (uint8_t)((uint32_t)cs >> (8 * lane));
    GLB uint8_t *out = E.dst + data0 + cs;
    const uint32_t x = E.states[(uint64_t)item * kRansLanes + lane];
    for (int q = 0; q < 4; q++) out[4 * lane + q] = (uint8_t)(x >> (8 * q));
    const GLB uint16_t *wsrc = E.words + (uint64_t)item * kRansChunk + (kRansChunk - nw);
    GLB uint8_t *wout = out + 4 * kRansLanes;
    const uint32_t bytes = (uint32_t)rans_chunk_bytes(nw) - 4 * kRansLanes;
    for (uint32_t t = lane; t < bytes; t += kRansLanes) {
        const uint32_t k = t / 2;
        wout[t] = k < nw ? (uint8_t)(wsrc[k] >> (8 * (t & 1))) : (uint8_t)0;
    }
}

// ---------------------------------------------------------------------------
// workspace of tmd_decode_static: device memory of the library itself, one
// array per GPU (the kernels never see its host-side name, only the address
// hipGetSymbolAddress gives for the current device)
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[TMD_STATIC_SCRATCH_BYTES];

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
constexpr int kStages = 7;  // the decode's stages
// (tmd_decode_rans's entropy decoding: stage kStages, "rans", of the track
// and attached arrays before the track-model decode; kStages + 1, "rans_un",
// of the unattached clusters into the output, beside the rank and attached
// kernels)
constexpr int kAllStages = kStages + 2;
const char *kStageNames[kAllStages] = {"tilesum",  "count",      "colscan", "offsets", "rank",
                                       "attached", "unattached", "rans",    "rans_un"};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct FrameLayout {
    size_t start, tilesum, hist, uin, ueff, recs, ckey, keyinfo, tkey, order;
    uint32_t ntile, tile0;
};

}  // namespace

struct tmd_plan {
    int device = 0;
    uint32_t simds = 1024;  // SIMDs of the device (CUs x 4): the attached decode balances its waves over them
    uint32_t tracks_per_wave = kWave;  // attached decode: tracks per wave (64..128; tmd_set_schedule)
    uint32_t persist = 0;              // attached decode: persistent grid of persist waves per SIMD (0: off)
    uint32_t *d_work = nullptr;        // its per-XCD work counters
    uint32_t n_frames = 0;
    uint32_t total_tiles = 0;
    tmd_params params{};
    std::vector<tmd_frame_shape> shapes;
    std::vector<FrameLayout> layout;
    size_t ws_bytes = 0;
    Geo *d_geo = nullptr;
    uint32_t *d_tile_frame = nullptr;
    FrameDesc *d_desc = nullptr;  // device table (FrameDescHost bytes)
    uint32_t *d_status = nullptr;
    uint32_t *h_status = nullptr;  // pinned
    FrameDescHost *h_desc = nullptr;   // pinned staging
    std::vector<FrameDescHost> last_desc;
    bool desc_valid = false;
    hipEvent_t desc_done = nullptr;
    hipEvent_t done = nullptr;
    bool called = false;  // `done` has been recorded at least once
    uint32_t profiling = 0;                            // stage mask
    uint32_t prof_rans = 0;                            // events around tmd_decode_rans's entropy decoding (2 bits)
    void *h_rans = nullptr;                            // pinned staging of its descriptors
    size_t h_rans_bytes = 0;
    hipEvent_t rans_copy = nullptr;                    // their last upload
    bool rans_staged = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rans_events[2];  // its stages: before, unattached
    std::vector<std::vector<hipEvent_t>> prof_events;  // per recorded call: 2 per stage (unrecorded: null)
    std::vector<hipEvent_t> event_pool;                // events ready for reuse
    hipGraphExec_t graph = nullptr;   // TMD_PLAN_GRAPH: the captured launch sequence
    hipStream_t capture = nullptr;    // stream the graph is captured on
    // tmd_decode_rans: the stream on which part of its entropy decoding runs
    // beside the track-model decode, and the events that order the two
    hipStream_t side = nullptr;
    hipEvent_t fork[2] = {}, join[2] = {};  // [0]: work before k_offsets, [1]: after
    // TMD_PLAN_GRAPH with profiling: a second graph with an event-record node
    // before and after each selected stage; each replay points those nodes
    // at fresh events from the pool
    hipGraph_t prof_src = nullptr;     // the captured graph (its nodes address the exec's)
    hipGraphExec_t prof_graph = nullptr;
    uint32_t prof_mask = 0;            // stages the profiling graph brackets
    std::vector<hipEvent_t> prof_marks;      // capture-time events, 2 per stage (null: unselected)
    std::vector<hipGraphNode_t> prof_nodes;  // their record nodes
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

// Device address of `scratch` on each device, looked up once per device
// (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int static_scratch(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return TMD_E_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TMD_E_HIP;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return TMD_OK;
}

template <class T>
bool aligned(const T *p)
{
    return ((uintptr_t)p % alignof(T)) == 0;
}

// Waves of the attached decode for a frame of nT tracks: ceil(nT / tpw) (tpw:
// the plan's tracks per wave, 64..128), or, for a single-frame call whose count
// is just above a multiple of the SIMD count, that multiple (tracks per wave
// up to tpw + 2, at most 128; see wave_lanes).
uint32_t attached_waves(uint32_t nT, bool single, uint32_t simds, uint32_t tpw)
{
    const uint32_t w0 = (uint32_t)(((uint64_t)nT + tpw - 1) / tpw);
    if (!single || simds == 0 || w0 <= simds || w0 % simds == 0) return w0;
    const uint32_t w = w0 / simds * simds;
    const uint64_t cap = std::min<uint64_t>((uint64_t)tpw + 2, kMaxWaveTracks);
    return (uint64_t)nT <= cap * w ? w : w0;
}

// Events for the stages selected in `mask` (2 per stage, null for the
// others), taken from the plan's pool.  Timing only: no system-scope fence
// (no cache write-back and invalidation around the timed kernels).
int take_events(tmd_plan_t *P, uint32_t mask, std::vector<hipEvent_t> &ev)
{
    ev.assign(2 * kStages, nullptr);
    for (int st = 0; st < kStages; st++) {
        if (!((mask >> st) & 1u)) continue;
        for (int e = 0; e < 2; e++) {
            if (!P->event_pool.empty()) {
                ev[2 * st + e] = P->event_pool.back();
                P->event_pool.pop_back();
            } else {
                HIP_TRY(hipEventCreateWithFlags(&ev[2 * st + e], hipEventDisableSystemFence));
            }
        }
    }
    return TMD_OK;
}

// Work that tmd_decode_rans runs on the plan's second stream beside the
// launch sequence, from the offsets on until its end: the unattached
// clusters' decoding into the output, in place of k_unattached.  It enqueues
// its kernels on the stream it is given.
using SideWork = std::function<int(hipStream_t)>;

// Enqueue side on the plan's second stream after what s holds so far, and
// record the plan's join event k after it.
int fork_side(tmd_plan_t *P, hipStream_t s, const SideWork &side, int k)
{
    if (!P->side) {
        HIP_TRY(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking));
        for (int e = 0; e < 2; e++) {
            HIP_TRY(hipEventCreateWithFlags(&P->fork[e], hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&P->join[e], hipEventDisableTiming));
        }
    }
    HIP_TRY(hipEventRecord(P->fork[k], s));
    HIP_TRY(hipStreamWaitEvent(P->side, P->fork[k], 0));
    const int rc = side(P->side);
    HIP_TRY(hipEventRecord(P->join[k], P->side));  // (also after a failed launch: s must not wait forever)
    return rc;
}

// Enqueue the pipeline on stream s, one kernel after the other.  Each stage
// with events in `ev` (2 per stage, or empty) is bracketed by them.  With
// `side`, once the offsets are known, side runs on the plan's second stream
// (fork_side) and s waits for it at its end (k_unattached has nothing to do).
// wait_early: work that the caller put on the second stream before (its join
// event 0) must be done before k_offsets.
int launch_all(tmd_plan_t *P, hipStream_t s, const std::vector<hipEvent_t> &ev, const SideWork *side = nullptr,
               bool wait_early = false)
{
    auto begin = [&](int st, hipStream_t q) -> int {
        return (ev.size() && ev[2 * st] && hipEventRecord(ev[2 * st], q) != hipSuccess) ? TMD_E_HIP : TMD_OK;
    };
    auto end = [&](int st, hipStream_t q) -> int {
        return (ev.size() && ev[2 * st + 1] && hipEventRecord(ev[2 * st + 1], q) != hipSuccess) ? TMD_E_HIP
                                                                                              : TMD_OK;
    };
    const uint32_t T = P->total_tiles;
    if (begin(0, s)) return TMD_E_HIP;
    uint32_t *work = P->persist ? P->d_work : nullptr;
    hipLaunchKernelGGL(k_tilesum, dim3(T + P->n_frames), dim3(kTile), 0, s, P->d_desc, P->d_tile_frame, T, work);
    if (end(0, s) || begin(1, s)) return TMD_E_HIP;
    if (T) hipLaunchKernelGGL(k_count, dim3(T), dim3(kCountThreads), 0, s, P->d_desc, P->d_tile_frame);
    if (end(1, s) || begin(2, s)) return TMD_E_HIP;
    hipLaunchKernelGGL(k_colscan, dim3((kHRow + kWave - 1) / kWave, P->n_frames), dim3(kWave * kScanWaves), 0,
                       s, P->d_desc);
    if (end(2, s)) return TMD_E_HIP;
    if (wait_early) HIP_TRY(hipStreamWaitEvent(s, P->join[0], 0));
    if (begin(3, s)) return TMD_E_HIP;
    hipLaunchKernelGGL(k_offsets, dim3(P->n_frames), dim3(kOffThreads), 0, s, P->d_desc);
    if (side)
        if (const int rc = fork_side(P, s, *side, 1)) return rc;
    if (end(3, s) || begin(4, s)) return TMD_E_HIP;
    if (T) hipLaunchKernelGGL(k_rank, dim3(T), dim3(kTile), 0, s, P->d_desc, P->d_tile_frame);
    if (end(4, s)) return TMD_E_HIP;
    // attached decode, then the unattached one.  (Run side by side on two
    // streams they take as long in all: the unattached waves slow the attached
    // decode by about what they take alone.)
    if (begin(5, s)) return TMD_E_HIP;
    if (T) {
        // wave slots: 4 per tile of the planned capacity; persistent: a grid
        // of persist waves per SIMD (a multiple of the XCD count) takes them
        const uint32_t slots = T * (kTileWaves / kAttWaves);
        uint32_t grid = slots;
        if (work) grid = std::max<uint32_t>(kXcds, std::min<uint32_t>(slots, P->simds * P->persist) / kXcds * kXcds);
        hipLaunchKernelGGL(k_attached, dim3(grid), dim3(kAttWaves * kWave), 0, s, P->d_desc, P->d_tile_frame, P->d_geo,
                           P->n_frames == 1 ? 1u : 0u, work, slots);
    }
    if (end(5, s) || begin(6, s)) return TMD_E_HIP;
    hipLaunchKernelGGL(k_unattached, dim3(NBIN, P->n_frames), dim3(kWave), 0, s, P->d_desc);
    if (end(6, s)) return TMD_E_HIP;
    if (side) HIP_TRY(hipStreamWaitEvent(s, P->join[1], 0));
    HIP_TRY(hipGetLastError());
    return TMD_OK;
}

// Capture the launch sequence on the plan's capture stream and instantiate it.
int capture_graph(tmd_plan_t *P, hipGraph_t *src, hipGraphExec_t *exec)
{
    hipGraph_t g = nullptr;
    *src = nullptr;
    *exec = nullptr;
    if (hipStreamBeginCapture(P->capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return TMD_E_HIP;
    const int rc = launch_all(P, P->capture, {});
    const hipError_t ec = hipStreamEndCapture(P->capture, &g);
    if (rc != TMD_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return TMD_E_HIP;
    }
    if (hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) {
        *exec = nullptr;
        (void)hipGraphDestroy(g);
        return TMD_E_HIP;
    }
    *src = g;
    return TMD_OK;
}

void drop_prof_graph(tmd_plan_t *P)
{
    if (P->prof_graph) (void)hipGraphExecDestroy(P->prof_graph);
    if (P->prof_src) (void)hipGraphDestroy(P->prof_src);
    for (hipEvent_t e : P->prof_marks)
        if (e) (void)hipEventDestroy(e);
    P->prof_graph = nullptr;
    P->prof_src = nullptr;
    P->prof_marks.clear();
    P->prof_nodes.clear();
    P->prof_mask = 0;
}

// The kernel each stage launches (graph nodes are matched to stages by it).
const void *stage_kernel(int st)
{
    switch (st) {
    case 0: return (const void *)k_tilesum;
    case 1: return (const void *)k_count;
    case 2: return (const void *)k_colscan;
    case 3: return (const void *)k_offsets;
    case 4: return (const void *)k_rank;
    case 5: return (const void *)k_attached;
    default: return (const void *)k_unattached;
    }
}

// The profiling graph for P->profiling, made once per stage mask: the launch
// sequence is captured (stream capture leaves event records out of a graph),
// then an event-record node is inserted before and after the kernel node of
// each selected stage (between it and its neighbours in the chain).  The
// nodes record placeholder events; each replay points them at fresh ones.
int prof_graph_ready(tmd_plan_t *P)
{
    if (P->prof_graph && P->prof_mask == P->profiling) return TMD_OK;
    drop_prof_graph(P);
    hipGraph_t g = nullptr;
    hipGraphExec_t unused = nullptr;
    int rc = capture_graph(P, &g, &unused);
    if (unused) (void)hipGraphExecDestroy(unused);
    if (rc != TMD_OK) return rc;
    P->prof_src = g;
    P->prof_marks.assign(2 * kStages, nullptr);
    P->prof_nodes.assign(2 * kStages, nullptr);
    size_t nn = 0;
    if (hipGraphGetNodes(g, nullptr, &nn) != hipSuccess) rc = TMD_E_HIP;
    std::vector<hipGraphNode_t> nodes(nn);
    if (rc == TMD_OK && nn && hipGraphGetNodes(g, nodes.data(), &nn) != hipSuccess) rc = TMD_E_HIP;
    for (size_t i = 0; rc == TMD_OK && i < nn; i++) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (t != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp;
        if (hipGraphKernelNodeGetParams(nodes[i], &kp) != hipSuccess) { rc = TMD_E_HIP; break; }
        int st = -1;
        for (int k = 0; k < kStages; k++)
            if (kp.func == stage_kernel(k)) st = k;
        if (st < 0 || !((P->profiling >> st) & 1u)) continue;
        hipGraphNode_t K = nodes[i];
        size_t np = 0, ns = 0;
        if (hipGraphNodeGetDependencies(K, nullptr, &np) != hipSuccess ||
            hipGraphNodeGetDependentNodes(K, nullptr, &ns) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        std::vector<hipGraphNode_t> pre(np), suc(ns);
        if ((np && hipGraphNodeGetDependencies(K, pre.data(), &np) != hipSuccess) ||
            (ns && hipGraphNodeGetDependentNodes(K, suc.data(), &ns) != hipSuccess)) {
            rc = TMD_E_HIP;
            break;
        }
        hipEvent_t &m0 = P->prof_marks[2 * st], &m1 = P->prof_marks[2 * st + 1];
        hipGraphNode_t &E0 = P->prof_nodes[2 * st], &E1 = P->prof_nodes[2 * st + 1];
        if (hipEventCreateWithFlags(&m0, hipEventDisableSystemFence) != hipSuccess ||
            hipEventCreateWithFlags(&m1, hipEventDisableSystemFence) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        // pre -> E0 -> K -> E1 -> suc
        if (hipGraphAddEventRecordNode(&E0, g, pre.data(), np, m0) != hipSuccess) { rc = TMD_E_HIP; break; }
        for (size_t q = 0; q < np && rc == TMD_OK; q++)
            if (hipGraphRemoveDependencies(g, &pre[q], &K, 1) != hipSuccess) rc = TMD_E_HIP;
        if (rc == TMD_OK && hipGraphAddDependencies(g, &E0, &K, 1) != hipSuccess) rc = TMD_E_HIP;
        if (rc == TMD_OK && hipGraphAddEventRecordNode(&E1, g, &K, 1, m1) != hipSuccess) rc = TMD_E_HIP;
        for (size_t q = 0; q < ns && rc == TMD_OK; q++)
            if (hipGraphRemoveDependencies(g, &K, &suc[q], 1) != hipSuccess ||
                hipGraphAddDependencies(g, &E1, &suc[q], 1) != hipSuccess)
                rc = TMD_E_HIP;
    }
    if (rc == TMD_OK && hipGraphInstantiate(&P->prof_graph, g, nullptr, nullptr, 0) != hipSuccess) {
        P->prof_graph = nullptr;
        rc = TMD_E_HIP;
    }
    if (rc != TMD_OK) {
        drop_prof_graph(P);
        return rc;
    }
    P->prof_mask = P->profiling;
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
    case TMD_E_SCRATCH: return "the plan's workspace exceeds the library's static scratch (TMD_STATIC_SCRATCH_BYTES)";
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
    int o = 0;
    for (int r = 0; r < NROW; r++) dst[o++] = g.row[r].x;
    for (int r = 0; r < NROW; r++) dst[o++] = g.row[r].pw;
    for (int r = 0; r < NROW; r++) dst[o++] = g.row[r].inv_pw;
    for (int r = 0; r < NROW; r++) dst[o++] = g.row[r].padoff;
    for (int r = 0; r < NROW; r++) dst[o++] = g.row[r].pwq;
    for (int r = 0; r < NROW; r++) dst[o++] = g.row[r].ks;
    for (int r = 0; r < NROW; r++) dst[o++] = g.row[r].kt;
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
        for (auto e : v)
            if (e) (void)hipEventDestroy(e);
    for (auto &L : P->rans_events)
        for (auto &v : L) {
            (void)hipEventDestroy(v.first);
            (void)hipEventDestroy(v.second);
        }
    for (auto e : P->event_pool) (void)hipEventDestroy(e);
    if (P->graph) (void)hipGraphExecDestroy(P->graph);
    drop_prof_graph(P);
    if (P->capture) (void)hipStreamDestroy(P->capture);
    if (P->side) (void)hipStreamDestroy(P->side);
    for (int k = 0; k < 2; k++) {
        if (P->fork[k]) (void)hipEventDestroy(P->fork[k]);
        if (P->join[k]) (void)hipEventDestroy(P->join[k]);
    }
    if (P->desc_done) (void)hipEventDestroy(P->desc_done);
    if (P->done) (void)hipEventDestroy(P->done);
    if (P->d_geo) (void)hipFree(P->d_geo);
    if (P->d_tile_frame) (void)hipFree(P->d_tile_frame);
    if (P->d_desc) (void)hipFree(P->d_desc);
    if (P->d_status) (void)hipFree(P->d_status);
    if (P->d_work) (void)hipFree(P->d_work);
    if (P->h_status) (void)hipHostFree(P->h_status);
    if (P->h_desc) (void)hipHostFree(P->h_desc);
    if (P->h_rans) (void)hipHostFree(P->h_rans);
    if (P->rans_copy) (void)hipEventDestroy(P->rans_copy);
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
        L.hist = off;    off += align256(4 * (size_t)L.ntile * kHRow);
        L.uin = off;     off += align256(4 * (size_t)NBIN);
        L.ueff = off;    off += align256(4 * (size_t)NBIN);
        L.recs = off;    off += align256(16 * (size_t)(S.n_attached ? S.n_attached : 1));
        L.ckey = off;    off += align256(2 * (size_t)(S.n_attached ? S.n_attached : 1));
        L.keyinfo = off; off += align256(4 * (size_t)(2 * kNKey));
        L.tkey = off;    off += align256(2 * (size_t)(S.n_tracks ? S.n_tracks : 1));
        L.order = off;   off += align256(4 * (size_t)(S.n_tracks ? S.n_tracks : 1));
        P->layout.push_back(L);
    }
    P->total_tiles = tiles;
    P->ws_bytes = off;
    int rc = TMD_OK;
    do {
        if (hipGetDevice(&P->device) != hipSuccess) { rc = TMD_E_HIP; break; }
        {
            void *sp = nullptr;  // set-up of tmd_decode_static's scratch on this device
            if ((rc = static_scratch(P->device, &sp)) != TMD_OK) break;
        }
        {
            int cus = 0;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess) {
                rc = TMD_E_HIP;
                break;
            }
            P->simds = cus > 0 ? 4u * (uint32_t)cus : 4u;
            // (tests set a small count to exercise the wave balancing on small frames)
            if (const char *e = getenv("TMD_ATTACHED_SIMDS")) {
                const long v = strtol(e, nullptr, 10);
                if (v > 0 && v < (1L << 20)) P->simds = (uint32_t)v;
            }
        }
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
        if (hipMalloc(&P->d_work, sizeof(uint32_t) * kXcds) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipMemset(P->d_status, 0, sizeof(uint32_t) * n_frames) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipHostMalloc((void **)&P->h_status, sizeof(uint32_t) * n_frames, 0) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        memset(P->h_status, 0, sizeof(uint32_t) * n_frames);
        if (hipHostMalloc((void **)&P->h_desc, sizeof(FrameDescHost) * n_frames, 0) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        if (hipEventCreateWithFlags(&P->desc_done, hipEventDisableTiming) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipEventCreateWithFlags(&P->done, hipEventDisableTiming) != hipSuccess) { rc = TMD_E_HIP; break; }
        if ((p->flags & TMD_PLAN_GRAPH) &&
            hipStreamCreateWithFlags(&P->capture, hipStreamNonBlocking) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
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
    if (!P) return TMD_E_ARG;
    return tmd_decode_shapes(P, P->shapes.data(), in, out, workspace, stream);
}

}  // extern "C"

namespace {
int decode_impl(tmd_plan_t *P, const tmd_frame_shape *shapes, const tmd_frame_in *in, tmd_frame_out *out,
                void *workspace, void *stream);
int decode_descs(tmd_plan_t *P, const tmd_frame_shape *shapes, const tmd_frame_in *in, tmd_frame_out *out,
                 void *workspace, const uint32_t *const *pre_status, bool un_fused,
                 std::vector<FrameDescHost> &desc);
int decode_enqueue(tmd_plan_t *P, const std::vector<FrameDescHost> &desc, void *stream, const SideWork *side,
                   bool wait_early);
}  // namespace

extern "C" {

int tmd_decode_shapes(tmd_plan_t *P, const tmd_frame_shape *shapes, const tmd_frame_in *in, tmd_frame_out *out,
                      void *workspace, void *stream)
{
    return decode_impl(P, shapes, in, out, workspace, stream);
}

}  // extern "C"

namespace {

// The argument checks of a decode call (nothing is enqueued) and its frame
// descriptors.  pre_status: an optional device word per frame that the
// frame's status starts from (flags of a step before the decode).  un_fused:
// the unattached clusters are decoded elsewhere (their input arrays may be
// null).
int decode_descs(tmd_plan_t *P, const tmd_frame_shape *shapes, const tmd_frame_in *in, tmd_frame_out *out,
                 void *workspace, const uint32_t *const *pre_status, bool un_fused,
                 std::vector<FrameDescHost> &desc)
{
    const bool post = un_fused;
    if (!P || !shapes || !in || !out || !workspace) return TMD_E_ARG;
    if ((uintptr_t)workspace % 256) return TMD_E_ARG;
    for (uint32_t f = 0; f < P->n_frames; f++) {
        const tmd_frame_shape &C = P->shapes[f], &S = shapes[f];
        if (S.n_tracks > C.n_tracks || S.n_attached > C.n_attached || S.n_unattached > C.n_unattached)
            return TMD_E_ARG;
    }
    desc.assign(P->n_frames, FrameDescHost{});
    for (uint32_t f = 0; f < P->n_frames; f++) {
        const tmd_frame_shape &S = shapes[f];
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
        if (S.n_unattached && !post && (!I.un_time_diff || !I.un_pad_diff || !I.un_qtot || !I.un_qmax))
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
        FrameDescHost &D = desc[f];
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
        D.recs = (uint4 *)(ws + L.recs);
        D.ckey = (uint16_t *)(ws + L.ckey);
        D.keyinfo = (uint32_t *)(ws + L.keyinfo);
        D.tkey = (uint16_t *)(ws + L.tkey);
        D.order = (uint32_t *)(ws + L.order);
        D.status = P->d_status + f;
        D.pre_status = pre_status ? pre_status[f] : nullptr;
        D.cap = O.capacity;
        D.nT = S.n_tracks; D.nA = S.n_attached; D.nU = S.n_unattached;
        D.ntile = (S.n_tracks + kTile - 1) / kTile;  // <= the planned L.ntile
        D.tile0 = L.tile0;
        D.awaves = attached_waves(S.n_tracks, P->n_frames == 1, P->simds, P->tracks_per_wave);
        D.un_fused = post ? 1u : 0u;
    }
    return TMD_OK;
}

// Enqueue a decode whose descriptors decode_descs built.  With `side`, the
// unattached clusters are not decoded by the sequence: side decodes them on
// the plan's second stream once the offsets are known (launch_all; the
// kernels are then launched one by one, also for a graph plan).  wait_early:
// see launch_all.
int decode_enqueue(tmd_plan_t *P, const std::vector<FrameDescHost> &desc, void *stream, const SideWork *side,
                   bool wait_early)
{
    hipStream_t s = (hipStream_t)stream;
    const bool post = side != nullptr;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != P->device) HIP_TRY(hipSetDevice(P->device));
    int rc = TMD_OK;
    do {
        // calls on one plan share its descriptor table and status words:
        // a call issued on another stream starts after the previous one ends
        if (P->called && hipStreamWaitEvent(s, P->done, 0) != hipSuccess) { rc = TMD_E_HIP; break; }
        const size_t dbytes = sizeof(FrameDescHost) * P->n_frames;
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
        if ((P->params.flags & TMD_PLAN_GRAPH) && !post && !wait_early) {
            // the kernels read only plan-owned buffers (descriptor table,
            // tables, tile map), so one captured graph serves every call
            if (P->profiling) {
                // the profiling graph, its record nodes pointed at fresh events
                if ((rc = prof_graph_ready(P)) != TMD_OK) break;
                // fresh events for the stages whose kernels are in the graph
                uint32_t have = 0;
                for (int st = 0; st < kStages; st++)
                    if (P->prof_nodes[2 * st]) have |= 1u << st;
                std::vector<hipEvent_t> ev;
                if ((rc = take_events(P, have, ev)) != TMD_OK) break;
                for (int k = 0; k < 2 * kStages && rc == TMD_OK; k++)
                    if (ev[k] && hipGraphExecEventRecordNodeSetEvent(P->prof_graph, P->prof_nodes[k], ev[k]) !=
                                     hipSuccess)
                        rc = TMD_E_HIP;
                if (rc == TMD_OK && hipGraphLaunch(P->prof_graph, s) != hipSuccess) rc = TMD_E_HIP;
                if (rc != TMD_OK) {
                    for (hipEvent_t e : ev)
                        if (e) P->event_pool.push_back(e);
                    break;
                }
                P->prof_events.push_back(ev);
            } else {
                if (!P->graph) {
                    hipGraph_t g = nullptr;
                    if ((rc = capture_graph(P, &g, &P->graph)) != TMD_OK) break;
                    (void)hipGraphDestroy(g);
                }
                if (hipGraphLaunch(P->graph, s) != hipSuccess) { rc = TMD_E_HIP; break; }
            }
        } else {
            std::vector<hipEvent_t> ev;
            if (P->profiling && (rc = take_events(P, P->profiling, ev)) != TMD_OK) break;
            rc = launch_all(P, s, ev, side, wait_early);
            if (rc != TMD_OK) {
                for (hipEvent_t e : ev)
                    if (e) P->event_pool.push_back(e);
                break;
            }
            if (P->profiling) P->prof_events.push_back(ev);
        }
        if (hipMemcpyAsync(P->h_status, P->d_status, sizeof(uint32_t) * P->n_frames, hipMemcpyDeviceToHost,
                           s) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        if (hipEventRecord(P->done, s) != hipSuccess) { rc = TMD_E_HIP; break; }
        P->called = true;
    } while (0);
    if (cur != P->device) (void)hipSetDevice(cur);
    return rc;
}

// tmd_decode_shapes: check, then enqueue
int decode_impl(tmd_plan_t *P, const tmd_frame_shape *shapes, const tmd_frame_in *in, tmd_frame_out *out,
                void *workspace, void *stream)
{
    std::vector<FrameDescHost> desc;
    if (const int rc = decode_descs(P, shapes, in, out, workspace, nullptr, false, desc)) return rc;
    return decode_enqueue(P, desc, stream, nullptr, false);
}

}  // namespace

extern "C" {

int tmd_status(tmd_plan_t *P, uint32_t frame, uint32_t *flags)
{
    if (!P || !flags || frame >= P->n_frames) return TMD_E_ARG;
    HIP_TRY(hipEventSynchronize(P->done));
    uint32_t f = P->h_status[frame];
    *flags = f;
    if (f & (TMD_F_COUNT | TMD_F_CODED)) return TMD_E_INPUT;
    if (f) return TMD_E_STREAM;
    return TMD_OK;
}

int tmd_decode_static(tmd_plan_t *P, const tmd_frame_shape *shapes, const tmd_frame_in *in, tmd_frame_out *out,
                      void *stream)
{
    if (!P) return TMD_E_ARG;
    if (P->ws_bytes > (size_t)TMD_STATIC_SCRATCH_BYTES) return TMD_E_SCRATCH;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != P->device) HIP_TRY(hipSetDevice(P->device));
    void *ws = nullptr;
    int rc = static_scratch(P->device, &ws);
    if (cur != P->device) (void)hipSetDevice(cur);
    if (rc != TMD_OK) return rc;
    return tmd_decode_shapes(P, shapes ? shapes : P->shapes.data(), in, out, ws, stream);
}

int tmd_set_schedule(tmd_plan_t *P, uint32_t tracks_per_wave, uint32_t persist_waves_per_simd)
{
    if (!P) return TMD_E_ARG;
    if (tracks_per_wave == 0) tracks_per_wave = kWave;
    if (tracks_per_wave < (uint32_t)kWave || tracks_per_wave > kMaxWaveTracks || persist_waves_per_simd > 64)
        return TMD_E_ARG;
    if (P->tracks_per_wave == tracks_per_wave && P->persist == persist_waves_per_simd) return TMD_OK;
    // the next call waits for the last one (it still uses the old settings)
    if (P->called) HIP_TRY(hipEventSynchronize(P->done));
    P->tracks_per_wave = tracks_per_wave;
    P->persist = persist_waves_per_simd;
    P->desc_valid = false;  // wave counts change: upload the descriptors again
    if (P->graph) {         // launch shapes change: capture again
        (void)hipGraphExecDestroy(P->graph);
        P->graph = nullptr;
    }
    drop_prof_graph(P);
    return TMD_OK;
}

int tmd_set_profiling(tmd_plan_t *P, uint32_t stage_mask)
{
    if (!P) return TMD_E_ARG;
    P->profiling = stage_mask & ((1u << kStages) - 1u);
    P->prof_rans = (stage_mask >> kStages) & 3u;
    return TMD_OK;
}

int tmd_stage_times(tmd_plan_t *P, double *ms, uint32_t n, uint32_t *calls)
{
    if (!P || (!ms && n)) return TMD_E_ARG;
    std::vector<double> acc(kStages, 0.0);
    for (auto &ev : P->prof_events) {
        for (int i = 0; i < kStages; i++) {
            if (!ev[2 * i]) continue;
            HIP_TRY(hipEventSynchronize(ev[2 * i + 1]));
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
            acc[i] += t;
        }
    }
    for (auto &L : P->rans_events) {
        double sum = 0.0;
        for (auto &v : L) {
            HIP_TRY(hipEventSynchronize(v.second));
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, v.first, v.second));
            sum += t;
        }
        acc.push_back(sum);
    }
    if (calls)
        *calls = (uint32_t)std::max({P->prof_events.size(), P->rans_events[0].size(), P->rans_events[1].size()});
    for (auto &ev : P->prof_events)
        for (auto e : ev)
            if (e) P->event_pool.push_back(e);
    P->prof_events.clear();
    for (auto &L : P->rans_events) {
        for (auto &v : L) {
            P->event_pool.push_back(v.first);
            P->event_pool.push_back(v.second);
        }
        L.clear();
    }
    for (uint32_t i = 0; i < n && i < (uint32_t)kAllStages; i++) ms[i] = acc[i];
    return kAllStages;
}

const char *tmd_stage_name(uint32_t stage) { return stage < (uint32_t)kAllStages ? kStageNames[stage] : ""; }

int tmd_selftest_math(const float *a, uint32_t *out, uint32_t n, void *stream)
{
    if (!a || !out) return TMD_E_ARG;
    if (n == 0) return TMD_OK;
    Geo g;
    build_geo(0.5f, &g);
    hipLaunchKernelGGL(k_selftest_math, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, a, g.snp_max,
                       out, n);
    HIP_TRY(hipGetLastError());
    return TMD_OK;
}

int tmd_selftest_sqrt(uint32_t lo_bits, uint32_t hi_bits, uint32_t *mismatches, void *stream)
{
    if (!mismatches || lo_bits > hi_bits) return TMD_E_ARG;
    hipLaunchKernelGGL(k_selftest_sqrt, dim3(4096), dim3(256), 0, (hipStream_t)stream, lo_bits, hi_bits,
                       mismatches);
    HIP_TRY(hipGetLastError());
    return TMD_OK;
}

int tmd_selftest_fp(const float *a, const float *b, float *out, uint32_t n, void *stream)
{
    if (!a || !b || !out) return TMD_E_ARG;
    if (n == 0) return TMD_OK;
    hipLaunchKernelGGL(k_selftest_fp, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, a, b, out, n);
    HIP_TRY(hipGetLastError());
    return TMD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Encoder host side
// ---------------------------------------------------------------------------
namespace {

struct EncLayout {
    size_t hn, htrk, rec, bsum, k0, k1, v0, v1, rhist, rflag, total;
    uint32_t nb, rblocks;
};

EncLayout enc_layout(uint32_t n, uint32_t nU)
{
    EncLayout L;
    L.nb = (n + 1023) / 1024;
    L.rblocks = (nU + kRadTile - 1) / kRadTile;
    size_t off = 0;
    L.hn = off;    off += align256(std::max<size_t>(n, 1));
    L.htrk = off;  off += align256(4 * std::max<size_t>(n, 1));
    L.rec = off;   off += align256(8 * std::max<size_t>(n, 1));
    L.bsum = off;  off += align256(4 * ((size_t)L.nb + 1));
    L.k0 = off;    off += align256(8 * std::max<size_t>(nU, 1));
    L.k1 = off;    off += align256(8 * std::max<size_t>(nU, 1));
    L.v0 = off;    off += align256(4 * std::max<size_t>(nU, 1));
    L.v1 = off;    off += align256(4 * std::max<size_t>(nU, 1));
    L.rhist = off; off += align256(4 * 256 * (std::max<size_t>(L.rblocks, 1) + 1));
    L.rflag = off; off += 256;
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

int tmd_encode_workspace(uint32_t n_tracks, uint32_t n_clusters, uint32_t n_unattached, size_t *bytes)
{
    (void)n_tracks;
    if (!bytes) return TMD_E_ARG;
    *bytes = enc_layout(n_clusters, n_unattached).total;
    return TMD_OK;
}

int tmd_encode(tmd_plan_t *P, const tmd_enc_in *in, tmd_enc_out *out, void *workspace, size_t workspace_bytes,
               void *stream)
{
    if (!P || !in || !out || !workspace || !out->counts) return TMD_E_ARG;
    if ((uintptr_t)workspace % 256) return TMD_E_ARG;
    const uint32_t nT = in->n_tracks, n = in->n_clusters, nU = in->n_unattached;
    const EncLayout L = enc_layout(n, nU);
    if (workspace_bytes < L.total) return TMD_E_CAPACITY;
    if (!in->trk_first || !out->un_count) return TMD_E_ARG;
    if (nT && (!in->trk_qpt || !in->trk_tgl)) return TMD_E_ARG;
    if (n && (!in->cl_sec || !in->cl_row || !in->cl_pad || !in->cl_time || !in->cl_snp || !in->cl_qtot ||
              !in->cl_qmax || !out->trk_ncls || !out->trk_sec0 || !out->trk_row0 || !out->trk_pad0 ||
              !out->trk_time0 || !out->trk_qpt || !out->trk_snp || !out->trk_tgl || !out->cls_row_diff ||
              !out->cls_sec_diff || !out->cls_pad_res || !out->cls_time_res || !out->cls_qtot || !out->cls_qmax))
        return TMD_E_ARG;
    if (nU && (!in->un_sec || !in->un_row || !in->un_pad || !in->un_time || !in->un_qtot || !in->un_qmax ||
               !out->un_time_diff || !out->un_pad_diff || !out->un_qtot || !out->un_qmax))
        return TMD_E_ARG;
    if (!aligned(in->trk_first) || !aligned(in->trk_qpt) || !aligned(in->trk_tgl) || !aligned(in->cl_pad) ||
        !aligned(in->cl_time) || !aligned(in->cl_snp) || !aligned(in->cl_qtot) || !aligned(in->cl_qmax) ||
        !aligned(in->un_pad) || !aligned(in->un_time) || !aligned(in->un_qtot) || !aligned(in->un_qmax) ||
        !aligned(out->trk_pad0) || !aligned(out->trk_time0) || !aligned(out->trk_qpt) || !aligned(out->trk_snp) ||
        !aligned(out->trk_tgl) || !aligned(out->cls_pad_res) || !aligned(out->cls_time_res) ||
        !aligned(out->cls_qtot) || !aligned(out->cls_qmax) || !aligned(out->un_count) ||
        !aligned(out->un_time_diff) || !aligned(out->un_pad_diff) || !aligned(out->un_qtot) ||
        !aligned(out->un_qmax) || !aligned(out->counts))
        return TMD_E_ARG;
    EncDesc E;
    memset(&E, 0, sizeof(E));
    E.nT = nT; E.n = n; E.nU = nU;
    E.first = (const GLB uint32_t *)in->trk_first;
    E.qpt = (const GLB double *)in->trk_qpt; E.tgl = (const GLB double *)in->trk_tgl;
    E.sec = (const GLB uint8_t *)in->cl_sec; E.row = (const GLB uint8_t *)in->cl_row;
    E.pad = (const GLB double *)in->cl_pad; E.time = (const GLB double *)in->cl_time;
    E.snp = (const GLB double *)in->cl_snp;
    E.qtot = (const GLB uint16_t *)in->cl_qtot; E.qmax = (const GLB uint16_t *)in->cl_qmax;
    E.usec = (const GLB uint8_t *)in->un_sec; E.urow = (const GLB uint8_t *)in->un_row;
    E.upad = (const GLB double *)in->un_pad; E.utime = (const GLB double *)in->un_time;
    E.uqtot = (const GLB uint16_t *)in->un_qtot; E.uqmax = (const GLB uint16_t *)in->un_qmax;
    E.ncls = (GLB uint8_t *)out->trk_ncls; E.sec0 = (GLB uint8_t *)out->trk_sec0;
    E.row0 = (GLB uint8_t *)out->trk_row0; E.pad0 = (GLB uint16_t *)out->trk_pad0;
    E.time0 = (GLB uint32_t *)out->trk_time0; E.oqpt = (GLB int16_t *)out->trk_qpt;
    E.osnp = (GLB int16_t *)out->trk_snp; E.otgl = (GLB int16_t *)out->trk_tgl;
    E.rdiff = (GLB int8_t *)out->cls_row_diff; E.sdiff = (GLB uint8_t *)out->cls_sec_diff;
    E.pres = (GLB int16_t *)out->cls_pad_res; E.tres = (GLB int16_t *)out->cls_time_res;
    E.cqtot = (GLB uint16_t *)out->cls_qtot; E.cqmax = (GLB uint16_t *)out->cls_qmax;
    E.ucount = (GLB uint32_t *)out->un_count; E.utdiff = (GLB uint32_t *)out->un_time_diff;
    E.updiff = (GLB uint16_t *)out->un_pad_diff; E.uoqtot = (GLB uint16_t *)out->un_qtot;
    E.uoqmax = (GLB uint16_t *)out->un_qmax; E.counts = (GLB uint32_t *)out->counts;
    char *ws = (char *)workspace;
    E.hn = (GLB uint8_t *)(ws + L.hn); E.htrk = (GLB uint32_t *)(ws + L.htrk);
    E.rec = (GLB unsigned long long *)(ws + L.rec);
    E.bsum = (GLB uint32_t *)(ws + L.bsum);
    E.k0 = (GLB unsigned long long *)(ws + L.k0); E.k1 = (GLB unsigned long long *)(ws + L.k1);
    E.v0 = (GLB uint32_t *)(ws + L.v0); E.v1 = (GLB uint32_t *)(ws + L.v1);
    E.rhist = (GLB uint32_t *)(ws + L.rhist);
    E.rflag = (GLB uint32_t *)(ws + L.rflag);
    E.rblocks = L.rblocks;
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != P->device) HIP_TRY(hipSetDevice(P->device));
    // calls on one plan are ordered on the device (they share its tables only,
    // but keep the plan's ordering rule)
    if (P->called) (void)hipStreamWaitEvent(s, P->done, 0);
    hipLaunchKernelGGL(k_enc_clear, dim3((NBIN + 255) / 256), dim3(256), 0, s, E);
    // the unattached clusters (keys, sort, differences) on the plan's second
    // stream, beside the track walk, which leaves most of the GPU idle
    if (nU) {
        const int rc = fork_side(P, s, [&](hipStream_t q) -> int {
            hipLaunchKernelGGL(k_enc_un_keys, dim3((nU + 255) / 256), dim3(256), 0, q, E);
            // the key's 8 passes, the runs of equal keys sorted by payload;
            // then, gated on a run too long for that, the full sort of the
            // result: the payload's 4 passes, then the key's 8.  Both counts
            // are even, so the result ends in (k0, v0) either way.
            unsigned long long *ka = (unsigned long long *)E.k0, *kb = (unsigned long long *)E.k1;
            uint32_t *va = (uint32_t *)E.v0, *vb = (uint32_t *)E.v1;
            auto pass = [&](uint32_t key_pass, uint32_t shift, uint32_t gated) {
                hipLaunchKernelGGL(k_rad_hist, dim3(L.rblocks), dim3(256), 0, q, E, ka, va, key_pass, shift, gated);
                hipLaunchKernelGGL(k_rad_offsets, dim3(256), dim3(256), 0, q, E, gated);
                hipLaunchKernelGGL(k_rad_scatter, dim3(L.rblocks), dim3(256), 0, q, E, ka, va, kb, vb, key_pass,
                                   shift, gated);
                std::swap(ka, kb);
                std::swap(va, vb);
            };
            for (uint32_t d = 0; d < 8; d++) pass(1u, 8u * d, 0u);
            hipLaunchKernelGGL(k_rad_fix, dim3((nU + 255) / 256), dim3(256), 0, q, E, ka, va);
            for (uint32_t d = 0; d < 4; d++) pass(0u, 8u * d, 1u);
            for (uint32_t d = 0; d < 8; d++) pass(1u, 8u * d, 1u);
            hipLaunchKernelGGL(k_enc_un_delta, dim3((nU + 255) / 256), dim3(256), 0, q, E, ka, va);
            return hipGetLastError() == hipSuccess ? TMD_OK : TMD_E_HIP;
        }, 0);
        if (rc != TMD_OK) {
            if (cur != P->device) (void)hipSetDevice(cur);
            return rc;
        }
    }
    if (n) hipLaunchKernelGGL(k_enc_pack, dim3((n + 255) / 256), dim3(256), 0, s, E);
    if (nT) hipLaunchKernelGGL(k_enc_tracks, dim3((nT + 255) / 256), dim3(256), 0, s, E, P->d_geo);
    if (n) {
        hipLaunchKernelGGL(k_enc_scan_blocks, dim3(L.nb), dim3(256), 0, s, E);
        hipLaunchKernelGGL(k_enc_scan_prefix, dim3(1), dim3(1024), 0, s, E, L.nb);
        hipLaunchKernelGGL(k_enc_headers, dim3(L.nb), dim3(256), 0, s, E);
    }
    hipError_t e = hipGetLastError();
    if (nU && hipStreamWaitEvent(s, P->join[0], 0) != hipSuccess) e = hipErrorUnknown;
    if (cur != P->device) (void)hipSetDevice(cur);
    return e == hipSuccess ? TMD_OK : TMD_E_HIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Entropy-coded frames: host side
// ---------------------------------------------------------------------------
namespace {

// element counts of the 19 arrays of a frame, in tmd_frame_in order
void rans_counts(const tmd_frame_shape &S, uint32_t *n)
{
    for (int i = 0; i < 8; i++) n[i] = S.n_tracks;
    for (int i = 8; i < 14; i++) n[i] = S.n_attached;
    n[14] = NBIN;
    for (int i = 15; i < 19; i++) n[i] = S.n_unattached;
}

constexpr uint8_t kRansWidthHost[kRansArrays] = {1, 1, 1, 2, 4, 2, 2, 2, 1, 1, 2, 2, 2, 2, 4, 4, 2, 2, 2};
constexpr int rans_width_sum(int a) { return a == kRansArrays ? 0 : kRansWidthHost[a] + rans_width_sum(a + 1); }
static_assert(rans_width_sum(0) == kRansPlanes, "one plane per byte of the element widths");
constexpr int rans_width_count(int w, int a = 0)
{
    return a == kRansArrays ? 0 : (kRansWidthHost[a] == w) + rans_width_count(w, a + 1);
}
static_assert(rans_width_count(1) <= 12 && rans_width_count(2) <= 12 && rans_width_count(4) <= 12 &&
                  rans_width_count(1) + rans_width_count(2) + rans_width_count(4) == kRansArrays,
              "arrays of 1, 2 or 4 bytes, at most 12 of each");
constexpr int rans_phase_count(int ph, int w, int a = 0)
{
    return a == kRansArrays ? 0 : (rans_phase(a) == ph && kRansWidthHost[a] == w) + rans_phase_count(ph, w, a + 1);
}
// (the kernels tmd_decode_rans launches for each phase)
static_assert(rans_phase_count(1, 1) == 0, "phase 1: 2- and 4-byte arrays");

// The entropy decoding's workspace: the error words of all frames, their
// descriptors and work-item offsets (copied in by each call), then for each
// frame its planes' decode tables and positions, its decoded arrays but the
// unattached ones (those go straight to the output) and the chunk records of
// the unattached time and pad differences (each section 256-byte aligned).
constexpr size_t kRansTabOff = 0;
constexpr size_t kRansInfoOff = kRansTabOff + 256 * ((kRansPlanes * (size_t)kRansTab + 255) / 256);
constexpr size_t kRansArrOff = kRansInfoOff + 256 * ((16 * kRansPlanes + 255) / 256);

struct RansHead {
    size_t err, desc, witem, frames;
};

RansHead rans_head(uint32_t nf)
{
    RansHead H;
    H.err = 0;
    H.desc = align256(4ull * nf);
    H.witem = H.desc + align256(sizeof(RansDesc) * nf);
    H.frames = H.witem + align256(4ull * 3 * kRansPhases * (nf + 1));
    return H;
}

uint32_t rans_chunks(uint32_t n) { return (uint32_t)(((uint64_t)n + kRansChunk - 1) / kRansChunk); }

size_t rans_frame_bytes(const tmd_frame_shape &S)
{
    uint32_t n[kRansArrays];
    rans_counts(S, n);
    size_t b = kRansArrOff;
    for (int a = 0; a < (int)kRansUn0; a++) b += align256((size_t)kRansWidthHost[a] * std::max<uint32_t>(n[a], 1));
    return b + align256(2 * sizeof(uint4) * std::max<uint32_t>(rans_chunks(S.n_unattached), 1));
}

}  // namespace

extern "C" {

int tmd_rans_workspace(const tmd_frame_shape *shapes, uint32_t n_frames, size_t *bytes)
{
    if (!shapes || !bytes || n_frames == 0) return TMD_E_ARG;
    size_t b = rans_head(n_frames).frames;
    for (uint32_t f = 0; f < n_frames; f++) b += rans_frame_bytes(shapes[f]);
    *bytes = b;
    return TMD_OK;
}

int tmd_decode_rans(tmd_plan_t *P, const tmd_frame_shape *shapes, const uint8_t *const *coded,
                    const uint64_t *coded_bytes, tmd_frame_out *out, void *workspace, void *rans_workspace,
                    void *stream)
{
    if (!P || !shapes || !coded || !coded_bytes || !out || !workspace || !rans_workspace) return TMD_E_ARG;
    if ((uintptr_t)rans_workspace % 256) return TMD_E_ARG;
    const uint32_t nf = P->n_frames;
    for (uint32_t f = 0; f < nf; f++) {
        const tmd_frame_shape &C = P->shapes[f], &S = shapes[f];
        if (!coded[f] || (uintptr_t)coded[f] % 16 || S.n_tracks > C.n_tracks || S.n_attached > C.n_attached ||
            S.n_unattached > C.n_unattached)
            return TMD_E_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != P->device) HIP_TRY(hipSetDevice(P->device));
    const RansHead H = rans_head(nf);
    char *ws = (char *)rans_workspace;
    std::vector<tmd_frame_in> in(nf);
    std::vector<const uint32_t *> pre(nf);
    // the descriptors and work-item offsets of every frame, staged in pinned memory
    const size_t hbytes = H.frames - H.desc;
    std::vector<uint8_t> hbuf(hbytes, 0);
    RansDesc *desc = (RansDesc *)hbuf.data();
    uint32_t *witem = (uint32_t *)(hbuf.data() + (H.witem - H.desc));
    char *fws = ws + H.frames;
    uint32_t maxch = 0;  // most chunks of an unattached array
    for (uint32_t f = 0; f < nf; f++) {
        const tmd_frame_shape &S = shapes[f];
        RansDesc &R = desc[f];
        R.src = (const GLB uint8_t *)coded[f];
        R.size = coded_bytes[f];
        R.nT = S.n_tracks;
        R.nA = S.n_attached;
        R.nU = S.n_unattached;
        rans_counts(S, R.n);
        R.err = (GLB uint32_t *)(ws + H.err) + f;
        R.tabs = (GLB uint8_t *)(fws + kRansTabOff);
        R.pinfo = (GLB uint64_t *)(fws + kRansInfoOff);
        size_t off = kRansArrOff;
        void *arr[kRansArrays] = {};
        for (int a = 0; a < (int)kRansUn0; a++) {
            arr[a] = fws + off;
            R.dst[a] = (GLB uint8_t *)arr[a];
            off += align256((size_t)kRansWidthHost[a] * std::max<uint32_t>(R.n[a], 1));
        }
        R.urec = (GLB uint4 *)(fws + off);
        // work items of each phase and width class: one per kRansWaves
        // chunks of its arrays
        for (int a = 0; a < kRansArrays; a++) {
            const int ph = rans_phase(a);
            const int wi = kRansWidthHost[a] == 1 ? 0 : (kRansWidthHost[a] == 2 ? 1 : 2);
            const uint32_t k = R.nw[ph][wi]++;
            R.warr[ph][wi][k] = (uint32_t)a;
            R.witem0[ph][wi][k + 1] = R.witem0[ph][wi][k] + (rans_chunks(R.n[a]) + kRansWaves - 1) / kRansWaves;
        }
        for (int ph = 0; ph < kRansPhases; ph++)
            for (int wi = 0; wi < 3; wi++) {
                uint32_t *t = witem + (3 * ph + wi) * (nf + 1);
                t[f + 1] = t[f] + R.witem0[ph][wi][R.nw[ph][wi]];
            }
        maxch = std::max(maxch, rans_chunks(S.n_unattached));
        tmd_frame_in &I = in[f];
        I.trk_ncls = (const uint8_t *)arr[0]; I.trk_sec0 = (const uint8_t *)arr[1]; I.trk_row0 = (const uint8_t *)arr[2];
        I.trk_pad0 = (const uint16_t *)arr[3]; I.trk_time0 = (const uint32_t *)arr[4];
        I.trk_qpt = (const int16_t *)arr[5]; I.trk_snp = (const int16_t *)arr[6]; I.trk_tgl = (const int16_t *)arr[7];
        I.cls_row_diff = (const int8_t *)arr[8]; I.cls_sec_diff = (const uint8_t *)arr[9];
        I.cls_pad_res = (const int16_t *)arr[10]; I.cls_time_res = (const int16_t *)arr[11];
        I.cls_qtot = (const uint16_t *)arr[12]; I.cls_qmax = (const uint16_t *)arr[13];
        I.un_count = (const uint32_t *)arr[14];  // (the unattached arrays: decoded into the output)
        pre[f] = (const uint32_t *)(ws + H.err) + f;
        fws += rans_frame_bytes(S);
    }
    // the decode's arguments are checked before anything is enqueued
    std::vector<FrameDescHost> fdesc;
    if (const int rc = decode_descs(P, shapes, in.data(), out, workspace, pre.data(), true, fdesc)) {
        if (cur != P->device) (void)hipSetDevice(cur);
        return rc;
    }
    // The kernels of one phase of the entropy decoding on stream q (phase 0
    // with the tables' set-up), between a pair of events if its stage is
    // profiled.
    const RansDesc *dd = (const RansDesc *)(ws + H.desc);
    const uint32_t *dw = (const uint32_t *)(ws + H.witem);
    auto launch_phase = [&](int ph, hipStream_t q) -> int {
        std::pair<hipEvent_t, hipEvent_t> ev(nullptr, nullptr);
        if ((P->prof_rans >> ph) & 1u) {
            std::vector<hipEvent_t> two;
            if (take_events(P, 1u, two) != TMD_OK) return TMD_E_HIP;
            ev = {two[0], two[1]};
            if (hipEventRecord(ev.first, q) != hipSuccess) {
                P->event_pool.push_back(ev.first);
                P->event_pool.push_back(ev.second);
                return TMD_E_HIP;
            }
        }
        const dim3 blk(kRansLanes * kRansWaves);
        const FrameDesc *fd = P->d_desc;
        auto items = [&](int wi) { return witem[(3 * ph + wi) * (nf + 1) + nf]; };
        int r = TMD_OK;
        if (ph == 0) {
            hipLaunchKernelGGL(k_rans_prep, dim3(kRansPlanes * nf), dim3(256), 0, q, dd);
            // the 4-byte arrays (track start times, bin counts: a few chunks
            // per frame, each a long dependent chain) on the plan's second
            // stream, beside the others; the decode waits for them before
            // k_offsets
            r = fork_side(P, q, [&](hipStream_t e) -> int {
                if (const uint32_t it = items(2)) hipLaunchKernelGGL((k_rans<4, 0>), dim3(it), blk, 0, e, dd, dw, nf, fd);
                return TMD_OK;
            }, 0);
            if (const uint32_t it = items(0)) hipLaunchKernelGGL((k_rans<1, 0>), dim3(it), blk, 0, q, dd, dw, nf, fd);
            if (const uint32_t it = items(1)) hipLaunchKernelGGL((k_rans<2, 0>), dim3(it), blk, 0, q, dd, dw, nf, fd);
        } else {
            if (const uint32_t it = items(2)) hipLaunchKernelGGL((k_rans<4, kRansUnPhase>), dim3(it), blk, 0, q, dd, dw, nf, fd);
            if (const uint32_t it = items(1)) hipLaunchKernelGGL((k_rans<2, kRansUnPhase>), dim3(it), blk, 0, q, dd, dw, nf, fd);
            if (maxch > 1) hipLaunchKernelGGL(k_rans_unfix, dim3(maxch, 2, nf), dim3(kRansLanes), 0, q, dd, fd);
        }
        if (r == TMD_OK && hipGetLastError() != hipSuccess) r = TMD_E_HIP;
        if (ev.second) {
            if (r == TMD_OK && hipEventRecord(ev.second, q) == hipSuccess) {
                P->rans_events[ph].push_back(ev);
            } else {
                P->event_pool.push_back(ev.first);
                P->event_pool.push_back(ev.second);
            }
        }
        return r;
    };
    int rc = TMD_OK;
    do {
        // (the previous call on this plan may still read the workspace, and
        // its upload may still read the staging buffer)
        if (P->called && hipStreamWaitEvent(s, P->done, 0) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (P->rans_staged && hipEventSynchronize(P->rans_copy) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (P->h_rans_bytes < hbytes) {
            if (P->h_rans) (void)hipHostFree(P->h_rans);
            P->h_rans = nullptr;
            P->h_rans_bytes = 0;
            if (hipHostMalloc(&P->h_rans, hbytes, 0) != hipSuccess) { rc = TMD_E_HIP; break; }
            P->h_rans_bytes = hbytes;
        }
        if (!P->rans_copy && hipEventCreateWithFlags(&P->rans_copy, hipEventDisableTiming) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        memcpy(P->h_rans, hbuf.data(), hbytes);
        if (hipMemcpyAsync(ws + H.desc, P->h_rans, hbytes, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipEventRecord(P->rans_copy, s) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
        P->rans_staged = true;
        // the error words start at 0 (a fill kernel, not a memset node)
        hipLaunchKernelGGL(k_fill32, dim3(1), dim3(256), 0, s, (uint32_t *)(ws + H.err), nf, 0u);
        rc = launch_phase(0, s);
    } while (0);
    if (cur != P->device) (void)hipSetDevice(cur);
    if (rc != TMD_OK) return rc;
    // once the offsets are known, on the plan's second stream beside the rank
    // and attached kernels: the unattached arrays into their output slots
    const SideWork side = [&](hipStream_t q) { return launch_phase(1, q); };
    return decode_enqueue(P, fdesc, stream, &side, true);
}

}  // extern "C"

namespace {

// bytes of a coded frame of this shape at most, and the encoder's workspace
struct RansEncLayout {
    uint32_t items = 0;
    uint32_t item0[kRansPlanes + 1];
    uint64_t bound = 0;
    size_t hist, freq, words, states, nwords, cstart, ppos, total;
};

int rans_enc_layout(const tmd_frame_shape &S, RansEncLayout &L)
{
    uint32_t n[kRansArrays];
    rans_counts(S, n);
    uint64_t bound = kRansMeta0;
    uint32_t plane = 0, items = 0;
    for (int a = 0; a < kRansArrays; a++) {
        if (n[a] > (1u << 30)) return TMD_E_ARG;  // a plane's offsets are 32-bit
        const uint32_t nch = (n[a] + kRansChunk - 1) / kRansChunk;
        for (int b = 0; b < kRansWidthHost[a]; b++) {
            L.item0[plane++] = items;
            items += nch;
            // alignment, model, chunk offsets, then per chunk its states, at
            // most one word per symbol, and padding
            bound += 16 + 512 + 4ull * (nch + 1) + 16 + (4ull * kRansLanes + 16) * nch + 2ull * n[a];
        }
    }
    L.item0[kRansPlanes] = items;
    L.items = items;
    L.bound = bound;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(std::max<size_t>(bytes, 1));
        return o;
    };
    L.hist = take(4ull * 256 * kRansPlanes);
    L.freq = take(2ull * 256 * kRansPlanes);
    L.words = take(2ull * kRansChunk * items);
    L.states = take(4ull * kRansLanes * items);
    L.nwords = take(4ull * items);
    L.cstart = take(8ull * items);
    L.ppos = take(8ull * (kRansPlanes + 1));
    L.total = off;
    return TMD_OK;
}

}  // namespace

extern "C" {

int tmd_rans_encode_workspace(const tmd_frame_shape *shape, size_t *workspace_bytes, uint64_t *coded_bound)
{
    if (!shape || !workspace_bytes || !coded_bound) return TMD_E_ARG;
    RansEncLayout L;
    const int rc = rans_enc_layout(*shape, L);
    if (rc != TMD_OK) return rc;
    *workspace_bytes = L.total;
    *coded_bound = L.bound;
    return TMD_OK;
}

int tmd_encode_rans(const tmd_frame_shape *shape, const tmd_frame_in *in, uint8_t *coded, uint64_t capacity,
                    uint64_t *coded_bytes, void *workspace, void *stream)
{
    if (!shape || !in || !coded || !coded_bytes || !workspace) return TMD_E_ARG;
    if ((uintptr_t)workspace % 256 || (uintptr_t)coded_bytes % 8) return TMD_E_ARG;
    RansEncLayout L;
    int rc = rans_enc_layout(*shape, L);
    if (rc != TMD_OK) return rc;
    if (capacity < L.bound) return TMD_E_CAPACITY;
    const void *arr[kRansArrays] = {in->trk_ncls, in->trk_sec0, in->trk_row0, in->trk_pad0, in->trk_time0,
                                    in->trk_qpt, in->trk_snp, in->trk_tgl, in->cls_row_diff, in->cls_sec_diff,
                                    in->cls_pad_res, in->cls_time_res, in->cls_qtot, in->cls_qmax, in->un_count,
                                    in->un_time_diff, in->un_pad_diff, in->un_qtot, in->un_qmax};
    RansEncDesc E;
    memset(&E, 0, sizeof(E));
    rans_counts(*shape, E.n);
    for (int a = 0; a < kRansArrays; a++) {
        if (E.n[a] && !arr[a]) return TMD_E_ARG;
        E.src[a] = (const GLB uint8_t *)arr[a];
    }
    memcpy(E.item0, L.item0, sizeof(E.item0));
    char *ws = (char *)workspace;
    E.hist = (GLB uint32_t *)(ws + L.hist);
    E.freq = (GLB uint16_t *)(ws + L.freq);
    E.words = (GLB uint16_t *)(ws + L.words);
    E.states = (GLB uint32_t *)(ws + L.states);
    E.nwords = (GLB uint32_t *)(ws + L.nwords);
    E.cstart = (GLB uint64_t *)(ws + L.cstart);
    E.ppos = (GLB uint64_t *)(ws + L.ppos);
    E.dst = (GLB uint8_t *)coded;
    E.size = (GLB uint64_t *)coded_bytes;
    E.nT = shape->n_tracks;
    E.nA = shape->n_attached;
    E.nU = shape->n_unattached;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill32, dim3(1), dim3(256), 0, s, (uint32_t *)(ws + L.hist), 256u * kRansPlanes, 0u);
    if (L.items) hipLaunchKernelGGL(k_renc_hist, dim3(L.items), dim3(256), 0, s, E);
    hipLaunchKernelGGL(k_renc_model, dim3(kRansPlanes), dim3(64), 0, s, E);
    if (L.items) hipLaunchKernelGGL(k_renc_code, dim3(L.items), dim3(kRansLanes), 0, s, E);
    hipLaunchKernelGGL(k_renc_place, dim3(1), dim3(256), 0, s, E);
    if (L.items) hipLaunchKernelGGL(k_renc_pack, dim3(L.items), dim3(kRansLanes), 0, s, E);
    if (hipGetLastError() != hipSuccess) return TMD_E_HIP;
    return TMD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Host-resident frames (the transfer-hiding scheme of the paper's Fig. 2):
// frames in host memory are decoded through `depth` slots used in turn.  A
// slot owns a decode stream, a capacity plan with its workspace, and device
// copies of one frame's inputs and outputs.  All uploads go through one
// stream and all downloads through another, ordered against the decodes by
// events, so that at any time one upload, one decode and one download can run
// side by side (PCIe carries both directions at once).
// ---------------------------------------------------------------------------
namespace {

enum CountKind { kCntT, kCntA, kCntU, kCntBin };
struct ArrSpec {
    size_t off;     // offset of the pointer in tmd_frame_in
    uint32_t elem;  // element size in bytes
    CountKind kind;
};
#define TMD_IN(f, e, k) {offsetof(tmd_frame_in, f), e, k}
const ArrSpec kPipeIn[] = {
    TMD_IN(trk_ncls, 1, kCntT),     TMD_IN(trk_sec0, 1, kCntT),      TMD_IN(trk_row0, 1, kCntT),
    TMD_IN(trk_pad0, 2, kCntT),     TMD_IN(trk_time0, 4, kCntT),     TMD_IN(trk_qpt, 2, kCntT),
    TMD_IN(trk_snp, 2, kCntT),      TMD_IN(trk_tgl, 2, kCntT),       TMD_IN(cls_row_diff, 1, kCntA),
    TMD_IN(cls_sec_diff, 1, kCntA), TMD_IN(cls_pad_res, 2, kCntA),   TMD_IN(cls_time_res, 2, kCntA),
    TMD_IN(cls_qtot, 2, kCntA),     TMD_IN(cls_qmax, 2, kCntA),      TMD_IN(un_count, 4, kCntBin),
    TMD_IN(un_time_diff, 4, kCntU), TMD_IN(un_pad_diff, 2, kCntU),   TMD_IN(un_qtot, 2, kCntU),
    TMD_IN(un_qmax, 2, kCntU),
};
#undef TMD_IN

size_t pipe_count(CountKind k, const tmd_frame_shape &S)
{
    switch (k) {
    case kCntT: return S.n_tracks;
    case kCntA: return S.n_attached;
    case kCntU: return S.n_unattached;
    default: return NBIN;
    }
}

const void *in_ptr(const tmd_frame_in &I, size_t off)
{
    const void *p;
    memcpy(&p, (const char *)&I + off, sizeof(p));
    return p;
}

void set_in_ptr(tmd_frame_in &I, size_t off, const void *p) { memcpy((char *)&I + off, &p, sizeof(p)); }

struct PipeSlot {
    hipStream_t stream = nullptr;  // decode
    hipEvent_t up = nullptr, dec = nullptr, down = nullptr;  // this slot's last upload, decode, download
    bool used = false;              // the events have been recorded
    tmd_plan_t *plan = nullptr;
    void *ws = nullptr;
    void *din = nullptr;  // device inputs, one allocation
    void *dout = nullptr;  // device outputs, one allocation
    tmd_frame_in in{};
    tmd_frame_out out{};
    int64_t frame = -1;  // frame of the current run whose result is still in flight
    void *dcoded = nullptr;  // coded frames (tmd_pipe_run_rans): device copy
    uint64_t coded_cap = 0;
    void *rws = nullptr;     // and the entropy decoding's workspace
};

}  // namespace

struct tmd_pipe {
    int device = 0;
    tmd_frame_shape cap{};
    std::vector<PipeSlot> slots;
    hipStream_t up = nullptr, down = nullptr;  // all uploads; all downloads
};

extern "C" {

void tmd_pipe_free(tmd_pipe_t *Q)
{
    if (!Q) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != Q->device) (void)hipSetDevice(Q->device);
    if (Q->up) (void)hipStreamSynchronize(Q->up);
    if (Q->down) (void)hipStreamSynchronize(Q->down);
    for (PipeSlot &sl : Q->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        for (hipEvent_t e : {sl.up, sl.dec, sl.down})
            if (e) (void)hipEventDestroy(e);
        tmd_free(sl.plan);
        if (sl.ws) (void)hipFree(sl.ws);
        if (sl.din) (void)hipFree(sl.din);
        if (sl.dout) (void)hipFree(sl.dout);
        if (sl.dcoded) (void)hipFree(sl.dcoded);
        if (sl.rws) (void)hipFree(sl.rws);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (Q->up) (void)hipStreamDestroy(Q->up);
    if (Q->down) (void)hipStreamDestroy(Q->down);
    if (cur != Q->device) (void)hipSetDevice(cur);
    delete Q;
}

int tmd_pipe_create(const tmd_frame_shape *capacity, uint32_t depth, const tmd_params *p, tmd_pipe_t **pipe)
{
    if (!capacity || !p || !pipe || depth == 0 || depth > TMD_PIPE_MAX_DEPTH) return TMD_E_ARG;
    if (capacity->n_tracks > TMD_MAX_TRACKS) return TMD_E_ARG;
    *pipe = nullptr;
    tmd_pipe_t *Q = new (std::nothrow) tmd_pipe_t();
    if (!Q) return TMD_E_HIP;
    Q->cap = *capacity;
    const tmd_params pp = {p->bz_tesla, 0u};  // eager launches: the slots' streams overlap
    int rc = TMD_OK;
    if (hipGetDevice(&Q->device) != hipSuccess) rc = TMD_E_HIP;
    if (rc == TMD_OK && (hipStreamCreateWithFlags(&Q->up, hipStreamNonBlocking) != hipSuccess ||
                         hipStreamCreateWithFlags(&Q->down, hipStreamNonBlocking) != hipSuccess))
        rc = TMD_E_HIP;
    Q->slots.resize(rc == TMD_OK ? depth : 0);
    for (PipeSlot &sl : Q->slots) {
        size_t wsb = 0;
        if ((rc = tmd_plan(capacity, 1, &pp, &sl.plan, &wsb)) != TMD_OK) break;
        if (hipMalloc(&sl.ws, wsb > 256 ? wsb : 256) != hipSuccess) { rc = TMD_E_HIP; break; }
        auto in_bytes = [&](const ArrSpec &a) {
            return align256((size_t)a.elem * std::max<size_t>(pipe_count(a.kind, Q->cap), 1));
        };
        size_t ib = 0;
        for (const ArrSpec &a : kPipeIn) ib += in_bytes(a);
        if (hipMalloc(&sl.din, ib) != hipSuccess) { rc = TMD_E_HIP; break; }
        size_t o = 0;
        for (const ArrSpec &a : kPipeIn) {
            set_in_ptr(sl.in, a.off, (char *)sl.din + o);
            o += in_bytes(a);
        }
        const size_t n = std::max<size_t>((size_t)Q->cap.n_attached + Q->cap.n_unattached, 1);
        const size_t ob = align256(4 * (size_t)(NBIN + 1)) + align256(4 * (size_t)NBIN) + align256(4 * n) +
                          3 * align256(2 * n);
        if (hipMalloc(&sl.dout, ob) != hipSuccess) { rc = TMD_E_HIP; break; }
        char *b = (char *)sl.dout;
        sl.out.row_offset = (uint32_t *)b; b += align256(4 * (size_t)(NBIN + 1));
        sl.out.row_nattached = (uint32_t *)b; b += align256(4 * (size_t)NBIN);
        sl.out.time = (uint32_t *)b; b += align256(4 * n);
        sl.out.pad = (uint16_t *)b; b += align256(2 * n);
        sl.out.qtot = (uint16_t *)b; b += align256(2 * n);
        sl.out.qmax = (uint16_t *)b;
        sl.out.capacity = n;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipEventCreateWithFlags(&sl.up, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&sl.dec, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&sl.down, hipEventDisableTiming) != hipSuccess) {
            rc = TMD_E_HIP;
            break;
        }
    }
    if (rc != TMD_OK) {
        tmd_pipe_free(Q);
        return rc;
    }
    *pipe = Q;
    return TMD_OK;
}

}  // extern "C"

namespace {

// Checks of the output buffers of frame i before anything is enqueued.
int pipe_check_out(const tmd_pipe_t *Q, const tmd_frame_shape &S, const tmd_frame_out &O)
{
    if (S.n_tracks > Q->cap.n_tracks || S.n_attached > Q->cap.n_attached || S.n_unattached > Q->cap.n_unattached)
        return TMD_E_ARG;
    const uint64_t nn = (uint64_t)S.n_attached + S.n_unattached;
    if (O.capacity < nn) return TMD_E_CAPACITY;
    if (!O.row_offset || !O.row_nattached || !aligned(O.row_offset) || !aligned(O.row_nattached)) return TMD_E_ARG;
    if (nn && (!O.time || !O.pad || !O.qtot || !O.qmax || !aligned(O.time) || !aligned(O.pad) || !aligned(O.qtot) ||
               !aligned(O.qmax)))
        return TMD_E_ARG;
    return TMD_OK;
}

// The pipeline over n frames: for frame i, `enqueue(i, slot)` puts its
// upload on Q->up and its decode on the slot's stream (ordered as described
// at tmd_pipe_run); the download and the slot bookkeeping are shared.
template <class Enqueue>
int pipe_execute(tmd_pipe_t *Q, uint32_t n_frames, const tmd_frame_shape *shapes, tmd_frame_out *out,
                 uint32_t *flags, Enqueue enqueue)
{
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != Q->device) HIP_TRY(hipSetDevice(Q->device));
    uint32_t any = 0;
    // wait for a slot's frame to be back and collect its flags
    auto finish = [&](PipeSlot &sl) -> int {
        if (sl.frame < 0) return TMD_OK;
        if (hipEventSynchronize(sl.down) != hipSuccess) return TMD_E_HIP;
        uint32_t f = 0;
        const int r = tmd_status(sl.plan, 0, &f);
        if (r == TMD_E_ARG || r == TMD_E_HIP) return r;
        flags[sl.frame] = f;
        any |= f;
        sl.frame = -1;
        return TMD_OK;
    };
    const uint32_t depth = (uint32_t)Q->slots.size();
    int rc = TMD_OK;
    for (uint32_t i = 0; i < n_frames && rc == TMD_OK; i++) {
        PipeSlot &sl = Q->slots[i % depth];
        if ((rc = finish(sl)) != TMD_OK) break;
        const tmd_frame_shape &S = shapes[i];
        // upload (after the slot's previous decode has read its inputs), then
        // decode (after the upload, and after the slot's previous download has
        // read its outputs)
        if (sl.used && hipStreamWaitEvent(Q->up, sl.dec, 0) != hipSuccess) { rc = TMD_E_HIP; break; }
        if ((rc = enqueue(i, sl)) != TMD_OK) break;
        if (hipEventRecord(sl.dec, sl.stream) != hipSuccess) { rc = TMD_E_HIP; break; }
        if (hipStreamWaitEvent(Q->down, sl.dec, 0) != hipSuccess) { rc = TMD_E_HIP; break; }
        const size_t nn = (size_t)S.n_attached + S.n_unattached;
        const tmd_frame_out &O = out[i];
        struct {
            void *dst;
            const void *src;
            size_t bytes;
        } dl[6] = {{O.row_offset, sl.out.row_offset, 4 * (size_t)(NBIN + 1)},
                   {O.row_nattached, sl.out.row_nattached, 4 * (size_t)NBIN},
                   {O.time, sl.out.time, 4 * nn},
                   {O.pad, sl.out.pad, 2 * nn},
                   {O.qtot, sl.out.qtot, 2 * nn},
                   {O.qmax, sl.out.qmax, 2 * nn}};
        for (auto &d : dl) {
            if (!d.bytes) continue;
            if (hipMemcpyAsync(d.dst, d.src, d.bytes, hipMemcpyDeviceToHost, Q->down) != hipSuccess) {
                rc = TMD_E_HIP;
                break;
            }
        }
        if (rc != TMD_OK) break;
        if (hipEventRecord(sl.down, Q->down) != hipSuccess) { rc = TMD_E_HIP; break; }
        sl.used = true;
        sl.frame = i;
    }
    // drain (also after an error, so that no copy is left running)
    int r = TMD_OK;
    if (hipStreamSynchronize(Q->up) != hipSuccess) r = TMD_E_HIP;
    for (PipeSlot &sl : Q->slots)
        if (hipStreamSynchronize(sl.stream) != hipSuccess) r = TMD_E_HIP;
    if (hipStreamSynchronize(Q->down) != hipSuccess) r = TMD_E_HIP;
    if (rc == TMD_OK) rc = r;
    for (PipeSlot &sl : Q->slots) {
        if (rc == TMD_OK) rc = finish(sl);
        sl.frame = -1;
    }
    if (cur != Q->device) (void)hipSetDevice(cur);
    if (rc != TMD_OK) return rc;
    if (any & TMD_F_COUNT) return TMD_E_INPUT;
    if (any) return TMD_E_STREAM;
    return TMD_OK;
}

}  // namespace

extern "C" {

int tmd_pipe_run(tmd_pipe_t *Q, uint32_t n_frames, const tmd_frame_shape *shapes, const tmd_frame_in *in,
                 tmd_frame_out *out, uint32_t *flags)
{
    if (!Q) return TMD_E_ARG;
    if (n_frames == 0) return TMD_OK;
    if (!shapes || !in || !out || !flags) return TMD_E_ARG;
    // host-side checks of every frame before anything is enqueued
    for (uint32_t i = 0; i < n_frames; i++) {
        const tmd_frame_shape &S = shapes[i];
        if (const int rc = pipe_check_out(Q, S, out[i])) return rc;
        for (const ArrSpec &a : kPipeIn) {
            const void *h = in_ptr(in[i], a.off);
            if (pipe_count(a.kind, S) && (!h || (uintptr_t)h % a.elem)) return TMD_E_ARG;
        }
        flags[i] = 0;
    }
    return pipe_execute(Q, n_frames, shapes, out, flags, [&](uint32_t i, PipeSlot &sl) -> int {
        const tmd_frame_shape &S = shapes[i];
        for (const ArrSpec &a : kPipeIn) {
            const size_t cnt = pipe_count(a.kind, S);
            if (!cnt) continue;
            if (hipMemcpyAsync((void *)in_ptr(sl.in, a.off), in_ptr(in[i], a.off), cnt * a.elem,
                               hipMemcpyHostToDevice, Q->up) != hipSuccess)
                return TMD_E_HIP;
        }
        if (hipEventRecord(sl.up, Q->up) != hipSuccess) return TMD_E_HIP;
        if (hipStreamWaitEvent(sl.stream, sl.up, 0) != hipSuccess) return TMD_E_HIP;
        if (sl.used && hipStreamWaitEvent(sl.stream, sl.down, 0) != hipSuccess) return TMD_E_HIP;
        tmd_frame_out dev = sl.out;
        return tmd_decode_shapes(sl.plan, &S, &sl.in, &dev, sl.ws, sl.stream);
    });
}

int tmd_pipe_run_rans(tmd_pipe_t *Q, uint32_t n_frames, const tmd_frame_shape *shapes,
                      const uint8_t *const *coded, const uint64_t *coded_bytes, tmd_frame_out *out,
                      uint32_t *flags)
{
    if (!Q) return TMD_E_ARG;
    if (n_frames == 0) return TMD_OK;
    if (!shapes || !coded || !coded_bytes || !out || !flags) return TMD_E_ARG;
    size_t enc_ws = 0;
    uint64_t bound = 0;
    if (const int rc = tmd_rans_encode_workspace(&Q->cap, &enc_ws, &bound)) return rc;
    for (uint32_t i = 0; i < n_frames; i++) {
        if (const int rc = pipe_check_out(Q, shapes[i], out[i])) return rc;
        if (!coded[i]) return TMD_E_ARG;
        if (coded_bytes[i] > bound) return TMD_E_CAPACITY;
        flags[i] = 0;
    }
    // the slots' buffers for coded frames, made on first use
    {
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != Q->device) HIP_TRY(hipSetDevice(Q->device));
        size_t rws = 0;
        int rc = tmd_rans_workspace(&Q->cap, 1, &rws);
        for (PipeSlot &sl : Q->slots) {
            if (rc != TMD_OK) break;
            if (!sl.dcoded) {
                if (hipMalloc(&sl.dcoded, std::max<uint64_t>(bound, 256)) != hipSuccess) { rc = TMD_E_HIP; break; }
                sl.coded_cap = bound;
            }
            if (!sl.rws && hipMalloc(&sl.rws, std::max<size_t>(rws, 256)) != hipSuccess) rc = TMD_E_HIP;
        }
        if (cur != Q->device) (void)hipSetDevice(cur);
        if (rc != TMD_OK) return rc;
    }
    return pipe_execute(Q, n_frames, shapes, out, flags, [&](uint32_t i, PipeSlot &sl) -> int {
        if (coded_bytes[i] &&
            hipMemcpyAsync(sl.dcoded, coded[i], coded_bytes[i], hipMemcpyHostToDevice, Q->up) != hipSuccess)
            return TMD_E_HIP;
        if (hipEventRecord(sl.up, Q->up) != hipSuccess) return TMD_E_HIP;
        if (hipStreamWaitEvent(sl.stream, sl.up, 0) != hipSuccess) return TMD_E_HIP;
        if (sl.used && hipStreamWaitEvent(sl.stream, sl.down, 0) != hipSuccess) return TMD_E_HIP;
        tmd_frame_out dev = sl.out;
        const uint8_t *dc = (const uint8_t *)sl.dcoded;
        return tmd_decode_rans(sl.plan, &shapes[i], &dc, &coded_bytes[i], &dev, sl.ws, sl.rws, sl.stream);
    });
}

}  // extern "C"
