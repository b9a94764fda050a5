/*
 * tmd.h -- C ABI of libtmd, TPC track-model decoding on AMD MI355X (gfx950).
 *
 * The library decodes compressed TPC time frames (arXiv:2411.02206, section 4,
 * "TPC track-model decoding on GPU"): attached clusters were stored as
 * residuals to their track, so decoding propagates every track through the
 * pad rows and adds the residuals (the paper's first GPU kernel, one thread
 * per track); unattached clusters were sorted by position and stored as
 * differences to the previous cluster, so decoding sums the differences within
 * each TPC region (the paper's second kernel, one region per thread).  The
 * track model (float32 helix propagate-and-update in the local sector frame,
 * rotation at sector crossings) is this project's own, because the paper does
 * not define one; its equations are documented with the implementation.
 *
 * Memory: every pointer in tmd_frame_in / tmd_frame_out and the workspace is
 * a DEVICE pointer owned by the caller.  The plan owns only its constant
 * tables, frame descriptors and status words.  No call waits for the GPU's
 * work except tmd_status, tmd_stage_times, tmd_free and the pipeline's
 * tmd_pipe_run / tmd_pipe_run_rans; a decode call whose frame descriptors
 * differ from the previous call's (and every tmd_decode_rans call) first
 * waits until the previous upload of the plan's descriptors (a small copy
 * from page-locked memory, enqueued by the previous call) has been made, as
 * the staging buffer is reused.
 *
 * Errors: every entry point returns TMD_OK (0) or a negative TMD_E_* code;
 * tmd_strerror() gives a message.  Argument errors are detected on the host
 * before anything is enqueued.  Data-dependent problems (inconsistent counts,
 * streams the model cannot follow) never make the decoder read or write out
 * of bounds: values are clamped or cut as documented, every output byte is
 * still defined, and the problem is reported as flag bits by tmd_status.
 */
#ifndef TMD_H
#define TMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TMD_NSEC 36                       /* 2 sides x 18 sectors */
#define TMD_NROW 152                      /* pad rows per sector */
#define TMD_NBIN (TMD_NSEC * TMD_NROW)    /* (sector,row) bins, bin = sector*152 + row */
#define TMD_MAX_TRACKS (1u << 24)         /* per frame */

/* return codes */
#define TMD_OK 0
#define TMD_E_ARG (-1)      /* null or misaligned pointer, bad size or shape */
#define TMD_E_CAPACITY (-2) /* output capacity < n_attached + n_unattached */
#define TMD_E_INPUT (-3)    /* (tmd_status) counts in the stream disagree with the shape */
#define TMD_E_STREAM (-4)   /* (tmd_status) the track model had to clamp values */
#define TMD_E_HIP (-5)      /* HIP runtime error (no device, out of memory, launch failure) */
#define TMD_E_SCRATCH (-6)  /* (tmd_decode_static) the plan's workspace exceeds TMD_STATIC_SCRATCH_BYTES */

/* status flag bits reported by tmd_status */
#define TMD_F_HDR 1u    /* track header out of range: n_clusters 0, sector >= 36 (wrapped), row >= 152 (clamped) */
#define TMD_F_SEC 2u    /* sector step >= 18 (wrapped modulo 18) */
#define TMD_F_ROW 4u    /* row left [0, 151] (clamped) */
#define TMD_F_ROT 8u    /* direction pointed backwards after a sector rotation */
#define TMD_F_SNP 16u   /* sin(phi) beyond +-0.999 or NaN (clamped, NaN -> 0) */
#define TMD_F_PAD 32u   /* decoded pad outside [0, 65535] (clamped) */
#define TMD_F_TIME 64u  /* decoded or header time outside [0, 2^24 - 1] (clamped) */
#define TMD_F_COUNT 128u /* sum of track lengths != n_attached, or sum of un_count != n_unattached:
                            streams are cut at the declared sizes */
#define TMD_F_CODED 256u /* (tmd_decode_rans) the entropy-coded input is not a well-formed coded frame of
                            its shape: the arrays decoded from it are undefined (the decode of them is
                            still safe) */

/* plan flags */
#define TMD_PLAN_GRAPH 1u   /* capture the launch sequence in a HIP graph and replay it */

typedef struct tmd_plan tmd_plan_t;

/* Sizes of one compressed frame. */
typedef struct {
    uint32_t n_tracks;     /* <= TMD_MAX_TRACKS */
    uint32_t n_attached;   /* clusters attached to tracks (sum of trk_ncls) */
    uint32_t n_unattached; /* unattached clusters (sum of un_count) */
} tmd_frame_shape;

/*
 * One compressed frame, structure of arrays (device pointers, read only).
 * Track header arrays have n_tracks entries:
 *   trk_ncls   number of clusters of the track (1..255)
 *   trk_sec0, trk_row0   sector (0..35) and pad row (0..151) of cluster 0
 *   trk_pad0   pad of cluster 0 in 1/32 pad (pad 0 is the -y edge of the row)
 *   trk_time0  time of cluster 0 in 1/32 time bin (< 2^24)
 *   trk_qpt, trk_snp, trk_tgl   q/pT * 2^10 (c/GeV), sin(phi) * 2^15, tan(lambda) * 2^12
 * Attached cluster arrays have n_attached entries, track after track, the
 * clusters of a track in order; entry 0 of a track only supplies qtot/qmax:
 *   cls_row_diff  row step from the previous cluster
 *   cls_sec_diff  sector step (0..17, modulo 18, same side) from the previous cluster
 *   cls_pad_res, cls_time_res   residual to the track prediction, 1/32 pad and 1/32 time bin
 *   cls_qtot, cls_qmax          charges, copied to the output
 * Unattached clusters: un_count[TMD_NBIN] per (sector,row) bin, then
 * n_unattached entries bin after bin; within a bin each value is the
 * difference to the previous cluster of the bin (the first to zero), time
 * modulo 2^32 and pad modulo 2^16:
 *   un_time_diff, un_pad_diff, un_qtot, un_qmax
 * Alignment: every pointer aligned to its element size.
 */
typedef struct {
    const uint8_t *trk_ncls, *trk_sec0, *trk_row0;
    const uint16_t *trk_pad0;
    const uint32_t *trk_time0;
    const int16_t *trk_qpt, *trk_snp, *trk_tgl;
    const int8_t *cls_row_diff;
    const uint8_t *cls_sec_diff;
    const int16_t *cls_pad_res, *cls_time_res;
    const uint16_t *cls_qtot, *cls_qmax;
    const uint32_t *un_count;
    const uint32_t *un_time_diff;
    const uint16_t *un_pad_diff, *un_qtot, *un_qmax;
} tmd_frame_in;

/*
 * Decoded clusters (device pointers, written).  Clusters are grouped by
 * (sector,row) bin: bin b occupies [row_offset[b], row_offset[b+1]); inside a
 * bin come first its row_nattached[b] attached clusters, in stream order
 * (track, then cluster), then its unattached clusters in stream order.
 * row_offset has TMD_NBIN + 1 entries, row_nattached TMD_NBIN.
 *   time  in 1/32 time bin, pad in 1/32 pad, qtot/qmax copied.
 * capacity: number of entries of time/pad/qtot/qmax, >= n_attached + n_unattached.
 */
typedef struct {
    uint32_t *row_offset, *row_nattached;
    uint32_t *time;
    uint16_t *pad, *qtot, *qmax;
    uint64_t capacity;
} tmd_frame_out;

typedef struct {
    float bz_tesla; /* solenoid field; the curvature of a track is q/pT * bz * 0.00299792458 per cm */
    uint32_t flags; /* TMD_PLAN_* */
} tmd_params;

/*
 * Defines: the set-up of the decode of the paper's section 4 (its first kernel
 * propagates each track through the TPC with the stored residuals; the track
 * model itself is deferred by the paper to its reference on global tracking,
 * so the float32 tables built here are those of this project's model, see the
 * implementation).  Frames of one plan are decoded together (the batched form;
 * section 4 runs several instances concurrently on streams instead).
 *
 * Prepare decoding of n_frames frames of the given shapes in one call of
 * tmd_decode (n_frames = 1: a plain single-frame decode; more: the batched
 * form, one launch sequence over all frames).  Builds the float32 constant
 * tables for p->bz_tesla on the host and uploads them to the current device.
 * *workspace_bytes receives the size of the device workspace tmd_decode needs
 * (256-byte aligned, caller-allocated, contents need not be initialised).
 * The plan reads the device's compute-unit count: a single-frame decode
 * balances its attached-decode waves over the device's SIMDs (results do not
 * depend on it).  The environment variable TMD_ATTACHED_SIMDS, if set to a
 * positive count, replaces that SIMD count (tests use it to exercise the
 * balancing on small frames).
 * Errors: TMD_E_ARG (null pointer, n_frames == 0, n_tracks > TMD_MAX_TRACKS),
 * TMD_E_HIP.
 */
int tmd_plan(const tmd_frame_shape *shapes, uint32_t n_frames, const tmd_params *p,
             tmd_plan_t **plan, size_t *workspace_bytes);

/*
 * Defines: the decoding of section 4 -- attached clusters rebuilt by
 * propagating each track and adding its residuals (the first kernel: one lane
 * per track), unattached clusters rebuilt by summing the differences within
 * each region (the second kernel: here a region is one (sector,row) bin), with
 * the indices into the structure-of-arrays input that section 4 precomputes on
 * the CPU computed here on the GPU.
 *
 * Enqueue the decode of n_frames frames (in[i], out[i] for frame i, shaped as
 * planned) on `stream` (a hipStream_t; NULL = the default stream) and return.
 * The kernels: track start offsets (scan of trk_ncls), per-cluster (sector,row)
 * keys with per-tile counts, per-bin offsets, stable ranks, attached decode,
 * unattached decode, status reduction.  Calls on one plan are serialised on
 * the device: a call enqueued on any stream waits for the previous call on the
 * same plan to finish (they share the plan's descriptor table and status
 * words), so independent work that should overlap needs plans of its own.
 * Errors: TMD_E_ARG (null plan/in/out/workspace, misaligned pointer),
 * TMD_E_CAPACITY, TMD_E_HIP.
 */
int tmd_decode(tmd_plan_t *plan, const tmd_frame_in *in, tmd_frame_out *out, void *workspace,
               void *stream);

/*
 * Defines: the decode of tmd_decode (section 4) over frames of changing sizes,
 * for a serving loop (the paper processes time frames of varying size one
 * after another; it prints no interface for this).
 *
 * As tmd_decode, for frames whose shapes (shapes[i], n_frames entries) are no
 * larger than the planned ones in every count: the plan's shapes are then
 * capacities, and one plan (and its workspace, and in TMD_PLAN_GRAPH mode its
 * captured graph) serves frames of any smaller shape, e.g. a serving loop's
 * changing batches.  A frame of shape (0, 0, 0) is an idle entry: it needs
 * only un_count (5472 zero words), row_offset and row_nattached.  The kernels
 * launched are those of the planned shapes; tiles beyond a frame's own track
 * count return at once.
 * Errors: those of tmd_decode, and TMD_E_ARG if a shape exceeds the plan's.
 */
int tmd_decode_shapes(tmd_plan_t *plan, const tmd_frame_shape *shapes, const tmd_frame_in *in,
                      tmd_frame_out *out, void *workspace, void *stream);

/*
 * Defines: the status of a decode.  The paper's decoding restores the stored
 * values exactly (section 4) and says nothing of invalid input; the flags are
 * this project's clamp-and-flag reading, under which every output byte of an
 * invalid stream is still defined.
 *
 * Flags of frame `frame` from the last tmd_decode on this plan; waits for that
 * decode to finish.  Returns TMD_OK if no flag is set, TMD_E_INPUT if
 * TMD_F_COUNT or TMD_F_CODED is set, TMD_E_STREAM if another flag is set,
 * TMD_E_ARG for a bad frame index; *flags receives the bits.
 */
int tmd_status(tmd_plan_t *plan, uint32_t frame, uint32_t *flags);

/* Release the plan and its device memory (waits for its work). NULL is a no-op.
 * (Resource management of this library; no passage of the paper defines it.) */
void tmd_free(tmd_plan_t *plan);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * tmd_decode_shapes, with the workspace taken from a scratch array of
 * TMD_STATIC_SCRATCH_BYTES that the library holds in device memory (one per
 * GPU, from the library's load until the process ends) instead of a caller
 * buffer.  shapes may be NULL (the planned shapes).  The call allocates no
 * device memory; the plan (made once by tmd_plan) and the caller's input and
 * output buffers are as for tmd_decode.  Every call on one GPU uses that GPU's
 * scratch array, and the decode needs nothing in it to be initialised; calls
 * that overlap on one GPU (other streams, other plans, or tmd_decode_static
 * beside itself) race on it and must be ordered by the caller.
 * Errors: those of tmd_decode_shapes, and TMD_E_SCRATCH if the plan's
 * workspace (the *workspace_bytes of tmd_plan) exceeds TMD_STATIC_SCRATCH_BYTES.
 */
#define TMD_STATIC_SCRATCH_BYTES (512ull << 20)
int tmd_decode_static(tmd_plan_t *plan, const tmd_frame_shape *shapes, const tmd_frame_in *in,
                      tmd_frame_out *out, void *stream);

/*
 * Host-resident frames (paper section 4, Fig. 2: per-stream transfers to the
 * GPU, decode kernels, transfers back, with the transfers of one stream
 * overlapping the kernels of another).  A pipeline owns `depth` slots
 * (1..TMD_PIPE_MAX_DEPTH); each slot has its own decode stream, a capacity
 * plan for frames up to *capacity, its workspace, and device buffers for one
 * frame's inputs and outputs.  One more stream carries every upload and
 * another every download.  All of it is allocated here (hipMalloc) and
 * released by tmd_pipe_free.  p->flags is ignored (the slots launch eagerly).
 * Errors: TMD_E_ARG (null pointer, depth out of range, n_tracks >
 * TMD_MAX_TRACKS), TMD_E_HIP (no device, out of memory).
 */
#define TMD_PIPE_MAX_DEPTH 8u
typedef struct tmd_pipe tmd_pipe_t;
int tmd_pipe_create(const tmd_frame_shape *capacity, uint32_t depth, const tmd_params *p, tmd_pipe_t **pipe);

/*
 * Decode n_frames frames held in HOST memory: in[i] has host pointers laid
 * out as tmd_frame_in describes, shaped shapes[i] (no count above the
 * pipeline's capacity), and out[i] host pointers for the outputs as
 * tmd_frame_out describes (row_offset, row_nattached, and n_attached +
 * n_unattached entries of time/pad/qtot/qmax; capacity >= that sum).  Frame i
 * goes to slot i % depth: its inputs are copied to the slot's buffers on the
 * upload stream, decoded on the slot's stream (tmd_decode_shapes), and the
 * outputs copied back on the download stream, each step ordered after the
 * previous one by events; a slot is reused once its previous frame is back.
 * Page-locked host memory
 * (hipHostMalloc, or a pinned torch tensor) lets the copies of one slot run
 * during another slot's kernels; pageable memory gives the same results
 * without that overlap.  Returns when every frame is back; flags[i] receives
 * frame i's status bits (as tmd_status).  The caller owns all host buffers;
 * they must stay valid and unchanged until the call returns.  Calls on one
 * pipeline must not overlap (one host thread at a time); separate pipelines
 * are independent.
 * Returns TMD_OK if no frame has a flag, TMD_E_INPUT if any has TMD_F_COUNT,
 * TMD_E_STREAM if any has another flag; errors: TMD_E_ARG (null pipeline,
 * null or misaligned pointer, a shape above the capacity; checked before
 * anything is enqueued), TMD_E_CAPACITY, TMD_E_HIP.
 */
int tmd_pipe_run(tmd_pipe_t *pipe, uint32_t n_frames, const tmd_frame_shape *shapes, const tmd_frame_in *in,
                 tmd_frame_out *out, uint32_t *flags);

/*
 * As tmd_pipe_run, for entropy-coded frames in HOST memory (coded[i],
 * coded_bytes[i]: the format of tmd_decode_rans): the coded bytes are what
 * crosses the bus, and each slot decodes them with tmd_decode_rans.  The
 * first call gives every slot a device buffer for coded frames up to the
 * largest size the capacity's coder may produce (tmd_rans_encode_workspace)
 * and the entropy decoding's workspace (hipMalloc, released by
 * tmd_pipe_free).  A frame whose coded data is malformed gets TMD_F_CODED
 * (TMD_E_STREAM).  Errors: as tmd_pipe_run, and TMD_E_CAPACITY if a coded
 * frame is larger than that buffer.
 */
int tmd_pipe_run_rans(tmd_pipe_t *pipe, uint32_t n_frames, const tmd_frame_shape *shapes,
                      const uint8_t *const *coded, const uint64_t *coded_bytes, tmd_frame_out *out,
                      uint32_t *flags);

/* Release a pipeline (waits for its streams). NULL is a no-op. */
void tmd_pipe_free(tmd_pipe_t *pipe);

/*
 * Defines: the compression that section 4's decode inverts: attached clusters
 * stored as residuals to their track's extrapolation, unattached clusters
 * sorted by position within their region and stored as differences to the
 * previous one.  The paper describes it only in words; this is this project's
 * encoder for its track model, the inverse of tmd_decode.
 *
 * Physical clusters (DEVICE pointers, read only): n_tracks tracks, track t
 * owning clusters [trk_first[t], trk_first[t + 1]) (trk_first[0] = 0,
 * trk_first[n_tracks] = n_clusters, non-decreasing), in the order they were
 * measured; trk_qpt = q/pT (c/GeV) and trk_tgl = tan(lambda) per track;
 * per cluster: sector (0..35), row (0..151), pad (in pads, 0 at the -y edge)
 * and time (in time bins) as doubles, the local sin(phi) of the track there
 * (used where a header is written), and the two charges.  Unattached
 * clusters: sector, row, pad, time, charges.
 */
typedef struct {
    uint32_t n_tracks, n_clusters, n_unattached;
    const uint32_t *trk_first;
    const double *trk_qpt, *trk_tgl;
    const uint8_t *cl_sec, *cl_row;
    const double *cl_pad, *cl_time, *cl_snp;
    const uint16_t *cl_qtot, *cl_qmax;
    const uint8_t *un_sec, *un_row;
    const double *un_pad, *un_time;
    const uint16_t *un_qtot, *un_qmax;
} tmd_enc_in;

/*
 * The compressed frame (DEVICE pointers, written), laid out as tmd_frame_in:
 * header arrays need n_clusters entries (a track splits into several headers
 * where the model cannot follow it), cluster arrays n_clusters (cluster i of
 * the input is cluster i of the output), unattached arrays n_unattached (in
 * bin order, sorted inside a bin by time, pad, qTot, qMax), un_count
 * TMD_NBIN.  counts: 3 device words written by the call: [0] headers
 * written (the frame's n_tracks), [1] headers opened inside a track, [2]
 * nonzero if an input was outside the codable range (pad beyond [0, 65535] or
 * time beyond [0, 2^24) in 1/32 units for attached clusters, [0, 2^32) for
 * unattached ones, a bin outside the detector, or a bad trk_first); the frame
 * is then not defined.
 */
typedef struct {
    uint8_t *trk_ncls, *trk_sec0, *trk_row0;
    uint16_t *trk_pad0;
    uint32_t *trk_time0;
    int16_t *trk_qpt, *trk_snp, *trk_tgl;
    int8_t *cls_row_diff;
    uint8_t *cls_sec_diff;
    int16_t *cls_pad_res, *cls_time_res;
    uint16_t *cls_qtot, *cls_qmax;
    uint32_t *un_count;
    uint32_t *un_time_diff;
    uint16_t *un_pad_diff, *un_qtot, *un_qmax;
    uint32_t *counts;
} tmd_enc_out;

/*
 * Bytes of device workspace tmd_encode needs for these sizes (256-byte
 * aligned, caller-allocated, contents need not be initialised).
 * Errors: TMD_E_ARG (null pointer).
 */
int tmd_encode_workspace(uint32_t n_tracks, uint32_t n_clusters, uint32_t n_unattached, size_t *bytes);

/*
 * Enqueue the encode on `stream`, with the float32 track model of the plan's
 * field (the plan's frame shapes do not matter).  Per track, every cluster is
 * quantised (rint of 32 x pad and 32 x time), the model predicts it from the
 * previous one and the residuals are stored; a new header is opened at the
 * first cluster, and wherever the row step leaves int8, the side changes, a
 * header already has 255 clusters, the prediction clamps or flags anything,
 * the cluster is not where the model puts it, or a residual leaves int16.
 * tmd_decode of the result restores the quantised clusters exactly.  The
 * unattached clusters are encoded on the plan's second stream, which forks
 * from `stream` after the call's first kernel and joins it again before the
 * call's work on `stream` ends, so the call is ordered on `stream` like a
 * single kernel.  Calls on one plan must not overlap on the host.
 * Errors: TMD_E_ARG (null or misaligned pointer), TMD_E_CAPACITY (workspace
 * too small), TMD_E_HIP; data problems are reported in out->counts[2].
 */
int tmd_encode(tmd_plan_t *plan, const tmd_enc_in *in, tmd_enc_out *out, void *workspace, size_t workspace_bytes,
               void *stream);

/*
 * Defines: the entropy decoding that comes right before the track-model
 * decoding (section 4; the paper's compressed time frames are ANS-coded, in a
 * format of its reference that this project does not have).  The coded format
 * here is this project's:
 *   - the 19 arrays of tmd_frame_in, in that order, as 39 byte planes (plane
 *     p of an array of w-byte little-endian elements holds byte p of each);
 *   - per plane a static model: frequencies f[0..255] summing to 2^12 (c_s:
 *     the sum of the frequencies below symbol s);
 *   - the plane's symbols in chunks of 64 lanes x 512 steps: symbol i of a
 *     chunk is step i / 64 of lane i % 64;
 *   - each lane is an rANS coder with a 32-bit state x in [2^16, 2^32) that
 *     is renormalised by 16-bit words, at most one per symbol, and the 64
 *     lanes of a chunk read one shared word stream.  Decoding: every lane's x
 *     starts at its stored state; step by step, and within a step lane by
 *     lane in ascending order, a lane with a symbol there takes the s whose
 *     [c_s, c_s + f_s) holds x % 2^12, sets x = f_s (x >> 12) + x % 2^12 - c_s,
 *     and, if x < 2^16, x = (x << 16) | the next word.  A chunk is well formed
 *     if at its end every x is 2^16 and every word has been read.
 * Bytes (little endian): a 64-byte header ("TMDR", version 2, n_tracks,
 * n_attached, n_unattached, 0, then zeros), the u64 offset of each of the 39
 * planes from the start, then the planes, each on a 16-byte boundary: f[256]
 * as u16, then ceil(n / 32768) + 1 u32 offsets of each chunk's data and of
 * the end of the last chunk (multiples of 16, from the start of the plane's
 * data, which is the next 16-byte boundary), then the chunks: the 64 lanes'
 * states (u32) and the word stream (u16), zero-padded to a multiple of 16
 * bytes.
 *
 * tmd_rans_workspace: bytes of the area where tmd_decode_rans puts the
 * decoded arrays of n_frames frames of these shapes (all but the unattached
 * ones) and its bookkeeping.
 * tmd_decode_rans: decode the coded frames (coded[i], coded_bytes[i]: DEVICE
 * buffers) as tmd_decode_shapes would decode the uncoded ones (shapes[i] no
 * larger than the plan's; workspace as for tmd_decode), all on `stream`: the
 * track and attached-cluster arrays are entropy-decoded into rans_workspace
 * and then decoded; the unattached clusters' arrays are entropy-decoded
 * straight into the output (their running sums and slots) once the output
 * offsets are known.  Part of the work runs on a second stream of the plan
 * (the 4-byte arrays beside the others, the unattached ones beside the
 * attached decode), which `stream` waits for.  The decode's kernels are
 * launched one by one, also for a TMD_PLAN_GRAPH plan.  A frame whose coded
 * data is malformed gets TMD_F_CODED in its status (tmd_status); its
 * malformed chunks count as zeros.
 * Errors: TMD_E_ARG (null or misaligned pointer, a shape above the plan's),
 * and those of tmd_decode_shapes.
 */
int tmd_rans_workspace(const tmd_frame_shape *shapes, uint32_t n_frames, size_t *bytes);
int tmd_decode_rans(tmd_plan_t *plan, const tmd_frame_shape *shapes, const uint8_t *const *coded,
                    const uint64_t *coded_bytes, tmd_frame_out *out, void *workspace, void *rans_workspace,
                    void *stream);

/*
 * Defines: the coding side of the format above (the paper's frames are
 * entropy-coded after the track-model encoding, section 4), on the device.
 * tmd_rans_encode_workspace: for a frame of `shape`, the workspace bytes of
 * tmd_encode_rans and the coded size it may reach (the capacity it needs).
 * tmd_encode_rans: code the frame `in` (DEVICE arrays of `shape`, as for
 * tmd_decode) into `coded` (DEVICE, `capacity` bytes, at least the bound),
 * and write the coded size to *coded_bytes (a DEVICE u64, 8-byte aligned),
 * all on `stream` of the current device.  `workspace`: DEVICE, 256-byte
 * aligned.  The model of each plane: every symbol that occurs gets
 * max(1, floor(count 2^12 / n)); while their sum is below 2^12 the symbol
 * with the smallest f n - count 2^12 gets one more, while it is above the
 * symbol with f > 1 and the largest f n - count 2^12 one less (ties: the
 * lowest symbol); a plane without symbols has f[0] = 2^12.  A chunk is
 * coded in the reverse order of its decoding (last step first, lanes
 * descending, every x starting at 2^16): before coding s a lane emits
 * x % 2^16 and shifts x right by 16 if x >= 2^20 f_s, then sets
 * x = (x / f_s) 2^12 + x % f_s + c_s; the stream is the emitted words in
 * reverse.  The bytes are those of the format above, alignment gaps zero.
 * Errors: TMD_E_ARG (null or misaligned pointer, an array of more than 2^30
 * elements), TMD_E_CAPACITY (capacity below the bound), TMD_E_HIP.
 */
int tmd_rans_encode_workspace(const tmd_frame_shape *shape, size_t *workspace_bytes, uint64_t *coded_bound);
int tmd_encode_rans(const tmd_frame_shape *shape, const tmd_frame_in *in, uint8_t *coded, uint64_t capacity,
                    uint64_t *coded_bytes, void *workspace, void *stream);

/* Static message for a return code. */
const char *tmd_strerror(int code);

/* Library version, e.g. "tmd 1.0 gfx950". */
const char *tmd_version(void);

/*
 * The float32 constant tables the decoder uses for field bz (host only, no
 * GPU needed): x, pw, inv_pw, padoff, pwq, ks, kt (152 each), cosb, sinb
 * (18 each), kb, vdq, inv_vd32, snp_max.  Returns the count written, or
 * -(count needed) if cap is too small.
 */
int tmd_tables(float bz, float *dst, int cap);

/*
 * Defines: the work split of the first kernel of section 4 (one thread per
 * track), which the paper does not tune further; these are this library's
 * scheduling knobs, picked per device and frame mix by the autotuner
 * (paper_2411_02206_amd/autotune.py).  Results never depend on them.
 *
 * Scheduling of the attached decode for later calls on the plan.
 * tracks_per_wave (64..128; 0 = 64): tracks a wave takes; above 64, the
 * tracks that start last are each decoded after a track that ends earlier, in
 * the same lane (length bucketing of tracks across the lanes).
 * persist_waves_per_simd (0..64; 0 = off): instead of one workgroup per wave
 * of work, launch a persistent grid of that many waves per SIMD which pull the
 * waves of work from per-XCD counters.  Waits for the plan's last call; a
 * TMD_PLAN_GRAPH plan captures its graph again at the next call.
 * Errors: TMD_E_ARG (null plan, a value out of range), TMD_E_HIP.
 */
int tmd_set_schedule(tmd_plan_t *plan, uint32_t tracks_per_wave, uint32_t persist_waves_per_simd);

/*
 * Stage timing.  tmd_set_profiling selects stages by bit (bit i = stage i as
 * named by tmd_stage_name; 0 = off, ~0u = all); tmd_decode then records a
 * pair of HIP events around each selected stage on its stream.  In
 * TMD_PLAN_GRAPH mode the plan captures a second graph (once per stage mask)
 * with an event-record node before and after each selected stage, and every
 * replay points those nodes at fresh events, so each call is timed on its
 * own.  The last two stages are tmd_decode_rans's entropy decoding, all its
 * frames between one pair of events each: "rans" before the track-model
 * decode, "rans_un" (the unattached arrays, decoded into the output) after
 * it.  tmd_stage_times waits for the
 * recorded calls, writes the summed milliseconds of each stage to
 * ms[0 .. n-1] (0 for unselected stages), the number of recorded calls to
 * *calls, and clears the record.  Returns the number of stages.
 */
int tmd_set_profiling(tmd_plan_t *plan, uint32_t stage_mask);
int tmd_stage_times(tmd_plan_t *plan, double *ms, uint32_t n, uint32_t *calls);
const char *tmd_stage_name(uint32_t stage);

/*
 * Arithmetic self-test on the device (device pointers, n floats each):
 * out[4i+0] = sqrtf(a[i]), out[4i+1] = a[i] / b[i], out[4i+2] = rintf(a[i]),
 * out[4i+3] = a[i] * b[i] + a[i] with two roundings.  The decoder relies on
 * these being the IEEE-754 correctly rounded results, as on the host.
 */
int tmd_selftest_fp(const float *a, const float *b, float *out, uint32_t n, void *stream);

/*
 * Self-test of the decode loop's own forms of three operations (device
 * pointers; a[n] in, out[4n] out, as raw 32-bit words):
 * out[4i+0] = square root of a[i] (meaningful for positive normal a[i], the
 * only arguments the loop gives it), out[4i+1] = a[i] clamped to the decoder's
 * |sin phi| limit with NaN -> 0, out[4i+2] = 1 if that clamp changed a[i] or
 * a[i] was NaN, else 0, out[4i+3] = rint(a[i]) as int32 clamped to
 * [-2^30, 2^30] with NaN -> 0.  Each must equal the plain definition.
 */
int tmd_selftest_math(const float *a, uint32_t *out, uint32_t n, void *stream);

/*
 * Counts into *mismatches (a device word, added to, not cleared) the floats
 * whose bit patterns lie in [lo_bits, hi_bits) for which the decode loop's
 * square root differs from the IEEE square root on the device.
 */
int tmd_selftest_sqrt(uint32_t lo_bits, uint32_t hi_bits, uint32_t *mismatches, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TMD_H */
