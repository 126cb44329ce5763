/*
 * xengine.h -- C ABI of the MI355X (gfx950) X-engine correlator.
 *
 * The correlator is the X stage of an FX correlator (Sec. I): for every
 * frequency channel it multiplies every input against every other input
 * and integrates over time (Sec. II-B), then the integrated matrix is
 * normalised for samples lost on the way (Sec. II-C).
 *
 * Data formats (all buffers are device memory unless stated otherwise, all
 * owned by the caller; the library never frees or keeps them):
 *
 *   packed     uint8 [T][F][N], time-major, then channel, then input: the
 *              channelised data of the UDP packets placed unmodified into a
 *              frame (Sec. II-A).  One byte per complex sample: high nibble
 *              = real part, low nibble = imaginary part, each offset-encoded
 *              0..15 meaning -8..7 (4+4-bit complex, Sec. I).
 *   loss_mask  uint8 [F][ceil(T/B)], one flag per channel and block of B
 *              samples, non-zero = lost.  The last block may be partial.
 *              A lost sample contributes nothing whatever its bytes hold
 *              (lost data are zeroed, Sec. II-A.2; the kernel applies the
 *              mask itself).  NULL = nothing lost.
 *   vis        int32 [F][N(N+1)/2][2], per channel the upper triangle of
 *              V[i][j] = sum over valid t of x_i * conj(x_j), i <= j,
 *              row-major packed: index(i,j) = i*N - i*(i-1)/2 + (j-i),
 *              (real, imaginary) interleaved.  8-byte aligned.
 *   count      int64 [F], valid samples integrated per channel (the packet
 *              loss counter of Sec. II-C).  8-byte aligned.
 *   out        float32 [F][N(N+1)/2][2], normalised visibilities.
 *
 * Integer sums are exact.  |Re V| <= 128 and |Im V| <= 120 per sample, so
 * int32 holds any integration of at most XE_MAX_SAMPLES valid samples; a
 * single call accepts at most that many samples (XE_ERR_OVERFLOW), and
 * keeping a running integration within it across calls is the caller's job.
 *
 * Calls are asynchronous: they validate their arguments on the host,
 * enqueue kernels on `stream` (a hipStream_t; NULL = the null stream of the
 * handle's device) and return.  They allocate nothing, and all but
 * xe_accumulate_batch and xe_batch_plan (which upload a work list) enqueue
 * kernels only and never synchronise, so they may be captured into a HIP
 * graph.  Argument errors
 * are reported before anything is enqueued; launch errors are reported as
 * XE_ERR_HIP; errors during execution surface at the caller's next
 * synchronisation.  A handle is not thread-safe: use one per host thread.
 * Nothing is thrown across the ABI.
 */
#ifndef XENGINE_H
#define XENGINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xe_handle_s *xe_handle;
typedef int32_t xe_status;

#define XE_OK 0
#define XE_ERR_ARG (-1)         /* bad size, null pointer, bad handle       */
#define XE_ERR_ALIGN (-2)       /* vis / count / out not 8-byte aligned     */
#define XE_ERR_OVERFLOW (-3)    /* T > XE_MAX_SAMPLES (int32 sums could wrap)*/
#define XE_ERR_WORKSPACE (-4)   /* batch does not fit the handle's workspace*/
#define XE_ERR_HIP (-5)         /* HIP runtime error; see xe_last_error     */
#define XE_ERR_UNSUPPORTED (-6) /* device is not gfx950                      */
#define XE_ERR_NO_DEVICE (-7)   /* validation-only handle: nothing launched */

#define XE_MAX_N 4096
#define XE_MAX_FN 4194304       /* F * N per call (bytes per sample time)  */
#define XE_MAX_SAMPLES 16777215 /* 128 * this < 2^31 */
#define XE_DEVICE_NONE (-1)

/* Create a handle on HIP device `hip_device`.  `workspace_bytes` of device
 * memory is allocated here, once, for the sums of time chunks that are
 * integrated by different workgroups (0 = the default, 1 GiB), beside 32 MB
 * for batch work lists; no later call allocates.  xe_plan_query and
 * xe_batch_query assume the default size.  With hip_device == XE_DEVICE_NONE the
 * handle is validation-only: every compute call checks its arguments and
 * then returns XE_ERR_NO_DEVICE without touching memory (for host tests).
 * Errors: XE_ERR_ARG (out == NULL), XE_ERR_HIP, XE_ERR_UNSUPPORTED. */
xe_status xe_create(xe_handle *out, int32_t hip_device, size_t workspace_bytes);

/* Free the handle and its workspace; NULL is accepted.  Work still queued
 * on the caller's streams must have finished. */
xe_status xe_destroy(xe_handle h);

/* Static text for a status code. */
const char *xe_status_string(xe_status s);

/* Text of the last error seen on this handle ("" if none); valid until the
 * next call on the handle. */
const char *xe_last_error(xe_handle h);

/* Tile geometry of frames with N <= 128 (at most four 32-input blocks).
 * The correlation of Sec. II-B runs 32 x 32 tile MFMAs in groups of eight
 * waves; a frame of at most four blocks has only the 10 tiles of a 4-block
 * triangle.  XE_GEOM_SUPER pads it to a 256-input super-block (36 tiles,
 * one 32-sample step per loop step); XE_GEOM_HALVES computes the 10 tiles
 * twice per loop step, over two consecutive 32-sample steps, and adds the
 * two halves; XE_GEOM_AUTO (the default) is XE_GEOM_HALVES.  Larger frames
 * are not affected.  Set per handle; it applies to later correlation calls
 * and to batch plans built afterwards (a plan keeps the geometry it was
 * built with).  The results are identical.  Errors: XE_ERR_ARG (NULL
 * handle, unknown value). */
#define XE_GEOM_AUTO 0
#define XE_GEOM_SUPER 1
#define XE_GEOM_HALVES 2
xe_status xe_set_geometry(xe_handle h, int32_t geometry);

/* Correlate one frame and OVERWRITE vis and count with its sums
 * (Sec. II-B: correlation of a staged frame; Sec. II-C: the loss counter).
 * 1 <= N <= XE_MAX_N, F >= 1, F * N <= XE_MAX_FN, 1 <= T <= XE_MAX_SAMPLES,
 * B >= 1. */
xe_status xe_correlate_frame(xe_handle h, const uint8_t *packed,
                             const uint8_t *loss_mask, int32_t N, int32_t F,
                             int32_t T, int32_t B, int32_t *vis,
                             int64_t *count, void *stream);

/* Correlate one frame and ADD its sums into vis and count: the kernels
 * extend the integration held in device memory, with no copy back per
 * frame (Sec. II-B).  Same arguments and limits as xe_correlate_frame. */
xe_status xe_accumulate(xe_handle h, const uint8_t *packed,
                        const uint8_t *loss_mask, int32_t N, int32_t F,
                        int32_t T, int32_t B, int32_t *vis, int64_t *count,
                        void *stream);

/* out = (float)((double)vis / (double)count[f]) element-wise, rounded once
 * to nearest; 0 where count[f] == 0 (Sec. II-C: the lost fraction applied
 * to the correlation matrix at the end of an integration).  vis and out may
 * not overlap. */
xe_status xe_normalize(xe_handle h, const int32_t *vis, const int64_t *count,
                       int32_t N, int32_t F, float *out, void *stream);

/* Per-input flags (Sec. II-C).  Besides lost packets, the F-engine flags
 * single data points (range and sampling faults).  They arrive as
 * bit-fields `flags`, uint32 [F][T][ceil(N/32)] (channel-major): bit i % 32
 * of word i / 32 is set when input i is flagged at that channel and sample;
 * bits past input N-1 in the last word are ignored.  Flagged points are
 * zeroed before correlation (xe_apply_flags), so baseline (i, j) integrates
 *     n_ij = count[f] - c_i - c_j + d_ij
 * samples, c_i = valid samples with i flagged, d_ij = valid samples with
 * both flagged (the method's per-input counters and per-sample
 * intersections).  All three calls take device pointers and are
 * capture-safe (kernels only). */

/* ADD the flag intersections of one frame into dcount, int32 [F][P], the
 * same packed upper triangle as vis: entry (i, j), i < j, counts the valid
 * samples where inputs i and j are both flagged; the diagonal entry (i, i)
 * counts those where input i is flagged (c_i).  Samples in lost blocks of
 * loss_mask (may be NULL) are not counted: their packet, footer included,
 * never arrived.  Computed on the matrix cores as a 0/1 Gram matrix per
 * channel over time; steps and blocks without flags are skipped.  Limits as
 * for xe_accumulate; flags and dcount 4-byte aligned.  Counts from several
 * frames add up exactly (integer sums). */
xe_status xe_flag_accumulate(xe_handle h, const uint32_t *flags,
                             const uint8_t *loss_mask, int32_t N, int32_t F,
                             int32_t T, int32_t B, int32_t *dcount,
                             void *stream);

/* Zero every flagged point of a frame in place: the byte becomes 0x88,
 * i.e. 0 + 0i (Sec. II-C: flagged data points are zeroed before they
 * reach the correlator).  Unflagged bytes are not written.  flags 4-byte
 * aligned; packed [T][F][N] as for xe_accumulate. */
xe_status xe_apply_flags(xe_handle h, uint8_t *packed, const uint32_t *flags,
                         int32_t N, int32_t F, int32_t T, void *stream);

/* out[f][p] = (float)((double)vis / (double)n_ij) per baseline (re and im),
 * rounded once to nearest; 0 where n_ij == 0, with
 *     n_ij = count[f] - dcount[f][(i,i)] - dcount[f][(j,j)] + dcount[f][(i,j)]
 * (Sec. II-C: the normalisation matrix, applied to the correlation matrix
 * at the end of an integration).  n_out (may be NULL) receives n_ij, int32
 * [F][P].  vis, count and dcount must cover the same frames, so that
 * n_ij >= 0.  vis, count, out and n_out 8-byte aligned (n_out 4), dcount
 * 4-byte aligned; out may not overlap vis or dcount. */
xe_status xe_normalize_flagged(xe_handle h, const int32_t *vis,
                               const int64_t *count, const int32_t *dcount,
                               int32_t N, int32_t F, float *out,
                               int32_t *n_out, void *stream);

/* Frame assembly from F-engine UDP packets (Sec. II-A: the network thread
 * places each packet's data by its sequence number, writes zeros where a
 * packet is missing, puts out-of-order packets in their own place and
 * ignores duplicates).  Packet layout, XE_PACKET_BYTES(N) bytes: a 16-byte
 * header (uint64 sequence number, uint32 stream id, uint32 input count N,
 * little-endian), the data of 4 samples x 8 bands x N inputs (one byte
 * each, in that order), then the flag bit-fields of the 4 x 8 (sample,
 * band) pairs, ceil(N/32) uint32 words each (bit i % 32 of word i / 32 =
 * input i, as for xe_flag_accumulate).  Stream stream_base + s carries
 * channels 8 s .. 8 s + 7 of the frame; the packet with sequence number
 * seq0 + k holds samples 4 k .. 4 k + 3. */
#define XE_PACKET_BYTES(N) (16 + 32 * (int64_t)(N) + 128 * (((int64_t)(N) + 31) / 32))

/* Build one frame from n_packets packets (device memory, arrival order,
 * XE_PACKET_BYTES(N) apart, 4-byte aligned): packed [T][8 n_streams][N],
 * loss_mask [8 n_streams][T/4] (block = one packet, B = 4), flags
 * [8 n_streams][T][ceil(N/32)] (may be NULL: not written).  For each
 * (stream, slot) the packet that arrived first (lowest index) is placed;
 * where none arrived the data is 0x88 (0 + 0i), the flags 0 and the block
 * lost.  Every output element is written.  stats (device, int64[6]):
 * packets inside the window, outside it (sequence number), of an unknown
 * stream, with another input count, places filled, places left empty;
 * duplicates = stats[0] - stats[4].  T a multiple of 4; the handle's
 * workspace holds 4 bytes per (stream, slot); n_packets < 2^31 - 1.
 * Capture-safe (kernels only). */
xe_status xe_assemble_frame(xe_handle h, const uint8_t *packets,
                            int64_t n_packets, int32_t N, int32_t n_streams,
                            int32_t stream_base, int64_t seq0, int32_t T,
                            uint8_t *packed, uint8_t *loss_mask,
                            uint32_t *flags, int64_t *stats, void *stream);

/* Per-input time shifting (the caption of Fig. 4, Sec. II-B, lists time
 * shifting among the extra operations of the GPU kernel stage and gives no
 * algorithm; this is an integer delay per input).  For every channel,
 *     packed_out[t][f][i] = packed_in[t - delays[i]][f][i]
 * when 0 <= t - delays[i] < T; otherwise 0x88 (0 + 0i).  flags_out
 * ([F][T][ceil(N/32)], may be NULL) receives the F-engine flags moved with
 * their data (flags_in, same layout, may be NULL = none), with the bit of
 * every sample shifted in from outside the frame set, so that
 * xe_flag_accumulate / xe_normalize_flagged count those samples out.
 * delays: device int32 [N], any values.  A channel's loss mask cannot
 * follow per-input delays: shift frames whose lost samples are already
 * flagged in flags_in, and pass no loss mask for the shifted frame.  The
 * outputs may not overlap the inputs.  Capture-safe (kernels only). */
xe_status xe_time_shift(xe_handle h, const uint8_t *packed_in,
                        const uint32_t *flags_in, const int32_t *delays,
                        int32_t N, int32_t F, int32_t T, uint8_t *packed_out,
                        uint32_t *flags_out, void *stream);

/* One correlator instance of a batch: a frame of one sub-array with its own
 * N, F, T and B, accumulated into its own vis and count.  Pointers are
 * device pointers; the array of instances itself is host memory. */
typedef struct {
    const uint8_t *packed;
    const uint8_t *loss_mask;
    int32_t N, F, T, B;
    int32_t *vis;
    int64_t *count;
} xe_instance;

/* Accumulate every instance of the batch in one persistent launch: the paper
 * pre-queues whole chains of operations to hide launch latency (Sec. II-B)
 * and several streams share one GPU (Sec. II).  The instances' work is cut
 * into items (channel x tile group x time chunk), longest first, and a grid
 * of one workgroup per compute unit drains them from a device queue.  Each
 * instance is validated as for xe_accumulate; the work list is copied to
 * one of four device slots with an asynchronous host-to-device copy from
 * pinned memory on `stream` (a slot is reused once the launch that last
 * used it has finished, which the call waits for).  Instances whose frame
 * is not 4-byte aligned or whose N is not a multiple of 4 run as plain
 * launches after the batch.  XE_ERR_WORKSPACE when the work list or the
 * time-chunk sums do not fit.  Like every call on a handle, batches must be
 * ordered on one stream (they share the handle's workspace). */
xe_status xe_accumulate_batch(xe_handle h, const xe_instance *inst,
                              int32_t n_inst, void *stream);

/* The same work list, built once and kept on the device (up to four plans
 * per handle) so that xe_batch_run can be replayed, e.g. from a captured
 * HIP graph: xe_batch_run only enqueues kernels (no copies, no host
 * synchronisation, no memset).  chunk_steps = time-chunk length in 32-sample
 * steps (0: automatic; the tuner in the Python package picks it).  The
 * halves-geometry instances, which drain in a launch of their own, take
 * shorter chunks when theirs would leave compute units idle: about their
 * total work / compute units, at least 32 steps and at most chunk_steps.  The
 * plan keeps the instances' pointers: the caller keeps those buffers alive
 * and refills them between runs.  xe_batch_plan synchronises the device
 * upload; *plan_id receives the plan. */
xe_status xe_batch_plan(xe_handle h, const xe_instance *inst, int32_t n_inst,
                        int32_t chunk_steps, int32_t *plan_id);
xe_status xe_batch_run(xe_handle h, int32_t plan_id, void *stream);
xe_status xe_batch_release(xe_handle h, int32_t plan_id);

/* Shape of a batch's work list (host only, no GPU). */
typedef struct {
    int64_t items;           /* work items in the persistent launch        */
    int32_t instances;       /* instances in the persistent launch         */
    int32_t unaligned;       /* instances run as plain launches            */
    int32_t chunk_steps;     /* time-chunk length used, in 32-sample steps */
    int64_t partial_bytes;   /* workspace for time-chunk sums              */
} xe_batch_info;

xe_status xe_batch_query(const xe_instance *inst, int32_t n_inst, int32_t n_cu,
                         int32_t chunk_steps, xe_batch_info *info);

/* How the library splits one frame into workgroups (host only, no GPU):
 * validates (N, F, T, B) as the compute calls do. */
typedef struct {
    int32_t blocks;          /* ceil(N / 32): 32-input tile edge            */
    int32_t groups;          /* workgroup tile groups per channel          */
    int32_t splits;          /* time chunks per (channel, group)           */
    int32_t steps_per_split; /* 32-sample steps per chunk                  */
    int64_t workgroups;      /* channels * groups * splits                 */
    int64_t mfma_tiles;      /* 32x32 tiles computed per channel           */
} xe_plan_info;

xe_status xe_plan_query(int32_t N, int32_t F, int32_t T, int32_t B,
                        int32_t n_cu, xe_plan_info *info);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * computation as xe_accumulate (ADD the frame's sums into vis and count,
 * same arguments and limits), on the current HIP device, without a handle:
 * nothing here calls hipMalloc, hipFree or any allocating routine.
 *
 * The partial sums of time chunks live in one static device array of
 * XE_NOALLOC_SCRATCH_BYTES per device, loaded with the library's code
 * object and held until the process ends; its address is looked up on the
 * first call on each device.  Nothing in it needs clearing between calls
 * (every chunk overwrites its own partials before they are read).  Every
 * call on a device shares that device's array, so calls that overlap on
 * one GPU (different streams, or other host threads) race: serialise them
 * on one stream.  A frame is planned into fewer time chunks when the usual
 * plan would not fit the array; a frame whose fewest possible chunks still
 * do not fit is rejected with XE_ERR_WORKSPACE before anything is touched.
 * Errors: as xe_accumulate; XE_ERR_HIP when no device is current;
 * XE_ERR_UNSUPPORTED when it is not gfx950. */
#define XE_NOALLOC_SCRATCH_BYTES (64u << 20)
xe_status xe_accumulate_noalloc(const uint8_t *packed, const uint8_t *loss_mask,
                                int32_t N, int32_t F, int32_t T, int32_t B,
                                int32_t *vis, int64_t *count, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* XENGINE_H */
