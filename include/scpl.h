/*
 * scpl.h -- C ABI of libscpl.so: SCPL video retargeting on AMD Instinct
 * MI355X (gfx950).
 *
 * Method: "Fast Video Retargeting Based on Seam Carving with Parental
 * Labeling" (C. Zhu, arXiv 1903.03180).  A clip is cut into dynamic
 * spatiotemporal buffers by the ASDE test (Sec. 3.2, eqs. 7-9); every buffer
 * is carved to the target width by repeated SCPL iterations (Sec. 3.1): the
 * uniform energy of the buffer (mean of its motion-aware energy maps, Sec.
 * 3.3) feeds the cumulative-energy DP of eq. (4), which also carries each
 * pixel's row-0 parent label; the least child of each parent (eq. 6) is
 * ranked, up to k seams are traced back and removed from every frame of the
 * buffer in one pass.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device pointers on the context's device; h_* are
 *    host pointers.  The caller owns every buffer it passes and the library
 *    never frees caller memory.  Arrays are dense, row-major, no padding.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    is asynchronous unless stated otherwise.  Entry points that return a
 *    value computed on the device to the host synchronise `stream`.
 *  - Arguments are validated before any launch; an invalid argument returns
 *    SCPL_ERR_INVALID_ARG and launches nothing.  On any error the outputs
 *    are undefined.  A device error raised by earlier asynchronous work is
 *    reported as SCPL_ERR_DEVICE by the next call that synchronises.
 *  - A context is used by one host thread at a time.
 *  - All arithmetic is exact integer arithmetic; results are bit-identical
 *    from run to run.
 *
 * Readings of points the paper leaves open (the same in every entry point):
 *  - luma Y = (77 R + 150 G + 29 B + 128) >> 8 of interleaved RGB;
 *  - gradient G = |Gx| + |Gy| of the 3x3 Sobel operator, borders replicated;
 *  - motion energy e = 2 G + 18 |Y_t - Y_{t-1}| (the 0.4 / 0.6 blend of
 *    Sec. 3.3 with the difference scaled to the gradient's range), no
 *    difference term for the clip's first frame; after carving, frame t-1 is
 *    carved with the same seams as frame t;
 *  - eq. (4) ties go to the leftmost predecessor; neighbours outside the
 *    image are skipped;
 *  - per iteration the per-parent least children are ranked by (cumulative
 *    energy, column) and k_iter = min(k, parents, width - target) of them
 *    are removed;
 *  - ASDE uses the population deviation, per pixel floor(sqrt(n S2 - S1^2));
 *    a candidate frame is rejected when ASDE > alpha * maxval * sqrt(n-1)/n
 *    (eq. 9 simplified; n counts the candidate; maxval = 1530 gradient, 7650
 *    motion), decided exactly; the rejected frame starts the next buffer;
 *  - the uniform energy is floor(sum of the buffer's energy maps / T).
 */
#ifndef SCPL_H
#define SCPL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCPL_OK = 0,
    SCPL_ERR_INVALID_ARG = 1,
    SCPL_ERR_OUT_OF_MEMORY = 2,
    SCPL_ERR_DEVICE = 3,
    SCPL_ERR_CAPACITY = 4,
    SCPL_ERR_NOT_READY = 5,
    SCPL_ERR_INTERNAL = 6
} scpl_status;

enum {
    SCPL_ENERGY_GRADIENT = 0, /* e = |Gx| + |Gy|                    (max 1530) */
    SCPL_ENERGY_MOTION = 1    /* e = 2 (|Gx| + |Gy|) + 18 |Yt - Yt-1| (max 7650) */
};

/* Limits checked by every entry point. */
#define SCPL_MAX_WIDTH 32767       /* columns fit int16 */
#define SCPL_MAX_HEIGHT 32767      /* cumulative energy fits int32 */
#define SCPL_MAX_PIXELS (1 << 27)  /* H * W, keeps the ASDE test in 128 bits */
#define SCPL_MAX_FRAMES 16384      /* frames per call */
#define SCPL_MAX_ALPHA_TERM 1024   /* alpha_num <= 1024, 1 <= alpha_den <= 1024 */
#define SCPL_MAX_DP_STAGE_HEIGHT 16383 /* scpl_dp: 4 x 16382 x H fits 32 bits */

typedef struct {
    int32_t n_frames;       /* N >= 1 */
    int32_t height;         /* H >= 1 */
    int32_t width;          /* W >= 1 */
    int32_t channels;       /* 1 (luma) or 3 (interleaved RGB), uint8 */
    int32_t target_width;   /* 1 <= Wt <= W */
    int32_t seams_per_iter; /* k >= 1; k >= W means every parent's least child (eq. 6) */
    int32_t energy_mode;    /* SCPL_ENERGY_GRADIENT or SCPL_ENERGY_MOTION */
    int32_t use_buffer;     /* 1: dynamic spatiotemporal buffer; 0: every frame alone */
    int32_t alpha_num;      /* alpha = alpha_num / alpha_den (paper: 0.15 .. 0.25) */
    int32_t alpha_den;
    int32_t max_buffer;     /* 0: unbounded (paper); > 0: force a new buffer at this length */
    int32_t target_height;  /* 0 or H: height kept; 1 <= Ht < H: horizontal seams, see below */
    int32_t memo_period;    /* 0 or 1: every buffer carved; m >= 2: seam memorisation, see below */
} scpl_params;

/* Seam memorisation (Sec. 5 names it as future work without defining it;
 * this is the library's reading).  With memo_period = m >= 2, buffer b of a
 * clip (0-based, in time order) is carved only when b mod m == 0.  Every
 * other buffer reuses the seams of buffer b - (b mod m): from each of its
 * frames exactly the pixels that buffer removed are removed, so its output
 * rows are its input rows without those pixels and its masks equal that
 * buffer's masks (iteration numbers included).  The buffer segmentation is
 * unchanged, memorised buffers add no record to scpl_last_log, and results
 * differ from m <= 1 wherever a memorised buffer's own seams would differ.
 * With a height pass the rule applies to each pass's buffers. */

typedef struct scpl_ctx scpl_ctx;

/* Create a context on HIP device `hip_device`.  The context owns a
 * workspace that grows on demand and is freed by scpl_destroy.  Creation
 * also allocates the host staging of a call with up to SCPL_MAX_FRAMES
 * frames (a few MiB of pinned memory) and the events of the plain path. */
scpl_status scpl_create(int32_t hip_device, scpl_ctx **out);
void scpl_destroy(scpl_ctx *ctx);
const char *scpl_status_str(scpl_status s);

/* Device bytes of the workspace scpl_retarget needs for one clip with
 * params p (the plain path, one buffer at a time): the tiled and
 * pixel-major luma of the clip, the buffer controller's state, one carving
 * job's workspace (bounded for every DP geometry) and, with a target height,
 * the temporaries of the height pass.  Pure host arithmetic; validates p. */
scpl_status scpl_workspace_size(const scpl_params *p, uint64_t *device_bytes);

/* Whole retarget of one clip (Secs. 3.1-3.3).
 * d_frames: N x H x W x C uint8.  d_out: N x Ht x Wt x C uint8 (Ht = H
 *   unless target_height is set).
 * d_masks (nullable): N x H x W uint16; 0 = kept, r + 1 = removed in
 *   iteration r of the frame's buffer (all frames of a buffer share a mask).
 * d_buffer_id (nullable): N int32, buffer index of each frame.
 * Height (Sec. 3.1, eq. 2: horizontal seams are vertical seams of the transposed
 * frames): with target_height Ht < H the clip is carved in width first (if
 * Wt < W), then its frames are transposed, carved from H to Ht columns the
 * same way (buffers, energies and seams of the transposed frames) and
 * transposed back.  Masks and buffer ids then describe the height pass when
 * Wt == W; when both dimensions shrink, buffer ids describe the width pass
 * and d_masks must be null.
 * h_n_buffers (nullable): receives the number of buffers.
 * d_workspace (nullable): device memory of workspace_bytes bytes (at least
 *   scpl_workspace_size(p), 256-byte aligned) that the call uses instead of
 *   the context's own workspace; owned by the caller, who keeps it alive
 *   and untouched until the work on `stream` is complete.  The call then
 *   allocates no device memory (its host staging may still grow).  Null:
 *   the context's workspace, grown on demand.  A region that is too small
 *   or misaligned returns SCPL_ERR_INVALID_ARG.
 * The segmentation step synchronises `stream` a few times; the carving is
 * asynchronous apart from one check of the iteration count per buffer.
 * Buffers are carved one after another (the plain path). */
scpl_status scpl_retarget(scpl_ctx *ctx, const scpl_params *p, const uint8_t *d_frames, uint8_t *d_out,
                          uint16_t *d_masks, int32_t *d_buffer_id, int32_t *h_n_buffers, void *d_workspace,
                          uint64_t workspace_bytes, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): scpl_retarget of
 * one clip on the plain path, with the same arguments apart from the
 * workspace and the same results, that allocates nothing.  Its device
 * workspace is a fixed array of SCPL_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends; its host staging
 * and events are made by scpl_create.
 *  - A clip whose workspace (scpl_workspace_size) exceeds
 *    SCPL_NOALLOC_SCRATCH_BYTES returns SCPL_ERR_CAPACITY and launches
 *    nothing.  Kernel timing (scpl_profile_enable) makes it return
 *    SCPL_ERR_INVALID_ARG.
 *  - Every call on one device, from any context, uses that device's one
 *    array, which keeps the last call's contents (the call initialises what
 *    it reads).  Calls whose work overlaps on one device race: issue them on
 *    one stream, or wait for the previous call's work before the next.
 *  - Synchronisation as scpl_retarget (the segmentation reads results back
 *    to the host). */
#define SCPL_NOALLOC_SCRATCH_BYTES (64u << 20)
scpl_status scpl_retarget_noalloc(scpl_ctx *ctx, const scpl_params *p, const uint8_t *d_frames, uint8_t *d_out,
                                  uint16_t *d_masks, int32_t *d_buffer_id, int32_t *h_n_buffers, void *stream);

/* Many clips at once (the batched path): every buffer of every clip is a job,
 * and each stage of an SCPL iteration runs as one launch over all jobs, the
 * iteration loop being captured once into a HIP graph and replayed.
 * Results are bit-identical to scpl_retarget on each clip alone. */
typedef struct {
    scpl_params p;
    const uint8_t *d_frames;
    uint8_t *d_out;
    uint16_t *d_masks;     /* nullable */
    int32_t *d_buffer_id;  /* nullable */
} scpl_clip;

scpl_status scpl_retarget_batch(scpl_ctx *ctx, const scpl_clip *clips, int32_t n_clips, void *stream);

/* Number of job groups of scpl_retarget_batch (default 3, at most
 * SCPL_MAX_STREAMS).  The jobs are dealt to the groups in order of
 * decreasing buffer length; each group advances in lock-step on a stream of
 * its own (default priority) that starts after the work already on the
 * caller's stream and that the caller's stream waits for.  Performance
 * only: results are identical for every count. */
#define SCPL_MAX_STREAMS 8
scpl_status scpl_batch_streams(scpl_ctx *ctx, int32_t n);

/* How scpl_retarget_batch runs the iterations of its jobs (performance
 * only: results are identical in both modes).
 * SCPL_BATCH_GROUPS (default): the job groups of scpl_batch_streams, each
 * replaying a captured graph of a few iterations (one launch per stage per
 * iteration over the group's jobs) while the host reads back the jobs'
 * states between replays.
 * SCPL_BATCH_PERSISTENT: one persistent launch for all jobs, captured as a
 * graph with the two small kernels that set up its work ring.  Its
 * workgroups take work items (a column range of a chunk of DP rows, a band
 * of the backtrack and compaction, 16 rows of the energy refresh, a job's
 * selection...) from the ring; the workgroup that finishes the last item of
 * a job's stage queues the job's next stage, so every job follows its own
 * iteration chain with no host in the loop and no lock-step between jobs
 * (Sec. 3.1 and 3.2: the same SCPL iterations, scheduled on the device).
 * On a device whose XCDs each have their own L2 cache, every job is dealt
 * to one XCD and only the workgroups running there take its items, so that
 * its data meet in one L2 and items publish their results without L2
 * write-backs; context creation checks with a probe launch that the
 * workgroups' XCD register follows the dispatcher's round robin, and
 * otherwise the batch runs as job groups.  SCPL_BATCH_PERSISTENT_AGENT (one
 * ring served by every workgroup, with agent-scope release and acquire
 * around each item) is switched off in this build: scpl_batch_mode refuses
 * it with SCPL_ERR_DEVICE.
 * A workgroup that waits longer than 4 s for an item stops the launch and
 * the call returns SCPL_ERR_INTERNAL.  Batches it does not serve (a clip
 * wider than 8192 columns) run as job groups.  The DP takes the column-split
 * chunking forced by scpl_dp_chunking when its rows R and columns P give
 * P + 2 R in (672, 896], else 256 x 384. */
enum { SCPL_BATCH_GROUPS = 0, SCPL_BATCH_PERSISTENT = 1, SCPL_BATCH_PERSISTENT_AGENT = 2 };
scpl_status scpl_batch_mode(scpl_ctx *ctx, int32_t mode);
/* Workgroups per compute unit of the persistent launch: 0 (default) as many
 * as fit at once, else at most per_cu (performance only). */
scpl_status scpl_persist_workgroups(scpl_ctx *ctx, int32_t per_cu);
/* XCDs the context's probe launch found (the persistent launch serves each
 * with a ring of its own), or 0 when XCD-local mode is unavailable and
 * SCPL_BATCH_PERSISTENT runs as job groups. */
scpl_status scpl_device_xcds(scpl_ctx *ctx, int32_t *h_n);
/* Where the last persistent launch made while kernels were timed
 * (scpl_profile_enable) spent its workgroups' time, summed over the
 * workgroups (device wall clock): h_ms[0..4] in items of the DP, band
 * origins, selection, band trace and compaction, and energy refresh, with
 * h_items[0..4] their counts; h_ms[5] waiting for an item (h_items[5]:
 * items taken, and the final waits); h_ms[6] counting items done and
 * queueing the next stages (h_items[6] = h_items[5]).  7 entries each.
 * SCPL_ERR_NOT_READY before any such launch. */
scpl_status scpl_persist_stats(scpl_ctx *ctx, double *h_ms, int64_t *h_items);

/* ---- request server (continuous batching) ----
 * Retarget requests are queued in arrival order.  Each of `lanes` worker
 * threads owns a context and a stream; whenever a lane is free it takes the
 * queued requests that fit the device-memory budget (in order, at most
 * max_batch) and retargets them as one batch (as scpl_retarget_batch, with
 * one job group on the lane's stream).
 * A request is admitted by an upper bound of the device memory its batch
 * share can claim (its tiled and pixel-major luma and buffer controller
 * plus one carving job per frame); the admitted requests' bounds never
 * exceed hbm_budget.
 * A request is done as soon as its own buffers are carved and its outputs
 * gathered (its gather runs beside the rest of the batch), unless
 * whole_batch is set: then every request of a batch is done when the batch
 * is.  Its bound counts against the budget until its batch ends.
 * Requests that arrive while batches run are admitted as lanes and memory
 * free up, and their work overlaps on the device with the batches in
 * flight.  Results are bit-identical to scpl_retarget on each clip alone.
 *
 * scpl_server_create: lanes in [1, SCPL_MAX_LANES], max_batch >= 1,
 *   hbm_budget in bytes (0: half the device memory free at creation).
 * scpl_server_submit: the clip's frames must be complete on the device and
 *   every buffer of the clip stays owned by the caller, untouched by the
 *   caller until the request is done.  Returns a ticket; SCPL_ERR_CAPACITY
 *   if the request's bound exceeds the whole budget (nothing is queued).
 * scpl_server_poll: *h_done = 1 once the outputs are complete on the device;
 *   *h_result (nullable) is then the request's status (SCPL_ERR_NOT_READY
 *   before, or for a request dropped by scpl_server_destroy).
 * scpl_server_wait: blocks until the request is done.
 * scpl_server_ticket_times: host steady-clock milliseconds from submission
 *   to the start of the request's batch and to its completion (done only).
 * scpl_server_release: forgets a done ticket (SCPL_ERR_NOT_READY while the
 *   request runs or another thread still waits on it).
 * scpl_server_destroy: requests already running finish; queued ones are
 *   dropped; then the lanes' contexts are destroyed. */
#define SCPL_MAX_LANES 16
typedef struct scpl_server scpl_server;
typedef struct {
    int32_t lanes;
    int32_t max_batch;
    uint64_t hbm_budget;
    int32_t whole_batch; /* 1: requests are done with their batch; 0 (default): with their own buffers */
} scpl_server_config;
scpl_status scpl_server_create(int32_t hip_device, const scpl_server_config *cfg, scpl_server **out);
scpl_status scpl_server_submit(scpl_server *srv, const scpl_clip *clip, int64_t *h_ticket);
scpl_status scpl_server_poll(scpl_server *srv, int64_t ticket, int32_t *h_done, scpl_status *h_result);
scpl_status scpl_server_wait(scpl_server *srv, int64_t ticket, scpl_status *h_result);
scpl_status scpl_server_ticket_times(scpl_server *srv, int64_t ticket, double *h_queue_ms, double *h_total_ms);
scpl_status scpl_server_release(scpl_server *srv, int64_t ticket);
void scpl_server_destroy(scpl_server *srv);
/* The admission bound of a request with params p (bytes; host arithmetic). */
scpl_status scpl_server_footprint(const scpl_params *p, uint64_t *h_bytes);

/* Per-iteration record of the last scpl_retarget / scpl_retarget_batch call:
 * for every buffer in order, for every iteration, four int32
 * (buffer index within its clip, W_r, P_eff, k_iter); clips in order.
 * Copies at most `cap` records into h_log and stores the total in *h_count. */
scpl_status scpl_last_log(scpl_ctx *ctx, int32_t *h_log, int64_t cap, int64_t *h_count);

/* ---- kernel timing (measurement) ----
 * When enabled, every launch of the library's kernels is bracketed by a pair
 * of HIP events recorded on the launch stream, and graph capture in
 * scpl_retarget_batch is skipped (the kernels are launched one by one).
 * scpl_profile_read synchronises the device, returns the summed duration
 * and launch count of one kernel kind since profiling was (re)enabled. */
enum {
    SCPL_KERNEL_LUMA = 0,    /* colour -> tiled luma */
    SCPL_KERNEL_SEGMENT = 1,
    SCPL_KERNEL_ENERGY = 2,
    SCPL_KERNEL_DP = 3,
    SCPL_KERNEL_BORG = 4,
    SCPL_KERNEL_SELECT = 5,
    SCPL_KERNEL_FILL = 6,
    SCPL_KERNEL_UPDATE = 7,  /* column-map compaction + energy update */
    SCPL_KERNEL_GATHER = 8,
    SCPL_KERNEL_INIT = 9,
    SCPL_KERNEL_REFRESH = 10, /* energies of the pixels whose neighbourhood changed */
    SCPL_KERNEL_PERSIST = 11, /* the persistent launch of SCPL_BATCH_PERSISTENT */
    SCPL_KERNEL_COUNT = 12
};
scpl_status scpl_profile_enable(scpl_ctx *ctx, int32_t on);
scpl_status scpl_profile_read(scpl_ctx *ctx, int32_t kernel, double *h_total_ms, int64_t *h_launches);
/* Which kernel kinds the timing brackets: bit k set = SCPL_KERNEL_k is
 * bracketed (default: all).  The others then run without events, which
 * keeps the instrumentation of a timed run to the kinds it needs.  Takes
 * effect at the next launch; bits at or above SCPL_KERNEL_COUNT are an
 * error. */
scpl_status scpl_profile_kinds(scpl_ctx *ctx, uint32_t mask);

/* ---- DP geometry and its autotuner (performance only: every geometry
 * gives bit-identical results) ----
 * The cumulative-energy DP of eq. (4) runs one workgroup per buffer; each
 * wavefront owns a run of columns, computes HB halo columns on each side with
 * Q columns per lane, meets the others every HB rows, and requests its
 * energy rows PF rows ahead.  EX = 1 makes each DP workgroup reserve the
 * whole LDS of its compute unit, so that no other workgroup (another
 * buffer's DP, or a concurrent stream's work) shares the unit.
 * scpl_dp_geometry forces (Q, HB, PF, EX) for every later launch it fits
 * (Q = 0: automatic; PF = 0: the default depth of (Q, HB)).  Valid (Q, HB,
 * PF): (2,8,8) (2,8,16) (4,8,8) (4,8,16) (4,16,8) (4,16,16) (8,16,4)
 * (8,16,8) (8,16,16) (8,32,4) (8,32,8) (16,32,2) (16,32,4) (16,32,8)
 * (16,64,2) (16,64,4), and (32,0,2) for the row-synchronous kernel; EX is
 * 0 or 1.
 * scpl_autotune_dp times every geometry that fits width W (the ones above
 * and a few column-split ones) with n_jobs
 * concurrent H x W synthetic energies per launch (as in a batched launch;
 * null stream, synchronises) and keeps the fastest for launches whose widest
 * job has width W; when the batched path runs more than one job group
 * (scpl_batch_streams) only EX = 1 geometries are timed.  Choices made for
 * several n_jobs at one width are all kept: a launch takes the one timed with
 * the nearest number of concurrent jobs (by ratio), counting every job of a
 * batched call, and one job for the plain path and the stage calls.  h_Q, h_HB, h_PF,
 * h_EX, h_us (nullable) receive the choice and its time per launch in
 * microseconds. */
scpl_status scpl_dp_geometry(scpl_ctx *ctx, int32_t Q, int32_t HB, int32_t PF, int32_t EX);
/* Column-split DP: every buffer's DP runs as one launch per R rows, with a
 * workgroup per P owned columns (each covering R more columns on either
 * side, which stay exact for the R rows).  scpl_dp_chunking(ctx, R, P)
 * applies to the geometry last forced by scpl_dp_geometry (R = 0: one
 * launch of one workgroup per buffer again); valid for (Q, HB, PF) in
 * (4,16,8) (4,16,16) (2,8,16) (4,8,8) with R and P multiples of Q, R >= HB,
 * and a cover of P + 2R columns that the workgroup's wavefronts can hold.
 * scpl_dp_chosen writes the geometry used for launches whose widest job has
 * width W and that run the most concurrent jobs any choice at W was timed
 * with: h_geom[6] = (Q, HB, PF, EX, R, P).
 * Without a forced or tuned geometry: (2,8,8) for W <= 448; up to W = 8960
 * the column-split (2,8,16) with EX = 1, R = 192 and P = 64 for launches of
 * at most four jobs, else the column-split (4,16,8) with EX = 1, R = 256 and
 * P = 384 (what scpl_dp_chosen reports); the row-synchronous kernel beyond. */
scpl_status scpl_dp_chunking(scpl_ctx *ctx, int32_t R, int32_t P);
scpl_status scpl_dp_chosen(scpl_ctx *ctx, int32_t W, int32_t *h_geom);
scpl_status scpl_autotune_dp(scpl_ctx *ctx, int32_t H, int32_t W, int32_t n_jobs, int32_t *h_Q, int32_t *h_HB,
                             int32_t *h_PF, int32_t *h_EX, double *h_us);

/* ---- launch variants and the batch autotuner (performance only: every
 * variant gives bit-identical results) ----
 * scpl_kernel_variants picks the compaction kernel's shape, update_variant
 * in [0, 7): rows per workgroup x new columns per pass of (4 x 2048) (the
 * default), (2 x 2048), (8 x 2048), (4 x 1024), (8 x 1024), (1 x 2048),
 * (2 x 1024); the energy refresh kernel's workgroup, refresh_variant 0
 * (automatic: 1024 threads when a launch has few workgroups, else 256), 1
 * (256) or 2 (1024); the band-origin kernel's columns per workgroup,
 * borg_variant 0 (256), 1 (128) or 2 (512); and the output gather's
 * frames per pass (rows of that many frames staged in LDS together),
 * gather_variant 0 (1), 1 (2), 2 (4) or 3 (8), fewer when the rows do not
 * fit 64 KiB, or 4 (the default): each row streamed over its frames, two
 * wavefronts loading rows two frames ahead and two assembling and storing
 * them (rows that are not 16-byte multiples or exceed 16 KiB as variant 0);
 * and whether the seam trace within bands and the compaction
 * run as two launches (fuse_variant 0) or as one kernel per band of rows
 * with 8 (1) or 16 (2) wavefronts per workgroup, which serves launches whose
 * buffers all have 32-row bands and at most 64 seams per iteration (the
 * others run the two launches).
 * scpl_autotune_batch times whole batched retargets of the given clips
 * (writing their outputs, identically, each time) and keeps the fastest
 * configuration for later batched calls of the context: first the number of
 * job groups (2, 3, 4) together with the DP geometry (the one launches would
 * take without it, the single-workgroup (8,16,8) and (4,16,16), the
 * column-split (4,16,8) with 256 rows x 384 columns and (2,8,16) with 128 x
 * 640, all with EX = 1), then the compaction variant, then the refresh
 * variant, then the band-origin and fused variants, then (where the context
 * found the XCDs) the persistent launch (SCPL_BATCH_PERSISTENT) with its DP
 * chunked 256 x 384, 192 x 512 or 128 x 640 and as many workgroups per
 * compute unit as fit, or one or two fewer, then the gather variant; each
 * candidate is run once untimed and then `reps` times, and its best time
 * counts.  The
 * configuration the calls would use before the call is timed first, and a
 * candidate replaces the best so far only when it is at least 1% faster
 * (so that run-to-run noise does not decide the choice).  Synchronises
 * `stream`.  h_choice (nullable, 15 int32): job groups, Q, HB, PF, EX, R, P
 * of the DP geometry (Q = 0: not forced), compaction variant, refresh
 * variant, 1 if a DP geometry is forced for batched calls, band-origin
 * variant, gather variant, fused variant, batch mode (scpl_batch_mode),
 * workgroups of the persistent launch; *h_ms (nullable): the best time of a
 * whole retarget in milliseconds.  A geometry forced with scpl_dp_geometry takes
 * precedence over the batch choice, and the batch autotuner then returns
 * SCPL_ERR_INVALID_ARG, as it does with kernel timing enabled. */
scpl_status scpl_kernel_variants(scpl_ctx *ctx, int32_t update_variant, int32_t refresh_variant,
                                 int32_t borg_variant, int32_t gather_variant, int32_t fuse_variant);
scpl_status scpl_autotune_batch(scpl_ctx *ctx, const scpl_clip *clips, int32_t n_clips, int32_t reps,
                                int32_t *h_choice, double *h_ms, void *stream);

/* ---- stage entry points (parity checks of single stages) ---- */

/* Luma of npx interleaved RGB pixels (reading of the colour step). */
scpl_status scpl_luma(scpl_ctx *ctx, const uint8_t *d_rgb, int64_t npx, uint8_t *d_y, void *stream);

/* Energy map of one H x W frame, Sec. 3.3.  d_yprev is nullable (no
 * difference term).  d_e: H x W int32. */
scpl_status scpl_energy(scpl_ctx *ctx, int32_t H, int32_t W, int32_t mode, const uint8_t *d_y,
                        const uint8_t *d_yprev, int32_t *d_e, void *stream);

/* Cumulative energy, eq. (4), with parent labels (Sec. 3.1) and the
 * indicator array.  d_u: H x W int32 in [0, 16382] (the DP keeps 4 U in 16
 * bits per column; the largest uniform energy is 7650), H <= 16383 (so that
 * 4 x the cumulative energy fits 32 bits).  A value of d_u outside
 * [0, 16382] returns SCPL_ERR_INVALID_ARG: the values are checked on the
 * device (one launch and a synchronisation) before the DP runs, and the
 * outputs are then left untouched.  d_ce_last, d_label_last:
 * W int32 (last row).  d_dir: H x W int8 in {-1, 0, 1} (predecessor column
 * minus column; row 0 is 0). */
scpl_status scpl_dp(scpl_ctx *ctx, int32_t H, int32_t W, const int32_t *d_u, int32_t *d_ce_last,
                    int32_t *d_label_last, int8_t *d_dir, void *stream);

/* Per-parent least child (eq. 6) and the k_iter = min(k, P_eff, limit) least
 * of them by (cumulative energy, column), from the DP's last row.
 * d_children: at least min(k, W) int32, k_iter columns in increasing order.
 * h_kiter, h_peff: host results (synchronises `stream`).  Labels must be a
 * DP's labels (non-decreasing, in [0, W)). */
scpl_status scpl_select(scpl_ctx *ctx, int32_t W, const int32_t *d_ce_last, const int32_t *d_label_last,
                        int32_t k, int32_t limit, int32_t *d_children, int32_t *h_kiter, int32_t *h_peff,
                        void *stream);

/* Trace kk children back through the indicator array (Sec. 3.1).
 * d_dir: H x W int8 from scpl_dp.  d_children: kk int32 in increasing order.
 * d_seams: kk x H int32, d_seams[s*H + i] = column of seam s in row i. */
scpl_status scpl_backtrack(scpl_ctx *ctx, int32_t H, int32_t W, const int8_t *d_dir, const int32_t *d_children,
                           int32_t kk, int32_t *d_seams, void *stream);

/* ASDE test of one candidate buffer (Sec. 3.2, eqs. 7-9): the n frames of
 * d_luma (n x H x W luma) with d_prev (nullable, H x W: the frame before
 * them, for the difference term of the first; motion energy only).
 * *h_S = sum over pixels of floor(sqrt(n S2 - S1^2)) (S1, S2: sums of the n
 * energies and of their squares; n times the population deviation of
 * eq. 8); *h_reject = 1 iff ASDE = S / (n H W) exceeds phi(n) of eq. (9)
 * with alpha = alpha_num / alpha_den (decided exactly in integers).
 * Synchronises `stream`. */
scpl_status scpl_asde(scpl_ctx *ctx, int32_t n, int32_t H, int32_t W, int32_t mode, const uint8_t *d_luma,
                      const uint8_t *d_prev, int32_t alpha_num, int32_t alpha_den, int64_t *h_S, int32_t *h_reject,
                      void *stream);

/* One-pass removal of kk seams from one frame (Sec. 3.1): d_in H x W x C
 * uint8 (C = 1 or 3), d_seams kk x H int32 with d_seams[s*H + i] the column
 * of seam s in row i (strictly increasing in s in every row, as
 * scpl_backtrack returns them; entries that break this give an undefined
 * but in-bounds result), 0 <= kk < W.  d_out: H x (W - kk) x C. */
scpl_status scpl_compact(scpl_ctx *ctx, int32_t H, int32_t W, int32_t C, const uint8_t *d_in, const int32_t *d_seams,
                         int32_t kk, uint8_t *d_out, void *stream);

/* Buffer segmentation alone (Sec. 3.2) on N x H x W luma.
 * h_buffer_id: N int32 (host).  h_s_trace (nullable, host): N int64, the
 * ASDE sum S of each tested candidate, -1 where no test was made.
 * Synchronises `stream`. */
scpl_status scpl_segment(scpl_ctx *ctx, const scpl_params *p, const uint8_t *d_luma, int32_t *h_buffer_id,
                         int64_t *h_s_trace, int32_t *h_n_buffers, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SCPL_H */
