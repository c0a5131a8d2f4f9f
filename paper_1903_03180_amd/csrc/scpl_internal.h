// Internal declarations shared by the HIP kernels and the host runtime of
// libscpl.so.  Nothing here is part of the C ABI (include/scpl.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scpl {

// Rows per band of the two-level backtrack: the DP's indicator array is cut
// into bands of B rows (B <= kBandMax); for every column at the last row of
// a band the column it reaches at the last row of the previous band is
// precomputed (fits int8 because a seam moves at most one column per row).
constexpr int kBandMax = 120;
// Affected pixels of one row recomputed in parallel by the partial update.
constexpr int kUpdList = 1024;
// Luma frames are stored in tiles of kTileH rows x kTileW columns (128
// bytes, one cache line) so that the few pixels around a seam in
// consecutive rows share lines.
constexpr int kTileH = 16;
constexpr int kTileW = 8;
__host__ __device__ inline int tiles_across(int W) { return (W + kTileW - 1) / kTileW; }
__host__ __device__ inline int64_t tiled_frame_bytes(int H, int W)
{
    return (int64_t)((H + kTileH - 1) / kTileH) * tiles_across(W) * (kTileH * kTileW);
}
// Byte offset of pixel (r, c) in a tiled frame with ntc tiles per row.
__host__ __device__ inline int tofs(int r, int c, int ntc)
{
    return (((r >> 4) * ntc + (c >> 3)) << 7) + ((r & 15) << 3) + (c & 7);
}
// Frames per launch of the speculative ASDE scan.
constexpr int kSegWindow = 64;
// candidates of the first scan of a new buffer: a rejection often comes
// right after another (a scene cut leaves a one-frame buffer), and a long
// scan that ends early wastes the candidates after the rejection
constexpr int kSegRestart = 8;
// buffers per clip whose first key rows the segmentation keeps (later ones are
// computed by the energy kernel)
constexpr int kSegKeepBuffers = 4;
constexpr int kDpThreads = 1024;

// One buffer of one clip: a carving job.  Every iteration of SCPL runs on
// all jobs of a launch at once; each job advances at its own pace (k_iter
// depends on its parents) and a finished job makes every kernel return.
struct Job {
    const uint8_t *frames;  // clip, N x H x W x C
    const uint8_t *luma;    // clip luma, N tiled frames of FS bytes
    const uint8_t *seq;     // clip luma pixel-major in 16-entry pieces (seq_kernel), seqp entries per pixel
    uint8_t *out;           // clip output, N x H x Wt x C
    uint16_t *masks;        // clip masks, N x H x W, or null
    int32_t H, W, C, Wt, k, mode;
    int32_t t0, T;          // frames [t0, t0 + T) of the clip
    int32_t has_prev;       // frame t0 - 1 is the (carved) predecessor of t0
    int32_t ntc;            // luma tiles per tile row
    int64_t FS;             // bytes per tiled luma frame
    int32_t seqp;           // entries per pixel of seq: N + 1 rounded up to 16
    int32_t Wp;             // padded row pitch of the job's 2-D workspace
    int32_t Kp, KL;         // key rows: pitch, and all-ones columns left of column 0
    int32_t dpnw;           // wavefronts the banded DP needs for this job
    int32_t B;              // rows per band of the backtrack
    int32_t nb;             // bands of B rows
    int32_t kcap;           // min(k, W): room for children / seams
    int32_t logcap;         // records in log
    int32_t buffer_index;   // index of the buffer within its clip
    int32_t ring;           // persistent launch: the work ring (XCD) that serves the job
    // workspace (device)
    int16_t *M;             // column map (carved column -> original column), H x Wp, compacted in place
    uint16_t *K;            // DP input rows: 4 floor(SE / T) of carved column j at [i Kp + KL + j],
                            // 0xffff left of column 0 and at and beyond W_r; (H + 1) rows, the
                            // extra row all 0xffff; compacted in place
    uint8_t *dir;           // indicator codes 0/1/2 = predecessor column - column + 1, H x Wp,
                            // then kDirScratch bytes the DP writes discarded codes to
    int8_t *borg;           // band origins, nb x Wp
    uint16_t *bmask;        // buffer mask in original columns, H x W
    int32_t *ce_last;       // DP last row, Wp
    uint32_t *bk;           // 2 x Wp: keys of a row chunk's last row (chunked DP)
    int32_t *lab_last;      // labels of the last row, Wp (stage entry points only)
    uint64_t *keys;         // 2 x Wp scratch for the selection
    int32_t *children;      // kcap
    int32_t *bcol;          // kcap x nb: seam column at the last row of each band
    int16_t *seams;         // H x kcap: columns of the seams in each row, increasing
    int32_t *log;           // logcap x 4: (W_r, P_eff, k_iter, 0)
    int32_t *state;         // [0]: iteration at which W_r reached Wt (-1 while running),
                            // [1]: current W_r, [2]: last k_iter, [3]: current iteration
    const uint16_t *u0;     // the first key rows 4 floor(SE / T), H x W, as the segmentation left them, or
                            // null (the energy kernel computes them)
};

struct SegArgs {
    const uint8_t *luma;  // N tiled frames
    int64_t FS;           // bytes per tiled frame
    int32_t ntc;          // tiles per tile row
    uint32_t *s1;         // H x W state
    uint64_t *s2;         // H x W state
    unsigned long long *sout;  // kSegWindow sums
    int32_t H, W, mode;
    int32_t t0;           // buffer start
    int32_t tb, te;       // candidate frames [tb, te)
    int32_t init;         // 1: start the moments from frame t0
};

// A buffer the segmentation has finished, [tlo - T, tlo), whose moments S1
// cover frames up to thi (seg_finish_kernel).
struct SegFinish {
    const uint8_t *luma;  // N tiled frames
    int64_t FS;           // bytes per tiled frame
    int32_t ntc;          // tiles per tile row
    const uint32_t *s1;   // H x W moments
    uint16_t *out;        // H x W key rows
    int32_t H, W, mode;
    int32_t tlo, thi;     // frames scanned past the buffer's end
    int32_t T;            // the buffer's frames
};

// Kernel launchers (scpl_kernels.hip).  All take the stream explicitly.
void launch_luma(const uint8_t *rgb, uint8_t *y, int64_t npx, hipStream_t s);
// N frames H x W x C (C = 1 or 3, row-major) -> tiled luma
void launch_tile_luma(const uint8_t *src, int C, int N, int H, int W, uint8_t *dst, hipStream_t s);
// N tiled luma frames -> pixel-major luma: entry s = 16 c + u of pixel p =
// row W + column at seq[(c H W + p) 16 + u] is frame max(s - 1, 0) (s <= N;
// later entries, up to seqp per pixel, repeat frame N - 1)
inline int seq_pitch(int N) { return (N + 1 + 15) / 16 * 16; }
void launch_seq(const uint8_t *tiled, int N, int H, int W, uint8_t *seq, int seqp, hipStream_t s);
// N tiled luma frames -> row-major H x W
void launch_untile(const uint8_t *src, int N, int H, int W, uint8_t *dst, hipStream_t s);
// window scans of n clips (d_args: n SegArgs in device memory), one grid layer each
void launch_seg_windows(const SegArgs *d_args, int n, int ntc_max, int Hmax, hipStream_t s);
// the first key rows of finished buffers (one grid layer per SegFinish)
void launch_seg_finish(const SegFinish *d_args, int n, int ntc_max, int Hmax, hipStream_t s);
void launch_init_jobs(const Job *d_jobs, int njobs, int Hmax, int Wmax, hipStream_t s);
void launch_energy(const Job *d_jobs, int njobs, int Hmax, int Wmax, hipStream_t s);
// DP geometry of a launch, chosen from its widest job: Q columns per
// thread; banded kernels give each wavefront C = 64 Q - 2 HB owned columns
// plus HB halo columns on each side and synchronise every HB rows; key rows
// are requested PF rows ahead.  EX = 1: the workgroup reserves the whole
// LDS of its compute unit, so no other workgroup shares that unit.
struct DpGeom {
    int Q, HB, banded, PF, EX;
    int R = 0, P = 0;  // chunked (R > 0): R rows per launch, P owned columns per workgroup
    int C() const { return 64 * Q - 2 * HB; }
    int waves(int W) const { return (W + C() - 1) / C(); }
    int chunk_waves() const { return (P + 2 * R + C() - 1) / C(); }
    int groups(int W) const { return R > 0 ? (W + P - 1) / P : 1; }
    // columns at or right of column 0 the DP may read for a job of width W
    int cover(int W) const;
    int threads(int Wmax) const;
};
DpGeom dp_geom(int Wmax);  // default for the widest job of a launch
bool dp_geom_fits(const DpGeom &g, int Wmax);
extern const DpGeom kDpVariants[];
extern const int kNumDpVariants;
extern const DpGeom kDpChunked[];
extern const int kNumDpChunked;
constexpr int kKeyLeft = 64;  // all-ones key columns left of column 0 (>= every HB)
constexpr int kDirScratch = 64 * 16;  // after the indicator rows: discarded codes of one row (64 lanes x Q <= 16)
void launch_dp(const Job *d_jobs, int njobs, const DpGeom &g, int Wmax, int Hmax, hipStream_t s);
void launch_tune_fill(uint16_t *K, int H, int W, int Kp, int KL, hipStream_t s);
// band-origin variants: 0 (256 columns per workgroup), 1 (128), 2 (512)
constexpr int kNumBorgVariants = 3;
void launch_borg(const Job *d_jobs, int njobs, int nbmax, int Bmax, int Wmax, int variant, hipStream_t s);
void launch_select(const Job *d_jobs, int njobs, int use_lab_array, size_t lds_cap, hipStream_t s);
void launch_labels(const Job *d_jobs, int njobs, int Wmax, hipStream_t s);
void launch_jump_only(const Job *d_jobs, int njobs, hipStream_t s);
void launch_fill(const Job *d_jobs, int njobs, int kmax, int nbmax, int Bmax, hipStream_t s);
// fill + compaction fused per band (variant 1: 8 wavefronts per workgroup,
// 2: 16), for launches whose jobs all have 32-row bands and at most 64 seams
// per iteration (band_update_fits)
constexpr int kNumFuseVariants = 3;  // 0: fill and compaction as two launches
bool band_update_fits(int kmax, int Bmax);
void launch_band_update(const Job *d_jobs, int njobs, int nbmax, int variant, hipStream_t s);
// compaction variants: (rows per workgroup, new columns per pass); 0 is the default
extern const int kUpdateVariants[][2];
extern const int kNumUpdateVariants;
void launch_update(const Job *d_jobs, int njobs, int Hmax, int Wmax, int variant, hipStream_t s);
// refresh variants: 0 automatic, 1: 256 threads per block, 2: 1024
constexpr int kNumRefreshVariants = 3;
void launch_refresh(const Job *d_jobs, int njobs, int kmax, int Hmax, int variant, hipStream_t s);
// gather variants: 1, 2, 4 or 8 frames of a row staged per pass (fewer when
// the launch's widest rows would not fit); inb_max / outb_max: the launch's
// largest source and output row in bytes
extern const int kNumGatherVariants;
void launch_gather(const Job *d_jobs, int njobs, int Hmax, int inb_max, int outb_max, int wmax, int variant,
                   hipStream_t s);
// U (H x W int32) -> key rows; *bad |= 1 if some U is outside [0, 16382]
void launch_u_to_keys(const int32_t *src, uint16_t *dst, int H, int W, int pitch, int32_t *bad, hipStream_t s);
void launch_keys_to_u(const uint16_t *src, int32_t *dst, int H, int W, int pitch, hipStream_t s);
// N frames H x W of C-byte pixels -> N frames W x H (and of 16-bit entries)
void launch_transpose(const uint8_t *src, int N, int H, int W, int C, uint8_t *dst, hipStream_t s);
void launch_transpose16(const uint16_t *src, int N, int H, int W, uint16_t *dst, hipStream_t s);
// one frame H x W x C minus kk seams (kk x H int32 columns) -> H x (W - kk) x C
void launch_compact_frame(const uint8_t *in, int H, int W, int C, const int32_t *seams, int kk, uint8_t *out,
                          hipStream_t s);
// row-major seams (H x pitch int16) -> kk x H int32
void launch_seams_out(const int16_t *src, int pitch, int32_t *dst, int kk, int H, hipStream_t s);
// indicator codes <-> int8 {-1, 0, 1} with pitch change (stage entry points)
void launch_dir_out(const uint8_t *codes, int pitch, int8_t *dst, int H, int W, hipStream_t s);
void launch_dir_in(const int8_t *src, uint8_t *codes, int pitch, int H, int W, hipStream_t s);
// Persistent launch: every iteration of every job of a batch in one launch
// of workgroups that take work items from a ring in device memory.
constexpr int kPersistThreads = 256;
struct PState {  // scheduler of one launch, one 256-byte line per field
    int head;    // next ring slot to take
    int pad0[63];
    int tail;    // next ring slot to fill
    int pad1[63];
    int active;  // jobs still carving
    int pad2[63];
    int abort;   // set by a workgroup that waited too long for an item
    int pad3[63];
};
struct PArgs {
    const Job *jobs;
    PState *st;                // per ring (the first one's abort flag serves all)
    int *cnt;                  // per job: items of its current phase done
    unsigned long long *seq;   // per ring slot: the slot number it holds (generation), all ones when empty
    unsigned long long *item;  // per ring slot: (job << 32) | (phase << 24) | part
    int njobs;
    int nring;                 // rings: one per XCD in XCD-local mode, else one
    int xcc_ring[16];          // XCD-local mode: ring of the workgroups on each XCC_ID (-1: none)
    int cap_mask;              // slots per ring - 1 (a power of two)
    int R, P;                  // DP: rows per chunk, columns per item (P + 2 R <= 896)
    int lds_bytes;             // dynamic LDS of a workgroup (persist_lds_bytes)
    int sel_lds;               // of which the selection may use
    long long wait_ticks;      // wall-clock ticks a workgroup waits for an item before it aborts
    unsigned long long *trace; // null, or kPTrace counters summed over the workgroups (wall-clock ticks)
};
// trace counters: [2 p] ticks in items of phase p (DP, BORG, SELECT, BAND,
// REFRESH), [2 p + 1] their count; [kPTraceWait] ticks waiting for an item,
// [kPTraceWait + 1] items taken (and final waits); [kPTraceDone] ticks
// counting items done and queueing the next phases
constexpr int kPTraceWait = 10;
constexpr int kPTraceDone = 12;
constexpr int kPTrace = 13;
size_t persist_lds_bytes();
int persist_blocks_per_cu();
void launch_persist_clear(const PArgs &a, hipStream_t s);
void launch_persist_seed(const PArgs &a, hipStream_t s);
// local: the XCD-local kernel (every job's ring served by the workgroups of
// one XCD), else the agent-scope one (one ring)
void launch_persist(const PArgs &a, int grid, bool local, hipStream_t s);
// XCC_ID of each of n workgroups of a probe launch (synchronises); 0 on success
int probe_xcc(int n, int *h_out);
size_t select_lds_bytes(size_t lds_cap);
void set_kernel_attributes(size_t lds_cap);

}  // namespace scpl
