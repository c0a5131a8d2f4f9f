// Host runtime of libscpl.so: argument validation, workspace, the ASDE
// buffer controller (Sec. 3.2), the SCPL iteration driver (Sec. 3.1) for the
// plain path (one buffer at a time) and the batched path (every buffer of
// every clip per launch, the iteration loop replayed from a HIP graph), and
// the stage entry points.  Declarations: include/scpl.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/scpl.h"
#include "scpl_internal.h"
#include "scpl_runtime.h"

using namespace scpl;

struct ProfPair {
    hipEvent_t a, b;
    int kind;
};

struct scpl_ctx {
    DpGeom forced{0, 0, 0, 0, 0};                       // DP geometry forced by the caller (Q = 0: none)
    struct Tuned {
        int W, n;  // widest-job width, concurrent jobs the timing launched
        DpGeom g;
    };
    std::vector<Tuned> tuned;  // autotuned geometries
    bool profiling = false;
    uint32_t prof_mask = ~0u;  // kernel kinds bracketed when profiling
    std::vector<ProfPair> prof_pending;  // recorded, not yet read
    std::vector<ProfPair> prof_free;     // reusable event pairs
    double prof_ms[SCPL_KERNEL_COUNT] = {};
    int64_t prof_n[SCPL_KERNEL_COUNT] = {};
    int device = 0;
    size_t lds_cap = 65536;
    void *ws = nullptr;        // device workspace: tiled luma, buffer controller, stage jobs
    size_t ws_size = 0;
    void *jws = nullptr;       // device workspace of the carving jobs
    size_t jws_size = 0;
    void *tws = nullptr;       // device temporaries of height retargeting
    size_t tws_size = 0;
    void *pinned = nullptr;    // host staging (job tables, sums, states)
    size_t pinned_size = 0;
    bool fixed_ws = false;     // ws / jws / tws point into a caller's region: never grown or freed
    bool fixed_pinned = false; // the host staging is never grown
    void *scratch = nullptr;   // this device's no-allocation workspace (device address of `scratch`)
    std::vector<int32_t> last_log;
    int nstreams = 3;                    // job groups of the batched path, one stream each
    DpGeom batch_forced{0, 0, 0, 0, 0};  // DP geometry the batch autotuner chose (Q = 0: none)
    int upd_variant = 0;                 // compaction kernel variant (kUpdateVariants)
    int refresh_variant = 0;             // refresh kernel variant (0 automatic)
    int borg_variant = 0;                // band-origin kernel variant
    int gather_variant = 4;              // gather kernel variant (frames per pass; 4: streamed)
    int fuse_variant = 0;                // fill + compaction: 0 two launches, 1/2 fused per band
    int batch_mode = SCPL_BATCH_GROUPS;  // how the batched path runs its iterations
    int persist_grid = 0;                // workgroups of the persistent launch (resident at once)
    int persist_max_per_cu = 0;          // of which per compute unit
    int ncu = 0;                         // compute units
    int nxcd = 0;                        // XCDs the probe found, 0: XCD-local mode unavailable
    int xcc_ring[16] = {};               // their XCC_IDs' rings
    long long wall_khz = 0;              // device wall clock (the persistent launch's wait bound)
    unsigned long long persist_trace[kPTrace] = {};  // the last timed persistent launch's counters
    bool persist_traced = false;
    std::vector<hipStream_t> gstreams;   // their streams (default priority)
    std::vector<hipEvent_t> gevents;     // one per group
    // per job group: its iteration graph and the launch arguments it was
    // captured with; a later call with the same arguments replays it
    struct GraphCache {
        std::vector<int64_t> key;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        void release()
        {
            if (ge) (void)hipGraphExecDestroy(ge);
            if (g) (void)hipGraphDestroy(g);
            ge = nullptr;
            g = nullptr;
            key.clear();
        }
    };
    std::vector<GraphCache> gcache;
    hipEvent_t fork = nullptr;           // groups start after the caller's stream reaches it
    hipEvent_t side_in = nullptr, side_out = nullptr;  // pixel-major lumas beside the segmentation
    hipStream_t gather_stream = nullptr;  // gathers of clips done early (default priority)
    std::vector<hipEvent_t> clip_events;  // one per clip gathered early
    hipEvent_t gathers_done = nullptr;
};

namespace {

typedef unsigned __int128 u128;

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

scpl_status dev_status(hipError_t e)
{
    if (e == hipSuccess) return SCPL_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SCPL_ERR_OUT_OF_MEMORY;
    return SCPL_ERR_DEVICE;
}

inline scpl_status dev_status(scpl_status s) { return s; }

#define SCPL_TRY(expr)                                     \
    do {                                                   \
        scpl_status st__ = dev_status((expr));             \
        if (st__ != SCPL_OK) return st__;                  \
    } while (0)

#define SCPL_CHECK_LAUNCH() SCPL_TRY(hipGetLastError())

scpl_status validate(const scpl_params *p)
{
    if (!p) return SCPL_ERR_INVALID_ARG;
    if (p->n_frames < 1 || p->n_frames > SCPL_MAX_FRAMES) return SCPL_ERR_INVALID_ARG;
    if (p->height < 1 || p->height > SCPL_MAX_HEIGHT) return SCPL_ERR_INVALID_ARG;
    if (p->width < 1 || p->width > SCPL_MAX_WIDTH) return SCPL_ERR_INVALID_ARG;
    if ((int64_t)p->height * p->width > SCPL_MAX_PIXELS) return SCPL_ERR_INVALID_ARG;
    if (p->channels != 1 && p->channels != 3) return SCPL_ERR_INVALID_ARG;
    if (p->target_width < 1 || p->target_width > p->width) return SCPL_ERR_INVALID_ARG;
    if (p->seams_per_iter < 1) return SCPL_ERR_INVALID_ARG;
    if (p->energy_mode != SCPL_ENERGY_GRADIENT && p->energy_mode != SCPL_ENERGY_MOTION) return SCPL_ERR_INVALID_ARG;
    if (p->use_buffer != 0 && p->use_buffer != 1) return SCPL_ERR_INVALID_ARG;
    if (p->alpha_num < 0 || p->alpha_num > SCPL_MAX_ALPHA_TERM) return SCPL_ERR_INVALID_ARG;
    if (p->alpha_den < 1 || p->alpha_den > SCPL_MAX_ALPHA_TERM) return SCPL_ERR_INVALID_ARG;
    if (p->max_buffer < 0) return SCPL_ERR_INVALID_ARG;
    if (p->target_height < 0 || p->target_height > p->height) return SCPL_ERR_INVALID_ARG;
    if (p->memo_period < 0 || p->memo_period > SCPL_MAX_FRAMES) return SCPL_ERR_INVALID_ARG;
    return SCPL_OK;
}

int32_t energy_max(int mode) { return mode == SCPL_ENERGY_GRADIENT ? 1530 : 7650; }

// Eq. (9) test: ASDE = S / (n H W) > alpha * maxval * sqrt(n - 1) / n,
// i.e. (S * aden)^2 > (anum * maxval * H W)^2 * (n - 1), exact in 128 bits
// under the limits of include/scpl.h.
bool asde_rejects(uint64_t S, int64_t n, int64_t npx, int32_t emax, int32_t anum, int32_t aden)
{
    if (n <= 1) return false;
    u128 lhs = (u128)S * (u128)(uint64_t)aden;
    lhs *= lhs;
    u128 b = (u128)(uint64_t)anum * (uint64_t)emax * (uint64_t)npx;
    return lhs > b * b * (u128)(uint64_t)(n - 1);
}

// ---------------------------------------------------------------- workspace

struct Bump {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count)
    {
        T *p = reinterpret_cast<T *>(base + off);
        off += align_up(count * sizeof(T));
        return p;
    }
};

// Rows per band: 32 (short band walks), or more for tall and wide frames so
// that the band origins of a whole frame (bands x width bytes) still fit in
// the selection kernel's LDS next to its keys (16 bytes per column); int8
// offsets cap it at 120.
int32_t band_rows(int32_t H, int32_t W, size_t lds_cap)
{
    const size_t keys = (size_t)16 * W;
    for (int32_t B : {32, 64, 96, 120}) {
        const size_t nb = (size_t)(H + B - 1) / B;
        if (keys + nb * (size_t)W <= lds_cap) return B;
    }
    return kBandMax;
}

size_t g_lds_cap = 65536;  // set from the device at context creation

// Columns right of the width that the DP may read under any geometry: a
// banded workgroup covers at most W + C + HB (C <= 1024), the row-synchronous
// kernel at most W + 64 Q (Q = 32), a column-split one at most W + 16 waves x
// C + HB (C <= 256).
constexpr int32_t kCoverSlack = 16 * 256 + 64;

struct JobShape {
    int32_t H, W, Wt, k;
    DpGeom g;  // DP geometry of the launch the job runs in
    bool bound = false;  // sizes for every geometry and band height (workspace bounds)
    int32_t band = 0;    // rows per band forced (the persistent launch: 32), 0: by the frame size
    int32_t Wp() const { return (int32_t)align_up((size_t)W, 64); }
    const DpGeom &geom() const { return g; }
    int32_t Kp() const
    {
        return kKeyLeft + (int32_t)align_up((size_t)(bound ? W + kCoverSlack : geom().cover(W)), 64);
    }
    int32_t B() const { return bound ? 32 : band > 0 ? band : band_rows(H, W, g_lds_cap); }
    int32_t nb() const { return (H + B() - 1) / B(); }
    int32_t kcap() const { return std::min(k, W); }
    int32_t logcap() const { return W - Wt + 2; }
};

size_t job_bytes(const JobShape &s)
{
    const size_t H = s.H, Wp = s.Wp(), W = s.W, nb = s.nb(), kc = s.kcap(), lc = s.logcap();
    size_t b = 0;
    b += align_up(H * Wp * 2);           // M
    b += align_up((H + 1) * (size_t)s.Kp() * 2);  // K
    b += align_up(H * Wp + kDirScratch);  // dir + scratch row of discarded codes
    b += align_up(nb * Wp);              // borg
    b += align_up(H * W * 2);            // bmask
    b += 2 * align_up(Wp * 4);           // ce_last, lab_last
    b += align_up(2 * Wp * 4);           // bk
    b += align_up(2 * Wp * 8);           // keys
    b += align_up(kc * 4);               // children
    b += align_up(kc * nb * 4);          // bcol
    b += align_up(kc * H * 2);           // seams
    b += align_up(lc * 16);              // log
    return b;
}

void carve_job(Job &J, const JobShape &s, Bump &bp, int32_t *state)
{
    const size_t H = s.H, Wp = s.Wp(), W = s.W, nb = s.nb(), kc = s.kcap(), lc = s.logcap();
    J.H = s.H;
    J.W = s.W;
    J.Wt = s.Wt;
    J.k = s.k;
    J.Wp = (int32_t)Wp;
    J.Kp = s.Kp();
    J.KL = kKeyLeft;
    J.dpnw = s.geom().banded ? s.geom().waves(s.W) : 0;
    J.B = s.B();
    J.nb = (int32_t)nb;
    J.kcap = (int32_t)kc;
    J.logcap = (int32_t)lc;
    J.M = bp.take<int16_t>(H * Wp);
    J.K = bp.take<uint16_t>((H + 1) * (size_t)J.Kp);
    J.dir = bp.take<uint8_t>(H * Wp + kDirScratch);
    J.borg = bp.take<int8_t>(nb * Wp);
    J.bmask = bp.take<uint16_t>(H * W);
    J.ce_last = bp.take<int32_t>(Wp);
    J.lab_last = bp.take<int32_t>(Wp);
    J.bk = bp.take<uint32_t>(2 * Wp);
    J.keys = bp.take<uint64_t>(2 * Wp);
    J.children = bp.take<int32_t>(kc);
    J.bcol = bp.take<int32_t>(kc * nb);
    J.seams = bp.take<int16_t>(kc * H);
    J.log = bp.take<int32_t>(lc * 4);
    J.state = state;
}

scpl_status grow(void *&buf, size_t &size, size_t bytes, bool fixed)
{
    if (bytes <= size) return SCPL_OK;
    if (fixed) return SCPL_ERR_CAPACITY;  // a caller's region is never replaced
    if (buf) {
        SCPL_TRY(hipFree(buf));  // implicitly waits for work using it
        buf = nullptr;
        size = 0;
    }
    size_t want = align_up(bytes, (size_t)1 << 20);
    SCPL_TRY(hipMalloc(&buf, want));
    size = want;
    return SCPL_OK;
}

scpl_status ensure_ws(scpl_ctx *ctx, size_t bytes) { return grow(ctx->ws, ctx->ws_size, bytes, ctx->fixed_ws); }
scpl_status ensure_jws(scpl_ctx *ctx, size_t bytes) { return grow(ctx->jws, ctx->jws_size, bytes, ctx->fixed_ws); }
scpl_status ensure_tws(scpl_ctx *ctx, size_t bytes) { return grow(ctx->tws, ctx->tws_size, bytes, ctx->fixed_ws); }

scpl_status ensure_pinned(scpl_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->pinned_size) return SCPL_OK;
    if (ctx->fixed_pinned) return SCPL_ERR_CAPACITY;
    if (ctx->pinned) {
        SCPL_TRY(hipHostFree(ctx->pinned));
        ctx->pinned = nullptr;
        ctx->pinned_size = 0;
    }
    size_t want = align_up(bytes, (size_t)1 << 16);
    SCPL_TRY(hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    ctx->pinned_size = want;
    return SCPL_OK;
}

// Streams and events for n job groups (streams only when n > 1: a single
// group runs on the caller's stream).
scpl_status ensure_side(scpl_ctx *ctx)
{
    if (!ctx->side_in) SCPL_TRY(hipEventCreateWithFlags(&ctx->side_in, hipEventDisableTiming));
    if (!ctx->side_out) SCPL_TRY(hipEventCreateWithFlags(&ctx->side_out, hipEventDisableTiming));
    return SCPL_OK;
}

scpl_status ensure_groups(scpl_ctx *ctx, int n)
{
    if (!ctx->fork) SCPL_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    while ((int)ctx->gevents.size() < n) {
        hipEvent_t e;
        SCPL_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->gevents.push_back(e);
    }
    while (n > 1 && (int)ctx->gstreams.size() < n) {
        hipStream_t st;
        SCPL_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        ctx->gstreams.push_back(st);
    }
    return SCPL_OK;
}

// DP geometry of a launch whose widest job is Wmax, with njobs jobs running
// concurrently (all job groups together): forced; else of the geometries
// autotuned for this width, the one timed with the nearest job count (by
// ratio); else the default table.
DpGeom select_geom(const scpl_ctx *ctx, int Wmax, int njobs = 1 << 20)
{
    if (ctx->forced.Q > 0 && dp_geom_fits(ctx->forced, Wmax)) return ctx->forced;
    const scpl_ctx::Tuned *best = nullptr;
    double bd = 0.0;
    const double ln = std::log((double)std::min(std::max(njobs, 1), 1 << 20));
    for (const auto &t : ctx->tuned)
        if (t.W == Wmax) {
            const double d = std::fabs(std::log((double)t.n) - ln);
            if (!best || d < bd) {
                best = &t;
                bd = d;
            }
        }
    if (best) return best->g;
    // untuned: launches of at most four buffers from 449 to 8960 columns take
    // the column split (2,8,16), 192 rows by 64 columns (the autotuner's pick
    // for one to three 1080- and 2160-row buffers); more buffers the default
    // of dp_geom.  The job workspaces are sized for dp_geom's, which covers
    // more columns.
    if (njobs <= 4 && Wmax > 448 && Wmax <= 8960) {
        DpGeom g{2, 8, 1, 16, 1};
        g.R = 192;
        g.P = 64;
        return g;
    }
    return dp_geom(Wmax);
}

// ----------------------------------------------------------- kernel timing

// Brackets the launches enqueued between prof_begin and prof_end with a
// pair of events when profiling is on.
struct ProfScope {
    scpl_ctx *ctx;
    hipStream_t s;
    int kind;
    ProfPair pp{};
    bool on = false;
    ProfScope(scpl_ctx *c, int k, hipStream_t st) : ctx(c), s(st), kind(k)
    {
        if (!ctx->profiling || !((ctx->prof_mask >> kind) & 1u)) return;
        if (!ctx->prof_free.empty()) {
            pp = ctx->prof_free.back();
            ctx->prof_free.pop_back();
        } else if (hipEventCreate(&pp.a) != hipSuccess || hipEventCreate(&pp.b) != hipSuccess) {
            return;
        }
        pp.kind = kind;
        on = hipEventRecord(pp.a, s) == hipSuccess;
    }
    ~ProfScope()
    {
        if (!on) return;
        if (hipEventRecord(pp.b, s) == hipSuccess) ctx->prof_pending.push_back(pp);
    }
};

scpl_status prof_drain(scpl_ctx *ctx)
{
    for (ProfPair &pp : ctx->prof_pending) {
        SCPL_TRY(hipEventSynchronize(pp.b));
        float ms = 0.f;
        SCPL_TRY(hipEventElapsedTime(&ms, pp.a, pp.b));
        ctx->prof_ms[pp.kind] += ms;
        ctx->prof_n[pp.kind] += 1;
        ctx->prof_free.push_back(pp);
    }
    ctx->prof_pending.clear();
    return SCPL_OK;
}

// ------------------------------------------------------------ segmentation

// Device state of one clip's buffer controller: moments S1, S2 per pixel
// and the window sums.
size_t seg_bytes(int64_t HW) { return align_up(HW * 4) + align_up(HW * 8); }

// Buffers of a clip whose first key rows the segmentation keeps, and the
// device bytes they take.
int seg_keep_buffers(const scpl_params &p)
{
    return (p.use_buffer && p.n_frames >= 2) ? std::min<int>(p.n_frames, kSegKeepBuffers) : 0;
}
size_t seg_keep_bytes(const scpl_params &p)
{
    return (size_t)seg_keep_buffers(p) * align_up((size_t)p.height * p.width * 2);
}

// Host staging of one run of nc clips with Ntot frames in all: window sums,
// segmentation arguments, buffer ids, job states and the job table.
size_t pinned_bytes(int nc, int64_t Ntot)
{
    return align_up((size_t)nc * kSegWindow * 8) + align_up(4 * (size_t)Ntot) + align_up(16 * (size_t)Ntot) +
           2 * align_up(sizeof(Job) * (size_t)Ntot) + align_up(sizeof(SegArgs) * (size_t)nc) +
           align_up(sizeof(SegFinish) * (size_t)nc);
}

// The gather stream and one event per clip of clips gathered early.
scpl_status ensure_clip_tracking(scpl_ctx *ctx, int nc)
{
    if (!ctx->gather_stream) SCPL_TRY(hipStreamCreateWithFlags(&ctx->gather_stream, hipStreamNonBlocking));
    if (!ctx->gathers_done) SCPL_TRY(hipEventCreateWithFlags(&ctx->gathers_done, hipEventDisableTiming));
    while ((int)ctx->clip_events.size() < nc) {
        hipEvent_t e;
        SCPL_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->clip_events.push_back(e);
    }
    return SCPL_OK;
}

// ------------------------------------------------------- height retargeting

bool height_pass(const scpl_params &p) { return p.target_height > 0 && p.target_height < p.height; }

// Parameters of the height pass: the transposed frames (W_src x H) carved
// from H to Ht columns; W_src is the width after the width pass.
scpl_params transposed_params(const scpl_params &p)
{
    scpl_params q = p;
    q.height = p.target_width;
    q.width = p.height;
    q.target_width = p.target_height;
    q.target_height = 0;
    return q;
}

// Temporaries of the height pass: the width-carved frames (when both
// dimensions shrink), the transposed input and output, transposed masks.
size_t height_temp_bytes(const scpl_params &p)
{
    if (!height_pass(p)) return 0;
    const size_t N = p.n_frames, H = p.height, C = p.channels, Ws = p.target_width;
    size_t b = 0;
    if (p.target_width < p.width) b += align_up(N * H * Ws * C);
    b += align_up(N * Ws * H * C) + align_up(N * Ws * p.target_height * C) + align_up(N * Ws * H * 2) +
         align_up(N * 4);
    return b;
}

// Device bytes of the plain path (one clip, one buffer at a time), by area:
// A holds the tiled and pixel-major luma, the buffer controller's state and
// the window sums; B one carving job's workspace (sized for every DP
// geometry and band height) with the job table and states; T the height
// pass's temporaries.  A pass of the width and a pass of the height reuse A
// and B one after the other.
struct PlainLayout {
    size_t ws = 0, jws = 0, tws = 0;
    size_t total() const { return ws + jws + tws; }
};

size_t area_a_bytes(const scpl_params &p)
{
    const size_t N = p.n_frames;
    return align_up(kSegWindow * 8) + align_up(N * tiled_frame_bytes(p.height, p.width)) +
           align_up((size_t)p.height * p.width * seq_pitch(p.n_frames)) + seg_bytes((int64_t)p.height * p.width) +
           align_up(sizeof(SegArgs)) + align_up(sizeof(SegFinish)) + seg_keep_bytes(p);
}

size_t area_b_bytes(const scpl_params &p)
{
    const size_t N = p.n_frames;  // at most one buffer per frame
    JobShape js{p.height, p.width, p.target_width, p.seams_per_iter, dp_geom(p.width), true};
    return job_bytes(js) + align_up(sizeof(Job) * N) + align_up(16 * N);
}

PlainLayout plain_layout(const scpl_params &p)
{
    PlainLayout L;
    if (!height_pass(p)) {
        L.ws = area_a_bytes(p);
        L.jws = area_b_bytes(p);
        return L;
    }
    if (p.target_width < p.width) {
        scpl_params w = p;
        w.target_height = 0;
        L.ws = area_a_bytes(w);
        L.jws = area_b_bytes(w);
    }
    const scpl_params q = transposed_params(p);
    L.ws = std::max(L.ws, area_a_bytes(q));
    L.jws = std::max(L.jws, area_b_bytes(q));
    L.tws = height_temp_bytes(p);
    return L;
}

// Points the context's three device workspaces (and, with fixed_host, its
// host staging as it stands) into one region laid out by L for the length of
// a call; the context's own allocations are restored afterwards and never
// freed or grown meanwhile.
struct FixedArena {
    scpl_ctx *ctx;
    void *ws, *jws, *tws;
    size_t ws_size, jws_size, tws_size;
    FixedArena(scpl_ctx *c, void *base, const PlainLayout &L, bool fixed_host)
        : ctx(c), ws(c->ws), jws(c->jws), tws(c->tws), ws_size(c->ws_size), jws_size(c->jws_size),
          tws_size(c->tws_size)
    {
        char *b = static_cast<char *>(base);
        c->ws = b;
        c->ws_size = L.ws;
        c->jws = b + L.ws;
        c->jws_size = L.jws;
        c->tws = b + L.ws + L.jws;
        c->tws_size = L.tws;
        c->fixed_ws = true;
        c->fixed_pinned = fixed_host;
    }
    ~FixedArena()
    {
        ctx->ws = ws;
        ctx->jws = jws;
        ctx->tws = tws;
        ctx->ws_size = ws_size;
        ctx->jws_size = jws_size;
        ctx->tws_size = tws_size;
        ctx->fixed_ws = false;
        ctx->fixed_pinned = false;
    }
};

struct SegClip {
    const scpl_params *p;
    const uint8_t *tiled;  // N tiled luma frames
    const uint8_t *seq;    // pixel-major luma, seq_pitch(N) entries per pixel
    int64_t FS;
    int ntc;
    void *state;           // seg_bytes(H W)
    int32_t *bid;          // host, N
    int64_t *trace;        // host, N, nullable
    uint16_t *keep = nullptr;  // device, nkeep x H x W: first key rows of finished buffers
    int nkeep = 0, kept = 0;
    std::vector<int> keep_of;  // per buffer: its slot of keep, or -1
    int32_t nbuf = 0;
    // controller
    int t0 = 0, n = 1, nb = 0, t = 1, te = 0;
    int win = kSegWindow;  // candidates per scan: kSegRestart after a rejection, doubled after none
    bool valid = false, done = false, launched = false;
};

// Dynamic spatiotemporal buffer (Sec. 3.2): frames join the current buffer
// while the ASDE of the grown buffer stays at or below phi(n).  Each round
// launches, for every clip still open, a speculative scan of a window of
// candidate frames; after one synchronisation the host accepts each clip's
// candidates in order and restarts that clip from its first rejected frame.
// With d_fin / h_fin (room for one per clip), the moments S1 of each
// finished buffer (up to SegClip::nkeep per clip, memorised buffers skipped)
// also give its first key rows, which the energy kernel then copies
// (seg_finish_kernel): before a clip's state is restarted, the frames
// scanned past the buffer's end are taken out of it.
scpl_status segment_clips(scpl_ctx *ctx, std::vector<SegClip> &cl, unsigned long long *d_sums,
                          unsigned long long *h_sums, SegArgs *d_args, SegArgs *h_args, hipStream_t s,
                          SegFinish *d_fin, SegFinish *h_fin)
{
    const int nc = (int)cl.size();
    int nfin = 0, fin_ntc = 0, fin_h = 0;
    // buffer b of clip c, frames [t0, tlo), its moments covering [t0, thi)
    auto finish = [&](SegClip &c, int b, int t0, int tlo, int thi) {
        const int m = c.p->memo_period;
        if (!h_fin || nfin >= nc || c.kept >= c.nkeep || (m >= 2 && b % m != 0)) return;
        if ((int)c.keep_of.size() <= b) c.keep_of.resize((size_t)b + 1, -1);
        const int64_t HW = (int64_t)c.p->height * c.p->width;
        c.keep_of[(size_t)b] = c.kept;
        SegFinish f{};
        f.luma = c.tiled;
        f.FS = c.FS;
        f.ntc = c.ntc;
        f.s1 = static_cast<const uint32_t *>(c.state);  // the first array of the state
        f.out = c.keep + (size_t)c.kept * (align_up((size_t)HW * 2) / 2);
        f.H = c.p->height;
        f.W = c.p->width;
        f.mode = c.p->energy_mode;
        f.tlo = tlo;
        f.thi = thi;
        f.T = tlo - t0;
        ++c.kept;
        h_fin[nfin++] = f;
        fin_ntc = std::max(fin_ntc, c.ntc);
        fin_h = std::max(fin_h, c.p->height);
    };
    // launched before the next window scan, which may restart the states
    auto launch_finish = [&]() -> scpl_status {
        if (nfin == 0) return SCPL_OK;
        SCPL_TRY(hipMemcpyAsync(d_fin, h_fin, sizeof(SegFinish) * (size_t)nfin, hipMemcpyHostToDevice, s));
        {
            ProfScope ps(ctx, SCPL_KERNEL_SEGMENT, s);
            launch_seg_finish(d_fin, nfin, fin_ntc, fin_h, s);
        }
        SCPL_CHECK_LAUNCH();
        nfin = fin_ntc = fin_h = 0;
        return SCPL_OK;
    };
    for (SegClip &c : cl) {
        const int N = c.p->n_frames;
        c.bid[0] = 0;
        if (c.trace) c.trace[0] = -1;
        if (!c.p->use_buffer) {
            for (int t = 0; t < N; ++t) {
                c.bid[t] = t;
                if (c.trace) c.trace[t] = -1;
            }
            c.nbuf = N;
            c.done = true;
        } else if (N == 1) {
            c.nbuf = 1;
            c.done = true;
        }
    }
    for (;;) {
        bool any = false;
        int na = 0, ntc_max = 0, h_max = 0;
        for (int ci = 0; ci < nc; ++ci) {
            SegClip &c = cl[ci];
            c.launched = false;
            if (c.done) continue;
            const scpl_params *p = c.p;
            const int N = p->n_frames;
            // frames forced into a new buffer by max_buffer need no test
            while (c.t < N && p->max_buffer > 0 && c.n >= p->max_buffer) {
                if (c.valid) finish(c, c.nb, c.t0, c.t, c.t);
                if (c.trace) c.trace[c.t] = -1;
                c.bid[c.t] = ++c.nb;
                c.t0 = c.t;
                c.n = 1;
                c.valid = false;
                ++c.t;
            }
            if (c.t >= N) {
                if (c.valid) finish(c, c.nb, c.t0, N, N);
                c.nbuf = c.nb + 1;
                c.done = true;
                continue;
            }
            c.te = std::min(N, c.t + c.win);
            if (p->max_buffer > 0) c.te = std::min(c.te, c.t + (p->max_buffer - c.n));
            const int64_t HW = (int64_t)p->height * p->width;
            Bump bp{static_cast<char *>(c.state)};
            SegArgs a{};
            a.luma = c.tiled;
            a.FS = c.FS;
            a.ntc = c.ntc;
            a.s1 = bp.take<uint32_t>(HW);
            a.s2 = bp.take<uint64_t>(HW);
            a.sout = d_sums + (size_t)ci * kSegWindow;
            a.H = p->height;
            a.W = p->width;
            a.mode = p->energy_mode;
            a.t0 = c.t0;
            a.tb = c.t;
            a.te = c.te;
            a.init = c.valid ? 0 : 1;
            h_args[na++] = a;
            ntc_max = std::max(ntc_max, c.ntc);
            h_max = std::max(h_max, p->height);
            c.launched = true;
            any = true;
        }
        // the buffers finished so far, before their states are restarted
        SCPL_TRY(launch_finish());
        if (!any) break;
        // one launch scans the windows of every open clip
        SCPL_TRY(hipMemsetAsync(d_sums, 0, (size_t)nc * kSegWindow * 8, s));
        SCPL_TRY(hipMemcpyAsync(d_args, h_args, sizeof(SegArgs) * (size_t)na, hipMemcpyHostToDevice, s));
        {
            ProfScope ps(ctx, SCPL_KERNEL_SEGMENT, s);
            launch_seg_windows(d_args, na, ntc_max, h_max, s);
        }
        SCPL_CHECK_LAUNCH();
        SCPL_TRY(hipMemcpyAsync(h_sums, d_sums, (size_t)nc * kSegWindow * 8, hipMemcpyDeviceToHost, s));
        SCPL_TRY(hipStreamSynchronize(s));
        for (int ci = 0; ci < nc; ++ci) {
            SegClip &c = cl[ci];
            if (!c.launched) continue;
            const scpl_params *p = c.p;
            const int64_t HW = (int64_t)p->height * p->width;
            const int32_t emax = energy_max(p->energy_mode);
            bool rejected = false;
            for (int tt = c.t; tt < c.te; ++tt) {
                const uint64_t S = h_sums[(size_t)ci * kSegWindow + (tt - c.t)];
                const int64_t nn = tt - c.t0 + 1;
                if (c.trace) c.trace[tt] = (int64_t)S;
                if (asde_rejects(S, nn, HW, emax, p->alpha_num, p->alpha_den)) {
                    finish(c, c.nb, c.t0, tt, c.te);
                    c.bid[tt] = ++c.nb;
                    c.t0 = tt;
                    c.n = 1;
                    c.valid = false;
                    c.t = tt + 1;
                    c.win = kSegRestart;
                    rejected = true;
                    break;
                }
                c.bid[tt] = c.nb;
                c.n = (int)nn;
            }
            if (!rejected) {
                c.valid = true;
                c.t = c.te;
                c.win = std::min(kSegWindow, 2 * c.win);
            }
        }
    }
    return SCPL_OK;
}

// ------------------------------------------------------------- iterations

struct LaunchShape {
    int Hmax = 0, Wmax = 0, nbmax = 0, kmax = 0, Bmax = 0;
    int gin = 0, gout = 0;  // largest source and output row in bytes (gather)
    DpGeom g{0, 0, 0, 0, 0};
    void add(const JobShape &s, int C = 1)
    {
        gin = std::max(gin, s.W * C);
        gout = std::max(gout, s.Wt * C);
        Hmax = std::max(Hmax, s.H);
        Wmax = std::max(Wmax, s.W);
        nbmax = std::max(nbmax, s.nb());
        kmax = std::max(kmax, s.kcap());
        Bmax = std::max(Bmax, s.B());
        g = s.g;
    }
};

// One SCPL iteration of every job of a launch (each job at its own
// iteration, kept on the device).
void enqueue_iteration(scpl_ctx *ctx, const Job *d_jobs, int nj, const LaunchShape &ls, hipStream_t s)
{
    {
        ProfScope ps(ctx, SCPL_KERNEL_DP, s);
        launch_dp(d_jobs, nj, ls.g, ls.Wmax, ls.Hmax, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_BORG, s);
        launch_borg(d_jobs, nj, ls.nbmax, ls.Bmax, ls.Wmax, ctx->borg_variant, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_SELECT, s);
        // LDS for the widest job's keys and band origins, not the whole CU, so
        // that the workgroups need not wait for an empty compute unit
        const size_t need = (size_t)16 * ls.Wmax + (size_t)ls.nbmax * (size_t)((ls.Wmax + 7) & ~3);
        launch_select(d_jobs, nj, 0, std::min(need, ctx->lds_cap), s);
    }
    if (ctx->fuse_variant > 0 && band_update_fits(ls.kmax, ls.Bmax)) {
        // fill and compaction fused per band (timed as the compaction)
        ProfScope ps(ctx, SCPL_KERNEL_UPDATE, s);
        launch_band_update(d_jobs, nj, ls.nbmax, ctx->fuse_variant, s);
    } else {
        {
            ProfScope ps(ctx, SCPL_KERNEL_FILL, s);
            launch_fill(d_jobs, nj, ls.kmax, ls.nbmax, ls.Bmax, s);
        }
        {
            ProfScope ps(ctx, SCPL_KERNEL_UPDATE, s);
            launch_update(d_jobs, nj, ls.Hmax, ls.Wmax, ctx->upd_variant, s);
        }
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_REFRESH, s);
        // also ends the iteration: moves every job still carving on
        launch_refresh(d_jobs, nj, ls.kmax, ls.Hmax, ctx->refresh_variant, s);
    }
}

// Iterations per replay of a group's graph.
constexpr int kGraphIters = 8;
// At most this many iterations of a group are enqueued per look at its
// states.  Enqueueing more can fill the stream's hardware queue, and then
// the host thread blocks inside the launch until the GPU drains it, while
// the other groups' read-backs wait unanswered.
constexpr int kMaxAhead = 32;

// A group of jobs that advances in lock-step on one stream: every stage of
// an iteration is one launch over the group's jobs.  Groups on different
// streams advance independently, so one group's bandwidth-bound stages run
// beside another's latency-bound DP.
struct Group {
    const Job *d_jobs = nullptr;
    const Job *h_jobs = nullptr;
    int32_t *d_states = nullptr;
    int32_t *h_states = nullptr;  // pinned
    int nj = 0;
    LaunchShape ls;
    int rfirst = 0;               // iterations enqueued before the first look at the states
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;      // completes with the group's latest state read-back
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    int slot = -1;                // index of the group in the context's graph cache (-1: none)
    bool cached = false;          // g and ge belong to the context's graph cache
    int r = 0;                    // iterations enqueued so far
    bool done = false;
    bool gather = true;           // gather the group's outputs when it is done (else its clips are gathered one by one)
    void release()
    {
        if (!cached) {
            if (ge) (void)hipGraphExecDestroy(ge);
            if (g) (void)hipGraphDestroy(g);
        }
        ge = nullptr;
        g = nullptr;
    }
};

// Everything enqueue_iteration's launches depend on besides the stream: the
// job table, the launch shape, the DP geometry and the kernel variants.
std::vector<int64_t> graph_key(const scpl_ctx *ctx, const Group &G)
{
    const LaunchShape &l = G.ls;
    return {(int64_t)(uintptr_t)G.d_jobs, G.nj,          l.Hmax,    l.Wmax,    l.nbmax,   l.kmax,
            l.Bmax,                       l.g.Q,         l.g.HB,    l.g.banded, l.g.PF,   l.g.EX,
            l.g.R,                        l.g.P,         ctx->borg_variant,    ctx->upd_variant,
            ctx->refresh_variant,         ctx->fuse_variant, (int64_t)ctx->lds_cap, kGraphIters};
}

scpl_status group_readback(Group &G)
{
    SCPL_TRY(hipMemcpyAsync(G.h_states, G.d_states, (size_t)G.nj * 4 * sizeof(int32_t), hipMemcpyDeviceToHost, G.st));
    SCPL_TRY(hipEventRecord(G.ev, G.st));
    return SCPL_OK;
}

// Enqueues at least n more iterations of the group: whole replays of its
// graph, or single launches when there is none (profiling, or a stream that
// cannot be captured).
scpl_status group_iterate(scpl_ctx *ctx, Group &G, int n)
{
    if (G.ge) {
        for (int q = 0; q < n; q += kGraphIters, G.r += kGraphIters) SCPL_TRY(hipGraphLaunch(G.ge, G.st));
        return SCPL_OK;
    }
    for (int q = 0; q < n; ++q, ++G.r) enqueue_iteration(ctx, G.d_jobs, G.nj, G.ls, G.st);
    SCPL_CHECK_LAUNCH();
    return SCPL_OK;
}

// Initial key rows, a graph of kGraphIters iterations (when use_graph), the
// first rfirst iterations, then a state read-back.
scpl_status group_start(scpl_ctx *ctx, Group &G, bool use_graph)
{
    const hipStream_t s = G.st;
    {
        ProfScope ps(ctx, SCPL_KERNEL_INIT, s);
        launch_init_jobs(G.d_jobs, G.nj, G.ls.Hmax, G.ls.Wmax, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_ENERGY, s);
        launch_energy(G.d_jobs, G.nj, G.ls.Hmax, G.ls.Wmax, s);
    }
    SCPL_CHECK_LAUNCH();
    if (use_graph && !ctx->profiling && s != nullptr && G.rfirst > 0) {
        // the graph of the previous call of this group when its launches
        // would be the same (the kernels read the job table when they run)
        std::vector<int64_t> key;
        scpl_ctx::GraphCache *c = nullptr;
        if (G.slot >= 0) {
            if ((int)ctx->gcache.size() <= G.slot) ctx->gcache.resize((size_t)G.slot + 1);
            c = &ctx->gcache[(size_t)G.slot];
            key = graph_key(ctx, G);
        }
        if (c && c->ge && c->key == key) {
            G.g = c->g;
            G.ge = c->ge;
            G.cached = true;
        } else {
            SCPL_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (int q = 0; q < kGraphIters; ++q) enqueue_iteration(ctx, G.d_jobs, G.nj, G.ls, s);
            hipError_t le = hipGetLastError();
            hipError_t ce = hipStreamEndCapture(s, &G.g);
            SCPL_TRY(le);
            SCPL_TRY(ce);
            SCPL_TRY(hipGraphInstantiate(&G.ge, G.g, nullptr, nullptr, 0));
            if (c) {  // the previous call's graph has finished running
                c->release();
                c->key = std::move(key);
                c->g = G.g;
                c->ge = G.ge;
                G.cached = true;
            }
        }
    }
    SCPL_TRY(group_iterate(ctx, G, std::min(G.rfirst, kMaxAhead)));
    return group_readback(G);
}

// After the group's read-back has completed: either every job has reached
// its target width (the outputs are gathered) or the jobs still carving
// (iterations that found fewer parents than k) get the iterations their
// width and last k_iter call for.
scpl_status group_advance(scpl_ctx *ctx, Group &G)
{
    bool all = true;
    int more = 1;
    for (int j = 0; j < G.nj; ++j) {
        if (G.h_states[4 * j] >= 0) continue;
        all = false;
        const int rem = G.h_states[4 * j + 1] - G.h_jobs[j].Wt;
        const int last = std::max(1, G.h_states[4 * j + 2]);
        more = std::max(more, (rem + last - 1) / last);
    }
    if (all) {
        if (G.gather) {
            ProfScope ps(ctx, SCPL_KERNEL_GATHER, G.st);
            launch_gather(G.d_jobs, G.nj, G.ls.Hmax, G.ls.gin, G.ls.gout, G.ls.Wmax, ctx->gather_variant, G.st);
        }
        SCPL_CHECK_LAUNCH();
        SCPL_TRY(hipEventRecord(G.ev, G.st));
        G.done = true;
        return SCPL_OK;
    }
    if (G.r > G.ls.Wmax + kGraphIters + 1) return SCPL_ERR_INTERNAL;  // each iteration removes >= 1 column
    SCPL_TRY(group_iterate(ctx, G, std::min(more, kMaxAhead)));
    return group_readback(G);
}

// Clips gathered as soon as their own buffers are carved (run_clips with a
// ClipDone).  After each state read-back the clips whose jobs have all
// reached their target width get their gather on the gather stream, and are
// reported once the gather's event has completed.  A state is read only
// once the read-back that wrote it has completed, so the job's last
// iteration has too (a job never leaves the done state); the host states
// start at -1 so that no state of an earlier call is taken for one.
struct ClipTracker {
    scpl_ctx *ctx = nullptr;
    const ClipDone *cb = nullptr;
    const int32_t *h_states = nullptr;      // every job's state (pinned), by slot
    std::vector<std::vector<int>> slots;   // per clip: its jobs' slots
    std::vector<const Job *> gjobs;         // per clip: its gather table (carving jobs, then memorised buffers)
    std::vector<int> ngj;
    std::vector<LaunchShape> ls;
    std::vector<char> launched, reported;
    // gathers of the clips whose jobs are all done
    scpl_status progress()
    {
        for (size_t c = 0; c < slots.size(); ++c) {
            if (launched[c]) continue;
            bool all = true;
            for (int q : slots[c]) all = all && h_states[4 * q] >= 0;
            if (!all) continue;
            if (ngj[c] > 0) {
                ProfScope ps(ctx, SCPL_KERNEL_GATHER, ctx->gather_stream);
                launch_gather(gjobs[c], ngj[c], ls[c].Hmax, ls[c].gin, ls[c].gout, ls[c].Wmax, ctx->gather_variant,
                              ctx->gather_stream);
            }
            SCPL_CHECK_LAUNCH();
            SCPL_TRY(hipEventRecord(ctx->clip_events[c], ctx->gather_stream));
            launched[c] = 1;
        }
        return poll();
    }
    // reports the clips whose gathers have completed
    scpl_status poll()
    {
        for (size_t c = 0; c < slots.size(); ++c) {
            if (!launched[c] || reported[c]) continue;
            const hipError_t q = hipEventQuery(ctx->clip_events[c]);
            if (q == hipErrorNotReady) continue;
            SCPL_TRY(q);
            reported[c] = 1;
            (*cb)((int)c);
        }
        return SCPL_OK;
    }
};

// Runs the groups to completion after the work already on stream s, and
// makes s wait for all of them.  The host polls the groups' read-backs and
// feeds whichever is ready.  trk (nullable): clips gathered one by one.
scpl_status run_groups(scpl_ctx *ctx, std::vector<Group> &gs, bool use_graph, hipStream_t s,
                       ClipTracker *trk = nullptr)
{
    struct Cleanup {
        std::vector<Group> &gs;
        bool ok = false;
        ~Cleanup()
        {
            for (Group &G : gs) {
                if (!ok) (void)hipStreamSynchronize(G.st);  // no graph is freed while it may run
                G.release();
            }
        }
    } cleanup{gs};
    bool forked = false;
    for (Group &G : gs)
        if (G.st != s) forked = true;
    if (forked) {
        SCPL_TRY(hipEventRecord(ctx->fork, s));
        for (Group &G : gs)
            if (G.st != s) SCPL_TRY(hipStreamWaitEvent(G.st, ctx->fork, 0));
    }
    for (Group &G : gs) SCPL_TRY(group_start(ctx, G, use_graph));
    int open = (int)gs.size();
    while (open > 0) {
        bool progressed = false;
        for (Group &G : gs) {
            if (G.done) continue;
            hipError_t q = open == 1 ? hipEventSynchronize(G.ev) : hipEventQuery(G.ev);
            if (q == hipErrorNotReady) continue;
            SCPL_TRY(q);
            if (trk) SCPL_TRY(trk->progress());  // the read-back has completed
            SCPL_TRY(group_advance(ctx, G));
            if (G.done) --open;
            progressed = true;
        }
        if (trk && !progressed) SCPL_TRY(trk->poll());
        if (!progressed) std::this_thread::yield();
    }
    if (trk) SCPL_TRY(trk->progress());
    for (Group &G : gs)
        if (G.st != s) SCPL_TRY(hipStreamWaitEvent(s, G.ev, 0));
    if (trk) {  // s waits for the clips' gathers too
        SCPL_TRY(hipEventRecord(ctx->gathers_done, ctx->gather_stream));
        SCPL_TRY(hipStreamWaitEvent(s, ctx->gathers_done, 0));
    }
    cleanup.ok = true;
    return SCPL_OK;
}

// The persistent launch's DP chunking: the caller's (or the batch
// autotuner's) column split when its four-wavefront cover is exact, else
// 256 rows by 384 columns.
DpGeom persist_geom(const scpl_ctx *ctx)
{
    for (const DpGeom *g : {&ctx->forced, &ctx->batch_forced})
        if (g->Q == 4 && g->HB == 16 && g->PF == 8 && g->R > 0 && g->chunk_waves() == 4 && dp_geom_fits(*g, 1))
            return DpGeom{4, 16, 1, 8, 0, g->R, g->P};
    return DpGeom{4, 16, 1, 8, 0, 256, 384};
}

// Ring slots of a persistent launch over jobs of these shapes: a power of
// two, at least 4 times the most items that can wait at once (each job has
// the items of one stage outstanding at a time), and at least 65536.
int persist_ring(const std::vector<JobShape> &shapes, const DpGeom &g)
{
    int64_t most = 0;
    for (const JobShape &s : shapes)
        most += std::max<int64_t>({(s.W + g.P - 1) / g.P, s.nb(), (s.H + 15) / 16, 1});
    int64_t cap = 65536;
    while (cap < 4 * most) cap *= 2;
    return (int)cap;
}

size_t persist_bytes(int njobs, int cap, int nring)
{
    return align_up(sizeof(PState) * (size_t)nring) + align_up((size_t)njobs * 4) +
           2 * align_up((size_t)cap * 8 * (size_t)nring) + align_up(kPTrace * 8);
}

// Rings of a persistent launch: one per XCD in XCD-local mode.
int persist_rings(const scpl_ctx *ctx)
{
    return ctx->batch_mode == SCPL_BATCH_PERSISTENT && ctx->nxcd > 0 ? ctx->nxcd : 1;
}

// Deals the jobs to the rings: heaviest first (rows x columns x columns to
// remove), each to the ring with the least work so far.
void deal_rings(std::vector<Job> &jobs, int nring)
{
    std::vector<int> order(jobs.size());
    std::iota(order.begin(), order.end(), 0);
    auto work = [&](const Job &J) { return (double)J.H * J.W * (double)std::max(J.W - J.Wt, 0); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(jobs[a]) > work(jobs[b]); });
    std::vector<double> load((size_t)nring, 0.0);
    for (int q : order) {
        const int r = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        jobs[q].ring = r;
        load[r] += work(jobs[q]);
    }
}

// Every iteration of the jobs d_jobs[0, nj) in one persistent launch on
// stream s (captured as a graph with the ring's set-up when use_graph),
// then their outputs gathered.  area: persist_bytes(nj, cap) of device
// memory.  With a graph it returns after the launch has run (the graph is
// freed then); the caller reads the states.
scpl_status run_persistent(scpl_ctx *ctx, const Job *d_jobs, int nj, const LaunchShape &ls, const DpGeom &g, int cap,
                           int nring, char *area, bool use_graph, hipStream_t s)
{
    const bool local = ctx->batch_mode == SCPL_BATCH_PERSISTENT && ctx->nxcd > 0;
    Bump b{area};
    PArgs a{};
    a.jobs = d_jobs;
    a.st = b.take<PState>((size_t)nring);
    a.cnt = b.take<int>((size_t)nj);
    a.seq = b.take<unsigned long long>((size_t)cap * nring);
    a.item = b.take<unsigned long long>((size_t)cap * nring);
    a.nring = nring;
    for (int q = 0; q < 16; ++q) a.xcc_ring[q] = local ? ctx->xcc_ring[q] : -1;
    unsigned long long *trace = b.take<unsigned long long>(kPTrace);
    a.trace = ctx->profiling ? trace : nullptr;  // counted while kernels are timed
    a.njobs = nj;
    a.cap_mask = cap - 1;
    a.R = g.R;
    a.P = g.P;
    a.lds_bytes = (int)persist_lds_bytes();
    a.sel_lds = a.lds_bytes;
    a.wait_ticks = 4000LL * ctx->wall_khz;  // 4 s
    {
        ProfScope ps(ctx, SCPL_KERNEL_INIT, s);
        launch_init_jobs(d_jobs, nj, ls.Hmax, ls.Wmax, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_ENERGY, s);
        launch_energy(d_jobs, nj, ls.Hmax, ls.Wmax, s);
    }
    SCPL_CHECK_LAUNCH();
    if (use_graph && !ctx->profiling && s != nullptr) {
        hipGraph_t gr = nullptr;
        hipGraphExec_t ge = nullptr;
        SCPL_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        launch_persist_clear(a, s);
        launch_persist_seed(a, s);
        launch_persist(a, ctx->persist_grid, local, s);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(s, &gr);
        SCPL_TRY(le);
        SCPL_TRY(ce);
        hipError_t ie = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        hipError_t xe = ie == hipSuccess ? hipGraphLaunch(ge, s) : ie;
        // the graph is freed only once it has run
        hipError_t se = hipStreamSynchronize(s);
        if (ge) (void)hipGraphExecDestroy(ge);
        (void)hipGraphDestroy(gr);
        SCPL_TRY(xe);
        SCPL_TRY(se);
    } else {
        if (a.trace) SCPL_TRY(hipMemsetAsync(a.trace, 0, kPTrace * 8, s));
        launch_persist_clear(a, s);
        launch_persist_seed(a, s);
        ProfScope ps(ctx, SCPL_KERNEL_PERSIST, s);
        launch_persist(a, ctx->persist_grid, local, s);
    }
    if (a.trace) {
        SCPL_TRY(hipMemcpyAsync(ctx->persist_trace, a.trace, sizeof(ctx->persist_trace), hipMemcpyDeviceToHost, s));
        SCPL_TRY(hipStreamSynchronize(s));
        ctx->persist_traced = true;
    }
    SCPL_CHECK_LAUNCH();
    {
        ProfScope ps(ctx, SCPL_KERNEL_GATHER, s);
        launch_gather(d_jobs, nj, ls.Hmax, ls.gin, ls.gout, ls.Wmax, ctx->gather_variant, s);
    }
    SCPL_CHECK_LAUNCH();
    return SCPL_OK;
}

// Copies the per-iteration records of the jobs into ctx->last_log.
scpl_status collect_logs(scpl_ctx *ctx, const std::vector<Job> &jobs, hipStream_t s)
{
    std::vector<int32_t> buf;
    for (const Job &J : jobs) {
        buf.resize((size_t)J.logcap * 4);
        SCPL_TRY(hipMemcpyAsync(buf.data(), J.log, buf.size() * 4, hipMemcpyDeviceToHost, s));
        SCPL_TRY(hipStreamSynchronize(s));
        for (int r = 0; r < J.logcap; ++r) {
            if (buf[4 * r] <= J.Wt || buf[4 * r + 2] <= 0) break;
            ctx->last_log.push_back(J.buffer_index);
            ctx->last_log.push_back(buf[4 * r]);
            ctx->last_log.push_back(buf[4 * r + 1]);
            ctx->last_log.push_back(buf[4 * r + 2]);
        }
    }
    return SCPL_OK;
}

Job clip_job(const scpl_params *p, const uint8_t *frames, const uint8_t *luma, uint8_t *out, uint16_t *masks,
             int t0, int T, int bindex)
{
    Job J{};
    J.frames = frames;
    J.luma = luma;
    J.ntc = tiles_across(p->width);
    J.FS = tiled_frame_bytes(p->height, p->width);
    J.out = out;
    J.masks = masks;
    J.C = p->channels;
    J.mode = p->energy_mode;
    J.t0 = t0;
    J.T = T;
    J.has_prev = (p->energy_mode == SCPL_ENERGY_MOTION && t0 > 0) ? 1 : 0;
    J.buffer_index = bindex;
    return J;
}

// Buffers (t0, T) from per-frame buffer ids.
std::vector<std::pair<int, int>> buffers_of(const int32_t *bid, int N)
{
    std::vector<std::pair<int, int>> v;
    int t0 = 0;
    for (int t = 1; t <= N; ++t)
        if (t == N || bid[t] != bid[t - 1]) {
            v.emplace_back(t0, t - t0);
            t0 = t;
        }
    return v;
}

int first_batch_iterations(const scpl_params *p)
{
    const int rem = p->width - p->target_width;
    return (rem + p->seams_per_iter - 1) / p->seams_per_iter;
}

}  // namespace

// ============================================== no-allocation workspace

// The device workspace of scpl_retarget_noalloc: one array per device,
// held from the library's load until the process ends.  Host code never
// passes `scratch` itself to a kernel or a copy (in host code the name is a
// stand-in, not a device address); scpl_create looks up each device's
// address once, with that device current, and the calls use that.
static __device__ __align__(256) unsigned char scratch[SCPL_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 256;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up once).
scpl_status scratch_address(int dev, void **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxScratchDevices) return SCPL_OK;  // no no-allocation workspace on this device
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        SCPL_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return SCPL_OK;
}
}  // namespace

// ===================================================================== C ABI

extern "C" {

const char *scpl_status_str(scpl_status s)
{
    // a C caller may pass any int: read it as one, not as the enumeration
    int v = 0;
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
    case SCPL_OK: return "ok";
    case SCPL_ERR_INVALID_ARG: return "invalid argument";
    case SCPL_ERR_OUT_OF_MEMORY: return "out of device memory";
    case SCPL_ERR_DEVICE: return "device error";
    case SCPL_ERR_CAPACITY: return "capacity exceeded";
    case SCPL_ERR_NOT_READY: return "not ready";
    case SCPL_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

scpl_status scpl_create(int32_t hip_device, scpl_ctx **out)
{
    if (!out) return SCPL_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    SCPL_TRY(hipGetDeviceCount(&n));
    if (hip_device < 0 || hip_device >= n) return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(hip_device));
    hipDeviceProp_t prop;
    SCPL_TRY(hipGetDeviceProperties(&prop, hip_device));
    scpl_ctx *c = new (std::nothrow) scpl_ctx();
    if (!c) return SCPL_ERR_OUT_OF_MEMORY;
    c->device = hip_device;
    // dynamic LDS of the selection kernel: all the device allows per block,
    // less the kernel's own static LDS
    c->lds_cap = prop.sharedMemPerBlock > 1024 ? prop.sharedMemPerBlock - 1024 : prop.sharedMemPerBlock;
    g_lds_cap = c->lds_cap;
    set_kernel_attributes(c->lds_cap);
    // the persistent launch: as many workgroups as are resident at once, and
    // the wall-clock rate its wait bound counts in
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, hip_device) == hipSuccess && khz > 0) {
        c->wall_khz = khz;
        c->ncu = prop.multiProcessorCount;
        c->persist_max_per_cu = persist_blocks_per_cu();
        c->persist_grid = std::min(c->persist_max_per_cu * c->ncu, 8192);
    }
    // XCD-local persistent mode: the XCC_ID of the workgroups of a probe
    // launch must follow the dispatcher's round robin over the XCDs
    // (workgroup i on the (i mod n)-th), else the mode stays off
    if (c->persist_grid > 0) {
        std::vector<int> ids(4096);
        if (probe_xcc((int)ids.size(), ids.data()) == 0) {
            std::vector<int> first;
            for (int v : ids) {
                if (std::find(first.begin(), first.end(), v) != first.end()) break;
                first.push_back(v);
            }
            const int n = (int)first.size();
            // (at least two XCDs: a register that read the same everywhere
            // would otherwise pass as a one-XCD device)
            bool ok = n >= 2 && n <= 16 && (n & (n - 1)) == 0;
            for (size_t i = 0; ok && i < ids.size(); ++i) ok = ids[i] == first[i % n];
            if (ok) {
                c->nxcd = n;
                for (int q = 0; q < 16; ++q) c->xcc_ring[q] = -1;
                for (int q = 0; q < n; ++q) c->xcc_ring[first[q] & 15] = q;
            }
        }
    }
    // everything the plain path needs besides its workspace is made here, so
    // that scpl_retarget_noalloc allocates nothing: the events of one job
    // group, host staging for the most frames a call may have, and this
    // device's address of the no-allocation workspace
    scpl_status st = ensure_side(c);
    if (st == SCPL_OK) st = ensure_groups(c, 1);
    if (st == SCPL_OK) st = ensure_pinned(c, pinned_bytes(1, SCPL_MAX_FRAMES));
    if (st == SCPL_OK) st = scratch_address(hip_device, &c->scratch);
    if (st != SCPL_OK) {
        scpl_destroy(c);
        return st;
    }
    *out = c;
    return SCPL_OK;
}

void scpl_destroy(scpl_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)prof_drain(ctx);
    for (ProfPair &pp : ctx->prof_free) {
        (void)hipEventDestroy(pp.a);
        (void)hipEventDestroy(pp.b);
    }
    for (hipStream_t st : ctx->gstreams) (void)hipStreamDestroy(st);
    for (scpl_ctx::GraphCache &c : ctx->gcache) c.release();
    for (hipEvent_t e : ctx->gevents) (void)hipEventDestroy(e);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->side_in) (void)hipEventDestroy(ctx->side_in);
    if (ctx->side_out) (void)hipEventDestroy(ctx->side_out);
    if (ctx->gather_stream) (void)hipStreamDestroy(ctx->gather_stream);
    for (hipEvent_t e : ctx->clip_events) (void)hipEventDestroy(e);
    if (ctx->gathers_done) (void)hipEventDestroy(ctx->gathers_done);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->jws) (void)hipFree(ctx->jws);
    if (ctx->tws) (void)hipFree(ctx->tws);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

scpl_status scpl_workspace_size(const scpl_params *p, uint64_t *device_bytes)
{
    scpl_status st = validate(p);
    if (st != SCPL_OK) return st;
    if (!device_bytes) return SCPL_ERR_INVALID_ARG;
    *device_bytes = plain_layout(*p).total();
    return SCPL_OK;
}

}  // extern "C"

scpl_status scpl::trim_workspace(scpl_ctx *ctx, uint64_t keep)
{
    if ((uint64_t)ctx->ws_size + ctx->jws_size + ctx->tws_size <= keep) return SCPL_OK;
    SCPL_TRY(hipSetDevice(ctx->device));
    if (ctx->ws) SCPL_TRY(hipFree(ctx->ws));  // waits for work that uses it
    if (ctx->jws) SCPL_TRY(hipFree(ctx->jws));
    if (ctx->tws) SCPL_TRY(hipFree(ctx->tws));
    ctx->ws = ctx->jws = ctx->tws = nullptr;
    ctx->ws_size = ctx->jws_size = ctx->tws_size = 0;
    return SCPL_OK;
}

// Upper bound of the device bytes a batched retarget of this clip can
// claim: its tiled luma and controller state, and one job per frame (the
// most buffers a clip can have) with its table entries.
uint64_t scpl::clip_footprint(const scpl_params &p)
{
    JobShape js{p.height, p.width, p.target_width, p.seams_per_iter, dp_geom(p.width)};
    const uint64_t N = (uint64_t)p.n_frames;
    uint64_t b = align_up((size_t)N * tiled_frame_bytes(p.height, p.width));
    b += align_up((size_t)p.height * p.width * seq_pitch((int)N));
    b += seg_bytes((int64_t)p.height * p.width) + seg_keep_bytes(p) + align_up(kSegWindow * 8);
    b += N * (job_bytes(js) + sizeof(Job) + 16) + 2 * kAlign;
    if (height_pass(p)) {
        const scpl_params q = transposed_params(p);
        JobShape jq{q.height, q.width, q.target_width, q.seams_per_iter, dp_geom(q.width)};
        uint64_t b2 = align_up((size_t)N * tiled_frame_bytes(q.height, q.width));
        b2 += align_up((size_t)q.height * q.width * seq_pitch((int)N));
        b2 += seg_bytes((int64_t)q.height * q.width) + seg_keep_bytes(q) + align_up(kSegWindow * 8);
        b2 += N * (job_bytes(jq) + sizeof(Job) + 16) + 2 * kAlign;
        b = std::max(b, b2) + height_temp_bytes(p);
    }
    return b;
}

// Retargets clips: tiled luma of every clip, buffer segmentation of all
// clips together, then the carving jobs (one per buffer) -- all at once
// (batched) or one buffer after another (plain).
scpl_status scpl::run_clips(scpl_ctx *ctx, const scpl_clip *clips, int nc, bool batched, int32_t *h_nbuf_first,
                            hipStream_t s, bool use_graph, const ClipDone *on_done)
{
    // area A: tiled lumas, controller states, window sums
    size_t a_bytes = align_up((size_t)nc * kSegWindow * 8);
    int64_t Ntot = 0;
    for (int c = 0; c < nc; ++c) {
        const scpl_params &p = clips[c].p;
        a_bytes += align_up((size_t)p.n_frames * tiled_frame_bytes(p.height, p.width));
        a_bytes += align_up((size_t)p.height * p.width * seq_pitch(p.n_frames));
        a_bytes += seg_bytes((int64_t)p.height * p.width) + seg_keep_bytes(p);
        Ntot += p.n_frames;
    }
    a_bytes += align_up(sizeof(SegArgs) * (size_t)nc) + align_up(sizeof(SegFinish) * (size_t)nc);
    SCPL_TRY(ensure_ws(ctx, a_bytes));
    SCPL_TRY(ensure_pinned(ctx, pinned_bytes(nc, Ntot)));
    Bump host{static_cast<char *>(ctx->pinned)};
    unsigned long long *h_sums = host.take<unsigned long long>((size_t)nc * kSegWindow);
    SegArgs *h_args = host.take<SegArgs>((size_t)nc);
    SegFinish *h_fin = host.take<SegFinish>((size_t)nc);
    int32_t *h_bid_all = host.take<int32_t>((size_t)Ntot);
    int32_t *h_states = host.take<int32_t>(4 * (size_t)Ntot);
    Job *h_jobs = host.take<Job>((size_t)Ntot);
    Job *h_gjobs = host.take<Job>((size_t)Ntot);  // gather tables of clips gathered early

    Bump dev{static_cast<char *>(ctx->ws)};
    unsigned long long *d_sums = dev.take<unsigned long long>((size_t)nc * kSegWindow);
    SegArgs *d_args = dev.take<SegArgs>((size_t)nc);
    SegFinish *d_fin = dev.take<SegFinish>((size_t)nc);
    std::vector<SegClip> seg(nc);
    int64_t off = 0;
    for (int c = 0; c < nc; ++c) {
        const scpl_params &p = clips[c].p;
        SegClip &sc = seg[c];
        sc.p = &p;
        sc.FS = tiled_frame_bytes(p.height, p.width);
        sc.ntc = tiles_across(p.width);
        uint8_t *tiled = dev.take<uint8_t>((size_t)p.n_frames * sc.FS);
        uint8_t *seq = dev.take<uint8_t>((size_t)p.height * p.width * seq_pitch(p.n_frames));
        sc.tiled = tiled;
        sc.seq = seq;
        sc.state = dev.take<char>(seg_bytes((int64_t)p.height * p.width));
        sc.nkeep = seg_keep_buffers(p);
        sc.keep = reinterpret_cast<uint16_t *>(dev.take<char>(seg_keep_bytes(p)));
        sc.bid = h_bid_all + off;
        sc.trace = nullptr;
        off += p.n_frames;
        ProfScope ps(ctx, SCPL_KERNEL_LUMA, s);
        launch_tile_luma(clips[c].d_frames, p.channels, p.n_frames, p.height, p.width, tiled, s);
    }
    SCPL_CHECK_LAUNCH();
    // the pixel-major lumas (read from the first iteration's refresh on) are
    // built while the segmentation runs, on the last job group's stream (no
    // stream of their own: more streams than hardware queues would share one)
    SCPL_TRY(ensure_side(ctx));
    SCPL_TRY(ensure_groups(ctx, batched ? ctx->nstreams : 1));
    const hipStream_t side = (batched && ctx->nstreams > 1) ? ctx->gstreams[ctx->nstreams - 1] : s;
    SCPL_TRY(hipEventRecord(ctx->side_in, s));
    SCPL_TRY(hipStreamWaitEvent(side, ctx->side_in, 0));
    for (int c = 0; c < nc; ++c) {
        const scpl_params &p = clips[c].p;
        ProfScope ps(ctx, SCPL_KERNEL_LUMA, side);
        launch_seq(seg[c].tiled, p.n_frames, p.height, p.width, const_cast<uint8_t *>(seg[c].seq),
                   seq_pitch(p.n_frames), side);
    }
    SCPL_CHECK_LAUNCH();
    SCPL_TRY(hipEventRecord(ctx->side_out, side));
    scpl_status st = segment_clips(ctx, seg, d_sums, h_sums, d_args, h_args, s, d_fin, h_fin);
    if (st != SCPL_OK) {
        (void)hipStreamSynchronize(side);  // no workspace is released under it
        return st;
    }
    for (int c = 0; c < nc; ++c)
        if (clips[c].d_buffer_id)
            SCPL_TRY(hipMemcpyAsync(clips[c].d_buffer_id, seg[c].bid, (size_t)clips[c].p.n_frames * 4,
                                    hipMemcpyHostToDevice, s));
    if (h_nbuf_first) *h_nbuf_first = seg[0].nbuf;
    SCPL_TRY(hipStreamWaitEvent(s, ctx->side_out, 0));

    // jobs: one per buffer of every clip
    struct Pending {
        int clip, t0, T, bindex;
    };
    std::vector<Pending> pend;
    // seam memorisation: buffers that are not carved but reuse the seams of
    // the last carved buffer of their clip (the pending job `src`)
    struct Memo {
        int src, t0, T, bindex;
    };
    std::vector<Memo> memo;
    for (int c = 0; c < nc; ++c) {
        const auto bufs = buffers_of(seg[c].bid, clips[c].p.n_frames);
        const size_t m = (size_t)clips[c].p.memo_period;
        int src = -1;
        for (size_t b = 0; b < bufs.size(); ++b) {
            if (m >= 2 && b % m != 0) {
                memo.push_back({src, bufs[b].first, bufs[b].second, (int)b});
                continue;
            }
            src = (int)pend.size();
            pend.push_back({c, bufs[b].first, bufs[b].second, (int)b});
        }
    }
    const int nj = (int)pend.size();
    const int nm = (int)memo.size();
    int Wall = 0;
    for (int c = 0; c < nc; ++c) Wall = std::max(Wall, clips[c].p.width);
    // the persistent launch serves batches up to 8192 columns wide
    // (only in XCD-local mode: without the probe's XCDs the batch runs as job
    // groups)
    const bool persist = batched && ctx->batch_mode == SCPL_BATCH_PERSISTENT && Wall <= 8192 && nj > 0 &&
                         ctx->persist_grid > 0 && ctx->nxcd > 0;
    const int nring = persist ? persist_rings(ctx) : 1;
    const DpGeom gpers = persist_geom(ctx);
    // a batched DP launch serves every job: its geometry follows the widest
    // (a geometry forced by the caller first, then the batch autotuner's)
    const DpGeom gall = persist ? gpers
                        : (ctx->forced.Q == 0 && ctx->batch_forced.Q > 0 && dp_geom_fits(ctx->batch_forced, Wall))
                            ? ctx->batch_forced
                            : select_geom(ctx, Wall, nj);
    auto shape_of = [&](const Pending &q) {
        const scpl_params &p = clips[q.clip].p;
        JobShape js{p.height, p.width, p.target_width, p.seams_per_iter, batched ? gall : select_geom(ctx, p.width, 1)};
        if (persist) js.band = 32;
        return js;
    };
    // area B: job workspaces (all jobs when batched; one shared per clip shape
    // when plain, buffers running one after another), job table, states
    size_t job_area = 0;
    for (const Pending &q : pend) {
        const size_t jb = job_bytes(shape_of(q));
        job_area = batched ? job_area + jb : std::max(job_area, jb);
    }
    int pcap = 0;
    if (persist) {
        std::vector<JobShape> shapes;
        for (const Pending &q : pend) shapes.push_back(shape_of(q));
        pcap = persist_ring(shapes, gpers);
    }
    const size_t pbytes = persist ? persist_bytes(nj, pcap, nring) : 0;
    // clips gathered as soon as their own buffers are done (job groups)
    const bool early = batched && !persist && on_done != nullptr && static_cast<bool>(*on_done);
    const size_t gbytes = early ? align_up(sizeof(Job) * (size_t)(nj + nm)) : 0;
    SCPL_TRY(ensure_jws(ctx, job_area + align_up(sizeof(Job) * (size_t)(nj + nm)) + align_up(16 * (size_t)nj) +
                                 pbytes + gbytes));
    Bump jdev{static_cast<char *>(ctx->jws)};
    char *job_ws = jdev.take<char>(job_area);
    Job *d_jobs = jdev.take<Job>((size_t)(nj + nm));  // carving jobs, then memorised buffers
    int32_t *d_states = jdev.take<int32_t>(4 * (size_t)nj);
    char *parea = persist ? jdev.take<char>(pbytes) : nullptr;
    Job *d_gjobs = early ? jdev.take<Job>((size_t)(nj + nm)) : nullptr;
    // batched: the jobs are dealt to the groups in order of decreasing
    // length, so that every group gets a share of the heavy buffers; a
    // group's jobs are consecutive in the job table
    const int ng = batched ? std::max(1, std::min(ctx->nstreams, nj)) : 1;
    std::vector<int> order(nj), slot(nj), gsize(ng, 0), gfirst(ng, 0);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pend[a].T > pend[b].T; });
    for (int i = 0; i < nj; ++i) ++gsize[i % ng];
    for (int g = 1; g < ng; ++g) gfirst[g] = gfirst[g - 1] + gsize[g - 1];
    {
        std::vector<int> fill(ng, 0);
        for (int i = 0; i < nj; ++i) slot[order[i]] = gfirst[i % ng] + fill[i % ng]++;
    }
    Bump jb{job_ws};
    std::vector<Job> jobs;
    for (int q = 0; q < nj; ++q) {
        const scpl_clip &cl = clips[pend[q].clip];
        const JobShape js = shape_of(pend[q]);
        Job J = clip_job(&cl.p, cl.d_frames, seg[pend[q].clip].tiled, cl.d_out, cl.d_masks, pend[q].t0, pend[q].T,
                         pend[q].bindex);
        J.seq = seg[pend[q].clip].seq;
        J.seqp = seq_pitch(cl.p.n_frames);
        {
            const SegClip &sc = seg[pend[q].clip];
            const int b = pend[q].bindex;
            const int64_t HW = (int64_t)cl.p.height * cl.p.width;
            if (b < (int)sc.keep_of.size() && sc.keep_of[(size_t)b] >= 0)
                J.u0 = sc.keep + (size_t)sc.keep_of[(size_t)b] * (align_up((size_t)HW * 2) / 2);
        }
        if (!batched) jb.off = 0;  // plain: every buffer reuses the same area
        carve_job(J, js, jb, d_states + 4 * slot[q]);
        h_jobs[slot[q]] = J;
        jobs.push_back(J);
    }
    if (persist) {  // each job's work ring (XCD)
        deal_rings(jobs, nring);
        for (int q = 0; q < nj; ++q) h_jobs[slot[q]].ring = jobs[q].ring;
    }
    // a memorised buffer is gathered like its source job (same column map
    // and mask, which hold that job's result once it is done) over its own
    // frames
    for (int q = 0; q < nm; ++q) {
        Job J = h_jobs[slot[memo[q].src]];
        J.t0 = memo[q].t0;
        J.T = memo[q].T;
        J.has_prev = 0;
        J.buffer_index = memo[q].bindex;
        h_jobs[nj + q] = J;
    }
    SCPL_TRY(hipMemcpyAsync(d_jobs, h_jobs, sizeof(Job) * (size_t)(nj + nm), hipMemcpyHostToDevice, s));
    // clips gathered early: per clip, its carving jobs and then its memorised
    // buffers, contiguous
    ClipTracker trk;
    if (early) {
        SCPL_TRY(ensure_clip_tracking(ctx, nc));
        trk.ctx = ctx;
        trk.cb = on_done;
        trk.h_states = h_states;
        trk.slots.assign(nc, {});
        trk.gjobs.assign(nc, nullptr);
        trk.ngj.assign(nc, 0);
        trk.ls.assign(nc, LaunchShape{});
        trk.launched.assign(nc, 0);
        trk.reported.assign(nc, 0);
        int at = 0;
        for (int c = 0; c < nc; ++c) {
            const int first = at;
            for (int q = 0; q < nj; ++q)
                if (pend[q].clip == c) {
                    trk.slots[c].push_back(slot[q]);
                    trk.ls[c].add(shape_of(pend[q]), clips[c].p.channels);
                    h_gjobs[at++] = h_jobs[slot[q]];
                }
            for (int q = 0; q < nm; ++q)
                if (pend[memo[q].src].clip == c) {
                    trk.ls[c].add(shape_of(pend[memo[q].src]), clips[c].p.channels);
                    h_gjobs[at++] = h_jobs[nj + q];
                }
            trk.gjobs[c] = d_gjobs + first;
            trk.ngj[c] = at - first;
        }
        SCPL_TRY(hipMemcpyAsync(d_gjobs, h_gjobs, sizeof(Job) * (size_t)at, hipMemcpyHostToDevice, s));
        // the gathers start after the work the call has put on s so far
        SCPL_TRY(hipEventRecord(ctx->gathers_done, s));
        SCPL_TRY(hipStreamWaitEvent(ctx->gather_stream, ctx->gathers_done, 0));
    }
    // gathers the memorised buffers [lo, hi) on stream s, after their sources
    auto gather_memo = [&](int lo, int hi) -> scpl_status {
        if (lo >= hi) return SCPL_OK;
        LaunchShape ls;
        for (int q = lo; q < hi; ++q) ls.add(shape_of(pend[memo[q].src]), clips[pend[memo[q].src].clip].p.channels);
        {
            ProfScope ps(ctx, SCPL_KERNEL_GATHER, s);
            launch_gather(d_jobs + nj + lo, hi - lo, ls.Hmax, ls.gin, ls.gout, ls.Wmax, ctx->gather_variant, s);
        }
        SCPL_CHECK_LAUNCH();
        return SCPL_OK;
    };
    SCPL_TRY(ensure_groups(ctx, ng));
    ctx->last_log.clear();
    auto make_group = [&](int first, int n, hipStream_t st, hipEvent_t ev) {
        Group G;
        G.d_jobs = d_jobs + first;
        G.h_jobs = h_jobs + first;
        G.d_states = d_states + 4 * first;
        G.h_states = h_states + 4 * first;
        G.nj = n;
        G.st = st;
        G.ev = ev;
        for (int q = 0; q < nj; ++q)
            if (slot[q] >= first && slot[q] < first + n) {
                G.ls.add(shape_of(pend[q]), clips[pend[q].clip].p.channels);
                G.rfirst = std::max(G.rfirst, first_batch_iterations(&clips[pend[q].clip].p));
            }
        return G;
    };
    if (persist) {
        LaunchShape ls;
        for (const Pending &q : pend) ls.add(shape_of(q), clips[q.clip].p.channels);
        st = run_persistent(ctx, d_jobs, nj, ls, gpers, pcap, nring, parea, use_graph, s);
        if (st != SCPL_OK) {
            (void)hipStreamSynchronize(s);
            return st;
        }
        // every job must have reached its target width, and no workgroup
        // may have given up waiting
        // (the abort flag lands in the window-sum staging, unused after the segmentation)
        int32_t *h_abort = reinterpret_cast<int32_t *>(h_sums);
        SCPL_TRY(hipMemcpyAsync(h_states, d_states, (size_t)nj * 16, hipMemcpyDeviceToHost, s));
        SCPL_TRY(hipMemcpyAsync(h_abort, &reinterpret_cast<PState *>(parea)->abort, 4, hipMemcpyDeviceToHost, s));
        SCPL_TRY(hipStreamSynchronize(s));
        if (*h_abort != 0) return SCPL_ERR_INTERNAL;
        for (int j = 0; j < nj; ++j)
            if (h_states[4 * j] < 0) return SCPL_ERR_INTERNAL;
        st = gather_memo(0, nm);
        if (st != SCPL_OK) return st;
        return collect_logs(ctx, jobs, s);
    }
    if (batched) {
        std::vector<Group> gs;
        for (int g = 0; g < ng; ++g) {
            gs.push_back(make_group(gfirst[g], gsize[g], ng > 1 ? ctx->gstreams[g] : s, ctx->gevents[g]));
            gs.back().slot = g;
        }
        if (early) {
            for (Group &G : gs) G.gather = false;
            for (int q = 0; q < 4 * nj; ++q) h_states[q] = -1;  // before any read-back is enqueued
        }
        st = run_groups(ctx, gs, use_graph, s, early ? &trk : nullptr);
        if (st != SCPL_OK) return st;
        if (!early) {
            st = gather_memo(0, nm);
            if (st != SCPL_OK) return st;
        }
        return collect_logs(ctx, jobs, s);
    }
    // plain: the next buffer reuses the job area, so a source's memorised
    // buffers are gathered right after it (they follow it in `memo`)
    int mq = 0;
    for (int q = 0; q < nj; ++q) {
        std::vector<Group> gs(1, make_group(slot[q], 1, s, ctx->gevents[0]));
        st = run_groups(ctx, gs, false, s);
        if (st != SCPL_OK) return st;
        int mend = mq;
        while (mend < nm && memo[mend].src == q) ++mend;
        st = gather_memo(mq, mend);
        if (st != SCPL_OK) return st;
        mq = mend;
        std::vector<Job> single(1, jobs[q]);
        st = collect_logs(ctx, single, s);
        if (st != SCPL_OK) return st;
    }
    return SCPL_OK;
}

// Width pass for every clip, then the height pass (transposed) for the clips
// with a target height.  Each pass is one run of the clips it concerns.
scpl_status scpl::run_clips_2d(scpl_ctx *ctx, const scpl_clip *clips, int nc, bool batched, int32_t *h_nbuf_first,
                               hipStream_t s, bool use_graph, const ClipDone *on_done)
{
    bool any = false;
    size_t tbytes = 0;
    for (int c = 0; c < nc; ++c)
        if (height_pass(clips[c].p)) {
            any = true;
            tbytes += height_temp_bytes(clips[c].p);
            if (clips[c].p.target_width < clips[c].p.width && clips[c].d_masks) return SCPL_ERR_INVALID_ARG;
        }
    if (!any) return run_clips(ctx, clips, nc, batched, h_nbuf_first, s, use_graph, on_done);
    SCPL_TRY(ensure_tws(ctx, tbytes));
    std::vector<scpl_clip> pass1, pass2;
    struct Back {
        const scpl_clip *clip;
        uint8_t *tout;
        uint16_t *tmask;
    };
    std::vector<Back> back;
    Bump tb{static_cast<char *>(ctx->tws)};
    std::vector<uint8_t *> src2(nc, nullptr);
    std::vector<int> orig1;  // clip of each width-pass entry, -1 for the width pass of a 2-D clip
    for (int c = 0; c < nc; ++c) {
        const scpl_clip &cl = clips[c];
        if (!height_pass(cl.p)) {
            pass1.push_back(cl);
            orig1.push_back(c);
            continue;
        }
        const size_t N = cl.p.n_frames, H = cl.p.height, C = cl.p.channels, Ws = cl.p.target_width;
        if (cl.p.target_width < cl.p.width) {  // width first, into a temporary
            scpl_clip w = cl;
            w.p.target_height = 0;
            w.d_out = tb.take<uint8_t>(N * H * Ws * C);
            w.d_masks = nullptr;
            src2[c] = w.d_out;
            pass1.push_back(w);
            orig1.push_back(-1);
        }
    }
    int32_t nb1 = 0;
    std::vector<int32_t> log1;
    if (!pass1.empty()) {
        const ClipDone done1 = [&](int i) {
            if (orig1[i] >= 0) (*on_done)(orig1[i]);
        };
        SCPL_TRY(run_clips(ctx, pass1.data(), (int)pass1.size(), batched, &nb1, s, use_graph,
                           on_done ? &done1 : nullptr));
        log1 = ctx->last_log;
    }
    for (int c = 0; c < nc; ++c) {
        const scpl_clip &cl = clips[c];
        if (!height_pass(cl.p)) continue;
        const size_t N = cl.p.n_frames, H = cl.p.height, C = cl.p.channels, Ws = cl.p.target_width;
        const size_t Ht = cl.p.target_height;
        const bool both = cl.p.target_width < cl.p.width;
        scpl_clip t{};
        t.p = transposed_params(cl.p);
        uint8_t *tin = tb.take<uint8_t>(N * Ws * H * C);
        launch_transpose(both ? src2[c] : cl.d_frames, (int)N, (int)H, (int)Ws, (int)C, tin, s);
        t.d_frames = tin;
        t.d_out = tb.take<uint8_t>(N * Ws * Ht * C);
        t.d_masks = (!both && cl.d_masks) ? tb.take<uint16_t>(N * Ws * H) : nullptr;
        int32_t *tbid = tb.take<int32_t>(N);
        t.d_buffer_id = both ? tbid : cl.d_buffer_id;
        pass2.push_back(t);
        back.push_back({&cl, t.d_out, t.d_masks});
    }
    SCPL_CHECK_LAUNCH();
    int32_t nb2 = 0;
    SCPL_TRY(run_clips(ctx, pass2.data(), (int)pass2.size(), batched, &nb2, s, use_graph));
    for (const Back &b : back) {
        const scpl_clip &cl = *b.clip;
        const int N = cl.p.n_frames, H = cl.p.height, Ws = cl.p.target_width, Ht = cl.p.target_height;
        launch_transpose(b.tout, N, Ws, Ht, cl.p.channels, cl.d_out, s);
        if (b.tmask) launch_transpose16(b.tmask, N, Ws, H, cl.d_masks, s);
    }
    SCPL_CHECK_LAUNCH();
    log1.insert(log1.end(), ctx->last_log.begin(), ctx->last_log.end());
    ctx->last_log.swap(log1);
    if (h_nbuf_first) *h_nbuf_first = height_pass(clips[0].p) && clips[0].p.target_width == clips[0].p.width ? nb2 : nb1;
    return SCPL_OK;
}

extern "C" {

scpl_status scpl_retarget(scpl_ctx *ctx, const scpl_params *p, const uint8_t *d_frames, uint8_t *d_out,
                          uint16_t *d_masks, int32_t *d_buffer_id, int32_t *h_n_buffers, void *d_workspace,
                          uint64_t workspace_bytes, void *stream)
{
    if (!ctx || !d_frames || !d_out) return SCPL_ERR_INVALID_ARG;
    scpl_status st = validate(p);
    if (st != SCPL_OK) return st;
    if (d_workspace) {
        if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign != 0) return SCPL_ERR_INVALID_ARG;
        if (workspace_bytes < plain_layout(*p).total()) return SCPL_ERR_INVALID_ARG;
    }
    SCPL_TRY(hipSetDevice(ctx->device));
    scpl_clip c{*p, d_frames, d_out, d_masks, d_buffer_id};
    if (!d_workspace) return run_clips_2d(ctx, &c, 1, false, h_n_buffers, static_cast<hipStream_t>(stream));
    FixedArena arena(ctx, d_workspace, plain_layout(*p), false);
    return run_clips_2d(ctx, &c, 1, false, h_n_buffers, static_cast<hipStream_t>(stream));
}

scpl_status scpl_retarget_noalloc(scpl_ctx *ctx, const scpl_params *p, const uint8_t *d_frames, uint8_t *d_out,
                                  uint16_t *d_masks, int32_t *d_buffer_id, int32_t *h_n_buffers, void *stream)
{
    if (!ctx || !d_frames || !d_out) return SCPL_ERR_INVALID_ARG;
    scpl_status st = validate(p);
    if (st != SCPL_OK) return st;
    if (ctx->profiling) return SCPL_ERR_INVALID_ARG;  // kernel timing creates events
    const PlainLayout L = plain_layout(*p);
    if (L.total() > SCPL_NOALLOC_SCRATCH_BYTES) return SCPL_ERR_CAPACITY;
    if (!ctx->scratch || pinned_bytes(1, p->n_frames) > ctx->pinned_size) return SCPL_ERR_INTERNAL;
    SCPL_TRY(hipSetDevice(ctx->device));
    scpl_clip c{*p, d_frames, d_out, d_masks, d_buffer_id};
    FixedArena arena(ctx, ctx->scratch, L, true);
    return run_clips_2d(ctx, &c, 1, false, h_n_buffers, static_cast<hipStream_t>(stream));
}

scpl_status scpl_retarget_batch(scpl_ctx *ctx, const scpl_clip *clips, int32_t n_clips, void *stream)
{
    if (!ctx || !clips || n_clips < 1) return SCPL_ERR_INVALID_ARG;
    for (int c = 0; c < n_clips; ++c) {
        scpl_status st = validate(&clips[c].p);
        if (st != SCPL_OK) return st;
        if (!clips[c].d_frames || !clips[c].d_out) return SCPL_ERR_INVALID_ARG;
    }
    SCPL_TRY(hipSetDevice(ctx->device));
    return run_clips_2d(ctx, clips, n_clips, true, nullptr, static_cast<hipStream_t>(stream));
}

scpl_status scpl_persist_stats(scpl_ctx *ctx, double *h_ms, int64_t *h_items)
{
    if (!ctx || !h_ms || !h_items) return SCPL_ERR_INVALID_ARG;
    if (!ctx->persist_traced || ctx->wall_khz <= 0) return SCPL_ERR_NOT_READY;
    const double ms_per_tick = 1.0 / (double)ctx->wall_khz;
    for (int q = 0; q < 7; ++q) {
        const int at = q < 5 ? 2 * q : q == 5 ? kPTraceWait : kPTraceDone;
        h_ms[q] = (double)ctx->persist_trace[at] * ms_per_tick;
        h_items[q] = q < 6 ? (int64_t)ctx->persist_trace[at + 1] : ctx->persist_trace[kPTraceWait + 1];
    }
    return SCPL_OK;
}

scpl_status scpl_persist_workgroups(scpl_ctx *ctx, int32_t per_cu)
{
    if (!ctx || per_cu < 0) return SCPL_ERR_INVALID_ARG;
    if (ctx->persist_max_per_cu <= 0) return SCPL_ERR_DEVICE;
    const int n = per_cu == 0 ? ctx->persist_max_per_cu : std::min<int>(per_cu, ctx->persist_max_per_cu);
    ctx->persist_grid = std::min(n * ctx->ncu, 8192);
    return SCPL_OK;
}

scpl_status scpl_device_xcds(scpl_ctx *ctx, int32_t *h_n)
{
    if (!ctx || !h_n) return SCPL_ERR_INVALID_ARG;
    *h_n = ctx->nxcd;
    return SCPL_OK;
}

scpl_status scpl_batch_mode(scpl_ctx *ctx, int32_t mode)
{
    if (!ctx || mode < SCPL_BATCH_GROUPS || mode > SCPL_BATCH_PERSISTENT_AGENT) return SCPL_ERR_INVALID_ARG;
    // the one-ring agent-scope kernel is switched off: a run of it faulted
    // the GPU with no cause found in its code
    if (mode == SCPL_BATCH_PERSISTENT_AGENT) return SCPL_ERR_DEVICE;
    if (mode != SCPL_BATCH_GROUPS && ctx->persist_grid <= 0) return SCPL_ERR_DEVICE;
    ctx->batch_mode = mode;
    return SCPL_OK;
}

scpl_status scpl_batch_streams(scpl_ctx *ctx, int32_t n)
{
    if (!ctx || n < 1 || n > SCPL_MAX_STREAMS) return SCPL_ERR_INVALID_ARG;
    ctx->nstreams = n;
    return SCPL_OK;
}

scpl_status scpl_profile_enable(scpl_ctx *ctx, int32_t on)
{
    if (!ctx) return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    SCPL_TRY(prof_drain(ctx));
    for (int k = 0; k < SCPL_KERNEL_COUNT; ++k) {
        ctx->prof_ms[k] = 0.0;
        ctx->prof_n[k] = 0;
    }
    ctx->profiling = on != 0;
    return SCPL_OK;
}

scpl_status scpl_profile_kinds(scpl_ctx *ctx, uint32_t mask)
{
    if (!ctx || (mask >> SCPL_KERNEL_COUNT) != 0) return SCPL_ERR_INVALID_ARG;
    ctx->prof_mask = mask;
    return SCPL_OK;
}

scpl_status scpl_profile_read(scpl_ctx *ctx, int32_t kernel, double *h_total_ms, int64_t *h_launches)
{
    if (!ctx || kernel < 0 || kernel >= SCPL_KERNEL_COUNT || !h_total_ms || !h_launches) return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    SCPL_TRY(prof_drain(ctx));
    *h_total_ms = ctx->prof_ms[kernel];
    *h_launches = ctx->prof_n[kernel];
    return SCPL_OK;
}

scpl_status scpl_last_log(scpl_ctx *ctx, int32_t *h_log, int64_t cap, int64_t *h_count)
{
    if (!ctx || !h_count || cap < 0 || (cap > 0 && !h_log)) return SCPL_ERR_INVALID_ARG;
    const int64_t n = (int64_t)ctx->last_log.size() / 4;
    *h_count = n;
    const int64_t m = std::min(n, cap);
    if (m > 0) std::memcpy(h_log, ctx->last_log.data(), (size_t)m * 16);
    return SCPL_OK;
}

// ------------------------------------------------------------------ stages

scpl_status scpl_luma(scpl_ctx *ctx, const uint8_t *d_rgb, int64_t npx, uint8_t *d_y, void *stream)
{
    if (!ctx || npx < 0 || (npx > 0 && (!d_rgb || !d_y))) return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    launch_luma(d_rgb, d_y, npx, static_cast<hipStream_t>(stream));
    SCPL_CHECK_LAUNCH();
    return SCPL_OK;
}

// A single-job workspace for the stage entry points.
static scpl_status stage_job(scpl_ctx *ctx, int32_t H, int32_t W, int32_t Wt, int32_t k, size_t extra, Job &J,
                             Job *&d_job, int32_t *&d_state, char *&d_extra, hipStream_t s)
{
    JobShape js{H, W, Wt, k, select_geom(ctx, W, 1)};
    const size_t total = job_bytes(js) + align_up(sizeof(Job)) + align_up(16) + align_up(extra);
    SCPL_TRY(ensure_ws(ctx, total));
    SCPL_TRY(ensure_pinned(ctx, align_up(sizeof(Job)) + 64));
    Bump dev{static_cast<char *>(ctx->ws)};
    char *job_ws = dev.take<char>(job_bytes(js));
    d_job = dev.take<Job>(1);
    d_state = dev.take<int32_t>(4);
    d_extra = dev.take<char>(extra);
    Bump jb{job_ws};
    carve_job(J, js, jb, d_state);
    Job *h = static_cast<Job *>(ctx->pinned);
    SCPL_TRY(hipStreamSynchronize(s));  // the staging slot may still feed an earlier copy
    *h = J;
    SCPL_TRY(hipMemcpyAsync(d_job, h, sizeof(Job), hipMemcpyHostToDevice, s));
    return SCPL_OK;
}

scpl_status scpl_energy(scpl_ctx *ctx, int32_t H, int32_t W, int32_t mode, const uint8_t *d_y,
                        const uint8_t *d_yprev, int32_t *d_e, void *stream)
{
    if (!ctx || !d_y || !d_e || H < 1 || W < 1 || H > SCPL_MAX_HEIGHT || W > SCPL_MAX_WIDTH ||
        (int64_t)H * W > SCPL_MAX_PIXELS || (mode != 0 && mode != 1))
        return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t FS = tiled_frame_bytes(H, W);
    Job J{};
    Job *d_job;
    int32_t *d_state;
    char *d_two;
    // the job sees a 2-frame tiled clip [yprev, y] and carves frame 1 with T = 1
    scpl_status st = stage_job(ctx, H, W, 1, 1, 2 * (size_t)FS, J, d_job, d_state, d_two, s);
    if (st != SCPL_OK) return st;
    uint8_t *two = reinterpret_cast<uint8_t *>(d_two);
    if (d_yprev) launch_tile_luma(d_yprev, 1, 1, H, W, two, s);
    launch_tile_luma(d_y, 1, 1, H, W, two + FS, s);
    J.frames = d_y;
    J.luma = two;
    J.ntc = tiles_across(W);
    J.FS = FS;
    J.C = 1;
    J.mode = mode;
    J.t0 = 1;
    J.T = 1;
    J.has_prev = (mode == SCPL_ENERGY_MOTION && d_yprev) ? 1 : 0;
    J.Wt = 0;  // never "done": the energy of the full width is wanted
    Job *h = static_cast<Job *>(ctx->pinned);
    SCPL_TRY(hipStreamSynchronize(s));
    *h = J;
    SCPL_TRY(hipMemcpyAsync(d_job, h, sizeof(Job), hipMemcpyHostToDevice, s));
    LaunchShape ls;
    ls.add(JobShape{H, W, 1, 1, select_geom(ctx, W, 1)});
    launch_init_jobs(d_job, 1, ls.Hmax, ls.Wmax, s);
    launch_energy(d_job, 1, H, W, s);
    launch_keys_to_u(J.K + J.KL, d_e, H, W, J.Kp, s);
    SCPL_CHECK_LAUNCH();
    SCPL_TRY(hipStreamSynchronize(s));  // the pinned job slot is reused by the next call
    return SCPL_OK;
}

scpl_status scpl_dp(scpl_ctx *ctx, int32_t H, int32_t W, const int32_t *d_u, int32_t *d_ce_last,
                    int32_t *d_label_last, int8_t *d_dir, void *stream)
{
    if (!ctx || !d_u || !d_ce_last || !d_label_last || !d_dir || H < 1 || W < 1 || H > SCPL_MAX_DP_STAGE_HEIGHT ||
        W > SCPL_MAX_WIDTH || (int64_t)H * W > SCPL_MAX_PIXELS)
        return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Job J{};
    Job *d_job;
    int32_t *d_state;
    char *d_flag;
    scpl_status st = stage_job(ctx, H, W, 0, 1, 4, J, d_job, d_state, d_flag, s);
    if (st != SCPL_OK) return st;
    LaunchShape ls;
    ls.add(JobShape{H, W, 0, 1, select_geom(ctx, W, 1)});
    int32_t *bad = reinterpret_cast<int32_t *>(d_flag);
    int32_t *h_bad = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned) + align_up(sizeof(Job)));
    SCPL_TRY(hipMemsetAsync(bad, 0, 4, s));
    launch_init_jobs(d_job, 1, H, W, s);
    launch_u_to_keys(d_u, J.K + J.KL, H, W, J.Kp, bad, s);
    SCPL_CHECK_LAUNCH();
    SCPL_TRY(hipMemcpyAsync(h_bad, bad, 4, hipMemcpyDeviceToHost, s));
    SCPL_TRY(hipStreamSynchronize(s));
    if (*h_bad) return SCPL_ERR_INVALID_ARG;  // eq. (4) keys hold 4 U in 16 bits
    launch_dp(d_job, 1, ls.g, W, H, s);
    launch_borg(d_job, 1, ls.nbmax, ls.Bmax, W, 0, s);
    launch_labels(d_job, 1, W, s);
    launch_dir_out(J.dir, J.Wp, d_dir, H, W, s);
    SCPL_CHECK_LAUNCH();
    SCPL_TRY(hipMemcpyAsync(d_ce_last, J.ce_last, (size_t)W * 4, hipMemcpyDeviceToDevice, s));
    SCPL_TRY(hipMemcpyAsync(d_label_last, J.lab_last, (size_t)W * 4, hipMemcpyDeviceToDevice, s));
    SCPL_TRY(hipStreamSynchronize(s));
    return SCPL_OK;
}

scpl_status scpl_select(scpl_ctx *ctx, int32_t W, const int32_t *d_ce_last, const int32_t *d_label_last, int32_t k,
                        int32_t limit, int32_t *d_children, int32_t *h_kiter, int32_t *h_peff, void *stream)
{
    if (!ctx || !d_ce_last || !d_label_last || !d_children || !h_kiter || W < 1 || W > SCPL_MAX_WIDTH || k < 1 ||
        limit < 1 || limit > W)
        return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Job J{};
    Job *d_job;
    int32_t *d_state;
    char *unused;
    const int H = 1;
    scpl_status st = stage_job(ctx, H, W, W - limit, k, 0, J, d_job, d_state, unused, s);
    if (st != SCPL_OK) return st;
    launch_init_jobs(d_job, 1, H, W, s);
    SCPL_TRY(hipMemcpyAsync(J.ce_last, d_ce_last, (size_t)W * 4, hipMemcpyDeviceToDevice, s));
    SCPL_TRY(hipMemcpyAsync(J.lab_last, d_label_last, (size_t)W * 4, hipMemcpyDeviceToDevice, s));
    launch_select(d_job, 1, 1, ctx->lds_cap, s);
    SCPL_CHECK_LAUNCH();
    int32_t rec[4];
    SCPL_TRY(hipMemcpyAsync(rec, J.log, 16, hipMemcpyDeviceToHost, s));
    SCPL_TRY(hipStreamSynchronize(s));
    *h_kiter = rec[2];
    if (h_peff) *h_peff = rec[1];
    if (rec[2] > 0)
        SCPL_TRY(hipMemcpyAsync(d_children, J.children, (size_t)rec[2] * 4, hipMemcpyDeviceToDevice, s));
    SCPL_TRY(hipStreamSynchronize(s));
    return SCPL_OK;
}

scpl_status scpl_backtrack(scpl_ctx *ctx, int32_t H, int32_t W, const int8_t *d_dir, const int32_t *d_children,
                           int32_t kk, int32_t *d_seams, void *stream)
{
    if (!ctx || !d_dir || H < 1 || W < 1 || H > SCPL_MAX_HEIGHT || W > SCPL_MAX_WIDTH ||
        (int64_t)H * W > SCPL_MAX_PIXELS || kk < 0 || kk > W || (kk > 0 && (!d_children || !d_seams)))
        return SCPL_ERR_INVALID_ARG;
    if (kk == 0) return SCPL_OK;
    SCPL_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Job J{};
    Job *d_job;
    int32_t *d_state;
    char *unused;
    scpl_status st = stage_job(ctx, H, W, 0, kk, 0, J, d_job, d_state, unused, s);
    if (st != SCPL_OK) return st;
    launch_init_jobs(d_job, 1, H, W, s);
    launch_dir_in(d_dir, J.dir, J.Wp, H, W, s);
    SCPL_TRY(hipMemcpyAsync(J.children, d_children, (size_t)kk * 4, hipMemcpyDeviceToDevice, s));
    int32_t rec[4] = {W, 0, kk, 0};
    int32_t *h = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned) + align_up(sizeof(Job)));
    SCPL_TRY(hipStreamSynchronize(s));
    std::memcpy(h, rec, 16);
    SCPL_TRY(hipMemcpyAsync(J.log, h, 16, hipMemcpyHostToDevice, s));
    LaunchShape ls;
    ls.add(JobShape{H, W, 0, kk, select_geom(ctx, W, 1)});
    launch_borg(d_job, 1, ls.nbmax, ls.Bmax, W, 0, s);
    launch_jump_only(d_job, 1, s);
    launch_fill(d_job, 1, kk, ls.nbmax, ls.Bmax, s);
    launch_seams_out(J.seams, J.kcap, d_seams, kk, H, s);
    SCPL_CHECK_LAUNCH();
    SCPL_TRY(hipStreamSynchronize(s));
    return SCPL_OK;
}

scpl_status scpl_dp_geometry(scpl_ctx *ctx, int32_t Q, int32_t HB, int32_t PF, int32_t EX)
{
    if (!ctx || (EX != 0 && EX != 1)) return SCPL_ERR_INVALID_ARG;
    if (Q == 0) {
        ctx->forced = DpGeom{0, 0, 0, 0, 0};
        return SCPL_OK;
    }
    for (int v = 0; v < kNumDpVariants; ++v)
        if (kDpVariants[v].Q == Q && kDpVariants[v].HB == HB && (PF == 0 || kDpVariants[v].PF == PF)) {
            ctx->forced = kDpVariants[v];
            ctx->forced.EX = EX;
            return SCPL_OK;
        }
    if (Q == 32 && HB == 0 && (PF == 0 || PF == 2)) {
        ctx->forced = DpGeom{32, 0, 0, 2, EX};
        return SCPL_OK;
    }
    return SCPL_ERR_INVALID_ARG;
}

scpl_status scpl_dp_chunking(scpl_ctx *ctx, int32_t R, int32_t P)
{
    if (!ctx || R < 0 || P < 0) return SCPL_ERR_INVALID_ARG;
    if (R == 0) {
        ctx->forced.R = 0;
        ctx->forced.P = 0;
        return SCPL_OK;
    }
    DpGeom g = ctx->forced;
    g.R = R;
    g.P = P;
    if (g.Q <= 0 || !g.banded || P > SCPL_MAX_WIDTH || R > SCPL_MAX_HEIGHT || !dp_geom_fits(g, 1))
        return SCPL_ERR_INVALID_ARG;
    ctx->forced = g;
    return SCPL_OK;
}

scpl_status scpl_dp_chosen(scpl_ctx *ctx, int32_t W, int32_t *h_geom)
{
    if (!ctx || !h_geom || W < 1 || W > SCPL_MAX_WIDTH) return SCPL_ERR_INVALID_ARG;
    const DpGeom g = select_geom(ctx, W);
    const int32_t v[6] = {g.Q, g.banded ? g.HB : 0, g.PF, g.EX, g.R, g.P};
    for (int q = 0; q < 6; ++q) h_geom[q] = v[q];
    return SCPL_OK;
}

scpl_status scpl_kernel_variants(scpl_ctx *ctx, int32_t update_variant, int32_t refresh_variant,
                                 int32_t borg_variant, int32_t gather_variant, int32_t fuse_variant)
{
    if (!ctx || update_variant < 0 || update_variant >= kNumUpdateVariants || refresh_variant < 0 ||
        refresh_variant >= kNumRefreshVariants || borg_variant < 0 || borg_variant >= kNumBorgVariants ||
        gather_variant < 0 || gather_variant >= kNumGatherVariants || fuse_variant < 0 ||
        fuse_variant >= kNumFuseVariants)
        return SCPL_ERR_INVALID_ARG;
    ctx->fuse_variant = fuse_variant;
    ctx->upd_variant = update_variant;
    ctx->refresh_variant = refresh_variant;
    ctx->borg_variant = borg_variant;
    ctx->gather_variant = gather_variant;
    return SCPL_OK;
}

scpl_status scpl_autotune_batch(scpl_ctx *ctx, const scpl_clip *clips, int32_t n_clips, int32_t reps,
                                int32_t *h_choice, double *h_ms, void *stream)
{
    if (!ctx || !clips || n_clips < 1 || reps < 1 || reps > 100 || ctx->profiling) return SCPL_ERR_INVALID_ARG;
    for (int c = 0; c < n_clips; ++c) {
        scpl_status st = validate(&clips[c].p);
        if (st != SCPL_OK) return st;
        if (!clips[c].d_frames || !clips[c].d_out) return SCPL_ERR_INVALID_ARG;
    }
    SCPL_TRY(hipSetDevice(ctx->device));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    struct Cfg {
        int streams;
        DpGeom g;  // Q = 0: whatever the launches would take unforced (tuned or default)
        int upd, refresh, borg, gather, fuse;
        int mode;   // SCPL_BATCH_GROUPS or SCPL_BATCH_PERSISTENT
        int pgrid;  // workgroups of the persistent launch
    };
    // the best of `reps` whole batched retargets after one untimed one (graphs,
    // workspace); the caller's outputs are written each time, identically
    auto time_cfg = [&](const Cfg &c, double *ms) -> scpl_status {
        ctx->nstreams = c.streams;
        ctx->batch_forced = c.g;
        ctx->upd_variant = c.upd;
        ctx->refresh_variant = c.refresh;
        ctx->borg_variant = c.borg;
        ctx->gather_variant = c.gather;
        ctx->fuse_variant = c.fuse;
        ctx->batch_mode = c.mode;
        ctx->persist_grid = c.pgrid;
        SCPL_TRY(run_clips_2d(ctx, clips, n_clips, true, nullptr, s, true));
        SCPL_TRY(hipStreamSynchronize(s));
        double best = 1e300;
        for (int q = 0; q < reps; ++q) {
            const auto t0 = std::chrono::steady_clock::now();
            SCPL_TRY(run_clips_2d(ctx, clips, n_clips, true, nullptr, s, true));
            SCPL_TRY(hipStreamSynchronize(s));
            const std::chrono::duration<double, std::milli> d = std::chrono::steady_clock::now() - t0;
            best = std::min(best, d.count());
        }
        *ms = best;
        return SCPL_OK;
    };
    if (ctx->forced.Q > 0) return SCPL_ERR_INVALID_ARG;  // a geometry forced by the caller would win anyway
    const Cfg start{ctx->nstreams,     ctx->batch_forced,   ctx->upd_variant, ctx->refresh_variant,
                    ctx->borg_variant, ctx->gather_variant, ctx->fuse_variant, ctx->batch_mode,
                    ctx->persist_grid};
    std::vector<DpGeom> geoms{DpGeom{0, 0, 0, 0, 0}, DpGeom{8, 16, 1, 8, 1}, DpGeom{4, 16, 1, 16, 1},
                              DpGeom{4, 16, 1, 8, 1, 256, 384}, DpGeom{2, 8, 1, 16, 1, 128, 640}};
    if (start.g.Q > 0) geoms[0] = start.g;
    // the configuration the calls would use now is the incumbent; a
    // candidate replaces it only when it is at least 1% faster, so that
    // run-to-run noise does not decide the choice
    Cfg best = start;
    best.g = geoms[0];
    double best_ms = 1e300, ms = 0.0;
    scpl_status st = time_cfg(best, &best_ms);
    auto challenge = [&](const Cfg &c) {
        if (st != SCPL_OK) return;
        st = time_cfg(c, &ms);
        if (st == SCPL_OK && ms < 0.99 * best_ms) {
            best_ms = ms;
            best = c;
        }
    };
    // coordinate descent: job groups with DP geometry, then the compaction,
    // refresh and band-origin variants
    const Cfg inc = best;
    for (int ns : {2, 3, 4})
        for (const DpGeom &g : geoms)
            if (inc.mode != SCPL_BATCH_GROUPS || ns != inc.streams || std::memcmp(&g, &inc.g, sizeof g) != 0)
                challenge(Cfg{ns, g, inc.upd, inc.refresh, inc.borg, inc.gather, inc.fuse, SCPL_BATCH_GROUPS,
                              inc.pgrid});
    for (int u = 0; u < kNumUpdateVariants; ++u)
        if (u != best.upd) {
            Cfg c = best;
            c.upd = u;
            challenge(c);
        }
    for (int r = 0; r < kNumRefreshVariants; ++r)
        if (r != best.refresh) {
            Cfg c = best;
            c.refresh = r;
            challenge(c);
        }
    for (int b = 0; b < kNumBorgVariants; ++b)
        if (b != best.borg) {
            Cfg c = best;
            c.borg = b;
            challenge(c);
        }
    for (int f = 0; f < kNumFuseVariants; ++f)
        if (f != best.fuse) {
            Cfg c = best;
            c.fuse = f;
            challenge(c);
        }
    // the persistent launch (where the probe found the XCDs): its DP
    // chunking and workgroups per compute unit
    if (ctx->nxcd > 0 && ctx->persist_max_per_cu > 0) {
        const Cfg gb = best;
        for (const DpGeom &g : {DpGeom{4, 16, 1, 8, 1, 256, 384}, DpGeom{4, 16, 1, 8, 1, 192, 512},
                                DpGeom{4, 16, 1, 8, 1, 128, 640}})
            for (int per_cu = ctx->persist_max_per_cu; per_cu >= std::max(2, ctx->persist_max_per_cu - 2); --per_cu) {
                Cfg c = gb;
                c.mode = SCPL_BATCH_PERSISTENT;
                c.g = g;
                c.pgrid = std::min(per_cu * ctx->ncu, 8192);
                challenge(c);
            }
    }
    for (int g = 0; g < kNumGatherVariants; ++g)
        if (g != best.gather) {
            Cfg c = best;
            c.gather = g;
            challenge(c);
        }
    const Cfg keep = st == SCPL_OK ? best : start;
    ctx->nstreams = keep.streams;
    ctx->batch_forced = keep.g;
    ctx->upd_variant = keep.upd;
    ctx->refresh_variant = keep.refresh;
    ctx->borg_variant = keep.borg;
    ctx->gather_variant = keep.gather;
    ctx->fuse_variant = keep.fuse;
    ctx->batch_mode = keep.mode;
    ctx->persist_grid = keep.pgrid;
    if (st != SCPL_OK) return st;
    if (h_choice) {
        const int32_t v[15] = {keep.streams, keep.g.Q,    keep.g.HB, keep.g.PF,    keep.g.EX,
                               keep.g.R,     keep.g.P,    keep.upd,  keep.refresh, keep.g.Q > 0 ? 1 : 0,
                               keep.borg,    keep.gather, keep.fuse, keep.mode,    keep.pgrid};
        std::memcpy(h_choice, v, sizeof v);
    }
    if (h_ms) *h_ms = best_ms;
    return SCPL_OK;
}

scpl_status scpl_autotune_dp(scpl_ctx *ctx, int32_t H, int32_t W, int32_t n_jobs, int32_t *h_Q, int32_t *h_HB,
                             int32_t *h_PF, int32_t *h_EX, double *h_us)
{
    if (!ctx || H < 2 || W < 1 || H > SCPL_MAX_HEIGHT || W > SCPL_MAX_WIDTH || (int64_t)H * W > SCPL_MAX_PIXELS ||
        n_jobs < 1 || n_jobs > 1024)
        return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    hipStream_t s = nullptr;
    std::vector<DpGeom> cand;
    // with several job groups the DP runs beside the other groups' kernels,
    // which a timing in isolation cannot see: it then keeps its compute
    // units to itself (EX = 1)
    const int ex0 = ctx->nstreams > 1 ? 1 : 0;
    for (int v = 0; v < kNumDpVariants + kNumDpChunked; ++v) {
        const DpGeom &gv = v < kNumDpVariants ? kDpVariants[v] : kDpChunked[v - kNumDpVariants];
        if (dp_geom_fits(gv, W))
            for (int ex = ex0; ex < 2; ++ex) {
                DpGeom g = gv;
                g.EX = ex;
                cand.push_back(g);
            }
    }
    if (cand.empty()) {
        DpGeom g = dp_geom(W);
        if (ex0 == 0) cand.push_back(g);
        g.EX = 1;
        cand.push_back(g);
    }
    hipEvent_t e0, e1;
    SCPL_TRY(hipEventCreate(&e0));
    SCPL_TRY(hipEventCreate(&e1));
    DpGeom best = cand[0];
    double best_us = 1e30;
    scpl_status st = SCPL_OK;
    for (const DpGeom &g : cand) {
        // n_jobs concurrent jobs of the same shape, each with its own workspace
        JobShape js{H, W, 0, 1, g};
        const size_t jb = job_bytes(js);
        const size_t total = jb * (size_t)n_jobs + align_up(sizeof(Job) * (size_t)n_jobs) + align_up(16 * (size_t)n_jobs);
        st = ensure_ws(ctx, total);
        if (st != SCPL_OK) break;
        st = ensure_pinned(ctx, align_up(sizeof(Job) * (size_t)n_jobs));
        if (st != SCPL_OK) break;
        Bump dev{static_cast<char *>(ctx->ws)};
        char *job_ws = dev.take<char>(jb * (size_t)n_jobs);
        Job *d_job = dev.take<Job>((size_t)n_jobs);
        int32_t *d_state = dev.take<int32_t>(4 * (size_t)n_jobs);
        Job *h = static_cast<Job *>(ctx->pinned);
        Bump bjb{job_ws};
        for (int q = 0; q < n_jobs; ++q) {
            Job J{};
            carve_job(J, js, bjb, d_state + 4 * q);
            h[q] = J;
        }
        SCPL_TRY(hipMemcpyAsync(d_job, h, sizeof(Job) * (size_t)n_jobs, hipMemcpyHostToDevice, s));
        launch_init_jobs(d_job, n_jobs, H, W, s);
        for (int q = 0; q < n_jobs; ++q) launch_tune_fill(h[q].K, H, W, h[q].Kp, h[q].KL, s);
        launch_dp(d_job, n_jobs, g, W, H, s);  // warm-up
        const int reps = 5;
        SCPL_TRY(hipEventRecord(e0, s));
        for (int q = 0; q < reps; ++q) launch_dp(d_job, n_jobs, g, W, H, s);
        SCPL_TRY(hipEventRecord(e1, s));
        SCPL_TRY(hipEventSynchronize(e1));
        SCPL_CHECK_LAUNCH();
        float ms = 0.f;
        SCPL_TRY(hipEventElapsedTime(&ms, e0, e1));
        const double us = 1e3 * ms / reps;
        if (us < best_us) {
            best_us = us;
            best = g;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SCPL_OK) return st;
    bool found = false;
    for (auto &t : ctx->tuned)
        if (t.W == W && t.n == n_jobs) {
            t.g = best;
            found = true;
        }
    if (!found) ctx->tuned.push_back({W, n_jobs, best});
    const DpGeom chosen = select_geom(ctx, W, n_jobs);
    if (h_Q) *h_Q = chosen.Q;
    if (h_HB) *h_HB = chosen.HB;
    if (h_PF) *h_PF = chosen.PF;
    if (h_EX) *h_EX = chosen.EX;
    if (h_us) *h_us = best_us;
    return SCPL_OK;
}

scpl_status scpl_segment(scpl_ctx *ctx, const scpl_params *p, const uint8_t *d_luma, int32_t *h_buffer_id,
                         int64_t *h_s_trace, int32_t *h_n_buffers, void *stream)
{
    if (!ctx || !d_luma || !h_buffer_id) return SCPL_ERR_INVALID_ARG;
    scpl_status st = validate(p);
    if (st != SCPL_OK) return st;
    SCPL_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t HW = (int64_t)p->height * p->width;
    const int64_t FS = tiled_frame_bytes(p->height, p->width);
    SCPL_TRY(ensure_ws(ctx, align_up(kSegWindow * 8) + align_up(sizeof(SegArgs)) + align_up((size_t)p->n_frames * FS) +
                                seg_bytes(HW)));
    SCPL_TRY(ensure_pinned(ctx, align_up(kSegWindow * 8) + align_up(sizeof(SegArgs))));
    Bump dev{static_cast<char *>(ctx->ws)};
    unsigned long long *d_sums = dev.take<unsigned long long>(kSegWindow);
    SegArgs *d_args = dev.take<SegArgs>(1);
    uint8_t *tiled = dev.take<uint8_t>((size_t)p->n_frames * FS);
    Bump host{static_cast<char *>(ctx->pinned)};
    unsigned long long *h_sums = host.take<unsigned long long>(kSegWindow);
    SegArgs *h_args = host.take<SegArgs>(1);
    std::vector<SegClip> seg(1);
    seg[0].p = p;
    seg[0].tiled = tiled;
    seg[0].FS = FS;
    seg[0].ntc = tiles_across(p->width);
    seg[0].state = dev.take<char>(seg_bytes(HW));
    seg[0].bid = h_buffer_id;
    seg[0].trace = h_s_trace;
    launch_tile_luma(d_luma, 1, p->n_frames, p->height, p->width, tiled, s);
    SCPL_CHECK_LAUNCH();
    st = segment_clips(ctx, seg, d_sums, h_sums, d_args, h_args, s, nullptr, nullptr);
    if (h_n_buffers) *h_n_buffers = seg[0].nbuf;
    return st;
}

scpl_status scpl_asde(scpl_ctx *ctx, int32_t n, int32_t H, int32_t W, int32_t mode, const uint8_t *d_luma,
                      const uint8_t *d_prev, int32_t alpha_num, int32_t alpha_den, int64_t *h_S, int32_t *h_reject,
                      void *stream)
{
    if (!ctx || !d_luma || !h_S || !h_reject || n < 1 || n > SCPL_MAX_FRAMES || H < 1 || W < 1 ||
        H > SCPL_MAX_HEIGHT || W > SCPL_MAX_WIDTH || (int64_t)H * W > SCPL_MAX_PIXELS || (mode != 0 && mode != 1) ||
        alpha_num < 0 || alpha_num > SCPL_MAX_ALPHA_TERM || alpha_den < 1 || alpha_den > SCPL_MAX_ALPHA_TERM)
        return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t HW = (int64_t)H * W;
    const int64_t FS = tiled_frame_bytes(H, W);
    const int pre = (d_prev && mode == SCPL_ENERGY_MOTION) ? 1 : 0;  // tiled frame 0 is the predecessor
    const int nt = n + pre;
    SCPL_TRY(ensure_ws(ctx, align_up(kSegWindow * 8) + align_up(sizeof(SegArgs)) + align_up((size_t)nt * FS) +
                                seg_bytes(HW)));
    SCPL_TRY(ensure_pinned(ctx, align_up(kSegWindow * 8) + align_up(sizeof(SegArgs))));
    Bump dev{static_cast<char *>(ctx->ws)};
    unsigned long long *d_sums = dev.take<unsigned long long>(kSegWindow);
    SegArgs *d_args = dev.take<SegArgs>(1);
    uint8_t *tiled = dev.take<uint8_t>((size_t)nt * FS);
    char *state = dev.take<char>(seg_bytes(HW));
    if (pre) launch_tile_luma(d_prev, 1, 1, H, W, tiled, s);
    launch_tile_luma(d_luma, 1, n, H, W, tiled + (size_t)pre * FS, s);
    SCPL_CHECK_LAUNCH();
    // the moments start from the first frame and take the others in windows
    // of candidates; the sum after the last one is S of the whole buffer
    uint64_t S = 0;  // a single frame has no deviation
    Bump host{static_cast<char *>(ctx->pinned)};
    unsigned long long *h_sums = host.take<unsigned long long>(kSegWindow);
    SegArgs *h_args = host.take<SegArgs>(1);
    for (int tb = pre + 1; tb < nt; tb += kSegWindow) {
        SegArgs a{};
        Bump bp{state};
        a.luma = tiled;
        a.FS = FS;
        a.ntc = tiles_across(W);
        a.s1 = bp.take<uint32_t>(HW);
        a.s2 = bp.take<uint64_t>(HW);
        a.sout = d_sums;
        a.H = H;
        a.W = W;
        a.mode = mode;
        a.t0 = pre;
        a.tb = tb;
        a.te = std::min(nt, tb + kSegWindow);
        a.init = tb == pre + 1 ? 1 : 0;
        SCPL_TRY(hipMemsetAsync(d_sums, 0, kSegWindow * 8, s));
        SCPL_TRY(hipStreamSynchronize(s));  // the pinned argument slot is reused
        *h_args = a;
        SCPL_TRY(hipMemcpyAsync(d_args, h_args, sizeof(SegArgs), hipMemcpyHostToDevice, s));
        launch_seg_windows(d_args, 1, tiles_across(W), H, s);
        SCPL_CHECK_LAUNCH();
        if (a.te == nt) {
            SCPL_TRY(hipMemcpyAsync(h_sums, d_sums, kSegWindow * 8, hipMemcpyDeviceToHost, s));
            SCPL_TRY(hipStreamSynchronize(s));
            S = h_sums[a.te - a.tb - 1];
        }
    }
    *h_S = (int64_t)S;
    *h_reject = asde_rejects(S, n, HW, energy_max(mode), alpha_num, alpha_den) ? 1 : 0;
    return SCPL_OK;
}

scpl_status scpl_compact(scpl_ctx *ctx, int32_t H, int32_t W, int32_t C, const uint8_t *d_in, const int32_t *d_seams,
                         int32_t kk, uint8_t *d_out, void *stream)
{
    if (!ctx || !d_in || !d_out || H < 1 || W < 1 || H > SCPL_MAX_HEIGHT || W > SCPL_MAX_WIDTH ||
        (int64_t)H * W > SCPL_MAX_PIXELS || (C != 1 && C != 3) || kk < 0 || kk >= W || (kk > 0 && !d_seams))
        return SCPL_ERR_INVALID_ARG;
    SCPL_TRY(hipSetDevice(ctx->device));
    launch_compact_frame(d_in, H, W, C, d_seams, kk, d_out, static_cast<hipStream_t>(stream));
    SCPL_CHECK_LAUNCH();
    return SCPL_OK;
}

}  // extern "C"
