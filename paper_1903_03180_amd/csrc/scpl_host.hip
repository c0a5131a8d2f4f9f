// Host runtime of libscpl.so: argument validation, workspace, the ASDE
// buffer controller (Sec. 3.2), the SCPL iteration driver (Sec. 3.1) for the
// plain path (one buffer at a time) and the batched path (every buffer of
// every clip per launch, the iteration loop replayed from a HIP graph), and
// the stage entry points.  Declarations: include/scpl.h.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/scpl.h"
#include "scpl_internal.h"

using namespace scpl;

struct ProfPair {
    hipEvent_t a, b;
    int kind;
};

struct scpl_ctx {
    bool profiling = false;
    std::vector<ProfPair> prof_pending;  // recorded, not yet read
    std::vector<ProfPair> prof_free;     // reusable event pairs
    double prof_ms[SCPL_KERNEL_COUNT] = {};
    int64_t prof_n[SCPL_KERNEL_COUNT] = {};
    int device = 0;
    size_t lds_cap = 65536;
    void *ws = nullptr;        // device workspace
    size_t ws_size = 0;
    void *pinned = nullptr;    // host staging (job tables, sums, states)
    size_t pinned_size = 0;
    std::vector<int32_t> last_log;
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

// Rows per band: 64, or more for wide frames so that the band origins of
// a whole frame (bands x width bytes) still fit in the selection kernel's
// LDS next to its keys (16 bytes per column); int8 offsets cap it at 120.
int32_t band_rows(int32_t H, int32_t W, size_t lds_cap)
{
    const size_t keys = (size_t)16 * W;
    for (int32_t B : {64, 96, 120}) {
        const size_t nb = (size_t)(H + B - 1) / B;
        if (keys + nb * (size_t)W <= lds_cap) return B;
    }
    return kBandMax;
}

size_t g_lds_cap = 65536;  // set from the device at context creation

struct JobShape {
    int32_t H, W, Wt, k;
    int32_t Q = 0;  // DP columns per thread of the launch the job runs in (0: its own width decides)
    int32_t Wp() const { return (int32_t)align_up((size_t)W, 64); }
    int32_t q() const { return Q > 0 ? Q : dp_columns_per_thread(W); }
    int32_t Wq() const { return q() * dp_threads(W, q()); }
    int32_t B() const { return band_rows(H, W, g_lds_cap); }
    int32_t nb() const { return (H + B() - 1) / B(); }
    int32_t kcap() const { return std::min(k, W); }
    int32_t logcap() const { return W - Wt + 2; }
};

size_t job_bytes(const JobShape &s)
{
    const size_t H = s.H, Wp = s.Wp(), W = s.W, nb = s.nb(), kc = s.kcap(), lc = s.logcap();
    size_t b = 0;
    b += 2 * align_up(H * Wp * 2);       // M0, M1
    b += 2 * align_up((H + 1) * (size_t)s.Wq() * 4);  // K0, K1
    b += 2 * align_up(H * Wp * 4);       // SE0, SE1
    b += align_up(H * Wp);               // dir
    b += align_up(nb * Wp);              // borg
    b += align_up(H * W * 2);            // bmask
    b += 2 * align_up(Wp * 4);           // ce_last, lab_last
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
    J.Wq = s.Wq();
    J.B = s.B();
    J.nb = (int32_t)nb;
    J.kcap = (int32_t)kc;
    J.logcap = (int32_t)lc;
    J.M0 = bp.take<int16_t>(H * Wp);
    J.M1 = bp.take<int16_t>(H * Wp);
    J.K0 = bp.take<uint32_t>((H + 1) * (size_t)J.Wq);
    J.K1 = bp.take<uint32_t>((H + 1) * (size_t)J.Wq);
    J.SE0 = bp.take<uint32_t>(H * Wp);
    J.SE1 = bp.take<uint32_t>(H * Wp);
    J.dir = bp.take<uint8_t>(H * Wp);
    J.borg = bp.take<int8_t>(nb * Wp);
    J.bmask = bp.take<uint16_t>(H * W);
    J.ce_last = bp.take<int32_t>(Wp);
    J.lab_last = bp.take<int32_t>(Wp);
    J.keys = bp.take<uint64_t>(2 * Wp);
    J.children = bp.take<int32_t>(kc);
    J.bcol = bp.take<int32_t>(kc * nb);
    J.seams = bp.take<int16_t>(kc * H);
    J.log = bp.take<int32_t>(lc * 4);
    J.state = state;
}

scpl_status ensure_ws(scpl_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->ws_size) return SCPL_OK;
    if (ctx->ws) {
        SCPL_TRY(hipFree(ctx->ws));  // implicitly waits for work using it
        ctx->ws = nullptr;
        ctx->ws_size = 0;
    }
    size_t want = align_up(bytes, (size_t)1 << 20);
    SCPL_TRY(hipMalloc(&ctx->ws, want));
    ctx->ws_size = want;
    return SCPL_OK;
}

scpl_status ensure_pinned(scpl_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->pinned_size) return SCPL_OK;
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
        if (!ctx->profiling) return;
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

size_t seg_bytes(int64_t HW) { return align_up(HW * 4) + align_up(HW * 8) + align_up(kSegWindow * 8); }

// Dynamic spatiotemporal buffer (Sec. 3.2): frames join the current buffer
// while the ASDE of the grown buffer stays at or below phi(n).  Each launch
// scans a window of candidates speculatively; the host accepts them in
// order and restarts from the first rejected frame.
scpl_status segment_clip(scpl_ctx *ctx, const scpl_params *p, const uint8_t *d_luma, void *seg_ws,
                         unsigned long long *h_sums, int32_t *bid, int64_t *trace, int32_t *nbuf, hipStream_t s)
{
    const int N = p->n_frames;
    const int64_t HW = (int64_t)p->height * p->width;
    if (!p->use_buffer) {
        for (int t = 0; t < N; ++t) {
            bid[t] = t;
            if (trace) trace[t] = -1;
        }
        *nbuf = N;
        return SCPL_OK;
    }
    Bump bp{static_cast<char *>(seg_ws)};
    SegArgs a{};
    a.luma = d_luma;
    a.s1 = bp.take<uint32_t>(HW);
    a.s2 = bp.take<uint64_t>(HW);
    a.sout = bp.take<unsigned long long>(kSegWindow);
    a.H = p->height;
    a.W = p->width;
    a.mode = p->energy_mode;
    const int32_t emax = energy_max(p->energy_mode);

    int t0 = 0, n = 1, nb = 0, t = 1;
    bool state_valid = false;
    bid[0] = 0;
    if (trace) trace[0] = -1;
    while (t < N) {
        if (p->max_buffer > 0 && n >= p->max_buffer) {
            if (trace) trace[t] = -1;
            bid[t] = ++nb;
            t0 = t;
            n = 1;
            state_valid = false;
            ++t;
            continue;
        }
        int te = std::min(N, t + kSegWindow);
        if (p->max_buffer > 0) te = std::min(te, t + (p->max_buffer - n));
        a.t0 = t0;
        a.tb = t;
        a.te = te;
        a.init = state_valid ? 0 : 1;
        SCPL_TRY(hipMemsetAsync(a.sout, 0, kSegWindow * 8, s));
        {
            ProfScope ps(ctx, SCPL_KERNEL_SEGMENT, s);
            launch_seg_window(a, s);
        }
        SCPL_CHECK_LAUNCH();
        SCPL_TRY(hipMemcpyAsync(h_sums, a.sout, (size_t)(te - t) * 8, hipMemcpyDeviceToHost, s));
        SCPL_TRY(hipStreamSynchronize(s));
        bool rejected = false;
        for (int tt = t; tt < te; ++tt) {
            const uint64_t S = h_sums[tt - t];
            const int64_t nn = tt - t0 + 1;
            if (trace) trace[tt] = (int64_t)S;
            if (asde_rejects(S, nn, HW, emax, p->alpha_num, p->alpha_den)) {
                bid[tt] = ++nb;
                t0 = tt;
                n = 1;
                state_valid = false;
                t = tt + 1;
                rejected = true;
                break;
            }
            bid[tt] = nb;
            n = (int)nn;
        }
        if (!rejected) {
            state_valid = true;
            t = te;
        }
    }
    *nbuf = nb + 1;
    return SCPL_OK;
}

// ------------------------------------------------------------- iterations

struct LaunchShape {
    int Hmax = 0, Wmax = 0, nbmax = 0, kmax = 0, Bmax = 0, Q = 0;
    void add(const JobShape &s)
    {
        Hmax = std::max(Hmax, s.H);
        Wmax = std::max(Wmax, s.W);
        nbmax = std::max(nbmax, s.nb());
        kmax = std::max(kmax, s.kcap());
        Bmax = std::max(Bmax, s.B());
        Q = std::max(Q, s.q());
    }
};

void enqueue_iteration(scpl_ctx *ctx, const Job *d_jobs, int nj, int r, const LaunchShape &ls, hipStream_t s)
{
    {
        ProfScope ps(ctx, SCPL_KERNEL_DP, s);
        launch_dp(d_jobs, nj, r, ls.Wmax, ls.Q, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_BORG, s);
        launch_borg(d_jobs, nj, r, ls.nbmax, ls.Bmax, ls.Wmax, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_SELECT, s);
        launch_select(d_jobs, nj, r, 0, ctx->lds_cap, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_FILL, s);
        launch_fill(d_jobs, nj, r, ls.kmax, ls.nbmax, ls.Bmax, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_COMPACT, s);
        launch_compact(d_jobs, nj, r, ls.Hmax, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_UPDATE, s);
        launch_update(d_jobs, nj, r, ls.Hmax, ls.Wmax, s);
    }
}

// Runs every SCPL iteration of jobs [0, nj) until all reach their target
// width, then gathers the outputs.  r_first_batch iterations are enqueued
// (captured into a graph when use_graph) before the first look at the
// per-job states; stragglers (iterations that found fewer parents than k)
// get further iterations.
scpl_status run_jobs(scpl_ctx *ctx, const Job *d_jobs, const Job *h_jobs, int32_t *d_states, int32_t *h_states,
                     int nj, const LaunchShape &ls, int r_first_batch, bool use_graph, hipStream_t s)
{
    {
        ProfScope ps(ctx, SCPL_KERNEL_INIT, s);
        launch_init_jobs(d_jobs, nj, ls.Hmax, ls.Wmax, s);
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_ENERGY, s);
        launch_energy(d_jobs, nj, ls.Hmax, ls.Wmax, s);
    }
    SCPL_CHECK_LAUNCH();
    int r = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    if (use_graph && !ctx->profiling && s != nullptr && r_first_batch > 0) {
        SCPL_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (; r < r_first_batch; ++r) enqueue_iteration(ctx, d_jobs, nj, r, ls, s);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(s, &g);
        SCPL_TRY(le);
        SCPL_TRY(ce);
        hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (ie == hipSuccess) ie = hipGraphLaunch(ge, s);
        if (ie != hipSuccess) {
            if (ge) (void)hipGraphExecDestroy(ge);
            (void)hipGraphDestroy(g);
            return dev_status(ie);
        }
    } else {
        for (; r < r_first_batch; ++r) enqueue_iteration(ctx, d_jobs, nj, r, ls, s);
        SCPL_CHECK_LAUNCH();
    }
    // the graph is released once the first state read-back has synchronised
    struct GraphGuard {
        hipGraph_t &g;
        hipGraphExec_t &ge;
        ~GraphGuard()
        {
            if (ge) (void)hipGraphExecDestroy(ge);
            if (g) (void)hipGraphDestroy(g);
        }
    } guard{g, ge};
    for (;;) {
        SCPL_TRY(hipMemcpyAsync(h_states, d_states, (size_t)nj * 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SCPL_TRY(hipStreamSynchronize(s));
        bool all = true;
        int more = 1;
        for (int j = 0; j < nj; ++j) {
            if (h_states[4 * j] >= 0) continue;
            all = false;
            // the job's width and last k_iter bound the iterations it still needs
            const int rem = h_states[4 * j + 1] - h_jobs[j].Wt;
            const int last = std::max(1, h_states[4 * j + 2]);
            more = std::max(more, (rem + last - 1) / last);
        }
        if (all) break;
        if (r > ls.Wmax + 1) return SCPL_ERR_INTERNAL;  // each iteration removes >= 1 column
        for (int q = 0; q < more; ++q, ++r) enqueue_iteration(ctx, d_jobs, nj, r, ls, s);
        SCPL_CHECK_LAUNCH();
    }
    {
        ProfScope ps(ctx, SCPL_KERNEL_GATHER, s);
        launch_gather(d_jobs, nj, ls.Hmax, s);
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

// ===================================================================== C ABI

extern "C" {

const char *scpl_status_str(scpl_status s)
{
    switch (s) {
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
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

scpl_status scpl_workspace_size(const scpl_params *p, uint64_t *device_bytes)
{
    scpl_status st = validate(p);
    if (st != SCPL_OK) return st;
    if (!device_bytes) return SCPL_ERR_INVALID_ARG;
    const int64_t HW = (int64_t)p->height * p->width;
    JobShape js{p->height, p->width, p->target_width, p->seams_per_iter};
    size_t b = 0;
    if (p->channels == 3) b += align_up((size_t)p->n_frames * HW);
    b += seg_bytes(HW) + job_bytes(js) + align_up(sizeof(Job)) + align_up(16);
    *device_bytes = b;
    return SCPL_OK;
}

scpl_status scpl_retarget(scpl_ctx *ctx, const scpl_params *p, const uint8_t *d_frames, uint8_t *d_out,
                          uint16_t *d_masks, int32_t *d_buffer_id, int32_t *h_n_buffers, void *stream)
{
    if (!ctx || !d_frames || !d_out) return SCPL_ERR_INVALID_ARG;
    scpl_status st = validate(p);
    if (st != SCPL_OK) return st;
    SCPL_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int N = p->n_frames;
    const int64_t HW = (int64_t)p->height * p->width;
    JobShape js{p->height, p->width, p->target_width, p->seams_per_iter};

    // device workspace: [luma] [segmentation] [job] [job table] [states]
    const size_t luma_b = p->channels == 3 ? align_up((size_t)N * HW) : 0;
    const size_t seg_b = seg_bytes(HW);
    const size_t job_b = job_bytes(js);
    const size_t total = luma_b + seg_b + job_b + align_up(sizeof(Job) * (size_t)N) + align_up(16 * (size_t)N);
    SCPL_TRY(ensure_ws(ctx, total));
    // host staging: [sums] [states] [jobs] [buffer ids] [trace unused]
    const size_t pin_b = align_up(kSegWindow * 8) + align_up(16 * (size_t)N) + align_up(sizeof(Job) * (size_t)N) +
                         align_up(4 * (size_t)N);
    SCPL_TRY(ensure_pinned(ctx, pin_b));

    Bump dev{static_cast<char *>(ctx->ws)};
    uint8_t *d_luma = luma_b ? dev.take<uint8_t>((size_t)N * HW) : nullptr;
    void *seg_ws = dev.take<char>(seg_b);
    char *job_ws = dev.take<char>(job_b);
    Job *d_jobs = dev.take<Job>((size_t)N);
    int32_t *d_states = dev.take<int32_t>(4 * (size_t)N);

    Bump host{static_cast<char *>(ctx->pinned)};
    unsigned long long *h_sums = host.take<unsigned long long>(kSegWindow);
    int32_t *h_states = host.take<int32_t>(4 * (size_t)N);
    Job *h_jobs = host.take<Job>((size_t)N);
    int32_t *h_bid = host.take<int32_t>((size_t)N);

    const uint8_t *luma = d_frames;
    if (p->channels == 3) {
        ProfScope ps(ctx, SCPL_KERNEL_LUMA, s);
        launch_luma(d_frames, d_luma, (int64_t)N * HW, s);
        SCPL_CHECK_LAUNCH();
        luma = d_luma;
    }
    int32_t nbuf = 0;
    st = segment_clip(ctx, p, luma, seg_ws, h_sums, h_bid, nullptr, &nbuf, s);
    if (st != SCPL_OK) return st;
    if (d_buffer_id) SCPL_TRY(hipMemcpyAsync(d_buffer_id, h_bid, (size_t)N * 4, hipMemcpyHostToDevice, s));
    if (h_n_buffers) *h_n_buffers = nbuf;

    // plain path: one buffer at a time, all sharing one job workspace
    const auto bufs = buffers_of(h_bid, N);
    std::vector<Job> jobs;
    for (size_t b = 0; b < bufs.size(); ++b) {
        Job J = clip_job(p, d_frames, luma, d_out, d_masks, bufs[b].first, bufs[b].second, (int)b);
        Bump jb{job_ws};
        carve_job(J, js, jb, d_states + 4 * b);
        h_jobs[b] = J;
        jobs.push_back(J);
    }
    SCPL_TRY(hipMemcpyAsync(d_jobs, h_jobs, sizeof(Job) * bufs.size(), hipMemcpyHostToDevice, s));
    LaunchShape ls;
    ls.add(js);
    ctx->last_log.clear();
    for (size_t b = 0; b < bufs.size(); ++b) {
        st = run_jobs(ctx, d_jobs + b, &jobs[b], d_states + 4 * b, h_states + 4 * b, 1, ls, first_batch_iterations(p),
                      false, s);
        if (st != SCPL_OK) return st;
        std::vector<Job> one(1, jobs[b]);
        st = collect_logs(ctx, one, s);
        if (st != SCPL_OK) return st;
    }
    return SCPL_OK;
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
    hipStream_t s = static_cast<hipStream_t>(stream);

    // pass 1: luma and segmentation of every clip (luma kept for carving)
    size_t luma_b = 0, seg_b = 0;
    int64_t Ntot = 0;
    for (int c = 0; c < n_clips; ++c) {
        const scpl_params &p = clips[c].p;
        const int64_t HW = (int64_t)p.height * p.width;
        if (p.channels == 3) luma_b += align_up((size_t)p.n_frames * HW);
        seg_b = std::max(seg_b, seg_bytes(HW));
        Ntot += p.n_frames;
    }
    const size_t pin_b = align_up(kSegWindow * 8) + align_up(4 * (size_t)Ntot) + align_up(16 * (size_t)Ntot) +
                         align_up(sizeof(Job) * (size_t)Ntot);
    SCPL_TRY(ensure_pinned(ctx, pin_b));
    Bump host{static_cast<char *>(ctx->pinned)};
    unsigned long long *h_sums = host.take<unsigned long long>(kSegWindow);
    int32_t *h_bid_all = host.take<int32_t>((size_t)Ntot);
    int32_t *h_states = host.take<int32_t>(4 * (size_t)Ntot);
    Job *h_jobs = host.take<Job>((size_t)Ntot);

    // segmentation needs only [luma][seg]; the job area is sized afterwards,
    // so reserve luma + seg first and grow (preserving nothing else) later.
    SCPL_TRY(ensure_ws(ctx, luma_b + seg_b));
    std::vector<const uint8_t *> lumas(n_clips);
    {
        Bump dev{static_cast<char *>(ctx->ws)};
        int64_t off = 0;
        for (int c = 0; c < n_clips; ++c) {
            const scpl_params &p = clips[c].p;
            const int64_t HW = (int64_t)p.height * p.width;
            if (p.channels == 3) {
                uint8_t *y = dev.take<uint8_t>((size_t)p.n_frames * HW);
                ProfScope ps(ctx, SCPL_KERNEL_LUMA, s);
                launch_luma(clips[c].d_frames, y, (int64_t)p.n_frames * HW, s);
                SCPL_CHECK_LAUNCH();
                lumas[c] = y;
            } else {
                lumas[c] = clips[c].d_frames;
            }
        }
        void *seg_ws = dev.take<char>(seg_b);
        for (int c = 0; c < n_clips; ++c) {
            int32_t nbuf = 0;
            scpl_status st = segment_clip(ctx, &clips[c].p, lumas[c], seg_ws, h_sums, h_bid_all + off, nullptr, &nbuf, s);
            if (st != SCPL_OK) return st;
            if (clips[c].d_buffer_id)
                SCPL_TRY(hipMemcpyAsync(clips[c].d_buffer_id, h_bid_all + off, (size_t)clips[c].p.n_frames * 4,
                                        hipMemcpyHostToDevice, s));
            off += clips[c].p.n_frames;
        }
    }

    // pass 2: one job per buffer of every clip
    struct Pending {
        int clip, t0, T, bindex;
    };
    std::vector<Pending> pend;
    {
        int64_t off = 0;
        for (int c = 0; c < n_clips; ++c) {
            const auto bufs = buffers_of(h_bid_all + off, clips[c].p.n_frames);
            for (size_t b = 0; b < bufs.size(); ++b) pend.push_back({c, bufs[b].first, bufs[b].second, (int)b});
            off += clips[c].p.n_frames;
        }
    }
    const int nj = (int)pend.size();
    int Wall = 0;
    for (int c = 0; c < n_clips; ++c) Wall = std::max(Wall, clips[c].p.width);
    const int Qall = dp_columns_per_thread(Wall);  // one DP launch serves every job
    size_t job_area = 0;
    for (const Pending &q : pend) {
        const scpl_params &p = clips[q.clip].p;
        JobShape js{p.height, p.width, p.target_width, p.seams_per_iter};
        js.Q = Qall;
        job_area += job_bytes(js);
    }
    const size_t head = luma_b + seg_b;
    const size_t total = head + job_area + align_up(sizeof(Job) * (size_t)nj) + align_up(16 * (size_t)nj);
    if (total > ctx->ws_size) {
        // growing frees the old area: the luma must be recomputed after
        SCPL_TRY(hipStreamSynchronize(s));
        SCPL_TRY(ensure_ws(ctx, total));
        Bump dev{static_cast<char *>(ctx->ws)};
        for (int c = 0; c < n_clips; ++c) {
            const scpl_params &p = clips[c].p;
            const int64_t HW = (int64_t)p.height * p.width;
            if (p.channels == 3) {
                uint8_t *y = dev.take<uint8_t>((size_t)p.n_frames * HW);
                ProfScope ps(ctx, SCPL_KERNEL_LUMA, s);
                launch_luma(clips[c].d_frames, y, (int64_t)p.n_frames * HW, s);
                SCPL_CHECK_LAUNCH();
                lumas[c] = y;
            }
        }
    }
    Bump dev{static_cast<char *>(ctx->ws)};
    dev.off = head;
    char *job_ws = dev.take<char>(job_area);
    Job *d_jobs = dev.take<Job>((size_t)nj);
    int32_t *d_states = dev.take<int32_t>(4 * (size_t)nj);
    Bump jb{job_ws};
    LaunchShape ls;
    int rfirst = 0;
    std::vector<Job> jobs;
    for (int q = 0; q < nj; ++q) {
        const scpl_clip &cl = clips[pend[q].clip];
        const scpl_params &p = cl.p;
        JobShape js{p.height, p.width, p.target_width, p.seams_per_iter};
        js.Q = Qall;
        Job J = clip_job(&p, cl.d_frames, lumas[pend[q].clip], cl.d_out, cl.d_masks, pend[q].t0, pend[q].T,
                         pend[q].bindex);
        carve_job(J, js, jb, d_states + 4 * q);
        h_jobs[q] = J;
        jobs.push_back(J);
        ls.add(js);
        rfirst = std::max(rfirst, first_batch_iterations(&p));
    }
    SCPL_TRY(hipMemcpyAsync(d_jobs, h_jobs, sizeof(Job) * (size_t)nj, hipMemcpyHostToDevice, s));
    ctx->last_log.clear();
    scpl_status st = run_jobs(ctx, d_jobs, jobs.data(), d_states, h_states, nj, ls, rfirst, true, s);
    if (st != SCPL_OK) return st;
    return collect_logs(ctx, jobs, s);
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
    JobShape js{H, W, Wt, k};
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
    const size_t HW = (size_t)H * W;
    Job J{};
    Job *d_job;
    int32_t *d_state;
    char *d_two;
    // the job sees a 2-frame clip [yprev, y] and carves frame 1 with T = 1
    scpl_status st = stage_job(ctx, H, W, 1, 1, 2 * HW, J, d_job, d_state, d_two, s);
    if (st != SCPL_OK) return st;
    if (d_yprev) SCPL_TRY(hipMemcpyAsync(d_two, d_yprev, HW, hipMemcpyDeviceToDevice, s));
    SCPL_TRY(hipMemcpyAsync(d_two + HW, d_y, HW, hipMemcpyDeviceToDevice, s));
    J.frames = reinterpret_cast<uint8_t *>(d_two);
    J.luma = reinterpret_cast<uint8_t *>(d_two);
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
    ls.add(JobShape{H, W, 1, 1});
    launch_init_jobs(d_job, 1, ls.Hmax, ls.Wmax, s);
    launch_energy(d_job, 1, H, W, s);
    launch_keys_to_u(J.K0, d_e, H, W, J.Wq, s);
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
    char *unused;
    scpl_status st = stage_job(ctx, H, W, 0, 1, 0, J, d_job, d_state, unused, s);
    if (st != SCPL_OK) return st;
    LaunchShape ls;
    ls.add(JobShape{H, W, 0, 1});
    launch_init_jobs(d_job, 1, H, W, s);
    launch_u_to_keys(d_u, J.K0, H, W, J.Wq, s);
    launch_dp(d_job, 1, 0, W, ls.Q, s);
    launch_borg(d_job, 1, 0, ls.nbmax, ls.Bmax, W, s);
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
    launch_select(d_job, 1, 0, 1, ctx->lds_cap, s);
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
    ls.add(JobShape{H, W, 0, kk});
    launch_borg(d_job, 1, 0, ls.nbmax, ls.Bmax, W, s);
    launch_jump_only(d_job, 1, 0, s);
    launch_fill(d_job, 1, 0, kk, ls.nbmax, ls.Bmax, s);
    launch_i16_to_i32(J.seams, d_seams, (int64_t)kk * H, s);
    SCPL_CHECK_LAUNCH();
    SCPL_TRY(hipStreamSynchronize(s));
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
    SCPL_TRY(ensure_ws(ctx, seg_bytes(HW)));
    SCPL_TRY(ensure_pinned(ctx, align_up(kSegWindow * 8)));
    int32_t nbuf = 0;
    st = segment_clip(ctx, p, d_luma, ctx->ws, static_cast<unsigned long long *>(ctx->pinned), h_buffer_id,
                      h_s_trace, &nbuf, s);
    if (h_n_buffers) *h_n_buffers = nbuf;
    return st;
}

}  // extern "C"
