// Request server of libscpl.so: continuous batching of retarget requests on
// one device.  Requests wait in a FIFO queue.  Each of `lanes` worker
// threads owns a context, a live job table and two streams: between
// iterations of its table it admits queued requests that fit the
// device-memory budget (their luma, buffer segmentation and first energies
// run on the lane's side stream while the table's iterations go on), and a
// request leaves the table as soon as its own buffers are carved, so a small
// request never waits for a large one that it shares a table with.  Each
// result is the one scpl_retarget gives for the clip alone: jobs never
// interact.  Declarations: include/scpl.h.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/scpl.h"
#include "scpl_runtime.h"

namespace {

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

struct Ticket {
    scpl_clip clip;
    uint64_t bytes = 0;
    int waiters = 0;  // threads inside scpl_server_wait on this ticket
    bool done = false;
    scpl_status result = SCPL_OK;
    double t_submit = 0, t_start = 0, t_done = 0;
};

}  // namespace

struct scpl_server {
    int device = 0;
    scpl_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Ticket> tickets;
    uint64_t in_use = 0;
    int64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> lanes;
    std::vector<scpl_ctx *> ctxs;
    std::vector<hipStream_t> streams;  // two per lane: iterations, admissions
    std::vector<scpl::LiveLane *> live;
    hipMemPool_t pool = nullptr;       // request memory of every lane
};

namespace {

// Marks request `id` done with `res` (caller holds S->mu).
void finish_locked(scpl_server *S, int64_t id, scpl_status res, double t)
{
    Ticket &tk = S->tickets[id];
    tk.done = true;
    tk.result = res;
    tk.t_done = t;
    S->in_use -= tk.bytes;
}

void lane_main(scpl_server *S, int li)
{
    (void)hipSetDevice(S->device);
    scpl::LiveLane *L = S->live[li];
    std::vector<std::pair<int64_t, scpl_clip>> take;
    std::vector<std::pair<int64_t, scpl_status>> done;
    for (;;) {
        take.clear();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            auto admissible = [&] {
                if (S->stop || S->queue.empty()) return false;
                if (scpl::live_requests(L) + (int)take.size() >= S->cfg.max_batch) return false;
                const Ticket &tk = S->tickets[S->queue.front()];
                return S->in_use + tk.bytes <= S->cfg.hbm_budget && scpl::live_fits(L, tk.clip.p);
            };
            if (scpl::live_requests(L) == 0) {
                S->cv_work.wait(lk, [&] { return S->stop || admissible(); });
                if (S->stop) return;  // requests already taken have finished
            }
            const double t = now_us();
            while (admissible()) {
                const int64_t id = S->queue.front();
                Ticket &tk = S->tickets[id];
                S->in_use += tk.bytes;
                tk.t_start = t;
                take.emplace_back(id, tk.clip);
                S->queue.pop_front();
            }
        }
        done.clear();
        for (const auto &q : take) {
            bool now = false;
            scpl_status res = SCPL_OK;
            const scpl_status st = scpl::live_admit(L, q.second, q.first, &now, &res);
            if (st != SCPL_OK) {  // this request fails alone
                now = true;
                res = st;
            }
            if (now) done.emplace_back(q.first, res);
        }
        if (scpl::live_requests(L) > 0) {
            const scpl_status st = scpl::live_advance(L, done);
            if (st != SCPL_OK) scpl::live_abort(L, st, done);
        }
        if (!done.empty()) {
            {
                std::lock_guard<std::mutex> lk(S->mu);
                const double t = now_us();
                for (const auto &d : done) finish_locked(S, d.first, d.second, t);
            }
            S->cv_done.notify_all();
            S->cv_work.notify_all();
        }
    }
}

}  // namespace

extern "C" {

scpl_status scpl_server_create(int32_t device, const scpl_server_config *cfg, scpl_server **out)
{
    if (!out || !cfg || cfg->lanes < 1 || cfg->lanes > SCPL_MAX_LANES || cfg->max_batch < 1) return SCPL_ERR_INVALID_ARG;
    *out = nullptr;
    scpl_server *S = new (std::nothrow) scpl_server();
    if (!S) return SCPL_ERR_OUT_OF_MEMORY;
    S->device = device;
    S->cfg = *cfg;
    scpl_status st = SCPL_OK;
    if (S->cfg.hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipSetDevice(device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) st = SCPL_ERR_DEVICE;
        S->cfg.hbm_budget = fr / 2;
    }
    if (st == SCPL_OK) {
        // request memory: a pool of its own that keeps freed memory for
        // later requests instead of returning it to the device
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = device;
        uint64_t keep = UINT64_MAX;
        if (hipSetDevice(device) != hipSuccess || hipMemPoolCreate(&S->pool, &props) != hipSuccess ||
            hipMemPoolSetAttribute(S->pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess)
            st = SCPL_ERR_DEVICE;
    }
    for (int l = 0; st == SCPL_OK && l < cfg->lanes; ++l) {
        scpl_ctx *c = nullptr;
        st = scpl_create(device, &c);
        if (st != SCPL_OK) break;
        // horizontal-seam requests run as one job group on the lane's side
        // stream
        st = scpl_batch_streams(c, 1);
        if (st != SCPL_OK) break;
        S->ctxs.push_back(c);
        hipStream_t s2[2] = {nullptr, nullptr};
        for (hipStream_t &x : s2)
            if (st == SCPL_OK && hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) st = SCPL_ERR_DEVICE;
        for (hipStream_t x : s2)
            if (x) S->streams.push_back(x);
        if (st != SCPL_OK) break;
        scpl::LiveLane *L = nullptr;
        st = scpl::live_create(c, s2[0], s2[1], S->pool, &L);
        if (st != SCPL_OK) break;
        S->live.push_back(L);
    }
    if (st != SCPL_OK) {
        for (scpl::LiveLane *L : S->live) scpl::live_destroy(L);
        for (scpl_ctx *c : S->ctxs) scpl_destroy(c);
        for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
        if (S->pool) (void)hipMemPoolDestroy(S->pool);
        delete S;
        return st;
    }
    for (int l = 0; l < cfg->lanes; ++l) S->lanes.emplace_back(lane_main, S, l);
    *out = S;
    return SCPL_OK;
}

scpl_status scpl_server_submit(scpl_server *S, const scpl_clip *clip, int64_t *h_ticket)
{
    if (!S || !clip || !h_ticket || !clip->d_frames || !clip->d_out) return SCPL_ERR_INVALID_ARG;
    uint64_t ws = 0;
    scpl_status st = scpl_workspace_size(&clip->p, &ws);  // validates the parameters
    if (st != SCPL_OK) return st;
    const uint64_t bytes = scpl::clip_footprint(clip->p);
    std::lock_guard<std::mutex> lk(S->mu);
    if (bytes > S->cfg.hbm_budget) return SCPL_ERR_CAPACITY;
    const int64_t id = S->next_id++;
    Ticket &tk = S->tickets[id];
    tk.clip = *clip;
    tk.bytes = bytes;
    tk.t_submit = now_us();
    S->queue.push_back(id);
    *h_ticket = id;
    S->cv_work.notify_one();
    return SCPL_OK;
}

scpl_status scpl_server_poll(scpl_server *S, int64_t ticket, int32_t *h_done, scpl_status *h_result)
{
    if (!S || !h_done) return SCPL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return SCPL_ERR_INVALID_ARG;
    *h_done = it->second.done ? 1 : 0;
    if (h_result) *h_result = it->second.done ? it->second.result : SCPL_ERR_NOT_READY;
    return SCPL_OK;
}

scpl_status scpl_server_wait(scpl_server *S, int64_t ticket, scpl_status *h_result)
{
    if (!S) return SCPL_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return SCPL_ERR_INVALID_ARG;
    // a submit may rehash the map while this thread waits: iterators then
    // go stale, element addresses do not; the waiter count keeps
    // scpl_server_release from erasing the ticket meanwhile
    Ticket *tk = &it->second;
    ++tk->waiters;
    S->cv_done.wait(lk, [&] { return tk->done; });
    --tk->waiters;
    if (h_result) *h_result = tk->result;
    return SCPL_OK;
}

scpl_status scpl_server_ticket_times(scpl_server *S, int64_t ticket, double *h_queue_ms, double *h_total_ms)
{
    if (!S) return SCPL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return SCPL_ERR_INVALID_ARG;
    if (!it->second.done) return SCPL_ERR_NOT_READY;
    if (h_queue_ms) *h_queue_ms = (it->second.t_start - it->second.t_submit) * 1e-3;
    if (h_total_ms) *h_total_ms = (it->second.t_done - it->second.t_submit) * 1e-3;
    return SCPL_OK;
}

scpl_status scpl_server_release(scpl_server *S, int64_t ticket)
{
    if (!S) return SCPL_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return SCPL_ERR_INVALID_ARG;
    if (!it->second.done || it->second.waiters > 0) return SCPL_ERR_NOT_READY;
    S->tickets.erase(it);
    return SCPL_OK;
}

scpl_status scpl_server_footprint(const scpl_params *p, uint64_t *h_bytes)
{
    if (!h_bytes) return SCPL_ERR_INVALID_ARG;
    uint64_t ws = 0;
    const scpl_status st = scpl_workspace_size(p, &ws);  // validates p
    if (st != SCPL_OK) return st;
    *h_bytes = scpl::clip_footprint(*p);
    return SCPL_OK;
}

void scpl_server_destroy(scpl_server *S)
{
    if (!S) return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        // requests already in a lane's table finish; queued ones are dropped
        S->stop = true;
        for (int64_t id : S->queue) {
            Ticket &tk = S->tickets[id];
            tk.done = true;
            tk.result = SCPL_ERR_NOT_READY;
        }
        S->queue.clear();
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
    for (std::thread &t : S->lanes) t.join();
    for (scpl::LiveLane *L : S->live) scpl::live_destroy(L);
    for (scpl_ctx *c : S->ctxs) scpl_destroy(c);
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    if (S->pool) (void)hipMemPoolDestroy(S->pool);
    delete S;
}

}  // extern "C"
