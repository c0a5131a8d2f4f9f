// Request server of libscpl.so: continuous batching of retarget requests on
// one device.  Requests wait in a FIFO queue; each of `lanes` worker threads
// owns a context and a stream, and whenever it is free takes every queued
// request that fits the device-memory budget (up to max_batch), admits them
// by their footprint bound and retargets them as one batch.  A request is
// done as soon as its own buffers are carved and its outputs gathered, while
// the rest of its batch carves on.  Requests that arrive while other batches
// run are admitted as lanes and memory free up, and their work overlaps on
// the device with the batches in flight.  Each result is the one
// scpl_retarget gives for the clip alone: jobs never interact.
// Declarations: include/scpl.h.
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

// A request the batched path would refuse for the whole batch: masks asked
// for a clip carved in both dimensions (the masks of the width pass and of
// the height pass do not fit one array).  Such a request fails alone.
bool refused_in_batch(const scpl_clip &c)
{
    const scpl_params &p = c.p;
    const bool height = p.target_height > 0 && p.target_height < p.height;
    return height && p.target_width < p.width && c.d_masks != nullptr;
}

// Workspace a lane keeps between batches (more is returned to the device;
// freeing device memory waits for the whole device, so it is kept rare).
constexpr uint64_t kLaneKeep = 16ull << 30;

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
    std::vector<hipStream_t> streams;
};

namespace {

void lane_main(scpl_server *S, int li)
{
    (void)hipSetDevice(S->device);
    scpl_ctx *ctx = S->ctxs[li];
    hipStream_t st = S->streams[li];
    std::vector<int64_t> batch;
    std::vector<scpl_clip> clips;
    for (;;) {
        batch.clear();
        clips.clear();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] {
                return S->stop ||
                       (!S->queue.empty() && S->in_use + S->tickets[S->queue.front()].bytes <= S->cfg.hbm_budget);
            });
            if (S->stop) return;
            const double t = now_us();
            bool refused = false;
            while (!S->queue.empty() && (int)batch.size() < S->cfg.max_batch) {
                Ticket &tk = S->tickets[S->queue.front()];
                if (refused_in_batch(tk.clip)) {  // completes with its error, outside any batch
                    tk.t_start = tk.t_done = t;
                    tk.result = SCPL_ERR_INVALID_ARG;
                    tk.done = true;
                    refused = true;
                    S->queue.pop_front();
                    continue;
                }
                if (S->in_use + tk.bytes > S->cfg.hbm_budget) break;
                S->in_use += tk.bytes;
                tk.t_start = t;
                batch.push_back(S->queue.front());
                clips.push_back(tk.clip);
                S->queue.pop_front();
            }
            if (refused) S->cv_done.notify_all();
        }
        if (batch.empty()) continue;
        // a request is done as soon as its own buffers are carved and
        // gathered; its memory counts against the budget until the batch ends
        // (the batch's workspace is one)
        std::vector<uint64_t> bytes;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (int64_t id : batch) bytes.push_back(S->tickets[id].bytes);
        }
        const scpl::ClipDone done = [&](int c) {
            {
                std::lock_guard<std::mutex> lk(S->mu);
                auto it = S->tickets.find(batch[c]);
                if (it != S->tickets.end() && !it->second.done) {
                    it->second.done = true;
                    it->second.result = SCPL_OK;
                    it->second.t_done = now_us();
                }
            }
            S->cv_done.notify_all();
        };
        // no graph capture here: the caller's threads may synchronise the
        // device at any time
        scpl_status res = scpl::run_clips_2d(ctx, clips.data(), (int)clips.size(), true, nullptr, st, false,
                                             S->cfg.whole_batch ? nullptr : &done);
        if (res == SCPL_OK && hipStreamSynchronize(st) != hipSuccess) res = SCPL_ERR_DEVICE;
        if (res == SCPL_OK) res = scpl::trim_workspace(ctx, kLaneKeep);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const double t = now_us();
            for (size_t q = 0; q < batch.size(); ++q) {
                S->in_use -= bytes[q];
                auto it = S->tickets.find(batch[q]);
                if (it == S->tickets.end() || it->second.done) continue;  // done early (and maybe released)
                it->second.done = true;
                it->second.result = res;
                it->second.t_done = t;
            }
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
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
    for (int l = 0; st == SCPL_OK && l < cfg->lanes; ++l) {
        scpl_ctx *c = nullptr;
        st = scpl_create(device, &c);
        if (st != SCPL_OK) break;
        // a lane runs its batch as one job group on its own stream: lanes
        // already overlap, and more streams than the device's hardware
        // queues would make streams share queues
        st = scpl_batch_streams(c, 1);
        if (st != SCPL_OK) break;
        S->ctxs.push_back(c);
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            st = SCPL_ERR_DEVICE;
            break;
        }
        S->streams.push_back(s);
    }
    if (st != SCPL_OK) {
        for (scpl_ctx *c : S->ctxs) scpl_destroy(c);
        for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
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
        // requests already taken by a lane finish; queued ones are dropped
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
    for (scpl_ctx *c : S->ctxs) scpl_destroy(c);
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    delete S;
}

}  // extern "C"
