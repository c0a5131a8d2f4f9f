// Host-runtime functions shared by the C ABI entry points of libscpl.so
// (scpl_host.hip) and the request server (scpl_server.hip).  Not part of
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "../../include/scpl.h"

namespace scpl {

// Retargets nc clips on stream s: tiled luma, buffer segmentation, then the
// carving jobs (one per buffer) all at once (batched) or one buffer after
// another (plain).  h_nbuf_first (nullable) receives the first clip's
// number of buffers.  use_graph: the batched iterations are replayed from
// HIP graphs (no other host thread may then synchronise the device while
// the graphs are captured).
scpl_status run_clips(scpl_ctx *ctx, const scpl_clip *clips, int nc, bool batched, int32_t *h_nbuf_first,
                      hipStream_t s, bool use_graph = true);

// run_clips with height retargeting: the width pass of every clip, then the
// transposed height pass of the clips with a target height.
scpl_status run_clips_2d(scpl_ctx *ctx, const scpl_clip *clips, int nc, bool batched, int32_t *h_nbuf_first,
                         hipStream_t s, bool use_graph = true);

// Upper bound of the device bytes a batched retarget of one clip claims.
uint64_t clip_footprint(const scpl_params &p);

// Frees the context's device workspaces if together they exceed keep bytes.
scpl_status trim_workspace(scpl_ctx *ctx, uint64_t keep);

// A server lane's live job table (iteration-level continuous batching):
// requests join between iterations and leave when their own buffers are
// carved.  `st` runs the iterations, `side` the admissions; request memory
// comes from `pool`.
struct LiveLane;
scpl_status live_create(scpl_ctx *ctx, hipStream_t st, hipStream_t side, hipMemPool_t pool, LiveLane **out);
void live_destroy(LiveLane *L);
// Requests in the table (carving or being released).
int live_requests(const LiveLane *L);
// Whether the table has a slot for every buffer the clip could have.
bool live_fits(const LiveLane *L, const scpl_params &p);
// Luma, segmentation and first energies of the clip (synchronises `side`),
// then its jobs join the table.  A clip with a target height runs whole on
// `side` instead, and *finished is set with its *result.
scpl_status live_admit(LiveLane *L, const scpl_clip &clip, int64_t tag, bool *finished, scpl_status *result);
// Enqueues iterations over the table, reads the jobs' states back, starts
// the gathers of the requests that are carved, and appends (tag, status) of
// every request whose outputs are complete.
scpl_status live_advance(LiveLane *L, std::vector<std::pair<int64_t, scpl_status>> &done);
// After a device error: every request of the table is reported with err.
void live_abort(LiveLane *L, scpl_status err, std::vector<std::pair<int64_t, scpl_status>> &done);

}  // namespace scpl
