// Host-runtime functions shared by the C ABI entry points of libscpl.so
// (scpl_host.hip) and the request server (scpl_server.hip).  Not part of
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

#include "../../include/scpl.h"

namespace scpl {

// Called on the calling thread, while a batched retarget runs, with the
// index of a clip whose outputs (frames, masks) are complete on the device:
// its buffers are carved and gathered, and no later work of the call reads
// or writes its memory.
using ClipDone = std::function<void(int)>;

// Retargets nc clips on stream s: tiled luma, buffer segmentation, then the
// carving jobs (one per buffer) all at once (batched) or one buffer after
// another (plain).  h_nbuf_first (nullable) receives the first clip's
// number of buffers.  use_graph: the batched iterations are replayed from
// HIP graphs (no other host thread may then synchronise the device while
// the graphs are captured).
// on_done (nullable, batched job groups only): clips are gathered as soon
// as their own buffers are carved, and reported as their gathers complete
// (clips still gathering when the call returns are not reported).
scpl_status run_clips(scpl_ctx *ctx, const scpl_clip *clips, int nc, bool batched, int32_t *h_nbuf_first,
                      hipStream_t s, bool use_graph = true, const ClipDone *on_done = nullptr);

// run_clips with height retargeting: the width pass of every clip, then the
// transposed height pass of the clips with a target height.
// (on_done: clips with a target width only; a clip with a height pass is
// complete when the call's work is.)
scpl_status run_clips_2d(scpl_ctx *ctx, const scpl_clip *clips, int nc, bool batched, int32_t *h_nbuf_first,
                         hipStream_t s, bool use_graph = true, const ClipDone *on_done = nullptr);

// Upper bound of the device bytes a batched retarget of one clip claims.
uint64_t clip_footprint(const scpl_params &p);

// Frees the context's device workspaces if together they exceed keep bytes.
scpl_status trim_workspace(scpl_ctx *ctx, uint64_t keep);

}  // namespace scpl
