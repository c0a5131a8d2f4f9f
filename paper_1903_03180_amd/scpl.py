"""Python binding of libscpl.so (C ABI in include/scpl.h).

Argument marshalling only: every step of the retarget runs in the library's
HIP kernels.  PyTorch supplies device memory and streams; tensors are passed
by data pointer.  The module raises at import if libscpl.so is missing:
there is no fallback implementation.

The `scpl_*` functions mirror the C entry points one to one (raw pointers
and sizes).  `Context` wraps them for torch tensors.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscpl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libscpl.so not built ({LIB_PATH}); run paper_1903_03180_amd/build.py")

_lib = C.CDLL(LIB_PATH)

SCPL_OK = 0
SCPL_ERR_INVALID_ARG = 1
SCPL_ERR_OUT_OF_MEMORY = 2
SCPL_ERR_DEVICE = 3
SCPL_ERR_CAPACITY = 4
SCPL_ERR_NOT_READY = 5
SCPL_ERR_INTERNAL = 6
SCPL_ENERGY_GRADIENT = 0
SCPL_ENERGY_MOTION = 1
SCPL_NOALLOC_SCRATCH_BYTES = 64 << 20
SCPL_BATCH_GROUPS = 0
SCPL_BATCH_PERSISTENT = 1
SCPL_BATCH_PERSISTENT_AGENT = 2

EXPORTS = [
    "scpl_create", "scpl_destroy", "scpl_status_str", "scpl_workspace_size", "scpl_retarget",
    "scpl_retarget_noalloc", "scpl_kernel_variants", "scpl_autotune_batch",
    "scpl_retarget_batch", "scpl_last_log", "scpl_luma", "scpl_energy", "scpl_dp", "scpl_select",
    "scpl_backtrack", "scpl_segment", "scpl_profile_enable", "scpl_profile_read", "scpl_profile_kinds", "scpl_dp_geometry",
    "scpl_autotune_dp", "scpl_dp_chunking", "scpl_dp_chosen", "scpl_batch_streams", "scpl_batch_mode", "scpl_device_xcds", "scpl_persist_stats", "scpl_persist_workgroups", "scpl_server_create",
    "scpl_server_submit", "scpl_server_poll",
    "scpl_server_wait", "scpl_server_ticket_times", "scpl_server_release", "scpl_server_destroy",
    "scpl_server_footprint", "scpl_asde", "scpl_compact",
]

DP_GEOMETRIES = [(2, 8, 8), (2, 8, 16), (4, 8, 8), (4, 8, 16), (4, 16, 8), (4, 16, 16), (8, 16, 4), (8, 16, 8),
                 (8, 16, 16), (8, 32, 4), (8, 32, 8), (16, 32, 2), (16, 32, 4), (16, 32, 8), (16, 64, 2), (16, 64, 4),
                 (32, 0, 2)]
# column-split DP (Q, HB, PF, R, P): one launch per R rows, a workgroup per P columns
DP_CHUNKED = [(4, 16, 8, 256, 384), (4, 16, 8, 384, 256), (4, 16, 8, 320, 384), (4, 16, 8, 192, 512),
              (4, 16, 8, 128, 640), (4, 16, 8, 512, 768), (4, 16, 8, 128, 768), (4, 16, 8, 128, 1024),
              (4, 16, 8, 192, 896), (4, 16, 8, 256, 768), (4, 16, 8, 256, 1024), (4, 16, 8, 320, 640),
              (4, 16, 8, 384, 128), (4, 16, 8, 352, 192), (4, 16, 8, 288, 320),
              (2, 8, 16, 128, 640), (2, 8, 16, 64, 768), (4, 8, 8, 128, 704),
              (2, 8, 16, 192, 64), (2, 8, 16, 160, 128), (2, 8, 16, 128, 192), (2, 8, 16, 208, 32),
              (2, 8, 16, 216, 16), (4, 16, 16, 256, 384), (4, 16, 16, 320, 384),
              (4, 16, 16, 192, 512)]

KERNELS = ["luma", "segment", "energy", "dp", "borg", "select", "fill", "update", "gather", "init", "refresh",
           "persist"]


class scpl_params(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "n_frames", "height", "width", "channels", "target_width", "seams_per_iter", "energy_mode",
        "use_buffer", "alpha_num", "alpha_den", "max_buffer", "target_height", "memo_period")]


class scpl_clip(C.Structure):
    _fields_ = [("p", scpl_params), ("d_frames", C.c_void_p), ("d_out", C.c_void_p), ("d_masks", C.c_void_p),
                ("d_buffer_id", C.c_void_p)]


class scpl_server_config(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("max_batch", C.c_int32), ("hbm_budget", C.c_uint64),
                ("whole_batch", C.c_int32)]


_P, _I32, _I64 = C.c_void_p, C.c_int32, C.c_int64
_sig = {
    "scpl_create": ([_I32, C.POINTER(C.c_void_p)], C.c_int),
    "scpl_destroy": ([_P], None),
    "scpl_status_str": ([C.c_int], C.c_char_p),
    "scpl_workspace_size": ([C.POINTER(scpl_params), C.POINTER(C.c_uint64)], C.c_int),
    "scpl_retarget": ([_P, C.POINTER(scpl_params), _P, _P, _P, _P, C.POINTER(_I32), _P, C.c_uint64, _P], C.c_int),
    "scpl_retarget_noalloc": ([_P, C.POINTER(scpl_params), _P, _P, _P, _P, C.POINTER(_I32), _P], C.c_int),
    "scpl_retarget_batch": ([_P, C.POINTER(scpl_clip), _I32, _P], C.c_int),
    "scpl_kernel_variants": ([_P, _I32, _I32, _I32, _I32, _I32], C.c_int),
    "scpl_autotune_batch": ([_P, C.POINTER(scpl_clip), _I32, _I32, C.POINTER(_I32), C.POINTER(C.c_double), _P],
                            C.c_int),
    "scpl_last_log": ([_P, _P, _I64, C.POINTER(_I64)], C.c_int),
    "scpl_luma": ([_P, _P, _I64, _P, _P], C.c_int),
    "scpl_energy": ([_P, _I32, _I32, _I32, _P, _P, _P, _P], C.c_int),
    "scpl_dp": ([_P, _I32, _I32, _P, _P, _P, _P, _P], C.c_int),
    "scpl_select": ([_P, _I32, _P, _P, _I32, _I32, _P, C.POINTER(_I32), C.POINTER(_I32), _P], C.c_int),
    "scpl_backtrack": ([_P, _I32, _I32, _P, _P, _I32, _P, _P], C.c_int),
    "scpl_segment": ([_P, C.POINTER(scpl_params), _P, _P, _P, C.POINTER(_I32), _P], C.c_int),
    "scpl_profile_enable": ([_P, _I32], C.c_int),
    "scpl_profile_read": ([_P, _I32, C.POINTER(C.c_double), C.POINTER(_I64)], C.c_int),
    "scpl_profile_kinds": ([_P, C.c_uint32], C.c_int),
    "scpl_dp_geometry": ([_P, _I32, _I32, _I32, _I32], C.c_int),
    "scpl_dp_chunking": ([_P, _I32, _I32], C.c_int),
    "scpl_dp_chosen": ([_P, _I32, C.POINTER(_I32)], C.c_int),
    "scpl_batch_streams": ([_P, _I32], C.c_int),
    "scpl_batch_mode": ([_P, _I32], C.c_int),
    "scpl_persist_stats": ([_P, _P, _P], C.c_int),
    "scpl_device_xcds": ([_P, _P], C.c_int),
    "scpl_persist_workgroups": ([_P, _I32], C.c_int),
    "scpl_server_create": ([_I32, C.POINTER(scpl_server_config), C.POINTER(C.c_void_p)], C.c_int),
    "scpl_server_submit": ([_P, C.POINTER(scpl_clip), C.POINTER(_I64)], C.c_int),
    "scpl_server_poll": ([_P, _I64, C.POINTER(_I32), C.POINTER(C.c_int)], C.c_int),
    "scpl_server_wait": ([_P, _I64, C.POINTER(C.c_int)], C.c_int),
    "scpl_server_ticket_times": ([_P, _I64, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "scpl_server_release": ([_P, _I64], C.c_int),
    "scpl_server_destroy": ([_P], None),
    "scpl_server_footprint": ([C.POINTER(scpl_params), C.POINTER(C.c_uint64)], C.c_int),
    "scpl_asde": ([_P, _I32, _I32, _I32, _I32, _P, _P, _I32, _I32, C.POINTER(_I64), C.POINTER(_I32), _P], C.c_int),
    "scpl_compact": ([_P, _I32, _I32, _I32, _P, _P, _I32, _P, _P], C.c_int),
    "scpl_autotune_dp": ([_P, _I32, _I32, _I32, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32),
                          C.POINTER(_I32), C.POINTER(C.c_double)], C.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()[_name] = _f


class ScplError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {scpl_status_str(status).decode()} ({status})")


def _check(st: int, what: str) -> None:
    if st != SCPL_OK:
        raise ScplError(st, what)


@dataclass
class Params:
    n_frames: int
    height: int
    width: int
    channels: int
    target_width: int
    seams_per_iter: int
    energy_mode: int = SCPL_ENERGY_MOTION
    use_buffer: int = 1
    alpha_num: int = 1
    alpha_den: int = 5
    max_buffer: int = 0
    target_height: int = 0
    memo_period: int = 0

    def c(self) -> scpl_params:
        return scpl_params(self.n_frames, self.height, self.width, self.channels, self.target_width,
                           self.seams_per_iter, self.energy_mode, self.use_buffer, self.alpha_num,
                           self.alpha_den, self.max_buffer, self.target_height, self.memo_period)


def _ptr(t) -> int | None:
    if t is None:
        return None
    assert t.is_contiguous(), "tensors passed to libscpl must be contiguous"
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def workspace_size(params: Params) -> int:
    """Device bytes scpl_retarget needs for a clip with these parameters."""
    b = C.c_uint64(0)
    cp = params.c()
    _check(scpl_workspace_size(C.byref(cp), C.byref(b)), "scpl_workspace_size")
    return int(b.value)


def params_for(frames, target_width: int, seams_per_iter: int, **kw) -> Params:
    if frames.dim() == 3:
        N, H, W = frames.shape
        Cc = 1
    elif frames.dim() == 4:
        N, H, W, Cc = frames.shape
    else:
        raise ValueError("frames must be N x H x W or N x H x W x 3 uint8")
    return Params(N, H, W, Cc, target_width, seams_per_iter, **kw)


class Context:
    """A libscpl context on one HIP device (one host thread at a time)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(scpl_create(device, C.byref(h)), "scpl_create")
        self.h = h
        self.device = device

    def close(self) -> None:
        if self.h:
            scpl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- whole path
    def retarget(self, frames, target_width: int, seams_per_iter: int, want_masks: bool = True, stream=None,
                 workspace=None, **kw):
        """frames: uint8 cuda tensor N x H x W (luma) or N x H x W x 3 (RGB).
        workspace: optional uint8 cuda tensor of at least workspace_size()
        bytes that the call uses instead of the context's own workspace.
        Returns dict(out, masks, buffer_id, n_buffers)."""
        import torch
        p = params_for(frames, target_width, seams_per_iter, **kw)
        Ht = p.target_height or p.height
        shp = (p.n_frames, Ht, p.target_width) + ((p.channels,) if frames.dim() == 4 else ())
        out = torch.empty(shp, dtype=torch.uint8, device=frames.device)
        both = Ht < p.height and p.target_width < p.width
        masks = torch.empty((p.n_frames, p.height, p.width), dtype=torch.int16, device=frames.device) \
            if want_masks and not both else None
        bid = torch.empty(p.n_frames, dtype=torch.int32, device=frames.device)
        nb = C.c_int32(0)
        cp = p.c()
        wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
        _check(scpl_retarget(self.h, C.byref(cp), _ptr(frames), _ptr(out), _ptr(masks), _ptr(bid), C.byref(nb),
                             _ptr(workspace), wsb, _stream(stream)), "scpl_retarget")
        return dict(out=out, masks=masks, buffer_id=bid, n_buffers=int(nb.value))

    def retarget_noalloc(self, frames, target_width: int, seams_per_iter: int, out=None, masks=None,
                         buffer_id=None, want_masks: bool = True, stream=None, **kw):
        """scpl_retarget_noalloc: as retarget(), with the library's fixed
        device workspace (SCPL_NOALLOC_SCRATCH_BYTES) and no allocation in
        the call.  out / masks / buffer_id: the caller's output tensors
        (those left None are allocated here, before the call).
        Returns dict(out, masks, buffer_id, n_buffers)."""
        import torch
        p = params_for(frames, target_width, seams_per_iter, **kw)
        Ht = p.target_height or p.height
        shp = (p.n_frames, Ht, p.target_width) + ((p.channels,) if frames.dim() == 4 else ())
        if out is None:
            out = torch.empty(shp, dtype=torch.uint8, device=frames.device)
        both = Ht < p.height and p.target_width < p.width
        if masks is None and want_masks and not both:
            masks = torch.empty((p.n_frames, p.height, p.width), dtype=torch.int16, device=frames.device)
        if buffer_id is None:
            buffer_id = torch.empty(p.n_frames, dtype=torch.int32, device=frames.device)
        nb = C.c_int32(0)
        cp = p.c()
        _check(scpl_retarget_noalloc(self.h, C.byref(cp), _ptr(frames), _ptr(out), _ptr(masks), _ptr(buffer_id),
                                     C.byref(nb), _stream(stream)), "scpl_retarget_noalloc")
        return dict(out=out, masks=masks, buffer_id=buffer_id, n_buffers=int(nb.value))

    def _clip_array(self, clips):
        import torch
        arr = (scpl_clip * len(clips))()
        for i, c in enumerate(clips):
            fr = c["frames"]
            kw = {k: c[k] for k in ("energy_mode", "use_buffer", "alpha_num", "alpha_den", "max_buffer",
                                    "target_height", "memo_period") if k in c}
            p = params_for(fr, c["target_width"], c["seams_per_iter"], **kw)
            shp = (p.n_frames, p.target_height or p.height, p.target_width) + ((p.channels,) if fr.dim() == 4 else ())
            if c.get("out") is None:
                c["out"] = torch.empty(shp, dtype=torch.uint8, device=fr.device)
            if c.get("masks") is None and c.get("want_masks", False):
                c["masks"] = torch.empty((p.n_frames, p.height, p.width), dtype=torch.int16, device=fr.device)
            if c.get("buffer_id") is None:
                c["buffer_id"] = torch.empty(p.n_frames, dtype=torch.int32, device=fr.device)
            arr[i] = scpl_clip(p.c(), _ptr(fr), _ptr(c["out"]), _ptr(c.get("masks")), _ptr(c["buffer_id"]))
        return arr

    def kernel_variants(self, update: int = 0, refresh: int = 0, borg: int = 0, gather: int = 4,
                        fuse: int = 0) -> None:
        """Compaction kernel variant (0-6), refresh kernel variant (0-2),
        band-origin kernel variant (0-2), gather variant (0-4), fill and
        compaction fused per band (0: no; 1, 2: 8 or 16 wavefronts); no
        arguments: the context's defaults."""
        _check(scpl_kernel_variants(self.h, update, refresh, borg, gather, fuse), "scpl_kernel_variants")

    def autotune_batch(self, clips, reps: int = 2, stream=None) -> dict:
        """scpl_autotune_batch on these clips (dicts as for retarget_batch,
        whose outputs it writes); returns the chosen configuration and the
        best time of a whole batched retarget."""
        arr = self._clip_array(clips)
        ch = (C.c_int32 * 15)()
        ms = C.c_double(0)
        _check(scpl_autotune_batch(self.h, arr, len(clips), reps, ch, C.byref(ms), _stream(stream)),
               "scpl_autotune_batch")
        v = [int(x) for x in ch]
        return {"streams": v[0], "dp_geometry": dict(zip(("cols_per_lane", "halo_rows", "prefetch_rows", "exclusive_cu",
                                                          "chunk_rows", "chunk_cols"), v[1:7])) if v[9] else None,
                "update_variant": v[7], "refresh_variant": v[8], "borg_variant": v[10], "gather_variant": v[11],
                "fuse_variant": v[12], "batch_mode": v[13], "persist_workgroups": v[14], "ms": ms.value}

    def retarget_batch(self, clips, stream=None):
        """clips: list of dicts with keys frames (cuda uint8 tensor),
        target_width, seams_per_iter and optional Params fields, and
        optionally out / masks / buffer_id tensors (allocated when absent,
        masks only when want_masks is true).  Returns the list of dicts with
        the outputs filled in."""
        arr = self._clip_array(clips)
        _check(scpl_retarget_batch(self.h, arr, len(clips), _stream(stream)), "scpl_retarget_batch")
        return clips

    def last_log(self):
        """(buffer, W_r, P_eff, k_iter) per iteration of the last call."""
        import numpy as np
        n = C.c_int64(0)
        _check(scpl_last_log(self.h, None, 0, C.byref(n)), "scpl_last_log")
        a = np.zeros((max(n.value, 1), 4), dtype=np.int32)
        _check(scpl_last_log(self.h, a.ctypes.data, n.value, C.byref(n)), "scpl_last_log")
        return a[:n.value]

    def batch_streams(self, n: int) -> None:
        """Number of independently advancing job groups (streams) of the
        batched path."""
        _check(scpl_batch_streams(self.h, n), "scpl_batch_streams")

    def batch_mode(self, mode: int) -> None:
        """How the batched path runs its iterations: SCPL_BATCH_GROUPS (job
        groups replaying graphs), SCPL_BATCH_PERSISTENT (one persistent
        launch whose workgroups take work items from rings on the device, one
        ring per XCD) or SCPL_BATCH_PERSISTENT_AGENT (the same with one ring
        and agent-scope ordering)."""
        _check(scpl_batch_mode(self.h, mode), "scpl_batch_mode")

    def persist_workgroups(self, per_cu: int = 0) -> None:
        """Workgroups per compute unit of the persistent launch (0: as many
        as fit at once)."""
        _check(scpl_persist_workgroups(self.h, per_cu), "scpl_persist_workgroups")

    def device_xcds(self) -> int:
        """XCDs whose workgroups each serve a ring of their own in the
        persistent launch (0: one ring, agent-scope ordering)."""
        n = C.c_int32(0)
        _check(scpl_device_xcds(self.h, C.byref(n)), "scpl_device_xcds")
        return n.value

    def persist_stats(self) -> dict:
        """Workgroup time of the last persistent launch made while kernels
        were timed: {part: (ms summed over workgroups, items)} for dp, borg,
        select, band (seam trace and compaction), refresh, wait (for an item)
        and done (counting items and queueing the next stages)."""
        ms = (C.c_double * 7)()
        n = (C.c_int64 * 7)()
        _check(scpl_persist_stats(self.h, ms, n), "scpl_persist_stats")
        keys = ["dp", "borg", "select", "band", "refresh", "wait", "done"]
        return {k: (ms[q], n[q]) for q, k in enumerate(keys)}

    # ---------------------------------------------------------- timing
    def profile(self, on: bool = True, kinds=None) -> None:
        """Start (and reset) or stop per-kernel event timing; kinds: the
        kernel names of KERNELS to bracket (None: all)."""
        mask = (1 << len(KERNELS)) - 1 if kinds is None else sum(1 << KERNELS.index(k) for k in kinds)
        _check(scpl_profile_kinds(self.h, mask), "scpl_profile_kinds")
        _check(scpl_profile_enable(self.h, 1 if on else 0), "scpl_profile_enable")

    def profile_read(self) -> dict:
        """{kernel: (total_ms, launches)} since profiling was enabled."""
        out = {}
        for i, name in enumerate(KERNELS):
            ms, n = C.c_double(0), C.c_int64(0)
            _check(scpl_profile_read(self.h, i, C.byref(ms), C.byref(n)), "scpl_profile_read")
            out[name] = (ms.value, n.value)
        return out

    # ---------------------------------------------------------- DP geometry
    def dp_geometry(self, Q: int = 0, HB: int = 0, PF: int = 0, EX: int = 0) -> None:
        """Force the DP geometry (Q columns per lane, HB halo, PF prefetch
        rows, PF = 0: default depth; EX = 1: one DP workgroup per compute
        unit and nothing beside it); Q = 0: automatic."""
        _check(scpl_dp_geometry(self.h, Q, HB, PF, EX), "scpl_dp_geometry")

    def dp_chunking(self, R: int = 0, P: int = 0) -> None:
        """Run the forced geometry's DP column-split: one launch per R rows,
        a workgroup per P owned columns (R = 0: one launch, one workgroup
        per buffer)."""
        _check(scpl_dp_chunking(self.h, R, P), "scpl_dp_chunking")

    def dp_chosen(self, W: int) -> dict:
        """The DP geometry used for launches whose widest job has width W."""
        g = (C.c_int32 * 6)()
        _check(scpl_dp_chosen(self.h, W, g), "scpl_dp_chosen")
        return dict(zip(("cols_per_lane", "halo_rows", "prefetch_rows", "exclusive_cu", "chunk_rows",
                         "chunk_cols"), [int(x) for x in g]))

    def autotune_dp(self, H: int, W: int, n_jobs: int = 1):
        """Time every DP geometry on launches of n_jobs H x W jobs; keep the
        fastest.  Returns (Q, HB, PF, EX, microseconds per launch)."""
        q, hb, pf, ex, us = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_double(0)
        _check(scpl_autotune_dp(self.h, H, W, n_jobs, C.byref(q), C.byref(hb), C.byref(pf), C.byref(ex),
                                C.byref(us)), "scpl_autotune_dp")
        return int(q.value), int(hb.value), int(pf.value), int(ex.value), float(us.value)

    # ---------------------------------------------------------- stages
    def luma(self, rgb, stream=None):
        import torch
        y = torch.empty(rgb.shape[:-1], dtype=torch.uint8, device=rgb.device)
        _check(scpl_luma(self.h, _ptr(rgb), y.numel(), _ptr(y), _stream(stream)), "scpl_luma")
        return y

    def energy(self, y, yprev=None, mode: int = SCPL_ENERGY_GRADIENT, stream=None):
        import torch
        H, W = y.shape
        e = torch.empty((H, W), dtype=torch.int32, device=y.device)
        _check(scpl_energy(self.h, H, W, mode, _ptr(y), _ptr(yprev), _ptr(e), _stream(stream)), "scpl_energy")
        return e

    def dp(self, u, stream=None):
        import torch
        H, W = u.shape
        ce = torch.empty(W, dtype=torch.int32, device=u.device)
        lab = torch.empty(W, dtype=torch.int32, device=u.device)
        d = torch.empty((H, W), dtype=torch.int8, device=u.device)
        _check(scpl_dp(self.h, H, W, _ptr(u), _ptr(ce), _ptr(lab), _ptr(d), _stream(stream)), "scpl_dp")
        return ce, lab, d

    def select(self, ce_last, label_last, k: int, limit: int | None = None, stream=None):
        import torch
        W = ce_last.shape[0]
        if limit is None:
            limit = W
        ch = torch.zeros(max(min(k, W), 1), dtype=torch.int32, device=ce_last.device)
        kk, pe = C.c_int32(0), C.c_int32(0)
        _check(scpl_select(self.h, W, _ptr(ce_last), _ptr(label_last), k, limit, _ptr(ch), C.byref(kk),
                           C.byref(pe), _stream(stream)), "scpl_select")
        return ch[:kk.value], int(pe.value)

    def backtrack(self, d, children, stream=None):
        import torch
        H, W = d.shape
        kk = children.shape[0]
        seams = torch.zeros((max(kk, 1), H), dtype=torch.int32, device=d.device)
        _check(scpl_backtrack(self.h, H, W, _ptr(d), _ptr(children), kk, _ptr(seams), _stream(stream)),
               "scpl_backtrack")
        return seams[:kk]

    def asde(self, luma, prev=None, energy_mode=SCPL_ENERGY_MOTION, alpha_num=1, alpha_den=5, stream=None):
        """(S, reject) of the candidate buffer luma (n x H x W)."""
        n, H, W = luma.shape
        S, rj = C.c_int64(0), C.c_int32(0)
        _check(scpl_asde(self.h, n, H, W, energy_mode, _ptr(luma), _ptr(prev), alpha_num, alpha_den, C.byref(S),
                         C.byref(rj), _stream(stream)), "scpl_asde")
        return int(S.value), bool(rj.value)

    def compact(self, frame, seams, stream=None):
        """frame H x W (x 3) uint8 minus the seams (kk x H int32 columns)."""
        import torch
        H, W = frame.shape[:2]
        Cc = frame.shape[2] if frame.dim() == 3 else 1
        kk = seams.shape[0]
        out = torch.empty((H, W - kk) + tuple(frame.shape[2:]), dtype=torch.uint8, device=frame.device)
        _check(scpl_compact(self.h, H, W, Cc, _ptr(frame), _ptr(seams) if kk else None, kk, _ptr(out),
                            _stream(stream)), "scpl_compact")
        return out

    def segment(self, luma, energy_mode=SCPL_ENERGY_MOTION, use_buffer=1, alpha_num=1, alpha_den=5, max_buffer=0,
                stream=None):
        import numpy as np
        N, H, W = luma.shape
        p = Params(N, H, W, 1, W, 1, energy_mode, use_buffer, alpha_num, alpha_den, max_buffer).c()
        bid = np.zeros(N, dtype=np.int32)
        tr = np.zeros(N, dtype=np.int64)
        nb = C.c_int32(0)
        _check(scpl_segment(self.h, C.byref(p), _ptr(luma), bid.ctypes.data, tr.ctypes.data, C.byref(nb),
                            _stream(stream)), "scpl_segment")
        return bid, tr


class Server:
    """Continuous-batching request server (scpl_server_* in include/scpl.h).

    submit() takes the same dict as one entry of Context.retarget_batch
    (frames must be complete on the device: synchronise first) and returns a
    ticket; the dict's tensors must stay alive and untouched until the
    ticket is done."""

    def __init__(self, device: int = 0, lanes: int = 4, max_batch: int = 8, hbm_budget: int = 0,
                 whole_batch: bool = False):
        h = C.c_void_p()
        cfg = scpl_server_config(lanes, max_batch, hbm_budget, 1 if whole_batch else 0)
        _check(scpl_server_create(device, C.byref(cfg), C.byref(h)), "scpl_server_create")
        self.h = h
        self._live = {}

    def close(self) -> None:
        if self.h:
            scpl_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, clip: dict) -> int:
        import torch
        fr = clip["frames"]
        kw = {k: clip[k] for k in ("energy_mode", "use_buffer", "alpha_num", "alpha_den", "max_buffer",
                                   "target_height", "memo_period") if k in clip}
        p = params_for(fr, clip["target_width"], clip["seams_per_iter"], **kw)
        shp = (p.n_frames, p.target_height or p.height, p.target_width) + ((p.channels,) if fr.dim() == 4 else ())
        if clip.get("out") is None:
            clip["out"] = torch.empty(shp, dtype=torch.uint8, device=fr.device)
        if clip.get("masks") is None and clip.get("want_masks", False):
            clip["masks"] = torch.empty((p.n_frames, p.height, p.width), dtype=torch.int16, device=fr.device)
        if clip.get("buffer_id") is None:
            clip["buffer_id"] = torch.empty(p.n_frames, dtype=torch.int32, device=fr.device)
        c = scpl_clip(p.c(), _ptr(fr), _ptr(clip["out"]), _ptr(clip.get("masks")), _ptr(clip["buffer_id"]))
        # the server's lanes write the outputs on streams of their own: the
        # frames, and whatever earlier work on this stream used the memory
        # the outputs were just given, must be complete first
        torch.cuda.current_stream(fr.device).synchronize()
        t = C.c_int64(0)
        _check(scpl_server_submit(self.h, C.byref(c), C.byref(t)), "scpl_server_submit")
        self._live[t.value] = clip  # keeps the tensors alive
        return int(t.value)

    def poll(self, ticket: int):
        """(done, status)"""
        d, st = C.c_int32(0), C.c_int(0)
        _check(scpl_server_poll(self.h, ticket, C.byref(d), C.byref(st)), "scpl_server_poll")
        return bool(d.value), int(st.value)

    def wait(self, ticket: int) -> dict:
        st = C.c_int(0)
        _check(scpl_server_wait(self.h, ticket, C.byref(st)), "scpl_server_wait")
        _check(st.value, "retarget request")
        return self._live[ticket]

    def times(self, ticket: int):
        """(queue_ms, total_ms) of a done request."""
        q, t = C.c_double(0), C.c_double(0)
        _check(scpl_server_ticket_times(self.h, ticket, C.byref(q), C.byref(t)), "scpl_server_ticket_times")
        return q.value, t.value

    def release(self, ticket: int) -> None:
        _check(scpl_server_release(self.h, ticket), "scpl_server_release")
        self._live.pop(ticket, None)

    @staticmethod
    def footprint(params: Params) -> int:
        """Admission bound (device bytes) of a request."""
        b = C.c_uint64(0)
        cp = params.c()
        _check(scpl_server_footprint(C.byref(cp), C.byref(b)), "scpl_server_footprint")
        return int(b.value)
