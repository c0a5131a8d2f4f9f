"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain CPU SCPL oracle.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The HIP library and its binding never do.  Every function
takes and returns numpy arrays and calls straight into scpl_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scpl_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

GRADIENT, MOTION = 0, 1


def build(force: bool = True) -> str:
    """Compile scpl_oracle.c with gcc -O2 into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        L.oracle_luma.argtypes = [P, i64, P]
        L.oracle_energy.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P]
        L.oracle_energy_max.argtypes = [C.c_int]
        L.oracle_energy_max.restype = i32
        L.oracle_dp.argtypes = [P, C.c_int, C.c_int, P, P, P]
        L.oracle_select.argtypes = [P, P, C.c_int, C.c_int, C.c_int, P, P]
        L.oracle_select.restype = C.c_int
        L.oracle_backtrack.argtypes = [P, C.c_int, C.c_int, P, C.c_int, P]
        L.oracle_isqrt.argtypes = [C.c_uint64]
        L.oracle_isqrt.restype = C.c_uint64
        L.oracle_asde_sum.argtypes = [P, P, i64, C.c_int]
        L.oracle_asde_sum.restype = i64
        L.oracle_reject.argtypes = [i64, C.c_int, i64, i32, i32, i32]
        L.oracle_reject.restype = C.c_int
        L.oracle_segment.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, i32, i32, C.c_int, P, P]
        L.oracle_segment.restype = C.c_int
        L.oracle_retarget.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_int, i32, i32, C.c_int, C.c_int, P, P, P, P, i64]
        L.oracle_retarget.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def luma(rgb: np.ndarray) -> np.ndarray:
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    y = np.empty(rgb.shape[:-1], dtype=np.uint8)
    lib().oracle_luma(_p(rgb), y.size, _p(y))
    return y


def energy(y: np.ndarray, yprev: np.ndarray | None = None, mode: int = GRADIENT) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.uint8)
    H, W = y.shape
    e = np.empty((H, W), dtype=np.int32)
    pp = None
    if yprev is not None:
        yprev = np.ascontiguousarray(yprev, dtype=np.uint8)
        assert yprev.shape == y.shape
        pp = _p(yprev)
    lib().oracle_energy(_p(y), pp, H, W, mode, _p(e))
    return e


def energy_max(mode: int) -> int:
    return int(lib().oracle_energy_max(mode))


def dp(u: np.ndarray):
    """Returns (ce, label, dir), each H x W."""
    u = np.ascontiguousarray(u, dtype=np.int32)
    H, W = u.shape
    ce = np.empty((H, W), dtype=np.int32)
    lab = np.empty((H, W), dtype=np.int32)
    d = np.empty((H, W), dtype=np.int8)
    lib().oracle_dp(_p(u), H, W, _p(ce), _p(lab), _p(d))
    return ce, lab, d


def select(ce_last: np.ndarray, label_last: np.ndarray, k: int, limit: int | None = None):
    """Returns (children sorted by column, p_eff)."""
    ce_last = np.ascontiguousarray(ce_last, dtype=np.int32)
    label_last = np.ascontiguousarray(label_last, dtype=np.int32)
    W = ce_last.shape[0]
    if limit is None:
        limit = W
    ch = np.zeros(max(W, 1), dtype=np.int32)
    pe = np.zeros(1, dtype=np.int32)
    kk = lib().oracle_select(_p(ce_last), _p(label_last), W, k, limit, _p(ch), _p(pe))
    return ch[:kk].copy(), int(pe[0])


def backtrack(d: np.ndarray, children: np.ndarray) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.int8)
    H, W = d.shape
    children = np.ascontiguousarray(children, dtype=np.int32)
    kk = children.shape[0]
    seams = np.zeros((max(kk, 1), H), dtype=np.int32)
    lib().oracle_backtrack(_p(d), H, W, _p(children), kk, _p(seams))
    return seams[:kk].copy()


def isqrt(q: int) -> int:
    return int(lib().oracle_isqrt(q))


def asde_sum(s1: np.ndarray, s2: np.ndarray, n: int) -> int:
    s1 = np.ascontiguousarray(s1, dtype=np.uint64)
    s2 = np.ascontiguousarray(s2, dtype=np.uint64)
    return int(lib().oracle_asde_sum(_p(s1), _p(s2), s1.size, n))


def reject(S: int, n: int, npx: int, emax: int, anum: int, aden: int) -> bool:
    return bool(lib().oracle_reject(S, n, npx, emax, anum, aden))


def segment(Y: np.ndarray, mode: int = MOTION, use_buffer: int = 1, anum: int = 1, aden: int = 5,
            max_buffer: int = 0):
    """Y: N x H x W luma.  Returns (buffer_id[N], s_trace[N])."""
    Y = np.ascontiguousarray(Y, dtype=np.uint8)
    N, H, W = Y.shape
    bid = np.empty(N, dtype=np.int32)
    st = np.empty(N, dtype=np.int64)
    lib().oracle_segment(_p(Y), N, H, W, mode, use_buffer, anum, aden, max_buffer, _p(bid), _p(st))
    return bid, st


def retarget(frames: np.ndarray, Wt: int, k: int, mode: int = MOTION, use_buffer: int = 1, anum: int = 1,
             aden: int = 5, max_buffer: int = 0, want_masks: bool = True, log_cap: int = 1 << 16,
             memo_period: int = 0):
    """frames: N x H x W (luma) or N x H x W x 3 (RGB) uint8.

    memo_period m >= 2: only buffers b with b mod m == 0 are carved; the
    others remove the pixels buffer b - (b mod m) removed (seam memorisation).
    Returns dict(out, masks, buffer_id, log) where log rows are
    (buffer, W_r, P_eff, k_iter) for every iteration of every carved buffer."""
    frames = np.ascontiguousarray(frames, dtype=np.uint8)
    if frames.ndim == 3:
        N, H, W = frames.shape
        Cc = 1
        out = np.empty((N, H, Wt), dtype=np.uint8)
    else:
        N, H, W, Cc = frames.shape
        out = np.empty((N, H, Wt, Cc), dtype=np.uint8)
    masks = np.empty((N, H, W), dtype=np.uint16) if want_masks else None
    bid = np.empty(N, dtype=np.int32)
    log = np.empty((log_cap, 4), dtype=np.int32)
    n = lib().oracle_retarget(_p(frames), N, H, W, Cc, Wt, k, mode, use_buffer, anum, aden, max_buffer,
                              memo_period, _p(out), _p(masks) if masks is not None else None, _p(bid), _p(log), log_cap)
    if n < 0:
        raise ValueError(f"oracle_retarget failed with {n}")
    return dict(out=out, masks=masks, buffer_id=bid, log=log[:min(n, log_cap)].copy())


def _t(a: np.ndarray) -> np.ndarray:
    """Frames N x H x W (x C) -> N x W x H (x C)."""
    return np.ascontiguousarray(np.swapaxes(a, 1, 2))


def retarget_2d(frames: np.ndarray, Wt: int, Ht: int, k: int, **kw):
    """Width, then height (Sec. 3.1, eq. 2: a horizontal seam is a vertical seam of
    the transposed frame): the frames are carved to width Wt as by
    retarget(), then transposed, carved to Ht columns, and transposed back.
    Masks and buffer ids describe the height pass when only the height
    shrinks; when both shrink, buffer ids are the width pass's and there are
    no masks.  The log holds the width pass's rows, then the height pass's."""
    H, W = frames.shape[1], frames.shape[2]
    if Ht >= H:
        return retarget(frames, Wt, k, **kw)
    first = retarget(frames, Wt, k, **kw) if Wt < W else None
    mid = first["out"] if first is not None else frames
    second = retarget(_t(mid), Ht, k, **kw)
    return dict(out=_t(second["out"]),
                masks=None if first is not None else _t(second["masks"]) if second["masks"] is not None else None,
                buffer_id=first["buffer_id"] if first is not None else second["buffer_id"],
                log=np.concatenate([first["log"], second["log"]]) if first is not None else second["log"])
