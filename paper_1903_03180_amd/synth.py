"""Seeded synthetic inputs for SCPL retargeting: still images and video clips.

This module only draws pixels.  It holds none of the retargeting arithmetic
(no energy, no dynamic programme, no seam logic), so both the HIP library's
callers and the CPU oracle's tests can take their inputs from it.

All pixel values are produced with integer arithmetic from numpy's PCG64
generator, so a (shape, seed) pair always yields the same bytes.

The paper measures on its own videos (Table 1) and images (Fig. 8), which are
not available; these generators stand in for them with the structure that
matters to the method: smooth textured backgrounds, bright or textured moving
objects (motion term, Sec. 3.3), slow camera pans, and hard scene cuts that
must break the spatiotemporal buffer (Sec. 3.2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "value_noise", "image_cfg1", "make_clip", "clip_1080p", "clip_4k", "batch_mix_specs",
    "clip_from_spec", "ClipSpec",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def value_noise(rng: np.random.Generator, H: int, W: int, lattice: int, lo: int, hi: int) -> np.ndarray:
    """Integer bilinear value noise: uniform lattice values in [lo, hi] every
    `lattice` pixels, interpolated in fixed point with round-half-up."""
    L = int(lattice)
    gh, gw = H // L + 2, W // L + 2
    g = rng.integers(lo, hi + 1, size=(gh, gw), dtype=np.int64)
    ii = np.arange(H, dtype=np.int64)
    jj = np.arange(W, dtype=np.int64)
    i0, fy = ii // L, ii % L
    j0, fx = jj // L, jj % L
    a = g[i0][:, j0]
    b = g[i0][:, j0 + 1]
    c = g[i0 + 1][:, j0]
    d = g[i0 + 1][:, j0 + 1]
    top = a * (L - fx)[None, :] + b * fx[None, :]
    bot = c * (L - fx)[None, :] + d * fx[None, :]
    v = (top * (L - fy)[:, None] + bot * fy[:, None] + (L * L) // 2) // (L * L)
    return np.clip(v, 0, 255).astype(np.uint8)


def image_cfg1(seed: int = 1, H: int = 48, W: int = 64) -> np.ndarray:
    """Single grey image: value-noise background (lattice 8, values 40-140)
    plus 3 constant rectangles of value 200-255 and size 6-20 x 5-16."""
    rng = _rng(seed)
    img = value_noise(rng, H, W, 8, 40, 140)
    for _ in range(3):
        w = int(rng.integers(6, 21))
        h = int(rng.integers(5, 17))
        w, h = min(w, W), min(h, H)
        x = int(rng.integers(0, W - w + 1))
        y = int(rng.integers(0, H - h + 1))
        img[y:y + h, x:x + w] = np.uint8(rng.integers(200, 256))
    return img


@dataclass
class _Obj:
    x: int
    y: int
    vx: int
    vy: int
    tex: np.ndarray  # h x w x C uint8


def _make_objects(rng, H, W, C, n_obj, max_speed, size_lo, size_hi):
    objs = []
    for _ in range(n_obj):
        w = int(rng.integers(size_lo, size_hi + 1))
        h = int(rng.integers(size_lo, size_hi + 1))
        w, h = max(1, min(w, W)), max(1, min(h, H))
        x = int(rng.integers(0, W - w + 1))
        y = int(rng.integers(0, H - h + 1))
        speed = int(rng.integers(1, max_speed + 1))
        vx = speed * (1 if rng.integers(0, 2) else -1)
        vy = int(rng.integers(-speed, speed + 1))
        if rng.integers(0, 2):
            lat = max(2, min(w, h) // 4)
            tex = np.stack([value_noise(rng, h, w, lat, 120, 255) for _ in range(C)], axis=-1)
        else:
            cell = int(rng.integers(4, 17))
            a = rng.integers(150, 256, size=C).astype(np.uint8)
            b = rng.integers(0, 90, size=C).astype(np.uint8)
            yy, xx = np.meshgrid(np.arange(h) // cell, np.arange(w) // cell, indexing="ij")
            chk = ((yy + xx) % 2 == 0)[..., None]
            tex = np.where(chk, a[None, None, :], b[None, None, :]).astype(np.uint8)
        objs.append(_Obj(x, y, vx, vy, tex))
    return objs


def _advance(o: _Obj, H: int, W: int) -> None:
    h, w = o.tex.shape[:2]
    nx, ny = o.x + o.vx, o.y + o.vy
    if nx < 0 or nx + w > W:
        o.vx = -o.vx
        nx = o.x + o.vx
    if ny < 0 or ny + h > H:
        o.vy = -o.vy
        ny = o.y + o.vy
    o.x = min(max(nx, 0), W - w)
    o.y = min(max(ny, 0), H - h)


def _background(rng, H, Wb, C, lattice, invert):
    chans = []
    for c in range(C):
        noise = value_noise(rng, H, Wb, lattice, 30, 150).astype(np.int64)
        gi = int(rng.integers(0, 60))
        gj = int(rng.integers(0, 60))
        ramp = (np.arange(H, dtype=np.int64)[:, None] * gi) // max(H, 1) + \
               (np.arange(Wb, dtype=np.int64)[None, :] * gj) // max(Wb, 1)
        v = noise + ramp
        if invert:
            v = 250 - v // 4
        chans.append(np.clip(v, 0, 255).astype(np.uint8))
    return np.stack(chans, axis=-1)


def make_clip(seed: int, N: int, H: int, W: int, C: int = 1, n_obj: int = 4, max_speed: int = 6,
              cut_at: int | None = None, pan_div: int = 0, lattice: int = 64,
              size_lo: int | None = None, size_hi: int | None = None) -> np.ndarray:
    """N x H x W x C uint8 clip (C = 1 returns N x H x W).

    Background: per-channel value noise (lattice `lattice`, values 30-150)
    plus a seeded linear ramp.  `n_obj` textured rectangles (value-noise or
    checker texture) move at integer velocities of magnitude 1..max_speed and
    bounce off the borders.  With pan_div > 0 the camera pans right by one
    pixel every pan_div frames (background sampled at x + t // pan_div).  At
    frame `cut_at` the scene changes: a new background and new objects are
    drawn from seed + 1 with an inverted ramp, so the mean luma difference
    across the cut is large."""
    if size_lo is None:
        size_lo = max(1, min(H, W) // 14)
    if size_hi is None:
        size_hi = max(size_lo, min(H, W) * 3 // 8)
    pan_max = (N - 1) // pan_div if pan_div > 0 else 0

    def scene(s, invert):
        rng = _rng(s)
        bg = _background(rng, H, W + pan_max, C, lattice, invert)
        objs = _make_objects(rng, H, W, C, n_obj, max_speed, size_lo, size_hi)
        return bg, objs

    bg, objs = scene(seed, False)
    out = np.empty((N, H, W, C), dtype=np.uint8)
    for t in range(N):
        if cut_at is not None and t == cut_at:
            bg, objs = scene(seed + 1, True)
        px = t // pan_div if pan_div > 0 else 0
        fr = out[t]
        fr[...] = bg[:, px:px + W, :]
        for o in objs:
            h, w = o.tex.shape[:2]
            fr[o.y:o.y + h, o.x:o.x + w, :] = o.tex
            _advance(o, H, W)
    return out[..., 0] if C == 1 else out


def clip_1080p(seed: int = 2, N: int = 120) -> np.ndarray:
    """1080p RGB clip: 120 frames of 1920x1080, 4 textured rectangles (80-400
    px) moving 1-6 px/frame, scene cut at frame 60."""
    return make_clip(seed, N, 1080, 1920, C=3, n_obj=4, max_speed=6, cut_at=60 if N > 60 else None,
                     lattice=64, size_lo=80, size_hi=400)


def clip_4k(seed: int = 3, N: int = 60) -> np.ndarray:
    """4K luma clip: 60 frames of 3840x2160, 8 objects, slow pan (1 px per 2
    frames)."""
    return make_clip(seed, N, 2160, 3840, C=1, n_obj=8, max_speed=6, cut_at=None, pan_div=2,
                     lattice=64, size_lo=120, size_hi=600)


@dataclass
class ClipSpec:
    seed: int
    N: int
    H: int
    W: int
    Wt: int


_ASPECTS = [(1, 1), (4, 3), (3, 2), (16, 9), (2, 1), (21, 9)]


def batch_mix_specs(n_clips: int = 64, seed0: int = 4000) -> list[ClipSpec]:
    """Uneven clip mix: aspect from {1:1, 4:3, 3:2, 16:9, 2:1, 21:9}, even
    height uniform in [360, 1440], width = clamp(round(h * a), 480, 2560),
    30-240 frames, target width floor(3 W / 4)."""
    specs = []
    for i in range(n_clips):
        rng = _rng(seed0 + i)
        an, ad = _ASPECTS[int(rng.integers(0, len(_ASPECTS)))]
        h = 2 * int(rng.integers(180, 721))
        w = (2 * h * an + ad) // (2 * ad)
        w = min(max(w, 480), 2560)
        n = int(rng.integers(30, 241))
        specs.append(ClipSpec(seed0 + i, n, h, w, (3 * w) // 4))
    return specs


def clip_from_spec(s: ClipSpec) -> np.ndarray:
    return make_clip(s.seed, s.N, s.H, s.W, C=1, n_obj=4, max_speed=6, lattice=64)
