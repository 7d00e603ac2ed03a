"""Seeded generators for exemplars, guides and jitter tables.

Everything here is plain numpy driven by ``numpy.random.default_rng(seed)``;
the same seed always yields the same bytes.  The shapes follow the paper's
three guidance scenarios (Sec. 4): a hand-drawn sphere exemplar transferred
onto a normal-mapped target, and a painted texture transferred through
texture coordinates.  The paper's own exemplars are not available, so
stochastic value-noise textures stand in for hand-drawn media.

Conventions shared by both consumers (oracle and HIP library):

* images are row-major ``(rows, cols, channels)``; pixel p = (x, y) with x the
  column and y the row;
* a guide has two channels, ``uint8`` (format ``GUIDE_U8X2``) or ``uint16``
  (format ``GUIDE_U16X2``), or three ``uint8`` channels stored in four bytes
  per pixel, the fourth zero (format ``GUIDE_U8X3``: a normal pair plus an
  appearance channel);
* a guide of C = 2..8 channels of 8 bits (format ``GUIDE_U8XN``) or 16 bits
  (format ``GUIDE_U16XN``) stores each pixel's channels in order in a texel
  of 4, 8 or 16 bytes (the smallest that holds them), the rest zero:
  ``(rows, cols, elements)`` of uint8 or uint16;
* the seed hierarchy has ``levels`` levels with spacings
  ``finest << (levels - 1 - i)`` for level i = 0 (coarsest) ... levels-1;
* level i's jitter table covers ``ceil(W/h) x ceil(H/h)`` cells, row-major,
  each entry ``jx | (jy << 16)`` with ``0 <= jx, jy < h``; the levels are
  concatenated coarsest first.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

GUIDE_U8X2 = 0
GUIDE_U16X2 = 1
GUIDE_U8X3 = 2
GUIDE_U8XN = 3
GUIDE_U16XN = 4


@dataclasses.dataclass
class Style:
    """A source exemplar C_S with its guide G_S."""

    rgb: np.ndarray  # (Sh, Sw, 3) uint8
    guide: np.ndarray  # (Sh, Sw, 2) uint8 or uint16
    fmt: int
    lut_bits: int

    @property
    def sw(self) -> int:
        return int(self.rgb.shape[1])

    @property
    def sh(self) -> int:
        return int(self.rgb.shape[0])


@dataclasses.dataclass
class Params:
    levels: int
    finest: int
    threshold: int
    radius: int


@dataclasses.dataclass
class Frame:
    """One target: its guide G_T, the source of its seeds' jitter (a table,
    or the seed of the jitter hash), parameters and style index."""

    guide: np.ndarray  # (H, W, 2)
    fmt: int
    jitter: Optional[np.ndarray]  # uint32 per-level tables, or None: the hash of `seed`
    params: Params
    style: int = 0
    seed: Optional[int] = None  # jitter hash seed when `jitter` is None

    @property
    def w(self) -> int:
        return int(self.guide.shape[1])

    @property
    def h(self) -> int:
        return int(self.guide.shape[0])


# ---------------------------------------------------------------------------
# seed-hierarchy jitter tables (the paper's RandomJitterTable, drawn up front)
# ---------------------------------------------------------------------------

def level_spacings(levels: int, finest: int) -> List[int]:
    return [finest << (levels - 1 - i) for i in range(levels)]


def jitter_cells(w: int, h: int, levels: int, finest: int) -> List[tuple]:
    """(cells_x, cells_y) per level, coarsest first."""
    out = []
    for sp in level_spacings(levels, finest):
        out.append(((w + sp - 1) // sp, (h + sp - 1) // sp))
    return out


def jitter_table(w: int, h: int, levels: int, finest: int, seed: Optional[int]) -> np.ndarray:
    """Uniform integer jitter per cell and level; ``seed=None`` gives all zeros
    (seeds on the cell corners)."""
    rng = np.random.default_rng(seed) if seed is not None else None
    parts = []
    for sp, (cx, cy) in zip(level_spacings(levels, finest), jitter_cells(w, h, levels, finest)):
        if rng is None:
            parts.append(np.zeros(cx * cy, np.uint32))
            continue
        jx = rng.integers(0, sp, size=cx * cy, dtype=np.uint32)
        jy = rng.integers(0, sp, size=cx * cy, dtype=np.uint32)
        parts.append(jx | (jy << np.uint32(16)))
    if not parts:
        return np.zeros(0, np.uint32)
    return np.ascontiguousarray(np.concatenate(parts).astype(np.uint32))


# ---------------------------------------------------------------------------
# textures and guides
# ---------------------------------------------------------------------------

def _value_noise(w: int, h: int, period: float, rng: np.random.Generator) -> np.ndarray:
    """Smoothstep-interpolated lattice noise in [0, 1), shape (h, w)."""
    nx = int(np.ceil(w / period)) + 2
    ny = int(np.ceil(h / period)) + 2
    lat = rng.random((ny, nx))
    gx = (np.arange(w) + 0.5) / period
    gy = (np.arange(h) + 0.5) / period
    ix = np.floor(gx).astype(np.int64)
    iy = np.floor(gy).astype(np.int64)
    fx = gx - ix
    fy = gy - iy
    sx = fx * fx * (3.0 - 2.0 * fx)
    sy = fy * fy * (3.0 - 2.0 * fy)
    a = lat[iy[:, None], ix[None, :]]
    b = lat[iy[:, None], ix[None, :] + 1]
    c = lat[iy[:, None] + 1, ix[None, :]]
    d = lat[iy[:, None] + 1, ix[None, :] + 1]
    top = a + (b - a) * sx[None, :]
    bot = c + (d - c) * sx[None, :]
    return top + (bot - top) * sy[:, None]


def value_noise_rgb(w: int, h: int, seed: int) -> np.ndarray:
    """Stochastic RGB texture: three octaves (periods 16/8/4 px, amplitudes
    1/.5/.25) per channel, rescaled to the full uint8 range."""
    rng = np.random.default_rng(seed)
    out = np.empty((h, w, 3), np.uint8)
    for ch in range(3):
        v = np.zeros((h, w))
        for period, amp in ((16, 1.0), (8, 0.5), (4, 0.25)):
            v += amp * _value_noise(w, h, period, rng)
        lo, hi = v.min(), v.max()
        out[:, :, ch] = np.floor(255.0 * (v - lo) / max(hi - lo, 1e-12) + 0.5).astype(np.uint8)
    return out


def _encode_normal(nx: np.ndarray, ny: np.ndarray) -> np.ndarray:
    e0 = np.clip(np.floor((nx + 1.0) * 127.5 + 0.5), 0, 255)
    e1 = np.clip(np.floor((ny + 1.0) * 127.5 + 0.5), 0, 255)
    return np.stack([e0, e1], axis=-1).astype(np.uint8)


def sphere_guide_u8(size: int) -> np.ndarray:
    """Normals (x, y components) of a sphere of radius size/2 centred in a
    size x size exemplar; outside the disk the rim normal is used."""
    c = size / 2.0
    x = (np.arange(size) + 0.5 - c) / c
    dx, dy = np.meshgrid(x, x)  # dx varies along columns, dy along rows
    r2 = dx * dx + dy * dy
    r = np.sqrt(np.maximum(r2, 1e-300))
    outside = r2 > 1.0
    nx = np.where(outside, dx / r, dx)
    ny = np.where(outside, dy / r, dy)
    return _encode_normal(nx, ny)


def _gradient(hf: np.ndarray):
    """Central differences per axis (one-sided at the ends); zero along an
    axis of a single sample."""
    gy = np.gradient(hf, axis=0) if hf.shape[0] > 1 else np.zeros_like(hf)
    gx = np.gradient(hf, axis=1) if hf.shape[1] > 1 else np.zeros_like(hf)
    return gy, gx


def bump_guide_u8(w: int, h: int, nbumps: int, seed: int) -> np.ndarray:
    """Normals of a heightfield made of Gaussian bumps (centres uniform,
    sigma in [0.03, 0.12]*min(w, h), signed amplitude in [0.5, 1.5]*sigma)."""
    rng = np.random.default_rng(seed)
    m = float(min(w, h))
    hf = np.zeros((h, w))
    for _ in range(nbumps):
        cx = rng.uniform(0, w)
        cy = rng.uniform(0, h)
        sig = rng.uniform(0.03, 0.12) * m
        amp = rng.uniform(0.5, 1.5) * sig * (1.0 if rng.random() < 0.5 else -1.0)
        rad = 5.0 * sig
        x0, x1 = max(0, int(cx - rad)), min(w, int(cx + rad) + 1)
        y0, y1 = max(0, int(cy - rad)), min(h, int(cy + rad) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1) + 0.5 - cx
        ys = np.arange(y0, y1) + 0.5 - cy
        hf[y0:y1, x0:x1] += amp * np.exp(-(ys[:, None] ** 2 + xs[None, :] ** 2) / (2 * sig * sig))
    gy, gx = _gradient(hf)
    norm = np.sqrt(gx * gx + gy * gy + 1.0)
    return _encode_normal(-gx / norm, -gy / norm)


def animated_bump_guides(w: int, h: int, nbumps: int, nframes: int, drift: float,
                         seed: int) -> List[np.ndarray]:
    """An animated target: the heightfield of bump_guide_u8 with every bump
    centre moving by up to ``drift`` pixels per frame in its own seeded
    direction; one normal guide per frame."""
    rng = np.random.default_rng(seed)
    m = float(min(w, h))
    bumps = []
    for _ in range(nbumps):
        cx, cy = rng.uniform(0, w), rng.uniform(0, h)
        sig = rng.uniform(0.03, 0.12) * m
        amp = rng.uniform(0.5, 1.5) * sig * (1.0 if rng.random() < 0.5 else -1.0)
        ang = rng.uniform(0, 2 * np.pi)
        spd = rng.uniform(0.5, 1.0) * drift
        bumps.append((cx, cy, sig, amp, spd * np.cos(ang), spd * np.sin(ang)))
    out = []
    for f in range(nframes):
        hf = np.zeros((h, w))
        for cx0, cy0, sig, amp, vx, vy in bumps:
            cx, cy = cx0 + vx * f, cy0 + vy * f
            rad = 5.0 * sig
            x0, x1 = max(0, int(cx - rad)), min(w, int(cx + rad) + 1)
            y0, y1 = max(0, int(cy - rad)), min(h, int(cy + rad) + 1)
            if x0 >= x1 or y0 >= y1:
                continue
            xs = np.arange(x0, x1) + 0.5 - cx
            ys = np.arange(y0, y1) + 0.5 - cy
            hf[y0:y1, x0:x1] += amp * np.exp(-(ys[:, None] ** 2 + xs[None, :] ** 2) / (2 * sig * sig))
        gy, gx = _gradient(hf)
        norm = np.sqrt(gx * gx + gy * gy + 1.0)
        out.append(_encode_normal(-gx / norm, -gy / norm))
    return out


def jitter_schedule(w: int, h: int, levels: int, finest: int, nframes: int, hold: int,
                    seed: int) -> List[np.ndarray]:
    """Per-frame jitter tables for an animation: a fresh table every ``hold``
    frames (hold = 1: seeds re-drawn every frame, the flickering
    hand-coloured look; hold >= nframes: one table for the whole sequence)."""
    return [jitter_table(w, h, levels, finest, seed + f // max(1, hold)) for f in range(nframes)]


def appearance_u8(rgb: np.ndarray, radius: int) -> np.ndarray:
    """Appearance channel: integer luma (77 R + 150 G + 29 B + 128) >> 8,
    box-averaged over a (2 radius + 1)^2 window clamped at the borders."""
    luma = ((77 * rgb[..., 0].astype(np.int64) + 150 * rgb[..., 1].astype(np.int64)
             + 29 * rgb[..., 2].astype(np.int64) + 128) >> 8)
    h, w = luma.shape
    k = 2 * radius + 1
    pad = np.pad(luma, radius, mode="edge")
    c = np.zeros((h + 2 * radius + 1, w + 2 * radius + 1), np.int64)
    c[1:, 1:] = pad.cumsum(0).cumsum(1)
    box = c[k:, k:] - c[:-k, k:] - c[k:, :-k] + c[:-k, :-k]
    return ((box + k * k // 2) // (k * k)).astype(np.uint8)


def guide_u8x3(two: np.ndarray, third: np.ndarray) -> np.ndarray:
    """A three-channel guide in its storage layout: (rows, cols, 4) uint8,
    channels 0-1 from ``two``, channel 2 from ``third``, byte 3 zero."""
    h, w = third.shape
    out = np.zeros((h, w, 4), np.uint8)
    out[..., :2] = two
    out[..., 2] = third
    return out


def texel_elements(depth: int, channels: int) -> int:
    """Elements per texel of a ``channels``-channel guide of ``depth`` bits."""
    b = channels * depth // 8
    return (4 if b <= 4 else 8 if b <= 8 else 16) * 8 // depth


def guide_n(chans, depth: int) -> np.ndarray:
    """A many-channel guide in its storage layout from a list of C (rows,
    cols) channel arrays: (rows, cols, elements) of uint8 (depth 8) or
    uint16 (depth 16), channel k in element k, the rest zero."""
    h, w = np.asarray(chans[0]).shape
    dt = np.uint8 if depth == 8 else np.uint16
    out = np.zeros((h, w, texel_elements(depth, len(chans))), dt)
    for k, c in enumerate(chans):
        out[..., k] = c
    return out


def _box_mean_u8(v: np.ndarray, radius: int) -> np.ndarray:
    """Integer box average over a (2 radius + 1)^2 window clamped at the
    borders, rounded to nearest."""
    h, w = v.shape
    k = 2 * radius + 1
    pad = np.pad(v.astype(np.int64), radius, mode="edge")
    c = np.zeros((h + 2 * radius + 1, w + 2 * radius + 1), np.int64)
    c[1:, 1:] = pad.cumsum(0).cumsum(1)
    box = c[k:, k:] - c[:-k, k:] - c[k:, :-k] + c[:-k, :-k]
    return ((box + k * k // 2) // (k * k)).astype(np.uint8)


def chroma_u8(rgb: np.ndarray, radius: int):
    """Two opponent-colour channels of an image, box-averaged like the
    appearance channel: (R - G + 255) / 2 and (R + G - 2 B + 510) / 4, in
    integers."""
    r, g, b = (rgb[..., k].astype(np.int64) for k in range(3))
    return (_box_mean_u8((r - g + 255) // 2, radius),
            _box_mean_u8((r + g - 2 * b + 510) // 4, radius))


def features_u8(rgb: np.ndarray, normals: np.ndarray) -> np.ndarray:
    """Five 8-bit guide channels: a normal pair, the appearance channel and
    the two chroma channels of ``rgb`` (8-byte texels)."""
    c1, c2 = chroma_u8(rgb, 4)
    return guide_n([normals[..., 0], normals[..., 1], appearance_u8(rgb, 4), c1, c2], 8)


def features_u16(uv: np.ndarray, normals: np.ndarray) -> np.ndarray:
    """Four 16-bit guide channels: texture coordinates and the normal pair
    widened to 16 bits (x 257) (8-byte texels)."""
    return guide_n([uv[..., 0], uv[..., 1], normals[..., 0].astype(np.uint16) * 257,
                    normals[..., 1].astype(np.uint16) * 257], 16)


def identity_uv_guide_u16(sw: int, sh: int) -> np.ndarray:
    """Texture coordinates of each texel centre, scaled to 16 bits."""
    gx = np.floor((np.arange(sw) + 0.5) * 65536.0 / sw).astype(np.int64)
    gy = np.floor((np.arange(sh) + 0.5) * 65536.0 / sh).astype(np.int64)
    g = np.empty((sh, sw, 2), np.uint16)
    g[:, :, 0] = np.minimum(gx, 65535)[None, :]
    g[:, :, 1] = np.minimum(gy, 65535)[:, None]
    return g


def warped_uv_guide_u16(w: int, h: int, sw: int, sh: int, seed: int,
                        lattice: int = 256, amplitude: float = 12.0) -> np.ndarray:
    """A texel-scale UV grid tiled over the target (wrapping at the texture
    size) and warped by a smooth value-noise displacement field."""
    rng = np.random.default_rng(seed)
    dx = (2.0 * _value_noise(w, h, lattice, rng) - 1.0) * amplitude
    dy = (2.0 * _value_noise(w, h, lattice, rng) - 1.0) * amplitude
    x = np.arange(w)[None, :] + dx + 0.5
    y = np.arange(h)[:, None] + dy + 0.5
    u = np.floor(np.mod(x, sw) * 65536.0 / sw)
    v = np.floor(np.mod(y, sh) * 65536.0 / sh)
    g = np.empty((h, w, 2), np.uint16)
    g[:, :, 0] = np.clip(u, 0, 65535)
    g[:, :, 1] = np.clip(v, 0, 65535)
    return g


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def voronoi_labels(w: int, h: int, nlabels: int, nsites: int, seed: int) -> np.ndarray:
    """A uint8 label map of (h, w): seeded sites at uniform random positions,
    site k labelled k mod nlabels, every pixel labelled by its nearest site
    (squared distance, ties to the lower site index).  Stands in for the
    segmentation maps of semantic regions."""
    rng = np.random.default_rng(seed)
    sx = rng.integers(0, w, size=nsites)
    sy = rng.integers(0, h, size=nsites)
    yy, xx = np.mgrid[0:h, 0:w]
    best = np.full((h, w), np.iinfo(np.int64).max, np.int64)
    lab = np.zeros((h, w), np.uint8)
    for k in range(nsites):
        d = (xx - int(sx[k])) ** 2 + (yy - int(sy[k])) ** 2
        take = d < best
        best[take] = d[take]
        lab[take] = k % nlabels
    return lab


CONFIG_NAMES = {
    1: "normal-256x256",
    2: "normal-1920x1080",
    3: "uv-3840x2160",
    4: "batch-64-uneven",
    5: "serve-poisson",
    6: "appearance-1920x1080",
    7: "features-1920x1080",
}

NORMAL_PARAMS = Params(levels=4, finest=8, threshold=32, radius=3)
UV_PARAMS = Params(levels=5, finest=8, threshold=4096, radius=3)


def _sphere_style(size: int, seed: int) -> Style:
    return Style(value_noise_rgb(size, size, seed), sphere_guide_u8(size), GUIDE_U8X2, 8)


def _uv_style(size: int, seed: int, lut_bits: int) -> Style:
    return Style(value_noise_rgb(size, size, seed), identity_uv_guide_u16(size, size),
                 GUIDE_U16X2, lut_bits)


APPEARANCE_PARAMS = Params(levels=4, finest=8, threshold=192, radius=3)


def _appearance_style(size: int, seed: int, lut_bits: int) -> Style:
    rgb = value_noise_rgb(size, size, seed)
    g = guide_u8x3(sphere_guide_u8(size), appearance_u8(rgb, 4))
    return Style(rgb, g, GUIDE_U8X3, lut_bits)


def appearance_target(w: int, h: int, nbumps: int, seed: int) -> np.ndarray:
    """Target of the appearance workload: bump normals plus the appearance
    channel of a value-noise image standing in for the subject."""
    return guide_u8x3(bump_guide_u8(w, h, nbumps, seed),
                      appearance_u8(value_noise_rgb(w, h, seed + 1), 4))


FEATURE_PARAMS = Params(levels=4, finest=8, threshold=160, radius=3)
FEATURE16_PARAMS = Params(levels=4, finest=8, threshold=1 << 22, radius=3)


def _features_style(size: int, seed: int, depth: int) -> Style:
    """Exemplar with a five-channel 8-bit guide (sphere normals, appearance,
    chroma), or a four-channel 16-bit one (texture coordinates and sphere
    normals)."""
    rgb = value_noise_rgb(size, size, seed)
    if depth == 8:
        return Style(rgb, features_u8(rgb, sphere_guide_u8(size)), GUIDE_U8XN, 0)
    return Style(rgb, features_u16(identity_uv_guide_u16(size, size), sphere_guide_u8(size)),
                 GUIDE_U16XN, 0)


def features_target(w: int, h: int, seed: int, depth: int, src_rgb: np.ndarray) -> np.ndarray:
    """Target of the features workload: an object textured with the exemplar
    through warped texture coordinates (``warped_uv_guide_u16`` over the
    exemplar's size).  Its normals are the exemplar's sphere normals at those
    coordinates plus bump detail ((bump - 128) / 8, clamped); with 8 bits the
    other channels are the appearance and chroma of the exemplar seen
    through the same coordinates, with 16 bits the coordinates themselves."""
    sh, sw = src_rgb.shape[:2]
    uv = warped_uv_guide_u16(w, h, sw, sh, seed + 1)
    iu = (uv[..., 0].astype(np.int64) * sw) >> 16
    iv = (uv[..., 1].astype(np.int64) * sh) >> 16
    bump = bump_guide_u8(w, h, 64, seed).astype(np.int64)
    n = sphere_guide_u8(sw)[iv, iu].astype(np.int64) + (bump - 128) // 8
    n = np.clip(n, 0, 255).astype(np.uint8)
    if depth == 8:
        return features_u8(src_rgb[iv, iu], n)
    return features_u16(uv, n)


def _frame(guide: np.ndarray, fmt: int, p: Params, seed: int, style: int = 0) -> Frame:
    """A workload frame whose seeds' jitter is the integer hash of (cell,
    level, seed): no table travels with it."""
    return Frame(np.ascontiguousarray(guide), fmt, None, p, style, seed)


def config(n: int, **kw):
    """Return ``(styles, frames)`` for workload n (1..4, 6, 7), or for n == 5 a
    dict describing the serving trace.  Keyword overrides: ``frames`` (cfg 4),
    ``requests`` and ``qps`` (cfg 5), ``lut_bits``, ``w`` and ``h`` (cfg 6),
    ``w``, ``h``, ``size`` (exemplar side) and ``depth`` (8 or 16) (cfg 7).
    A workload-7 style's ``guide`` holds 5 channels (8 bits) or 4 (16 bits)
    and its ``lut_bits`` is 0 (its lookups are exact searches)."""
    if n == 1:
        st = _sphere_style(256, 101)
        p = Params(levels=3, finest=8, threshold=48, radius=2)
        return [st], [_frame(bump_guide_u8(256, 256, 8, 102), GUIDE_U8X2, p, 1)]
    if n == 2:
        st = _sphere_style(512, 201)
        return [st], [_frame(bump_guide_u8(1920, 1080, 64, 202), GUIDE_U8X2, NORMAL_PARAMS, 1)]
    if n == 3:
        st = _uv_style(2048, 301, 11)
        g = warped_uv_guide_u16(3840, 2160, 2048, 2048, 302)
        return [st], [_frame(g, GUIDE_U16X2, UV_PARAMS, 1)]
    if n == 4:
        nframes = int(kw.get("frames", 64))
        styles = [_sphere_style(512, 411), _sphere_style(512, 412),
                  _uv_style(512, 413, 9), _uv_style(512, 414, 9)]
        rng = np.random.default_rng(401)
        frames = []
        half = nframes // 2
        for i in range(nframes):
            w = int(rng.integers(320, 1921))
            h = int(rng.integers(240, 1081))
            if i < half:
                g = bump_guide_u8(w, h, 16, 4100 + i)
                frames.append(_frame(g, GUIDE_U8X2, NORMAL_PARAMS, 4200 + i, style=i % 2))
            else:
                g = warped_uv_guide_u16(w, h, 512, 512, 4100 + i)
                frames.append(_frame(g, GUIDE_U16X2, UV_PARAMS, 4200 + i, style=2 + i % 2))
        return styles, frames
    if n == 5:
        nreq = int(kw.get("requests", 10000))
        qps = float(kw.get("qps", 2000.0))
        pool = int(kw.get("pool", 2))
        styles = ([_sphere_style(512, 510 + k) for k in range(4)]
                  + [_uv_style(512, 520 + k, 9) for k in range(4)])
        sizes = [(640, 480), (1280, 720), (1920, 1080)]
        # a small pool of distinct guides per (size, guidance type); requests
        # reference them, each with its own jitter table (per-frame seeds)
        guides = {}
        for si, (w, h) in enumerate(sizes):
            for k in range(pool):
                guides[(si, GUIDE_U8X2, k)] = bump_guide_u8(w, h, 16, 5000 + 10 * si + k)
                guides[(si, GUIDE_U16X2, k)] = warped_uv_guide_u16(w, h, 512, 512, 5100 + 10 * si + k)
        rng = np.random.default_rng(501)
        gaps = rng.exponential(1.0 / qps, size=nreq)
        arrivals = np.cumsum(gaps) - gaps[0]
        size_idx = rng.integers(0, len(sizes), size=nreq)
        style_idx = rng.integers(0, len(styles), size=nreq)
        pool_idx = rng.integers(0, pool, size=nreq)
        return {
            "styles": styles,
            "sizes": sizes,
            "guides": guides,
            "arrivals": arrivals,
            "size_idx": size_idx,
            "style_idx": style_idx,
            "pool_idx": pool_idx,
            # every request's own jitter hash seed (a fresh seed pattern per frame)
            "seeds": 7000 + np.arange(nreq),
            "params": {GUIDE_U8X2: NORMAL_PARAMS, GUIDE_U16X2: UV_PARAMS},
        }
    if n == 6:
        st = _appearance_style(512, 601, int(kw.get("lut_bits", 8)))
        w, h = int(kw.get("w", 1920)), int(kw.get("h", 1080))
        return [st], [_frame(appearance_target(w, h, 64, 602), GUIDE_U8X3, APPEARANCE_PARAMS, 1)]
    if n == 7:
        depth = int(kw.get("depth", 8))
        size = int(kw.get("size", 512))
        st = _features_style(size, 701, depth)
        w, h = int(kw.get("w", 1920)), int(kw.get("h", 1080))
        g = features_target(w, h, 702, depth, st.rgb)
        p = FEATURE_PARAMS if depth == 8 else FEATURE16_PARAMS
        return [st], [_frame(g, GUIDE_U8XN if depth == 8 else GUIDE_U16XN, p, 1)]
    raise ValueError(f"unknown workload {n}")
