"""Pins of the oracle's per-pixel level loop (Algorithm 2) and voting blend
(end of Sec. 3.2): hand-worked cases, special cases that reduce to texture
mapping, and the paper's invariants, checked on random and workload-shaped
inputs."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from tests.test_oracle_lut import brute_lut

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def frame_jitter(fr):
    """A workload frame's jitter table: its own, or the one the jitter hash
    of its seed defines."""
    if fr.jitter is not None:
        return fr.jitter
    return oracle.jitter_hash(fr.w, fr.h, fr.params.levels, fr.params.finest, fr.seed)


def grid_guide(w, h):
    """G_S(x, y) = (16x, 16y): unique values for images up to 16x16."""
    g = np.zeros((h, w, 2), np.uint8)
    g[:, :, 0] = (16 * np.arange(w))[None, :]
    g[:, :, 1] = (16 * np.arange(h))[:, None]
    return g


def unpack(nnf):
    return (nnf & 0xFFFF).astype(np.int64), (nnf >> 16).astype(np.int64)


def gather_rgb(src, nnf):
    x, y = unpack(nnf)
    return src[y, x]


# ------------------------------------------------------------- hand-worked

def test_level_loop_hand(ora):
    case = GOLD["level_loop"]
    gs = grid_guide(8, 8)
    gt = gs.copy()
    gt[:, 4:] = gs[:, 2:6]
    lut = brute_lut(gs, 8)
    nnf, chunk = ora.assign(gs, lut, 8, gt, None, case["levels"], case["finest"],
                            case["threshold"])
    lvl, qx, qy = ora.decode_chunk(chunk)
    for c in case["cases"]:
        x, y = c["p"]
        assert [nnf[y, x] & 0xFFFF, nnf[y, x] >> 16] == c["nnf"]
        assert lvl[y, x] == c["level"] and [qx[y, x], qy[y, x]] == c["q"]


def test_identity_hand(ora):
    """G_T = G_S with unique guide values: every pixel maps to itself and the
    stylised image is the exemplar, for any threshold >= 1 and radius."""
    gs = grid_guide(8, 8)
    rng = np.random.default_rng(0)
    src = rng.integers(0, 256, size=(8, 8, 3), dtype=np.uint8)
    lut = brute_lut(gs, 8)
    for t in (1, 5, 1000):
        for r in (0, 1, 2, 3):
            rgb, chunk, nnf = ora.stylize(src, gs, lut, 8, gs, None, 2, 2, t, r)
            x, y = unpack(nnf)
            assert np.all(x == np.arange(8)[None, :]) and np.all(y == np.arange(8)[:, None])
            np.testing.assert_array_equal(rgb, src)


@pytest.mark.parametrize("name", ["blend_1d", "blend_half_up", "blend_outside_source"])
def test_blend_hand(ora, name):
    case = GOLD[name]
    red = np.array(case["src_red"], np.uint8)
    src = np.zeros((1, red.size, 3), np.uint8)
    src[0, :, 0] = red
    src[0, :, 1] = 255 - red
    nnf = np.array(case["nnf_x"], np.uint32).reshape(1, -1)
    out = ora.blend(src, nnf, case["radius"])
    np.testing.assert_array_equal(out[0, :, 0], case["out_red"])
    # the other channel rounds the complementary sums the same way
    assert out.shape == (1, nnf.size, 3)


def test_blend_2d_hand(ora):
    """3x3 target, r = 1, two chunks with x-offsets 0 and +4 split by column;
    centre pixel: 6 votes at offset 0 and 3 at offset 4."""
    src = np.zeros((3, 8, 3), np.uint8)
    src[:, :, 0] = (10 * np.arange(8))[None, :]
    nnf = np.zeros((3, 3), np.uint32)
    for y in range(3):
        for x in range(3):
            ox = 4 if x == 2 else 0
            nnf[y, x] = (x + ox) | (y << 16)
    out = ora.blend(src, nnf, 1)
    # p=(1,1): six votes of C_S[1] = 10 and three of C_S[1+4] = 50:
    # (210 + 4) // 9 = 23
    assert out[1, 1, 0] == 23
    # p=(0,0): window {(0,0),(1,0),(0,1),(1,1)}: all offset 0 -> C_S[0] = 0
    assert out[0, 0, 0] == 0
    # p=(2,0): n=(1,0),(1,1) vote C_S[2] = 20; n=(2,0),(2,1) vote C_S[6] = 60 -> 40
    assert out[0, 2, 0] == 40


# ------------------------------------------------------------- special cases

def _rand_case(seed, w, h, sw, sh, u16, lut_bits):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, 256, size=(sh, sw, 3), dtype=np.uint8)
    if u16:
        gs = rng.integers(0, 65536, size=(sh, sw, 2), dtype=np.uint16)
        gt = rng.integers(0, 65536, size=(h, w, 2), dtype=np.uint16)
    else:
        gs = rng.integers(0, 256, size=(sh, sw, 2), dtype=np.uint8)
        gt = rng.integers(0, 256, size=(h, w, 2), dtype=np.uint8)
    return src, gs, gt, brute_lut(gs, lut_bits)


@pytest.mark.parametrize("u16", [False, True])
def test_threshold_zero_is_texture_mapping(ora, u16):
    """t = 0 accepts no level, so every pixel takes its own lookup: exactly
    per-pixel texture mapping (Lit Sphere)."""
    lb = 6 if u16 else 8
    src, gs, gt, lut = _rand_case(1, 21, 17, 13, 11, u16, lb)
    jit = workloads.jitter_table(21, 17, 3, 2, 5)
    rgb, chunk, nnf = ora.stylize(src, gs, lut, lb, gt, jit, 3, 2, 0, 0)
    depth = 16 if u16 else 8
    g = gt.astype(np.int64) >> (depth - lb)
    expect = lut[g[:, :, 1] * (1 << lb) + g[:, :, 0]]
    np.testing.assert_array_equal(nnf, expect)
    np.testing.assert_array_equal(rgb, gather_rgb(src, expect))
    lvl, qx, qy = ora.decode_chunk(chunk)
    assert np.all(lvl == 3)
    assert np.all(qx == np.arange(21)[None, :]) and np.all(qy == np.arange(17)[:, None])
    # zero levels gives the same mapping
    rgb0, chunk0, nnf0 = ora.stylize(src, gs, lut, lb, gt, None, 0, 2, 1000, 0)
    np.testing.assert_array_equal(nnf0, expect)
    np.testing.assert_array_equal(rgb0, rgb)


def test_identity_uv_reproduces_source(ora):
    g = workloads.identity_uv_guide_u16(64, 48)
    src = workloads.value_noise_rgb(64, 48, 4)
    lut = ora.lut_build(g, 6)
    for levels, finest, t, r in [(3, 4, 1, 2), (5, 1, 4096, 3), (2, 8, 1 << 30, 1)]:
        jit = workloads.jitter_table(64, 48, levels, finest, 8)
        rgb, chunk, nnf = ora.stylize(src, g, lut, 6, g, jit, levels, finest, t, r)
        np.testing.assert_array_equal(rgb, src)
        x, y = unpack(nnf)
        assert np.all(x == np.arange(64)[None, :]) and np.all(y == np.arange(48)[:, None])


# ------------------------------------------------------------- invariants

def _invariants(ora, src, gs, gt, lut, lb, jit, levels, finest, t, r):
    rgb, chunk, nnf = ora.stylize(src, gs, lut, lb, gt, jit, levels, finest, t, r)
    h, w = gt.shape[:2]
    lvl, qx, qy = ora.decode_chunk(chunk)
    x, y = unpack(nnf)
    sh, sw = gs.shape[:2]
    assert np.all((x < sw) & (y < sh))
    # accepted pixels: error below threshold at their source coordinate
    acc = lvl < levels
    e = ((gt.astype(np.int64) - gs[y, x].astype(np.int64)) ** 2).sum(2)
    assert np.all(e[acc] < t)
    # fallback pixels: own lookup, q = p
    depth = 8 if gs.dtype == np.uint8 else 16
    g = gt.astype(np.int64) >> (depth - lb)
    own = lut[g[:, :, 1] * (1 << lb) + g[:, :, 0]]
    assert np.all(nnf[~acc] == own[~acc])
    xs, ys = np.meshgrid(np.arange(w), np.arange(h))
    assert np.all(qx[~acc] == xs[~acc]) and np.all(qy[~acc] == ys[~acc])
    # a chunk is a pure translation: one offset per (level, seed)
    off = (x - xs) * 100003 + (y - ys)
    keys = chunk[acc].astype(np.int64)
    o = off[acc]
    order = np.argsort(keys, kind="stable")
    ks, os_ = keys[order], o[order]
    same = ks[1:] == ks[:-1]
    assert np.all(os_[1:][same] == os_[:-1][same])
    # accepted seeds are the level's nearest seed and lie on the seed grid
    for i in range(levels):
        sel = np.argwhere(acc & (lvl == i))
        for yy, xx in sel[:: max(1, len(sel) // 50)]:
            found, nqx, nqy = ora.nearest_seed(w, h, levels, finest, jit, i, int(xx), int(yy))
            assert found and (nqx, nqy) == (qx[yy, xx], qy[yy, xx])
    # r = 0 is a plain copy through the NNF
    if r == 0:
        np.testing.assert_array_equal(rgb, gather_rgb(src, nnf))
    return rgb, chunk, nnf


@pytest.mark.parametrize("seed", range(6))
def test_invariants_random(ora, seed):
    rng = np.random.default_rng(seed)
    u16 = bool(seed % 2)
    w, h = int(rng.integers(5, 60)), int(rng.integers(5, 60))
    sw, sh = int(rng.integers(4, 40)), int(rng.integers(4, 40))
    lb = int(rng.integers(4, 9)) if u16 else 8
    # smooth guides so that chunks form
    yy, xx = np.mgrid[0:h, 0:w]
    syy, sxx = np.mgrid[0:sh, 0:sw]
    scale = 65535 if u16 else 255
    dt = np.uint16 if u16 else np.uint8
    gt = np.stack([(xx * scale // w), (yy * scale // h)], 2).astype(dt)
    gs = np.stack([(sxx * scale // sw), (syy * scale // sh)], 2).astype(dt)
    src = rng.integers(0, 256, size=(sh, sw, 3), dtype=np.uint8)
    lut = brute_lut(gs, lb)
    levels = int(rng.integers(1, 5))
    finest = int(2 ** rng.integers(0, 4))
    jit = workloads.jitter_table(w, h, levels, finest, seed)
    t = int(rng.integers(1, 4 * scale))
    r = int(rng.integers(0, 4))
    _invariants(ora, src, gs, gt, lut, lb, jit, levels, finest, t, r)


def test_invariants_workload1(ora):
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    lut = ora.lut_build(st.guide, st.lut_bits)
    p = fr.params
    _invariants(ora, st.rgb, st.guide, fr.guide, lut, st.lut_bits, frame_jitter(fr), p.levels, p.finest,
                p.threshold, p.radius)
    _invariants(ora, st.rgb, st.guide, fr.guide, lut, st.lut_bits, frame_jitter(fr), p.levels, p.finest,
                p.threshold, 0)


def test_threshold_monotone(ora):
    """Raising t never moves a pixel to a finer level: the candidate sequence of
    a pixel does not depend on t, and a level accepted at t stays acceptable
    at any larger t (larger threshold, larger chunks)."""
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    lut = ora.lut_build(st.guide, st.lut_bits)
    p = fr.params
    prev = None
    sizes = []
    for t in (0, 8, 32, 48, 128, 512, 4096):
        nnf, chunk = ora.assign(st.guide, lut, 8, fr.guide, frame_jitter(fr), p.levels, p.finest, t)
        lvl = chunk >> 26
        if prev is not None:
            assert np.all(lvl <= prev)
        prev = lvl
        sizes.append(np.unique(chunk).size)
    # fewer, hence larger, chunks as the threshold grows
    assert all(a >= b for a, b in zip(sizes, sizes[1:]))


def test_row_range_matches_full(ora):
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    lut = ora.lut_build(st.guide, st.lut_bits)
    p = fr.params
    nnf, chunk = ora.assign(st.guide, lut, 8, fr.guide, frame_jitter(fr), p.levels, p.finest,
                            p.threshold)
    nnf2, chunk2 = ora.assign(st.guide, lut, 8, fr.guide, frame_jitter(fr), p.levels, p.finest,
                              p.threshold, rows=(100, 20))
    np.testing.assert_array_equal(nnf2[100:120], nnf[100:120])
    np.testing.assert_array_equal(chunk2[100:120], chunk[100:120])
    out = ora.blend(st.rgb, nnf, p.radius)
    out2 = ora.blend(st.rgb, nnf, p.radius, rows=(37, 5))
    np.testing.assert_array_equal(out2[37:42], out[37:42])


def test_invalid_args(ora):
    g = np.zeros((4, 4, 2), np.uint8)
    with pytest.raises(ValueError):
        ora.lut_build(g, 9)
    with pytest.raises(ValueError):
        ora.assign(g, np.zeros(1 << 16, np.uint32), 8, g, None, 2, 3, 10)  # finest not 2^k
