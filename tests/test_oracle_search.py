"""Pins for the oracle's guides of many channels (formats 3 and 4: 2..8
channels of 8 or 16 bits, each lookup the exact nearest source pixel; the
additional guiding channels of Sec. 3.1, where the paper suggests a search
tree).

The exact lookup against the pinned two- and three-channel tables, a closed
form with ties at 16 bits, the removal of zero-weight channels and channel
permutations; the channel-0 sweep against brute force; the level loop
against the pinned two- and three-channel paths, texture mapping at t = 0, a
translation whose NNF is known in closed form, and the level loop's
invariants."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def _pack(chans, depth):
    return workloads.guide_n(chans, depth)


def _coords(idx, sw):
    idx = np.asarray(idx, np.int64)
    return ((idx % sw) | ((idx // sw) << 16)).astype(np.uint32)


def hand_case():
    case = GOLD["search_weighted_tie"]
    src = np.zeros((case["sh"], case["sw"], 8), np.uint8)
    src.reshape(-1, 8)[:, :case["channels"]] = case["src_texels"]
    q = np.zeros((len(case["queries"]), 8), np.uint8)
    q[:, :case["channels"]] = case["queries"]
    want = np.array([x | (y << 16) for x, y in case["expect_xy"]], np.uint32)
    return case, src, q, want


def test_hand_case_weighted_tie():
    """A hand-worked lookup (tests/golden): weights, an ignored channel, and a
    tie won by the smaller raster index although the other texel lies nearer
    along channel 0."""
    case, src, q, want = hand_case()
    for fn in (oracle.nn_query_n, oracle.nn_sweep_n):
        np.testing.assert_array_equal(fn(src, case["channels"], q, weights=case["weights"]), want)


@pytest.mark.parametrize("depth,channels,want", [
    (8, 2, 4), (8, 4, 4), (8, 5, 8), (8, 8, 8), (16, 2, 4), (16, 3, 8), (16, 4, 8),
    (16, 5, 16), (16, 8, 16), (8, 1, 0), (8, 9, 0), (12, 3, 0)])
def test_texel_bytes(depth, channels, want):
    assert oracle.texel_bytes(depth, channels) == want


def test_two_channels_equal_the_pinned_table():
    """Two 8-bit channels: the exact lookup of every value (c0, c1) is the
    pinned two-channel table's entry at 8 bits per channel, whose bins are
    the values themselves."""
    rng = np.random.default_rng(11)
    two = rng.integers(0, 256, (23, 37, 2)).astype(np.uint8)
    two[rng.random((23, 37)) < 0.3] = (90, 160)  # many duplicates: ties by raster order
    lut = oracle.lut_build(two, 8)
    v = np.arange(1 << 16)
    q = _pack([(v & 255)[None], (v >> 8)[None]], 8).reshape(-1, 4)  # query c = c0 + 256 c1
    np.testing.assert_array_equal(oracle.nn_sweep_n(_pack([two[..., 0], two[..., 1]], 8), 2, q),
                                  lut)


@pytest.mark.parametrize("weights", [None, (3, 1, 7), (0, 5, 1)])
def test_three_channels_equal_the_pinned_table(weights):
    """Three 8-bit channels with weights: sampled values against the pinned
    three-channel table's brute-force entries (8 bits per channel)."""
    rng = np.random.default_rng(12)
    src = np.zeros((19, 21, 4), np.uint8)
    src[..., :3] = rng.integers(0, 256, (19, 21, 3))
    bins = rng.integers(0, 1 << 24, 3000)
    want = oracle.lut_query(src, 8, bins, weights=weights)
    q = _pack([(bins & 255)[None], ((bins >> 8) & 255)[None], (bins >> 16)[None]], 8).reshape(-1, 4)
    got = oracle.nn_query_n(src, 3, q, weights=weights)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("weights", [(1, 1, 1, 1), (3, 5, 1, 2), (7, 1, 7, 1)])
def test_closed_form_with_ties_16bit(weights):
    """Source channels (x, y, x, y) at 16 bits: the lookup of (a, b, c, d)
    separates per axis; x minimises w0 (a - x)^2 + w2 (c - x)^2, i.e. the
    integer nearest (w0 a + w2 c) / (w0 + w2) with a half-way tie to the
    smaller x (the smaller raster index), clamped to the source; y likewise.
    a != c makes ties frequent."""
    sw, sh = 40, 30
    yy, xx = np.mgrid[0:sh, 0:sw]
    src = _pack([xx, yy, xx, yy], 16)
    rng = np.random.default_rng(13)
    n = 4000
    a, c = rng.integers(0, sw + 12, n) - 6, rng.integers(0, sw + 12, n) - 6
    b, d = rng.integers(0, sh + 12, n) - 6, rng.integers(0, sh + 12, n) - 6
    q = _pack([np.clip(a, 0, None)[None], np.clip(b, 0, None)[None],
               np.clip(c, 0, None)[None], np.clip(d, 0, None)[None]], 16).reshape(-1, 4)
    a, b, c, d = (q[:, k].astype(np.int64) for k in range(4))
    w0, w1, w2, w3 = weights

    def nearest(u, v, wu, wv, hi):
        num = 2 * (wu * u + wv * v) - (wu + wv)  # ceil(m - 1/2), m = (wu u + wv v) / (wu + wv)
        den = 2 * (wu + wv)
        return np.clip(-((-num) // den), 0, hi)

    x = nearest(a, c, w0, w2, sw - 1)
    y = nearest(b, d, w1, w3, sh - 1)
    want = (x | (y << 16)).astype(np.uint32)
    np.testing.assert_array_equal(oracle.nn_query_n(src, 4, q, weights=weights), want)
    np.testing.assert_array_equal(oracle.nn_sweep_n(src, 4, q, weights=weights), want)


def _random_guides(rng, depth, channels, sw, sh, nq, levels_of_values):
    top = (1 << depth) - 1
    vals = np.linspace(0, top, levels_of_values).astype(np.int64)
    src = [vals[rng.integers(0, levels_of_values, (sh, sw))] for _ in range(channels)]
    qs = [rng.integers(0, top + 1, (1, nq)) for _ in range(channels)]
    return _pack(src, depth), _pack(qs, depth).reshape(nq, -1), src, qs


@pytest.mark.parametrize("depth", [8, 16])
@pytest.mark.parametrize("channels", [2, 3, 4, 5, 8])
def test_sweep_equals_brute_force(depth, channels):
    rng = np.random.default_rng(depth * 10 + channels)
    src, q, _, _ = _random_guides(rng, depth, channels, 17, 13, 600, 5)
    w = rng.integers(0, 128, channels)
    w[rng.integers(0, channels)] = 0
    for weights in (None, w):
        np.testing.assert_array_equal(oracle.nn_sweep_n(src, channels, q, weights=weights),
                                      oracle.nn_query_n(src, channels, q, weights=weights))


@pytest.mark.parametrize("depth", [8, 16])
def test_all_zero_weights_mean_unit(depth):
    """Weights that are all zero select unit weights (they would otherwise
    make every texel equally near, so the lookup would always be texel 0)."""
    rng = np.random.default_rng(17 + depth)
    src, q, _, _ = _random_guides(rng, depth, 4, 21, 12, 500, 9)
    unit = oracle.nn_query_n(src, 4, q)
    np.testing.assert_array_equal(oracle.nn_query_n(src, 4, q, weights=[0, 0, 0, 0]), unit)
    np.testing.assert_array_equal(oracle.nn_query_n(src, 4, q, weights=[1, 1, 1, 1]), unit)
    assert np.unique(unit).size > 10


@pytest.mark.parametrize("depth", [8, 16])
def test_zero_weight_removes_a_channel(depth):
    """A channel of weight 0 takes no part: the lookups equal those of the
    guide without it (one channel fewer, another texel layout)."""
    rng = np.random.default_rng(21 + depth)
    _, _, src, qs = _random_guides(rng, depth, 5, 23, 11, 800, 7)
    w = np.array([3, 1, 0, 2, 5])
    full = oracle.nn_query_n(_pack(src, depth), 5, _pack(qs, depth).reshape(800, -1), weights=w)
    keep = [0, 1, 3, 4]
    less = oracle.nn_query_n(_pack([src[k] for k in keep], depth), 4,
                             _pack([qs[k] for k in keep], depth).reshape(800, -1),
                             weights=w[keep])
    np.testing.assert_array_equal(full, less)


@pytest.mark.parametrize("depth", [8, 16])
def test_channel_order_does_not_matter(depth):
    rng = np.random.default_rng(31 + depth)
    _, _, src, qs = _random_guides(rng, depth, 6, 19, 14, 700, 6)
    w = rng.integers(1, 128, 6)
    base = oracle.nn_sweep_n(_pack(src, depth), 6, _pack(qs, depth).reshape(700, -1), weights=w)
    perm = rng.permutation(6)
    got = oracle.nn_sweep_n(_pack([src[k] for k in perm], depth), 6,
                            _pack([qs[k] for k in perm], depth).reshape(700, -1), weights=w[perm])
    np.testing.assert_array_equal(got, base)


def test_extra_texel_elements_are_ignored():
    rng = np.random.default_rng(41)
    _, q, src, _ = _random_guides(rng, 8, 5, 15, 9, 300, 9)
    a = _pack(src, 8)
    b = a.copy()
    b[..., 5:] = rng.integers(0, 256, b[..., 5:].shape)
    q2 = q.copy()
    q2[:, 5:] = 255
    np.testing.assert_array_equal(oracle.nn_query_n(a, 5, q), oracle.nn_query_n(b, 5, q2))


# ------------------------------------------------------------- level loop

def test_two_channel_frame_equals_the_pinned_path():
    """Workload 1 (two 8-bit channels) through the many-channel path equals
    the pinned two-channel path with its exact 8-bit table."""
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    p = fr.params
    lut = oracle.lut_build(st.guide, 8)
    want = oracle.stylize(st.rgb, st.guide, lut, 8, fr.guide, None, p.levels, p.finest,
                          p.threshold, p.radius, seed=fr.seed)
    sg = _pack([st.guide[..., 0], st.guide[..., 1]], 8)
    tg = _pack([fr.guide[..., 0], fr.guide[..., 1]], 8)
    got = oracle.stylize_n(st.rgb, sg, 2, tg, None, p.levels, p.finest, p.threshold, p.radius,
                           seed=fr.seed)
    for g, e in zip(got, want):
        np.testing.assert_array_equal(g, e)


@pytest.mark.parametrize("weights", [None, (2, 2, 1)])
def test_three_channel_frame_equals_the_pinned_path(weights):
    """A three-channel frame equals the pinned three-channel path at 8 bits
    per channel.  Its table holds 2^24 bins; only the bins the frame can look
    up (every target pixel's value, which includes every seed's) are filled,
    each from the pinned brute-force query."""
    styles, frames = workloads.config(6, lut_bits=8, w=72, h=56)
    st, fr = styles[0], frames[0]
    rng = np.random.default_rng(51)
    src_rgb = st.rgb[:40, :48].copy()
    sg = np.ascontiguousarray(st.guide[100:140, 200:248])  # 48 x 40 crop of the sphere style
    tg = fr.guide
    p = workloads.Params(levels=3, finest=4, threshold=300, radius=2)
    bins = np.unique(tg[..., 0].astype(np.int64) | (tg[..., 1].astype(np.int64) << 8)
                     | (tg[..., 2].astype(np.int64) << 16))
    lut = np.zeros(1 << 24, np.uint32)
    lut[bins] = oracle.lut_query(sg, 8, bins, weights=weights)
    jit = workloads.jitter_table(fr.w, fr.h, p.levels, p.finest, int(rng.integers(1 << 30)))
    want = oracle.stylize(src_rgb, sg, lut, 8, tg, jit, p.levels, p.finest, p.threshold,
                          p.radius, weights=weights)
    got = oracle.stylize_n(src_rgb, sg, 3, tg, jit, p.levels, p.finest, p.threshold, p.radius,
                           weights=weights)
    for g, e in zip(got, want):
        np.testing.assert_array_equal(g, e)


def test_constant_extra_channel_changes_nothing():
    styles, frames = workloads.config(7, w=96, h=64, size=64)
    st, fr = styles[0], frames[0]
    p = fr.params
    five = oracle.stylize_n(st.rgb, st.guide, 5, fr.guide, None, p.levels, p.finest, p.threshold,
                            p.radius, seed=fr.seed)
    sg, tg = st.guide.copy(), fr.guide.copy()
    sg[..., 5] = 77
    tg[..., 5] = 77
    six = oracle.stylize_n(st.rgb, sg, 6, tg, None, p.levels, p.finest, p.threshold, p.radius,
                           seed=fr.seed)
    for a, b in zip(five, six):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("depth", [8, 16])
def test_threshold_zero_is_texture_mapping(depth):
    styles, frames = workloads.config(7, depth=depth, w=80, h=48, size=48)
    st, fr = styles[0], frames[0]
    ch = 5 if depth == 8 else 4
    p = fr.params
    nnf, chunk = oracle.assign_n(st.guide, ch, fr.guide, None, p.levels, p.finest, 0,
                                 seed=fr.seed)
    want = oracle.nn_query_n(st.guide, ch, fr.guide.reshape(fr.h * fr.w, -1)).reshape(fr.h, fr.w)
    np.testing.assert_array_equal(nnf, want)
    lvl, qx, qy = oracle.decode_chunk(chunk)
    yy, xx = np.mgrid[0:fr.h, 0:fr.w]
    assert np.all(lvl == p.levels) and np.all(qx == xx) and np.all(qy == yy)


def test_translation_closed_form_16bit():
    """Source channels (x, y, 2x, 3y) at 16 bits and a target holding the same
    function at p + d: every exact lookup of a target value is p + d, so
    every seed's chunk is that translation with guide error 0, and every
    pixel takes level 0 (t = 1) from its level-0 NearestSeed."""
    sw, sh, w, h, dx, dy = 90, 70, 64, 48, 13, 9
    yy, xx = np.mgrid[0:sh, 0:sw]
    src = _pack([xx, yy, 2 * xx, 3 * yy], 16)
    ty, tx = np.mgrid[0:h, 0:w]
    tgt = _pack([tx + dx, ty + dy, 2 * (tx + dx), 3 * (ty + dy)], 16)
    levels, finest = 3, 4
    jit = workloads.jitter_table(w, h, levels, finest, 61)
    nnf, chunk = oracle.assign_n(src, 4, tgt, jit, levels, finest, 1)
    np.testing.assert_array_equal(nnf, ((tx + dx) | ((ty + dy) << 16)).astype(np.uint32))
    lvl, qx, qy = oracle.decode_chunk(chunk)
    assert np.all(lvl == 0)
    for (py, px) in [(0, 0), (47, 63), (20, 31), (5, 60)]:
        found, sx, sy = oracle.nearest_seed(w, h, levels, finest, jit, 0, px, py)
        assert found and (qx[py, px], qy[py, px]) == (sx, sy)


@pytest.mark.parametrize("depth", [8, 16])
def test_level_loop_invariants(depth):
    """Accepted pixels have weighted error below t (recomputed with numpy
    from the NNF); every chunk is one translation; fallback pixels hold their
    own lookup."""
    styles, frames = workloads.config(7, depth=depth, w=120, h=72, size=64)
    st, fr = styles[0], frames[0]
    ch = 5 if depth == 8 else 4
    p = fr.params
    w8 = np.array([2, 3, 1, 1, 2][:ch])
    nnf, chunk = oracle.assign_n(st.guide, ch, fr.guide, None, p.levels, p.finest, p.threshold,
                                 weights=w8, seed=fr.seed)
    lvl, qx, qy = oracle.decode_chunk(chunk)
    sx, sy = (nnf & 0xFFFF).astype(np.int64), (nnf >> 16).astype(np.int64)
    assert np.all(sx < st.sw) and np.all(sy < st.sh)
    src_vals = st.guide[sy, sx][..., :ch].astype(np.int64)
    tgt_vals = fr.guide[..., :ch].astype(np.int64)
    err = ((src_vals - tgt_vals) ** 2 * w8).sum(axis=2)
    acc = lvl < p.levels
    assert acc.any() and (~acc).any()
    assert np.all(err[acc] < p.threshold)
    yy, xx = np.mgrid[0:fr.h, 0:fr.w]
    key = chunk[acc]
    ox, oy = (sx - xx)[acc], (sy - yy)[acc]
    for k in np.unique(key)[:400]:
        sel = key == k
        assert np.unique(ox[sel]).size == 1 and np.unique(oy[sel]).size == 1
    fb = ~acc
    own = oracle.nn_query_n(st.guide, ch, fr.guide[fb], weights=w8)
    np.testing.assert_array_equal(nnf[fb], own)
