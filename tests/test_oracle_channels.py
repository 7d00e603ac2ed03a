"""Pins for the oracle's three-channel guides (additional guiding channels,
Sec. 3.1; format 2: three uint8 channels in four bytes per pixel).

The lookup table against an independent vectorised argmin and a closed form;
the reduction to the pinned two-channel path when the third channel is
constant; invariants of the level loop with the three-channel error."""
import numpy as np
import pytest

import oracle
import workloads


def _numpy_lut3(src, lut_bits):
    """argmin over pixels of the squared distance from every bin centre,
    first (smallest raster index) minimum -- written out with numpy."""
    n = 1 << lut_bits
    s = 8 - lut_bits
    cen = (np.arange(n) << s) + ((1 << (s - 1)) if s else 0)
    c0, c1, c2 = np.meshgrid(cen, cen, cen, indexing="ij")  # c0 slowest here
    # bin index c = b0 + b1 n + b2 n^2: order the centres by that index
    q = np.stack([c0.ravel(), c1.ravel(), c2.ravel()], axis=1)  # row = b0 * n^2 + b1 * n + b2
    g = src[..., :3].reshape(-1, 3).astype(np.int64)
    d = ((q[:, None, :] - g[None, :, :]) ** 2).sum(axis=2)
    best = np.argmin(d, axis=1)
    sw = src.shape[1]
    coords = (best % sw) | ((best // sw) << 16)
    out = np.zeros(n ** 3, np.uint32)
    b0, b1, b2 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    out[(b0 + b1 * n + b2 * n * n).ravel()] = coords
    return out


@pytest.mark.parametrize("lut_bits,levels_of_values", [(1, 4), (3, 3), (4, 256)])
def test_lut3_matches_vectorised_argmin(lut_bits, levels_of_values):
    rng = np.random.default_rng(lut_bits * 7 + levels_of_values)
    src = np.zeros((12, 17, 4), np.uint8)
    vals = np.linspace(0, 255, levels_of_values).astype(np.uint8)
    src[..., :3] = vals[rng.integers(0, levels_of_values, (12, 17, 3))]  # many ties
    src[..., 3] = rng.integers(0, 256, (12, 17))  # byte 3 must be ignored
    np.testing.assert_array_equal(oracle.lut_build(src, lut_bits), _numpy_lut3(src, lut_bits))


def test_lut3_closed_form_full_coverage():
    """A source holding every bin centre exactly once (lut_bits 3: centres
    32 c + 16) maps every bin to the pixel holding its centre."""
    n = 8
    rng = np.random.default_rng(5)
    order = rng.permutation(n ** 3)
    src = np.zeros((16, 32, 4), np.uint8)
    flat = src.reshape(-1, 4)
    for pos, c in enumerate(order):
        b0, b1, b2 = c % n, (c // n) % n, c // (n * n)
        flat[pos, :3] = (32 * b0 + 16, 32 * b1 + 16, 32 * b2 + 16)
    lut = oracle.lut_build(src, 3)
    where = np.empty(n ** 3, np.int64)
    where[order] = np.arange(n ** 3)
    want = ((where % 32) | ((where // 32) << 16)).astype(np.uint32)
    np.testing.assert_array_equal(lut, want)


def test_lut3_with_constant_third_channel_reduces_to_two_channels():
    g2 = workloads.sphere_guide_u8(64)
    g3 = workloads.guide_u8x3(g2, np.zeros((64, 64), np.uint8))
    for bits in (2, 5):
        n = 1 << bits
        l2 = oracle.lut_build(g2, bits)
        l3 = oracle.lut_build(g3, bits).reshape(n, n * n)  # [c2][c1 c0]
        for c2 in range(n):
            np.testing.assert_array_equal(l3[c2], l2)


def test_lut_query_equals_built_entries():
    rng = np.random.default_rng(9)
    st = workloads.config(6, lut_bits=4, w=64, h=64)[0][0]
    src = st.guide[:48, :40]
    lut = oracle.lut_build(src, 4)
    bins = rng.integers(0, lut.size, 300)
    np.testing.assert_array_equal(oracle.lut_query(src, 4, bins), lut[bins])
    g2 = workloads.sphere_guide_u8(40)
    lut2 = oracle.lut_build(g2, 6)
    bins = rng.integers(0, lut2.size, 300)
    np.testing.assert_array_equal(oracle.lut_query(g2, 6, bins), lut2[bins])


def test_stylize_with_zero_third_channel_equals_two_channel_path():
    rgb = workloads.value_noise_rgb(96, 96, 3)
    g2s = workloads.sphere_guide_u8(96)
    g2t = workloads.bump_guide_u8(120, 80, 5, 4)
    g3s = workloads.guide_u8x3(g2s, np.zeros((96, 96), np.uint8))
    g3t = workloads.guide_u8x3(g2t, np.zeros((80, 120), np.uint8))
    jit = workloads.jitter_table(120, 80, 3, 4, 8)
    bits = 5
    l2, l3 = oracle.lut_build(g2s, bits), oracle.lut_build(g3s, bits)
    for t, r in ((0, 1), (40, 2), (400, 0)):
        a = oracle.stylize(rgb, g2s, l2, bits, g2t, jit, 3, 4, t, r)
        b = oracle.stylize(rgb, g3s, l3, bits, g3t, jit, 3, 4, t, r)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_three_channel_level_loop_invariants():
    st = workloads.config(6, lut_bits=4, w=96, h=72)[0][0]
    src = st.guide[:80, :80]
    rgb = st.rgb[:80, :80]
    tgt = workloads.appearance_target(96, 72, 5, 31)
    p = workloads.APPEARANCE_PARAMS
    jit = workloads.jitter_table(96, 72, p.levels, p.finest, 32)
    bits = 4
    lut = oracle.lut_build(src, bits)
    prev = None
    for t in (0, 30, 64, 300):
        out, chunk, nnf = oracle.stylize(rgb, src, lut, bits, tgt, jit, p.levels, p.finest, t,
                                         p.radius)
        lv = chunk >> 26
        vx, vy = nnf & 0xFFFF, nnf >> 16
        acc = lv < p.levels
        # accepted pixels: the three-channel error at the transferred pixel is below t
        d = tgt[..., :3].astype(np.int64) - src[vy, vx, :3].astype(np.int64)
        e = (d * d).sum(axis=2)
        assert np.all(e[acc] < t)
        # fallback pixels take their own lookup
        q = tgt[..., :3].astype(np.int64) >> (8 - bits)
        own = lut[q[..., 0] + (q[..., 1] << bits) + (q[..., 2] << (2 * bits))]
        np.testing.assert_array_equal(nnf[~acc], own[~acc])
        if t == 0:
            assert not acc.any()
        if prev is not None:  # a larger threshold never picks a finer level
            assert np.all(lv <= prev)
        prev = lv


def test_label_tables_three_channels_one_label_is_the_plain_table():
    st = workloads.config(6, lut_bits=3, w=64, h=64)[0][0]
    src = st.guide[:40, :48]
    lab = np.zeros((40, 48), np.uint8)
    luts = oracle.lut_build_labels(src, lab, 2, 3)
    plain = oracle.lut_build(src, 3)
    np.testing.assert_array_equal(luts[0], plain)
    np.testing.assert_array_equal(luts[1], plain)  # absent label: the plain table


def test_third_channel_decides_acceptance():
    """Every source pixel has appearance 128 and every target pixel 0 or 255,
    so each candidate's error is at least 127^2 from the third channel alone:
    below that threshold no level can accept, above it the normals decide."""
    g2s = workloads.sphere_guide_u8(64)
    g2t = workloads.bump_guide_u8(72, 56, 4, 12)
    src = workloads.guide_u8x3(g2s, np.full((64, 64), 128, np.uint8))
    yy, xx = np.mgrid[0:56, 0:72]
    tgt = workloads.guide_u8x3(g2t, (((xx >> 2) + (yy >> 2)) % 2 * 255).astype(np.uint8))
    rgb = workloads.value_noise_rgb(64, 64, 2)
    jit = workloads.jitter_table(72, 56, 3, 4, 13)
    lut = oracle.lut_build(src, 4)
    _, chunk, _ = oracle.stylize(rgb, src, lut, 4, tgt, jit, 3, 4, 127 * 127, 1)
    assert np.all((chunk >> 26) == 3)
    _, chunk, _ = oracle.stylize(rgb, src, lut, 4, tgt, jit, 3, 4, 127 * 127 + 400, 1)
    assert np.any((chunk >> 26) < 3)


# --------------------------------------------------------- channel weights

def _numpy_lut3_weighted(src, lut_bits, w):
    n = 1 << lut_bits
    s = 8 - lut_bits
    cen = (np.arange(n) << s) + ((1 << (s - 1)) if s else 0)
    b0, b1, b2 = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    q = np.stack([cen[b0.ravel()], cen[b1.ravel()], cen[b2.ravel()]], axis=1)
    g = src[..., :3].reshape(-1, 3).astype(np.int64)
    d = (np.asarray(w, np.int64)[None, None, :] * (q[:, None, :] - g[None, :, :]) ** 2).sum(axis=2)
    best = np.argmin(d, axis=1)
    sw = src.shape[1]
    out = np.zeros(n ** 3, np.uint32)
    out[(b0 + b1 * n + b2 * n * n).ravel()] = (best % sw) | ((best // sw) << 16)
    return out


@pytest.mark.parametrize("weights", [(1, 1, 1), (3, 1, 7), (0, 2, 5), (127, 0, 1)])
def test_weighted_lut3_matches_vectorised_argmin(weights):
    rng = np.random.default_rng(sum(weights))
    src = np.zeros((10, 13, 4), np.uint8)
    src[..., :3] = np.linspace(0, 255, 5).astype(np.uint8)[rng.integers(0, 5, (10, 13, 3))]
    src[..., 3] = rng.integers(0, 256, (10, 13))
    for bits in (2, 4):
        np.testing.assert_array_equal(oracle.lut_build(src, bits, weights),
                                      _numpy_lut3_weighted(src, bits, weights))
        bins = rng.integers(0, 1 << (3 * bits), 50)
        np.testing.assert_array_equal(oracle.lut_query(src, bits, bins, weights),
                                      _numpy_lut3_weighted(src, bits, weights)[bins])


def test_zero_weight_drops_the_channel():
    """Weights (1, 1, 0) make a three-channel guide behave exactly as its
    first two channels (table and frames), whatever the third channel holds."""
    rgb = workloads.value_noise_rgb(80, 80, 7)
    g2s = workloads.sphere_guide_u8(80)
    g2t = workloads.bump_guide_u8(100, 70, 5, 8)
    g3s = workloads.guide_u8x3(g2s, workloads.appearance_u8(rgb, 3))
    g3t = workloads.appearance_target(100, 70, 5, 9)
    g3t[..., :2] = g2t
    jit = workloads.jitter_table(100, 70, 3, 4, 10)
    bits = 4
    w = (1, 1, 0)
    l2 = oracle.lut_build(g2s, bits)
    l3 = oracle.lut_build(g3s, bits, w).reshape(1 << bits, -1)
    for c2 in range(1 << bits):
        np.testing.assert_array_equal(l3[c2], l2)
    for t in (0, 40, 300):
        a = oracle.stylize(rgb, g2s, l2, bits, g2t, jit, 3, 4, t, 2)
        b = oracle.stylize(rgb, g3s, l3.ravel(), bits, g3t, jit, 3, 4, t, 2, weights=w)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_uniform_weight_scales_the_threshold():
    """Weights (k, k, k) with threshold k t equal unit weights with t."""
    st = workloads.config(6, lut_bits=4, w=64, h=64)[0][0]
    src, rgb = st.guide[:72, :72], st.rgb[:72, :72]
    tgt = workloads.appearance_target(90, 60, 4, 15)
    jit = workloads.jitter_table(90, 60, 3, 8, 16)
    l1 = oracle.lut_build(src, 4)
    l3 = oracle.lut_build(src, 4, (3, 3, 3))
    np.testing.assert_array_equal(l1, l3)
    for t in (50, 200):
        a = oracle.stylize(rgb, src, l1, 4, tgt, jit, 3, 8, t, 1)
        b = oracle.stylize(rgb, src, l3, 4, tgt, jit, 3, 8, 3 * t, 1, weights=(3, 3, 3))
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


def test_weights_are_validated():
    g3 = workloads.guide_u8x3(workloads.sphere_guide_u8(16), np.zeros((16, 16), np.uint8))
    with pytest.raises(ValueError):
        oracle.lut_build(g3, 3, (1, 128, 1))
    with pytest.raises(ValueError):
        oracle.lut_build(workloads.sphere_guide_u8(16), 3, (2, 1, 1))  # two channels: unit only
    np.testing.assert_array_equal(oracle.lut_build(workloads.sphere_guide_u8(16), 3, (1, 1, 1)),
                                  oracle.lut_build(workloads.sphere_guide_u8(16), 3))


@pytest.mark.parametrize("fmt,case", [(2, 0), (2, 1), (2, 2), (0, 0), (0, 1), (1, 0), (1, 1)])
def test_lut_query_sweep_equals_definition(fmt, case):
    """The channel-0 sweep returns exactly the brute-force argmin (the
    definition, lut_query) on small random sources with many ties (few
    distinct values), for every guide format, with unit and with skewed
    channel weights (channel-0 weight 0 turns the stopping bound off)."""
    rng = np.random.default_rng(100 * fmt + case)
    sh, sw = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    if fmt == 2:
        src = np.zeros((sh, sw, 4), np.uint8)
        src[..., :3] = rng.choice(np.array([0, 7, 100, 101, 255], np.uint8), (sh, sw, 3))
        src[..., 3] = rng.integers(0, 256, (sh, sw))
        bits = int(rng.integers(1, 9))
        nb = 1 << (3 * bits)
        weights = [None, (0, 3, 1), (127, 1, 9)][case]
    elif fmt == 0:
        src = rng.choice(np.array([3, 4, 200, 201], np.uint8), (sh, sw, 2))
        bits = int(rng.integers(1, 9))
        nb = 1 << (2 * bits)
        weights = None
    else:
        src = rng.choice(np.array([0, 1000, 1001, 65535], np.uint16), (sh, sw, 2))
        bits = int(rng.integers(1, 13))
        nb = 1 << (2 * bits)
        weights = None
    bins = rng.integers(0, nb, size=min(nb, 600))
    np.testing.assert_array_equal(oracle.lut_query_sweep(src, bits, bins, weights=weights),
                                  oracle.lut_query(src, bits, bins, weights=weights))


def test_lut_query_sweep_on_appearance_style():
    """The 512^2 appearance style at 8 bits (the table of the three-channel
    1080p workload): sampled bins, sweep against the definition."""
    st = workloads.config(6, w=64, h=64)[0][0]
    rng = np.random.default_rng(3)
    bins = rng.integers(0, 1 << 24, size=300)
    np.testing.assert_array_equal(oracle.lut_query_sweep(st.guide, 8, bins),
                                  oracle.lut_query(st.guide, 8, bins))
