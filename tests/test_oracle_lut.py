"""Pins of the oracle's lookup table (Sec. 3.1) against brute force and closed
forms.  The oracle uses a ring search; these tests compute the plain
definition (argmin over every source pixel, first index on ties) directly."""
import json
import os

import numpy as np
import pytest

import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def brute_lut(guide: np.ndarray, lut_bits: int, bins=None) -> np.ndarray:
    """argmin_u |centre(c) - G_S[u]|^2 by exhaustive search; np.argmin keeps the
    first (smallest raster index) minimum."""
    depth = 8 if guide.dtype == np.uint8 else 16
    s = depth - lut_bits
    n = 1 << lut_bits
    g = guide.reshape(-1, 2).astype(np.int64)
    sw = guide.shape[1]
    if bins is None:
        bins = np.arange(n * n)
    bins = np.asarray(bins, dtype=np.int64)
    cx, cy = bins % n, bins // n
    if s == 0:
        qx, qy = cx, cy
    else:
        qx, qy = (cx << s) + (1 << (s - 1)), (cy << s) + (1 << (s - 1))
    out = np.empty(bins.size, np.uint32)
    step = max(1, (1 << 24) // max(g.shape[0], 1))
    for a in range(0, bins.size, step):
        b = slice(a, a + step)
        d = (qx[b, None] - g[None, :, 0]) ** 2 + (qy[b, None] - g[None, :, 1]) ** 2
        i = np.argmin(d, axis=1)
        out[b] = (i % sw).astype(np.uint32) | ((i // sw).astype(np.uint32) << 16)
    return out


@pytest.mark.parametrize("size", [(8, 8), (32, 32), (13, 7)])
def test_lut_u8_random_small(ora, size):
    rng = np.random.default_rng(11 + size[0])
    g = rng.integers(0, 256, size=(size[1], size[0], 2), dtype=np.uint8)
    np.testing.assert_array_equal(ora.lut_build(g, 8), brute_lut(g, 8))


def test_lut_u8_duplicates_and_ties(ora):
    # few distinct values, many duplicates: every bin ties between pixels
    rng = np.random.default_rng(5)
    vals = np.array([[0, 0], [255, 255], [128, 0], [0, 128], [64, 192]], np.uint8)
    g = vals[rng.integers(0, len(vals), size=24 * 20)].reshape(20, 24, 2)
    np.testing.assert_array_equal(ora.lut_build(g, 8), brute_lut(g, 8))


def test_lut_u8_sphere64(ora):
    g = workloads.sphere_guide_u8(64)
    np.testing.assert_array_equal(ora.lut_build(g, 8), brute_lut(g, 8))


@pytest.mark.parametrize("lut_bits", [1, 3, 6, 8])
def test_lut_u16_random(ora, lut_bits):
    rng = np.random.default_rng(100 + lut_bits)
    g = rng.integers(0, 65536, size=(17, 23, 2), dtype=np.uint16)
    np.testing.assert_array_equal(ora.lut_build(g, lut_bits), brute_lut(g, lut_bits))


def test_lut_u16_clustered(ora):
    # all guides packed into one corner: most bins search far outward
    rng = np.random.default_rng(7)
    g = rng.integers(0, 3000, size=(16, 16, 2), dtype=np.uint16)
    np.testing.assert_array_equal(ora.lut_build(g, 7), brute_lut(g, 7))


@pytest.mark.parametrize("lut_bits", [6, 7])
def test_lut_u8_coarse_bins(ora, lut_bits):
    g = workloads.sphere_guide_u8(48)
    np.testing.assert_array_equal(ora.lut_build(g, lut_bits), brute_lut(g, lut_bits))


def test_lut_sampled_bins_512(ora):
    """4096 random bins of full-size 512x512 exemplars (sphere and UV)."""
    rng = np.random.default_rng(3)
    g = workloads.sphere_guide_u8(512)
    lut = ora.lut_build(g, 8)
    bins = rng.integers(0, 1 << 16, size=4096)
    np.testing.assert_array_equal(lut[bins], brute_lut(g, 8, bins))
    gu = workloads.identity_uv_guide_u16(512, 512)
    gu[100:140, 30:90] = rng.integers(0, 65536, size=(40, 60, 2))  # break the closed form
    lutu = ora.lut_build(gu, 9)
    bins = rng.integers(0, 1 << 18, size=4096)
    np.testing.assert_array_equal(lutu[bins], brute_lut(gu, 9, bins))


@pytest.mark.parametrize("side,lut_bits", [(64, 6), (512, 9), (2048, 11)])
def test_lut_identity_uv_closed_form(ora, side, lut_bits):
    """Texel-centre UV guides at lut_bits = log2(side): bin c's centre is
    exactly texel c's guide, so LUT[c] = c."""
    g = workloads.identity_uv_guide_u16(side, side)
    lut = ora.lut_build(g, lut_bits)
    c = np.arange(side, dtype=np.uint32)
    expect = (c[None, :] | (c[:, None] << np.uint32(16))).ravel()
    np.testing.assert_array_equal(lut, expect)


def test_lut_tie_across_rings(ora):
    case = GOLD["lut_tie_across_rings"]
    g = np.array(case["src_guide"], np.uint8).reshape(1, -1, 2)
    lut = ora.lut_build(g, 8)
    bx, by = case["bin"]
    ex, ey = case["lut"]
    assert lut[by * 256 + bx] == ex | (ey << 16)
    np.testing.assert_array_equal(lut, brute_lut(g, 8))


def test_lut_invariant_nearest(ora):
    """|centre(c) - G_S[LUT[c]]|^2 <= |centre(c) - G_S[u]|^2 for all u."""
    rng = np.random.default_rng(9)
    g = rng.integers(0, 65536, size=(9, 11, 2), dtype=np.uint16)
    lut = ora.lut_build(g, 5)
    n = 32
    c = np.arange(n * n)
    q = np.stack([(c % n) * 2048 + 1024, (c // n) * 2048 + 1024], 1)
    src = g.reshape(-1, 2).astype(np.int64)
    chosen = src[(lut >> 16).astype(np.int64) * 11 + (lut & 0xFFFF)]
    dch = ((q - chosen) ** 2).sum(1)
    dall = ((q[:, None, :] - src[None, :, :]) ** 2).sum(2)
    assert np.all(dch <= dall.min(1))
