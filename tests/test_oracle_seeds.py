"""Pins of the oracle's seed hierarchy (Sec. 3.2, SeedPoint and NearestSeed of
Algorithm 2): seed positions against the jitter table read directly,
brute-force nearest seeds on tiny images, and hand-worked tie cases."""
import json
import os

import numpy as np
import pytest

import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def table_offsets(w, h, levels, finest):
    cells = workloads.jitter_cells(w, h, levels, finest)
    offs = np.cumsum([0] + [cx * cy for cx, cy in cells])
    return cells, offs


@pytest.mark.parametrize("w,h,levels,finest", [(37, 21, 3, 2), (64, 64, 4, 4), (5, 40, 2, 8),
                                               (100, 3, 1, 1)])
def test_jitter_len_matches_cells(ora, w, h, levels, finest):
    cells, offs = table_offsets(w, h, levels, finest)
    assert ora.jitter_len(w, h, levels, finest) == offs[-1]
    assert workloads.jitter_table(w, h, levels, finest, 3).size == offs[-1]


def test_spacings(ora):
    assert workloads.level_spacings(3, 8) == [32, 16, 8]
    assert workloads.level_spacings(5, 8) == [128, 64, 32, 16, 8]
    assert workloads.level_spacings(3, 2) == [8, 4, 2]  # the paper's 2^l, l = L..1


@pytest.mark.parametrize("w,h,levels,finest", [(37, 21, 3, 2), (29, 33, 2, 8)])
def test_seed_point_reads_table(ora, w, h, levels, finest):
    jit = workloads.jitter_table(w, h, levels, finest, 17)
    cells, offs = table_offsets(w, h, levels, finest)
    for lvl, sp in enumerate(workloads.level_spacings(levels, finest)):
        cx, cy = cells[lvl]
        tab = jit[offs[lvl]:offs[lvl + 1]].reshape(cy, cx)
        for by in range(-1, cy + 1):
            for bx in range(-1, cx + 1):
                ok, sx, sy = ora.seed_point(w, h, levels, finest, jit, lvl, bx, by)
                if not (0 <= bx < cx and 0 <= by < cy):
                    assert not ok
                    continue
                e = int(tab[by, bx])
                ex, ey = sp * bx + (e & 0xFFFF), sp * by + (e >> 16)
                # each seed stays inside its own cell
                assert sp * bx <= ex < sp * (bx + 1) and sp * by <= ey < sp * (by + 1)
                assert ok == (ex < w and ey < h)
                if ok:
                    assert (sx, sy) == (ex, ey)


def test_no_jitter_seeds_on_corners(ora):
    for lvl, sp in enumerate(workloads.level_spacings(3, 4)):
        for by in range(0, 3):
            for bx in range(0, 3):
                ok, sx, sy = ora.seed_point(40, 40, 3, 4, None, lvl, bx, by)
                assert ok == (sp * bx < 40 and sp * by < 40)
                if ok:
                    assert (sx, sy) == (sp * bx, sp * by)


def test_jitter_uniform_chi2():
    """The generator's jitter is uniform over [0, h)^2 (chi-square, 64 bins)."""
    jit = workloads.jitter_table(4096, 4096, 1, 8, 123)  # 512^2 cells at h = 8
    jx = jit & 0xFFFF
    jy = jit >> 16
    counts = np.bincount((jy * 8 + jx).astype(np.int64), minlength=64)
    exp = jit.size / 64
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 120  # 63 dof; p ~ 1e-5


def brute_nearest(w, h, levels, finest, jit, lvl):
    """All pixels at once: the 9 candidate seeds of each pixel, first strict
    minimum in (dx outer, dy inner) order."""
    cells, offs = table_offsets(w, h, levels, finest)
    sp = workloads.level_spacings(levels, finest)[lvl]
    cx, cy = cells[lvl]
    tab = jit[offs[lvl]:offs[lvl + 1]].reshape(cy, cx).astype(np.int64)
    ys, xs = np.mgrid[0:h, 0:w]
    best = np.full((h, w), np.iinfo(np.int64).max)
    qx = np.full((h, w), -1)
    qy = np.full((h, w), -1)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            bx = xs // sp + dx
            by = ys // sp + dy
            inside = (bx >= 0) & (by >= 0) & (bx < cx) & (by < cy)
            e = np.where(inside, tab[np.clip(by, 0, cy - 1), np.clip(bx, 0, cx - 1)], 0)
            sx = sp * bx + (e & 0xFFFF)
            sy = sp * by + (e >> 16)
            ok = inside & (sx < w) & (sy < h)
            d = np.where(ok, (sx - xs) ** 2 + (sy - ys) ** 2, np.iinfo(np.int64).max)
            take = d < best
            best = np.where(take, d, best)
            qx = np.where(take, sx, qx)
            qy = np.where(take, sy, qy)
    return qx, qy


@pytest.mark.parametrize("w,h,levels,finest,seed", [(23, 19, 3, 2, 1), (40, 12, 2, 8, 2),
                                                    (7, 30, 3, 1, 3), (50, 50, 1, 32, 4)])
def test_nearest_seed_brute(ora, w, h, levels, finest, seed):
    jit = workloads.jitter_table(w, h, levels, finest, seed)
    for lvl in range(levels):
        bqx, bqy = brute_nearest(w, h, levels, finest, jit, lvl)
        for y in range(h):
            for x in range(w):
                found, qx, qy = ora.nearest_seed(w, h, levels, finest, jit, lvl, x, y)
                if bqx[y, x] < 0:
                    assert not found
                else:
                    assert found and (qx, qy) == (bqx[y, x], bqy[y, x])


def test_nearest_seed_hand_ties(ora):
    case = GOLD["nearest_seed_ties"]
    for c in case["cases"]:
        found, qx, qy = ora.nearest_seed(case["w"], case["h"], case["levels"], case["finest"],
                                         None, case["level"], *c["p"])
        assert found and [qx, qy] == c["q"]


def test_nearest_seed_x_outer(ora):
    case = GOLD["nearest_seed_x_outer"]
    jit = np.array([jx | (jy << 16) for jx, jy in case["jitter"]], np.uint32)
    found, qx, qy = ora.nearest_seed(case["w"], case["h"], case["levels"], case["finest"], jit,
                                     0, *case["p"])
    assert found and [qx, qy] == case["q"]


# ---------------------------------------------------------------------------
# RandomJitterTable defined by an integer hash of (cell, log2 h, seed)
# (Algorithm 2, SeedPoint: the paper leaves the table's contents open; this
# reading makes them a function of one 32-bit seed).
# ---------------------------------------------------------------------------

M32 = 0xFFFFFFFF


def py_mix(x):
    """The mixing step written with Python integers."""
    x ^= x >> 16
    x = (x * 0x9E3779B9) & M32
    x ^= x >> 15
    x = (x * 0x6A09E667) & M32
    x ^= x >> 16
    return x


def py_key(seed, lg, bx, by):
    k = py_mix((seed + 0xBB67AE85) & M32)
    k = py_mix(k ^ lg)
    k = py_mix(k ^ (bx & M32))
    return py_mix(k ^ (by & M32))


def np_keys(seed, lg, bx, by):
    """The same hash vectorised over cell arrays (numpy uint32 wraps)."""
    def mix(x):
        x = x ^ (x >> np.uint32(16))
        x = x * np.uint32(0x9E3779B9)
        x = x ^ (x >> np.uint32(15))
        x = x * np.uint32(0x6A09E667)
        return x ^ (x >> np.uint32(16))
    with np.errstate(over="ignore"):
        k = mix(np.full(bx.shape, (seed + 0xBB67AE85) & M32, np.uint32))
        k = mix(k ^ np.uint32(lg))
        k = mix(k ^ bx.astype(np.uint32))
        return mix(k ^ by.astype(np.uint32))


def test_hash_key_definition(ora):
    """The oracle's 32-bit key equals the definition restated with Python
    integers, over random seeds, levels and cells (including the cast of a
    negative cell index to uint32)."""
    rng = np.random.default_rng(5)
    for _ in range(400):
        seed = int(rng.integers(0, 2**32))
        lg = int(rng.integers(0, 14))
        bx, by = int(rng.integers(-2, 5000)), int(rng.integers(-2, 5000))
        assert ora.jitter_hash_key(seed, lg, bx, by) == py_key(seed, lg, bx, by)
    # the seed's additive constant keeps the first mix off its fixed point at 0
    assert ora.jitter_hash_key((0 - 0xBB67AE85) & M32, 0, 0, 0) == py_key((0 - 0xBB67AE85) & M32, 0, 0, 0)
    assert py_mix(0) == 0


@pytest.mark.parametrize("w,h,levels,finest,seed", [(37, 21, 3, 2, 1), (300, 170, 4, 8, 7),
                                                    (64, 64, 1, 1, 3), (1000, 9, 2, 16, 2**32 - 1)])
def test_hash_table_positions(ora, w, h, levels, finest, seed):
    """Every entry of the hash-defined table, recomputed from the definition
    with numpy: jx = k & (h-1), jy = (k >> 16) & (h-1); seed_point with the
    seed gives h*b + j, inside the cell."""
    jit = ora.jitter_hash(w, h, levels, finest, seed)
    cells, offs = table_offsets(w, h, levels, finest)
    assert jit.size == offs[-1]
    for lvl, sp in enumerate(workloads.level_spacings(levels, finest)):
        cx, cy = cells[lvl]
        by, bx = np.mgrid[0:cy, 0:cx]
        k = np_keys(seed, sp.bit_length() - 1, bx.ravel(), by.ravel())
        jx = k & np.uint32(sp - 1)
        jy = (k >> np.uint32(16)) & np.uint32(sp - 1)
        np.testing.assert_array_equal(jit[offs[lvl]:offs[lvl + 1]], jx | (jy << np.uint32(16)))
        for e in range(0, cx * cy, max(1, cx * cy // 25)):
            bxe, bye = e % cx, e // cx
            ok, sx, sy = ora.seed_point(w, h, levels, finest, None, lvl, bxe, bye, seed=seed)
            ex, ey = sp * bxe + int(jx[e]), sp * bye + int(jy[e])
            assert sp * bxe <= ex < sp * (bxe + 1) and sp * bye <= ey < sp * (bye + 1)
            assert ok == (ex < w and ey < h)
            if ok:
                assert (sx, sy) == (ex, ey)


@pytest.mark.parametrize("sp_log2", [3, 6])
def test_hash_uniform_chi2(ora, sp_log2):
    """The hash jitter is uniform over [0, h)^2: chi-square over 64 bins of
    (jx, jy) for 512^2 cells of one level (spacing 8: every value a bin;
    spacing 64: the top 3 bits of each coordinate)."""
    sp = 1 << sp_log2
    jit = ora.jitter_hash(512 * sp, 512 * sp, 1, sp, 11)
    jx, jy = jit & 0xFFFF, jit >> 16
    sh = sp_log2 - 3
    counts = np.bincount(((jy >> sh) * 8 + (jx >> sh)).astype(np.int64), minlength=64)
    exp = jit.size / 64
    assert ((counts - exp) ** 2 / exp).sum() < 120  # 63 dof; p ~ 1e-5


def test_hash_levels_and_seeds_decorrelated(ora):
    """One cell index at two levels, or under two seeds, gets unrelated
    jitter: the low 3 bits of (jx, jy) agree for about 1/64 of the cells."""
    a = ora.jitter_hash(2048, 2048, 2, 8, 1)  # spacings 16, 8
    n16 = (2048 // 16) ** 2
    lv0 = a[:n16] & np.uint32(0x00070007)
    lv1 = a[n16:].reshape(256, 256)[:128, :128].ravel() & np.uint32(0x00070007)
    assert abs((lv0 == lv1).mean() - 1 / 64) < 0.01
    b = ora.jitter_hash(2048, 2048, 2, 8, 2)
    assert abs((a[n16:] == b[n16:]).mean() - 1 / 64) < 0.01  # spacing 8: 64 values
