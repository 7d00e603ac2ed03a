"""The animation extension (Sec. 3.3) on the oracle: a sequence is frames
of the plain path, each with the jitter table of a per-frame seed schedule.
Pins: seeds that do not move leave a static target unchanged; with
threshold 0 no seed is ever accepted, so the result does not depend on the
seeds; re-drawn seeds change more pixels under a larger threshold (larger
chunks move as a whole); the change counts equal a brute-force count."""
import numpy as np

import oracle
import workloads

W = H = 128


def _seq(t, hold, nframes=4, drift=1.5):
    styles, frames = workloads.config(1)
    st = styles[0]
    p = frames[0].params
    guides = workloads.animated_bump_guides(W, H, 6, nframes, drift, 21)
    jits = workloads.jitter_schedule(W, H, p.levels, p.finest, nframes, hold, 31)
    lut = oracle.lut_build(st.guide, st.lut_bits)
    return [oracle.stylize(st.rgb, st.guide, lut, st.lut_bits, g, j, p.levels, p.finest, t,
                           p.radius) for g, j in zip(guides, jits)], p


def _src_changed(seq):
    """Mean fraction of pixels whose source coordinate changes between
    consecutive frames."""
    return float(np.mean([oracle.frame_change(a[1], b[1], a[2], b[2])[1] / (W * H)
                          for a, b in zip(seq, seq[1:])]))


def test_generators_are_deterministic_and_shaped():
    a = workloads.animated_bump_guides(40, 24, 3, 3, 2.0, 5)
    b = workloads.animated_bump_guides(40, 24, 3, 3, 2.0, 5)
    assert len(a) == 3 and all(x.shape == (24, 40, 2) and x.dtype == np.uint8 for x in a)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[0], a[2])  # the bumps move
    s = workloads.animated_bump_guides(40, 24, 3, 3, 0.0, 5)
    assert all(np.array_equal(s[0], x) for x in s)  # no drift: a static target
    js = workloads.jitter_schedule(40, 24, 3, 2, 6, 2, 9)
    assert np.array_equal(js[0], js[1]) and np.array_equal(js[2], js[3])
    assert not np.array_equal(js[1], js[2])
    assert len(js[0]) == oracle.jitter_len(40, 24, 3, 2)


def test_frame_change_counts_by_brute_force():
    rng = np.random.default_rng(3)
    for n in (0, 1, 7, 97):
        a = rng.integers(0, 4, n).astype(np.uint32)
        b = rng.integers(0, 4, n).astype(np.uint32)
        c = rng.integers(0, 3, n).astype(np.uint32)
        d = rng.integers(0, 3, n).astype(np.uint32)
        code = sum(1 for i in range(n) if int(a[i]) != int(b[i]))
        src = sum(1 for i in range(n) if int(c[i]) != int(d[i]))
        assert oracle.frame_change(a, b, c, d) == (code, src)
        assert oracle.frame_change(a, b) == (code, 0)
        assert oracle.frame_change(a, a, c, c) == (0, 0)


def test_static_target_with_held_seeds_does_not_change():
    seq, _ = _seq(48, hold=100, drift=0.0)
    for a, b in zip(seq, seq[1:]):
        assert oracle.frame_change(a[1], b[1], a[2], b[2]) == (0, 0)
        assert np.array_equal(a[0], b[0])


def test_threshold_zero_ignores_the_seeds():
    seq, p = _seq(0, hold=1, drift=0.0)
    assert _src_changed(seq) == 0.0
    for x in seq:
        assert np.all((x[1] >> 26) == p.levels)  # every pixel fell back


def test_moving_target_with_held_seeds_changes_less_than_redrawn_seeds():
    held, _ = _seq(400, hold=100)
    redrawn, _ = _seq(400, hold=1)
    assert _src_changed(redrawn) > _src_changed(held)


def test_redrawn_seeds_change_more_pixels_with_larger_threshold():
    small = _src_changed(_seq(16, hold=1, drift=0.0)[0])
    large = _src_changed(_seq(2000, hold=1, drift=0.0)[0])
    assert large > small + 0.05, (small, large)
