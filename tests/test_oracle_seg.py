"""Pins of the oracle's segmentation-guide variant (the extra guide of the
paper's results section that keeps chunks inside semantic regions, read as a
hard constraint): its reduction to the plain path, brute-force per-label
lookup tables, a hand-worked case and the label invariants."""
import numpy as np

import oracle
import workloads


def frame_jitter(fr):
    """A workload frame's jitter table: its own, or the one the jitter hash
    of its seed defines."""
    if fr.jitter is not None:
        return fr.jitter
    return oracle.jitter_hash(fr.w, fr.h, fr.params.levels, fr.params.finest, fr.seed)


def brute_lut_labels(gs, labels, label, lut_bits):
    """argmin over source pixels labelled `label` of the squared distance to
    each bin centre, ties to the smallest raster index; None if none."""
    depth = 8 if gs.dtype == np.uint8 else 16
    s = depth - lut_bits
    n = 1 << lut_bits
    c = np.arange(n, dtype=np.int64)
    centre = c if s == 0 else (c << s) + (1 << (s - 1))
    flat = gs.reshape(-1, 2).astype(np.int64)
    idx = np.nonzero(labels.reshape(-1) == label)[0]
    if idx.size == 0:
        return None
    g0, g1 = flat[idx, 0], flat[idx, 1]
    out = np.zeros(n * n, np.uint32)
    sw = gs.shape[1]
    for cy in range(n):
        d = (centre[:, None] - g0[None, :]) ** 2 + (centre[cy] - g1[None, :]) ** 2
        best = idx[np.argmin(d, axis=1)]  # argmin keeps the first (smallest raster index)
        out[cy * n:(cy + 1) * n] = (best % sw).astype(np.uint32) | ((best // sw).astype(np.uint32) << 16)
    return out


def test_one_label_reduces_to_plain_path():
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    p = fr.params
    lut = oracle.lut_build(st.guide, st.lut_bits)
    zs = np.zeros(st.guide.shape[:2], np.uint8)
    zt = np.zeros(fr.guide.shape[:2], np.uint8)
    luts = oracle.lut_build_labels(st.guide, zs, 1, st.lut_bits)
    np.testing.assert_array_equal(luts[0], lut)
    a = oracle.stylize(st.rgb, st.guide, lut, st.lut_bits, fr.guide, frame_jitter(fr), p.levels,
                       p.finest, p.threshold, p.radius)
    b = oracle.stylize_seg(st.rgb, st.guide, zs, luts, 1, st.lut_bits, fr.guide, zt, frame_jitter(fr),
                           p.levels, p.finest, p.threshold, p.radius)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_label_luts_against_brute_force():
    rng = np.random.default_rng(3)
    for dt, bits, shape in [(np.uint8, 8, (13, 17)), (np.uint8, 5, (20, 9)),
                            (np.uint16, 6, (11, 23)), (np.uint16, 9, (7, 7))]:
        hi = 256 if dt == np.uint8 else 65536
        gs = rng.integers(0, hi, size=shape + (2,)).astype(dt)
        labels = rng.integers(0, 3, size=shape).astype(np.uint8)
        labels[labels == 1] = 0  # label 1 absent: it takes the unconstrained table
        luts = oracle.lut_build_labels(gs, labels, 4, bits)
        plain = oracle.lut_build(gs, bits)
        for lab in range(4):
            expect = brute_lut_labels(gs, labels, lab, bits)
            np.testing.assert_array_equal(luts[lab], plain if expect is None else expect,
                                          err_msg=f"{dt} bits={bits} label={lab}")


def test_hand_worked_label_rejection():
    """Source 4x1 with guide (10x, 0) and labels [0,0,1,1]; identity target
    guide with labels [0,1,1,1]; one level of spacing 4 with its seed at
    (0,0), t = 1000.  p=1 would be accepted at offset 0 without labels, but
    its source pixel carries label 0: it falls back to label 1's table, whose
    nearest guide to (10,0) is x=2."""
    gs = np.zeros((1, 4, 2), np.uint8)
    gs[0, :, 0] = [0, 10, 20, 30]
    ls = np.array([[0, 0, 1, 1]], np.uint8)
    gt = gs.copy()
    lt = np.array([[0, 1, 1, 1]], np.uint8)
    rgb = np.zeros((1, 4, 3), np.uint8)
    luts = oracle.lut_build_labels(gs, ls, 2, 8)
    jit = np.zeros(1, np.uint32)
    _, chunk, nnf = oracle.stylize_seg(rgb, gs, ls, luts, 2, 8, gt, lt, jit, 1, 4, 1000, 0)
    assert [int(v & 0xFFFF) for v in nnf[0]] == [0, 2, 2, 3]
    assert [int(c >> 26) for c in chunk[0]] == [0, 1, 0, 0]
    assert int(chunk[0, 1] & 0x1FFF) == 1  # fallback chunk: q = p
    # without labels every pixel takes level 0 at offset 0
    lut = oracle.lut_build(gs, 8)
    _, chunk0, nnf0 = oracle.stylize(rgb, gs, lut, 8, gt, jit, 1, 4, 1000, 0)
    assert [int(v & 0xFFFF) for v in nnf0[0]] == [0, 1, 2, 3]
    assert all(int(c >> 26) == 0 for c in chunk0[0])


def test_label_invariants_on_a_frame():
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    p = fr.params
    ls = workloads.voronoi_labels(st.guide.shape[1], st.guide.shape[0], 3, 12, 5)
    lt = workloads.voronoi_labels(fr.w, fr.h, 3, 20, 6)
    luts = oracle.lut_build_labels(st.guide, ls, 3, st.lut_bits)
    for t in (48, 400, 4000):
        _, chunk, nnf = oracle.stylize_seg(st.rgb, st.guide, ls, luts, 3, st.lut_bits, fr.guide,
                                           lt, frame_jitter(fr), p.levels, p.finest, t, p.radius)
        vx, vy = (nnf & 0xFFFF).astype(np.int64), (nnf >> 16).astype(np.int64)
        got = ls[vy, vx]
        # every pixel, accepted or fallen back, lands on a source pixel of its
        # own label (all three labels occur in the exemplar)
        np.testing.assert_array_equal(got, lt)
        # chunks stay pure translations
        lv, qx, qy = oracle.decode_chunk(chunk)
        acc = lv < p.levels
        key = chunk[acc]
        off = (vx - np.arange(fr.w)[None, :])[acc] * 100000 + (vy - np.arange(fr.h)[:, None])[acc]
        for k in np.unique(key)[:200]:
            assert np.unique(off[key == k]).size == 1
