"""Segmentation guide on the GPU against the oracle, bit for bit
(tolerance 0): per-label lookup tables, frames of both guide formats under
every kernel choice, random small cases, the one-label reduction, label
values past the last table, and batches mixing labelled and plain frames."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def sb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1807_03249_amd as m

    m.lib()
    return m


def check(sb, st, ls, nlabels, tgt_guide, lt, jit, levels, finest, t, r, name, tunes=(None,),
          style=None, seed=None):
    """GPU frame with labels against the oracle; the seeds' jitter is the
    table ``jit``, else the hash of ``seed``."""
    import torch

    luts = oracle.lut_build_labels(st.guide, ls, nlabels, st.lut_bits)
    e_rgb, e_chunk, e_nnf = oracle.stylize_seg(st.rgb, st.guide, ls, luts, nlabels, st.lut_bits,
                                               tgt_guide, lt, jit, levels, finest, t, r,
                                               seed=seed)
    if style is None:
        style = sb.Style(st.rgb, st.guide, st.lut_bits, labels=ls, nlabels=nlabels)
    np.testing.assert_array_equal(style.label_luts.cpu().numpy().view(np.uint32), luts,
                                  err_msg=f"{name}: label tables")
    for tune in tunes:
        say(f"{name} {tgt_guide.shape[1]}x{tgt_guide.shape[0]} L={levels} t={t} r={r} tune={tune}")
        rgb, chunk, nnf = sb.stylize(style, tgt_guide, jit, sb.params(levels, finest, t, r, seed),
                                     want_nnf=True, tune=tune, tgt_labels=lt)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(chunk.cpu().numpy().view(np.uint32), e_chunk,
                                      err_msg=f"{name} {tune}: chunk")
        np.testing.assert_array_equal(nnf.cpu().numpy().view(np.uint32), e_nnf,
                                      err_msg=f"{name} {tune}: nnf")
        np.testing.assert_array_equal(rgb.cpu().numpy(), e_rgb, err_msg=f"{name} {tune}: rgb")
    return style


def test_normal_frame_all_tunes(sb):
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    p = fr.params
    ls = workloads.voronoi_labels(st.guide.shape[1], st.guide.shape[0], 3, 12, 5)
    lt = workloads.voronoi_labels(fr.w, fr.h, 3, 20, 6)
    style = None
    for t in (p.threshold, 600):
        style = check(sb, st, ls, 3, fr.guide, lt, fr.jitter, p.levels, p.finest, t, p.radius,
                      "normal 256", tunes=[None] + list(sb.TUNES), style=style, seed=fr.seed)


def test_uv_frame_with_absent_label(sb):
    """16-bit guides; label 2 occurs in the target but not in the exemplar:
    its pixels use the unconstrained table and can only fall back."""
    styles, frames = workloads.config(4, frames=2)
    f = frames[1]  # the UV-guided one
    st = styles[f.style]
    h, w = min(f.h, 300), min(f.w, 400)
    g = np.ascontiguousarray(f.guide[:h, :w])
    ls = workloads.voronoi_labels(st.guide.shape[1], st.guide.shape[0], 2, 9, 7)
    lt = workloads.voronoi_labels(w, h, 3, 15, 8)
    p = f.params
    jit = workloads.jitter_table(w, h, p.levels, p.finest, 9)
    check(sb, st, ls, 3, g, lt, jit, p.levels, p.finest, p.threshold, p.radius, "uv absent label",
          tunes=[None, (2, 16, 4, 1), (4, 8, 2, 2)])


@pytest.mark.parametrize("seed", range(8))
def test_random_small(sb, seed):
    rng = np.random.default_rng(100 + seed)
    u16 = seed % 2 == 1
    w, h = int(rng.integers(1, 200)), int(rng.integers(1, 150))
    sw, sh = int(rng.integers(2, 90)), int(rng.integers(2, 90))
    bits = int(rng.integers(3, 10)) if u16 else int(rng.integers(5, 9))
    scale = 65535 if u16 else 255
    dt = np.uint16 if u16 else np.uint8
    yy, xx = np.mgrid[0:h, 0:w]
    noise = rng.integers(-scale // 40, scale // 40 + 1, size=(h, w, 2))
    gt = np.clip(np.stack([xx * scale // max(w, 1), yy * scale // max(h, 1)], 2) + noise, 0,
                 scale).astype(dt)
    syy, sxx = np.mgrid[0:sh, 0:sw]
    gs = np.stack([sxx * scale // max(sw, 1), syy * scale // max(sh, 1)], 2).astype(dt)
    st = workloads.Style(rng.integers(0, 256, size=(sh, sw, 3), dtype=np.uint8), gs,
                         1 if u16 else 0, bits)
    nl = int(rng.integers(1, 5))
    ls = rng.integers(0, nl, size=(sh, sw)).astype(np.uint8)
    lt = rng.integers(0, nl + 1, size=(h, w)).astype(np.uint8)  # nl is past the last table
    levels = int(rng.integers(0, 6))
    finest = int(2 ** rng.integers(0, 5))
    while levels and finest << (levels - 1) > 8192:
        levels -= 1
    # half the cases take their seeds from the jitter hash
    hseed = 31 * seed + 5 if seed % 2 == 0 else None
    jit = None if hseed is not None else workloads.jitter_table(w, h, levels, finest, seed)
    t = int(rng.integers(0, 8 * scale))
    r = int(rng.integers(0, 8))
    check(sb, st, ls, nl, gt, lt, jit, levels, finest, t, r, f"seg random {seed} u16={u16}",
          tunes=[None, (2, 8, 4, 1)], seed=hseed)


@pytest.mark.parametrize("u16,levels", [(False, 9), (True, 10)])
def test_deep_hierarchy(sb, u16, levels):
    """Nine or ten levels with labels: the block level loop stages two seed
    records per lane from the seed table."""
    rng = np.random.default_rng(500 + levels)
    w, h, sw, sh = 251, 163, 47, 41
    scale = 65535 if u16 else 255
    dt = np.uint16 if u16 else np.uint8
    yy, xx = np.mgrid[0:h, 0:w]
    noise = rng.integers(-scale // 40, scale // 40 + 1, size=(h, w, 2))
    gt = np.clip(np.stack([xx * scale // w, yy * scale // h], 2) + noise, 0, scale).astype(dt)
    syy, sxx = np.mgrid[0:sh, 0:sw]
    gs = np.stack([sxx * scale // sw, syy * scale // sh], 2).astype(dt)
    st = workloads.Style(rng.integers(0, 256, size=(sh, sw, 3), dtype=np.uint8), gs,
                         1 if u16 else 0, 7 if u16 else 8)
    ls = (sxx * 3 // sw).astype(np.uint8)
    lt = (xx * 3 // w).astype(np.uint8)
    jit = workloads.jitter_table(w, h, levels, 8, levels)
    check(sb, st, ls, 3, gt, lt, jit, levels, 8, (1 << 22) if u16 else 80, 2,
          f"seg deep L={levels} u16={u16}", tunes=[None, (2, 8, 4, 1), (4, 16, 2, 2)])


def test_one_label_equals_plain(sb):
    import torch

    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    p = fr.params
    prm = sb.params(p.levels, p.finest, p.threshold, p.radius, seed=fr.seed)
    zs = np.zeros(st.guide.shape[:2], np.uint8)
    zt = np.zeros(fr.guide.shape[:2], np.uint8)
    say("one label vs plain")
    style = sb.Style(st.rgb, st.guide, st.lut_bits, labels=zs, nlabels=1)
    a = sb.stylize(style, fr.guide, fr.jitter, prm)
    b = sb.stylize(style, fr.guide, fr.jitter, prm, tgt_labels=zt)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_batch_mixes_labelled_and_plain_frames(sb):
    import torch

    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    ls = workloads.voronoi_labels(st.guide.shape[1], st.guide.shape[0], 3, 12, 5)
    style = sb.Style(st.rgb, st.guide, st.lut_bits, labels=ls, nlabels=3)
    rng = np.random.default_rng(4)
    jobs, expect = [], []
    for i in range(6):
        w, h = int(rng.integers(40, 257)), int(rng.integers(30, 257))
        g = np.ascontiguousarray(fr.guide[:h, :w])
        jit = workloads.jitter_table(w, h, 3, 8, 200 + i)
        lt = workloads.voronoi_labels(w, h, 3, 10, 300 + i) if i % 2 == 0 else None
        prm = sb.params(3, 8, 300, 1 + i % 5)
        jobs.append(sb.FrameJob(style, g, jit, prm, tgt_labels=lt))
        expect.append(sb.stylize(style, g, jit, prm, tgt_labels=lt))
    torch.cuda.synchronize()
    say("batch of labelled and plain frames")
    b = sb.Batch(use_graph=True)
    b.run(jobs)
    torch.cuda.synchronize()
    for j, (rgb, chunk) in zip(jobs, expect):
        np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), rgb.cpu().numpy())
        np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), chunk.cpu().numpy())
    b.close()
