"""Three-channel guides on the GPU (format 2: two normal channels plus an
appearance channel, the additional guiding channels of Sec. 3.1), through the
C ABI against the CPU oracle, bit-exact: the exact lookup table built by the
separable transform (whole tables at small sizes, sampled bins of the
2^24-entry table of the 1080p appearance workload), whole frames under every
kernel choice, the 1080p workload at sampled pixels, the segmentation guide,
and batches that mix formats."""
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


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def small_style(size, seed, lut_bits):
    rgb = workloads.value_noise_rgb(size, size, seed)
    g = workloads.guide_u8x3(workloads.sphere_guide_u8(size), workloads.appearance_u8(rgb, 4))
    return workloads.Style(rgb, g, workloads.GUIDE_U8X3, lut_bits)


@pytest.mark.parametrize("lut_bits,nvals,h,w", [(1, 4, 12, 17), (3, 3, 33, 20), (5, 256, 40, 64),
                                                (4, 2, 1, 1)])
def test_table_matches_oracle(sb, lut_bits, nvals, h, w):
    import torch

    say(f"three-channel table bits={lut_bits} values={nvals} {w}x{h}")
    rng = np.random.default_rng(lut_bits + 10 * nvals)
    src = np.zeros((h, w, 4), np.uint8)
    vals = np.linspace(0, 255, nvals).astype(np.uint8)
    src[..., :3] = vals[rng.integers(0, nvals, (h, w, 3))]
    src[..., 3] = rng.integers(0, 256, (h, w))  # ignored
    rgb = rng.integers(0, 256, (h, w, 3)).astype(np.uint8)
    st = sb.Style(rgb, src, lut_bits)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(st.lut), oracle.lut_build(src, lut_bits))


def test_two_channel_tables_match_oracle(sb):
    """The 8-bit two-channel table now comes from the same separable build."""
    import torch

    for size, bits, seed in ((64, 8, 1), (37, 5, 2), (128, 7, 3)):
        say(f"two-channel table {size} bits={bits}")
        rng = np.random.default_rng(seed)
        g = rng.integers(0, 256, (size, size, 2)).astype(np.uint8)
        g[: size // 2] = workloads.sphere_guide_u8(size)[: size // 2]
        st = sb.Style(workloads.value_noise_rgb(size, size, seed), g, bits)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(u32(st.lut), oracle.lut_build(g, bits))


def test_full_size_table_sampled(sb):
    import torch

    st_np = workloads.config(6, w=64, h=64)[0][0]  # the 512^2 appearance style, 8 bits
    say("512x512 three-channel style, 2^24-entry table, 3000 sampled bins")
    st = sb.Style(st_np.rgb, st_np.guide, st_np.lut_bits)
    torch.cuda.synchronize()
    lut = u32(st.lut)
    assert lut.size == 1 << 24
    rng = np.random.default_rng(77)
    bins = np.concatenate([rng.integers(0, 1 << 24, 2990), [0, (1 << 24) - 1, 1 << 23, 255,
                                                             65535, 65536, 12345678, 8421504,
                                                             4210752, 16711935]])
    np.testing.assert_array_equal(lut[bins], oracle.lut_query(st_np.guide, 8, bins))


@pytest.mark.parametrize("w,h,levels,finest,t,r", [(200, 136, 4, 8, 64, 3), (97, 61, 3, 4, 300, 2),
                                                  (64, 64, 0, 8, 0, 1), (131, 70, 4, 2, 25, 0),
                                                  (221, 143, 9, 8, 200, 2)])
def test_frames_match_oracle_all_tunes(sb, w, h, levels, finest, t, r):
    import torch

    st_np = small_style(128, 41, 5)
    style = sb.Style(st_np.rgb, st_np.guide, st_np.lut_bits)
    lut = oracle.lut_build(st_np.guide, 5)
    g = workloads.appearance_target(w, h, 5, 42 + w)
    jit = workloads.jitter_table(w, h, levels, finest, 43 + h)
    e_rgb, e_chunk, e_nnf = oracle.stylize(st_np.rgb, st_np.guide, lut, 5, g, jit, levels, finest,
                                           t, r)
    prm = sb.params(levels, finest, t, r)
    for tune in [None] + list(sb.TUNES):
        say(f"three-channel frame {w}x{h} L={levels} f={finest} t={t} r={r} tune={tune}")
        rgb, chunk, nnf = sb.stylize(style, g, jit, prm, want_nnf=True, tune=tune)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(u32(chunk), e_chunk, err_msg=f"tune={tune}")
        np.testing.assert_array_equal(u32(nnf), e_nnf, err_msg=f"tune={tune}")
        np.testing.assert_array_equal(rgb.cpu().numpy(), e_rgb, err_msg=f"tune={tune}")


def test_full_size_workload(sb):
    """The 1080p appearance workload in the configuration the benchmark times,
    element by element over the whole frame: every chunk code, NNF entry and
    RGB triple against the oracle.  The oracle's table holds exactly the
    entries the frame reads -- the bins of every seed, then of every pixel
    that falls back -- each computed by the oracle's exact query."""
    import torch

    styles, frames = workloads.config(6)
    st_np, fr = styles[0], frames[0]
    p = fr.params
    w, h = fr.w, fr.h
    bits = st_np.lut_bits

    def bins_at(xs, ys):
        c = fr.guide[ys, xs, :3].astype(np.int64) >> (8 - bits)
        return c[:, 0] + (c[:, 1] << bits) + (c[:, 2] << (2 * bits))

    jit = oracle.jitter_hash(w, h, p.levels, p.finest, fr.seed)
    sx, sy, off = [], [], 0
    for (cx, cy), sp in zip(workloads.jitter_cells(w, h, p.levels, p.finest),
                            workloads.level_spacings(p.levels, p.finest)):
        j = jit[off:off + cx * cy].astype(np.int64)
        off += cx * cy
        by, bx = np.divmod(np.arange(cx * cy), cx)
        x, y = bx * sp + (j & 0xFFFF), by * sp + (j >> 16)
        ok = (x < w) & (y < h)
        sx.append(x[ok])
        sy.append(y[ok])
    seed_bins = np.unique(bins_at(np.concatenate(sx), np.concatenate(sy)))
    say(f"appearance 1080p: {seed_bins.size} seed bins")
    lut = np.zeros(1 << (3 * bits), np.uint32)
    lut[seed_bins] = oracle.lut_query_sweep(st_np.guide, bits, seed_bins)
    # which pixels fall back depends only on the seeds' entries
    _, chunk0 = oracle.assign(st_np.guide, lut, bits, fr.guide, None, p.levels, p.finest,
                              p.threshold, seed=fr.seed)
    fy, fx = np.nonzero((chunk0 >> 26) == p.levels)
    own_bins = np.setdiff1d(np.unique(bins_at(fx, fy)), seed_bins)
    say(f"appearance 1080p: {fy.size} fallback pixels, {own_bins.size} more bins")
    lut[own_bins] = oracle.lut_query_sweep(st_np.guide, bits, own_bins)
    e_rgb, e_chunk, e_nnf = oracle.stylize(st_np.rgb, st_np.guide, lut, bits, fr.guide, fr.jitter,
                                           p.levels, p.finest, p.threshold, p.radius, seed=fr.seed)
    np.testing.assert_array_equal(e_chunk, chunk0)
    say("appearance 1080p: GPU frame")
    style = sb.Style(st_np.rgb, st_np.guide, bits)
    rgb, chunk, nnf = sb.stylize(style, fr.guide, fr.jitter,
                                 sb.params(p.levels, p.finest, p.threshold, p.radius, seed=fr.seed),
                                 want_nnf=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(chunk), e_chunk)
    np.testing.assert_array_equal(u32(nnf), e_nnf)
    np.testing.assert_array_equal(rgb.cpu().numpy(), e_rgb)
    lv = e_chunk >> 26
    assert 0.0 < float((lv == p.levels).mean()) < 0.9  # the level loop does accept


def test_segmentation_with_three_channels(sb):
    import torch

    st_np = small_style(96, 51, 4)
    ls = workloads.voronoi_labels(96, 96, 4, 9, 52)
    w, h = 150, 90
    lt = workloads.voronoi_labels(w, h, 5, 12, 53)  # label 4 lies past the exemplar's labels
    g = workloads.appearance_target(w, h, 4, 54)
    jit = workloads.jitter_table(w, h, 3, 8, 55)
    luts = oracle.lut_build_labels(st_np.guide, ls, 4, 4)
    say("three-channel frame with the segmentation guide")
    e = oracle.stylize_seg(st_np.rgb, st_np.guide, ls, luts, 4, 4, g, lt, jit, 3, 8, 200, 2)
    style = sb.Style(st_np.rgb, st_np.guide, 4, labels=ls, nlabels=4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(style.label_luts).reshape(4, -1), luts)
    rgb, chunk, nnf = sb.stylize(style, g, jit, sb.params(3, 8, 200, 2), want_nnf=True,
                                 tgt_labels=lt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(chunk), e[1])
    np.testing.assert_array_equal(u32(nnf), e[2])
    np.testing.assert_array_equal(rgb.cpu().numpy(), e[0])


def test_batch_mixes_formats(sb):
    import torch

    st3 = small_style(128, 61, 5)
    s3 = sb.Style(st3.rgb, st3.guide, 5)
    s2_np = workloads.config(1)[0][0]
    s2 = sb.Style(s2_np.rgb, s2_np.guide, s2_np.lut_bits)
    jobs = []
    rng = np.random.default_rng(62)
    for k in range(10):
        w, h = int(rng.integers(40, 400)), int(rng.integers(30, 300))
        if k % 2:
            g, st = workloads.appearance_target(w, h, 4, 63 + k), s3
        else:
            g, st = workloads.bump_guide_u8(w, h, 4, 63 + k), s2
        jit = workloads.jitter_table(w, h, 3, 8, 70 + k)
        jobs.append(sb.FrameJob(st, g, jit, sb.params(3, 8, 64, 3), out_nnf=torch.empty(
            (h, w), dtype=torch.int32, device="cuda")))
    say("batch of 10 frames mixing two- and three-channel guides")
    b = sb.Batch(use_graph=True)
    for _ in range(2):
        b.run(jobs)
        torch.cuda.synchronize()
        for j in jobs:
            rgb, chunk, nnf = sb.stylize(j.style, j.guide, j.jitter, j.params, want_nnf=True)
            torch.cuda.synchronize()
            assert torch.equal(j.out_rgb, rgb) and torch.equal(j.out_chunk, chunk)
            assert torch.equal(j.out_nnf, nnf)
    b.close()


@pytest.mark.parametrize("weights", [(3, 1, 7), (1, 1, 0), (0, 2, 5), (127, 127, 1)])
def test_weighted_tables_and_frames(sb, weights):
    """Channel weights (strong or weak appearance guide): the weighted table
    and frames under every kernel choice against the oracle."""
    import torch

    st_np = small_style(96, 71, 4)
    style = sb.Style(st_np.rgb, st_np.guide, 4, weights=weights)
    torch.cuda.synchronize()
    lut = oracle.lut_build(st_np.guide, 4, weights)
    say(f"weighted table {weights}")
    np.testing.assert_array_equal(u32(style.lut), lut)
    w, h = 150, 94
    g = workloads.appearance_target(w, h, 4, 72)
    jit = workloads.jitter_table(w, h, 3, 8, 73)
    t = 60 * max(weights)
    e_rgb, e_chunk, e_nnf = oracle.stylize(st_np.rgb, st_np.guide, lut, 4, g, jit, 3, 8, t, 2,
                                           weights=weights)
    prm = sb.params(3, 8, t, 2)
    for tune in [None] + list(sb.TUNES)[::3]:
        say(f"weighted frame {weights} tune={tune}")
        rgb, chunk, nnf = sb.stylize(style, g, jit, prm, want_nnf=True, tune=tune)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(u32(chunk), e_chunk, err_msg=f"tune={tune}")
        np.testing.assert_array_equal(u32(nnf), e_nnf, err_msg=f"tune={tune}")
        np.testing.assert_array_equal(rgb.cpu().numpy(), e_rgb, err_msg=f"tune={tune}")


def test_weighted_segmentation_and_batch(sb):
    import torch

    weights = (5, 2, 9)
    st_np = small_style(80, 81, 4)
    ls = workloads.voronoi_labels(80, 80, 3, 7, 82)
    style = sb.Style(st_np.rgb, st_np.guide, 4, labels=ls, nlabels=3, weights=weights)
    torch.cuda.synchronize()
    luts = oracle.lut_build_labels(st_np.guide, ls, 3, 4, weights)
    np.testing.assert_array_equal(u32(style.label_luts).reshape(3, -1), luts)
    w, h = 120, 77
    lt = workloads.voronoi_labels(w, h, 3, 9, 83)
    g = workloads.appearance_target(w, h, 4, 84)
    jit = workloads.jitter_table(w, h, 3, 8, 85)
    say("weighted frame with the segmentation guide")
    e = oracle.stylize_seg(st_np.rgb, st_np.guide, ls, luts, 3, 4, g, lt, jit, 3, 8, 900, 2,
                           weights=weights)
    rgb, chunk, nnf = sb.stylize(style, g, jit, sb.params(3, 8, 900, 2), want_nnf=True,
                                 tgt_labels=lt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(chunk), e[1])
    np.testing.assert_array_equal(u32(nnf), e[2])
    np.testing.assert_array_equal(rgb.cpu().numpy(), e[0])
    say("batch mixing weighted and unweighted three-channel styles")
    plain = sb.Style(st_np.rgb, st_np.guide, 4)
    jobs = [sb.FrameJob(style if k % 2 else plain, workloads.appearance_target(w + k, h, 4, 86 + k),
                        workloads.jitter_table(w + k, h, 3, 8, 87 + k), sb.params(3, 8, 900, 2))
            for k in range(6)]
    b = sb.Batch(use_graph=True)
    b.run(jobs)
    torch.cuda.synchronize()
    for j in jobs:
        r, c = sb.stylize(j.style, j.guide, j.jitter, j.params)
        torch.cuda.synchronize()
        assert torch.equal(j.out_rgb, r) and torch.equal(j.out_chunk, c)
    b.close()


@pytest.mark.parametrize("case", range(10))
def test_random_three_channel_cases(sb, case):
    """Random sizes, hierarchies, thresholds, radii, weights and (half the
    cases) label maps, against the oracle."""
    import torch

    rng = np.random.default_rng(1000 + case)
    ssz = int(rng.integers(24, 80))
    bits = int(rng.integers(1, 6))
    st_np = small_style(ssz, 2000 + case, bits)
    weights = tuple(int(v) for v in rng.integers(0, 12, 3)) if case % 3 else None
    w, h = int(rng.integers(1, 150)), int(rng.integers(1, 120))
    levels = int(rng.integers(0, 5))
    finest = int(2 ** rng.integers(0, 4))
    while levels > 0 and (finest << (levels - 1)) > 8192:
        levels -= 1
    t = int(rng.integers(0, 3000))
    r = int(rng.integers(0, 4))
    g = workloads.appearance_target(w, h, 3, 3000 + case)
    jit = oracle.jitter_fill(w, h, levels, finest, 4000 + case, case)
    seg = case % 2 == 1
    say(f"random three-channel case {case}: src {ssz} bits {bits} {w}x{h} L={levels} "
        f"f={finest} t={t} r={r} w={weights} seg={seg}")
    prm = sb.params(levels, finest, t, r)
    if seg:
        nl = int(rng.integers(1, 5))
        ls = workloads.voronoi_labels(ssz, ssz, nl, 6, 5000 + case)
        lt = workloads.voronoi_labels(w, h, nl + 1, 5, 6000 + case)
        style = sb.Style(st_np.rgb, st_np.guide, bits, labels=ls, nlabels=nl, weights=weights)
        luts = oracle.lut_build_labels(st_np.guide, ls, nl, bits, weights)
        e = oracle.stylize_seg(st_np.rgb, st_np.guide, ls, luts, nl, bits, g, lt, jit, levels,
                               finest, t, r, weights=weights)
        rgb, chunk, nnf = sb.stylize(style, g, jit, prm, want_nnf=True, tgt_labels=lt)
    else:
        style = sb.Style(st_np.rgb, st_np.guide, bits, weights=weights)
        lut = oracle.lut_build(st_np.guide, bits, weights)
        e = oracle.stylize(st_np.rgb, st_np.guide, lut, bits, g, jit, levels, finest, t, r,
                           weights=weights)
        rgb, chunk, nnf = sb.stylize(style, g, jit, prm, want_nnf=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(chunk), e[1])
    np.testing.assert_array_equal(u32(nnf), e[2])
    np.testing.assert_array_equal(rgb.cpu().numpy(), e[0])
