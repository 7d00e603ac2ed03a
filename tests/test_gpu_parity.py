"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element
by element and bit-exact (chunk map, NNF and uint8 RGB are all integer
results).  Cases: the single-frame workloads at full size, random small
shapes and parameters that span several tiles with ragged edges, and the
degenerate cases of the method."""
import numpy as np
import pytest

import oracle
import workloads
from tests.test_oracle_lut import brute_lut

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


def to_np(t):
    return t.cpu().numpy()


def u32(t):
    return to_np(t).view(np.uint32)


def run_gpu(sb, style_np, lut_bits, frame_guide, jit, levels, finest, t, r, style_obj=None,
            tune=None, seed=None):
    import torch

    st = style_obj or sb.Style(style_np.rgb, style_np.guide, lut_bits)
    p = sb.params(levels, finest, t, r, seed=seed)
    rgb, chunk, nnf = sb.stylize(st, frame_guide, jit, p, want_nnf=True, tune=tune)
    torch.cuda.synchronize()
    return to_np(rgb), u32(chunk), u32(nnf), st


def check_frame(sb, st_np, fr_guide, jit, levels, finest, t, r, lut=None, style_obj=None,
                name="", tunes=(None,), seed=None):
    """GPU frame against the oracle, element by element, under each kernel
    choice.  The seeds' jitter: the table ``jit``, else the hash of ``seed``,
    else none (cell corners)."""
    if lut is None:
        lut = oracle.lut_build(st_np.guide, st_np.lut_bits)
    e_rgb, e_chunk, e_nnf = oracle.stylize(st_np.rgb, st_np.guide, lut, st_np.lut_bits, fr_guide,
                                           jit, levels, finest, t, r, seed=seed)
    st = style_obj
    for tune in tunes:
        say(f"{name} {fr_guide.shape[1]}x{fr_guide.shape[0]} L={levels} f={finest} t={t} r={r} "
            f"tune={tune} seed={seed}")
        g_rgb, g_chunk, g_nnf, st = run_gpu(sb, st_np, st_np.lut_bits, fr_guide, jit, levels,
                                            finest, t, r, st, tune, seed)
        msg = f"{name} tune={tune}"
        np.testing.assert_array_equal(g_chunk, e_chunk, err_msg=f"{msg}: chunk map")
        np.testing.assert_array_equal(g_nnf, e_nnf, err_msg=f"{msg}: nnf")
        np.testing.assert_array_equal(g_rgb, e_rgb, err_msg=f"{msg}: rgb")
    return st


def all_tunes(sb):
    return [None] + list(sb.TUNES)


# ----------------------------------------------------------------- LUT

def lut_gpu(sb, st_np):
    import torch

    st = sb.Style(st_np.rgb, st_np.guide, st_np.lut_bits)
    torch.cuda.synchronize()
    return u32(st.lut), st


@pytest.mark.parametrize("n", [1, 2, 3])
def test_lut_workload_styles(sb, n):
    styles, _ = workloads.config(n)
    for s in styles:
        say(f"lut workload {n} {s.sw}x{s.sh} bits={s.lut_bits}")
        g, _ = lut_gpu(sb, s)
        np.testing.assert_array_equal(g, oracle.lut_build(s.guide, s.lut_bits))


def test_lut_batch_styles(sb):
    styles, _ = workloads.config(4, frames=2)
    for s in styles:
        say(f"lut batch style {s.sw}x{s.sh} fmt={s.fmt} bits={s.lut_bits}")
        g, _ = lut_gpu(sb, s)
        np.testing.assert_array_equal(g, oracle.lut_build(s.guide, s.lut_bits))


@pytest.mark.parametrize("seed", range(8))
def test_lut_random(sb, seed):
    rng = np.random.default_rng(1000 + seed)
    u16 = seed % 2 == 1
    sw, sh = int(rng.integers(1, 70)), int(rng.integers(1, 70))
    if u16:
        bits = int(rng.integers(1, 11))
        hi = int(rng.choice([65536, 4000]))
        gs = rng.integers(0, hi, size=(sh, sw, 2), dtype=np.uint16)
    else:
        bits = int(rng.integers(1, 9))
        gs = rng.integers(0, 256, size=(sh, sw, 2), dtype=np.uint8)
        if seed % 4 == 0:
            gs[:] = gs[0, 0]  # a single guide value: every bin ties everywhere
    st = workloads.Style(rng.integers(0, 256, size=(sh, sw, 3), dtype=np.uint8), gs,
                         1 if u16 else 0, bits)
    say(f"lut random seed={seed} {sw}x{sh} u16={u16} bits={bits}")
    g, _ = lut_gpu(sb, st)
    # the plain definition (exhaustive argmin) directly: for sparse, clustered
    # sources the oracle's ring search would walk far for every bin
    np.testing.assert_array_equal(g, brute_lut(gs, bits))


# ----------------------------------------------------------- full frames

@pytest.mark.parametrize("n", [1, 2, 3])
def test_workload_frames(sb, n):
    styles, frames = workloads.config(n)
    st, fr = styles[0], frames[0]
    p = fr.params
    assert fr.jitter is None and fr.seed is not None  # the workloads' seeds come from the hash
    check_frame(sb, st, fr.guide, fr.jitter, p.levels, p.finest, p.threshold, p.radius,
                name=f"workload {n}", tunes=all_tunes(sb), seed=fr.seed)


def test_workload2_param_sweep(sb):
    """The 1080p frame under other thresholds and radii (one resident style)."""
    styles, frames = workloads.config(2)
    st, fr = styles[0], frames[0]
    lut = oracle.lut_build(st.guide, st.lut_bits)
    style_obj = None
    for t, r in [(0, 0), (1, 1), (200, 2), (5000, 7), (1 << 31, 3)]:
        style_obj = check_frame(sb, st, fr.guide, fr.jitter, 4, 8, t, r, lut=lut,
                                style_obj=style_obj, name="workload 2 sweep",
                                tunes=[None, sb.TUNES[0]], seed=fr.seed)


@pytest.mark.parametrize("seed", range(24))
def test_random_small(sb, seed):
    rng = np.random.default_rng(seed)
    u16 = seed % 2 == 1
    w, h = int(rng.integers(1, 300)), int(rng.integers(1, 200))
    sw, sh = int(rng.integers(1, 120)), int(rng.integers(1, 120))
    bits = int(rng.integers(3, 11)) if u16 else int(rng.integers(5, 9))
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
    levels = int(rng.integers(0, 7))
    finest = int(2 ** rng.integers(0, 5))
    while levels and finest << (levels - 1) > 8192:
        levels -= 1
    # every third case draws its seeds from the jitter hash (its seed drawn
    # over all 32 bits), the others from a table
    hseed = int(rng.integers(0, 2**32)) if seed % 3 == 0 else None
    jit = None if hseed is not None else workloads.jitter_table(w, h, levels, finest, seed)
    t = int(rng.integers(0, 8 * scale))
    r = int(rng.integers(0, 8))
    check_frame(sb, st, gt, jit, levels, finest, t, r, name=f"random {seed} u16={u16}",
                tunes=all_tunes(sb), seed=hseed)


def _gradient_case(rng, w, h, sw, sh, u16):
    scale = 65535 if u16 else 255
    dt = np.uint16 if u16 else np.uint8
    yy, xx = np.mgrid[0:h, 0:w]
    noise = rng.integers(-scale // 40, scale // 40 + 1, size=(h, w, 2))
    gt = np.clip(np.stack([xx * scale // w, yy * scale // h], 2) + noise, 0, scale).astype(dt)
    syy, sxx = np.mgrid[0:sh, 0:sw]
    gs = np.stack([sxx * scale // sw, syy * scale // sh], 2).astype(dt)
    st = workloads.Style(rng.integers(0, 256, size=(sh, sw, 3), dtype=np.uint8), gs,
                         1 if u16 else 0, 9 if u16 else 8)
    return st, gt


@pytest.mark.parametrize("u16,levels,finest,t", [(False, 8, 8, 60), (False, 11, 8, 30),
                                                 (True, 9, 8, 1 << 22), (False, 12, 2, 60),
                                                 (True, 10, 8, 0), (False, 7, 16, 60)])
def test_deep_hierarchies(sb, u16, levels, finest, t):
    """Eight or more levels: an 8 x 8 block stages 9 L > 64 seed records, so
    lanes take a second record each (made in the level loop for 8-bit guides,
    read from the seed table for 16-bit ones); spacings up to 8192 exceed the
    frame.  L = 12 at finest 2 takes the per-pixel path."""
    rng = np.random.default_rng(levels * 100 + finest + int(u16))
    st, gt = _gradient_case(rng, 333, 217, 97, 83, u16)
    jit = workloads.jitter_table(333, 217, levels, finest, levels + 7)
    check_frame(sb, st, gt, jit, levels, finest, t, 2, name=f"deep u16={u16}",
                tunes=all_tunes(sb))
    # the same hierarchy with the seeds from the jitter hash
    check_frame(sb, st, gt, None, levels, finest, t, 2, name=f"deep hash u16={u16}",
                tunes=[None, sb.TUNES[0], sb.TUNES[-1]], seed=levels * 977 + finest)


def test_degenerate_shapes(sb):
    rng = np.random.default_rng(77)
    st = workloads.Style(workloads.value_noise_rgb(64, 64, 1), workloads.sphere_guide_u8(64), 0, 8)
    lut = oracle.lut_build(st.guide, 8)
    style_obj = None
    for w, h, levels, finest in [(1, 1, 3, 2), (1, 37, 2, 1), (53, 1, 4, 2), (7, 5, 3, 8),
                                 (8192, 2, 2, 8), (3, 8192, 3, 64), (300, 9, 1, 8192)]:
        gt = rng.integers(0, 256, size=(h, w, 2), dtype=np.uint8)
        jit = workloads.jitter_table(w, h, levels, finest, w * 31 + h)
        style_obj = check_frame(sb, st, gt, jit, levels, finest, 64, 3, lut=lut,
                                style_obj=style_obj, name="degenerate", tunes=all_tunes(sb))
        style_obj = check_frame(sb, st, gt, None, levels, finest, 64, 3, lut=lut,
                                style_obj=style_obj, name="degenerate hash",
                                tunes=[None, sb.TUNES[-1]], seed=w * 31 + h)


def test_no_jitter_and_zero_levels(sb):
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    lut = oracle.lut_build(st.guide, 8)
    o = check_frame(sb, st, fr.guide, None, 3, 8, 48, 2, lut=lut, name="no jitter",
                    tunes=all_tunes(sb))
    check_frame(sb, st, fr.guide, np.zeros(0, np.uint32), 0, 8, 48, 2, lut=lut, style_obj=o,
                name="zero levels", tunes=all_tunes(sb))


def test_identity_reproduces_source(sb):
    import torch

    g = workloads.identity_uv_guide_u16(512, 512)
    src = workloads.value_noise_rgb(512, 512, 9)
    st = sb.Style(src, g, 9)
    jit = workloads.jitter_table(512, 512, 5, 8, 3)
    say("identity 512x512")
    rgb, chunk = sb.stylize(st, g, jit, sb.params(5, 8, 1, 3))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(rgb), src)


def test_rejects_format_mismatch(sb):
    import torch

    st = sb.Style(workloads.value_noise_rgb(32, 32, 1), workloads.sphere_guide_u8(32), 8)
    g16 = np.zeros((8, 8, 2), np.uint16)
    # the binding passes the style's format; a u16 guide for a u8 style is a
    # different byte size and must be refused before launch
    with pytest.raises(Exception):
        sb.stylize(st, g16.view(np.int16), np.zeros(sb.jitter_len(8, 8, 1, 8), np.uint32),
                   sb.params(1, 8, 10, 1))
    torch.cuda.synchronize()


def test_unaligned_output_rows(sb):
    """Odd widths: rows start unaligned, so the vote takes its byte and
    16-bit store paths and its partial pixel groups."""
    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    lut = oracle.lut_build(st.guide, 8)
    g = np.ascontiguousarray(fr.guide[:, :253])
    jit = workloads.jitter_table(253, 256, 3, 8, 5)
    check_frame(sb, st, g, jit, 3, 8, 48, 2, lut=lut, name="width 253", tunes=all_tunes(sb))




def test_library_owned_style(sb):
    """sb_style_create builds the same padded exemplar and lookup table as
    the caller-owned path, and a frame through it equals the oracle;
    sb_style_destroy frees it."""
    import ctypes

    import torch

    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    p = fr.params
    rgb_d = torch.from_numpy(st.rgb).cuda()
    guide_d = torch.from_numpy(st.guide).cuda()
    h = ctypes.POINTER(sb.SbStyle)()
    say("sb_style_create 256x256")
    rc = sb.lib().sb_style_create(rgb_d.data_ptr(), guide_d.data_ptr(), st.sw, st.sh, st.fmt,
                                  st.lut_bits, torch.cuda.current_stream().cuda_stream,
                                  ctypes.cast(ctypes.byref(h), ctypes.POINTER(ctypes.c_void_p)))
    assert rc == sb.SB_OK
    del rgb_d, guide_d  # the style holds its own copies
    s = h.contents
    assert (s.sw, s.sh, s.fmt, s.lut_bits, s.nlabels) == (st.sw, st.sh, st.fmt, st.lut_bits, 0)
    class DevView:  # a view of library-owned device memory as a tensor
        def __init__(self, ptr, n):
            self.__cuda_array_interface__ = {"shape": (n,), "typestr": "<i4",
                                             "data": (ptr, False), "version": 2}

    lut = oracle.lut_build(st.guide, st.lut_bits)
    got = torch.as_tensor(DevView(s.lut, 1 << (2 * st.lut_bits)), device="cuda")
    np.testing.assert_array_equal(u32(got), lut)
    ref = sb.Style(st.rgb, st.guide, st.lut_bits)
    ex = torch.as_tensor(DevView(s.rgba, ref.rgba.numel()), device="cuda")
    assert torch.equal(ex, ref.rgba)

    class Owned:  # the binding's Style interface over the library-owned struct
        c = s
        fmt = st.fmt

    e_rgb, e_chunk, e_nnf = oracle.stylize(st.rgb, st.guide, lut, st.lut_bits, fr.guide, None,
                                           p.levels, p.finest, p.threshold, p.radius, seed=fr.seed)
    rgb, chunk, nnf = sb.stylize(Owned, fr.guide, None,
                                 sb.params(p.levels, p.finest, p.threshold, p.radius, seed=fr.seed),
                                 want_nnf=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(u32(chunk), e_chunk)
    np.testing.assert_array_equal(u32(nnf), e_nnf)
    np.testing.assert_array_equal(to_np(rgb), e_rgb)
    assert sb.lib().sb_style_destroy(h) == sb.SB_OK


def test_round_robin_two_streams_match_oracle(sb):
    """The launch configuration the benchmark times: prepared frames over six
    buffer sets launched round robin on two streams, three passes with no
    synchronisation between launches, each set's frame with its own jitter
    seed; every set's result equals the oracle's, element by element."""
    import torch

    styles, frames = workloads.config(2)
    st_np, fr = styles[0], frames[0]
    p = fr.params
    style = sb.Style(st_np.rgb, st_np.guide, st_np.lut_bits)
    lut = oracle.lut_build(st_np.guide, st_np.lut_bits)
    g = torch.from_numpy(fr.guide).cuda()
    seeds = [fr.seed + 17 * i for i in range(6)]
    say(f"round robin on two streams: {fr.w}x{fr.h}, seeds {seeds}")
    sets, plans = [], []
    for sd in seeds:
        prm = sb.params(p.levels, p.finest, p.threshold, p.radius, seed=sd)
        rgb = torch.empty((fr.h, fr.w, 3), dtype=torch.uint8, device="cuda")
        chunk = torch.empty((fr.h, fr.w), dtype=torch.int32, device="cuda")
        ws = torch.empty(sb.workspace_bytes(fr.w, fr.h, prm), dtype=torch.uint8, device="cuda")
        sets.append((rgb, chunk))
        plans.append(sb.FramePlan(style, g, None, prm, rgb, chunk, ws))
    other = torch.cuda.Stream()
    streams = [torch.cuda.current_stream().cuda_stream, other.cuda_stream]
    for _ in range(3):
        for k, plan in enumerate(plans):
            plan.launch(streams[k % 2])
    torch.cuda.synchronize()
    for sd, (rgb, chunk) in zip(seeds, sets):
        e_rgb, e_chunk, _ = oracle.stylize(st_np.rgb, st_np.guide, lut, st_np.lut_bits, fr.guide,
                                           None, p.levels, p.finest, p.threshold, p.radius,
                                           seed=sd)
        np.testing.assert_array_equal(u32(chunk), e_chunk, err_msg=f"chunk seed={sd}")
        np.testing.assert_array_equal(to_np(rgb), e_rgb, err_msg=f"rgb seed={sd}")


def test_frame_plan_equals_stylize():
    """FramePlan (arguments marshalled once, one C call per launch) gives the
    frame sb_stylize gives, on the current stream and on an explicit one."""
    import torch

    import paper_1807_03249_amd as sb

    styles, frames = workloads.config(2)
    st_np, fr = styles[0], frames[0]
    p = fr.params
    style = sb.Style(st_np.rgb, st_np.guide, st_np.lut_bits)
    prm = sb.params(p.levels, p.finest, p.threshold, p.radius, seed=fr.seed)
    g = torch.from_numpy(fr.guide).cuda()
    e_rgb, e_chunk = sb.stylize(style, g, None, prm)
    ws = torch.empty(sb.workspace_bytes(fr.w, fr.h, prm), dtype=torch.uint8, device="cuda")
    for tune in (None, (2, 8, 4, 1, 1)):
        rgb = torch.empty_like(e_rgb)
        chunk = torch.empty_like(e_chunk)
        plan = sb.FramePlan(style, g, None, prm, rgb, chunk, ws, tune=tune)
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(rgb, e_rgb) and torch.equal(chunk, e_chunk)
        s = torch.cuda.Stream()
        rgb.zero_()
        torch.cuda.synchronize()
        plan.launch(s.cuda_stream)
        s.synchronize()
        assert torch.equal(rgb, e_rgb) and torch.equal(chunk, e_chunk)
