"""Batched form on the GPU: many frames of uneven size and mixed guidance in
one graph launch must equal per-frame launches bit for bit (and the oracle),
across repeated replays of the same captured graphs."""
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


@pytest.fixture(scope="module")
def mix(sb):
    """12 uneven frames, half normal-guided and half UV-guided, 4 styles."""
    styles_np, frames_np = workloads.config(4, frames=12)
    styles = [sb.Style(s.rgb, s.guide, s.lut_bits) for s in styles_np]
    return styles_np, frames_np, styles


def jobs_for(sb, styles, frames_np, idx):
    out = []
    for i in idx:
        f = frames_np[i]
        p = f.params
        out.append(sb.FrameJob(styles[f.style], f.guide, f.jitter,
                               sb.params(p.levels, p.finest, p.threshold, p.radius, seed=f.seed)))
    return out


def single(sb, styles, f):
    import torch

    p = f.params
    rgb, chunk = sb.stylize(styles[f.style], f.guide, f.jitter,
                            sb.params(p.levels, p.finest, p.threshold, p.radius, seed=f.seed))
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), chunk.cpu().numpy()


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_equals_single(sb, mix, use_graph):
    import torch

    styles_np, frames_np, styles = mix
    b = sb.Batch(use_graph=use_graph)
    idx = list(range(len(frames_np)))
    say(f"batch of {len(idx)} graph={use_graph}")
    jobs = jobs_for(sb, styles, frames_np, idx)
    b.run(jobs)
    torch.cuda.synchronize()
    for i, j in zip(idx, jobs):
        rgb, chunk = single(sb, styles, frames_np[i])
        np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), rgb, err_msg=f"frame {i} rgb")
        np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), chunk, err_msg=f"frame {i} chunk")
    b.close()


@pytest.mark.parametrize("tune,bpc", [((2, 8, 4, 2), 2), ((4, 8, 2, 1), 1), ((2, 16, 2, 2), 16),
                                      ((4, 16, 4, 2), 8)])
def test_batch_tunes_equal_single(sb, mix, tune, bpc):
    """Every kernel choice and persistent grid size gives the same bits."""
    import torch

    styles_np, frames_np, styles = mix
    b = sb.Batch(use_graph=True, tune=tune, blocks_per_cu=bpc)
    idx = [0, 3, 6, 7, 10]
    say(f"batch tune={tune} blocks_per_cu={bpc}")
    jobs = jobs_for(sb, styles, frames_np, idx)
    b.run(jobs)
    torch.cuda.synchronize()
    for i, j in zip(idx, jobs):
        rgb, chunk = single(sb, styles, frames_np[i])
        np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), rgb, err_msg=f"frame {i} rgb")
        np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), chunk, err_msg=f"frame {i} chunk")
    b.close()


def test_batch_matches_oracle(sb, mix):
    import torch

    styles_np, frames_np, styles = mix
    b = sb.Batch(use_graph=True)
    idx = [0, 7]  # one normal-guided, one UV-guided frame
    jobs = jobs_for(sb, styles, frames_np, idx)
    b.run(jobs)
    torch.cuda.synchronize()
    for i, j in zip(idx, jobs):
        f = frames_np[i]
        st = styles_np[f.style]
        p = f.params
        say(f"oracle frame {i} {f.w}x{f.h}")
        lut = oracle.lut_build(st.guide, st.lut_bits)
        e_rgb, e_chunk, _ = oracle.stylize(st.rgb, st.guide, lut, st.lut_bits, f.guide, f.jitter,
                                           p.levels, p.finest, p.threshold, p.radius, seed=f.seed)
        np.testing.assert_array_equal(j.out_chunk.cpu().numpy().view(np.uint32), e_chunk)
        np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), e_rgb)
    b.close()


def test_graph_replays_any_shapes(sb, mix):
    """One plan, many replays with different frame sets and eager work and
    synchronisation in between; every replay matches the eager results."""
    import torch

    styles_np, frames_np, styles = mix
    b = sb.Batch(use_graph=True)
    expect = {i: single(sb, styles, frames_np[i]) for i in range(len(frames_np))}
    rng = np.random.default_rng(5)
    for rep in range(6):
        idx = sorted(rng.choice(len(frames_np), size=int(rng.integers(1, len(frames_np) + 1)),
                                replace=False).tolist())
        say(f"replay {rep}: frames {idx}")
        jobs = jobs_for(sb, styles, frames_np, idx)
        b.run(jobs)
        # eager work on the same device between replays
        _ = single(sb, styles, frames_np[idx[0]])
        torch.cuda.synchronize()
        for i, j in zip(idx, jobs):
            np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), expect[i][0])
            np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), expect[i][1])
    b.close()


def test_back_to_back_runs(sb, mix):
    """Runs enqueued without waiting: the two descriptor halves alternate."""
    import torch

    styles_np, frames_np, styles = mix
    b = sb.Batch(use_graph=True)
    sets = [[0, 1, 2], [3, 4, 5, 6], [7, 8], [9, 10, 11], [0, 6, 11]]
    runs = []
    for idx in sets:
        jobs = jobs_for(sb, styles, frames_np, idx)
        b.run(jobs)
        runs.append((idx, jobs))
    torch.cuda.synchronize()
    for idx, jobs in runs:
        for i, j in zip(idx, jobs):
            rgb, chunk = single(sb, styles, frames_np[i])
            np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), rgb)
            np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), chunk)
    b.close()


def test_batch_rejects_bad_frames(sb, mix):
    import torch

    styles_np, frames_np, styles = mix
    b = sb.Batch(use_graph=True)
    jobs = jobs_for(sb, styles, frames_np, [0])
    bad = sb.FrameJob(styles[0], frames_np[0].guide, frames_np[0].jitter, sb.params(4, 8, 10, 9))
    with pytest.raises(sb.StyleBlitError):
        b.run(jobs + [bad])
    with pytest.raises(sb.StyleBlitError):
        b.run(jobs * (b.max_frames + 1))
    torch.cuda.synchronize()
    b.close()


def test_batch_mixed_radii(sb):
    """Frames of radius 0..7 in one batch: both vote kernels (radius 0-3 and
    4-7) run in the same replay, each over its own frames' tiles."""
    import torch

    styles_np, frames_np = workloads.config(1)
    st = sb.Style(styles_np[0].rgb, styles_np[0].guide, styles_np[0].lut_bits)
    f = frames_np[0]
    rng = np.random.default_rng(11)
    jobs, expect = [], []
    for i, r in enumerate([7, 0, 4, 3, 6, 1, 5, 2]):
        w, h = int(rng.integers(40, 257)), int(rng.integers(30, 257))
        g = np.ascontiguousarray(f.guide[:h, :w])
        jit = workloads.jitter_table(w, h, 3, 8, 100 + i)
        p = sb.params(3, 8, 48, r)
        jobs.append(sb.FrameJob(st, g, jit, p))
        rgb, chunk = sb.stylize(st, g, jit, p)
        expect.append((rgb, chunk))
    torch.cuda.synchronize()
    for tune in [None, (2, 16, 4, 1)]:
        say(f"mixed radii batch tune={tune}")
        b = sb.Batch(use_graph=True, tune=tune)
        b.run(jobs)
        torch.cuda.synchronize()
        for j, (rgb, chunk) in zip(jobs, expect):
            np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), rgb.cpu().numpy(),
                                          err_msg=f"r={j.params.radius}")
            np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), chunk.cpu().numpy())
        b.close()


def test_batch_deep_hierarchy_matches_oracle(sb):
    """A batch frame with 9 levels (9 L > 64 seed records per block, so the
    second record per lane) next to a shallow one, against the oracle."""
    import torch

    rng = np.random.default_rng(909)
    st_np = workloads.Style(workloads.value_noise_rgb(96, 80, 5), workloads.sphere_guide_u8(96)[:80],
                            0, 8)
    style = sb.Style(st_np.rgb, st_np.guide, st_np.lut_bits)
    lut = oracle.lut_build(st_np.guide, st_np.lut_bits)
    cases = [(301, 177, 9, 8, 90, 2), (150, 90, 3, 8, 40, 1)]
    jobs, want = [], []
    for w, h, levels, finest, t, r in cases:
        g = rng.integers(0, 256, size=(h, w, 2), dtype=np.uint8)
        jit = workloads.jitter_table(w, h, levels, finest, w + h)
        jobs.append(sb.FrameJob(style, g, jit, sb.params(levels, finest, t, r)))
        want.append(oracle.stylize(st_np.rgb, st_np.guide, lut, st_np.lut_bits, g, jit, levels,
                                   finest, t, r))
    b = sb.Batch(use_graph=True)
    say("batch with a 9-level frame")
    b.run(jobs)
    torch.cuda.synchronize()
    for k, (j, (e_rgb, e_chunk, _)) in enumerate(zip(jobs, want)):
        np.testing.assert_array_equal(j.out_chunk.cpu().numpy().view(np.uint32), e_chunk,
                                      err_msg=f"frame {k} chunk")
        np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), e_rgb, err_msg=f"frame {k} rgb")
    b.close()


@pytest.mark.parametrize("tune,bpc", [(None, 0), ((4, 8, 2, 2), 16), ((2, 16, 4, 1), 4)])
def test_full_workload_batch(sb, tune, bpc):
    """The whole 64-frame mix of uneven sizes (half normal-guided, half
    UV-guided, four styles) as one batch, as the benchmark runs it: every
    frame equals its single-frame launch, and eight frames of both guide
    formats equal the oracle."""
    import torch

    styles_np, frames_np = workloads.config(4)
    assert len(frames_np) == 64
    styles = [sb.Style(s.rgb, s.guide, s.lut_bits) for s in styles_np]
    idx = list(range(64))
    jobs = jobs_for(sb, styles, frames_np, idx)
    b = sb.Batch(use_graph=True, tune=tune, blocks_per_cu=bpc)
    say(f"full 64-frame batch tune={tune} blocks_per_cu={bpc}")
    b.run(jobs)
    torch.cuda.synchronize()
    for i, j in zip(idx, jobs):
        rgb, chunk = single(sb, styles, frames_np[i])
        np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), rgb, err_msg=f"frame {i} rgb")
        np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), chunk, err_msg=f"frame {i} chunk")
    if tune is None:
        luts = {}
        for i in [0, 5, 17, 31, 32, 40, 51, 63]:
            f = frames_np[i]
            st = styles_np[f.style]
            p = f.params
            say(f"oracle frame {i} {f.w}x{f.h} fmt={f.fmt}")
            if f.style not in luts:
                luts[f.style] = oracle.lut_build(st.guide, st.lut_bits)
            e_rgb, e_chunk, _ = oracle.stylize(st.rgb, st.guide, luts[f.style], st.lut_bits,
                                               f.guide, None, p.levels, p.finest, p.threshold,
                                               p.radius, seed=f.seed)
            np.testing.assert_array_equal(jobs[i].out_chunk.cpu().numpy().view(np.uint32),
                                          e_chunk, err_msg=f"frame {i} chunk")
            np.testing.assert_array_equal(jobs[i].out_rgb.cpu().numpy(), e_rgb,
                                          err_msg=f"frame {i} rgb")
    b.close()


def test_stylize_frames_equals_single(sb, mix):
    """sb_stylize_frames (the per-frame baseline of the batch bench: all
    frames through the per-frame kernels from one call, one shared
    workspace) gives every frame exactly what a lone sb_stylize gives, under
    the default and a non-default kernel choice."""
    import torch

    styles_np, frames_np, styles = mix
    idx = list(range(len(frames_np)))
    for tune in (None, (2, 16, 4, 1, 1)):
        say(f"stylize_frames {len(idx)} frames tune={tune}")
        jobs = jobs_for(sb, styles, frames_np, idx)
        sb.stylize_frames(jobs, tune=tune)
        torch.cuda.synchronize()
        for i, j in zip(idx, jobs):
            rgb, chunk = single(sb, styles, frames_np[i])
            np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), chunk, err_msg=f"frame {i}")
            np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), rgb, err_msg=f"frame {i}")
