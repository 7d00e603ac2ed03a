"""The animation extension (Sec. 3.3) on the GPU: frames of an animated
target with a per-frame seed schedule, equal to the oracle bit for bit; the
frame-to-frame change counts of sb_frame_change equal the oracle's; served
sessions complete in order and every frame equals the frame stylised alone
(tolerance 0 throughout: the outputs and counts are integers)."""
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
    import paper_1807_03249_amd as sb

    return sb


@pytest.fixture(scope="module")
def style1():
    return workloads.config(1)[0][0]


def _seq(w, h, nframes, hold, seed):
    p = workloads.config(1)[1][0].params
    guides = workloads.animated_bump_guides(w, h, 6, nframes, 2.0, seed)
    jits = workloads.jitter_schedule(w, h, p.levels, p.finest, nframes, hold, seed + 1)
    return guides, jits, p


@pytest.mark.parametrize("w,h,hold,t", [(200, 136, 1, 48), (200, 136, 2, 400), (97, 61, 1, 2000)])
def test_sequence_and_changes_match_oracle(sb, style1, w, h, hold, t):
    import torch

    say(f"animated sequence {w}x{h} hold={hold} t={t}")
    st = style1
    guides, jits, p = _seq(w, h, 5, hold, 70 + w)
    style = sb.Style(st.rgb, st.guide, st.lut_bits)
    prm = sb.params(p.levels, p.finest, t, p.radius)
    lut = oracle.lut_build(st.guide, st.lut_bits)
    got, want = [], []
    for g, j in zip(guides, jits):
        rgb, chunk, nnf = sb.stylize(style, g, j, prm, want_nnf=True)
        torch.cuda.synchronize()
        got.append((rgb, chunk, nnf))
        want.append(oracle.stylize(st.rgb, st.guide, lut, st.lut_bits, g, j, p.levels, p.finest,
                                   t, p.radius))
    for k, ((rgb, chunk, nnf), (orgb, ochunk, onnf)) in enumerate(zip(got, want)):
        np.testing.assert_array_equal(rgb.cpu().numpy(), orgb, err_msg=f"frame {k}")
        np.testing.assert_array_equal(chunk.cpu().numpy().view(np.uint32), ochunk,
                                      err_msg=f"frame {k}")
        np.testing.assert_array_equal(nnf.cpu().numpy().view(np.uint32), onnf,
                                      err_msg=f"frame {k}")
    for k in range(len(got) - 1):
        a, b = got[k], got[k + 1]
        c = sb.frame_change(a[1], b[1], a[2], b[2]).cpu().numpy()
        assert tuple(int(x) for x in c) == oracle.frame_change(want[k][1], want[k + 1][1],
                                                               want[k][2], want[k + 1][2])
        c = sb.frame_change(a[1], b[1]).cpu().numpy()
        assert tuple(int(x) for x in c) == oracle.frame_change(want[k][1], want[k + 1][1])


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 1021, 4 * 256 * 1024 * 4 + 13])
@pytest.mark.parametrize("offset", [0, 1])
def test_frame_change_sizes_and_alignment(sb, n, offset):
    """Ragged tails, empty and single-pixel maps, maps larger than one
    grid-stride pass, and maps that are only 4-byte aligned (scalar path)."""
    import torch

    say(f"frame_change n={n} offset={offset}")
    rng = np.random.default_rng(n + 17 * offset)
    maps = [rng.integers(0, 3, n + offset).astype(np.uint32) for _ in range(4)]
    dev = [torch.from_numpy(m.view(np.int32)).cuda()[offset:] for m in maps]
    c = sb.frame_change(dev[0], dev[1], dev[2], dev[3]).cpu().numpy()
    want = oracle.frame_change(maps[0][offset:], maps[1][offset:], maps[2][offset:],
                               maps[3][offset:])
    assert (int(c[0]), int(c[1])) == want
    c = sb.frame_change(dev[0], dev[1]).cpu().numpy()
    assert (int(c[0]), int(c[1])) == (want[0], 0)


def test_frame_change_rejects_bad_arguments(sb):
    import torch

    a = torch.zeros(16, dtype=torch.int32, device="cuda")
    L = sb.lib()
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    ws = torch.empty(L.sb_change_workspace_bytes(), dtype=torch.uint8, device="cuda")
    p = a.data_ptr()
    assert L.sb_frame_change(p, p, p, None, 16, cnt.data_ptr(), ws.data_ptr(), ws.numel(),
                             None) == sb.SB_EINVAL
    assert L.sb_frame_change(p, p, None, None, -1, cnt.data_ptr(), ws.data_ptr(), ws.numel(),
                             None) == sb.SB_EINVAL
    assert L.sb_frame_change(p, p, None, None, 16, cnt.data_ptr(), ws.data_ptr(), 8,
                             None) == sb.SB_ENOMEM


def test_sessions_complete_in_order_and_match_alone(sb):
    """Four sessions of eight frames each, all arriving at once, interleaved
    frame by frame; batches of two over four slots put consecutive frames of
    a session on different slots, so the session order needs the
    cross-slot waits."""
    import torch
    import paper_1807_03249_amd.serve as sv

    styles, frames = workloads.config(1)
    st = styles[0]
    style = sb.Style(st.rgb, st.guide, st.lut_bits)
    p = frames[0].params
    prm = sb.params(p.levels, p.finest, p.threshold, p.radius)
    sizes = [(640, 360), (320, 200), (200, 136), (1280, 720)]
    nf = 8
    seqs = []
    for s, (w, h) in enumerate(sizes):
        g, j, _ = _seq(w, h, nf, 1, 300 + s)
        seqs.append(([torch.from_numpy(x).cuda() for x in g],
                     [torch.from_numpy(x.view(np.int32)).cuda() for x in j]))
    reqs = []
    for k in range(nf):
        for s, (w, h) in enumerate(sizes):
            reqs.append(sv.Request(0.0, style, seqs[s][0][k], seqs[s][1][k], prm,
                                   torch.empty((h, w, 3), dtype=torch.uint8, device="cuda"),
                                   torch.empty((h, w), dtype=torch.int32, device="cuda"),
                                   torch.empty((h, w), dtype=torch.int32, device="cuda"),
                                   session=s))
    say(f"serve {len(reqs)} session frames, 4 slots, batches of 2")
    out = sv.run(reqs, slots=4, max_batch=2, budget_bytes=1 << 30)
    assert np.all(out["status"] == sb.SB_OK)
    moved = 0
    for s in range(len(sizes)):
        idx = np.nonzero(out["session"] == s)[0]
        assert np.all(np.diff(out["completed"][idx]) >= 0), f"session {s} out of order"
        moved += int(np.sum(np.diff(out["slot"][idx]) != 0))
    assert moved > 0  # some consecutive frames ran on different slots
    for i, r in enumerate(reqs):
        rgb, chunk, nnf = sb.stylize(r.style, r.guide, r.jitter, r.params, want_nnf=True)
        torch.cuda.synchronize()
        assert torch.equal(r.out_rgb, rgb), f"request {i}"
        assert torch.equal(r.out_chunk, chunk), f"request {i}"
        assert torch.equal(r.out_nnf, nnf), f"request {i}"


def test_plain_serving_keeps_nnf_and_sessions(sb):
    import torch
    import paper_1807_03249_amd.serve as sv

    styles, frames = workloads.config(1)
    st = styles[0]
    style = sb.Style(st.rgb, st.guide, st.lut_bits)
    p = frames[0].params
    prm = sb.params(p.levels, p.finest, p.threshold, p.radius)
    g, j, _ = _seq(200, 136, 4, 1, 400)
    reqs = [sv.Request(0.0, style, torch.from_numpy(x).cuda(),
                       torch.from_numpy(y.view(np.int32)).cuda(), prm,
                       torch.empty((136, 200, 3), dtype=torch.uint8, device="cuda"),
                       torch.empty((136, 200), dtype=torch.int32, device="cuda"),
                       torch.empty((136, 200), dtype=torch.int32, device="cuda"), session=0)
            for x, y in zip(g, j)]
    say("plain serving of one session")
    out = sv.run(reqs, plain=True)
    assert np.all(out["status"] == sb.SB_OK)
    assert np.all(np.diff(out["completed"]) >= 0)
    for r in reqs:
        rgb, chunk, nnf = sb.stylize(r.style, r.guide, r.jitter, r.params, want_nnf=True)
        torch.cuda.synchronize()
        assert torch.equal(r.out_nnf, nnf)


@pytest.mark.parametrize("w,h,levels,finest,seed,stream", [
    (200, 136, 4, 8, 1, 0), (97, 61, 3, 4, 2**64 - 1, 2**63), (3840, 2160, 5, 8, 42, 7),
    (1, 1, 1, 1, 5, 5), (64, 64, 0, 8, 1, 1)])
def test_device_jitter_matches_oracle(sb, w, h, levels, finest, seed, stream):
    import torch

    say(f"device jitter {w}x{h} L={levels} f={finest} seed={seed} stream={stream}")
    j = sb.jitter_fill(w, h, levels, finest, seed, stream)
    torch.cuda.synchronize()
    n = sb.jitter_len(w, h, levels, finest)
    np.testing.assert_array_equal(j.cpu().numpy().view(np.uint32)[:n],
                                  oracle.jitter_fill(w, h, levels, finest, seed, stream))


def test_frames_with_device_seed_schedule(sb, style1):
    """An animated sequence whose per-frame jitter comes from the device
    generator (seed fixed, stream = frame index / hold) equals the oracle fed
    the oracle's tables."""
    import torch

    st = style1
    w, h, hold = 160, 120, 2
    p = workloads.config(1)[1][0].params
    guides = workloads.animated_bump_guides(w, h, 5, 4, 2.0, 91)
    style = sb.Style(st.rgb, st.guide, st.lut_bits)
    lut = oracle.lut_build(st.guide, st.lut_bits)
    prm = sb.params(p.levels, p.finest, p.threshold, p.radius)
    for f, g in enumerate(guides):
        say(f"device seed schedule frame {f}")
        j = sb.jitter_fill(w, h, p.levels, p.finest, 1234, f // hold)
        rgb, chunk = sb.stylize(style, g, j, prm)
        torch.cuda.synchronize()
        e = oracle.stylize(st.rgb, st.guide, lut, st.lut_bits, g,
                           oracle.jitter_fill(w, h, p.levels, p.finest, 1234, f // hold),
                           p.levels, p.finest, p.threshold, p.radius)
        np.testing.assert_array_equal(chunk.cpu().numpy().view(np.uint32), e[1])
        np.testing.assert_array_equal(rgb.cpu().numpy(), e[0])
