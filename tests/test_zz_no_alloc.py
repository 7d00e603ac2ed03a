"""sb_stylize_noalloc (static scratch, no workspace) against sb_stylize, bit
for bit, through the C ABI: three calls in a row on one device, each smaller
than the one before, so each call runs over the previous call's leftovers in
the shared scratch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _case(n):
    import workloads

    styles, frames = workloads.config(n)
    return styles[frames[0].style], frames[0]


def test_noalloc_matches_stylize_on_shrinking_frames():
    import torch

    import paper_1807_03249_amd as sb

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    for n in (3, 2, 1):  # 3840x2160 UV, 1920x1080 normal, 256x256 normal
        st_np, fr = _case(n)
        p = fr.params
        say(f"noalloc: workload {n} {fr.w}x{fr.h} L={p.levels} t={p.threshold} r={p.radius}")
        style = sb.Style(st_np.rgb, st_np.guide, st_np.lut_bits)
        prm = sb.params(p.levels, p.finest, p.threshold, p.radius, seed=fr.seed)
        g = fr.guide.view("int16") if fr.guide.dtype == np.uint16 else fr.guide
        guide = torch.from_numpy(np.ascontiguousarray(g)).cuda()
        e_rgb, e_chunk, e_nnf = sb.stylize(style, guide, None, prm, want_nnf=True)
        rgb = torch.full((fr.h, fr.w, 3), 7, dtype=torch.uint8, device="cuda")
        chunk = torch.full((fr.h, fr.w), -1, dtype=torch.int32, device="cuda")
        nnf = torch.full((fr.h, fr.w), -1, dtype=torch.int32, device="cuda")
        sb.stylize_noalloc(style, guide, None, prm, rgb, chunk, nnf)
        torch.cuda.synchronize()
        assert torch.equal(chunk, e_chunk), f"workload {n}: chunk map differs"
        assert torch.equal(nnf, e_nnf), f"workload {n}: nnf differs"
        assert torch.equal(rgb, e_rgb), f"workload {n}: rgb differs"


def test_noalloc_table_jitter_and_repeat():
    """A drawn jitter table (SB_JITTER_TABLE) with finest spacing 4, so the
    seed pass fills the scratch's seed table and the per-pixel level loop
    reads it: twice in a row on the same frame, then a smaller frame."""
    import torch

    import paper_1807_03249_amd as sb
    import workloads

    st_np, fr = _case(2)
    p = fr.params
    style = sb.Style(st_np.rgb, st_np.guide, st_np.lut_bits)
    for (w, h) in ((fr.w, fr.h), (fr.w, fr.h), (333, 77)):
        say(f"noalloc table jitter {w}x{h}")
        g = torch.from_numpy(np.ascontiguousarray(fr.guide[:h, :w])).cuda()
        jt = workloads.jitter_table(w, h, p.levels, 4, 11)
        jd = torch.from_numpy(jt.view(np.int32)).cuda()
        prm = sb.params(p.levels, 4, p.threshold, p.radius)
        e_rgb, e_chunk = sb.stylize(style, g, jd, prm)
        rgb = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
        chunk = torch.empty((h, w), dtype=torch.int32, device="cuda")
        sb.stylize_noalloc(style, g, jd, prm, rgb, chunk)
        torch.cuda.synchronize()
        assert torch.equal(chunk, e_chunk)
        assert torch.equal(rgb, e_rgb)
