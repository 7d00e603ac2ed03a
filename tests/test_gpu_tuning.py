"""Kernel choices on the GPU: the timed entry point and the autotuner.
Every choice must give the same bits (tolerance 0), and the tuner may only
pick a choice whose outputs it checked against the default's."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1807_03249_amd as sb

    styles, frames = workloads.config(1)
    st, fr = styles[0], frames[0]
    style = sb.Style(st.rgb, st.guide, st.lut_bits)
    p = fr.params
    return sb, style, fr, sb.params(p.levels, p.finest, p.threshold, p.radius, seed=fr.seed)


def test_timed_entry_matches_plain_and_orders_events(env):
    import torch

    sb, style, fr, prm = env
    say("sb_stylize_timed vs sb_stylize")
    ref_rgb, ref_chunk = sb.stylize(style, fr.guide, fr.jitter, prm)
    ev = sb.TimingEvents()
    rgb, chunk = sb.stylize(style, fr.guide, fr.jitter, prm, events=ev, tune=(2, 8, 4, 2))
    torch.cuda.synchronize()
    assert torch.equal(rgb, ref_rgb) and torch.equal(chunk, ref_chunk)
    d = ev.pass_ms()
    assert all(x >= 0 for x in d), d
    assert ev.elapsed_ms(0, 3) >= max(d)
    ev.close()


def test_tune_frame_picks_an_exact_choice(env, tmp_path):
    import paper_1807_03249_amd.autotune as at

    sb, style, fr, prm = env
    cache = str(tmp_path / "tune.json")
    say("tune_frame")
    r = at.tune_frame(style, fr.guide, fr.jitter, prm, reps=3, cache_path=cache)
    assert not r["cached"]
    assert set(r["candidates"]) == {",".join(map(str, t)) for t in sb.TUNES}
    assert all(v["exact"] for v in r["candidates"].values())
    assert tuple(r["tune"]) in sb.TUNES
    r2 = at.tune_frame(style, fr.guide, fr.jitter, prm, reps=3, cache_path=cache)
    assert r2["cached"] and tuple(r2["tune"]) == tuple(r["tune"])


def test_tune_batch_picks_an_exact_choice(env, tmp_path):
    import torch

    import paper_1807_03249_amd.autotune as at

    sb = env[0]
    styles_np, frames_np = workloads.config(4, frames=6)
    styles = [sb.Style(s.rgb, s.guide, s.lut_bits) for s in styles_np]
    jobs = []
    for f in frames_np:
        p = f.params
        jobs.append(sb.FrameJob(styles[f.style], f.guide, f.jitter,
                                sb.params(p.levels, p.finest, p.threshold, p.radius, seed=f.seed)))
    say(f"tune_batch over {len(jobs)} frames")
    r = at.tune_batch(jobs, candidates=[(4, 16, 2, 1), (2, 8, 4, 2)], blocks_per_cu=(2, 8), reps=2,
                      cache_path=str(tmp_path / "tune.json"))
    assert all(v["exact"] for v in r["candidates"].values()), r["candidates"]
    b = sb.Batch(use_graph=True, tune=r["tune"], blocks_per_cu=r["blocks_per_cu"])
    b.run(jobs)
    torch.cuda.synchronize()
    for j in jobs:
        rgb, chunk = sb.stylize(j.style, j.guide, j.jitter, j.params)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(j.out_rgb.cpu().numpy(), rgb.cpu().numpy())
        np.testing.assert_array_equal(j.out_chunk.cpu().numpy(), chunk.cpu().numpy())
    b.close()
