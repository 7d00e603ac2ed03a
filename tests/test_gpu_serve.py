"""Serving on the GPU: a Poisson request trace through the native request
loop (memory-budget admission, continuous batching over several streams).
Each request's result in the mix must equal the same request stylised alone
and, for a sample, the oracle (tolerance 0: the outputs are integers)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1807_03249_amd as sb
    import paper_1807_03249_amd.serve as sv

    trace = workloads.config(5, requests=48, qps=3000.0, pool=1)
    styles = [sb.Style(s.rgb, s.guide, s.lut_bits) for s in trace["styles"]]
    return sb, sv, trace, styles


def make_requests(env, explicit_outputs, n=None, burst=False):
    """Requests of the trace: every fourth with its own jitter table, the
    rest with their own jitter hash seed.  ``burst``: all arrive at once, so
    the free slots take batches of several requests and run side by side."""
    import torch

    sb, sv, trace, styles = env
    reqs = []
    guides = {}
    n = n or len(trace["arrivals"])
    for i in range(n):
        si, st = int(trace["size_idx"][i]), int(trace["style_idx"][i])
        fmt = trace["styles"][st].fmt
        key = (si, fmt, int(trace["pool_idx"][i]))
        if key not in guides:
            g = trace["guides"][key]
            g = g.view(np.int16) if g.dtype == np.uint16 else g
            guides[key] = torch.from_numpy(g).cuda()
        g = guides[key]
        h, w = int(g.shape[0]), int(g.shape[1])
        p = trace["params"][fmt]
        if i % 4 == 0:
            jit = workloads.jitter_table(w, h, p.levels, p.finest, 9000 + i)
            jt = torch.from_numpy(jit.view(np.int32)).cuda()
            prm = sb.params(p.levels, p.finest, p.threshold, p.radius)
        else:
            jt = None
            prm = sb.params(p.levels, p.finest, p.threshold, p.radius,
                            seed=int(trace["seeds"][i]))
        out_rgb = out_chunk = None
        if explicit_outputs:
            out_rgb = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
            out_chunk = torch.empty((h, w), dtype=torch.int32, device="cuda")
        arrival = 0.0 if burst else float(trace["arrivals"][i])
        reqs.append(sv.Request(arrival, styles[st], g, jt, prm, out_rgb, out_chunk))
    return reqs


def alone(sb, r):
    import torch

    rgb, chunk = sb.stylize(r.style, r.guide, r.jitter, r.params)
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), chunk.cpu().numpy()


@pytest.mark.parametrize("plain,burst", [(False, False), (False, True), (True, False)])
def test_each_result_same_alone_and_in_mix(env, plain, burst):
    sb, sv, trace, styles = env
    reqs = make_requests(env, explicit_outputs=True, burst=burst)
    say(f"serve {len(reqs)} requests plain={plain} burst={burst}")
    out = sv.run(reqs, slots=3, max_batch=8, budget_bytes=1 << 30, plain=plain)
    assert np.all(out["status"] == sb.SB_OK)
    assert np.all(out["completed"] >= out["arrival"])
    if burst:
        # continuous batching really ran: batches of several requests, and
        # two slots' batches in flight at the same time
        assert out["batch_size"].max() > 1
        assert len(np.unique(out["batch"][out["batch_size"] > 1])) >= 2
        sl, la, co = out["slot"], out["launched"], out["completed"]
        overlap = any(sl[i] != sl[j] and la[i] < co[j] and la[j] < co[i]
                      for i in range(len(reqs)) for j in range(i + 1, len(reqs)))
        assert overlap, "no two slots were busy at once"
    for i, r in enumerate(reqs):
        rgb, chunk = alone(sb, r)
        np.testing.assert_array_equal(r.out_rgb.cpu().numpy(), rgb, err_msg=f"request {i}")
        np.testing.assert_array_equal(r.out_chunk.cpu().numpy(), chunk, err_msg=f"request {i}")


def test_budget_bounds_bytes_in_flight(env):
    sb, sv, trace, styles = env
    reqs = make_requests(env, explicit_outputs=False)
    budget = 24 << 20  # room for about one 1080p request plus a small one
    say(f"serve with a {budget >> 20} MiB budget")
    out = sv.run(reqs, slots=4, max_batch=8, budget_bytes=budget)
    assert np.all(out["status"] == sb.SB_OK)
    sizes = np.array([sv._bind().sb_frame_bytes(r.w, r.h) for r in reqs], dtype=np.int64)
    # at every admission instant, bytes admitted and not yet completed fit the budget
    for t in out["admitted"]:
        live = (out["admitted"] <= t) & (out["completed"] > t)
        assert sizes[live].sum() <= budget


def test_request_larger_than_budget_is_refused(env):
    sb, sv, trace, styles = env
    reqs = make_requests(env, explicit_outputs=False, n=16)
    budget = 4 << 20  # smaller than a 1280x720 request
    out = sv.run(reqs, slots=2, max_batch=4, budget_bytes=budget)
    sizes = np.array([sv._bind().sb_frame_bytes(r.w, r.h) for r in reqs])
    assert np.all(out["status"][sizes > budget] == sb.SB_EBUDGET)
    assert np.all(out["status"][sizes <= budget] == sb.SB_OK)


def test_mixed_guides_labels_and_sessions(env):
    """One trace mixing two-channel, three-channel (appearance) and
    segmentation-guided requests, some in sessions: every result equals the
    request run alone, and sessions complete in order."""
    import torch

    sb, sv, trace, styles = env
    s2_np = workloads.config(1)[0][0]
    s2 = sb.Style(s2_np.rgb, s2_np.guide, s2_np.lut_bits)
    s3_np = workloads.config(6, lut_bits=6, w=64, h=64)[0][0]
    s3 = sb.Style(s3_np.rgb, s3_np.guide, 6)
    ls = workloads.voronoi_labels(s2_np.sw, s2_np.sh, 4, 10, 81)
    sl = sb.Style(s2_np.rgb, s2_np.guide, s2_np.lut_bits, labels=ls, nlabels=4)
    prm = sb.params(3, 8, 64, 2)
    rng = np.random.default_rng(82)
    reqs = []
    for i in range(36):
        w, h = int(rng.integers(64, 700)), int(rng.integers(48, 500))
        kind = i % 3
        if kind == 0:
            st, g, lab = s2, workloads.bump_guide_u8(w, h, 4, 900 + i), None
        elif kind == 1:
            st, g, lab = s3, workloads.appearance_target(w, h, 4, 900 + i), None
        else:
            st, g = sl, workloads.bump_guide_u8(w, h, 4, 900 + i)
            lab = torch.from_numpy(workloads.voronoi_labels(w, h, 5, 8, 950 + i)).cuda()
        jit = torch.from_numpy(workloads.jitter_table(w, h, 3, 8, 990 + i).view(np.int32)).cuda()
        reqs.append(sv.Request(i * 2e-5, st, torch.from_numpy(g).cuda(), jit, prm,
                               torch.empty((h, w, 3), dtype=torch.uint8, device="cuda"),
                               torch.empty((h, w), dtype=torch.int32, device="cuda"),
                               torch.empty((h, w), dtype=torch.int32, device="cuda"),
                               session=(i % 4) if i < 24 else -1, tgt_labels=lab))
    say("serve 36 mixed requests (two/three channels, labels, sessions)")
    out = sv.run(reqs, slots=3, max_batch=4, budget_bytes=1 << 30)
    assert np.all(out["status"] == sb.SB_OK)
    for s in range(4):
        idx = np.nonzero(out["session"] == s)[0]
        assert np.all(np.diff(out["completed"][idx]) >= 0)
    for i, r in enumerate(reqs):
        rgb, chunk, nnf = sb.stylize(r.style, r.guide, r.jitter, r.params, want_nnf=True,
                                     tgt_labels=r.tgt_labels)
        torch.cuda.synchronize()
        assert torch.equal(r.out_rgb, rgb), f"request {i}"
        assert torch.equal(r.out_chunk, chunk), f"request {i}"
        assert torch.equal(r.out_nnf, nnf), f"request {i}"


def test_served_results_match_oracle(env):
    """A burst through the batched loop; a sample of the served frames (both
    guide formats, every size, table and hash jitter) against the oracle."""
    sb, sv, trace, styles = env
    reqs = make_requests(env, explicit_outputs=True, burst=True)
    say(f"serve {len(reqs)} requests in a burst, sample against the oracle")
    out = sv.run(reqs, slots=3, max_batch=8, budget_bytes=1 << 30)
    assert np.all(out["status"] == sb.SB_OK)
    assert out["batch_size"].max() > 1
    picked = {}
    for i in range(len(reqs)):
        key = (int(trace["size_idx"][i]), trace["styles"][int(trace["style_idx"][i])].fmt, i % 4 == 0)
        picked.setdefault(key, i)
    luts = {}
    for i in sorted(picked.values()):
        r = reqs[i]
        st_i = int(trace["style_idx"][i])
        st = trace["styles"][st_i]
        p = trace["params"][st.fmt]
        g = trace["guides"][(int(trace["size_idx"][i]), st.fmt, int(trace["pool_idx"][i]))]
        jit = r.jitter.cpu().numpy().view(np.uint32) if r.jitter is not None else None
        seed = None if r.jitter is not None else int(trace["seeds"][i])
        if st_i not in luts:
            luts[st_i] = oracle.lut_build(st.guide, st.lut_bits)
        say(f"oracle request {i} {r.w}x{r.h} fmt={st.fmt} table={jit is not None} "
            f"batch_size={out['batch_size'][i]}")
        e_rgb, e_chunk, _ = oracle.stylize(st.rgb, st.guide, luts[st_i], st.lut_bits, g, jit,
                                           p.levels, p.finest, p.threshold, p.radius, seed=seed)
        np.testing.assert_array_equal(r.out_chunk.cpu().numpy().view(np.uint32), e_chunk,
                                      err_msg=f"request {i} chunk")
        np.testing.assert_array_equal(r.out_rgb.cpu().numpy(), e_rgb, err_msg=f"request {i} rgb")


def test_many_channel_requests_run_alone(env):
    """Requests of a many-channel style (exact search) mixed into a burst of
    table-format requests: each runs in a batch of its own, and every result
    equals the request stylised alone."""
    import torch

    sb, sv, trace, styles = env
    reqs = make_requests(env, explicit_outputs=True, n=24, burst=True)
    st_np = workloads.config(7, w=64, h=64, size=64)[0][0]
    sst = sb.Style(st_np.rgb, st_np.guide, channels=5)
    rng = np.random.default_rng(61)
    p = workloads.FEATURE_PARAMS
    prm = sb.params(p.levels, p.finest, p.threshold, p.radius, seed=5)
    many = []
    for i in range(8):
        w, h = int(rng.integers(100, 400)), int(rng.integers(80, 300))
        g = torch.from_numpy(workloads.features_target(w, h, 640 + i, 8, st_np.rgb)).cuda()
        many.append(sv.Request(0.0, sst, g, None, prm,
                               torch.empty((h, w, 3), dtype=torch.uint8, device="cuda"),
                               torch.empty((h, w), dtype=torch.int32, device="cuda")))
    mixed = []
    for i, r in enumerate(reqs):
        mixed.append(r)
        if i % 3 == 0 and many:
            mixed.append(many.pop())
    say(f"serve {len(mixed)} requests, some of a many-channel style")
    out = sv.run(mixed, slots=3, max_batch=8, budget_bytes=1 << 30)
    assert np.all(out["status"] == sb.SB_OK)
    assert out["batch_size"].max() > 1
    for i, r in enumerate(mixed):
        if r.style is sst:
            assert out["batch_size"][i] == 1
        rgb, chunk = sb.stylize(r.style, r.guide, r.jitter, r.params)
        torch.cuda.synchronize()
        assert torch.equal(r.out_rgb, rgb), f"request {i}"
        assert torch.equal(r.out_chunk, chunk), f"request {i}"
