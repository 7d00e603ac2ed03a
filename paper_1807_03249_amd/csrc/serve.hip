// serve.hip -- a request loop with HBM-budget admission and continuous
// batching on top of the batch plans.
//
// One host thread runs the whole trace.  Each turn it
//   1. moves requests whose arrival time has passed to the pending queue;
//   2. admits pending requests in arrival order while their output bytes fit
//      in the device arena (the memory budget); a request larger than the
//      whole arena is refused with SB_EBUDGET;
//   3. retires finished batches (event query), freeing their arena bytes and
//      their slot;
//   4. gives every free slot (its own stream, batch plan and workspace) all
//      admitted requests up to max_batch, launched as one graph replay (a
//      single request takes the per-frame kernels on the slot's stream).
//      When a request belongs to a session (the frames of one animation)
//      whose previous frame still runs on another slot, the slot's stream
//      first waits for that slot's batch, so a session's frames complete in
//      order.
// Requests that arrive while batches run are admitted as memory frees up and
// start on the next free slot, so their work overlaps batches already on the
// device.  The plain mode launches every request alone on one stream, in
// arrival order, as the baseline.
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "sb_internal.h"

namespace sb {
namespace {

// First-fit allocator over [0, size) of the arena, 256-byte granules.
class Arena {
 public:
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t *off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

size_t out_bytes(int32_t w, int32_t h) {
  return ((size_t(w) * h * 3 + 255) & ~size_t(255)) + size_t(w) * h * 4;
}

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  sb_batch *plan = nullptr;
  void *workspace = nullptr;
  bool busy = false;
  int32_t batch = -1;  // id of the batch in flight
  std::vector<int32_t> reqs;
};

// One frame through the per-frame entry points (with the segmentation guide
// when the frame carries target labels).
int run_one(const sb_frame &f, void *ws, size_t ws_bytes, const sb_tune *tune, hipStream_t s) {
  if (f.tgt_labels)
    return sb_stylize_seg(f.style, f.tgt_guide, f.tgt_labels, f.w, f.h, f.jitter, &f.params,
                          f.out_rgb, f.out_chunk, f.out_nnf, ws, ws_bytes, tune, s);
  return sb_stylize_ex(f.style, f.tgt_guide, f.w, f.h, f.jitter, &f.params, f.out_rgb,
                       f.out_chunk, f.out_nnf, ws, ws_bytes, tune, s);
}

// Where the latest launched frame of a session runs.
struct SessionTail {
  int32_t slot, batch;
};

}  // namespace
}  // namespace sb

using namespace sb;

extern "C" {

size_t sb_frame_bytes(int32_t w, int32_t h) {
  if (w < 1 || h < 1 || w > SB_MAX_SIDE || h > SB_MAX_SIDE) return 0;
  return out_bytes(w, h);
}

int sb_serve_run(const sb_serve_config *cfg, const sb_request *reqs, int32_t n,
                 sb_request_result *res) {
  if (!cfg || !reqs || !res || n < 1) return SB_EINVAL;
  if (!cfg->arena || cfg->arena_bytes < 256) return SB_EINVAL;
  const bool plain = cfg->plain != 0;
  const int32_t slots = plain ? 1 : cfg->slots;
  const int32_t maxb = plain ? 1 : cfg->max_batch;
  if (slots < 1 || slots > 8 || maxb < 1 || maxb > sb_batch_max_frames()) return SB_EINVAL;
  if (!plain && (!cfg->desc_dev || !cfg->desc_host || !cfg->workspace)) return SB_EINVAL;
  if (!cfg->workspace) return SB_EINVAL;
  Tune tune;
  if (!resolve_tune(&cfg->tune, &tune)) return SB_EINVAL;
  if (cfg->blocks_per_cu < 0 || cfg->blocks_per_cu > 16) return SB_EINVAL;
  for (int32_t i = 0; i < n; ++i) {
    const sb_request &r = reqs[i];
    FrameArgs a;
    uint8_t *probe_rgb = r.out_rgb ? r.out_rgb : reinterpret_cast<uint8_t *>(1);
    uint32_t *probe_chunk = r.out_chunk ? r.out_chunk : reinterpret_cast<uint32_t *>(1);
    if (!fill_frame(r.style, r.tgt_guide, r.w, r.h, r.jitter, &r.params, probe_rgb, probe_chunk,
                    nullptr, &a, r.tgt_labels))
      return SB_EINVAL;
    if (i > 0 && r.arrival_s < reqs[i - 1].arrival_s) return SB_EINVAL;  // sorted arrivals
    if ((r.out_rgb == nullptr) != (r.out_chunk == nullptr)) return SB_EINVAL;  // both or neither
    // a batch of max_batch requests of this size must fit one slot's workspace
    if (sb_workspace_bytes(r.w, r.h, &r.params) * size_t(maxb) + 256 * size_t(maxb) >
        cfg->workspace_bytes_per_slot)
      return SB_ENOMEM;
    memset(&res[i], 0, sizeof res[i]);
    res[i].status = 1;  // not finished
  }

  std::vector<Slot> sl(static_cast<size_t>(slots));
  hipError_t e = hipSuccess;
  for (int32_t s = 0; s < slots && e == hipSuccess; ++s) {
    e = hipStreamCreateWithFlags(&sl[s].stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl[s].done, hipEventDisableTiming);
    sl[s].workspace = static_cast<char *>(cfg->workspace) + size_t(s) * cfg->workspace_bytes_per_slot;
    if (e == hipSuccess && !plain) {
      const int rc = sb_batch_create(static_cast<char *>(cfg->desc_dev) + s * sb_batch_desc_bytes(),
                                     static_cast<char *>(cfg->desc_host) + s * sb_batch_desc_bytes(),
                                     cfg->use_graph, &cfg->tune, cfg->blocks_per_cu, sl[s].stream,
                                     &sl[s].plan);
      if (rc != SB_OK) e = hipErrorUnknown;
    }
  }
  // plain mode: one event per launch, retired in order
  std::vector<hipEvent_t> pev;
  if (e == hipSuccess && plain) {
    pev.resize(256);
    for (auto &ev : pev)
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  }

  Arena arena(cfg->arena_bytes);
  std::vector<size_t> aoff(static_cast<size_t>(n), 0);
  std::vector<sb_frame> fr(static_cast<size_t>(n));
  std::deque<int32_t> pending, admitted, plain_inflight;
  std::map<int32_t, SessionTail> tails;  // session -> slot and batch of its latest frame
  std::vector<Slot *> done;               // slots found finished in one polling pass
  done.reserve(sl.size());
  int32_t next = 0, finished = 0, batch_id = 0, rc = SB_OK;
  const auto t0 = std::chrono::steady_clock::now();
  auto finish = [&](int32_t i, double t) {
    res[i].completed_s = t;
    res[i].status = SB_OK;
    if (!reqs[i].out_rgb) arena.release(aoff[i], out_bytes(reqs[i].w, reqs[i].h));
    ++finished;
  };

  while (e == hipSuccess && rc == SB_OK && finished < n) {
    const double t = now_s(t0);
    while (next < n && reqs[next].arrival_s <= t) pending.push_back(next++);
    // admission by memory budget, in arrival order
    while (!pending.empty()) {
      const int32_t i = pending.front();
      const sb_request &r = reqs[i];
      if (!r.out_rgb) {
        const size_t need = out_bytes(r.w, r.h);
        if (need > cfg->arena_bytes) {  // can never fit
          res[i].status = SB_EBUDGET;
          res[i].completed_s = now_s(t0);
          ++finished;
          pending.pop_front();
          continue;
        }
        if (!arena.alloc(need, &aoff[i])) break;
      }
      sb_frame &f = fr[i];
      f.style = r.style;
      f.tgt_guide = r.tgt_guide;
      f.jitter = r.jitter;
      f.w = r.w;
      f.h = r.h;
      f.params = r.params;
      char *base = static_cast<char *>(cfg->arena) + aoff[i];
      f.out_rgb = r.out_rgb ? r.out_rgb : reinterpret_cast<uint8_t *>(base);
      f.out_chunk = r.out_chunk ? r.out_chunk
                                : reinterpret_cast<uint32_t *>(
                                      base + ((size_t(r.w) * r.h * 3 + 255) & ~size_t(255)));
      f.out_nnf = r.out_nnf;
      f.tgt_labels = r.tgt_labels;
      res[i].admitted_s = now_s(t0);
      admitted.push_back(i);
      pending.pop_front();
    }
    // retire finished work
    if (plain) {
      while (!plain_inflight.empty()) {
        const int32_t i = plain_inflight.front();
        const hipError_t q = hipEventQuery(pev[size_t(res[i].batch) % pev.size()]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
          e = q;
          break;
        }
        finish(i, now_s(t0));
        plain_inflight.pop_front();
      }
    } else {
      // query every slot first, then retire them at one time stamp: a slot
      // that waited for another completes after it, and the two must not be
      // stamped in the opposite order
      done.clear();
      for (auto &s : sl) {
        if (!s.busy) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
          e = q;
          break;
        }
        done.push_back(&s);
      }
      const double tc = now_s(t0);
      for (Slot *s : done) {
        for (int32_t i : s->reqs) finish(i, tc);
        s->reqs.clear();
        s->busy = false;
        s->batch = -1;
      }
    }
    // launch: continuous batching over free slots
    if (plain) {
      while (!admitted.empty() && plain_inflight.size() < pev.size()) {
        const int32_t i = admitted.front();
        const sb_frame &f = fr[i];
        const int r = run_one(f, sl[0].workspace, cfg->workspace_bytes_per_slot, &cfg->tune,
                              sl[0].stream);
        if (r != SB_OK) {
          rc = r;
          break;
        }
        res[i].batch = batch_id++;
        res[i].launched_s = now_s(t0);
        res[i].batch_size = 1;
        e = hipEventRecord(pev[size_t(res[i].batch) % pev.size()], sl[0].stream);
        admitted.pop_front();
        plain_inflight.push_back(i);
      }
    } else {
      for (int32_t s = 0; s < slots && !admitted.empty(); ++s) {
        Slot &S = sl[size_t(s)];
        if (S.busy) continue;
        std::vector<sb_frame> bf;
        while (!admitted.empty() && int32_t(S.reqs.size()) < maxb) {
          // a request of a search format (many-channel guide) runs through
          // the per-frame kernels, in a batch of its own, in arrival order
          const bool alone = fmt_search(fr[size_t(admitted.front())].style->fmt);
          if (alone && !S.reqs.empty()) break;
          S.reqs.push_back(admitted.front());
          bf.push_back(fr[size_t(admitted.front())]);
          admitted.pop_front();
          if (alone) break;
        }
        // sessions whose previous frame still runs on another slot: wait
        // for that slot's batch (each slot once)
        uint32_t waited = 0;
        for (int32_t i : S.reqs) {
          const int32_t ses = reqs[i].session;
          if (ses < 0) continue;
          const auto it = tails.find(ses);
          if (it == tails.end()) continue;
          const SessionTail &tl = it->second;
          if (tl.slot == s || (waited >> tl.slot) & 1u) continue;
          const Slot &P = sl[size_t(tl.slot)];
          if (!P.busy || P.batch != tl.batch) continue;  // already retired
          if (e == hipSuccess) e = hipStreamWaitEvent(S.stream, P.done, 0);
          waited |= 1u << tl.slot;
        }
        if (e != hipSuccess) break;
        // a batch of one goes straight to the per-frame kernels (sized to the
        // frame, no descriptor upload); larger batches replay the plan
        const sb_frame &f0 = bf[0];
        const int r = bf.size() == 1
                          ? run_one(f0, S.workspace, cfg->workspace_bytes_per_slot, &cfg->tune,
                                    S.stream)
                          : sb_batch_run(S.plan, bf.data(), int32_t(bf.size()), S.workspace,
                                         cfg->workspace_bytes_per_slot, S.stream);
        if (r != SB_OK) {
          rc = r;
          break;
        }
        const double tl = now_s(t0);
        for (int32_t i : S.reqs) {
          res[i].batch = batch_id;
          res[i].slot = s;
          res[i].launched_s = tl;
          res[i].batch_size = int32_t(S.reqs.size());
          if (reqs[i].session >= 0) tails[reqs[i].session] = SessionTail{s, batch_id};
        }
        S.batch = batch_id;
        ++batch_id;
        e = hipEventRecord(S.done, S.stream);
        S.busy = true;
      }
    }
  }
  // drain and release
  for (auto &s : sl) {
    if (s.stream) hipStreamSynchronize(s.stream);
    if (s.plan) sb_batch_destroy(s.plan);
    if (s.done) hipEventDestroy(s.done);
    if (s.stream) hipStreamDestroy(s.stream);
  }
  for (auto &ev : pev)
    if (ev) hipEventDestroy(ev);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_serve_run");
    return SB_EHIP;
  }
  return rc;
}

}  // extern "C"
