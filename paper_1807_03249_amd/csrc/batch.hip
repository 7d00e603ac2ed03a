// batch.hip -- many frames of uneven size and mixed guidance in one launch.
//
// A batch plan owns two descriptor buffers (device + pinned host, supplied by
// the caller) and, when graphs are on, two instantiated hipGraphs, each the
// upload of one descriptor buffer followed by the three persistent passes.
// Every shape lives in the descriptors, so the graphs are captured once and
// replayed for any batch.  Runs alternate between the two buffers: filling
// buffer k waits only for run k-2, so the host prepares the next batch while
// the previous one executes.
#include <stdio.h>
#include <string.h>

#include <new>

#include "sb_internal.h"

struct sb_batch {
  unsigned char *desc_dev[2];
  unsigned char *desc_host[2];
  hipGraph_t graph[2];
  hipGraphExec_t exec[2];
  hipEvent_t done[2];
  bool used[2];
  bool use_graph;
  uint32_t grid;
  sb::Tune tune;
  int next;
};

namespace sb {
namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

hipError_t batch_cleanup(sb_batch *b) {
  hipError_t first = hipSuccess;
  for (int k = 0; k < 2; ++k) {
    if (b->used[k] && b->done[k]) {
      hipError_t e = hipEventSynchronize(b->done[k]);
      if (first == hipSuccess) first = e;
    }
    if (b->exec[k]) hipGraphExecDestroy(b->exec[k]);
    if (b->graph[k]) hipGraphDestroy(b->graph[k]);
    if (b->done[k]) hipEventDestroy(b->done[k]);
  }
  return first;
}
}  // namespace
}  // namespace sb

using namespace sb;

extern "C" {

size_t sb_batch_desc_bytes(void) { return 2 * batch_desc_bytes(); }

int32_t sb_batch_max_frames(void) { return int32_t(kMaxBatchFrames); }

size_t sb_batch_workspace_bytes(const sb_frame *frames, int32_t n) {
  if (!frames || n < 1 || n > int32_t(kMaxBatchFrames)) return 0;
  size_t total = 0;
  for (int32_t f = 0; f < n; ++f) {
    const size_t b = sb_workspace_bytes(frames[f].w, frames[f].h, &frames[f].params);
    if (b == 0) return 0;
    total += align256(b);
  }
  return total;
}

int sb_batch_create(void *desc_dev, void *desc_host, int32_t use_graph, const sb_tune *tune,
                    int32_t blocks_per_cu, hipStream_t stream, sb_batch **out) {
  if (!desc_dev || !desc_host || !out) return SB_EINVAL;
  if (use_graph && stream == nullptr) return SB_EINVAL;  // capture needs a created stream
  if (blocks_per_cu < 0 || blocks_per_cu > 16) return SB_EINVAL;
  Tune t;
  if (!resolve_tune(tune, &t)) return SB_EINVAL;
  sb_batch *b = new (std::nothrow) sb_batch;
  if (!b) return SB_ENOMEM;
  memset(b, 0, sizeof *b);
  b->use_graph = use_graph != 0;
  b->tune = t;
  for (int k = 0; k < 2; ++k) {
    b->desc_dev[k] = static_cast<unsigned char *>(desc_dev) + k * batch_desc_bytes();
    b->desc_host[k] = static_cast<unsigned char *>(desc_host) + k * batch_desc_bytes();
  }
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  b->grid = uint32_t(cus > 0 ? cus : 256) * uint32_t(blocks_per_cu > 0 ? blocks_per_cu : 8);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&b->done[k], hipEventDisableTiming);
  for (int k = 0; k < 2 && e == hipSuccess && b->use_graph; ++k) {
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) break;
    hipError_t ec = hipMemcpyAsync(b->desc_dev[k], b->desc_host[k], batch_desc_bytes(),
                                   hipMemcpyHostToDevice, stream);
    if (ec == hipSuccess) ec = launch_batch(b->desc_dev[k], b->grid, b->tune, stream);
    e = hipStreamEndCapture(stream, &b->graph[k]);
    if (ec != hipSuccess) e = ec;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[k], b->graph[k], nullptr, nullptr, 0);
  }
  if (e != hipSuccess) {
    set_hip_error(e, "sb_batch_create");
    batch_cleanup(b);
    delete b;
    return SB_EHIP;
  }
  *out = b;
  return SB_OK;
}

int sb_batch_run(sb_batch *b, const sb_frame *frames, int32_t n, void *workspace,
                 size_t workspace_bytes, hipStream_t stream) {
  if (!b || !frames || n < 1 || n > int32_t(kMaxBatchFrames) || !workspace) return SB_EINVAL;
  const size_t need = sb_batch_workspace_bytes(frames, n);
  if (need == 0) return SB_EINVAL;
  if (workspace_bytes < need) return SB_ENOMEM;
  // validate every frame before touching the descriptor buffer; frames of
  // the table formats go to the batch kernels (args[0 .. nt)), frames of
  // the search formats (many-channel guides) to the per-frame kernels after
  // them on the same stream (search[0 .. ns)), each in its own workspace
  static thread_local FrameArgs args[kMaxBatchFrames], search[kMaxBatchFrames];
  char *ws = static_cast<char *>(workspace);
  int32_t nt = 0, ns = 0;
  for (int32_t f = 0; f < n; ++f) {
    const sb_frame &fr = frames[f];
    const bool srch = fr.style && fmt_search(fr.style->fmt);
    FrameArgs &a = srch ? search[ns++] : args[nt++];
    if (!fill_frame(fr.style, fr.tgt_guide, fr.w, fr.h, fr.jitter, &fr.params, fr.out_rgb,
                    fr.out_chunk, fr.out_nnf, &a, fr.tgt_labels))
      return SB_EINVAL;
    // graphs: the batch's seed pass is one persistent launch over every
    // frame, so each record is built once there rather than per block;
    // direct launches keep single frames' choice (records made in the level
    // loop for 8-bit styles), which saves a pass and its wait
    if (b->use_graph && !srch) a.own_seeds = 0;
    carve_workspace(&a, ws);
    ws += align256(sb_workspace_bytes(fr.w, fr.h, &fr.params));
  }
  const int k = b->next;
  if (b->used[k]) {  // run k-2 must have finished reading this buffer
    hipError_t e = hipEventSynchronize(b->done[k]);
    if (e != hipSuccess) {
      set_hip_error(e, "sb_batch_run");
      return SB_EHIP;
    }
  }
  unsigned char *hd = b->desc_host[k];
  BatchHeader hdr;
  memset(&hdr, 0, sizeof hdr);
  hdr.nframes = uint32_t(nt);
  memcpy(hd, &hdr, sizeof hdr);
  uint32_t *pre[kBatchKinds];
  for (int kind = 0; kind < kBatchKinds; ++kind) {
    pre[kind] = reinterpret_cast<uint32_t *>(hd + batch_prefix_offset(kind));
    pre[kind][0] = 0;
  }
  for (int32_t f = 0; f < nt; ++f) {
    uint32_t c[kBatchKinds];
    tile_counts(args[f], b->tune, c);
    for (int kind = 0; kind < kBatchKinds; ++kind) pre[kind][f + 1] = pre[kind][f] + c[kind];
  }
  memcpy(hd + batch_frames_offset(), args, size_t(nt) * sizeof(FrameArgs));
  hipError_t e = hipSuccess;
  if (nt > 0 && b->use_graph) {
    e = hipGraphLaunch(b->exec[k], stream);
  } else if (nt > 0) {
    // direct launches know the batch's shape: exact grids, one tile per
    // workgroup, so kernels on other streams interleave with them
    e = hipMemcpyAsync(b->desc_dev[k], hd, batch_desc_bytes(), hipMemcpyHostToDevice, stream);
    uint32_t totals[kBatchKinds];
    for (int kind = 0; kind < kBatchKinds; ++kind) totals[kind] = pre[kind][nt];
    if (e == hipSuccess) e = launch_batch_exact(b->desc_dev[k], totals, b->tune, stream);
  }
  for (int32_t f = 0; f < ns && e == hipSuccess; ++f)
    e = launch_stylize(search[f], search[f].fmt, b->tune, nullptr, stream);
  if (e == hipSuccess) e = hipEventRecord(b->done[k], stream);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_batch_run");
    return SB_EHIP;
  }
  b->used[k] = true;
  b->next = k ^ 1;
  return SB_OK;
}

int sb_batch_destroy(sb_batch *b) {
  if (!b) return SB_EINVAL;
  hipError_t e = batch_cleanup(b);
  delete b;
  if (e != hipSuccess) {
    set_hip_error(e, "sb_batch_destroy");
    return SB_EHIP;
  }
  return SB_OK;
}

int sb_stylize_frames(const sb_frame *frames, int32_t n, void *workspace,
                      size_t workspace_bytes, const sb_tune *tune, hipStream_t stream) {
  if (!frames || n < 1 || !workspace) return SB_EINVAL;
  Tune t;
  if (!resolve_tune(tune, &t)) return SB_EINVAL;
  // every frame is checked before the first is enqueued
  for (int32_t f = 0; f < n; ++f) {
    const sb_frame &fr = frames[f];
    FrameArgs a;
    if (!fill_frame(fr.style, fr.tgt_guide, fr.w, fr.h, fr.jitter, &fr.params, fr.out_rgb,
                    fr.out_chunk, fr.out_nnf, &a, fr.tgt_labels))
      return SB_EINVAL;
    if (workspace_bytes < sb_workspace_bytes(fr.w, fr.h, &fr.params)) return SB_ENOMEM;
  }
  // the frames run one after another on one stream, so they share the workspace
  for (int32_t f = 0; f < n; ++f) {
    const sb_frame &fr = frames[f];
    const int rc = stylize_impl(fr.style, fr.tgt_guide, fr.w, fr.h, fr.jitter, &fr.params,
                                fr.out_rgb, fr.out_chunk, fr.out_nnf, workspace, workspace_bytes,
                                tune, nullptr, stream, fr.tgt_labels);
    if (rc != SB_OK) return rc;
  }
  return SB_OK;
}

}  // extern "C"
