// capi.hip -- the C ABI (include/styleblit.h): argument validation, workspace
// carving and kernel dispatch.  No device memory is allocated here; every
// buffer comes from the caller.
#include <stdio.h>
#include <string.h>

#include "sb_internal.h"

namespace sb {

namespace {
thread_local char g_err[256] = "";

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int32_t ilog2(int32_t v) {
  int32_t l = 0;
  while ((int32_t(1) << (l + 1)) <= v) ++l;
  return l;
}

bool side_ok(int32_t v) { return v >= 1 && v <= SB_MAX_SIDE; }

bool style_ok(const sb_style *s) {
  if (!s || !s->rgba || !s->guide) return false;
  if (!side_ok(s->sw) || !side_ok(s->sh)) return false;
  if (fmt_search(s->fmt)) {
    // many channels: the search tree instead of tables; no labels
    uint32_t wn[2];
    return s->tree && search_texel_bytes(s->fmt, s->channels) != 0 && s->lut_bits == 0 &&
           s->nlabels == 0 && resolve_weights_n(s->weights, s->channels, wn);
  }
  if (!s->lut || !fmt_ok(s->fmt)) return false;
  int32_t wt[3];
  if (!resolve_weights(s->fmt, s->weights, wt)) return false;
  if (s->nlabels < 0 || s->nlabels > SB_MAX_LABELS) return false;
  if (s->nlabels > 0 && (!s->labels || !s->label_luts)) return false;
  return s->lut_bits >= 1 && s->lut_bits <= fmt_depth(s->fmt) && s->lut_bits <= SB_MAX_LUT_BITS;
}

bool params_ok(const sb_params *p) {
  if (!p) return false;
  if (p->radius < 0 || p->radius > SB_MAX_RADIUS) return false;
  if (p->jitter != SB_JITTER_HASH && p->jitter != SB_JITTER_NONE && p->jitter != SB_JITTER_TABLE)
    return false;
  Levels lv;
  return make_levels(1, 1, p->levels, p->finest, &lv);
}
}  // namespace

void set_error_text(const char *msg) { snprintf(g_err, sizeof g_err, "%s", msg); }

void set_hip_error(hipError_t e, const char *where) {
  snprintf(g_err, sizeof g_err, "%s: %s (%d)", where, hipGetErrorString(e), int(e));
}

bool make_levels(int32_t w, int32_t h, int32_t levels, int32_t finest, Levels *out) {
  if (levels < 0 || levels > SB_MAX_LEVELS) return false;
  if (finest < 1 || (finest & (finest - 1)) != 0) return false;
  const int32_t lf = ilog2(finest);
  if (levels > 0 && lf + levels - 1 > ilog2(SB_MAX_SIDE)) return false;
  memset(out, 0, sizeof *out);
  out->count = levels;
  int32_t off = 0, poff = 0;
  for (int32_t i = 0; i < levels; ++i) {
    const int32_t ls = lf + (levels - 1 - i);
    const int32_t sp = int32_t(1) << ls;
    out->log2_spacing[i] = ls;
    out->cells_x[i] = (w + sp - 1) / sp;
    out->cells_y[i] = (h + sp - 1) / sp;
    out->offset[i] = off;
    out->poffset[i] = poff;
    off += out->cells_x[i] * out->cells_y[i];
    poff += (out->cells_x[i] + 2) * (out->cells_y[i] + 2);
  }
  out->offset[levels] = off;
  out->poffset[levels] = poff;
  return true;
}

bool fill_frame(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                uint32_t *out_chunk, uint32_t *out_nnf, FrameArgs *a,
                const uint8_t *tgt_labels) {
  if (!style_ok(style) || !tgt_guide || !out_rgb || !out_chunk) return false;
  if (tgt_labels && style->nlabels < 1) return false;  // labels on one side only
  if (!side_ok(w) || !side_ok(h) || !params_ok(params)) return false;
  if (params->jitter == SB_JITTER_TABLE && params->levels > 0 && !jitter) return false;
  memset(a, 0, sizeof *a);
  make_levels(w, h, params->levels, params->finest, &a->lv);
  a->jmode = params->jitter;
  if (params->jitter == SB_JITTER_HASH) {
    // the hash state after the seed and level words; the kernels add the cell
    const uint32_t k0 = hash_mix(params->seed + 0xBB67AE85u);
    for (int32_t i = 0; i < a->lv.count; ++i)
      a->jhash[i] = hash_mix(k0 ^ uint32_t(a->lv.log2_spacing[i]));
  }
  a->src_rgba = style->rgba;
  a->src_guide = style->guide;
  a->lut = style->lut;
  a->tgt_guide = tgt_guide;
  a->jitter = params->jitter == SB_JITTER_TABLE ? jitter : nullptr;
  a->out_rgb = out_rgb;
  a->out_chunk = out_chunk;
  a->out_nnf = out_nnf;
  a->sw = style->sw;
  a->sh = style->sh;
  a->w = w;
  a->h = h;
  a->lut_bits = style->lut_bits;
  a->lut_shift = fmt_depth(style->fmt) - style->lut_bits;
  a->lut_log2 = fmt_channels(style->fmt) * style->lut_bits;
  int32_t wt[3];
  resolve_weights(style->fmt, style->weights, wt);  // checked by style_ok
  a->wt02 = uint32_t(wt[0]) | (uint32_t(wt[2]) << 16);
  a->wt1 = wt[1];
  // records made in the level loop cost a table lookup per block and cell;
  // worth it when the one table (256 KiB) stays in cache and blocks hold
  // whole cells, otherwise a separate pass builds each record once
  const Levels &lv = a->lv;
  a->own_seeds = style->fmt == SB_GUIDE_U8X2 && tgt_labels == nullptr &&
                 (lv.count == 0 || lv.log2_spacing[lv.count - 1] >= 3);
  if (fmt_search(style->fmt)) fill_tree_args(style, a);
  a->threshold = params->threshold;
  a->radius = params->radius;
  a->fmt = style->fmt;
  a->ex_stride = ex_stride(style->sw);
  a->ex_zero = uint32_t(ex_stride(style->sw)) * uint32_t(style->sh + 2 * kExMargin);
  if (tgt_labels) {
    a->src_labels = style->labels;
    a->tgt_labels = tgt_labels;
    a->label_luts = style->label_luts;
    a->nlabels = style->nlabels;
  }
  return true;
}

bool resolve_weights(int32_t fmt, const uint8_t *in, int32_t out[3]) {
  out[0] = out[1] = out[2] = 1;
  if (!in || (in[0] == 0 && in[1] == 0 && in[2] == 0)) return true;
  for (int32_t k = 0; k < 3; ++k) {
    if (in[k] > 127) return false;
    out[k] = in[k];
  }
  return fmt == SB_GUIDE_U8X3 || (out[0] == 1 && out[1] == 1 && out[2] == 1);
}

bool resolve_tune(const sb_tune *in, Tune *out) {
  out->ppt = 4;
  out->rows = 16;
  out->group = 2;
  out->apx = 2;
  out->split = 2;
  if (!in) return true;
  if (in->blend_ppt != 0) {
    if (in->blend_ppt != 2 && in->blend_ppt != 4) return false;
    out->ppt = in->blend_ppt;
  }
  if (in->blend_rows != 0) {
    if (in->blend_rows != 8 && in->blend_rows != 16) return false;
    out->rows = in->blend_rows;
  }
  if (in->level_group != 0) {
    if (in->level_group != 2 && in->level_group != 4) return false;
    out->group = in->level_group;
  }
  if (in->level_ppt != 0) {
    if (in->level_ppt != 1 && in->level_ppt != 2 && in->level_ppt != 4) return false;
    out->apx = in->level_ppt;
  }
  if (in->blend_split != 0) {
    if (in->blend_split != 1 && in->blend_split != 2) return false;
    out->split = in->blend_split;
  }
  return true;
}

void carve_workspace(FrameArgs *a, void *workspace) {
  char *ws = static_cast<char *>(workspace);
  a->seeds = reinterpret_cast<uint2 *>(ws);
  a->offsets = reinterpret_cast<uint32_t *>(ws + align256(size_t(a->lv.poffset[a->lv.count]) * 8));
}

}  // namespace sb

using namespace sb;

extern "C" {

const char *sb_version(void) { return "styleblit-gfx950 0.3"; }

const char *sb_status_string(int status) {
  switch (status) {
    case SB_OK: return "ok";
    case SB_EINVAL: return "invalid argument";
    case SB_ENOMEM: return "workspace too small or host allocation failed";
    case SB_EHIP: return "HIP error";
    case SB_EBUDGET: return "request exceeds the memory budget";
    default: return "unknown status";
  }
}

const char *sb_last_hip_error(void) { return g_err; }

int64_t sb_jitter_len(int32_t w, int32_t h, int32_t levels, int32_t finest) {
  Levels lv;
  if (!side_ok(w) || !side_ok(h) || !make_levels(w, h, levels, finest, &lv)) return -1;
  return lv.offset[levels];
}

size_t sb_exemplar_texels(int32_t sw, int32_t sh) {
  if (!side_ok(sw) || !side_ok(sh)) return 0;
  return ex_texels(sw, sh);
}

int sb_pack_exemplar(const uint8_t *rgb, int32_t sw, int32_t sh, uint32_t *rgba,
                     hipStream_t stream) {
  if (!rgb || !rgba || !side_ok(sw) || !side_ok(sh)) return SB_EINVAL;
  hipError_t e = launch_pack_exemplar(rgb, sw, sh, rgba, stream);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_pack_exemplar");
    return SB_EHIP;
  }
  return SB_OK;
}

size_t sb_lut_workspace_bytes(int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits) {
  if (!fmt_ok(fmt) || !side_ok(sw) || !side_ok(sh)) return 0;
  if (lut_bits < 1 || lut_bits > fmt_depth(fmt) || lut_bits > SB_MAX_LUT_BITS) return 0;
  return lut_workspace_bytes(fmt, sw, sh, lut_bits);
}

int sb_lut_build(const void *guide, int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits,
                 uint32_t *lut, void *workspace, size_t workspace_bytes, hipStream_t stream) {
  return sb_lut_build_w(guide, fmt, sw, sh, lut_bits, nullptr, lut, workspace, workspace_bytes,
                        stream);
}

int sb_lut_build_w(const void *guide, int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits,
                   const uint8_t *weights, uint32_t *lut, void *workspace,
                   size_t workspace_bytes, hipStream_t stream) {
  if (!guide || !lut || !workspace) return SB_EINVAL;
  int32_t wt[3];
  if (!resolve_weights(fmt, weights, wt)) return SB_EINVAL;
  const size_t need = sb_lut_workspace_bytes(fmt, sw, sh, lut_bits);
  if (need == 0) return SB_EINVAL;
  if (workspace_bytes < need) return SB_ENOMEM;
  hipError_t e = launch_lut_build(guide, fmt, sw, sh, lut_bits, wt, lut, workspace, stream);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_lut_build");
    return SB_EHIP;
  }
  return SB_OK;
}

int sb_lut_build_labels(const void *guide, const uint8_t *labels, int32_t fmt, int32_t sw,
                        int32_t sh, int32_t lut_bits, int32_t nlabels, const uint32_t *lut,
                        uint32_t *luts, void *workspace, size_t workspace_bytes,
                        hipStream_t stream) {
  return sb_lut_build_labels_w(guide, labels, fmt, sw, sh, lut_bits, nullptr, nlabels, lut, luts,
                               workspace, workspace_bytes, stream);
}

int sb_lut_build_labels_w(const void *guide, const uint8_t *labels, int32_t fmt, int32_t sw,
                          int32_t sh, int32_t lut_bits, const uint8_t *weights, int32_t nlabels,
                          const uint32_t *lut, uint32_t *luts, void *workspace,
                          size_t workspace_bytes, hipStream_t stream) {
  if (!guide || !labels || !lut || !luts || !workspace) return SB_EINVAL;
  if (nlabels < 1 || nlabels > SB_MAX_LABELS) return SB_EINVAL;
  int32_t wt[3];
  if (!resolve_weights(fmt, weights, wt)) return SB_EINVAL;
  const size_t need = sb_lut_workspace_bytes(fmt, sw, sh, lut_bits);
  if (need == 0) return SB_EINVAL;
  if (workspace_bytes < need) return SB_ENOMEM;
  const hipError_t e = launch_lut_build_labels(guide, labels, fmt, sw, sh, lut_bits, wt, nlabels,
                                               lut, luts, workspace, stream);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_lut_build_labels");
    return SB_EHIP;
  }
  return SB_OK;
}

size_t sb_workspace_bytes(int32_t w, int32_t h, const sb_params *params) {
  if (!side_ok(w) || !side_ok(h) || !params_ok(params)) return 0;
  Levels lv;
  make_levels(w, h, params->levels, params->finest, &lv);
  return align256(size_t(lv.poffset[lv.count]) * 8) + align256(size_t(w) * size_t(h) * 4);
}

}  // extern "C"

namespace sb {
int stylize_impl(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                 const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                 uint32_t *out_chunk, uint32_t *out_nnf, void *workspace, size_t workspace_bytes,
                 const sb_tune *tune, hipEvent_t *events, hipStream_t stream,
                 const uint8_t *tgt_labels) {
  FrameArgs a;
  if (!fill_frame(style, tgt_guide, w, h, jitter, params, out_rgb, out_chunk, out_nnf, &a,
                  tgt_labels))
    return SB_EINVAL;
  Tune t;
  if (!resolve_tune(tune, &t)) return SB_EINVAL;
  if (!workspace) return SB_EINVAL;
  if (workspace_bytes < sb_workspace_bytes(w, h, params)) return SB_ENOMEM;
  carve_workspace(&a, workspace);
  const hipError_t e = launch_stylize(a, style->fmt, t, events, stream);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_stylize");
    return SB_EHIP;
  }
  return SB_OK;
}
}  // namespace sb

extern "C" {

int sb_stylize_ex(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                  const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                  uint32_t *out_chunk, uint32_t *out_nnf, void *workspace,
                  size_t workspace_bytes, const sb_tune *tune, hipStream_t stream) {
  return stylize_impl(style, tgt_guide, w, h, jitter, params, out_rgb, out_chunk, out_nnf,
                      workspace, workspace_bytes, tune, nullptr, stream, nullptr);
}

int sb_stylize_seg(const sb_style *style, const void *tgt_guide, const uint8_t *tgt_labels,
                   int32_t w, int32_t h, const uint32_t *jitter, const sb_params *params,
                   uint8_t *out_rgb, uint32_t *out_chunk, uint32_t *out_nnf, void *workspace,
                   size_t workspace_bytes, const sb_tune *tune, hipStream_t stream) {
  if (!tgt_labels) return SB_EINVAL;
  return stylize_impl(style, tgt_guide, w, h, jitter, params, out_rgb, out_chunk, out_nnf,
                      workspace, workspace_bytes, tune, nullptr, stream, tgt_labels);
}

int sb_stylize_timed(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                     const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                     uint32_t *out_chunk, uint32_t *out_nnf, void *workspace,
                     size_t workspace_bytes, const sb_tune *tune, hipEvent_t events[4],
                     hipStream_t stream) {
  if (!events || !events[0] || !events[1] || !events[2] || !events[3]) return SB_EINVAL;
  return stylize_impl(style, tgt_guide, w, h, jitter, params, out_rgb, out_chunk, out_nnf,
                      workspace, workspace_bytes, tune, events, stream, nullptr);
}

int sb_timing_events_create(hipEvent_t events[4]) {
  if (!events) return SB_EINVAL;
  for (int i = 0; i < 4; ++i) events[i] = nullptr;
  for (int i = 0; i < 4; ++i) {
    const hipError_t e =
        hipEventCreateWithFlags(&events[i], hipEventDisableSystemFence);
    if (e != hipSuccess) {
      set_hip_error(e, "sb_timing_events_create");
      for (int k = 0; k < i; ++k) hipEventDestroy(events[k]);
      for (int k = 0; k < 4; ++k) events[k] = nullptr;
      return SB_EHIP;
    }
  }
  return SB_OK;
}

int sb_timing_events_destroy(hipEvent_t events[4]) {
  if (!events) return SB_EINVAL;
  hipError_t first = hipSuccess;
  for (int i = 0; i < 4; ++i) {
    if (!events[i]) continue;
    const hipError_t e = hipEventDestroy(events[i]);
    if (first == hipSuccess) first = e;
    events[i] = nullptr;
  }
  if (first != hipSuccess) {
    set_hip_error(first, "sb_timing_events_destroy");
    return SB_EHIP;
  }
  return SB_OK;
}

int sb_event_elapsed_ms(hipEvent_t start, hipEvent_t stop, float *ms) {
  if (!start || !stop || !ms) return SB_EINVAL;
  const hipError_t e = hipEventElapsedTime(ms, start, stop);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_event_elapsed_ms");
    return SB_EHIP;
  }
  return SB_OK;
}

int sb_stylize(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
               const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
               uint32_t *out_chunk, uint32_t *out_nnf, void *workspace, size_t workspace_bytes,
               hipStream_t stream) {
  // the plain entry point keeps one contract whichever path runs: the
  // workspace must be there and large enough
  if (!workspace) return SB_EINVAL;
  const size_t need = sb_workspace_bytes(w, h, params);
  if (need == 0) return SB_EINVAL;
  if (workspace_bytes < need) return SB_ENOMEM;
  return sb_stylize_ex(style, tgt_guide, w, h, jitter, params, out_rgb, out_chunk, out_nnf,
                       workspace, workspace_bytes, nullptr, stream);
}

}  // extern "C"
