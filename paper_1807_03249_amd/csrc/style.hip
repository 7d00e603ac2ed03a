// style.hip -- library-owned styles (sb_style_create, sb_style_create_n,
// sb_style_destroy).
//
// The one place the library allocates device memory: a style's padded
// exemplar, a copy of its guide and its exact lookup table (Sec. 3.1), or for
// guides of many channels its search tree, in one block, built on the
// caller's stream with the same launchers the caller-owned path uses.  The
// build workspace is freed before returning.
#include <new>

#include "sb_internal.h"

namespace sb {
namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The handed-out pointer is the address of `s`, the first member, so
// sb_style_destroy finds the block again; `magic` rejects other styles.
struct OwnedStyle {
  sb_style s;
  void *block;
  uint32_t magic;
};
constexpr uint32_t kStyleMagic = 0x53545931u;

bool side_ok(int32_t v) { return v >= 1 && v <= SB_MAX_SIDE; }

}  // namespace
}  // namespace sb

using namespace sb;

extern "C" {

int sb_style_create(const uint8_t *src_rgb, const void *src_guide, int32_t sw, int32_t sh,
                    int32_t fmt, int32_t lut_bits, hipStream_t stream, sb_style **out) {
  if (!src_rgb || !src_guide || !out || !side_ok(sw) || !side_ok(sh) || !fmt_ok(fmt))
    return SB_EINVAL;
  const size_t wsb = sb_lut_workspace_bytes(fmt, sw, sh, lut_bits);
  if (wsb == 0) return SB_EINVAL;  // lut_bits out of range for the format
  const size_t ex_bytes = align256(ex_texels(sw, sh) * 4);
  const size_t guide_bytes = size_t(sw) * size_t(sh) * (fmt == SB_GUIDE_U8X2 ? 2 : 4);
  const size_t lut_bytes = (size_t(1) << (fmt_channels(fmt) * lut_bits)) * 4;
  OwnedStyle *o = new (std::nothrow) OwnedStyle;
  if (!o) return SB_ENOMEM;
  memset(o, 0, sizeof *o);
  void *ws = nullptr;
  char *blk = nullptr;
  hipError_t e = hipMalloc(&o->block, ex_bytes + align256(guide_bytes) + lut_bytes);
  if (e == hipSuccess) e = hipMalloc(&ws, wsb);
  if (e == hipSuccess) {
    blk = static_cast<char *>(o->block);
    uint32_t *rgba = reinterpret_cast<uint32_t *>(blk);
    void *guide = blk + ex_bytes;
    uint32_t *lut = reinterpret_cast<uint32_t *>(blk + ex_bytes + align256(guide_bytes));
    const int32_t unit[3] = {1, 1, 1};
    e = hipMemcpyAsync(guide, src_guide, guide_bytes, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = launch_pack_exemplar(src_rgb, sw, sh, rgba, stream);
    if (e == hipSuccess) e = launch_lut_build(guide, fmt, sw, sh, lut_bits, unit, lut, ws, stream);
    // the workspace is released only once the build has run
    const hipError_t es = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = es;
    o->s.rgba = rgba;
    o->s.guide = guide;
    o->s.lut = lut;
  }
  if (ws) hipFree(ws);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_style_create");
    if (o->block) hipFree(o->block);
    delete o;
    return SB_EHIP;
  }
  o->s.sw = sw;
  o->s.sh = sh;
  o->s.fmt = fmt;
  o->s.lut_bits = lut_bits;
  o->magic = kStyleMagic;
  *out = &o->s;
  return SB_OK;
}

int sb_style_create_n(const uint8_t *src_rgb, const void *src_guide, int32_t sw, int32_t sh,
                      int32_t fmt, int32_t channels, const uint8_t *weights, hipStream_t stream,
                      sb_style **out) {
  const int32_t t = sb_texel_bytes(fmt, channels);
  uint32_t wn[2];
  if (!src_rgb || !src_guide || !out || !side_ok(sw) || !side_ok(sh) || t == 0 ||
      !resolve_weights_n(weights, channels, wn))
    return SB_EINVAL;
  const size_t ex_bytes = align256(ex_texels(sw, sh) * 4);
  const size_t guide_bytes = align256(size_t(sw) * size_t(sh) * size_t(t));
  const size_t tree_bytes = sb_tree_bytes(fmt, channels, sw, sh);
  const size_t wsb = sb_tree_workspace_bytes(fmt, channels, sw, sh);
  OwnedStyle *o = new (std::nothrow) OwnedStyle;
  if (!o) return SB_ENOMEM;
  memset(o, 0, sizeof *o);
  void *ws = nullptr;
  hipError_t e = hipMalloc(&o->block, ex_bytes + guide_bytes + tree_bytes);
  if (e == hipSuccess) e = hipMalloc(&ws, wsb);
  int rc = SB_OK;
  if (e == hipSuccess) {
    char *blk = static_cast<char *>(o->block);
    uint32_t *rgba = reinterpret_cast<uint32_t *>(blk);
    void *guide = blk + ex_bytes;
    void *tree = blk + ex_bytes + guide_bytes;
    e = hipMemcpyAsync(guide, src_guide, size_t(sw) * size_t(sh) * size_t(t),
                       hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = launch_pack_exemplar(src_rgb, sw, sh, rgba, stream);
    // the build synchronises the stream, so the workspace is idle after it
    if (e == hipSuccess)
      rc = sb_tree_build(guide, fmt, channels, sw, sh, weights, tree, tree_bytes, ws, wsb, stream);
    else
      hipStreamSynchronize(stream);
    o->s.rgba = rgba;
    o->s.guide = guide;
    o->s.tree = tree;
  }
  if (ws) hipFree(ws);
  if (e != hipSuccess || rc != SB_OK) {
    if (e != hipSuccess) set_hip_error(e, "sb_style_create_n");
    if (o->block) hipFree(o->block);
    delete o;
    return rc != SB_OK ? rc : SB_EHIP;
  }
  o->s.sw = sw;
  o->s.sh = sh;
  o->s.fmt = fmt;
  o->s.lut_bits = 0;
  o->s.channels = channels;
  for (int32_t k = 0; weights && k < channels; ++k) o->s.weights[k] = weights[k];
  o->magic = kStyleMagic;
  *out = &o->s;
  return SB_OK;
}

int sb_style_destroy(sb_style *style) {
  if (!style) return SB_OK;
  OwnedStyle *o = reinterpret_cast<OwnedStyle *>(style);
  if (o->magic != kStyleMagic) return SB_EINVAL;
  o->magic = 0;
  const hipError_t e = hipFree(o->block);
  delete o;
  if (e != hipSuccess) {
    set_hip_error(e, "sb_style_destroy");
    return SB_EHIP;
  }
  return SB_OK;
}

}  // extern "C"
