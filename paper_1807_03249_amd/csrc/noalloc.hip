// noalloc.hip -- sb_stylize_noalloc: one frame whose scratch (the seed table
// and the per-pixel offset map that sb_stylize carves from the caller's
// workspace) lives in a fixed device array of the library, so the call
// allocates nothing and needs no workspace argument.
//
// The array is a file-scope __device__ variable.  Its name in host code is a
// host-side stand-in, not a device address, so host code never passes it to
// a kernel or a copy: on the first call on each device (with that device
// current) the device address is looked up once with hipGetSymbolAddress and
// kept per device, and only that address is used afterwards.
#include <stdio.h>

#include <mutex>

#include "sb_internal.h"

namespace sb {
namespace {

static __device__ __align__(256) unsigned char scratch[SB_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` per device, once looked up

// The current device's address of the scratch array (looked up on its first
// use there), or SB_EHIP if the device or the lookup fails.
int scratch_ptr(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_hip_error(e, "sb_stylize_noalloc: hipGetDevice");
    return SB_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_error_text("sb_stylize_noalloc: device index beyond the library's table");
    return SB_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                    "sb_stylize_noalloc: hipGetSymbolAddress");
      return SB_EHIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return SB_OK;
}

}  // namespace
}  // namespace sb

using namespace sb;

extern "C" {

size_t sb_noalloc_scratch_bytes(void) { return SB_NOALLOC_SCRATCH_BYTES; }

int sb_stylize_noalloc(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                       const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                       uint32_t *out_chunk, uint32_t *out_nnf, hipStream_t stream) {
  const size_t need = sb_workspace_bytes(w, h, params);
  if (need == 0) return SB_EINVAL;
  if (need > SB_NOALLOC_SCRATCH_BYTES) {
    char msg[160];
    snprintf(msg, sizeof msg,
             "sb_stylize_noalloc: a %dx%d frame needs %zu bytes of scratch; the static "
             "scratch holds %zu",
             int(w), int(h), need, size_t(SB_NOALLOC_SCRATCH_BYTES));
    set_error_text(msg);
    return SB_ENOMEM;
  }
  // arguments are checked (stylize_impl) before the scratch address is
  // looked up, so a bad call touches no device state
  FrameArgs probe;
  if (!fill_frame(style, tgt_guide, w, h, jitter, params, out_rgb, out_chunk, out_nnf, &probe))
    return SB_EINVAL;
  void *ws = nullptr;
  const int rc = scratch_ptr(&ws);
  if (rc != SB_OK) return rc;
  // every byte the kernels read from the seed table and the offset map is
  // written earlier in the same call, so nothing needs clearing between calls
  return stylize_impl(style, tgt_guide, w, h, jitter, params, out_rgb, out_chunk, out_nnf, ws,
                      need, nullptr, nullptr, stream, nullptr);
}

}  // extern "C"
