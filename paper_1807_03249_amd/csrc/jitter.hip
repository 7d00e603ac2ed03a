// jitter.hip -- the seed hierarchy's jitter table drawn on the device.
//
// The paper's RandomJitterTable holds one random offset per cell and level
// (SeedPoint in Algorithm 2).  Callers may pass their own table; this fills
// one from Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011), a
// counter-based generator, so a frame's table follows from (seed, stream)
// alone -- the per-frame seed schedule of an animation needs no host
// random numbers and no upload.  Entry e takes word 0 of the block at counter
// (e, 0, 0, 0) under key (seed, stream): jx = word mod h_i, jy = (word >> 32)
// mod h_i for its level's spacing h_i (a power of two, so the modulus is a
// mask and uniform).
#include "sb_internal.h"

namespace sb {
namespace {

__global__ __launch_bounds__(256) void k_jitter_fill(Levels lv, uint64_t seed, uint64_t stream,
                                                     uint32_t *__restrict__ out) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= uint32_t(lv.offset[lv.count])) return;
  int32_t i = 0;
  while (e >= uint32_t(lv.offset[i + 1])) ++i;
  // Philox4x64-10: round constants and the key's Weyl increments
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t k0 = seed, k1 = stream;
  uint64_t c0 = e, c1 = 0, c2 = 0, c3 = 0;
#pragma unroll
  for (int32_t r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  const uint32_t hm = (1u << lv.log2_spacing[i]) - 1u;
  out[e] = (uint32_t(c0) & hm) | ((uint32_t(c0 >> 32) & hm) << 16);
}

}  // namespace
}  // namespace sb

using namespace sb;

extern "C" {

int sb_jitter_fill(int32_t w, int32_t h, int32_t levels, int32_t finest, uint64_t seed,
                   uint64_t stream_id, uint32_t *jitter, hipStream_t stream) {
  if (w < 1 || h < 1 || w > SB_MAX_SIDE || h > SB_MAX_SIDE) return SB_EINVAL;
  Levels lv;
  if (!make_levels(w, h, levels, finest, &lv)) return SB_EINVAL;
  const uint32_t n = uint32_t(lv.offset[lv.count]);
  if (n == 0) return SB_OK;
  if (!jitter) return SB_EINVAL;
  hipLaunchKernelGGL(k_jitter_fill, dim3((n + 255) / 256), dim3(256), 0, stream, lv, seed,
                     stream_id, jitter);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_hip_error(e, "sb_jitter_fill");
    return SB_EHIP;
  }
  return SB_OK;
}

}  // extern "C"
