// sb_device.h -- device helpers shared by the frame kernels of the table
// formats (stylize.hip) and of the search formats (search.hip): seed records,
// offsets, chunk codes, vote distances, seed jitter, the NearestSeed key and
// the XCD-aware tile order.
#pragma once

#include "sb_internal.h"

namespace sb {

typedef short short2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Seed records as plain vectors in global memory.
__device__ __forceinline__ SB_GLOBAL u32x2 *seed_table(const FrameArgs &a) {
  return reinterpret_cast<SB_GLOBAL u32x2 *>(glb(a.seeds));
}

// Offsets are two int16 in one word; x in the low half.
__device__ inline uint32_t pack_off(int32_t dx, int32_t dy) {
  return (uint32_t(dx) & 0xFFFFu) | (uint32_t(dy) << 16);
}
__device__ inline int32_t off_x(uint32_t o) { return int32_t(int16_t(o & 0xFFFFu)); }
__device__ inline int32_t off_y(uint32_t o) { return int32_t(int16_t(o >> 16)); }

// Chunk code of the seed whose position word (4x | 4y << 16) is q4.
__device__ inline uint32_t chunk_code(int32_t level, uint32_t q4) {
  return (uint32_t(level) << 26) | ((q4 >> 18) << 13) | ((q4 & 0xFFFFu) >> 2);
}

// What the vote needs of a pixel's offset o = NNF[p] - p: the byte distance
// 4 (oy P + ox) it adds to a pixel's position in the padded exemplar (rows of
// P texels) to reach the co-located texel of that source patch.
__device__ inline uint32_t vote_distance(const FrameArgs &a, uint32_t off) {
  return uint32_t(4 * (__mul24(off_y(off), a.ex_stride) + off_x(off)));
}

// Jitter word jx | jy << 16 of cell (cx, cy) of a level with log2 spacing ls
// and a ncx-wide cell grid: from the hash (level hash state hk), zero, or the
// caller's table (the level's entries from joff on).
__device__ inline uint32_t cell_jitter(const FrameArgs &a, int32_t ls, int32_t ncx, int32_t joff,
                                       uint32_t hk, int32_t cx, int32_t cy) {
  if (a.jmode == SB_JITTER_HASH) return hash_jitter(hk, ls, uint32_t(cx), uint32_t(cy));
  if (a.jmode == SB_JITTER_NONE) return 0u;
  return glb(a.jitter)[uint32_t(joff) + __umul24(uint32_t(cy), uint32_t(ncx)) + uint32_t(cx)];
}

// NearestSeed key of candidate k (k = (dx+1)*3 + (dy+1): x outer, y inner):
// 16 d + k for the squared distance d, from the packed int16 pair 4q - 4p
// (|4 dx| <= 4 * 8191 fits int16, so 16 d + k <= 2146959400 < 2^31 - 1).
// The empty record (-32768, -32768) saturates the subtraction and then the
// dot product, giving INT32_MAX, above every real key.  The minimum key over
// k = 0..8 is NearestSeed's first strict minimum; INT32_MAX means no seed.
__device__ inline int32_t seed_key(uint32_t q4, short2_t p4, int32_t k) {
  const short2_t dv = __builtin_elementwise_sub_sat(__builtin_bit_cast(short2_t, q4), p4);
  return __builtin_amdgcn_sdot2(dv, dv, k, true);
}

// Tile of workgroup `bid` out of n: workgroups are dealt to the 8 XCDs in
// turn (bid mod 8), so XCD x takes the x-th contiguous run of tiles -- a band
// of rows -- and its L2 sees the source regions of one band instead of
// scraps of all of them.  A bijection on [0, n) for any n.
__device__ inline uint32_t xcd_tile(uint32_t bid, uint32_t n) {
  const uint32_t x = bid & 7u, local = bid >> 3, q = n >> 3, r = n & 7u;
  return x * q + min(x, r) + local;
}

}  // namespace sb
