// change.hip -- frame-to-frame change of an animation.
//
// With the extension to animation (Sec. 3.3) every frame of a sequence draws
// its seeds anew (or keeps them for a few frames); the local guidance keeps
// most of the mosaic in place while the new seeds move some chunks, which is
// the flicker the paper controls with the threshold t.  The measure here is
// how many pixels changed between two frames of one sequence: pixels whose
// chunk code differs, and pixels whose source coordinate (NNF entry)
// differs -- the latter is what the viewer sees move.
//
// Two passes, no atomics: every block of the first pass counts a grid-stride
// share of the pixels and stores its two partial sums; one block of the
// second pass adds the partial sums.  HBM bound: 8 bytes per pixel and map
// pair.
#include "sb_internal.h"

namespace sb {
namespace {

constexpr int32_t kChangeThreads = 256;
constexpr int32_t kChangeBlocks = 1024;

__device__ inline uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int32_t o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int32_t o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline uint32_t differ4(const uint4 &a, const uint4 &b) {
  return uint32_t(a.x != b.x) + uint32_t(a.y != b.y) + uint32_t(a.z != b.z) + uint32_t(a.w != b.w);
}

// Partial counts of one block: out[2 * blockIdx.x + m] for map m (0 = chunk
// codes, 1 = source coordinates; map 1 is skipped when its pointers are
// null).  vec: every pointer is 16-byte aligned, so whole uint4 groups are
// read; the ragged tail (n % 4 pixels) is read one by one.
__global__ __launch_bounds__(kChangeThreads) void k_change_partial(
    const uint32_t *__restrict__ ca, const uint32_t *__restrict__ cb,
    const uint32_t *__restrict__ na, const uint32_t *__restrict__ nb, int64_t n, int32_t vec,
    uint64_t *__restrict__ out) {
  const int64_t tid = int64_t(blockIdx.x) * kChangeThreads + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * kChangeThreads;
  const bool two = na != nullptr;
  uint32_t c0 = 0, c1 = 0;  // per thread at most n / stride + 4 <= 2^22 + 4 pixels
  int64_t done = 0;
  if (vec) {
    const int64_t groups = n >> 2;
    const uint4 *a4 = reinterpret_cast<const uint4 *>(ca);
    const uint4 *b4 = reinterpret_cast<const uint4 *>(cb);
    const uint4 *p4 = reinterpret_cast<const uint4 *>(na);
    const uint4 *q4 = reinterpret_cast<const uint4 *>(nb);
    for (int64_t g = tid; g < groups; g += stride) {
      c0 += differ4(a4[g], b4[g]);
      if (two) c1 += differ4(p4[g], q4[g]);
    }
    done = groups << 2;
  }
  for (int64_t i = done + tid; i < n; i += stride) {
    c0 += uint32_t(ca[i] != cb[i]);
    if (two) c1 += uint32_t(na[i] != nb[i]);
  }
  __shared__ uint32_t part[2][kChangeThreads / 64];
  c0 = wave_sum(c0);
  c1 = wave_sum(c1);
  const int32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    part[0][wave] = c0;
    part[1][wave] = c1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint64_t s = 0;
    for (int32_t k = 0; k < kChangeThreads / 64; ++k) s += part[threadIdx.x][k];
    out[2 * blockIdx.x + threadIdx.x] = s;
  }
}

// One block: counts[m] = sum of the nblocks partial sums of map m.
__global__ __launch_bounds__(kChangeThreads) void k_change_sum(const uint64_t *__restrict__ part,
                                                              int32_t nblocks,
                                                              uint64_t *__restrict__ counts) {
  uint64_t s0 = 0, s1 = 0;
  for (int32_t b = threadIdx.x; b < nblocks; b += kChangeThreads) {
    s0 += part[2 * b];
    s1 += part[2 * b + 1];
  }
  s0 = wave_sum64(s0);
  s1 = wave_sum64(s1);
  __shared__ uint64_t acc[2][kChangeThreads / 64];
  const int32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    acc[0][wave] = s0;
    acc[1][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint64_t s = 0;
    for (int32_t k = 0; k < kChangeThreads / 64; ++k) s += acc[threadIdx.x][k];
    counts[threadIdx.x] = s;
  }
}

}  // namespace
}  // namespace sb

using namespace sb;

extern "C" {

size_t sb_change_workspace_bytes(void) { return size_t(kChangeBlocks) * 2 * sizeof(uint64_t); }

int sb_frame_change(const uint32_t *chunk_a, const uint32_t *chunk_b, const uint32_t *nnf_a,
                    const uint32_t *nnf_b, int64_t n, uint64_t *counts, void *workspace,
                    size_t workspace_bytes, hipStream_t stream) {
  if (!counts || n < 0) return SB_EINVAL;
  if (n > 0 && (!chunk_a || !chunk_b || (nnf_a == nullptr) != (nnf_b == nullptr)))
    return SB_EINVAL;
  if (n == 0) nnf_a = nnf_b = nullptr;
  if (n > int64_t(1) << 40) return SB_EINVAL;
  if (!workspace || workspace_bytes < sb_change_workspace_bytes()) return SB_ENOMEM;
  if (reinterpret_cast<uintptr_t>(workspace) % 8 || reinterpret_cast<uintptr_t>(counts) % 8)
    return SB_EINVAL;
  auto al16 = [](const void *p) { return p == nullptr || reinterpret_cast<uintptr_t>(p) % 16 == 0; };
  const int32_t vec = al16(chunk_a) && al16(chunk_b) && al16(nnf_a) && al16(nnf_b);
  // enough blocks to fill the chip, at most one per 4 * 256 pixels
  int64_t blocks = (n + 4 * kChangeThreads - 1) / (4 * kChangeThreads);
  if (blocks < 1) blocks = 1;
  if (blocks > kChangeBlocks) blocks = kChangeBlocks;
  uint64_t *part = static_cast<uint64_t *>(workspace);
  hipLaunchKernelGGL(k_change_partial, dim3(uint32_t(blocks)), dim3(kChangeThreads), 0, stream,
                     chunk_a, chunk_b, nnf_a, nnf_b, n, vec, part);
  hipLaunchKernelGGL(k_change_sum, dim3(1), dim3(kChangeThreads), 0, stream, part,
                     int32_t(blocks), counts);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_hip_error(e, "sb_frame_change");
    return SB_EHIP;
  }
  return SB_OK;
}

}  // extern "C"
