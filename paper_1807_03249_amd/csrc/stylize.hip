// stylize.hip -- per-frame StyleBlit kernels for gfx950.
//
//   k_seeds   one thread per cell of every level: the jittered seed
//             (SeedPoint, Algorithm 2), whether it is inside the target, and
//             the translation u* - q its lookup (Sec. 3.1) gives the chunk it
//             starts.  Tiny: one record per seed.
//   k_assign  one thread per target pixel: the level loop of Algorithm 2,
//             NearestSeed over the 3x3 cells from the seed records, the exact
//             integer guide error at u* + (p - q) against the threshold, and
//             the own-lookup fallback.  Writes the chunk code and the offset
//             NNF[p] - p.
//   k_blend   the voting step (end of Sec. 3.2): a tile of offsets plus an
//             r-pixel halo in LDS, (2r+1)^2 votes per pixel gathered from the
//             RGBA exemplar, integer average rounded half up.
#include "sb_internal.h"

namespace sb {
namespace {

template <int FMT>
__device__ inline uint32_t guide_word(const void *g, uint32_t i) {
  if (FMT == SB_GUIDE_U8X2) {
    uint32_t v = static_cast<const uint16_t *>(g)[i];
    return (v & 0xFFu) | ((v >> 8) << 16);  // unpack to the u16 pair layout
  } else {
    return static_cast<const uint32_t *>(g)[i];
  }
}

// Lookup-table bin of a guide word (two channels, 16 bits apart).
__device__ inline uint32_t lut_bin(uint32_t g, int32_t shift, int32_t bits) {
  return ((g & 0xFFFFu) >> shift) | (((g >> 16) >> shift) << bits);
}

// Exact squared L2 error of two guide words compared with t: true iff e < t.
__device__ inline bool error_below(uint32_t a, uint32_t b, uint32_t t) {
  const int32_t d0 = int32_t(a & 0xFFFFu) - int32_t(b & 0xFFFFu);
  const int32_t d1 = int32_t(a >> 16) - int32_t(b >> 16);
  const uint64_t e = uint64_t(uint32_t(d0 * d0)) + uint64_t(uint32_t(d1 * d1));
  return e < uint64_t(t);
}

// Offsets are two int16 in one word; x in the low half.
__device__ inline uint32_t pack_off(int32_t dx, int32_t dy) {
  return (uint32_t(dx) & 0xFFFFu) | (uint32_t(dy) << 16);
}
__device__ inline int32_t off_x(uint32_t o) { return int32_t(int16_t(o & 0xFFFFu)); }
__device__ inline int32_t off_y(uint32_t o) { return int32_t(int16_t(o >> 16)); }

__global__ void k_pack_exemplar(const uint8_t *rgb, uint32_t n, uint32_t *rgba) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  rgba[i] = uint32_t(rgb[3 * i]) | (uint32_t(rgb[3 * i + 1]) << 8) | (uint32_t(rgb[3 * i + 2]) << 16);
}

template <int FMT>
__global__ void k_seeds(FrameArgs a) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  const Levels &lv = a.lv;
  if (idx >= uint32_t(lv.offset[lv.count])) return;
  int32_t i = 0;
  while (idx >= uint32_t(lv.offset[i + 1])) ++i;
  const uint32_t local = idx - uint32_t(lv.offset[i]);
  const uint32_t cx = local % uint32_t(lv.cells_x[i]);
  const uint32_t cy = local / uint32_t(lv.cells_x[i]);
  const uint32_t j = a.jitter[idx];
  const uint32_t sx = (cx << lv.log2_spacing[i]) + (j & 0xFFFFu);
  const uint32_t sy = (cy << lv.log2_spacing[i]) + (j >> 16);
  uint2 rec = make_uint2(kNoSeed, 0u);
  if (sx < uint32_t(a.w) && sy < uint32_t(a.h)) {
    const uint32_t g = guide_word<FMT>(a.tgt_guide, sy * uint32_t(a.w) + sx);
    const uint32_t u = a.lut[lut_bin(g, a.lut_shift, a.lut_bits)];
    rec.x = pack_xy(sx, sy);
    rec.y = pack_off(int32_t(u & 0xFFFFu) - int32_t(sx), int32_t(u >> 16) - int32_t(sy));
  }
  a.seeds[idx] = rec;
}

template <int FMT>
__global__ void __launch_bounds__(256) k_assign(FrameArgs a) {
  const int32_t x = int32_t(blockIdx.x * 16 + (threadIdx.x & 15));
  const int32_t y = int32_t(blockIdx.y * 16 + (threadIdx.x >> 4));
  if (x >= a.w || y >= a.h) return;
  const uint32_t pidx = uint32_t(y) * uint32_t(a.w) + uint32_t(x);
  const uint32_t gt = guide_word<FMT>(a.tgt_guide, pidx);
  const Levels &lv = a.lv;
  uint32_t chunk = 0, off = 0;
  bool done = false;
  for (int32_t i = 0; i < lv.count && !done; ++i) {
    const int32_t ls = lv.log2_spacing[i];
    const int32_t bx = x >> ls, by = y >> ls;
    const int32_t ncx = lv.cells_x[i], ncy = lv.cells_y[i];
    const uint2 *tab = a.seeds + lv.offset[i];
    uint32_t best = ~0u, bq = 0, bo = 0;
    for (int32_t dx = -1; dx <= 1; ++dx) {      // NearestSeed: x outer,
      const int32_t cx = bx + dx;
      if (cx < 0 || cx >= ncx) continue;
      for (int32_t dy = -1; dy <= 1; ++dy) {    // y inner, first strict minimum
        const int32_t cy = by + dy;
        if (cy < 0 || cy >= ncy) continue;
        const uint2 rec = tab[cy * ncx + cx];
        if (rec.x == kNoSeed) continue;
        const int32_t ex = int32_t(rec.x & 0xFFFFu) - x, ey = int32_t(rec.x >> 16) - y;
        const uint32_t d = uint32_t(ex * ex + ey * ey);
        if (d < best) {
          best = d;
          bq = rec.x;
          bo = rec.y;
        }
      }
    }
    if (best == ~0u) continue;  // no in-image seed around p at this level
    const int32_t vx = x + off_x(bo), vy = y + off_y(bo);
    if (uint32_t(vx) >= uint32_t(a.sw) || uint32_t(vy) >= uint32_t(a.sh)) continue;
    const uint32_t gs = guide_word<FMT>(a.src_guide, uint32_t(vy) * uint32_t(a.sw) + uint32_t(vx));
    if (error_below(gt, gs, a.threshold)) {
      chunk = (uint32_t(i) << 26) | ((bq >> 16) << 13) | (bq & 0xFFFFu);
      off = bo;
      done = true;
    }
  }
  if (!done) {  // no level accepted: the pixel's own lookup
    const uint32_t u = a.lut[lut_bin(gt, a.lut_shift, a.lut_bits)];
    chunk = (uint32_t(lv.count) << 26) | (uint32_t(y) << 13) | uint32_t(x);
    off = pack_off(int32_t(u & 0xFFFFu) - x, int32_t(u >> 16) - y);
  }
  a.out_chunk[pidx] = chunk;
  a.offsets[pidx] = off;
  if (a.out_nnf) a.out_nnf[pidx] = pack_xy(uint32_t(x + off_x(off)), uint32_t(y + off_y(off)));
}

// Exact n / k for n < 2^20 and 1 <= k <= 225 via a float reciprocal and one
// correction step each way.
__device__ inline uint32_t div_small(uint32_t n, uint32_t k) {
  uint32_t q = uint32_t(float(n) * __builtin_amdgcn_rcpf(float(k)));
  int32_t r = int32_t(n) - int32_t(q * k);
  if (r < 0) --q;
  else if (r >= int32_t(k)) ++q;
  return q;
}

constexpr int kBlendTW = 32, kBlendTH = 8;

__global__ void __launch_bounds__(256) k_blend(FrameArgs a) {
  extern __shared__ uint32_t tile[];  // (TW + 2r) x (TH + 2r) offsets
  const int32_t r = a.radius;
  const int32_t lw = kBlendTW + 2 * r, lh = kBlendTH + 2 * r;
  const int32_t x0 = int32_t(blockIdx.x) * kBlendTW - r, y0 = int32_t(blockIdx.y) * kBlendTH - r;
  for (int32_t t = threadIdx.x; t < lw * lh; t += 256) {
    const int32_t tx = x0 + t % lw, ty = y0 + t / lw;
    uint32_t o = kNoVote;
    if (tx >= 0 && ty >= 0 && tx < a.w && ty < a.h) o = a.offsets[uint32_t(ty) * a.w + uint32_t(tx)];
    tile[t] = o;
  }
  __syncthreads();
  const int32_t lx = threadIdx.x & (kBlendTW - 1), ly = threadIdx.x / kBlendTW;
  const int32_t x = x0 + r + lx, y = y0 + r + ly;
  if (x >= a.w || y >= a.h) return;
  uint32_t rb = 0, g = 0, k = 0;
  for (int32_t dy = 0; dy <= 2 * r; ++dy) {
    for (int32_t dx = 0; dx <= 2 * r; ++dx) {
      const uint32_t o = tile[(ly + dy) * lw + lx + dx];
      // the neighbour's source patch, co-located with p: p + (NNF[n] - n)
      const int32_t sx = x + off_x(o), sy = y + off_y(o);
      if (uint32_t(sx) < uint32_t(a.sw) && uint32_t(sy) < uint32_t(a.sh) && o != kNoVote) {
        const uint32_t c = a.src_rgba[uint32_t(sy) * uint32_t(a.sw) + uint32_t(sx)];
        rb += c & 0x00FF00FFu;
        g += c & 0x0000FF00u;
        ++k;
      }
    }
  }
  const uint32_t h = k >> 1;
  uint8_t *o = a.out_rgb + 3 * (uint32_t(y) * uint32_t(a.w) + uint32_t(x));
  o[0] = uint8_t(div_small((rb & 0xFFFFu) + h, k));
  o[1] = uint8_t(div_small((g >> 8) + h, k));
  o[2] = uint8_t(div_small((rb >> 16) + h, k));
}

unsigned blocks_for(uint64_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_pack_exemplar(const uint8_t *rgb, int32_t sw, int32_t sh, uint32_t *rgba,
                                hipStream_t stream) {
  const uint32_t n = uint32_t(sw) * uint32_t(sh);
  k_pack_exemplar<<<blocks_for(n, 256), 256, 0, stream>>>(rgb, n, rgba);
  return hipGetLastError();
}

hipError_t launch_stylize(const FrameArgs &a, int32_t fmt, hipStream_t stream) {
  const uint32_t ncells = uint32_t(a.lv.offset[a.lv.count]);
  if (ncells) {
    if (fmt == SB_GUIDE_U8X2)
      k_seeds<SB_GUIDE_U8X2><<<blocks_for(ncells, 256), 256, 0, stream>>>(a);
    else
      k_seeds<SB_GUIDE_U16X2><<<blocks_for(ncells, 256), 256, 0, stream>>>(a);
  }
  dim3 ga(blocks_for(a.w, 16), blocks_for(a.h, 16));
  if (fmt == SB_GUIDE_U8X2)
    k_assign<SB_GUIDE_U8X2><<<ga, 256, 0, stream>>>(a);
  else
    k_assign<SB_GUIDE_U16X2><<<ga, 256, 0, stream>>>(a);
  dim3 gb(blocks_for(a.w, kBlendTW), blocks_for(a.h, kBlendTH));
  const size_t lds = size_t(kBlendTW + 2 * a.radius) * (kBlendTH + 2 * a.radius) * 4;
  k_blend<<<gb, 256, lds, stream>>>(a);
  return hipGetLastError();
}

}  // namespace sb
