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

// Seed record of table entry idx (idx == total writes the sentinel record
// that out-of-table cells read).
template <int FMT>
__device__ inline void seeds_body(const FrameArgs &a, uint32_t idx) {
  const Levels &lv = a.lv;
  const uint32_t total = uint32_t(lv.offset[lv.count]);
  if (idx > total) return;
  uint2 rec = make_uint2(kNoSeed, 0u);
  if (idx < total) {
    int32_t i = 0;
    while (idx >= uint32_t(lv.offset[i + 1])) ++i;
    const uint32_t local = idx - uint32_t(lv.offset[i]);
    const uint32_t cx = local % uint32_t(lv.cells_x[i]);
    const uint32_t cy = local / uint32_t(lv.cells_x[i]);
    const uint32_t j = a.jitter[idx];
    const uint32_t sx = (cx << lv.log2_spacing[i]) + (j & 0xFFFFu);
    const uint32_t sy = (cy << lv.log2_spacing[i]) + (j >> 16);
    if (sx < uint32_t(a.w) && sy < uint32_t(a.h)) {
      const uint32_t g = guide_word<FMT>(a.tgt_guide, sy * uint32_t(a.w) + sx);
      const uint32_t u = a.lut[lut_bin(g, a.lut_shift, a.lut_bits)];
      rec.x = pack_xy(sx, sy);
      rec.y = pack_off(int32_t(u & 0xFFFFu) - int32_t(sx), int32_t(u >> 16) - int32_t(sy));
    }
  }
  a.seeds[idx] = rec;
}

template <int FMT>
__global__ void __launch_bounds__(256) k_seeds(FrameArgs a) {
  seeds_body<FMT>(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// Candidate of one level for pixel (x, y) from the nine seed records around
// its cell (loaded by the caller, out-of-table cells read the sentinel):
// NearestSeed's first strict minimum, then the source index to test (0 when
// the translated coordinate leaves the source, so the gather is issued
// unconditionally).
struct LevelCand {
  bool ok;
  uint32_t q, off, idx;
};

__device__ inline LevelCand pick(const uint2 rec[9], int32_t x, int32_t y, int32_t sw, int32_t sh) {
  uint32_t best = ~0u, bq = 0, bo = 0;
#pragma unroll
  for (int32_t k = 0; k < 9; ++k) {  // k = (dx+1)*3 + (dy+1): x outer, y inner
    const uint32_t ex = (rec[k].x & 0xFFFFu) - uint32_t(x), ey = (rec[k].x >> 16) - uint32_t(y);
    const uint32_t d = rec[k].x == kNoSeed ? ~0u : ex * ex + ey * ey;
    if (d < best) {
      best = d;
      bq = rec[k].x;
      bo = rec[k].y;
    }
  }
  LevelCand c;
  const int32_t vx = x + off_x(bo), vy = y + off_y(bo);
  c.ok = best != ~0u && uint32_t(vx) < uint32_t(sw) && uint32_t(vy) < uint32_t(sh);
  c.q = bq;
  c.off = bo;
  c.idx = c.ok ? uint32_t(vy) * uint32_t(sw) + uint32_t(vx) : 0u;
  return c;
}

__device__ inline void load_level(const FrameArgs &a, int32_t i, int32_t x, int32_t y,
                                  uint2 rec[9]) {
  const Levels &lv = a.lv;
  const int32_t ls = lv.log2_spacing[i];
  const int32_t bx = x >> ls, by = y >> ls;
  const int32_t ncx = lv.cells_x[i], ncy = lv.cells_y[i];
  const uint32_t none = uint32_t(lv.offset[lv.count]);  // the sentinel record
#pragma unroll
  for (int32_t k = 0; k < 9; ++k) {
    const int32_t cx = bx + k / 3 - 1, cy = by + k % 3 - 1;
    const bool in = cx >= 0 && cy >= 0 && cx < ncx && cy < ncy;
    rec[k] = a.seeds[in ? uint32_t(lv.offset[i] + cy * ncx + cx) : none];
  }
}

// One 16 x 16 pixel tile (tile index row-major over the frame's tiles).
template <int FMT>
__device__ inline void assign_body(const FrameArgs &a, uint32_t tile, uint32_t tid) {
  const uint32_t tiles_x = (uint32_t(a.w) + 15) / 16;
  const int32_t x = int32_t((tile % tiles_x) * 16 + (tid & 15));
  const int32_t y = int32_t((tile / tiles_x) * 16 + (tid >> 4));
  if (x >= a.w || y >= a.h) return;
  const uint32_t pidx = uint32_t(y) * uint32_t(a.w) + uint32_t(x);
  const uint32_t gt = guide_word<FMT>(a.tgt_guide, pidx);
  const int32_t L = a.lv.count;
  uint32_t chunk = 0, off = 0;
  bool done = false;
  // two levels per step: their 18 seed records, then both source-guide
  // gathers, are in flight together
  for (int32_t i = 0; i < L && !done; i += 2) {
    uint2 r0[9], r1[9];
    load_level(a, i, x, y, r0);
    const bool two = i + 1 < L;
    if (two) load_level(a, i + 1, x, y, r1);
    const LevelCand c0 = pick(r0, x, y, a.sw, a.sh);
    LevelCand c1;
    c1.ok = false;
    c1.idx = 0;
    c1.q = 0;
    c1.off = 0;
    if (two) c1 = pick(r1, x, y, a.sw, a.sh);
    const uint32_t g0 = guide_word<FMT>(a.src_guide, c0.idx);
    const uint32_t g1 = guide_word<FMT>(a.src_guide, c1.idx);
    if (c0.ok && error_below(gt, g0, a.threshold)) {
      chunk = (uint32_t(i) << 26) | ((c0.q >> 16) << 13) | (c0.q & 0xFFFFu);
      off = c0.off;
      done = true;
    } else if (c1.ok && error_below(gt, g1, a.threshold)) {
      chunk = (uint32_t(i + 1) << 26) | ((c1.q >> 16) << 13) | (c1.q & 0xFFFFu);
      off = c1.off;
      done = true;
    }
  }
  if (!done) {  // no level accepted: the pixel's own lookup
    const uint32_t u = a.lut[lut_bin(gt, a.lut_shift, a.lut_bits)];
    chunk = (uint32_t(L) << 26) | (uint32_t(y) << 13) | uint32_t(x);
    off = pack_off(int32_t(u & 0xFFFFu) - x, int32_t(u >> 16) - y);
  }
  a.out_chunk[pidx] = chunk;
  a.offsets[pidx] = off;
  if (a.out_nnf) a.out_nnf[pidx] = pack_xy(uint32_t(x + off_x(off)), uint32_t(y + off_y(off)));
}

typedef short short2_t __attribute__((ext_vector_type(2)));

// The level loop for one 8 x 8 block whose pixels share one cell at every
// level (every spacing >= 8 and <= 4096): the nine seed records of a level
// are wave-uniform scalar loads, and each lane scans them with a packed
// difference and a dot product, keeping min((d << 4) | k) -- the smallest
// squared distance d, ties to the first candidate k in scan order (x outer,
// y inner), exactly NearestSeed's first strict minimum.
// NearestSeed for a block's pixel at level i from the level's nine records
// (scalar loads at wave-uniform addresses): min over (d << 4) | k, i.e. the
// smallest squared distance d, ties to the first k in scan order.  Returns the
// record index of the winner, or `none` when the block has no in-image seed.
__device__ inline uint32_t scan_level(const FrameArgs &a, const uint2 *__restrict__ seeds,
                                      int32_t i, int32_t bx0, int32_t by0, short2_t pv,
                                      uint32_t none) {
  const Levels &lv = a.lv;
  const int32_t ls = lv.log2_spacing[i];
  const int32_t cx = bx0 >> ls, cy = by0 >> ls;
  const int32_t ncx = lv.cells_x[i], ncy = lv.cells_y[i], base = lv.offset[i];
  uint32_t key = ~0u;
#pragma unroll
  for (int32_t k = 0; k < 9; ++k) {
    const int32_t ccx = cx + k / 3 - 1, ccy = cy + k % 3 - 1;
    const bool tab = ccx >= 0 && ccy >= 0 && ccx < ncx && ccy < ncy;
    const uint32_t ridx = tab ? uint32_t(base + ccy * ncx + ccx) : none;
    const uint32_t pos = seeds[ridx].x;  // uniform address: scalar load
    if (pos != kNoSeed) {
      const short2_t dv = __builtin_bit_cast(short2_t, pos) - pv;
      const uint32_t d = uint32_t(__builtin_amdgcn_sdot2(dv, dv, 0, false));
      key = min(key, (d << 4) | uint32_t(k));
    }
  }
  if (key == ~0u) return none;
  const int32_t kk = int32_t(key & 15u);
  const int32_t kdx = (kk * 11) >> 5;  // kk / 3 for kk < 9
  return uint32_t(base + (cy + kk - 3 * kdx - 1) * ncx + (cx + kdx - 1));
}

// The level loop for one 8 x 8 block whose pixels share one cell at every
// level (every spacing >= 8 and <= 4096, so d << 4 stays below 2^31).  Two
// levels per step: both scans, both winning records, both source-guide
// gathers in flight together, then the tests in level order.
template <int FMT>
__device__ inline void assign_block(const FrameArgs &a, int32_t bx0, int32_t by0,
                                    int32_t lane) {
  const int32_t x = bx0 + (lane & 7), y = by0 + (lane >> 3);
  const bool in = x < a.w && y < a.h;
  const uint32_t pidx = in ? uint32_t(y) * uint32_t(a.w) + uint32_t(x) : 0u;
  const uint32_t gt = guide_word<FMT>(a.tgt_guide, pidx);
  const short2_t pv = __builtin_bit_cast(short2_t, pack_xy(uint32_t(x), uint32_t(y)));
  const uint2 *__restrict__ seeds = a.seeds;
  const int32_t L = a.lv.count;
  const uint32_t none = uint32_t(a.lv.offset[L]);  // the sentinel record
  uint32_t chunk = 0, off = 0;
  bool done = !in;
  for (int32_t i = 0; i < L; i += 2) {
    if (__all(done)) break;
    const uint32_t r0 = scan_level(a, seeds, i, bx0, by0, pv, none);
    const uint32_t r1 = i + 1 < L ? scan_level(a, seeds, i + 1, bx0, by0, pv, none) : none;
    const uint2 c0 = seeds[r0], c1 = seeds[r1];  // the sentinel when none
    const int32_t vx0 = x + off_x(c0.y), vy0 = y + off_y(c0.y);
    const int32_t vx1 = x + off_x(c1.y), vy1 = y + off_y(c1.y);
    const bool ok0 = c0.x != kNoSeed && uint32_t(vx0) < uint32_t(a.sw) && uint32_t(vy0) < uint32_t(a.sh);
    const bool ok1 = c1.x != kNoSeed && uint32_t(vx1) < uint32_t(a.sw) && uint32_t(vy1) < uint32_t(a.sh);
    const uint32_t g0 = guide_word<FMT>(a.src_guide, ok0 ? uint32_t(vy0) * uint32_t(a.sw) + uint32_t(vx0) : 0u);
    const uint32_t g1 = guide_word<FMT>(a.src_guide, ok1 ? uint32_t(vy1) * uint32_t(a.sw) + uint32_t(vx1) : 0u);
    if (!done && ok0 && error_below(gt, g0, a.threshold)) {
      chunk = (uint32_t(i) << 26) | ((c0.x >> 16) << 13) | (c0.x & 0xFFFFu);
      off = c0.y;
      done = true;
    }
    if (!done && ok1 && error_below(gt, g1, a.threshold)) {
      chunk = (uint32_t(i + 1) << 26) | ((c1.x >> 16) << 13) | (c1.x & 0xFFFFu);
      off = c1.y;
      done = true;
    }
  }
  if (!in) return;
  if (!done) {  // no level accepted: the pixel's own lookup
    const uint32_t u = a.lut[lut_bin(gt, a.lut_shift, a.lut_bits)];
    chunk = (uint32_t(L) << 26) | (uint32_t(y) << 13) | uint32_t(x);
    off = pack_off(int32_t(u & 0xFFFFu) - x, int32_t(u >> 16) - y);
  }
  a.out_chunk[pidx] = chunk;
  a.offsets[pidx] = off;
  if (a.out_nnf) a.out_nnf[pidx] = pack_xy(uint32_t(x + off_x(off)), uint32_t(y + off_y(off)));
}

// Whether every level's cells hold whole 8 x 8 blocks and distances stay
// below 2^27 (spacings 8 ... 4096).
__device__ inline bool uniform_cells(const Levels &lv) {
  return lv.count == 0 || (lv.log2_spacing[lv.count - 1] >= 3 && lv.log2_spacing[0] <= 12);
}

// One 16 x 16 tile: four 8 x 8 blocks, one per wave, on the uniform-cell
// path; otherwise one pixel per thread on the general path.
template <int FMT>
__device__ inline void assign_tile(const FrameArgs &a, uint32_t tile, uint32_t tid) {
  if (uniform_cells(a.lv)) {
    const uint32_t tiles_x = (uint32_t(a.w) + 15) / 16;
    const int32_t wave = __builtin_amdgcn_readfirstlane(int32_t(tid >> 6));
    const int32_t bx0 = int32_t((tile % tiles_x) * 16) + (wave & 1) * 8;
    const int32_t by0 = int32_t((tile / tiles_x) * 16) + (wave >> 1) * 8;
    assign_block<FMT>(a, bx0, by0, int32_t(tid & 63));
  } else {
    assign_body<FMT>(a, tile, tid);
  }
}

template <int FMT>
__global__ void __launch_bounds__(256) k_assign(FrameArgs a) {
  assign_tile<FMT>(a, blockIdx.x, threadIdx.x);
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

// The votes of one pixel: (2r+1)^2 gathers issued in batches of up to ~25
// with out-of-source votes reading texel 0 and masked out of the sums.
template <int R>
__device__ inline uint32_t vote(const uint32_t *tile, int32_t lw, int32_t lx, int32_t ly,
                                int32_t x, int32_t y, const uint32_t *rgba, uint32_t sw,
                                uint32_t sh) {
  constexpr int W = 2 * R + 1;
  constexpr int ROWS = W * W <= 9 ? W : 1;  // gathers of one row in flight together
  uint32_t rb = 0, g = 0, k = 0;
#pragma unroll 1
  for (int32_t r0 = 0; r0 < W; r0 += ROWS) {
    uint32_t idx[ROWS * W];
    bool ok[ROWS * W];
#pragma unroll
    for (int32_t q = 0; q < ROWS * W; ++q) {
      ok[q] = false;
      idx[q] = 0;
      if (r0 + q / W < W) {
        const uint32_t o = tile[(ly + r0 + q / W) * lw + lx + q % W];
        const int32_t sx = x + off_x(o), sy = y + off_y(o);
        ok[q] = uint32_t(sx) < sw && uint32_t(sy) < sh;
        idx[q] = ok[q] ? uint32_t(sy) * sw + uint32_t(sx) : 0u;
      }
    }
    uint32_t t[ROWS * W];
#pragma unroll
    for (int32_t q = 0; q < ROWS * W; ++q) t[q] = rgba[idx[q]];
#pragma unroll
    for (int32_t q = 0; q < ROWS * W; ++q) {
      const uint32_t c = ok[q] ? t[q] : 0u;
      rb += c & 0x00FF00FFu;
      g += c & 0x0000FF00u;
      k += ok[q] ? 1u : 0u;
    }
  }
  const uint32_t h = k >> 1;
  return div_small((rb & 0xFFFFu) + h, k) | (div_small((g >> 8) + h, k) << 8) |
         (div_small((rb >> 16) + h, k) << 16);
}

// The votes of one pixel when every neighbour's source patch lies inside the
// source.  `lin` holds, per tile cell n, 4 * (raster index of NNF[n]) with two
// flags in the low bits: bit 0 when n has the same offset NNF[n] - n as its
// left neighbour, bit 1 when it has the same offset as the neighbour above.
// A vote's texel address is a per-row scalar base plus that byte offset (flags
// cleared) plus a per-column immediate.  Moving one column right within a run
// of equal offsets reads the same texel (and likewise one row down), so a lane
// loads only where its window's run starts and reuses the texel otherwise.
// The vote count is the constant (2r+1)^2.
template <int R>
__device__ inline uint32_t vote_inside(const uint32_t *lin, int32_t lw, int32_t lx, int32_t ly,
                                       const unsigned char *texels, uint32_t sw) {
  constexpr int W = 2 * R + 1;
  uint32_t rb = 0, g = 0;
  uint32_t up[W];
#pragma unroll
  for (int32_t dx = 0; dx < W; ++dx) up[dx] = 0;
#pragma unroll 1
  for (int32_t dy = 0; dy < W; ++dy) {
    // neighbour n = p + (dx - R, dy - R) votes with NNF[n] - (dx - R, dy - R)
    const unsigned char *row = texels - int64_t(dy - R) * int64_t(sw) * 4;
    const uint32_t *lrow = lin + (ly + dy) * lw + lx;
    uint32_t left = 0;
#pragma unroll
    for (int32_t dx = 0; dx < W; ++dx) {
      const uint32_t v = lrow[dx];
      uint32_t t;
      if (dx > 0 && (v & 1u)) t = left;
      else if (dy > 0 && (v & 2u)) t = up[dx];
      else t = *reinterpret_cast<const uint32_t *>(row + uint64_t(v & ~3u) - 4 * (dx - R));
      rb += t & 0x00FF00FFu;
      g += t & 0x0000FF00u;
      left = t;
      up[dx] = t;
    }
  }
  constexpr uint32_t k = W * W, hk = k / 2;
  return (((rb & 0xFFFFu) + hk) / k) | ((((g >> 8) + hk) / k) << 8) |
         ((((rb >> 16) + hk) / k) << 16);
}

__device__ inline uint32_t vote_inside_any(int32_t r, const uint32_t *lin, int32_t lw, int32_t lx,
                                           int32_t ly, const unsigned char *texels, uint32_t sw) {
  switch (r) {
    case 0: return vote_inside<0>(lin, lw, lx, ly, texels, sw);
    case 1: return vote_inside<1>(lin, lw, lx, ly, texels, sw);
    case 2: return vote_inside<2>(lin, lw, lx, ly, texels, sw);
    case 3: return vote_inside<3>(lin, lw, lx, ly, texels, sw);
    case 4: return vote_inside<4>(lin, lw, lx, ly, texels, sw);
    case 5: return vote_inside<5>(lin, lw, lx, ly, texels, sw);
    case 6: return vote_inside<6>(lin, lw, lx, ly, texels, sw);
    default: return vote_inside<7>(lin, lw, lx, ly, texels, sw);
  }
}

// One 32 x 8 pixel tile.  `tile` is LDS for two (32 + 2r) x (8 + 2r) arrays:
// the offsets NNF[n] - n and, when the whole tile votes inside the source,
// the texel byte offsets of NNF[n].  Each wave covers two rows; a wave whose
// voting footprint holds one offset copies C_S[NNF[p]] (every vote is that
// texel).  Ends with all threads past their last LDS read (callers that reuse
// the tile synchronise before refilling it).
__device__ inline void blend_body(const FrameArgs &a, uint32_t t_index, uint32_t tid,
                                  uint32_t *tile) {
  const int32_t r = a.radius;
  const int32_t lw = kBlendTW + 2 * r, lh = kBlendTH + 2 * r;
  const int32_t nel = lw * lh;  // <= 46 * 22, at most 4 per thread
  uint32_t *toff = tile, *tlin = tile + nel;
  const uint32_t tiles_x = (uint32_t(a.w) + kBlendTW - 1) / kBlendTW;
  const int32_t x0 = int32_t(t_index % tiles_x) * kBlendTW - r;
  const int32_t y0 = int32_t(t_index / tiles_x) * kBlendTH - r;
  const uint32_t sw = uint32_t(a.sw), sh = uint32_t(a.sh);
  uint32_t ov[4];
  bool inside = true;
#pragma unroll
  for (int32_t e = 0; e < 4; ++e) {
    const int32_t t = int32_t(tid) + 256 * e;
    ov[e] = kNoVote;
    if (t < nel) {
      const int32_t tx = x0 + t % lw, ty = y0 + t / lw;
      if (tx >= 0 && ty >= 0 && tx < a.w && ty < a.h) ov[e] = a.offsets[uint32_t(ty) * a.w + uint32_t(tx)];
      const int32_t nx = tx + off_x(ov[e]), ny = ty + off_y(ov[e]);
      inside &= ov[e] != kNoVote && nx >= r && ny >= r && nx < int32_t(sw) - r &&
                ny < int32_t(sh) - r;
    }
  }
#pragma unroll
  for (int32_t e = 0; e < 4; ++e) {
    const int32_t t = int32_t(tid) + 256 * e;
    if (t < nel) toff[t] = ov[e];
  }
  const bool all_inside = __syncthreads_and(inside);  // also orders the toff writes
  if (all_inside) {
#pragma unroll
    for (int32_t e = 0; e < 4; ++e) {
      const int32_t t = int32_t(tid) + 256 * e;
      if (t < nel) {
        const int32_t cx = t % lw, cy = t / lw;
        const int32_t tx = x0 + cx, ty = y0 + cy;
        uint32_t v = (uint32_t(ty + off_y(ov[e])) * sw + uint32_t(tx + off_x(ov[e]))) * 4u;
        if (cx > 0 && toff[t - 1] == ov[e]) v |= 1u;
        if (cy > 0 && toff[t - lw] == ov[e]) v |= 2u;
        tlin[t] = v;
      }
    }
  }
  __syncthreads();
  const int32_t lx = int32_t(tid) & (kBlendTW - 1), ly = int32_t(tid) / kBlendTW;
  const int32_t x = x0 + r + lx, y = y0 + r + ly;
  // a wave's footprint: rows [2w, 2w + 2 + 2r) of the tile, all columns
  const int32_t lane = int32_t(tid) & 63, wrow = (int32_t(tid) >> 6) * 2;
  const uint32_t ref = toff[(wrow + r) * lw + r];
  bool same = ref != kNoVote;
  for (int32_t q = lane; q < lw * (2 + 2 * r); q += 64) same &= toff[wrow * lw + q] == ref;
  const bool copy = __all(same);
  if (x >= a.w || y >= a.h) return;
  uint32_t c;
  if (copy) {
    c = a.src_rgba[uint32_t(y + off_y(ref)) * sw + uint32_t(x + off_x(ref))];
  } else if (all_inside) {
    c = vote_inside_any(r, tlin, lw, lx, ly, reinterpret_cast<const unsigned char *>(a.src_rgba), sw);
  } else {
    switch (r) {
      case 0: c = vote<0>(toff, lw, lx, ly, x, y, a.src_rgba, sw, sh); break;
      case 1: c = vote<1>(toff, lw, lx, ly, x, y, a.src_rgba, sw, sh); break;
      case 2: c = vote<2>(toff, lw, lx, ly, x, y, a.src_rgba, sw, sh); break;
      case 3: c = vote<3>(toff, lw, lx, ly, x, y, a.src_rgba, sw, sh); break;
      case 4: c = vote<4>(toff, lw, lx, ly, x, y, a.src_rgba, sw, sh); break;
      case 5: c = vote<5>(toff, lw, lx, ly, x, y, a.src_rgba, sw, sh); break;
      case 6: c = vote<6>(toff, lw, lx, ly, x, y, a.src_rgba, sw, sh); break;
      default: c = vote<7>(toff, lw, lx, ly, x, y, a.src_rgba, sw, sh); break;
    }
  }
  uint8_t *o = a.out_rgb + 3 * (uint32_t(y) * uint32_t(a.w) + uint32_t(x));
  o[0] = uint8_t(c);
  o[1] = uint8_t(c >> 8);
  o[2] = uint8_t(c >> 16);
}

__global__ void __launch_bounds__(256) k_blend(FrameArgs a) {
  extern __shared__ uint32_t tile[];
  blend_body(a, blockIdx.x, threadIdx.x, tile);
}

// ------------------------------------------------------------------ batches
//
// A batch runs the same three passes over many frames: each kernel is
// persistent (a fixed grid striding over the concatenated tiles of all
// frames) and reads the frames' arguments from a descriptor block in device
// memory, so one captured graph serves any mix of sizes and formats.

// Frame owning global tile t: the last f with pre[f] <= t (pre in LDS).
__device__ inline uint32_t frame_of(const uint32_t *pre, uint32_t n, uint32_t t) {
  uint32_t lo = 0, hi = n;  // pre[lo] <= t < pre[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (pre[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int KIND>
__global__ void __launch_bounds__(256) k_batch(const unsigned char *desc) {
  extern __shared__ uint32_t dyn[];  // blend tile
  __shared__ uint32_t pre[kMaxBatchFrames + 1];
  const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(desc);
  const uint32_t n = hd->nframes;
  const uint32_t *gpre = reinterpret_cast<const uint32_t *>(desc + batch_prefix_offset(KIND));
  for (uint32_t i = threadIdx.x; i <= n; i += 256) pre[i] = gpre[i];
  __syncthreads();
  const FrameArgs *frames = reinterpret_cast<const FrameArgs *>(desc + batch_frames_offset());
  const uint32_t total = pre[n];
  for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
    const uint32_t f = frame_of(pre, n, t);
    const FrameArgs &a = frames[f];
    const uint32_t local = t - pre[f];
    if (KIND == 0) {
      const uint32_t idx = local * 256 + threadIdx.x;
      if (a.fmt == SB_GUIDE_U8X2) seeds_body<SB_GUIDE_U8X2>(a, idx);
      else seeds_body<SB_GUIDE_U16X2>(a, idx);
    } else if (KIND == 1) {
      if (a.fmt == SB_GUIDE_U8X2) assign_tile<SB_GUIDE_U8X2>(a, local, threadIdx.x);
      else assign_tile<SB_GUIDE_U16X2>(a, local, threadIdx.x);
    } else {
      blend_body(a, local, threadIdx.x, dyn);
      __syncthreads();  // the next tile refills the LDS tile
    }
  }
}

unsigned blocks_for(uint64_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_pack_exemplar(const uint8_t *rgb, int32_t sw, int32_t sh, uint32_t *rgba,
                                hipStream_t stream) {
  const uint32_t n = uint32_t(sw) * uint32_t(sh);
  k_pack_exemplar<<<blocks_for(n, 256), 256, 0, stream>>>(rgb, n, rgba);
  return hipGetLastError();
}

void tile_counts(const FrameArgs &a, uint32_t counts[3]) {
  counts[0] = (uint32_t(a.lv.offset[a.lv.count]) + 1 + 255) / 256;  // + sentinel
  counts[1] = ((uint32_t(a.w) + 15) / 16) * ((uint32_t(a.h) + 15) / 16);
  counts[2] = ((uint32_t(a.w) + kBlendTW - 1) / kBlendTW) * ((uint32_t(a.h) + kBlendTH - 1) / kBlendTH);
}

hipError_t launch_stylize(const FrameArgs &a, int32_t fmt, hipStream_t stream) {
  uint32_t c[3];
  tile_counts(a, c);
  if (fmt == SB_GUIDE_U8X2)
    k_seeds<SB_GUIDE_U8X2><<<c[0], 256, 0, stream>>>(a);
  else
    k_seeds<SB_GUIDE_U16X2><<<c[0], 256, 0, stream>>>(a);
  if (fmt == SB_GUIDE_U8X2)
    k_assign<SB_GUIDE_U8X2><<<c[1], 256, 0, stream>>>(a);
  else
    k_assign<SB_GUIDE_U16X2><<<c[1], 256, 0, stream>>>(a);
  const size_t lds = size_t(kBlendTW + 2 * a.radius) * (kBlendTH + 2 * a.radius) * 8;
  k_blend<<<c[2], 256, lds, stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_batch(const unsigned char *desc_dev, uint32_t grid, hipStream_t stream) {
  const size_t lds = size_t(kBlendTW + 2 * SB_MAX_RADIUS) * (kBlendTH + 2 * SB_MAX_RADIUS) * 8;
  k_batch<0><<<grid, 256, 0, stream>>>(desc_dev);
  k_batch<1><<<grid, 256, 0, stream>>>(desc_dev);
  k_batch<2><<<grid, 256, lds, stream>>>(desc_dev);
  return hipGetLastError();
}

}  // namespace sb
