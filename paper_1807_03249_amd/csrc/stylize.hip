// stylize.hip -- per-frame StyleBlit kernels for gfx950.
//
//   k_seeds   one thread per record of the padded seed table: the jittered
//             seed of a cell (SeedPoint, Algorithm 2) if it lies in the
//             target, and the translation u* - q its lookup (Sec. 3.1) gives
//             the chunk it starts; the ring around each level's grid and
//             out-of-image seeds hold the empty record.
//   k_assign  the level loop of Algorithm 2 per pixel: NearestSeed over the
//             3x3 cells, the exact integer guide error at u* + (p - q)
//             against the threshold (with the segmentation guide, also the
//             label test), and the own-lookup fallback.  Writes the chunk
//             code and the offset NNF[p] - p as the byte distance the vote
//             adds in the padded exemplar.
//   k_blend   the voting step (end of Sec. 3.2): a tile of offsets with an
//             r-pixel halo in LDS; each lane averages the (2r+1)^2 votes of
//             four adjacent pixels, one vector gather per (cell, pixel run).
//
// Every side is at most SB_MAX_SIDE = 8192 (the chunk code holds 13-bit
// coordinates), so pixel and texel indices are formed with full-rate 24-bit
// multiplies (__umul24 / __mul24) instead of 32- or 64-bit ones.
#include "sb_device.h"

namespace sb {
namespace {

// Dword-aligned vectors of 2..4 texels (global loads need dword alignment
// only).
typedef uint32_t u32x2a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32x3a4 __attribute__((ext_vector_type(3), aligned(4)));
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// A guide texel as stored (2 x u8, 2 x u16 or 3 x u8 in a word) and unpacked
// to its guide word: two channels as a u16 pair (channel 1 in the high
// half), or three u8 channels in bytes 0..2 (byte 3 cleared).
template <int FMT>
__device__ inline uint32_t guide_raw(const void *g, uint32_t i) {
  if (FMT == SB_GUIDE_U8X2) return glb(static_cast<const uint16_t *>(g))[i];
  return glb(static_cast<const uint32_t *>(g))[i];
}
template <int FMT>
__device__ inline uint32_t guide_unpack(uint32_t v) {
  if (FMT == SB_GUIDE_U8X2) return (v & 0xFFu) | ((v >> 8) << 16);
  if (FMT == SB_GUIDE_U8X3) return v & 0xFFFFFFu;
  return v;
}
template <int FMT>
__device__ inline uint32_t guide_word(const void *g, uint32_t i) {
  return guide_unpack<FMT>(guide_raw<FMT>(g, i));
}

// Lookup-table bin of a guide word: c0 | c1 << bits (| c2 << 2 bits), each
// channel's top `bits` bits.
template <int FMT>
__device__ inline uint32_t lut_bin(uint32_t g, int32_t shift, int32_t bits) {
  if (FMT == SB_GUIDE_U8X3)
    return ((g & 0xFFu) >> shift) | ((((g >> 8) & 0xFFu) >> shift) << bits) |
           (((g >> 16) >> shift) << (2 * bits));
  return ((g & 0xFFFFu) >> shift) | (((g >> 16) >> shift) << bits);
}

// Exact squared L2 error of two guide words compared with t: true iff e < t.
// 8-bit channels: the differences fit int16, one packed subtract and one
// dot product.  Three channels carry weights w0..w2 <= 127 (w02 = w0 | w2 <<
// 16, w1): channels 0 and 2 as the packed pair against their weighted
// differences (|w d| <= 127 * 255 fits int16), channel 1's weighted square as
// the accumulator; e <= 3 * 127 * 255^2.  16-bit channels: 24-bit multiplies
// (|d| < 2^16, d^2 < 2^32) and a saturating add (a sum that saturates is >=
// 2^32 - 1 >= t anyway).
template <int FMT>
__device__ inline bool error_below(uint32_t a, uint32_t b, uint32_t t, uint32_t w02, int32_t w1) {
  if (FMT == SB_GUIDE_U8X2) {
    const short2_t d = __builtin_bit_cast(short2_t, a) - __builtin_bit_cast(short2_t, b);
    return uint32_t(__builtin_amdgcn_sdot2(d, d, 0, false)) < t;
  } else if (FMT == SB_GUIDE_U8X3) {
    const uint32_t m = 0x00FF00FFu;
    const short2_t d = __builtin_bit_cast(short2_t, a & m) - __builtin_bit_cast(short2_t, b & m);
    const short2_t dw = d * __builtin_bit_cast(short2_t, w02);
    const int32_t d1 = int32_t((a >> 8) & 0xFFu) - int32_t((b >> 8) & 0xFFu);
    return uint32_t(__builtin_amdgcn_sdot2(d, dw, __mul24(d1, __mul24(d1, w1)), false)) < t;
  } else {
    const int32_t d0 = int32_t(a & 0xFFFFu) - int32_t(b & 0xFFFFu);
    const int32_t d1 = int32_t(a >> 16) - int32_t(b >> 16);
    const uint32_t e0 = uint32_t(__mul24(d0, d0));
    const uint32_t e1 = uint32_t(__mul24(d1, d1));
    return __builtin_elementwise_add_sat(e0, e1) < t;
  }
}

// Every texel of the padded exemplar: source texels with alpha 1, margins and
// zero rows 0.
__global__ void k_pack_exemplar(const uint8_t *rgb, int32_t sw, int32_t sh, uint32_t n,
                                uint32_t *rgba) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t P = ex_stride(sw);
  const int32_t x = int32_t(i % uint32_t(P)) - kExMargin, y = int32_t(i / uint32_t(P)) - kExMargin;
  uint32_t t = 0;
  if (x >= 0 && y >= 0 && x < sw && y < sh) {
    const uint8_t *c = rgb + 3 * (size_t(y) * size_t(sw) + size_t(x));
    t = uint32_t(c[0]) | (uint32_t(c[1]) << 8) | (uint32_t(c[2]) << 16) | (1u << 24);
  }
  rgba[i] = t;
}

// The lookup table a target pixel uses: the unconstrained one, or with the
// segmentation guide the table of the pixel's label (past the last label:
// the last table).
__device__ inline const uint32_t *lut_of(const FrameArgs &a, uint32_t pidx) {
  if (!a.tgt_labels) return a.lut;
  const uint32_t l = min(uint32_t(glb(a.tgt_labels)[pidx]), uint32_t(a.nlabels - 1));
  return a.label_luts + (size_t(l) << a.lut_log2);
}

// The seed record of cell (cx, cy) of a level with log2 spacing ls, a
// ncx x ncy cell grid, its jitter entries from joff on and hash state hk
// (SeedPoint and the seed's lookup): position 4x | 4y << 16 and the
// translation u* - q, or the empty record for a cell outside the grid or a
// seed outside the target.
template <int FMT>
__device__ inline u32x2 seed_record(const FrameArgs &a, int32_t ls, int32_t ncx, int32_t ncy,
                                    int32_t joff, uint32_t hk, int32_t cx, int32_t cy) {
  u32x2 rec = {kNoSeed, 0u};
  if (cx >= 0 && cy >= 0 && cx < ncx && cy < ncy) {
    const uint32_t j = cell_jitter(a, ls, ncx, joff, hk, cx, cy);
    const uint32_t sx = (uint32_t(cx) << ls) + (j & 0xFFFFu);
    const uint32_t sy = (uint32_t(cy) << ls) + (j >> 16);
    if (sx < uint32_t(a.w) && sy < uint32_t(a.h)) {
      const uint32_t at = __umul24(sy, uint32_t(a.w)) + sx;
      const uint32_t g = guide_word<FMT>(a.tgt_guide, at);
      const uint32_t u = glb(lut_of(a, at))[lut_bin<FMT>(g, a.lut_shift, a.lut_bits)];
      rec.x = pack_xy(4 * sx, 4 * sy);
      rec.y = pack_off(int32_t(u & 0xFFFFu) - int32_t(sx), int32_t(u >> 16) - int32_t(sy));
    }
  }
  return rec;
}

// The table of a pixel's own lookup: the unconstrained one, or with the
// segmentation guide the table of its label lt (past the last: the last).
template <bool SEG>
__device__ inline const uint32_t *own_table(const FrameArgs &a, uint32_t lt) {
  return SEG ? a.label_luts + (size_t(min(lt, uint32_t(a.nlabels - 1))) << a.lut_log2) : a.lut;
}

// Record idx of the padded seed table (read by the per-pixel level loop of
// hierarchies finer than 8 pixels; the block level loop makes its own).
template <int FMT>
__device__ inline void seeds_body(const FrameArgs &a, uint32_t idx) {
  const Levels &lv = a.lv;
  if (idx >= uint32_t(lv.poffset[lv.count])) return;
  int32_t i = 0;
  while (idx >= uint32_t(lv.poffset[i + 1])) ++i;
  const uint32_t local = idx - uint32_t(lv.poffset[i]), pc = uint32_t(lv.cells_x[i] + 2);
  seed_table(a)[idx] = seed_record<FMT>(a, lv.log2_spacing[i], lv.cells_x[i], lv.cells_y[i],
                                        lv.offset[i], a.jhash[i], int32_t(local % pc) - 1,
                                        int32_t(local / pc) - 1);
}

template <int FMT>
__global__ void __launch_bounds__(256) k_seeds(FrameArgs a) {
  seeds_body<FMT>(a, blockIdx.x * blockDim.x + threadIdx.x);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Records staged per wave: level i's nine at [kRecStride * i, + 9) of each
// block's record array (its 3 x 3 neighbourhood, x outer, y inner).
constexpr int32_t kRecStride = 12;
constexpr int32_t kWaveRecs = SB_MAX_LEVELS * kRecStride;
// Union grid of a multi-block wave: per level the 4 x 4 cells around the
// wave's region (16 slots, row-major), positions then offsets.
constexpr int32_t kUnion = 16;
constexpr int32_t kUnionWords = 2 * kUnion * SB_MAX_LEVELS;
// LDS words per wave of the block level loop for B blocks.
__host__ __device__ constexpr int32_t wave_recs_words(int32_t b) {
  return 2 * b * kWaveRecs + (b > 1 ? kUnionWords : 0);
}

// N levels i0 .. i0+N-1 of the block level loop for the lane's B pixels
// (pixel b in block b, whose records start at lpos + b * kWaveRecs): NearestSeed
// over each level's nine staged records, then all N * B source-guide gathers
// in flight together, then the tests in level order.  Straight-line code
// (levels past L rescan level L-1 and are never taken), so the gathers issue
// back to back.
template <int FMT, int N, int B, bool SEG>
__device__ __forceinline__ void level_group(const FrameArgs &a, const uint32_t *lpos,
                                            const uint32_t *loff, int32_t i0, const int32_t *x,
                                            const int32_t *y, const short2_t *p4,
                                            const uint32_t *gt, const uint32_t *lt,
                                            uint32_t *chunk, uint32_t *off, bool *done) {
  const int32_t L = a.lv.count;
  const uint32_t sw = uint32_t(a.sw), sh = uint32_t(a.sh);
  uint32_t g[B][N], wq[B][N], wo[B][N];
  bool ok[B][N];
#pragma unroll
  for (int32_t b = 0; b < B; ++b) {
#pragma unroll
    for (int32_t u = 0; u < N; ++u) {
      const int32_t li = min(i0 + u, L - 1);
      const uint32_t *P = lpos + b * kWaveRecs + kRecStride * li;
      const uint32_t *O = loff + b * kWaveRecs + kRecStride * li;
      const i32x4 q03 = *reinterpret_cast<const i32x4 *>(P);
      const i32x4 q47 = *reinterpret_cast<const i32x4 *>(P + 4);
      int32_t key = seed_key(uint32_t(q03.x), p4[b], 0);
      key = min(key, seed_key(uint32_t(q03.y), p4[b], 1));
      key = min(key, seed_key(uint32_t(q03.z), p4[b], 2));
      key = min(key, seed_key(uint32_t(q03.w), p4[b], 3));
      key = min(key, seed_key(uint32_t(q47.x), p4[b], 4));
      key = min(key, seed_key(uint32_t(q47.y), p4[b], 5));
      key = min(key, seed_key(uint32_t(q47.z), p4[b], 6));
      key = min(key, seed_key(uint32_t(q47.w), p4[b], 7));
      key = min(key, seed_key(P[8], p4[b], 8));
      wq[b][u] = P[key & 15];
      wo[b][u] = O[key & 15];
      const int32_t vx = x[b] + off_x(wo[b][u]), vy = y[b] + off_y(wo[b][u]);
      // non-short-circuit: keeps the group one straight-line block
      ok[b][u] = (i0 + u < L) & (key != INT32_MAX) & (uint32_t(vx) < sw) & (uint32_t(vy) < sh);
      g[b][u] = ok[b][u] ? __umul24(uint32_t(vy), sw) + uint32_t(vx) : 0u;
    }
  }
  uint32_t ls[B][N];
#pragma unroll
  for (int32_t b = 0; b < B; ++b) {
#pragma unroll
    for (int32_t u = 0; u < N; ++u) {
      // with the segmentation guide the source label is gathered beside the guide
      ls[b][u] = SEG ? uint32_t(glb(a.src_labels)[g[b][u]]) : 0u;
      g[b][u] = guide_raw<FMT>(a.src_guide, g[b][u]);
    }
  }
#pragma unroll
  for (int32_t b = 0; b < B; ++b) {
#pragma unroll
    for (int32_t u = 0; u < N; ++u) {
      const bool below =
          error_below<FMT>(gt[b], guide_unpack<FMT>(g[b][u]), a.threshold, a.wt02, a.wt1);
      const bool same = !SEG || ls[b][u] == lt[b];
      const bool take = (!done[b]) & ok[b][u] & below & same;
      chunk[b] = take ? chunk_code(i0 + u, wq[b][u]) : chunk[b];
      off[b] = take ? wo[b][u] : off[b];
      done[b] = done[b] || take;
    }
  }
}

// The level's first jitter entry (own records) or first seed-table record,
// and its hash state, for a lane whose level is `i`: a select per level, so
// nothing is indexed per lane in the kernel arguments.
__device__ __forceinline__ void level_select(const FrameArgs &a, uint32_t i, int32_t lo,
                                             int32_t hi, int32_t &f, uint32_t &hk) {
  const int32_t *first = a.own_seeds ? a.lv.offset : a.lv.poffset;
  f = first[lo];
  hk = a.jhash[lo];
#pragma unroll 1
  for (int32_t l = lo + 1; l < hi; ++l) {
    f = i >= uint32_t(l) ? first[l] : f;
    hk = i >= uint32_t(l) ? a.jhash[l] : hk;
  }
}

// The record of cell (cx, cy) of a level with log2 spacing ls: made from the
// jitter, the target guide and the table (own records), or read from the
// padded seed table (first record f of the level).
template <int FMT>
__device__ __forceinline__ u32x2 level_record(const FrameArgs &a, int32_t ls, int32_t f,
                                              uint32_t hk, int32_t cx, int32_t cy) {
  const int32_t ncx = ((a.w - 1) >> ls) + 1, ncy = ((a.h - 1) >> ls) + 1;
  if (a.own_seeds) return seed_record<FMT>(a, ls, ncx, ncy, f, hk, cx, cy);
  return seed_table(a)[uint32_t(f + (cy + 1) * (ncx + 2) + cx + 1)];
}

// The level loop for a wave's region of BX x BY blocks of 8 x 8 pixels at
// (bx0, by0) whose pixels share one cell per block at every level (every
// spacing >= 8); lane l takes pixel (l & 7, l >> 3) of every block.  The
// wave stages each block's 9 L seed records in LDS: with one block, one
// lane per record (two when 9 L > 64); with several, the region's blocks
// draw on one union grid per level (the cells the region touches and a
// ring, at most 4 x 4), staged 16 lanes per level and then copied into each
// block's record array, so a record shared by the blocks is made once.
// The union pays where records are made in the kernel (jitter -> target
// guide -> table); records read from the seed table are read per block.
// Levels run in groups of G (level_group).  The target guide, the records
// and the pixels' own lookups (their fallback) are all requested up front,
// so the chain of dependent memory round trips is guide -> lookup and
// records -> source guide, side by side.
template <int FMT, int G, int BX, int BY, bool SEG>
__device__ inline void assign_block(const FrameArgs &a, int32_t bx0, int32_t by0, int32_t lane,
                                    uint32_t *lds) {
  constexpr int32_t B = BX * BY;
  uint32_t *lpos = lds, *loff = lds + B * kWaveRecs;
  const Levels &lv = a.lv;
  const int32_t L = lv.count;
  int32_t x[B], y[B];
  bool in[B];
  uint32_t pidx[B], gt[B], lt[B];
#pragma unroll
  for (int32_t b = 0; b < B; ++b) {
    x[b] = bx0 + 8 * (b % BX) + (lane & 7);
    y[b] = by0 + 8 * (b / BX) + (lane >> 3);
    in[b] = x[b] < a.w && y[b] < a.h;
    pidx[b] = in[b] ? __umul24(uint32_t(y[b]), uint32_t(a.w)) + uint32_t(x[b]) : 0u;
    gt[b] = guide_word<FMT>(a.tgt_guide, pidx[b]);
    lt[b] = SEG ? uint32_t(glb(a.tgt_labels)[pidx[b]]) : 0u;
  }
  // a lane's level geometry follows from the spacings h_i = h_0 / 2^i: log2
  // spacing ls0 - i and ceil(extent / h_i) cells per axis
  const int32_t ls0 = L > 0 ? lv.log2_spacing[0] : 0;
  if (B == 1 || !a.own_seeds) {
    // records read from the seed table (or a lone block's own records):
    // record j (level j / 9, neighbour j % 9) of block b for lanes j and
    // j + 64; a block wholly outside the frame stages the region's first
    // block's cells (its pixels are never used)
    u32x2 rec[B][2];
    int32_t slot[B][2];
#pragma unroll
    for (int32_t h = 0; h < 2; ++h) {
      const uint32_t j = uint32_t(lane + 64 * h);
      const uint32_t i = (j * 57u) >> 9;  // j / 9 for j < 128
      const uint32_t k = j - 9u * i;
      const uint32_t kx = (k * 11u) >> 5;  // k / 3 for k < 9: x outer, y inner
      const bool staged = (h == 0 || 9 * L > 64) && j < uint32_t(9 * L);
      const int32_t ls = ls0 - int32_t(min(i, uint32_t(max(L - 1, 0))));
      int32_t f = 0;
      uint32_t hk = 0;
      if (staged) level_select(a, i, 0, L, f, hk);
#pragma unroll
      for (int32_t b = 0; b < B; ++b) {
        const int32_t X0 = bx0 + (bx0 + 8 * (b % BX) < a.w ? 8 * (b % BX) : 0);
        const int32_t Y0 = by0 + (by0 + 8 * (b / BX) < a.h ? 8 * (b / BX) : 0);
        slot[b][h] = staged ? b * kWaveRecs + kRecStride * int32_t(i) + int32_t(k) : -1;
        rec[b][h] = u32x2{0, 0};
        if (staged)
          rec[b][h] = level_record<FMT>(a, ls, f, hk, (X0 >> ls) - 1 + int32_t(kx),
                                        (Y0 >> ls) - 1 + int32_t(k - 3u * kx));
      }
    }
#pragma unroll
    for (int32_t b = 0; b < B; ++b) {
#pragma unroll
      for (int32_t h = 0; h < 2; ++h) {
        if (slot[b][h] >= 0) {
          lpos[slot[b][h]] = rec[b][h].x;
          loff[slot[b][h]] = rec[b][h].y;
        }
      }
    }
  } else {
    // own records for several blocks: one union grid, each shared record made once
    uint32_t *upos = lds + 2 * B * kWaveRecs, *uoff = upos + kUnion * SB_MAX_LEVELS;
    // the region's last in-frame pixel
    const int32_t rx1 = min(bx0 + 8 * BX, a.w) - 1, ry1 = min(by0 + 8 * BY, a.h) - 1;
    // union cell t = (ux, uy) of level 4r + (lane >> 4), four levels per round
    for (int32_t r = 0; 4 * r < L; ++r) {
      const int32_t i = 4 * r + (lane >> 4), t = lane & 15, ux = t & 3, uy = t >> 2;
      const int32_t ls = ls0 - min(i, L - 1);
      const int32_t c0x = bx0 >> ls, c0y = by0 >> ls;
      if (i < L && ux <= (rx1 >> ls) - c0x + 2 && uy <= (ry1 >> ls) - c0y + 2) {
        int32_t f;
        uint32_t hk;
        level_select(a, uint32_t(i), 4 * r, min(4 * r + 4, L), f, hk);
        const u32x2 rec = level_record<FMT>(a, ls, f, hk, c0x - 1 + ux, c0y - 1 + uy);
        upos[kUnion * i + t] = rec.x;
        uoff[kUnion * i + t] = rec.y;
      }
    }
    wave_lds_sync();
    // each block's neighbourhood out of the union: record j = (level j / 9,
    // neighbour j % 9) of block b; a block wholly outside the frame copies
    // the region's first block's cells (its pixels are never used)
#pragma unroll
    for (int32_t b = 0; b < B; ++b) {
      const int32_t X0 = bx0 + (bx0 + 8 * (b % BX) < a.w ? 8 * (b % BX) : 0);
      const int32_t Y0 = by0 + (by0 + 8 * (b / BX) < a.h ? 8 * (b / BX) : 0);
#pragma unroll
      for (int32_t h = 0; h < 2; ++h) {
        if (h > 0 && 9 * L <= 64) continue;
        const uint32_t j = uint32_t(lane + 64 * h);
        if (j >= uint32_t(9 * L)) continue;
        const uint32_t i = (j * 57u) >> 9, k = j - 9u * i, kx = (k * 11u) >> 5;
        const int32_t ls = ls0 - int32_t(i);
        const int32_t u = kUnion * int32_t(i) + ((Y0 >> ls) - (by0 >> ls) + int32_t(k - 3u * kx)) * 4 +
                          (X0 >> ls) - (bx0 >> ls) + int32_t(kx);
        const int32_t s = b * kWaveRecs + kRecStride * int32_t(i) + int32_t(k);
        lpos[s] = upos[u];
        loff[s] = uoff[u];
      }
    }
  }
  wave_lds_sync();
  // the pixels' own lookups, used when no level accepts: requested up front
  // from a table that stays in cache (up to 2^18 entries, 1 MiB), else only
  // for the pixels that end up needing them (a large table is mostly cold,
  // and few pixels fall back)
  const bool eager = a.lut_log2 <= 18;
  uint32_t own[B], chunk[B], off[B];
  short2_t p4[B];
  bool done[B];
#pragma unroll
  for (int32_t b = 0; b < B; ++b) {
    own[b] = 0;
    if (eager) own[b] = glb(own_table<SEG>(a, lt[b]))[lut_bin<FMT>(gt[b], a.lut_shift, a.lut_bits)];
    p4[b] = __builtin_bit_cast(short2_t, pack_xy(uint32_t(4 * x[b]), uint32_t(4 * y[b])));
    chunk[b] = off[b] = 0;
    done[b] = !in[b];
  }
  // groups of G levels (one round trip of gathers each) until every pixel of
  // the blocks has a level or the levels run out
  for (int32_t i0 = 0; i0 < L; i0 += G) {
    bool all = true;
#pragma unroll
    for (int32_t b = 0; b < B; ++b) all = all && done[b];
    if (__all(all)) break;
    level_group<FMT, G, B, SEG>(a, lpos, loff, i0, x, y, p4, gt, lt, chunk, off, done);
  }
#pragma unroll
  for (int32_t b = 0; b < B; ++b) {
    if (!in[b]) continue;
    if (!done[b]) {  // no level accepted: the pixel's own lookup
      if (!eager) own[b] = glb(own_table<SEG>(a, lt[b]))[lut_bin<FMT>(gt[b], a.lut_shift, a.lut_bits)];
      chunk[b] = (uint32_t(L) << 26) | (uint32_t(y[b]) << 13) | uint32_t(x[b]);
      off[b] = pack_off(int32_t(own[b] & 0xFFFFu) - x[b], int32_t(own[b] >> 16) - y[b]);
    }
    glb(a.out_chunk)[pidx[b]] = chunk[b];
    glb(a.offsets)[pidx[b]] = vote_distance(a, off[b]);
    if (a.out_nnf)
      glb(a.out_nnf)[pidx[b]] =
          pack_xy(uint32_t(x[b] + off_x(off[b])), uint32_t(y[b] + off_y(off[b])));
  }
}

// The level loop for one pixel when cells are smaller than 8 x 8 blocks:
// each lane reads its own nine records per level.
template <int FMT, bool SEG>
__device__ inline void assign_pixel(const FrameArgs &a, int32_t x, int32_t y) {
  if (x >= a.w || y >= a.h) return;
  const Levels &lv = a.lv;
  const int32_t L = lv.count;
  const uint32_t pidx = __umul24(uint32_t(y), uint32_t(a.w)) + uint32_t(x);
  const uint32_t gt = guide_word<FMT>(a.tgt_guide, pidx);
  const short2_t p4 = __builtin_bit_cast(short2_t, pack_xy(uint32_t(4 * x), uint32_t(4 * y)));
  const uint32_t sw = uint32_t(a.sw), sh = uint32_t(a.sh);
  uint32_t chunk = 0, off = 0;
  bool done = false;
  for (int32_t i = 0; i < L && !done; ++i) {
    const int32_t ls = lv.log2_spacing[i], pc = lv.cells_x[i] + 2;
    const SB_GLOBAL u32x2 *top = seed_table(a) + lv.poffset[i] + (y >> ls) * pc + (x >> ls);
    int32_t key = INT32_MAX;
#pragma unroll
    for (int32_t k = 0; k < 9; ++k) key = min(key, seed_key(top[(k % 3) * pc + k / 3].x, p4, k));
    if (key == INT32_MAX) continue;
    const int32_t k = key & 15, kx = (k * 11) >> 5;
    const u32x2 w = top[(k - 3 * kx) * pc + kx];
    const int32_t vx = x + off_x(w.y), vy = y + off_y(w.y);
    if (uint32_t(vx) >= sw || uint32_t(vy) >= sh) continue;
    const uint32_t vidx = __umul24(uint32_t(vy), sw) + uint32_t(vx);
    if (SEG && glb(a.src_labels)[vidx] != glb(a.tgt_labels)[pidx]) continue;
    const uint32_t g = guide_word<FMT>(a.src_guide, vidx);
    if (error_below<FMT>(gt, g, a.threshold, a.wt02, a.wt1)) {
      chunk = chunk_code(i, w.x);
      off = w.y;
      done = true;
    }
  }
  if (!done) {
    const uint32_t u = glb(lut_of(a, pidx))[lut_bin<FMT>(gt, a.lut_shift, a.lut_bits)];
    chunk = (uint32_t(L) << 26) | (uint32_t(y) << 13) | uint32_t(x);
    off = pack_off(int32_t(u & 0xFFFFu) - x, int32_t(u >> 16) - y);
  }
  glb(a.out_chunk)[pidx] = chunk;
  glb(a.offsets)[pidx] = vote_distance(a, off);
  if (a.out_nnf) glb(a.out_nnf)[pidx] = pack_xy(uint32_t(x + off_x(off)), uint32_t(y + off_y(off)));
}

// Whether every level's cells hold whole 8 x 8 blocks.
__host__ __device__ inline bool uniform_cells(const Levels &lv) {
  return lv.count == 0 || lv.log2_spacing[lv.count - 1] >= 3;
}

// One (16 BX) x (16 BY) tile with BX BY = B: four regions of BX x BY blocks
// of 8 x 8 pixels, one per wave, on the uniform-cell path; otherwise B
// pixels per thread.  `lds` holds 4 waves' records (wave_recs_words(B) each).
template <int FMT, int G, int B, bool SEG>
__device__ inline void assign_tile(const FrameArgs &a, uint32_t tile, uint32_t tid,
                                   uint32_t *lds) {
  constexpr int32_t BX = B >= 2 ? 2 : 1, BY = B / BX;
  static_assert(BX * BY == B && (B == 1 || B == 2 || B == 4), "regions of 1, 2 or 4 blocks");
  const uint32_t tw = 16 * BX, th = 16 * BY;
  const uint32_t tiles_x = (uint32_t(a.w) + tw - 1) / tw;
  const int32_t tx0 = int32_t((tile % tiles_x) * tw), ty0 = int32_t((tile / tiles_x) * th);
  if (uniform_cells(a.lv)) {
    const int32_t wave = __builtin_amdgcn_readfirstlane(int32_t(tid >> 6));
    const int32_t bx0 = tx0 + (wave & 1) * 8 * BX, by0 = ty0 + (wave >> 1) * 8 * BY;
    // a region wholly outside the frame has no cells in the table
    if (bx0 >= a.w || by0 >= a.h) return;
    assign_block<FMT, G, BX, BY, SEG>(a, bx0, by0, int32_t(tid & 63),
                                      lds + wave * wave_recs_words(B));
  } else {
#pragma unroll
    for (int32_t b = 0; b < B; ++b)
      assign_pixel<FMT, SEG>(a, tx0 + int32_t(tid & 15) + 16 * (b % BX),
                             ty0 + int32_t(tid >> 4) + 16 * (b / BX));
  }
}

template <int FMT, int G, int B, bool SEG>
__global__ void __launch_bounds__(256) k_assign(FrameArgs a) {
  __shared__ __attribute__((aligned(16))) uint32_t lds[4 * wave_recs_words(B)];
  assign_tile<FMT, G, B, SEG>(a, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x, lds);
}

// Exact floor(n / k) for n < 2^16 and 1 <= k <= 225, given rk within one ulp
// of 1/k (v_rcp_f32): (n + 1/2) * rk lies within 0.5/k of (n + 1/2)/k, whose
// fractional part keeps at least 0.5/k from the next integer, so truncation
// gives floor(n / k).  (Checked exhaustively over every such n and k and the
// three floats nearest 1/k.)  Written as fma(n, rk, hk) with hk = rk / 2:
// the same exact product rounded once.
__device__ inline uint32_t div_small(uint32_t n, float rk, float hk) {
  return uint32_t(__builtin_fmaf(float(n), rk, hk));
}

// LDS row length and rows of a voting tile of TW x TH pixels and radius R
// (rows padded to a multiple of 4 cells so each lane's cells start aligned).
__host__ __device__ constexpr int32_t blend_lw(int32_t tw, int32_t r) { return (tw + 2 * r + 3) & ~3; }
__host__ __device__ constexpr int32_t blend_lh(int32_t th, int32_t r) { return th + 2 * r; }
// LDS words of a voting tile: the rows and one unused row in front, so the
// row above any tile row is an address inside the array.
__host__ __device__ constexpr int32_t blend_words(int32_t tw, int32_t th, int32_t r) {
  return blend_lw(tw, r) * (blend_lh(th, r) + 1);
}

// Load n = 1..4 consecutive texels at byte offset `at` of the exemplar.
template <int N>
__device__ __forceinline__ void load_texels(const SB_GLOBAL unsigned char *ex, uint32_t at,
                                            uint32_t *t) {
  const SB_GLOBAL unsigned char *p = ex + uint64_t(at);
  if (N == 4) {
    const u32x4a4 v = *reinterpret_cast<const SB_GLOBAL u32x4a4 *>(p);
    t[0] = v.x, t[1] = v.y, t[2] = v.z, t[3] = v.w;
  } else if (N == 3) {
    const u32x3a4 v = *reinterpret_cast<const SB_GLOBAL u32x3a4 *>(p);
    t[0] = v.x, t[1] = v.y, t[2] = v.z;
  } else if (N == 2) {
    const u32x2a4 v = *reinterpret_cast<const SB_GLOBAL u32x2a4 *>(p);
    t[0] = v.x, t[1] = v.y;
  } else {
    t[0] = *reinterpret_cast<const SB_GLOBAL uint32_t *>(p);
  }
}

// Per-lane select r = (lane's bit of mask) ? a : b as one v_cndmask, and
// the lane mask of a == b as one v_cmp: written out so the compiler neither
// branches around copies nor turns a mask into a 0/1 value and back.
__device__ __forceinline__ uint32_t lane_select(uint64_t mask, uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
  return r;
}
__device__ __forceinline__ uint64_t lane_equal(int32_t a, int32_t b) {
  uint64_t m;
  asm("v_cmp_eq_u32_e64 %0, %1, %2" : "=s"(m) : "v"(a), "v"(b));
  return m;
}

// Texels of the lane's PPT pixels for one window cell, indexed by pixel J
// (only J0(c)..J1(c) are meaningful).
template <int PPT>
struct TexelsN {
  uint32_t t[PPT];
};

// Cell column C (0 .. 2R+PPT-1) of one window row votes for the lane's
// pixels J = C - 2R .. C (clipped to 0..PPT-1).  Every vote of a cell with
// offset o for pixel p is the texel at p + o, so a cell with the same offset
// as the cell above it (same column, previous row) or, from column PPT on, as
// its left neighbour needs texels the lane already holds; only lanes whose
// cell starts a new offset issue the gather, one vector load of the pixels'
// adjacent texels.  Two phases per row: first every cell's gather, landing
// over the upper cell's texels (so no gather waits for another), then in
// column order the left-neighbour reuse (one select) and the sums.
template <int R, int PPT, int C>
__device__ __forceinline__ void vote_gather(const SB_GLOBAL unsigned char *ex, uint32_t pbase,
                                            const int32_t *cells, const int32_t *up_cells,
                                            bool has_up, TexelsN<PPT> *row,
                                            const TexelsN<PPT> *up_row) {
  if constexpr (C < 2 * R + PPT) {
    constexpr int J0 = C - 2 * R > 0 ? C - 2 * R : 0;
    constexpr int J1 = C < PPT - 1 ? C : PPT - 1;
    constexpr int N = J1 - J0 + 1;
    const int32_t lin = cells[C];
    const bool up = has_up && lin == up_cells[C];
    const bool left = C >= PPT && lin == cells[C > 0 ? C - 1 : 0];
    uint32_t t[PPT];
#pragma unroll
    for (int m = 0; m < N; ++m) t[m] = up_row[C].t[J0 + m];
    if (!up && !left) load_texels<N>(ex, pbase + 4u * J0 + uint32_t(lin), t);
#pragma unroll
    for (int m = 0; m < N; ++m) row[C].t[J0 + m] = t[m];
    vote_gather<R, PPT, C + 1>(ex, pbase, cells, up_cells, has_up, row, up_row);
  }
}

template <int R, int PPT, int C>
__device__ __forceinline__ void vote_sum(const int32_t *cells, TexelsN<PPT> *row, uint32_t *S,
                                         uint32_t *RB) {
  if constexpr (C < 2 * R + PPT) {
    constexpr int J0 = C - 2 * R > 0 ? C - 2 * R : 0;
    constexpr int J1 = C < PPT - 1 ? C : PPT - 1;
    constexpr int N = J1 - J0 + 1;
    if constexpr (C >= PPT) {
      const uint64_t left = lane_equal(cells[C], cells[C - 1]);
#pragma unroll
      for (int m = 0; m < N; ++m)
        row[C].t[J0 + m] = lane_select(left, row[C - 1].t[J0 + m], row[C].t[J0 + m]);
    }
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const uint32_t v = row[C].t[J0 + m];
      S[J0 + m] += v;
      RB[J0 + m] += v & 0x00FF00FFu;
    }
    vote_sum<R, PPT, C + 1>(cells, row, S, RB);
  }
}

template <int R, int PPT, int C>
__device__ __forceinline__ void vote_row(const SB_GLOBAL unsigned char *ex, uint32_t pbase,
                                         const int32_t *cells, const int32_t *up_cells,
                                         bool has_up, TexelsN<PPT> *row,
                                         const TexelsN<PPT> *up_row, uint32_t *S, uint32_t *RB) {
  vote_gather<R, PPT, C>(ex, pbase, cells, up_cells, has_up, row, up_row);
  vote_sum<R, PPT, C>(cells, row, S, RB);
}

// Store the RGB of a lane's PPT pixels (c[j] = R | G << 8 | B << 16) at (x, y):
// one 12-byte (PPT 4) or 6-byte (PPT 2) write when the row holds them all
// and the address allows, else byte by byte.
template <int PPT>
__device__ __forceinline__ void store_rgb(const FrameArgs &a, int32_t x, int32_t y,
                                          const uint32_t *c) {
  const uint32_t at = 3u * (__umul24(uint32_t(y), uint32_t(a.w)) + uint32_t(x));  // < 2^28
  SB_GLOBAL uint8_t *o = glb(a.out_rgb) + at;
  const uint32_t oa = uint32_t(reinterpret_cast<uintptr_t>(a.out_rgb)) + at;  // alignment only
  if (PPT == 4 && x + 4 <= a.w && (oa & 3) == 0) {
    u32x3a4 v;
    v.x = (c[0] & 0xFFFFFFu) | (c[1 % PPT] << 24);
    v.y = ((c[1 % PPT] >> 8) & 0xFFFFu) | (c[2 % PPT] << 16);
    v.z = ((c[2 % PPT] >> 16) & 0xFFu) | (c[3 % PPT] << 8);
    *reinterpret_cast<SB_GLOBAL u32x3a4 *>(o) = v;
  } else if (PPT == 2 && x + 2 <= a.w && (oa & 1) == 0) {
    SB_GLOBAL uint16_t *o16 = reinterpret_cast<SB_GLOBAL uint16_t *>(o);
    o16[0] = uint16_t(c[0]);
    o16[1] = uint16_t(((c[0] >> 16) & 0xFFu) | (c[1 % PPT] << 8));
    o16[2] = uint16_t(c[1 % PPT] >> 8);
  } else {
#pragma unroll
    for (int32_t j = 0; j < PPT; ++j) {
      if (x + j < a.w) {
        o[3 * j] = uint8_t(c[j]);
        o[3 * j + 1] = uint8_t(c[j] >> 8);
        o[3 * j + 2] = uint8_t(c[j] >> 16);
      }
    }
  }
}

// The full vote of one lane's PPT pixels (group gx of tile row ly): every
// window row's gathers and sums, then the average.  `lin` as in blend_tile.
template <int R, int PPT, int TH>
__device__ __forceinline__ void vote_group(const FrameArgs &a, int32_t X0, int32_t Y0, int32_t gx,
                                           int32_t ly, const int32_t *lin) {
  constexpr int32_t TW = 16 * PPT;
  constexpr int32_t LW = blend_lw(TW, R);
  const int32_t P = a.ex_stride;
  const int32_t x = X0 + PPT * gx, y = Y0 + ly;
  const uint32_t pbase =
      4u * (__umul24(uint32_t(y + kExMargin), uint32_t(P)) + uint32_t(x + kExMargin));
  const SB_GLOBAL unsigned char *ex = glb(reinterpret_cast<const unsigned char *>(a.src_rgba));
  uint32_t S[PPT] = {}, RB[PPT] = {};
  // the lane's cells of a window row: 2R + PPT, read as aligned PPT-vectors
  // and, for the last 2R mod PPT cells (0 or 2), one aligned pair (reading
  // only the cells used keeps the kernel within 64 VGPRs, 8 waves per SIMD)
  constexpr int32_t NCL = 2 * R + PPT, NQ = NCL / PPT, NTAIL = NCL % PPT;
  static_assert(NTAIL == 0 || NTAIL == 2, "cells per row are a multiple of 2");
  typedef int32_t lvec __attribute__((ext_vector_type(PPT)));
  typedef int32_t lvec2 __attribute__((ext_vector_type(2)));
  // the previous row's texels (unused in the first row, which has no row
  // above: every lane there gathers or takes its left neighbour's texels);
  // the previous row's cells are read again from LDS rather than carried
  TexelsN<PPT> up_row[NCL];
#pragma unroll
  for (int32_t c = 0; c < NCL; ++c) up_row[c] = TexelsN<PPT>{};
  // (the tile starts one row into `lin`, so row dy - 1 is in the array for dy = 0 too)
  const int32_t *lane_above = lin + ly * LW + PPT * gx;
#pragma unroll 1
  for (int32_t dy = 0; dy < 2 * R + 1; ++dy) {
    const lvec *qu = reinterpret_cast<const lvec *>(lane_above + dy * LW);
    const lvec *q = reinterpret_cast<const lvec *>(lane_above + (dy + 1) * LW);
    int32_t cells[NCL], up_cells[NCL];
#pragma unroll
    for (int32_t i = 0; i < NQ; ++i) {
      const lvec v = q[i], u = qu[i];
#pragma unroll
      for (int32_t j = 0; j < PPT; ++j) cells[PPT * i + j] = v[j], up_cells[PPT * i + j] = u[j];
    }
    if constexpr (NTAIL == 2) {
      const lvec2 v = *reinterpret_cast<const lvec2 *>(q + NQ);
      const lvec2 u = *reinterpret_cast<const lvec2 *>(qu + NQ);
      cells[NCL - 2] = v.x, cells[NCL - 1] = v.y;
      up_cells[NCL - 2] = u.x, up_cells[NCL - 1] = u.y;
    }
    TexelsN<PPT> row[NCL];
    vote_row<R, PPT, 0>(ex, pbase, cells, up_cells, dy > 0, row, up_row, S, RB);
#pragma unroll
    for (int32_t c = 0; c < NCL; ++c) up_row[c] = row[c];
  }
  if (y >= a.h || x >= a.w) return;
  uint32_t c[PPT];
#pragma unroll
  for (int32_t j = 0; j < PPT; ++j) {
    // S = sum R + 2^8 sum G + 2^16 sum B + 2^24 k and RB = sum R + 2^16 sum B
    // (mod 2^32); every channel sum is < 2^16 and k <= 225
    const uint32_t gk = S[j] - RB[j];
    const uint32_t k = gk >> 24, hk = k >> 1;
    const float rk = __builtin_amdgcn_rcpf(float(k)), rh = 0.5f * rk;
    c[j] = div_small((RB[j] & 0xFFFFu) + hk, rk, rh) |
           (div_small(((gk >> 8) & 0xFFFFu) + hk, rk, rh) << 8) |
           (div_small((RB[j] >> 16) + hk, rk, rh) << 16);
  }
  store_rgb<PPT>(a, x, y, c);
}

// Extra LDS words of a voting tile with SPLIT: per window row of the tile
// one flag byte per lane group (16 per row), the list of groups that need
// the full vote (one word per thread) and its length.
__host__ __device__ constexpr int32_t blend_split_words(int32_t th, int32_t r) {
  return 4 * blend_lh(th, r) + 16 * th + 4;
}

// One (16 PPT) x TH pixel voting tile with 16 TH threads: thread t votes for
// PPT horizontally adjacent pixels.  `lin` is LDS for blend_words words (plus
// blend_split_words with SPLIT): an unused row, then blend_lw x blend_lh
// cells; cell n holds 4 * (oy * P + ox) for its offset o = NNF[n] - n and the
// padded exemplar's row length P: a vote of n for pixel p is the texel at
// p's own padded position plus that many bytes.  Cells outside the target
// hold the distance to the exemplar's zero rows instead, so their votes read
// zeros, which count for nothing (alpha 0).  Pixel p's average is
// (sum + floor(k/2)) / k per channel over its k in-source votes, the vote
// rule at the end of Sec. 3.2.
//
// With SPLIT, groups whose whole window (2R + 1 rows of 2R + PPT cells)
// holds one offset -- every vote then lands on the same in-source texel, so
// the average is that texel exactly, which is the paper's remark that
// voting only blends at chunk boundaries -- copy their texels with one
// gather; the others are listed in LDS and voted by the tile's threads in
// list order, so the full votes run in packed waves.  Uniformity is tested
// separably: per window row, whether the group's cells are all equal (min =
// max) and whether its first cell equals the one below, as flag bytes.
// Ends with all threads past their last LDS read (callers that reuse `lin`
// synchronise before refilling it).
template <int R, int PPT, int TH, bool SPLIT>
__device__ inline void blend_tile(const FrameArgs &a, uint32_t t_index, uint32_t tid,
                                  int32_t *lin) {
  constexpr int32_t TW = 16 * PPT, NT = 16 * TH;
  constexpr int32_t LW = blend_lw(TW, R), LH = blend_lh(TH, R);
  static_assert(TW <= kBlendMaxTW && TH <= kBlendMaxTH, "tile exceeds the exemplar zero rows");
  const uint32_t tiles_x = (uint32_t(a.w) + TW - 1) / TW;
  const int32_t X0 = int32_t(t_index % tiles_x) * TW;
  const int32_t Y0 = int32_t(t_index / tiles_x) * TH;
  const int32_t P = a.ex_stride;
  const int32_t zero_rel = 4 * (int32_t(a.ex_zero) - ((Y0 + kExMargin) * P + (X0 + kExMargin)));
  // the tile's cells in runs of 4 along a row (LW is a multiple of 4), one
  // dword-aligned 16-byte load per run and every thread's runs requested
  // together; a run reaching past the target (border tiles only) reads its
  // cells one by one, and cells outside the target take zero_rel
  constexpr int32_t QW = LW / 4, NCH = QW * LH, CPER = (NCH + NT - 1) / NT;
  static_assert(LW % 4 == 0, "tile rows are whole runs of 4 cells");
  u32x4a4 run[CPER];
  uint32_t inside[CPER];  // bit m: cell m of the run lies in the target
#pragma unroll
  for (int32_t n = 0; n < CPER; ++n) {
    const int32_t ch = int32_t(tid) + n * NT;
    const int32_t tx = X0 - R + 4 * (ch % QW), ty = Y0 - R + ch / QW;
    const bool row_in = ch < NCH && ty >= 0 && ty < a.h;
    const SB_GLOBAL uint32_t *src =
        glb(a.offsets) + (row_in ? __umul24(uint32_t(ty), uint32_t(a.w)) : 0u);
    if (row_in && tx >= 0 && tx + 4 <= a.w) {
      run[n] = *reinterpret_cast<const SB_GLOBAL u32x4a4 *>(src + tx);
      inside[n] = 15u;
    } else {
      inside[n] = 0u;
#pragma unroll
      for (int32_t m = 0; m < 4; ++m) {
        const bool in = row_in && tx + m >= 0 && tx + m < a.w;
        run[n][m] = src[in ? uint32_t(tx + m) : 0u];
        inside[n] |= uint32_t(in) << m;
      }
    }
  }
#pragma unroll
  for (int32_t n = 0; n < CPER; ++n) {
    const int32_t ch = int32_t(tid) + n * NT;
    if (n + 1 < CPER || ch < NCH) {
      i32x4 v;
#pragma unroll
      for (int32_t m = 0; m < 4; ++m)
        v[m] = (inside[n] >> m) & 1u ? int32_t(run[n][m]) : zero_rel;
      *reinterpret_cast<i32x4 *>(lin + LW + 4 * ch) = v;
    }
  }
  constexpr bool split = SPLIT && R > 0;
  uint8_t *flags = reinterpret_cast<uint8_t *>(lin + blend_words(TW, TH, R));
  uint32_t *list = reinterpret_cast<uint32_t *>(flags) + 4 * LH;
  uint32_t *count = list + NT;
  if (split && tid == 0) *count = 0u;
  __syncthreads();
  const int32_t gx = int32_t(tid & 15), ly = int32_t(tid >> 4);
  if constexpr (!split) {
    vote_group<R, PPT, TH>(a, X0, Y0, gx, ly, lin);
    return;
  } else {
    constexpr int32_t NCL = 2 * R + PPT;
    // flag byte of (window row yy, group gx): bit 0 the group's NCL cells in
    // that row are equal, bit 1 its first cell equals the one below
#pragma unroll
    for (int32_t h = 0; h * TH < LH; ++h) {
      const int32_t yy = ly + TH * h;
      if (yy < LH) {
        const int32_t *c = lin + LW + yy * LW + PPT * gx;
        int32_t mn = c[0], mx = c[0];
#pragma unroll
        for (int32_t i = 1; i < NCL; ++i) mn = min(mn, c[i]), mx = max(mx, c[i]);
        const bool down = yy + 1 < LH && c[LW] == c[0];
        flags[yy * 16 + gx] = uint8_t((mn == mx ? 1u : 0u) | (down ? 2u : 0u));
      }
    }
    __syncthreads();
    uint32_t f = 3u;
#pragma unroll
    for (int32_t dy = 0; dy < 2 * R; ++dy) f &= flags[(ly + dy) * 16 + gx];
    const bool uni = f == 3u && (flags[(ly + 2 * R) * 16 + gx] & 1u) != 0u;
    const int32_t x = X0 + PPT * gx, y = Y0 + ly;
    const bool live = x < a.w && y < a.h;
    if (uni && live) {
      // one offset over the whole window: every pixel's average is its texel
      const uint32_t pbase =
          4u * (__umul24(uint32_t(y + kExMargin), uint32_t(P)) + uint32_t(x + kExMargin));
      const SB_GLOBAL unsigned char *ex =
          glb(reinterpret_cast<const unsigned char *>(a.src_rgba));
      uint32_t c[PPT];
      load_texels<PPT>(ex, pbase + uint32_t(lin[LW + (ly + R) * LW + PPT * gx + R]), c);
      store_rgb<PPT>(a, x, y, c);
    }
    const bool need = live && !uni;
    const uint64_t bal = __builtin_amdgcn_ballot_w64(need);
    uint32_t base = 0;
    if ((tid & 63) == 0 && bal != 0)
      base = atomicAdd(count, uint32_t(__builtin_popcountll(bal)));
    base = __builtin_amdgcn_readfirstlane(base);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
    if (need) list[base + below] = tid;
    __syncthreads();
    const uint32_t n = *count;
    for (uint32_t e = tid; e < n; e += NT) {
      const uint32_t t = list[e];
      vote_group<R, PPT, TH>(a, X0, Y0, int32_t(t & 15), int32_t(t >> 4), lin);
    }
  }
}

// Radius dispatch over [RLO, RHI] for the batch kernels.
template <int PPT, int TH, int RLO, int RHI, bool SPLIT>
__device__ inline void blend_tile_r(const FrameArgs &a, uint32_t t_index, uint32_t tid,
                                    int32_t *lin) {
  if constexpr (RLO <= RHI) {
    if (a.radius == RLO) blend_tile<RLO, PPT, TH, SPLIT>(a, t_index, tid, lin);
    else blend_tile_r<PPT, TH, RLO + 1, RHI, SPLIT>(a, t_index, tid, lin);
  }
}

// LDS words of a voting tile of radius R.
__host__ __device__ constexpr int32_t blend_tile_words(int32_t ppt, int32_t th, int32_t r,
                                                       bool split) {
  return blend_words(16 * ppt, th, r) + (split ? blend_split_words(th, r) : 0);
}

template <int R, int PPT, int TH, bool SPLIT>
__global__ void __launch_bounds__(16 * TH) k_blend(FrameArgs a) {
  __shared__ __attribute__((aligned(16))) int32_t lin[blend_tile_words(PPT, TH, R, SPLIT)];
  blend_tile<R, PPT, TH, SPLIT>(a, xcd_tile(blockIdx.x, gridDim.x), threadIdx.x, lin);
}

// ------------------------------------------------------------------ batches
//
// A batch runs the same passes over many frames: each kernel is persistent
// (a fixed grid striding over the concatenated tiles of all frames) and reads
// the frames' arguments from a descriptor block in device memory, so one
// captured graph serves any mix of sizes and formats.  A block copies the
// arguments of the frame it is working on into LDS.  The vote pass runs as
// two kernels, radius 0..3 and 4..7, each over its own frames' tiles, so the
// common small radii do not pay the register budget of the large ones.

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

// The arguments of frame f of a batch descriptor, read in place: the
// descriptor is read-only for the whole launch and the frame index is
// wave-uniform, so the compiler loads the fields the kernels use through the
// scalar cache, as it does a single frame's kernel arguments.
__device__ __forceinline__ const FrameArgs &batch_frame(const unsigned char *__restrict__ desc,
                                                        uint32_t f) {
  f = __builtin_amdgcn_readfirstlane(f);
  return *reinterpret_cast<const FrameArgs *>(desc + batch_frames_offset() +
                                              size_t(f) * sizeof(FrameArgs));
}

// Batch pass KIND over the descriptor's frames; BODY(frame args, local tile, work).
template <int KIND, int NT, int WORDS, class Body>
__device__ __forceinline__ void batch_loop(const unsigned char *__restrict__ desc, Body body) {
  __shared__ __attribute__((aligned(16))) uint32_t work[WORDS];
  __shared__ uint32_t pre[kMaxBatchFrames + 1];
  const BatchHeader *hd = reinterpret_cast<const BatchHeader *>(desc);
  const uint32_t n = hd->nframes;
  const uint32_t *gpre = reinterpret_cast<const uint32_t *>(desc + batch_prefix_offset(KIND));
  for (uint32_t i = threadIdx.x; i <= n; i += NT) pre[i] = gpre[i];
  __syncthreads();
  const uint32_t total = pre[n];
  if (gridDim.x == total) {
    // an exact grid (direct launches): one tile per workgroup, dealt to the
    // XCDs by contiguous bands like a single frame's, and short-lived
    // workgroups that other streams' kernels can interleave with
    const uint32_t t = xcd_tile(blockIdx.x, total);
    const uint32_t f = frame_of(pre, n, t);
    body(batch_frame(desc, f), t - pre[f], work);
    return;
  }
  // persistent grid: XCD-aware order: runs of kXcdRun consecutive tiles go to
  // the XCDs in turn, and the workgroups on XCD x (those with blockIdx mod 8
  // = x) stride through the runs of x, so an XCD's L2 serves neighbouring
  // tiles while the runs keep the XCDs' shares balanced across the batch (a
  // grid of fewer than 8 workgroups strides plainly: some XCDs would own
  // runs but have no workgroup)
  constexpr uint32_t kXcdRun = 32;
  const bool xcd = gridDim.x >= 8u;
  const uint32_t x = xcd ? blockIdx.x & 7u : 0u, local = xcd ? blockIdx.x >> 3 : blockIdx.x;
  const uint32_t per = xcd ? (gridDim.x >> 3) + (x < (gridDim.x & 7u) ? 1u : 0u) : gridDim.x;
  for (uint32_t s = local;; s += per) {
    const uint32_t t = xcd ? ((s / kXcdRun) * 8u + x) * kXcdRun + s % kXcdRun : s;
    if (!xcd && t >= total) break;
    if (t >= total) {
      // runs of this XCD beyond the end: the next may still hold tiles only
      // if this one was the partly filled last run
      if ((s / kXcdRun) * 8u * kXcdRun >= total) break;
      continue;
    }
    const uint32_t f = frame_of(pre, n, t);
    body(batch_frame(desc, f), t - pre[f], work);
    __syncthreads();  // the next tile restages its LDS
  }
}

__global__ void __launch_bounds__(256) k_batch_seeds(const unsigned char *__restrict__ desc) {
  batch_loop<0, 256, 1>(desc, [](const FrameArgs &fa, uint32_t local, uint32_t *)
                                  __attribute__((always_inline)) {
    const uint32_t idx = local * 256 + threadIdx.x;
    if (fa.fmt == SB_GUIDE_U8X2) seeds_body<SB_GUIDE_U8X2>(fa, idx);
    else if (fa.fmt == SB_GUIDE_U8X3) seeds_body<SB_GUIDE_U8X3>(fa, idx);
    else seeds_body<SB_GUIDE_U16X2>(fa, idx);
  });
}

template <int G, int B>
__global__ void __launch_bounds__(256) k_batch_assign(const unsigned char *__restrict__ desc) {
  batch_loop<1, 256, 4 * wave_recs_words(B)>(desc, [](const FrameArgs &fa, uint32_t local,
                                                     uint32_t *w) __attribute__((always_inline)) {
    const bool seg = fa.tgt_labels != nullptr;
    if (fa.fmt == SB_GUIDE_U8X2) {
      if (seg) assign_tile<SB_GUIDE_U8X2, G, B, true>(fa, local, threadIdx.x, w);
      else assign_tile<SB_GUIDE_U8X2, G, B, false>(fa, local, threadIdx.x, w);
    } else if (fa.fmt == SB_GUIDE_U8X3) {
      if (seg) assign_tile<SB_GUIDE_U8X3, G, B, true>(fa, local, threadIdx.x, w);
      else assign_tile<SB_GUIDE_U8X3, G, B, false>(fa, local, threadIdx.x, w);
    } else {
      if (seg) assign_tile<SB_GUIDE_U16X2, G, B, true>(fa, local, threadIdx.x, w);
      else assign_tile<SB_GUIDE_U16X2, G, B, false>(fa, local, threadIdx.x, w);
    }
  });
}

template <int PPT, int TH, int RLO, int RHI, bool SPLIT>
__global__ void __launch_bounds__(16 * TH) k_batch_blend(const unsigned char *__restrict__ desc) {
  constexpr int WORDS = blend_tile_words(PPT, TH, RHI, SPLIT);
  batch_loop<RLO == 0 ? 2 : 3, 16 * TH, WORDS>(desc, [](const FrameArgs &fa, uint32_t local,
                                                        uint32_t *w)
                                                         __attribute__((always_inline)) {
    blend_tile_r<PPT, TH, RLO, RHI, SPLIT>(fa, local, threadIdx.x, reinterpret_cast<int32_t *>(w));
  });
}

unsigned blocks_for(uint64_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

template <int FMT, int G, int B>
void launch_assign(const FrameArgs &a, uint32_t blocks, hipStream_t stream) {
  if (a.tgt_labels) k_assign<FMT, G, B, true><<<blocks, 256, 0, stream>>>(a);
  else k_assign<FMT, G, B, false><<<blocks, 256, 0, stream>>>(a);
}

template <int FMT>
void launch_assign_any(const FrameArgs &a, const Tune &t, uint32_t blocks, hipStream_t stream) {
  if (t.group == 4) {
    if (t.apx == 4) launch_assign<FMT, 4, 4>(a, blocks, stream);
    else if (t.apx == 2) launch_assign<FMT, 4, 2>(a, blocks, stream);
    else launch_assign<FMT, 4, 1>(a, blocks, stream);
  } else {
    if (t.apx == 4) launch_assign<FMT, 2, 4>(a, blocks, stream);
    else if (t.apx == 2) launch_assign<FMT, 2, 2>(a, blocks, stream);
    else launch_assign<FMT, 2, 1>(a, blocks, stream);
  }
}

template <int PPT, int TH, bool SPLIT>
void launch_blend(const FrameArgs &a, uint32_t blocks, hipStream_t stream) {
  switch (a.radius) {
    case 0: k_blend<0, PPT, TH, SPLIT><<<blocks, 16 * TH, 0, stream>>>(a); break;
    case 1: k_blend<1, PPT, TH, SPLIT><<<blocks, 16 * TH, 0, stream>>>(a); break;
    case 2: k_blend<2, PPT, TH, SPLIT><<<blocks, 16 * TH, 0, stream>>>(a); break;
    case 3: k_blend<3, PPT, TH, SPLIT><<<blocks, 16 * TH, 0, stream>>>(a); break;
    case 4: k_blend<4, PPT, TH, SPLIT><<<blocks, 16 * TH, 0, stream>>>(a); break;
    case 5: k_blend<5, PPT, TH, SPLIT><<<blocks, 16 * TH, 0, stream>>>(a); break;
    case 6: k_blend<6, PPT, TH, SPLIT><<<blocks, 16 * TH, 0, stream>>>(a); break;
    default: k_blend<7, PPT, TH, SPLIT><<<blocks, 16 * TH, 0, stream>>>(a); break;
  }
}

template <int PPT, int TH>
void launch_blend_any(const FrameArgs &a, bool split, uint32_t blocks, hipStream_t stream) {
  if (split) launch_blend<PPT, TH, true>(a, blocks, stream);
  else launch_blend<PPT, TH, false>(a, blocks, stream);
}

template <int PPT, int TH, bool SPLIT>
void launch_batch_blend(const unsigned char *desc, uint32_t grid, hipStream_t stream) {
  k_batch_blend<PPT, TH, 0, 3, SPLIT><<<grid, 16 * TH, 0, stream>>>(desc);
  k_batch_blend<PPT, TH, 4, SB_MAX_RADIUS, SPLIT><<<grid, 16 * TH, 0, stream>>>(desc);
}

template <int PPT, int TH>
void launch_batch_blend_any(const unsigned char *desc, bool split, uint32_t grid,
                            hipStream_t stream) {
  if (split) launch_batch_blend<PPT, TH, true>(desc, grid, stream);
  else launch_batch_blend<PPT, TH, false>(desc, grid, stream);
}

template <int PPT, int TH, bool SPLIT>
void launch_batch_blend_exact(const unsigned char *desc, const uint32_t *totals,
                              hipStream_t stream) {
  if (totals[2]) k_batch_blend<PPT, TH, 0, 3, SPLIT><<<totals[2], 16 * TH, 0, stream>>>(desc);
  if (totals[3])
    k_batch_blend<PPT, TH, 4, SB_MAX_RADIUS, SPLIT><<<totals[3], 16 * TH, 0, stream>>>(desc);
}

template <int PPT, int TH>
void launch_batch_blend_exact_any(const unsigned char *desc, bool split, const uint32_t *totals,
                                  hipStream_t stream) {
  if (split) launch_batch_blend_exact<PPT, TH, true>(desc, totals, stream);
  else launch_batch_blend_exact<PPT, TH, false>(desc, totals, stream);
}

}  // namespace

hipError_t launch_pack_exemplar(const uint8_t *rgb, int32_t sw, int32_t sh, uint32_t *rgba,
                                hipStream_t stream) {
  const uint32_t n = uint32_t(ex_texels(sw, sh));
  k_pack_exemplar<<<blocks_for(n, 256), 256, 0, stream>>>(rgb, sw, sh, n, rgba);
  return hipGetLastError();
}

void tile_counts(const FrameArgs &a, const Tune &t, uint32_t counts[4]) {
  const uint32_t tw = 16 * uint32_t(t.ppt), th = uint32_t(t.rows);
  const uint32_t blend = ((uint32_t(a.w) + tw - 1) / tw) * ((uint32_t(a.h) + th - 1) / th);
  // no seed table when the block level loop makes its own records
  counts[0] = a.own_seeds ? 0u : (uint32_t(a.lv.poffset[a.lv.count]) + 255) / 256;
  const uint32_t aw = t.apx >= 2 ? 32u : 16u, ah = t.apx == 4 ? 32u : 16u;
  counts[1] = ((uint32_t(a.w) + aw - 1) / aw) * ((uint32_t(a.h) + ah - 1) / ah);
  counts[2] = a.radius <= 3 ? blend : 0;
  counts[3] = a.radius <= 3 ? 0 : blend;
}

hipError_t launch_stylize(const FrameArgs &a, int32_t fmt, const Tune &t, hipEvent_t *ev,
                          hipStream_t stream) {
  uint32_t c[4];
  tile_counts(a, t, c);
  hipError_t e = hipSuccess;
  if (ev) e = hipEventRecord(ev[0], stream);
  if (fmt_search(fmt)) {
    // seed and level-loop passes of the search formats; the vote is shared
    if (e == hipSuccess) e = launch_search_frame(a, ev, stream);
  } else {
    if (e == hipSuccess && c[0] > 0) {
      if (fmt == SB_GUIDE_U8X2)
        k_seeds<SB_GUIDE_U8X2><<<c[0], 256, 0, stream>>>(a);
      else if (fmt == SB_GUIDE_U8X3)
        k_seeds<SB_GUIDE_U8X3><<<c[0], 256, 0, stream>>>(a);
      else
        k_seeds<SB_GUIDE_U16X2><<<c[0], 256, 0, stream>>>(a);
    }
    if (ev && e == hipSuccess) e = hipEventRecord(ev[1], stream);
    if (e == hipSuccess) {
      if (fmt == SB_GUIDE_U8X2) launch_assign_any<SB_GUIDE_U8X2>(a, t, c[1], stream);
      else if (fmt == SB_GUIDE_U8X3) launch_assign_any<SB_GUIDE_U8X3>(a, t, c[1], stream);
      else launch_assign_any<SB_GUIDE_U16X2>(a, t, c[1], stream);
    }
  }
  if (ev && e == hipSuccess) e = hipEventRecord(ev[2], stream);
  if (e == hipSuccess) {
    const uint32_t nb = c[2] + c[3];
    const bool sp = t.split == 2;
    if (t.ppt == 4 && t.rows == 16) launch_blend_any<4, 16>(a, sp, nb, stream);
    else if (t.ppt == 4) launch_blend_any<4, 8>(a, sp, nb, stream);
    else if (t.rows == 16) launch_blend_any<2, 16>(a, sp, nb, stream);
    else launch_blend_any<2, 8>(a, sp, nb, stream);
  }
  if (ev && e == hipSuccess) e = hipEventRecord(ev[3], stream);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_batch_exact(const unsigned char *desc_dev, const uint32_t totals[kBatchKinds],
                              const Tune &t, hipStream_t stream) {
  if (totals[0]) k_batch_seeds<<<totals[0], 256, 0, stream>>>(desc_dev);
  if (totals[1]) {
    if (t.group == 4) {
      if (t.apx == 4) k_batch_assign<4, 4><<<totals[1], 256, 0, stream>>>(desc_dev);
      else if (t.apx == 2) k_batch_assign<4, 2><<<totals[1], 256, 0, stream>>>(desc_dev);
      else k_batch_assign<4, 1><<<totals[1], 256, 0, stream>>>(desc_dev);
    } else {
      if (t.apx == 4) k_batch_assign<2, 4><<<totals[1], 256, 0, stream>>>(desc_dev);
      else if (t.apx == 2) k_batch_assign<2, 2><<<totals[1], 256, 0, stream>>>(desc_dev);
      else k_batch_assign<2, 1><<<totals[1], 256, 0, stream>>>(desc_dev);
    }
  }
  const bool sp = t.split == 2;
  if (t.ppt == 4 && t.rows == 16) launch_batch_blend_exact_any<4, 16>(desc_dev, sp, totals, stream);
  else if (t.ppt == 4) launch_batch_blend_exact_any<4, 8>(desc_dev, sp, totals, stream);
  else if (t.rows == 16) launch_batch_blend_exact_any<2, 16>(desc_dev, sp, totals, stream);
  else launch_batch_blend_exact_any<2, 8>(desc_dev, sp, totals, stream);
  return hipGetLastError();
}

hipError_t launch_batch(const unsigned char *desc_dev, uint32_t grid, const Tune &t,
                        hipStream_t stream) {
  k_batch_seeds<<<grid, 256, 0, stream>>>(desc_dev);
  if (t.group == 4) {
    if (t.apx == 4) k_batch_assign<4, 4><<<grid, 256, 0, stream>>>(desc_dev);
    else if (t.apx == 2) k_batch_assign<4, 2><<<grid, 256, 0, stream>>>(desc_dev);
    else k_batch_assign<4, 1><<<grid, 256, 0, stream>>>(desc_dev);
  } else {
    if (t.apx == 4) k_batch_assign<2, 4><<<grid, 256, 0, stream>>>(desc_dev);
    else if (t.apx == 2) k_batch_assign<2, 2><<<grid, 256, 0, stream>>>(desc_dev);
    else k_batch_assign<2, 1><<<grid, 256, 0, stream>>>(desc_dev);
  }
  const bool sp = t.split == 2;
  if (t.ppt == 4 && t.rows == 16) launch_batch_blend_any<4, 16>(desc_dev, sp, grid, stream);
  else if (t.ppt == 4) launch_batch_blend_any<4, 8>(desc_dev, sp, grid, stream);
  else if (t.rows == 16) launch_batch_blend_any<2, 16>(desc_dev, sp, grid, stream);
  else launch_batch_blend_any<2, 8>(desc_dev, sp, grid, stream);
  return hipGetLastError();
}

}  // namespace sb
