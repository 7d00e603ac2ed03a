// frame.hip -- the fused single-kernel StyleBlit frame path for gfx950.
//
// One workgroup (256 threads, 4 wave64s) owns a TW x TH tile of target pixels
// and runs every step of the per-frame path for it:
//
//  1. Seed staging.  For each level, the cells around the tile (plus the
//     voting halo and one ring of neighbour cells) get their jittered seed
//     (SeedPoint, Algorithm 2), its in-image flag and the translation u* - q
//     from the seed's lookup (Sec. 3.1), written to LDS once per tile.
//  2. Candidate pruning.  For every 8x8 pixel block of the tile and every
//     level whose spacing is >= 8 (so the whole block shares one cell), a
//     9-bit mask keeps only the neighbour seeds that can be the first strict
//     minimum of NearestSeed for some pixel of the block: a seed is dropped
//     when its smallest distance to the block exceeds another seed's largest
//     distance to it, so it is strictly farther for every pixel.  Scan order
//     is kept, so the first strict minimum is unchanged.
//  3. Level loop (Algorithm 2) for every pixel of the tile and of the r-pixel
//     halo the vote needs.  A wave takes one 8x8 block at a time, so the
//     candidate list is wave-uniform; halo pixels go through the same loop
//     with all nine candidates.  Offsets NNF[p] - p land in LDS; chunk codes
//     are staged for row-wise stores.
//  4. Voting blend (end of Sec. 3.2).  If the offsets over a block's whole
//     voting footprint are one and the same, every vote of every pixel reads
//     the same texel C_S[NNF[p]] and the average is that texel (copy);
//     otherwise each pixel sums its (2r+1)^2 votes and rounds half up.
//  5. Row-wise stores of the chunk map and of the packed RGB.
#include "sb_internal.h"

namespace sb {
namespace {

template <int FMT>
__device__ inline uint32_t guide_at(const void *g, uint32_t i) {
  if (FMT == SB_GUIDE_U8X2) {
    uint32_t v = static_cast<const uint16_t *>(g)[i];
    return (v & 0xFFu) | ((v >> 8) << 16);
  } else {
    return static_cast<const uint32_t *>(g)[i];
  }
}

__device__ inline uint32_t bin_of(uint32_t g, int32_t shift, int32_t bits) {
  return ((g & 0xFFFFu) >> shift) | (((g >> 16) >> shift) << bits);
}

__device__ inline bool below(uint32_t a, uint32_t b, uint32_t t) {
  const int32_t d0 = int32_t(a & 0xFFFFu) - int32_t(b & 0xFFFFu);
  const int32_t d1 = int32_t(a >> 16) - int32_t(b >> 16);
  const uint32_t s0 = uint32_t(d0 * d0), s1 = uint32_t(d1 * d1);
  // exact: s0 + s1 < t  without 64-bit arithmetic (each square < 2^32)
  return s0 < t && s1 < t - s0;
}

__device__ inline int32_t sx16(uint32_t o) { return int32_t(int16_t(o & 0xFFFFu)); }
__device__ inline int32_t sy16(uint32_t o) { return int32_t(int16_t(o >> 16)); }
__device__ inline uint32_t pk16(int32_t x, int32_t y) { return (uint32_t(x) & 0xFFFFu) | (uint32_t(y) << 16); }

__device__ inline uint32_t div_small(uint32_t n, uint32_t k) {
  uint32_t q = uint32_t(float(n) * __builtin_amdgcn_rcpf(float(k)));
  int32_t r = int32_t(n) - int32_t(q * k);
  if (r < 0) --q;
  else if (r >= int32_t(k)) ++q;
  return q;
}

// NearestSeed over the staged seeds of one level: the first strict minimum of
// the squared distance among the candidates selected by `m` (bit k = (dx+1)*3
// + (dy+1), scanned x outer, y inner).  False when none is in the image.
__device__ __forceinline__ bool nearest(const uint2 *lvl, int32_t gw, int32_t lcx, int32_t lcy,
                                        uint32_t m, int32_t x, int32_t y, uint32_t &bq,
                                        uint32_t &bo) {
  uint32_t best = ~0u;
  // m is wave-uniform: a scalar loop over the kept candidates, in scan order
#pragma unroll 1
  for (uint32_t mm = m; mm; mm &= mm - 1) {
    const int32_t k = __builtin_ctz(mm);
    const uint2 rec = lvl[(lcy + k % 3 - 1) * gw + (lcx + k / 3 - 1)];
    const uint32_t ex = (rec.x & 0xFFFFu) - uint32_t(x), ey = (rec.x >> 16) - uint32_t(y);
    const uint32_t d = rec.x == kNoSeed ? ~0u : ex * ex + ey * ey;  // wraps to the exact square
    if (d < best) {
      best = d;
      bq = rec.x;
      bo = rec.y;
    }
  }
  return best != ~0u;
}

// Candidate of one level for pixel (x, y): whether it exists and lands in the
// source, and the source raster index to test (0 when it does not, so the
// gather can be issued unconditionally).
struct Cand {
  bool ok;
  uint32_t q, off, idx;
};

__device__ __forceinline__ Cand level_cand(const FrameArgs &a, const TileGeom &tg,
                                           const uint2 *seeds, const uint32_t *bmask, int32_t nb,
                                           int32_t ox, int32_t oy, int32_t i, int32_t x,
                                           int32_t y) {
  const int32_t ls = a.lv.log2_spacing[i];
  // the staged grid of a level starts one cell before the region's first cell
  const int32_t lcx = (x >> ls) - ((ox >> ls) - 1), lcy = (y >> ls) - ((oy >> ls) - 1);
  const uint32_t m = bmask ? __builtin_amdgcn_readfirstlane(bmask[i * nb]) : 0x1FFu;
  Cand c;
  c.q = 0;
  c.off = 0;
  c.ok = nearest(seeds + tg.seed_off[i], tg.grid_w[i], lcx, lcy, m, x, y, c.q, c.off);
  const int32_t vx = x + sx16(c.off), vy = y + sy16(c.off);
  c.ok = c.ok && uint32_t(vx) < uint32_t(a.sw) && uint32_t(vy) < uint32_t(a.sh);
  c.idx = c.ok ? uint32_t(vy) * uint32_t(a.sw) + uint32_t(vx) : 0u;
  return c;
}

// The level loop of Algorithm 2 for one pixel, two levels per step so that
// both source-guide gathers are in flight together.  Returns the chunk code
// and the offset NNF[p] - p.
template <int FMT>
__device__ __forceinline__ void assign_one(const FrameArgs &a, const TileGeom &tg,
                                           const uint2 *seeds, const uint32_t *bmask, int32_t nb,
                                           int32_t ox, int32_t oy, int32_t x, int32_t y,
                                           uint32_t &chunk, uint32_t &off) {
  const uint32_t gt = guide_at<FMT>(a.tgt_guide, uint32_t(y) * uint32_t(a.w) + uint32_t(x));
  const int32_t L = a.lv.count;
  // levels in groups of four: every candidate of the group first (LDS only),
  // then their source-guide gathers all in flight, then the tests in order
  for (int32_t i0 = 0; i0 < L; i0 += 4) {
    bool ok0 = false, ok1 = false, ok2 = false, ok3 = false;
    uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, f0 = 0, f1 = 0, f2 = 0, f3 = 0;
    uint32_t x0i = 0, x1i = 0, x2i = 0, x3i = 0;
#define SB_CAND(K)                                                                   \
    if (i0 + K < L) {                                                                \
      const Cand c = level_cand(a, tg, seeds, bmask, nb, ox, oy, i0 + K, x, y);      \
      ok##K = c.ok;                                                                  \
      q##K = c.q;                                                                    \
      f##K = c.off;                                                                  \
      x##K##i = c.idx;                                                               \
    }
    SB_CAND(0) SB_CAND(1) SB_CAND(2) SB_CAND(3)
#undef SB_CAND
    const uint32_t g0 = guide_at<FMT>(a.src_guide, x0i);
    const uint32_t g1 = guide_at<FMT>(a.src_guide, x1i);
    const uint32_t g2 = guide_at<FMT>(a.src_guide, x2i);
    const uint32_t g3 = guide_at<FMT>(a.src_guide, x3i);
#define SB_TEST(K)                                                                   \
    if (ok##K && below(gt, g##K, a.threshold)) {                                     \
      chunk = (uint32_t(i0 + K) << 26) | ((q##K >> 16) << 13) | (q##K & 0xFFFFu);    \
      off = f##K;                                                                    \
      return;                                                                        \
    }
    SB_TEST(0) SB_TEST(1) SB_TEST(2) SB_TEST(3)
#undef SB_TEST
  }
  // no level accepted: the pixel's own lookup (only these lanes gather it)
  const uint32_t fb = a.lut[bin_of(gt, a.lut_shift, a.lut_bits)];
  chunk = (uint32_t(L) << 26) | (uint32_t(y) << 13) | uint32_t(x);
  off = pk16(int32_t(fb & 0xFFFFu) - x, int32_t(fb >> 16) - y);
}

// Voting for one 8x8 block (one pixel per lane).
//
// The block's voting footprint (the block plus an r-pixel ring) holds few
// distinct offsets NNF[n] - n, because chunks are pure translations.  The
// wave labels them (one label per distinct offset, found with ballots),
// gathers for each label the co-located texels C_S[p + o] of all 64 pixels at
// once -- a coalesced 8x8 read -- into an LDS texel buffer, and then every
// pixel sums its (2r+1)^2 votes from LDS through the labels of its window.
// A texel outside the source is stored as 0 with its valid bit clear, so it
// neither adds colour nor counts.  With a single label the window average is
// that texel (the copy case).  More labels than the buffer holds are handled
// in further passes, each summing only the votes whose label it gathered.
constexpr int kDMax = 16;  // labels per pass

// One wave's voting scratch in LDS: the texel buffer (row kDMax stays 0 for
// votes outside the current pass), the pass's label offsets and the
// footprint's labels.
struct VoteLds {
  uint32_t (*tex)[64];
  uint32_t *offs;
  uint16_t *lbl;
};

__host__ __device__ constexpr uint32_t vote_lds_bytes(int32_t r) {
  return uint32_t((kDMax + 1) * 64 * 4 + kDMax * 4 + (((8 + 2 * r) * (8 + 2 * r) * 2 + 15) & ~15));
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

template <int R>
__device__ __forceinline__ uint32_t vote_block(const uint32_t *reg, int32_t RW, int32_t bxl,
                                               int32_t byl, int32_t lane, int32_t x, int32_t y,
                                               bool inimg, const uint32_t *rgba, uint32_t sw,
                                               uint32_t sh, uint32_t P, const VoteLds &v) {
  constexpr int FW = 8 + 2 * R, NC = FW * FW, NS = (NC + 63) / 64;
  constexpr int W = 2 * R + 1;
  uint32_t o[NS], lab[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int q = lane + 64 * s;
    o[s] = q < NC ? reg[(byl + q / FW) * RW + bxl + q % FW] : 0u;
    lab[s] = q < NC ? 0xFFFFu : 0xFFFEu;  // 0xFFFF: not labelled yet
  }
  const int32_t lx = lane & 7, ly = lane >> 3;
  v.tex[kDMax][lane] = 0u;
  uint32_t rb = 0, gk = 0, base = 0;
  for (;;) {
    // label up to kDMax new distinct offsets
    uint32_t nj = 0;
    for (; nj < kDMax; ++nj) {
      bool pend = false;
      uint32_t first = 0;
#pragma unroll
      for (int s = NS - 1; s >= 0; --s)
        if (lab[s] == 0xFFFFu) {
          pend = true;
          first = o[s];
        }
      const uint64_t bal = __ballot(pend);
      if (bal == 0) break;
      const uint32_t os = __builtin_amdgcn_readlane(first, __builtin_ctzll(bal));
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (lab[s] == 0xFFFFu && o[s] == os) lab[s] = base + nj;
      v.offs[nj] = os;
    }
    const bool more = __ballot([&] {
                        bool p = false;
#pragma unroll
                        for (int s = 0; s < NS; ++s) p |= lab[s] == 0xFFFFu;
                        return p;
                      }()) != 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int q = lane + 64 * s;
      if (q < NC) v.lbl[q] = uint16_t(lab[s]);
    }
    wave_lds_sync();
    // texels of this pass's labels: one coalesced block gather each, all in
    // flight before the first is stored
    {
      uint32_t tv[kDMax];
      bool tok[kDMax];
#pragma unroll
      for (uint32_t j = 0; j < kDMax; ++j) {
        const uint32_t os = j < nj ? v.offs[j] : kNoVote;
        const int32_t sx = x + sx16(os), sy = y + sy16(os);
        tok[j] = inimg && uint32_t(sx) < sw && uint32_t(sy) < sh;
        tv[j] = rgba[tok[j] ? uint32_t(sy + kExMargin) * P + uint32_t(sx + kExMargin) : 0u];
      }
#pragma unroll
      for (uint32_t j = 0; j < kDMax; ++j)
        if (j < nj) v.tex[j][lane] = tok[j] ? (tv[j] | 0x01000000u) : 0u;
    }
    wave_lds_sync();
    if (base == 0 && !more && nj == 1) return v.tex[0][lane] & 0x00FFFFFFu;  // one offset: copy
    // opaque per block: keeps the compiler from hoisting all (2r+1)^2 window
    // addresses out of the block loop into registers
    int32_t woff = ly * FW + lx;
    __asm__ volatile("" : "+v"(woff));
    const uint16_t *wl = v.lbl + woff;
    if (base == 0 && !more) {
      for (int32_t dy = 0; dy < W; ++dy) {
#pragma unroll
        for (int32_t dx = 0; dx < W; ++dx) {
          const uint32_t t = v.tex[wl[dy * FW + dx]][lane];
          rb += t & 0x00FF00FFu;
          gk += t & 0xFF00FF00u;
        }
      }
    } else {
      for (int32_t dy = 0; dy < W; ++dy) {
#pragma unroll
        for (int32_t dx = 0; dx < W; ++dx) {
          const uint32_t l = uint32_t(wl[dy * FW + dx]) - base;
          const uint32_t t = v.tex[l < nj ? l : uint32_t(kDMax)][lane];
          rb += t & 0x00FF00FFu;
          gk += t & 0xFF00FF00u;
        }
      }
    }
    base += nj;
    if (!more) break;
    wave_lds_sync();
  }
  const uint32_t k = gk >> 24, hk = k >> 1;
  if (k == 0) return 0u;
  return div_small((rb & 0xFFFFu) + hk, k) | (div_small(((gk >> 8) & 0xFFFFu) + hk, k) << 8) |
         (div_small((rb >> 16) + hk, k) << 16);
}

__device__ __forceinline__ uint32_t vote_any(int32_t r, const uint32_t *reg, int32_t RW,
                                             int32_t bxl, int32_t byl, int32_t lane, int32_t x,
                                             int32_t y, bool inimg, const uint32_t *rgba,
                                             uint32_t sw, uint32_t sh, uint32_t P, const VoteLds &v) {
  switch (r) {
    case 0: return vote_block<0>(reg, RW, bxl, byl, lane, x, y, inimg, rgba, sw, sh, P, v);
    case 1: return vote_block<1>(reg, RW, bxl, byl, lane, x, y, inimg, rgba, sw, sh, P, v);
    case 2: return vote_block<2>(reg, RW, bxl, byl, lane, x, y, inimg, rgba, sw, sh, P, v);
    case 3: return vote_block<3>(reg, RW, bxl, byl, lane, x, y, inimg, rgba, sw, sh, P, v);
    case 4: return vote_block<4>(reg, RW, bxl, byl, lane, x, y, inimg, rgba, sw, sh, P, v);
    case 5: return vote_block<5>(reg, RW, bxl, byl, lane, x, y, inimg, rgba, sw, sh, P, v);
    case 6: return vote_block<6>(reg, RW, bxl, byl, lane, x, y, inimg, rgba, sw, sh, P, v);
    default: return vote_block<7>(reg, RW, bxl, byl, lane, x, y, inimg, rgba, sw, sh, P, v);
  }
}

}  // namespace

constexpr int kThreads = 512, kWaves = kThreads / 64;

template <int FMT, int TW, int TH>
__global__ void __launch_bounds__(kThreads) k_frame(FrameArgs a, TileGeom tg) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int NBX = TW / 8, NBY = TH / 8, NB = NBX * NBY;
  uint2 *seeds = reinterpret_cast<uint2 *>(lds + tg.lds_seeds);
  uint32_t *masks = reinterpret_cast<uint32_t *>(lds + tg.lds_masks);   // [level][block]
  uint32_t *reg = reinterpret_cast<uint32_t *>(lds + tg.lds_region);    // RW x RH offsets
  uint32_t *o_rgb = reinterpret_cast<uint32_t *>(lds + tg.lds_rgb);     // TW x TH

  // XCD-aware tile order: consecutive workgroups land on different XCDs, so
  // give each XCD a contiguous run of tiles (shared halos and source texels
  // then meet in the same L2).
  const uint32_t nt = gridDim.x;
  uint32_t t = blockIdx.x;
  if (nt % 8 == 0) t = (t % 8) * (nt / 8) + t / 8;
  const int32_t tiles_x = tg.tiles_x;
  const int32_t x0 = int32_t(t % uint32_t(tiles_x)) * TW, y0 = int32_t(t / uint32_t(tiles_x)) * TH;
  const int32_t r = a.radius;
  const int32_t RW = TW + 2 * r, RH = TH + 2 * r;
  const int32_t L = a.lv.count;
  const int32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t ox = x0 - r, oy = y0 - r;  // region origin

  // 1. seed staging
  for (int32_t s = tid; s < tg.seed_off[L]; s += kThreads) {
    int32_t i = 0;
    while (s >= tg.seed_off[i + 1]) ++i;
    const int32_t loc = s - tg.seed_off[i];
    const int32_t ls = a.lv.log2_spacing[i];
    const int32_t cx = (ox >> ls) - 1 + loc % tg.grid_w[i];
    const int32_t cy = (oy >> ls) - 1 + loc / tg.grid_w[i];
    uint2 rec = make_uint2(kNoSeed, 0u);
    if (cx >= 0 && cy >= 0 && cx < a.lv.cells_x[i] && cy < a.lv.cells_y[i]) {
      const uint32_t j = a.jitter[a.lv.offset[i] + cy * a.lv.cells_x[i] + cx];
      const uint32_t sx = (uint32_t(cx) << ls) + (j & 0xFFFFu);
      const uint32_t sy = (uint32_t(cy) << ls) + (j >> 16);
      if (sx < uint32_t(a.w) && sy < uint32_t(a.h)) {
        const uint32_t g = guide_at<FMT>(a.tgt_guide, sy * uint32_t(a.w) + sx);
        const uint32_t u = a.lut[bin_of(g, a.lut_shift, a.lut_bits)];
        rec.x = sx | (sy << 16);
        rec.y = pk16(int32_t(u & 0xFFFFu) - int32_t(sx), int32_t(u >> 16) - int32_t(sy));
      }
    }
    seeds[s] = rec;
  }
  __syncthreads();

  // 2. per-block candidate masks for levels whose cells hold whole blocks
  for (int32_t s = tid; s < L * NB; s += kThreads) {
    const int32_t i = s / NB, b = s % NB;
    const int32_t ls = a.lv.log2_spacing[i];
    const int32_t bx0 = x0 + (b % NBX) * 8, by0 = y0 + (b / NBX) * 8;
    const int32_t bx1 = min(bx0 + 7, a.w - 1), by1 = min(by0 + 7, a.h - 1);
    uint32_t m = 0x1FFu;
    if (ls >= 3 && bx0 < a.w && by0 < a.h) {
      const int32_t lcx = (bx0 >> ls) - ((ox >> ls) - 1), lcy = (by0 >> ls) - ((oy >> ls) - 1);
      const uint2 *lvl = seeds + tg.seed_off[i];
      uint32_t mind[9], best_max = ~0u;
      m = 0;
#pragma unroll
      for (int32_t k = 0; k < 9; ++k) {
        const uint2 rec = lvl[(lcy + k % 3 - 1) * tg.grid_w[i] + (lcx + k / 3 - 1)];
        mind[k] = ~0u;
        if (rec.x == kNoSeed) continue;
        const int32_t sx = int32_t(rec.x & 0xFFFFu), sy = int32_t(rec.x >> 16);
        const int32_t nx = sx < bx0 ? bx0 - sx : (sx > bx1 ? sx - bx1 : 0);
        const int32_t ny = sy < by0 ? by0 - sy : (sy > by1 ? sy - by1 : 0);
        const int32_t fx = max(abs(sx - bx0), abs(sx - bx1));
        const int32_t fy = max(abs(sy - by0), abs(sy - by1));
        mind[k] = uint32_t(nx * nx + ny * ny);
        best_max = min(best_max, uint32_t(fx * fx + fy * fy));
        m |= 1u << k;
      }
#pragma unroll
      for (int32_t k = 0; k < 9; ++k)
        if (mind[k] > best_max) m &= ~(1u << k);
    }
    masks[s] = m;
  }
  __syncthreads();

  // 3a. level loop over the tile's 8x8 blocks (wave-uniform candidate masks)
#pragma unroll 1
  for (int32_t b = wave; b < NB; b += kWaves) {
    const int32_t lx = (b % NBX) * 8 + (lane & 7), ly = (b / NBX) * 8 + (lane >> 3);
    const int32_t x = x0 + lx, y = y0 + ly;
    uint32_t chunk = 0, off = kNoVote;
    if (x < a.w && y < a.h) {
      assign_one<FMT>(a, tg, seeds, masks + b, NB, ox, oy, x, y, chunk, off);
      const uint32_t pix = uint32_t(y) * uint32_t(a.w) + uint32_t(x);
      a.out_chunk[pix] = chunk;
      if (a.out_nnf) a.out_nnf[pix] = pk16(x + sx16(off), y + sy16(off));
    }
    reg[(ly + r) * RW + lx + r] = off;
  }
  // 3b. the voting halo around the tile
  {
    const int32_t band = RW * r;  // top and bottom bands
    const int32_t side = r * TH;  // left and right bands
    const int32_t nh = 2 * band + 2 * side;
    for (int32_t h = tid; h < nh; h += kThreads) {
      int32_t rx, ry;
      if (h < band) { rx = h % RW; ry = h / RW; }
      else if (h < 2 * band) { rx = (h - band) % RW; ry = r + TH + (h - band) / RW; }
      else if (h < 2 * band + side) { rx = (h - 2 * band) % r; ry = r + (h - 2 * band) / r; }
      else { rx = r + TW + (h - 2 * band - side) % r; ry = r + (h - 2 * band - side) / r; }
      const int32_t x = ox + rx, y = oy + ry;
      uint32_t off = kNoVote, chunk;
      if (x >= 0 && y >= 0 && x < a.w && y < a.h)
        assign_one<FMT>(a, tg, seeds, nullptr, 0, ox, oy, x, y, chunk, off);
      reg[ry * RW + rx] = off;
    }
  }
  __syncthreads();

  // 4. voting blend, one 8x8 block per wave at a time
  VoteLds vl;
  {
    unsigned char *vb = lds + tg.lds_vote + wave * vote_lds_bytes(r);
    vl.tex = reinterpret_cast<uint32_t(*)[64]>(vb);
    vl.offs = reinterpret_cast<uint32_t *>(vb + (kDMax + 1) * 64 * 4);
    vl.lbl = reinterpret_cast<uint16_t *>(vb + (kDMax + 1) * 64 * 4 + kDMax * 4);
  }
#pragma unroll 1
  for (int32_t b = wave; b < NB; b += kWaves) {
    const int32_t bxl = (b % NBX) * 8, byl = (b / NBX) * 8;
    const int32_t lx = bxl + (lane & 7), ly = byl + (lane >> 3);
    const int32_t x = x0 + lx, y = y0 + ly;
    const bool inimg = x < a.w && y < a.h;
    o_rgb[ly * TW + lx] = vote_any(r, reg, RW, bxl, byl, lane, x, y, inimg, a.src_rgba,
                                   uint32_t(a.sw), uint32_t(a.sh), uint32_t(a.ex_stride), vl);
    wave_lds_sync();
  }
  __syncthreads();

  // 5. row-wise stores of the packed RGB
  const int32_t vw = min(TW, a.w - x0), vh = min(TH, a.h - y0);
  if (vw == TW && (a.w & 3) == 0 && (reinterpret_cast<uintptr_t>(a.out_rgb) & 3) == 0) {
    // 3*TW bytes per row, dword aligned: each thread packs one dword
    constexpr int DW = 3 * TW / 4;
    for (int32_t q = tid; q < DW * vh; q += kThreads) {
      const int32_t ly = q / DW, d = q % DW;
      uint32_t word = 0;
#pragma unroll
      for (int32_t e = 0; e < 4; ++e) {
        const int32_t byte = 4 * d + e;
        const uint32_t px = o_rgb[ly * TW + byte / 3];
        word |= ((px >> (8 * (byte % 3))) & 0xFFu) << (8 * e);
      }
      uint32_t *dst = reinterpret_cast<uint32_t *>(a.out_rgb + 3 * (uint32_t(y0 + ly) * uint32_t(a.w) + uint32_t(x0)));
      dst[d] = word;
    }
  } else {
    for (int32_t q = tid; q < TW * TH; q += kThreads) {
      const int32_t lx = q % TW, ly = q / TW;
      if (lx < vw && ly < vh) {
        const uint32_t px = o_rgb[q];
        uint8_t *dst = a.out_rgb + 3 * (uint32_t(y0 + ly) * uint32_t(a.w) + uint32_t(x0 + lx));
        dst[0] = uint8_t(px);
        dst[1] = uint8_t(px >> 8);
        dst[2] = uint8_t(px >> 16);
      }
    }
  }
}

namespace {

template <int TW, int TH>
bool plan_tile(const FrameArgs &a, TileGeom *tg) {
  const int32_t r = a.radius, L = a.lv.count;
  int32_t off = 0;
  for (int32_t i = 0; i < L; ++i) {
    const int32_t h = 1 << a.lv.log2_spacing[i];
    tg->grid_w[i] = (TW + 2 * r - 1) / h + 4;
    tg->grid_h[i] = (TH + 2 * r - 1) / h + 4;
    tg->seed_off[i] = off;
    off += tg->grid_w[i] * tg->grid_h[i];
  }
  tg->seed_off[L] = off;
  size_t p = 0;
  auto take = [&](size_t bytes) { size_t at = p; p += (bytes + 15) & ~size_t(15); return int32_t(at); };
  tg->lds_seeds = take(size_t(off) * 8);
  tg->lds_masks = take(size_t(L) * (TW / 8) * (TH / 8) * 4);
  tg->lds_region = take(size_t(TW + 2 * r) * (TH + 2 * r) * 4);
  tg->lds_chunk = 0;
  tg->lds_rgb = take(size_t(TW) * TH * 4);
  tg->lds_vote = take(size_t(vote_lds_bytes(r)) * kWaves);
  tg->lds_bytes = int32_t(p);
  tg->tiles_x = (a.w + TW - 1) / TW;
  tg->tiles_y = (a.h + TH - 1) / TH;
  tg->tile_w = TW;
  tg->tile_h = TH;
  return p <= kMaxLds;
}

template <int FMT, int TW, int TH>
hipError_t launch_t(const FrameArgs &a, hipStream_t stream) {
  TileGeom tg;
  memset(&tg, 0, sizeof tg);
  if (!plan_tile<TW, TH>(a, &tg)) return hipErrorInvalidValue;
  const uint32_t n = uint32_t(tg.tiles_x) * uint32_t(tg.tiles_y);
  k_frame<FMT, TW, TH><<<n, kThreads, tg.lds_bytes, stream>>>(a, tg);
  return hipGetLastError();
}

}  // namespace

bool frame_tile_fits(const FrameArgs &a, int32_t tile) {
  TileGeom tg;
  switch (tile) {
    case kTile32x16: return plan_tile<32, 16>(a, &tg);
    case kTile32x32: return plan_tile<32, 32>(a, &tg);
    case kTile64x16: return plan_tile<64, 16>(a, &tg);
    case kTile64x32: return plan_tile<64, 32>(a, &tg);
    default: return false;
  }
}

hipError_t launch_frame(const FrameArgs &a, int32_t fmt, int32_t tile, hipStream_t stream) {
#define SB_TILE_CASE(T, TW, TH)                                                            \
  case T:                                                                                  \
    return fmt == SB_GUIDE_U8X2 ? launch_t<SB_GUIDE_U8X2, TW, TH>(a, stream)               \
                                : launch_t<SB_GUIDE_U16X2, TW, TH>(a, stream);
  switch (tile) {
    SB_TILE_CASE(kTile32x16, 32, 16)
    SB_TILE_CASE(kTile32x32, 32, 32)
    SB_TILE_CASE(kTile64x16, 64, 16)
    SB_TILE_CASE(kTile64x32, 64, 32)
    default: return hipErrorInvalidValue;
  }
#undef SB_TILE_CASE
}

}  // namespace sb
