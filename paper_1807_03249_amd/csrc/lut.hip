// lut.hip -- device-side build of the guide-to-source lookup table (Sec. 3.1).
//
// LUT[c] = argmin_u |centre(c) - G_S[u]|^2 over all source pixels u, ties to
// the smallest raster index.
//
// 8-bit guides (two or three channels) take a separable exact transform:
// every value tuple a source pixel holds is a site keyed by the smallest
// raster index holding it, and since the squared distance is a sum over
// channels, the (distance, index) minimum over all sites can be taken one
// channel at a time -- first over channel 0 for every fixed value of the
// other channels, then over channel 1, ... -- on the grid of bin centres.
// Keys are uint64 (distance << 32 | index), so the lexicographic minimum is
// the integer minimum, and adding one channel's (weighted) squared distance
// to every key of a line keeps their order.  Each pass is a brute-force minimum over
// the 256 values of one channel, restricted to the values that hold a site.
//
// 16-bit guides (too many value tuples for a grid) bucket the source pixels
// on a grid whose
// cells are at least twice as wide as a lookup bin (counting sort: count,
// scan, scatter), and each bin then searches square rings of buckets around
// the bucket holding its centre.  After ring k the searched box is known, so
// every unsearched pixel is at least `gap` away along one axis, where gap is
// the distance from the centre to the nearest open side of the box; the
// search ends once the best squared distance is strictly below gap^2 (an
// equal distance further out could still win the raster-index tie).
#include "sb_internal.h"

namespace sb {
namespace {

struct LutGeom {
  int32_t depth;       // guide bits per channel: 8 or 16
  int32_t lut_bits;    // bins per channel = 1 << lut_bits
  int32_t bucket_bits; // buckets per channel = 1 << bucket_bits
  int32_t npix;
};

LutGeom lut_geom(int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits) {
  LutGeom g;
  g.depth = fmt == SB_GUIDE_U8X2 ? 8 : 16;
  g.lut_bits = lut_bits;
  g.npix = sw * sh;
  // about one bucket per few source pixels, never finer than half a bin
  int32_t side_bits = 0;
  while ((int64_t(1) << (2 * (side_bits + 1))) <= int64_t(g.npix)) ++side_bits;
  int32_t bb = side_bits - 1;
  if (bb > lut_bits - 1) bb = lut_bits - 1;
  if (bb < 1) bb = 1;
  if (bb > g.depth) bb = g.depth;
  g.bucket_bits = bb;
  return g;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct LutWs {
  uint32_t *count;  // nb  (counts, then scatter cursors)
  uint32_t *start;  // nb + 1
  uint2 *pts;       // npix: {g0 | g1 << 16, raster index}
};

LutWs lut_ws(void *base, const LutGeom &g) {
  size_t nb = size_t(1) << (2 * g.bucket_bits);
  char *p = static_cast<char *>(base);
  LutWs w;
  w.count = reinterpret_cast<uint32_t *>(p);
  p += align256(nb * 4);
  w.start = reinterpret_cast<uint32_t *>(p);
  p += align256((nb + 1) * 4);
  w.pts = reinterpret_cast<uint2 *>(p);
  return w;
}

// ------------------------------------------------ separable (8-bit guides)

constexpr uint64_t kNoKey = ~0ull;
constexpr int32_t kSepTile = 16;  // columns of one pass block

// f0[value tuple c0 | c1 << 8 (| c2 << 16)] = smallest raster index holding
// it (pre-filled with ~0u); with `labels`, only pixels labelled `want`.
template <int FMT>
__global__ void k_sep_sites(const void *guide, int32_t npix, uint32_t *f0, const uint8_t *labels,
                            int32_t want) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= uint32_t(npix)) return;
  if (labels && labels[i] != want) return;
  const uint32_t v = FMT == SB_GUIDE_U8X2 ? uint32_t(static_cast<const uint16_t *>(guide)[i])
                                          : static_cast<const uint32_t *>(guide)[i] & 0xFFFFFFu;
  atomicMin(&f0[v], i);
}

// One channel of the minimisation.  The input is [outer][256][inner]: keys,
// or with SITES the site indices of f0 (~0u: none).  The output is
// [outer][nb][inner] keys, or with FINAL the table entries (coordinates;
// where no site exists at all -- a label absent from the exemplar -- the
// entry of `fallback`).  A block takes one outer index and `ti` adjacent
// columns: it stages the 256 x ti input keys in LDS, lists the channel
// values that hold a key in any of its columns, and computes nb x ti
// minima over that list.
template <bool SITES, bool FINAL>
__global__ __launch_bounds__(256) void k_sep_pass(const void *in, uint64_t *out, uint32_t *lut,
                                                  const uint32_t *fallback, int32_t inner,
                                                  int32_t ti, int32_t lut_bits, int32_t weight,
                                                  int32_t sw) {
  __shared__ uint64_t key[256 * kSepTile];
  __shared__ uint8_t vlist[256];
  __shared__ uint32_t wcount[4];
  const int32_t t = threadIdx.x;
  const int32_t tiles = inner / ti;
  const size_t o = blockIdx.x / uint32_t(tiles);
  const int32_t i0 = int32_t(blockIdx.x % uint32_t(tiles)) * ti;
  for (int32_t e = t; e < 256 * ti; e += 256) {
    const int32_t v = e / ti, j = e - v * ti;
    const size_t src = (o * 256 + size_t(v)) * size_t(inner) + size_t(i0 + j);
    uint64_t k;
    if (SITES) {
      const uint32_t idx = static_cast<const uint32_t *>(in)[src];
      k = idx == ~0u ? kNoKey : uint64_t(idx);
    } else {
      k = static_cast<const uint64_t *>(in)[src];
    }
    key[v * kSepTile + j] = k;
  }
  __syncthreads();
  // compact list of the channel values with a key (thread t examines v = t)
  bool any = false;
  for (int32_t j = 0; j < ti; ++j) any |= key[t * kSepTile + j] != kNoKey;
  const uint64_t mask = __ballot(any);
  const int32_t wave = t >> 6, lane = t & 63;
  if (lane == 0) wcount[wave] = uint32_t(__popcll(mask));
  __syncthreads();
  uint32_t base = 0;
  for (int32_t w = 0; w < wave; ++w) base += wcount[w];
  const uint32_t count = wcount[0] + wcount[1] + wcount[2] + wcount[3];
  if (any) vlist[base + uint32_t(__popcll(mask & ((1ull << lane) - 1ull)))] = uint8_t(t);
  __syncthreads();
  const int32_t nb = 1 << lut_bits, sft = 8 - lut_bits;
  const int32_t half = sft ? 1 << (sft - 1) : 0;
  const int32_t j = t % ti;
  for (int32_t b = t / ti; b < nb; b += 256 / ti) {
    const int32_t centre = (b << sft) + half;
    uint64_t best = kNoKey;
    for (uint32_t n = 0; n < count; ++n) {
      const int32_t v = vlist[n];
      const uint64_t k = key[v * kSepTile + j];
      const int32_t d = centre - v;
      const uint64_t cand = k + (uint64_t(uint32_t(weight * d * d)) << 32);
      best = (k != kNoKey && cand < best) ? cand : best;
    }
    const size_t dst = (o * size_t(nb) + size_t(b)) * size_t(inner) + size_t(i0 + j);
    if (FINAL) {
      const uint32_t idx = uint32_t(best);
      lut[dst] = best == kNoKey ? (fallback ? fallback[dst] : 0u)
                                : pack_xy(idx % uint32_t(sw), idx / uint32_t(sw));
    } else {
      out[dst] = best;
    }
  }
}

// ------------------------------------------------ bucketed (16-bit guides)

__device__ inline void read_guide(const void *g, uint32_t i, uint32_t &c0, uint32_t &c1) {
  const uint32_t v = static_cast<const uint32_t *>(g)[i];
  c0 = v & 0xFFFFu;
  c1 = v >> 16;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Counting sort over the source pixels; with `labels`, only the pixels
// labelled `want` (one per-label table of the segmentation guide).
__global__ void k_lut_count(const void *guide, int32_t npix, int32_t shift, int32_t bb,
                            uint32_t *count, const uint8_t *labels, int32_t want) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= uint32_t(npix)) return;
  if (labels && labels[i] != want) return;
  uint32_t c0, c1;
  read_guide(guide, i, c0, c1);
  atomicAdd(&count[((c1 >> shift) << bb) | (c0 >> shift)], 1u);
}

// Exclusive scan of n counts into start[0..n], one workgroup of 1024 threads;
// each thread owns a contiguous run.  Also turns count[] into the scatter
// cursors (= start).
__global__ void __launch_bounds__(1024) k_lut_scan(uint32_t *count, uint32_t *start, uint32_t n) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (n + 1023) / 1024;
  const uint32_t b0 = t * per < n ? t * per : n;
  const uint32_t b1 = b0 + per < n ? b0 + per : n;
  uint32_t s = 0;
  for (uint32_t i = b0; i < b1; ++i) s += count[i];
  part[t] = s;
  __syncthreads();
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    uint32_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - s;  // exclusive prefix of this thread's run
  for (uint32_t i = b0; i < b1; ++i) {
    uint32_t c = count[i];
    start[i] = run;
    count[i] = run;
    run += c;
  }
  if (t == 1023) start[n] = part[1023];
}

__global__ void k_lut_scatter(const void *guide, int32_t npix, int32_t shift, int32_t bb,
                              uint32_t *cursor, uint2 *pts, const uint8_t *labels, int32_t want) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= uint32_t(npix)) return;
  if (labels && labels[i] != want) return;
  uint32_t c0, c1;
  read_guide(guide, i, c0, c1);
  uint32_t pos = atomicAdd(&cursor[((c1 >> shift) << bb) | (c0 >> shift)], 1u);
  pts[pos] = make_uint2(c0 | (c1 << 16), i);
}

// `fallback` (may be null): when no pixel was bucketed (a label absent from
// the exemplar), copy this table instead.
__global__ void k_lut_query(const uint32_t *start, const uint2 *pts, int32_t lut_bits,
                            int32_t bin_shift, int32_t bucket_bits, int32_t bucket_shift,
                            int32_t sw, uint32_t *lut, const uint32_t *fallback) {
  const uint32_t nbins = 1u << (2 * lut_bits);
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nbins) return;
  if (fallback && start[1u << (2 * bucket_bits)] == 0) {
    lut[c] = fallback[c];
    return;
  }
  const uint32_t half = bin_shift ? (1u << (bin_shift - 1)) : 0u;
  const uint32_t qx = ((c & ((1u << lut_bits) - 1)) << bin_shift) + half;
  const uint32_t qy = ((c >> lut_bits) << bin_shift) + half;
  const int32_t nb = 1 << bucket_bits;
  const int32_t bw = 1 << bucket_shift;  // bucket width in guide units
  const int32_t bx0 = int32_t(qx >> bucket_shift), by0 = int32_t(qy >> bucket_shift);
  uint64_t best_d = ~0ull;
  uint32_t best_i = ~0u;
  for (int32_t k = 0;; ++k) {
    const int32_t x0 = bx0 - k, x1 = bx0 + k, y0 = by0 - k, y1 = by0 + k;
    const int32_t ya = y0 > 0 ? y0 : 0, yb = y1 < nb - 1 ? y1 : nb - 1;
    for (int32_t by = ya; by <= yb; ++by) {
      const bool full = (by == y0) || (by == y1);
      const int32_t step = full ? 1 : (x1 - x0);
      for (int32_t bx = x0; bx <= x1; bx += (step > 0 ? step : 1)) {
        if (bx < 0 || bx >= nb) continue;
        const uint32_t b = (uint32_t(by) << bucket_bits) | uint32_t(bx);
        const uint32_t e1 = start[b + 1];
        for (uint32_t e = start[b]; e < e1; ++e) {
          const uint2 p = pts[e];
          const int64_t dx = int64_t(qx) - int64_t(p.x & 0xFFFFu);
          const int64_t dy = int64_t(qy) - int64_t(p.x >> 16);
          const uint64_t d = uint64_t(dx * dx) + uint64_t(dy * dy);
          if (d < best_d || (d == best_d && p.y < best_i)) {
            best_d = d;
            best_i = p.y;
          }
        }
      }
    }
    // distance from the centre to the nearest side of the searched box that
    // still has buckets beyond it
    uint32_t gap = ~0u;
    if (x0 > 0) gap = min(gap, qx - uint32_t(x0 * bw) + 1u);
    if (x1 < nb - 1) gap = min(gap, uint32_t((x1 + 1) * bw) - qx);
    if (y0 > 0) gap = min(gap, qy - uint32_t(y0 * bw) + 1u);
    if (y1 < nb - 1) gap = min(gap, uint32_t((y1 + 1) * bw) - qy);
    if (gap == ~0u) break;  // every bucket searched
    if (best_i != ~0u && best_d < uint64_t(gap) * gap) break;
  }
  lut[c] = pack_xy(best_i % uint32_t(sw), best_i / uint32_t(sw));
}

unsigned blocks_for(uint64_t n, unsigned bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

namespace {
// Workspace of the separable build: X holds the keys after channel 0; Y
// first the site grid, then (three channels) the keys after channel 1.
struct SepWs {
  uint64_t *x;
  void *y;
};
size_t sep_x_bytes(int32_t nch, int32_t lut_bits) {
  return align256((size_t(1) << (8 * (nch - 1))) * (size_t(1) << lut_bits) * 8);
}
size_t sep_y_bytes(int32_t nch, int32_t lut_bits) {
  const size_t sites = (size_t(1) << (8 * nch)) * 4;
  const size_t keys1 = nch == 3 ? size_t(256) * (size_t(1) << (2 * lut_bits)) * 8 : 0;
  return align256(sites > keys1 ? sites : keys1);
}
}  // namespace

size_t lut_workspace_bytes(int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits) {
  if (fmt != SB_GUIDE_U16X2) {
    const int32_t nch = fmt_channels(fmt);
    return sep_x_bytes(nch, lut_bits) + sep_y_bytes(nch, lut_bits);
  }
  LutGeom g = lut_geom(fmt, sw, sh, lut_bits);
  size_t nb = size_t(1) << (2 * g.bucket_bits);
  return align256(nb * 4) + align256((nb + 1) * 4) + align256(size_t(g.npix) * 8);
}

namespace {
// Launch one pass over [outer][256][inner] -> [outer][nb][inner].
template <bool SITES, bool FINAL>
void sep_pass(const void *in, uint64_t *out, uint32_t *lut, const uint32_t *fallback,
              size_t outer, int32_t inner, int32_t lut_bits, int32_t weight, int32_t sw,
              hipStream_t stream) {
  // up to kSepTile columns per block, fewer when that leaves the chip
  // short of blocks (the last pass of a two-channel table has one line of
  // 2^lut_bits columns)
  int32_t ti = inner < kSepTile ? inner : kSepTile;
  while (ti > 1 && outer * size_t(inner / ti) < 2048) ti >>= 1;
  const size_t blocks = outer * size_t(inner / ti);
  k_sep_pass<SITES, FINAL><<<unsigned(blocks), 256, 0, stream>>>(in, out, lut, fallback, inner,
                                                                  ti, lut_bits, weight, sw);
}

hipError_t build_sep(const void *guide, int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits,
                     const int32_t *wt, uint32_t *lut, void *workspace, const uint8_t *labels,
                     int32_t want, const uint32_t *fallback, hipStream_t stream) {
  const int32_t nch = fmt_channels(fmt);
  const int32_t nb = 1 << lut_bits, npix = sw * sh;
  uint64_t *x = static_cast<uint64_t *>(workspace);
  char *y = static_cast<char *>(workspace) + sep_x_bytes(nch, lut_bits);
  uint32_t *f0 = reinterpret_cast<uint32_t *>(y);
  const uint32_t nsites = 1u << (8 * nch);
  k_fill_u32<<<blocks_for(nsites, 256) < 4096 ? blocks_for(nsites, 256) : 4096, 256, 0, stream>>>(
      f0, nsites, ~0u);
  if (fmt == SB_GUIDE_U8X2)
    k_sep_sites<SB_GUIDE_U8X2><<<blocks_for(npix, 256), 256, 0, stream>>>(guide, npix, f0, labels,
                                                                          want);
  else
    k_sep_sites<SB_GUIDE_U8X3><<<blocks_for(npix, 256), 256, 0, stream>>>(guide, npix, f0, labels,
                                                                          want);
  // channel 0: [v_rest][v0] -> [v_rest][b0]
  sep_pass<true, false>(f0, x, nullptr, nullptr, size_t(1) << (8 * (nch - 1)), 1, lut_bits,
                        wt[0], sw, stream);
  if (nch == 2) {
    // channel 1: [v1][b0] -> [b1][b0], the table
    sep_pass<false, true>(x, nullptr, lut, fallback, 1, nb, lut_bits, wt[1], sw, stream);
  } else {
    uint64_t *k1 = reinterpret_cast<uint64_t *>(y);  // the site grid is no longer needed
    // channel 1: [v2][v1][b0] -> [v2][b1][b0]
    sep_pass<false, false>(x, k1, nullptr, nullptr, 256, nb, lut_bits, wt[1], sw, stream);
    // channel 2: [v2][b1 b0] -> [b2][b1 b0], the table
    sep_pass<false, true>(k1, nullptr, lut, fallback, 1, nb * nb, lut_bits, wt[2], sw, stream);
  }
  return hipGetLastError();
}

// One table: over all source pixels (labels null) or those labelled `want`.
hipError_t build_one(const void *guide, int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits,
                     const int32_t *wt, uint32_t *lut, void *workspace, const uint8_t *labels,
                     int32_t want, const uint32_t *fallback, hipStream_t stream) {
  if (fmt != SB_GUIDE_U16X2)
    return build_sep(guide, fmt, sw, sh, lut_bits, wt, lut, workspace, labels, want, fallback,
                     stream);
  const LutGeom g = lut_geom(fmt, sw, sh, lut_bits);
  const LutWs w = lut_ws(workspace, g);
  const uint32_t nb = 1u << (2 * g.bucket_bits);
  const int32_t shift = g.depth - g.bucket_bits;
  k_fill_u32<<<blocks_for(nb, 256) < 4096 ? blocks_for(nb, 256) : 4096, 256, 0, stream>>>(
      w.count, nb, 0u);
  k_lut_count<<<blocks_for(g.npix, 256), 256, 0, stream>>>(guide, g.npix, shift, g.bucket_bits,
                                                           w.count, labels, want);
  k_lut_scan<<<1, 1024, 0, stream>>>(w.count, w.start, nb);
  k_lut_scatter<<<blocks_for(g.npix, 256), 256, 0, stream>>>(guide, g.npix, shift, g.bucket_bits,
                                                             w.count, w.pts, labels, want);
  const uint64_t nbins = uint64_t(1) << (2 * lut_bits);
  k_lut_query<<<blocks_for(nbins, 256), 256, 0, stream>>>(
      w.start, w.pts, lut_bits, g.depth - lut_bits, g.bucket_bits, shift, sw, lut, fallback);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_lut_build(const void *guide, int32_t fmt, int32_t sw, int32_t sh,
                            int32_t lut_bits, const int32_t wt[3], uint32_t *lut,
                            void *workspace, hipStream_t stream) {
  return build_one(guide, fmt, sw, sh, lut_bits, wt, lut, workspace, nullptr, 0, nullptr, stream);
}

hipError_t launch_lut_build_labels(const void *guide, const uint8_t *labels, int32_t fmt,
                                   int32_t sw, int32_t sh, int32_t lut_bits, const int32_t wt[3],
                                   int32_t nlabels, const uint32_t *lut, uint32_t *luts,
                                   void *workspace, hipStream_t stream) {
  const size_t bins = size_t(1) << (fmt_channels(fmt) * lut_bits);
  for (int32_t l = 0; l < nlabels; ++l) {
    const hipError_t e = build_one(guide, fmt, sw, sh, lut_bits, wt, luts + size_t(l) * bins,
                                   workspace, labels, l, lut, stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sb
