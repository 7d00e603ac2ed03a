// sb_internal.h -- shared definitions of the gfx950 StyleBlit library (kernels
// and host entry points).  Not part of the public ABI (see include/styleblit.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "styleblit.h"

namespace sb {

// Position word of an invalid seed record (no in-image seed for that cell):
// the int16 pair (-32768, -32768), farther from every pixel than any seed.
constexpr uint32_t kNoSeed = 0x80008000u;
// Offset of an out-of-target neighbour in the voting tile: adding it to any
// in-range pixel coordinate lands at x or y >= 32768, outside every source.
constexpr uint32_t kNoVote = 0x80008000u;

// Geometry of the seed hierarchy of one frame, passed by value to kernels.
struct Levels {
  int32_t count;                       // L
  int32_t log2_spacing[SB_MAX_LEVELS]; // level i (0 = coarsest)
  int32_t cells_x[SB_MAX_LEVELS];
  int32_t cells_y[SB_MAX_LEVELS];
  int32_t offset[SB_MAX_LEVELS + 1];   // first jitter entry of level i; offset[L] = total
  // seed records: per level a (cells_x + 2) x (cells_y + 2) grid, the cells
  // plus a ring of empty records, so every 3x3 neighbourhood is in the table
  int32_t poffset[SB_MAX_LEVELS + 1];  // first record of level i; poffset[L] = total
};

// Guide formats: channels and bits per channel.
__host__ __device__ constexpr bool fmt_ok(int32_t fmt) {
  return fmt == SB_GUIDE_U8X2 || fmt == SB_GUIDE_U16X2 || fmt == SB_GUIDE_U8X3;
}
__host__ __device__ constexpr int32_t fmt_channels(int32_t fmt) {
  return fmt == SB_GUIDE_U8X3 ? 3 : 2;
}
__host__ __device__ constexpr int32_t fmt_depth(int32_t fmt) {
  return fmt == SB_GUIDE_U16X2 || fmt == SB_GUIDE_U16XN ? 16 : 8;
}
// Guides of 2..8 channels looked up by the exact search (search.hip).
__host__ __device__ constexpr bool fmt_search(int32_t fmt) {
  return fmt == SB_GUIDE_U8XN || fmt == SB_GUIDE_U16XN;
}
// Bytes per texel of a search-format guide of `channels` channels: 4, 8 or
// 16; 0 if invalid.
__host__ __device__ constexpr int32_t search_texel_bytes(int32_t fmt, int32_t channels) {
  return !fmt_search(fmt) || channels < 2 || channels > SB_MAX_CHANNELS ? 0
         : channels * fmt_depth(fmt) <= 32                               ? 4
         : channels * fmt_depth(fmt) <= 64                               ? 8
                                                                         : 16;
}

// The search tree of an n-texel source guide of t-byte texels, in one
// buffer: node records of 2t + 8 bytes -- the node's box (the lowest and the
// highest value of every element over its texels, as two texels) and its
// link (inner: {first child, 0}, the two children adjacent; leaf: {first
// texel, count | kTreeLeaf}) -- then the leaves' texels and their source
// coordinates (x | y << 16).  A tree has at most 2n - 1 nodes.
constexpr uint32_t kTreeLeaf = 0x80000000u;
__host__ __device__ constexpr size_t tree_record_bytes(size_t t) { return 2 * t + 8; }
constexpr size_t kLeafGroup = 4;
struct TreeLayout {
  size_t nodes, vals, keys, total;
};
inline TreeLayout tree_layout(size_t n, size_t t) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  TreeLayout l;
  l.nodes = 256;
  l.vals = l.nodes + al(2 * n * tree_record_bytes(t));
  // room for kLeafGroup - 1 entries past the last texel and key: a search
  // reads a leaf's texels and keys in groups of kLeafGroup
  l.keys = l.vals + al((n + kLeafGroup) * t);
  l.total = l.keys + al((n + kLeafGroup) * 4);
  return l;
}

// Largest voting tile of the blend (pixels): 256 threads, 4 horizontal
// pixels each.
constexpr int32_t kBlendMaxTW = 64, kBlendMaxTH = 16;

// A resolved kernel choice (see sb_tune): pixels per thread and tile rows of
// the vote pass, levels per gather round and pixels per thread of the level
// loop, and whether the vote copies uniform windows and lists the rest
// (split = 2) or votes every pixel in place (1).
struct Tune {
  int32_t ppt, rows, group, apx, split;
};
// Fill a Tune from the caller's sb_tune (NULL or 0 fields = defaults); false
// if a field holds an unsupported value.
bool resolve_tune(const sb_tune *in, Tune *out);

// Padded exemplar: texels of Sw x Sh sit in rows of sw + 2 * kExMargin
// texels with kExMargin empty (zero) texels on every side, followed by zero
// rows that hold one voting tile.  Inside texels carry alpha 1, so a sum of
// votes counts its in-source votes in byte 3.  Every vote lands within
// SB_MAX_RADIUS of the source, so no vote needs a bounds check.
constexpr int32_t kExMargin = 8;
__host__ __device__ constexpr int32_t ex_stride(int32_t sw) { return sw + 2 * kExMargin; }
__host__ __device__ constexpr int32_t ex_zero_rows(int32_t sw) {
  return kBlendMaxTH - 1 + (kBlendMaxTW + ex_stride(sw) - 1) / ex_stride(sw);
}
__host__ __device__ constexpr size_t ex_texels(int32_t sw, int32_t sh) {
  return size_t(ex_stride(sw)) * size_t(sh + 2 * kExMargin + ex_zero_rows(sw));
}

// Everything one frame's kernels read: device pointers plus sizes.
struct FrameArgs {
  const uint32_t *src_rgba;   // padded exemplar, ex_texels(sw, sh)
  const void *src_guide;      // Sw*Sh*2 channels
  const uint32_t *lut;        // (1 << lut_bits)^2
  const void *tgt_guide;      // W*H*2 channels
  const uint32_t *jitter;     // Levels.offset[L] entries (SB_JITTER_TABLE only)
  uint8_t *out_rgb;           // W*H*3
  uint32_t *out_chunk;        // W*H
  uint32_t *out_nnf;          // W*H or null
  uint2 *seeds;               // workspace: per padded cell {4x | 4y << 16, dx | dy << 16}
  uint32_t *offsets;          // workspace: per pixel the vote's byte distance
                              // 4 (oy ex_stride + ox) of its offset o = NNF[p] - p
  int32_t sw, sh, w, h;
  int32_t lut_bits, lut_shift; // lut_shift = guide depth - lut_bits
  int32_t lut_log2;            // log2 of the table's entries: channels * lut_bits
  uint32_t wt02;               // channel weights w0 | w2 << 16 (three-channel guides)
  int32_t wt1;                 // channel weight w1
  int32_t own_seeds;           // the block level loop makes its seed records itself
                               // (8-bit two-channel table, finest spacing >= 8);
                               // otherwise a seed pass fills the seed table first
  uint32_t threshold;
  int32_t radius;
  int32_t fmt;                 // sb_guide_fmt (read by the batch kernels)
  int32_t ex_stride;           // texels per padded exemplar row
  uint32_t ex_zero;            // first texel of the padded exemplar's zero rows
  // segmentation guide: all null / 0 without it
  const uint8_t *src_labels;   // Sw*Sh
  const uint8_t *tgt_labels;   // W*H
  const uint32_t *label_luts;  // nlabels tables of (1 << lut_bits)^2 entries
  int32_t nlabels;
  // seed jitter: sb_jitter mode, and for SB_JITTER_HASH level i's hash state
  // after the seed and level words, mix(mix(seed + 0xBB67AE85) ^ lg_i), so a
  // cell's jitter is two more mixing steps (hash_jitter)
  int32_t jmode;
  uint32_t jhash[SB_MAX_LEVELS];
  // search formats (SB_GUIDE_U8XN / U16XN): the tree's sections, the
  // texel size and the eight channel weights (byte k = weight of element k,
  // 0 past the guide's channels)
  const void *t_nodes;
  const void *t_vals;
  const uint32_t *t_keys;
  int32_t texel;
  uint32_t wn[2];
  Levels lv;
};

// The 32-bit mixing step of the jitter hash (xor-shift, multiply by
// floor(2^32 / golden ratio), xor-shift, multiply by the first 32 fraction
// bits of sqrt(2), xor-shift; wrapping arithmetic).
__host__ __device__ inline uint32_t hash_mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x9E3779B9u;
  x ^= x >> 15;
  x *= 0x6A09E667u;
  x ^= x >> 16;
  return x;
}

// Jitter word jx | jy << 16 of cell (cx, cy) at a level of spacing 2^ls whose
// hash state is hk (FrameArgs::jhash).
__host__ __device__ inline uint32_t hash_jitter(uint32_t hk, int32_t ls, uint32_t cx,
                                                uint32_t cy) {
  const uint32_t k = hash_mix(hash_mix(hk ^ cx) ^ cy);
  const uint32_t m = (1u << ls) - 1u;
  return (k & m) | (((k >> 16) & m) << 16);
}

// Batch descriptor block in device memory: header, per-pass tile prefix sums
// (kMaxBatchFrames + 1 entries each: seeds, assign, blend of radius 0..3,
// blend of radius 4..7) and the frames.
constexpr uint32_t kMaxBatchFrames = 128;
constexpr int kBatchKinds = 4;
struct BatchHeader {
  uint32_t nframes, pad[3];
};
__host__ __device__ constexpr size_t batch_prefix_offset(int kind) {
  return 16 + size_t(kind) * (kMaxBatchFrames + 1) * 4;
}
__host__ __device__ constexpr size_t batch_frames_offset() {
  return (batch_prefix_offset(kBatchKinds) + 255) & ~size_t(255);
}
__host__ __device__ constexpr size_t batch_desc_bytes() {
  return batch_frames_offset() + kMaxBatchFrames * sizeof(FrameArgs);
}

// Fill the level geometry for a W x H frame; false if the parameters are out
// of range.
bool make_levels(int32_t w, int32_t h, int32_t levels, int32_t finest, Levels *out);

// Validate one frame's arguments and fill its kernel arguments (workspace
// pointers are left null).  False on any invalid argument.
bool fill_frame(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                uint32_t *out_chunk, uint32_t *out_nnf, FrameArgs *a,
                const uint8_t *tgt_labels = nullptr);
// Point a frame's seed table and offset map into a workspace of at least
// sb_workspace_bytes() bytes.
void carve_workspace(FrameArgs *a, void *workspace);

// One frame through the per-frame kernels after validation (the body of the
// sb_stylize family): SB_EINVAL / SB_ENOMEM before anything is enqueued,
// SB_EHIP if a launch fails.  events: NULL, or 4 events bracketing the passes.
int stylize_impl(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                 const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                 uint32_t *out_chunk, uint32_t *out_nnf, void *workspace, size_t workspace_bytes,
                 const sb_tune *tune, hipEvent_t *events, hipStream_t stream,
                 const uint8_t *tgt_labels);

// Thread-local error text of the last failed HIP call.
void set_hip_error(hipError_t e, const char *where);
void set_error_text(const char *msg);

// Launchers (stylize.hip, lut.hip).  Each returns hipSuccess or the launch
// error.
hipError_t launch_pack_exemplar(const uint8_t *rgb, int32_t sw, int32_t sh, uint32_t *rgba,
                                hipStream_t stream);
// One frame's three passes; with ev (4 events) records ev[0..3] before the
// seed, assignment and vote passes and after the vote pass.
hipError_t launch_stylize(const FrameArgs &a, int32_t fmt, const Tune &t, hipEvent_t *ev,
                          hipStream_t stream);
// The seed and level-loop passes of a search-format frame (search.hip); with
// ev, records ev[1] between them.
hipError_t launch_search_frame(const FrameArgs &a, hipEvent_t *ev, hipStream_t stream);
// Element weights of a search-format guide: `channels` bytes 0..127 (NULL or
// all zero: unit), packed as FrameArgs::wn; false if a weight exceeds 127.
bool resolve_weights_n(const uint8_t *in, int32_t channels, uint32_t out[2]);
// Point a frame's tree fields at a search-format style's tree.
void fill_tree_args(const sb_style *style, FrameArgs *a);
// Tiles of one frame per batch pass kind (seeds, assign, vote r <= 3, vote r >= 4).
void tile_counts(const FrameArgs &a, const Tune &t, uint32_t counts[kBatchKinds]);
// The passes over a batch described at desc_dev, persistent grids.
hipError_t launch_batch(const unsigned char *desc_dev, uint32_t grid, const Tune &t,
                        hipStream_t stream);
// The same passes with exact grids: totals[kind] workgroups (the batch's
// tiles of that pass), one tile each; passes without tiles are not launched.
hipError_t launch_batch_exact(const unsigned char *desc_dev, const uint32_t totals[kBatchKinds],
                              const Tune &t, hipStream_t stream);
// Channel weights from the caller's three bytes (NULL or all zero: unit);
// false if a weight exceeds 127 or a two-channel format gets non-unit ones.
bool resolve_weights(int32_t fmt, const uint8_t *in, int32_t out[3]);
size_t lut_workspace_bytes(int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits);
hipError_t launch_lut_build(const void *guide, int32_t fmt, int32_t sw, int32_t sh,
                            int32_t lut_bits, const int32_t wt[3], uint32_t *lut,
                            void *workspace, hipStream_t stream);
hipError_t launch_lut_build_labels(const void *guide, const uint8_t *labels, int32_t fmt,
                                   int32_t sw, int32_t sh, int32_t lut_bits, const int32_t wt[3],
                                   int32_t nlabels, const uint32_t *lut, uint32_t *luts,
                                   void *workspace, hipStream_t stream);

__host__ __device__ inline uint32_t pack_xy(uint32_t x, uint32_t y) { return x | (y << 16); }

// A frame pointer as a global-memory pointer.  Kernels that read their
// FrameArgs from memory (the batch kernels) would otherwise address through
// flat instructions.
#define SB_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ SB_GLOBAL T *glb(T *p) {
  return (SB_GLOBAL T *)p;
}

}  // namespace sb
