// sb_internal.h -- shared definitions of the gfx950 StyleBlit library (kernels
// and host entry points).  Not part of the public ABI (see include/styleblit.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "styleblit.h"

namespace sb {

// An invalid seed record: no in-image seed for that cell.
constexpr uint32_t kNoSeed = 0xFFFFFFFFu;
// Offset of an out-of-target neighbour in the voting tile: adding it to any
// in-range pixel coordinate lands at x or y >= 32768, outside every source.
constexpr uint32_t kNoVote = 0x80008000u;

// Geometry of the seed hierarchy of one frame, passed by value to kernels.
struct Levels {
  int32_t count;                       // L
  int32_t log2_spacing[SB_MAX_LEVELS]; // level i (0 = coarsest)
  int32_t cells_x[SB_MAX_LEVELS];
  int32_t cells_y[SB_MAX_LEVELS];
  int32_t offset[SB_MAX_LEVELS + 1];   // first table entry of level i; offset[L] = total
};

// Everything one frame's kernels read: device pointers plus sizes.
struct FrameArgs {
  const uint32_t *src_rgba;   // Sw*Sh texels
  const void *src_guide;      // Sw*Sh*2 channels
  const uint32_t *lut;        // (1 << lut_bits)^2
  const void *tgt_guide;      // W*H*2 channels
  const uint32_t *jitter;     // Levels.offset[L] entries
  uint8_t *out_rgb;           // W*H*3
  uint32_t *out_chunk;        // W*H
  uint32_t *out_nnf;          // W*H or null
  uint2 *seeds;               // workspace: per cell {position x|y<<16, offset dx|dy<<16}
  uint32_t *offsets;          // workspace: per pixel NNF[p] - p as two int16
  int32_t sw, sh, w, h;
  int32_t lut_bits, lut_shift; // lut_shift = guide depth - lut_bits
  uint32_t threshold;
  int32_t radius;
  Levels lv;
};

// Fill the level geometry for a W x H frame; false if the parameters are out
// of range.
bool make_levels(int32_t w, int32_t h, int32_t levels, int32_t finest, Levels *out);

// Thread-local error text of the last failed HIP call.
void set_hip_error(hipError_t e, const char *where);
void set_error_text(const char *msg);

// Launchers (stylize.hip, lut.hip).  Each returns hipSuccess or the launch
// error.
hipError_t launch_pack_exemplar(const uint8_t *rgb, int32_t sw, int32_t sh, uint32_t *rgba,
                                hipStream_t stream);
hipError_t launch_stylize(const FrameArgs &a, int32_t fmt, hipStream_t stream);
size_t lut_workspace_bytes(int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits);
hipError_t launch_lut_build(const void *guide, int32_t fmt, int32_t sw, int32_t sh,
                            int32_t lut_bits, uint32_t *lut, void *workspace, hipStream_t stream);

__host__ __device__ inline uint32_t pack_xy(uint32_t x, uint32_t y) { return x | (y << 16); }

}  // namespace sb
