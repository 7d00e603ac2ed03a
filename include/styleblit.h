/*
 * styleblit.h -- C ABI of the MI355X (gfx950) StyleBlit library.
 *
 * StyleBlit (Sykora et al., EGSR 2018) stylises a target image by copying
 * coherent chunks of a source exemplar C_S.  Every target pixel p walks a
 * hierarchy of jittered seed grids from coarse to fine (Sec. 3.2,
 * Algorithm 2); at each level the nearest seed q's guide value is mapped to
 * a source pixel u* through a lookup table (Sec. 3.1), and p takes the source
 * coordinate u* + (p - q) as soon as the guide error there is below a
 * threshold.  A voting pass then averages, for every target pixel, the
 * co-located colours of the source patches around its neighbours' source
 * coordinates (end of Sec. 3.2).
 *
 * Conventions (all functions):
 *   - pointers marked [device] are HIP device pointers, [host] host pointers;
 *     the caller owns every buffer; the library allocates device memory only
 *     in sb_style_create (released by sb_style_destroy);
 *   - images are row-major; pixel p = (x, y), x the column; raster index
 *     y*W + x;
 *   - a guide has two interleaved channels, uint8 (SB_GUIDE_U8X2, 2 B/px) or
 *     uint16 (SB_GUIDE_U16X2, 4 B/px, native little-endian), or three uint8
 *     channels in 4 B/px (SB_GUIDE_U8X3: channels in bytes 0..2, byte 3
 *     ignored) -- the additional guiding channels of Sec. 3.1, e.g. a
 *     normal pair plus an appearance channel; or 2..8 channels of uint8
 *     (SB_GUIDE_U8XN) or uint16 (SB_GUIDE_U16XN) in texels of 4, 8 or 16
 *     bytes (sb_texel_bytes), channel k in element k, later elements
 *     ignored -- looked up by an exact search instead of a table;
 *   - source coordinates are packed x | (y << 16);
 *   - work is enqueued asynchronously on `stream` (0 = the null stream); the
 *     caller synchronises.  Arguments are validated before anything is
 *     enqueued: on an error code nothing has been written;
 *   - functions return sb_status codes and never throw; after SB_EHIP,
 *     sb_last_hip_error() names the HIP error (per calling thread).
 */
#ifndef STYLEBLIT_H
#define STYLEBLIT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SB_OK = 0,
    SB_EINVAL = -1,  /* bad argument; nothing enqueued */
    SB_ENOMEM = -2,  /* workspace too small, or a host allocation failed */
    SB_EHIP = -3,    /* a HIP call or launch failed; see sb_last_hip_error() */
    SB_EBUDGET = -4  /* serving: request larger than the memory budget */
} sb_status;

typedef enum {
    SB_GUIDE_U8X2 = 0,
    SB_GUIDE_U16X2 = 1,
    SB_GUIDE_U8X3 = 2,
    SB_GUIDE_U8XN = 3,   /* 2..8 uint8 channels, exact search (sb_style.channels) */
    SB_GUIDE_U16XN = 4   /* 2..8 uint16 channels, exact search */
} sb_guide_fmt;

/* Largest target and source side, and limits of the parameters. */
#define SB_MAX_SIDE 8192
#define SB_MAX_LEVELS 12
#define SB_MAX_RADIUS 7
#define SB_MAX_LUT_BITS 12
#define SB_MAX_LABELS 256
#define SB_MAX_CHANNELS 8

/* A style: the exemplar C_S, its guide G_S and the lookup table built from
 * G_S (Sec. 3.1).  A plain struct of caller-owned device pointers; it must
 * stay alive while work that reads it is in flight. */
typedef struct {
    const uint32_t *rgba;   /* [device] padded exemplar of sb_exemplar_texels(sw, sh)
                               texels, written by sb_pack_exemplar */
    const void *guide;      /* [device] Sw*Sh guide texels (2 or 4 B each, by fmt;
                               sb_texel_bytes for SB_GUIDE_U8XN / U16XN) */
    const uint32_t *lut;    /* [device] (1<<lut_bits)^2 source coordinates, bin index
                               c = c0 + (c1 << lut_bits); SB_GUIDE_U8X3: (1<<lut_bits)^3,
                               c = c0 + (c1 << lut_bits) + (c2 << 2*lut_bits); written
                               by sb_lut_build; not read (may be NULL) for
                               SB_GUIDE_U8XN / U16XN */
    int32_t sw, sh;         /* source size, 1..SB_MAX_SIDE */
    int32_t fmt;            /* sb_guide_fmt */
    int32_t lut_bits;       /* bits per channel of the lookup table: U8X2 and U8X3
                               1..8, U16X2 1..SB_MAX_LUT_BITS; 0 for U8XN / U16XN */
    /* Segmentation guide (optional; nlabels = 0 and NULLs without it): a
     * label per source pixel and one lookup table per label, so chunks stay
     * inside regions of equal label (the extra segmentation guide of the
     * paper's results section, read as a hard constraint: see
     * sb_stylize_seg). */
    const uint8_t *labels;      /* [device] Sw*Sh labels 0..nlabels-1 */
    const uint32_t *label_luts; /* [device] nlabels tables of (1<<lut_bits)^2 entries,
                                   written by sb_lut_build_labels */
    int32_t nlabels;            /* 0, or 1..SB_MAX_LABELS */
    /* Channel weights of a guide of three or more channels (the paper's
     * strong or weak appearance guide): the error and the lookup's argmin
     * sum w_k * d_k^2.  weights[k] in 0..127 for the guide's channels k
     * (SB_GUIDE_U8X3: 0..2); all zero means unit weights, the only choice
     * for two-channel table formats.  Tables must have been built with the
     * same weights (sb_lut_build_w). */
    uint8_t weights[8];
    /* SB_GUIDE_U8XN / U16XN only (0 / NULL otherwise): the number of
     * channels, 2..SB_MAX_CHANNELS, and the search tree over the source
     * guide written by sb_tree_build. */
    int32_t channels;
    const void *tree;       /* [device] sb_tree_bytes() bytes */
} sb_style;

/* Where the seed hierarchy's jitter comes from (SeedPoint in Algorithm 2
 * offsets each cell's seed by RandomJitterTable[b]; the paper leaves the
 * table's contents open).  Every mode gives integer jitter (jx, jy) in
 * [0, h)^2 for a cell b = (bx, by) of spacing h = 2^lg, and the seed
 * (h*bx + jx, h*by + jy):
 *   SB_JITTER_HASH   an integer hash of (cell, lg, seed), computed in the
 *                    kernels (no table is read).  With wrapping uint32
 *                    arithmetic, mix(x) = x ^= x >> 16; x *= 0x9E3779B9;
 *                    x ^= x >> 15; x *= 0x6A09E667; x ^= x >> 16, and
 *                    k = mix(mix(mix(mix(seed + 0xBB67AE85) ^ lg) ^ bx) ^ by),
 *                    jx = k & (h - 1), jy = (k >> 16) & (h - 1).  One 32-bit
 *                    seed per frame is the whole per-frame seed schedule of
 *                    an animation (Sec. 3.3).
 *   SB_JITTER_NONE   jx = jy = 0: seeds on the cell corners.
 *   SB_JITTER_TABLE  read from a caller-owned table (sb_jitter_len entries;
 *                    the `jitter` argument of the stylize calls), e.g. drawn
 *                    on the device by sb_jitter_fill. */
typedef enum { SB_JITTER_HASH = 0, SB_JITTER_NONE = 1, SB_JITTER_TABLE = 2 } sb_jitter;

/* Per-frame parameters of Algorithm 2 and of the voting blend. */
typedef struct {
    int32_t levels;         /* L, 0..SB_MAX_LEVELS; 0 = plain lookup (texture mapping) */
    int32_t finest;         /* spacing of the finest level, a power of two >= 1; level i
                               (0 = coarsest) has spacing finest << (L-1-i), at most
                               SB_MAX_SIDE.  The paper's hierarchy is finest = 2. */
    uint32_t threshold;     /* t: a level is accepted iff the exact squared L2 guide
                               error over all channels is < t (so t = 0 accepts
                               nothing) */
    int32_t radius;         /* r, 0..SB_MAX_RADIUS: voting window (2r+1)^2; 0 = copy */
    uint32_t seed;          /* jitter hash seed (SB_JITTER_HASH; per frame for animation) */
    int32_t jitter;         /* sb_jitter: where the seeds' jitter comes from */
} sb_params;

/* --------------------------------------------------------------- general */

const char *sb_version(void);
const char *sb_status_string(int status);
const char *sb_last_hip_error(void);

/* Entries of the jitter table of a W x H target (SB_JITTER_TABLE): level i
 * (coarsest first) has ceil(W/h_i) x ceil(H/h_i) cells, row-major; each entry
 * is jx | (jy << 16) with 0 <= jx, jy < h_i, and the cell's seed is
 * (h_i*cx + jx, h_i*cy + jy) (SeedPoint in Algorithm 2, whose
 * RandomJitterTable this is; the caller supplies it).  Returns -1 on invalid
 * arguments. */
int64_t sb_jitter_len(int32_t w, int32_t h, int32_t levels, int32_t finest);

/* Draw that table on the device from a counter-based generator, so the
 * per-frame seed schedule of an animation (Sec. 3.3: seeds re-drawn every
 * frame, or every few frames) needs no host random numbers: Philox4x64-10
 * (Salmon et al., SC 2011) under key (seed, stream_id); entry e takes word 0
 * of the block at counter (e, 0, 0, 0), jx = word mod h_i and
 * jy = (word >> 32) mod h_i.  jitter [device] sb_jitter_len() entries.
 * SB_EINVAL on invalid sizes (nothing enqueued); no work when L = 0. */
int sb_jitter_fill(int32_t w, int32_t h, int32_t levels, int32_t finest, uint64_t seed,
                   uint64_t stream_id, uint32_t *jitter, hipStream_t stream);

/* ------------------------------------------------- style registration */

/* Texels of the padded exemplar of an Sw x Sh source (0 on invalid sizes).
 * Layout: rows of Sw + 16 texels; source texel (x, y) at (y + 8) * (Sw + 16)
 * + (x + 8); an 8-texel zero margin on every side, then zero rows.  A texel
 * is R | G<<8 | B<<16 | A<<24 with A = 1 inside the source and 0 elsewhere,
 * so the blend's (2r+1)^2 gathers need no bounds checks and count their
 * in-source votes in A (the vote rule at the end of Sec. 3.2). */
size_t sb_exemplar_texels(int32_t sw, int32_t sh);

/* Write the padded exemplar (every texel, margins included) from 3 B/px RGB.
 * rgb [device] Sw*Sh*3; rgba [device] sb_exemplar_texels(sw, sh) texels. */
int sb_pack_exemplar(const uint8_t *rgb, int32_t sw, int32_t sh, uint32_t *rgba,
                     hipStream_t stream);

/* Device workspace needed by sb_lut_build. */
size_t sb_lut_workspace_bytes(int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits);

/* Build the guide-to-source lookup table of Sec. 3.1 on the device:
 *   LUT[c] = argmin_u |centre(c) - G_S[u]|^2, ties to the smallest raster
 *   index of u, where bin c = (c0, c1[, c2]) holds the guide values whose top
 *   lut_bits bits per channel are c0, c1[, c2] and centre(c) = (c << s) +
 *   2^(s-1) per channel for s = depth - lut_bits > 0, centre(c) = c for s = 0.
 *   With three channels this exact table stands in for the search tree the
 *   paper suggests for additional guiding channels (Sec. 3.1): same argmin,
 *   one load per query.
 * guide [device] Sw*Sh texels; lut [device] (1<<lut_bits)^2 entries, or
 * (1<<lut_bits)^3 for SB_GUIDE_U8X3 (64 MiB at 8 bits);
 * workspace [device] of at least sb_lut_workspace_bytes() bytes (8-bit
 * guides: about 2^(8*(channels-1)+lut_bits+4) bytes, 256 MiB for three
 * channels at 8 bits). */
int sb_lut_build(const void *guide, int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits,
                 uint32_t *lut, void *workspace, size_t workspace_bytes, hipStream_t stream);
/* The same with channel weights: LUT[c] = argmin_u sum_k w_k (centre_k(c) -
 * G_S[u]_k)^2, ties as above.  weights [host] three values 0..127 (NULL or
 * all zero: unit weights); non-unit weights need SB_GUIDE_U8X3. */
int sb_lut_build_w(const void *guide, int32_t fmt, int32_t sw, int32_t sh, int32_t lut_bits,
                   const uint8_t *weights, uint32_t *lut, void *workspace,
                   size_t workspace_bytes, hipStream_t stream);

/* A library-owned style in one call: copies the exemplar and its guide into
 * device memory the library allocates, packs the exemplar and builds the
 * exact lookup table of Sec. 3.1 (as sb_pack_exemplar + sb_lut_build), and
 * returns a style usable wherever an sb_style is taken.  Unit channel
 * weights, no labels.
 *   src_rgb    [device] Sw*Sh*3 bytes; src_guide [device] Sw*Sh texels of fmt;
 *              both may be freed once `stream` has been synchronised (this
 *              call synchronises it before returning)
 *   lut_bits   as sb_style.lut_bits (8 for 8-bit guides; 1..SB_MAX_LUT_BITS
 *              for SB_GUIDE_U16X2)
 *   out        [host] receives the style
 * Allocates with hipMalloc (the build workspace is freed before returning).
 * SB_EINVAL on bad arguments, SB_EHIP if an allocation or launch fails
 * (nothing is left allocated then). */
int sb_style_create(const uint8_t *src_rgb, const void *src_guide, int32_t sw, int32_t sh,
                    int32_t fmt, int32_t lut_bits, hipStream_t stream, sb_style **out);
/* Free a style from sb_style_create (only those), once no work that reads
 * it is in flight.  NULL is ignored. */
int sb_style_destroy(sb_style *style);

/* ----------------------------------------- guides of many channels (search)
 *
 * The additional guiding channels of Sec. 3.1, for which the paper suggests
 * a search tree in place of the table: SB_GUIDE_U8XN / SB_GUIDE_U16XN guides
 * of 2..8 channels, each lookup the exact nearest source pixel
 *   u*(g) = argmin_u sum_k w_k (g_k - G_S[u]_k)^2, ties to the smallest
 *   raster index of u,
 * over the raw channel values (no quantisation), with the style's weights.
 * The search runs on a k-d tree of the source guide built on the device:
 * every node holds the tight bounding box of its texels, inner nodes split
 * the widest (weighted) channel at the middle of the box, leaves hold at
 * most 8 texels (texels equal in every weighted channel collapse to the one
 * of smallest raster index), and a search skips a subtree only when its box
 * lies strictly farther than the best texel found, so the result is the
 * exact argmin for any tree shape.  Per frame: a seed pass searches each
 * seed's lookup (eight lanes per seed, over disjoint subtrees); the level
 * loop then runs as for the table formats, and a pass of its own searches
 * the own lookup of every pixel no level accepts (one thread per pixel,
 * starting from the nearest candidate its level loop measured); the vote is
 * unchanged.  Not available with labels.  In a batch (sb_batch_run) such
 * frames run through the per-frame kernels after the batch kernels, on the
 * same stream; sb_serve_run runs each such request alone on a slot. */

/* Bytes per texel of a `channels`-channel guide of fmt SB_GUIDE_U8XN or
 * SB_GUIDE_U16XN: the smallest of 4, 8, 16 that holds the channels; 0 if
 * the pair is invalid. */
int32_t sb_texel_bytes(int32_t fmt, int32_t channels);
/* Bytes of the search tree of an Sw x Sh source (an upper bound: the tree
 * has at most 2 Sw Sh - 1 nodes); 0 on invalid arguments. */
size_t sb_tree_bytes(int32_t fmt, int32_t channels, int32_t sw, int32_t sh);
/* Device workspace of sb_tree_build. */
size_t sb_tree_workspace_bytes(int32_t fmt, int32_t channels, int32_t sw, int32_t sh);
/* Build the search tree of a source guide.
 *   guide     [device] Sw*Sh texels of sb_texel_bytes(fmt, channels) bytes
 *   weights   [host] `channels` values 0..127 (NULL or all zero: unit); they
 *             steer the splits only -- the tree answers exactly for any
 *             weights, the style's weights decide the lookups
 *   tree      [device] sb_tree_bytes() bytes; workspace [device] of
 *             sb_tree_workspace_bytes()
 * Builds one tree level per round of launches and reads each level's node
 * count back, so it synchronises `stream` (and returns after the tree is
 * complete).  SB_EINVAL / SB_ENOMEM on bad arguments or small buffers,
 * SB_EHIP if a launch or copy fails. */
int sb_tree_build(const void *guide, int32_t fmt, int32_t channels, int32_t sw, int32_t sh,
                  const uint8_t *weights, void *tree, size_t tree_bytes, void *workspace,
                  size_t workspace_bytes, hipStream_t stream);
/* Exact lookups of n query texels through a style's tree:
 * out[i] = u*(queries[i]) as x | y << 16.  style: an SB_GUIDE_U8XN / U16XN
 * style (its weights apply); queries [device] n texels; out [device] n. */
int sb_tree_query(const sb_style *style, const void *queries, int64_t n, uint32_t *out,
                  hipStream_t stream);
/* A library-owned style of a many-channel guide in one call: copies the
 * exemplar and guide, packs the exemplar and builds the search tree, as
 * sb_style_create does for the table formats.  weights [host] `channels`
 * values 0..127 or NULL (unit); synchronises `stream`.  Free with
 * sb_style_destroy. */
int sb_style_create_n(const uint8_t *src_rgb, const void *src_guide, int32_t sw, int32_t sh,
                      int32_t fmt, int32_t channels, const uint8_t *weights, hipStream_t stream,
                      sb_style **out);

/* Per-label lookup tables for the segmentation guide: table l holds, for
 * every bin, the source pixel labelled l whose guide is nearest to the bin
 * centre (ties to the smallest raster index, as sb_lut_build); a label with
 * no source pixel gets the unconstrained table `lut` (from sb_lut_build).
 * guide [device] Sw*Sh texels; labels [device] Sw*Sh (values >= nlabels
 * belong to no table); lut [device] the unconstrained table; luts [device]
 * nlabels tables (each the size of `lut`), label-major; workspace [device]
 * of sb_lut_workspace_bytes(). */
int sb_lut_build_labels(const void *guide, const uint8_t *labels, int32_t fmt, int32_t sw,
                        int32_t sh, int32_t lut_bits, int32_t nlabels, const uint32_t *lut,
                        uint32_t *luts, void *workspace, size_t workspace_bytes,
                        hipStream_t stream);
/* The same with channel weights, as sb_lut_build_w (the unconstrained
 * table `lut` must use the same weights). */
int sb_lut_build_labels_w(const void *guide, const uint8_t *labels, int32_t fmt, int32_t sw,
                          int32_t sh, int32_t lut_bits, const uint8_t *weights, int32_t nlabels,
                          const uint32_t *lut, uint32_t *luts, void *workspace,
                          size_t workspace_bytes, hipStream_t stream);

/* -------------------------------------------------------- one frame */

/* Device workspace needed by sb_stylize for a W x H frame. */
size_t sb_workspace_bytes(int32_t w, int32_t h, const sb_params *params);

/* Stylise one frame (Algorithm 2 for every pixel, then the voting blend).
 *   style      [host] struct of device pointers, see sb_style
 *   tgt_guide  [device] W*H texels, same format as the style's guide
 *   jitter     [device] sb_jitter_len(W, H, L, finest) entries when
 *              params->jitter is SB_JITTER_TABLE; not read (may be NULL)
 *              with SB_JITTER_HASH or SB_JITTER_NONE
 *   out_rgb    [device] W*H*3 bytes: the stylised image C_T
 *   out_chunk  [device] W*H: chunk code (level << 26) | (qy << 13) | qx of the
 *              seed q whose chunk covers the pixel; level = L and q = p when
 *              no level accepted and the pixel took its own lookup
 *   out_nnf    [device, may be NULL] W*H source coordinates (x | y << 16)
 *   workspace  [device] at least sb_workspace_bytes() bytes
 * The output buffers must not overlap the inputs. */
int sb_stylize(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
               const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
               uint32_t *out_chunk, uint32_t *out_nnf, void *workspace, size_t workspace_bytes,
               hipStream_t stream);

/* Bytes of the library's static per-device scratch (40 MiB): the largest
 * sb_workspace_bytes() that sb_stylize_noalloc accepts, enough for a
 * 3840 x 2160 frame with finest spacing 8 (about 34.6 MB). */
#define SB_NOALLOC_SCRATCH_BYTES 41943040u

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): sb_stylize without the workspace argument, bit-identical to
 * it.  The seed table and offset map live in a static array of
 * SB_NOALLOC_SCRATCH_BYTES bytes that the library holds on every device it
 * runs on until the process ends; this call allocates nothing (no hipMalloc,
 * no hipFree).  Its device address is looked up on the first call on each
 * device, so the device current at the call must be the one `stream` runs
 * on.  Every call on one device shares that device's array and keeps the
 * last call's contents (nothing in it needs clearing: each call writes every
 * byte it reads before reading it), so calls whose work overlaps on one
 * device -- on two streams, or from two threads without ordering -- race
 * and must be serialised by the caller.
 * Returns SB_ENOMEM (with sb_last_hip_error() naming the sizes) when
 * sb_workspace_bytes(w, h, params) exceeds SB_NOALLOC_SCRATCH_BYTES,
 * SB_EINVAL as sb_stylize, SB_EHIP if the address lookup or a launch fails;
 * nothing is enqueued on an error. */
int sb_stylize_noalloc(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                       const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                       uint32_t *out_chunk, uint32_t *out_nnf, hipStream_t stream);
/* SB_NOALLOC_SCRATCH_BYTES, for bindings that cannot read the macro. */
size_t sb_noalloc_scratch_bytes(void);

/* Kernel choice.  Every choice computes the same result bit for bit; they
 * differ only in speed, so an autotuner may pick any.  0 in a field takes the
 * library's default.
 *   blend_ppt    pixels per thread of the voting pass, adjacent in a row: 2 or
 *                4 (default 4); each vote gather loads that many texels
 *   blend_rows   rows of the voting tile: 8 or 16 (default 16); the tile is
 *                (16 * blend_ppt) x blend_rows pixels, one thread per
 *                blend_ppt pixels
 *   level_group  levels of Algorithm 2 whose source-guide gathers are in
 *                flight together before their tests: 2 or 4 (default 2)
 *   level_ppt    pixels per thread of the level loop, i.e. 8x8 blocks per
 *                wave: 1, 2 (side by side) or 4 (2 x 2) (default 2); the
 *                blocks of a wave share the seed records they have in common
 *   blend_split  2: the voting pass copies the texel of every pixel group
 *                whose whole window holds one offset (their exact average)
 *                and votes the other groups from a per-tile list; 1: every
 *                group votes in place (default 2) */
typedef struct {
    int32_t blend_ppt;
    int32_t blend_rows;
    int32_t level_group;
    int32_t level_ppt;
    int32_t blend_split;
} sb_tune;

/* sb_stylize with an explicit kernel choice (tune may be NULL = defaults);
 * SB_EINVAL for an unsupported field value. */
int sb_stylize_ex(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                  const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                  uint32_t *out_chunk, uint32_t *out_nnf, void *workspace,
                  size_t workspace_bytes, const sb_tune *tune, hipStream_t stream);

/* sb_stylize_ex that also records events[0..3] (timing events, e.g. from
 * sb_timing_events_create) on `stream` before the seed-record pass, before
 * the level-loop pass, before the voting pass and after it, for per-pass
 * timing.  (Single frames of 8-bit two-channel styles without labels make
 * their seed records inside the level loop, with no seed pass: events 0 and
 * 1 are then recorded back to back.) */
int sb_stylize_timed(const sb_style *style, const void *tgt_guide, int32_t w, int32_t h,
                     const uint32_t *jitter, const sb_params *params, uint8_t *out_rgb,
                     uint32_t *out_chunk, uint32_t *out_nnf, void *workspace,
                     size_t workspace_bytes, const sb_tune *tune, hipEvent_t events[4],
                     hipStream_t stream);

/* sb_stylize_ex with the segmentation guide.  tgt_labels [device] W*H: the
 * target's label map; the style must carry labels (nlabels >= 1).  A seed q
 * takes its lookup from the table of its label L_T[q]; a level is accepted
 * only if, besides the error test, the transferred source pixel v carries
 * the pixel's label (L_S[v] == L_T[p]); a pixel no level accepts takes its
 * own lookup in the table of its label.  A label value >= nlabels selects
 * table nlabels-1 and is compared as is.  Voting is unchanged. */
int sb_stylize_seg(const sb_style *style, const void *tgt_guide, const uint8_t *tgt_labels,
                   int32_t w, int32_t h, const uint32_t *jitter, const sb_params *params,
                   uint8_t *out_rgb, uint32_t *out_chunk, uint32_t *out_nnf, void *workspace,
                   size_t workspace_bytes, const sb_tune *tune, hipStream_t stream);

/* Four timing events for sb_stylize_timed, created without the system-scope
 * fence (hipEventDisableSystemFence), so recording them
 * between passes adds no cache write-back or invalidation to the timed work.
 * The caller owns them and frees them with sb_timing_events_destroy. */
int sb_timing_events_create(hipEvent_t events[4]);
int sb_timing_events_destroy(hipEvent_t events[4]);
/* Milliseconds between two completed events (hipEventElapsedTime). */
int sb_event_elapsed_ms(hipEvent_t start, hipEvent_t stop, float *ms);

/* ------------------------------------------------------------- animation */

/* Frame-to-frame change of an animated sequence (Sec. 3.3, extension to
 * animation: seeds re-drawn per frame perturb the mosaic, and a larger
 * threshold t gives larger chunks and more change).  Counts, over n pixels
 * of two frames of the same size:
 *   counts[0]  pixels whose chunk code differs (chunk_a[i] != chunk_b[i]),
 *   counts[1]  pixels whose source coordinate differs (nnf_a[i] != nnf_b[i]);
 *              0 when nnf_a and nnf_b are both NULL.
 * chunk_a, chunk_b, nnf_a, nnf_b [device] n entries each, as written by
 *   sb_stylize (out_chunk, out_nnf); any alignment (16-byte aligned maps are
 *   read as vectors).
 * counts     [device, 8-byte aligned] 2 entries, written on `stream`.
 * workspace  [device, 8-byte aligned] at least sb_change_workspace_bytes().
 * n = 0 writes two zeros (the maps may then be NULL).  Returns SB_EINVAL
 * (null maps, only one NNF map, n < 0 or n > 2^40, misaligned
 * counts/workspace) or SB_ENOMEM (workspace too small) before enqueuing
 * anything. */
size_t sb_change_workspace_bytes(void);
int sb_frame_change(const uint32_t *chunk_a, const uint32_t *chunk_b, const uint32_t *nnf_a,
                    const uint32_t *nnf_b, int64_t n, uint64_t *counts, void *workspace,
                    size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- batches */

/* One frame of a batch: the arguments of sb_stylize for that frame. */
typedef struct {
    const sb_style *style;      /* [host] */
    const void *tgt_guide;      /* [device] W*H texels in the style's format */
    const uint32_t *jitter;     /* [device] sb_jitter_len() entries (SB_JITTER_TABLE only;
                                   may be NULL otherwise) */
    int32_t w, h;
    sb_params params;
    uint8_t *out_rgb;           /* [device] W*H*3 */
    uint32_t *out_chunk;        /* [device] W*H */
    uint32_t *out_nnf;          /* [device, may be NULL] W*H */
    const uint8_t *tgt_labels;  /* [device, may be NULL] W*H target labels: the frame
                                   runs as sb_stylize_seg (the style must carry labels) */
} sb_frame;

typedef struct sb_batch sb_batch;  /* opaque: descriptor buffers and captured graphs */

/* Most frames per batch run. */
int32_t sb_batch_max_frames(void);
/* Bytes of the descriptor buffers a plan needs, both on the device and in
 * pinned host memory (two halves, used alternately by successive runs). */
size_t sb_batch_desc_bytes(void);
/* Device workspace for running these frames as one batch (0 if invalid). */
size_t sb_batch_workspace_bytes(const sb_frame *frames, int32_t n);

/* A batch plan.  desc_dev [device] and desc_host [host, pinned, e.g. from
 * hipHostMalloc] of sb_batch_desc_bytes() each stay owned by the caller and
 * must outlive the plan.  With use_graph != 0 the plan captures, once, two
 * hipGraphs on `stream` (which must not be the null stream): the upload of
 * one descriptor half followed by persistent kernels (seed records,
 * per-pixel level loop, voting for radius 0..3 and for 4..7) that stride
 * over the concatenated tiles of all frames of the batch.  The graphs hold
 * no shapes, so they serve every later batch.  With use_graph == 0 each run
 * enqueues the upload and the same kernels directly, each with an exact
 * grid (one workgroup per tile of the batch, no persistent loop), so batches
 * on several streams interleave on the device as separate frames would.
 * tune (may be NULL) fixes the kernel choice of every run; blocks_per_cu
 * (0 = 8, else 1..16) sets the persistent grid of the graphs to that many
 * blocks per compute unit. */
int sb_batch_create(void *desc_dev, void *desc_host, int32_t use_graph, const sb_tune *tune,
                    int32_t blocks_per_cu, hipStream_t stream, sb_batch **out);
/* Stylise n frames (1..sb_batch_max_frames()) with one graph launch on
 * `stream` (frames of many-channel styles follow it through the per-frame
 * kernels); the results equal n separate sb_stylize calls bit for bit.
 * Validates every frame first (SB_EINVAL / SB_ENOMEM and nothing enqueued
 * on a bad argument).  Blocks only while the run two calls back still reads
 * the descriptor half this run reuses.  workspace [device] of at least
 * sb_batch_workspace_bytes() bytes, not shared with a run still in flight. */
int sb_batch_run(sb_batch *b, const sb_frame *frames, int32_t n, void *workspace,
                 size_t workspace_bytes, hipStream_t stream);
/* Wait for the plan's runs, then release its graphs and events. */
int sb_batch_destroy(sb_batch *b);

/* The per-frame alternative to a batch: the n frames one after another on
 * `stream`, each through the per-frame kernels exactly as sb_stylize_ex (or
 * sb_stylize_seg for frames with target labels) would run it, from one
 * call.  They share workspace [device], which must hold the largest frame's
 * sb_workspace_bytes().  Every frame is validated before anything is
 * enqueued (SB_EINVAL / SB_ENOMEM); SB_EHIP if a launch fails. */
int sb_stylize_frames(const sb_frame *frames, int32_t n, void *workspace,
                      size_t workspace_bytes, const sb_tune *tune, hipStream_t stream);

/* ---------------------------------------------------------------- serving */

/* Device bytes a request's outputs take from the serving arena. */
size_t sb_frame_bytes(int32_t w, int32_t h);

typedef struct {
    int32_t slots;      /* batches in flight, each on its own stream, 1..8 */
    int32_t max_batch;  /* frames per batch, 1..sb_batch_max_frames() */
    int32_t use_graph;  /* batches as graph replays (1) or direct launches (0) */
    int32_t plain;      /* 1: no batching; every request is its own sb_stylize on one
                           stream, in arrival order (the per-request baseline) */
    void *arena;        /* [device] outputs of requests in flight are carved from here:
                           its size is the memory budget for admission */
    size_t arena_bytes;
    void *desc_dev;     /* [device] slots * sb_batch_desc_bytes() (unused when plain) */
    void *desc_host;    /* [host, pinned] slots * sb_batch_desc_bytes() (unused when plain) */
    void *workspace;    /* [device] slots * workspace_bytes_per_slot */
    size_t workspace_bytes_per_slot;  /* >= max_batch * (sb_workspace_bytes + 256) of the
                                         largest request */
    sb_tune tune;       /* kernel choice of every launch (zeros = defaults) */
    int32_t blocks_per_cu;  /* batch plans' persistent grid, as in sb_batch_create */
} sb_serve_config;

typedef struct {
    double arrival_s;           /* arrival time, seconds after the run starts; sorted */
    const sb_style *style;      /* [host] resident style */
    const void *tgt_guide;      /* [device] */
    const uint32_t *jitter;     /* [device] jitter table (SB_JITTER_TABLE only; may be
                                   NULL otherwise) */
    int32_t w, h;
    sb_params params;
    uint8_t *out_rgb;           /* [device] or NULL: taken from the arena on admission and
                                   released at completion */
    uint32_t *out_chunk;        /* [device] or NULL (with out_rgb) */
    uint32_t *out_nnf;          /* [device] or NULL: source coordinates, as in sb_stylize */
    int32_t session;            /* >= 0: a frame of an animated sequence; frames of one
                                   session complete in arrival order (a later frame's
                                   kernels wait for the earlier frame's batch when it runs
                                   on another slot).  < 0: independent request */
    const uint8_t *tgt_labels;  /* [device] or NULL: W*H target labels, the frame runs with
                                   the segmentation guide (the style must carry labels) */
} sb_request;

typedef struct {
    double admitted_s, launched_s, completed_s;  /* seconds after the run starts, host
                                                    clock; completion as seen by polling */
    int32_t batch, slot, batch_size;
    int32_t status;             /* SB_OK, or SB_EBUDGET if it can never fit the arena */
} sb_request_result;

/* Run a request trace in real time on the calling thread: arrivals at their
 * times, admission in arrival order while the outputs fit in the arena,
 * frames of one session completing in order,
 * continuous batching over `slots` streams (a free slot takes every admitted
 * request up to max_batch and runs them as one batch-plan replay, or, for a
 * single request, as one sb_stylize_ex on the slot's stream; a request of a
 * many-channel style always runs alone that way), completion by event
 * polling.  Every result is
 * the one sb_stylize gives for that request alone.  Returns after the last
 * request finished and the slots' streams drained. */
int sb_serve_run(const sb_serve_config *cfg, const sb_request *reqs, int32_t n,
                 sb_request_result *res);

#ifdef __cplusplus
}
#endif
#endif /* STYLEBLIT_H */
