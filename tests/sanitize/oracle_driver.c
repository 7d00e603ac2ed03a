/* Sanitizer driver for the CPU oracle: exercises every exported oracle
 * function on small random and ragged inputs (all guide formats, labels,
 * table and hash jitter, every radius, level counts, finest spacings and
 * frame shapes smaller than the coarsest cell) so that an AddressSanitizer /
 * UndefinedBehaviorSanitizer build reports any out-of-bounds access, use of
 * freed memory, overflow or misaligned access.  Exit code 0 when every call
 * returned its documented status.  Test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int ora_lut_build_w(const void *, int, int, int, int, const uint8_t *, uint32_t *);
int ora_lut_build(const void *, int, int, int, int, uint32_t *);
int ora_lut_query_w(const void *, int, int, int, int, const uint8_t *, const int64_t *, int64_t,
                    uint32_t *);
int ora_lut_query_sweep_w(const void *, int, int, int, int, const uint8_t *, const int64_t *,
                          int64_t, uint32_t *);
int ora_lut_build_labels_w(const void *, const uint8_t *, int, int, int, int, int,
                           const uint8_t *, uint32_t *);
int64_t ora_jitter_len(int, int, int, int);
int ora_jitter_fill(int, int, int, int, uint64_t, uint64_t, uint32_t *);
int ora_jitter_hash(int, int, int, int, uint32_t, uint32_t *);
int ora_nearest_seed(int, int, int, int, const uint32_t *, int, int64_t, int64_t, int64_t *,
                     int64_t *);
int ora_stylize_w(const uint8_t *, const void *, int, int, const uint32_t *, int, int,
                  const uint8_t *, const void *, int, int, const uint32_t *, int, int, uint32_t,
                  int, uint8_t *, uint32_t *, uint32_t *);
int ora_stylize_seg_w(const uint8_t *, const void *, const uint8_t *, int, int, const uint32_t *,
                      int, int, int, const uint8_t *, const void *, const uint8_t *, int, int,
                      const uint32_t *, int, int, uint32_t, int, uint8_t *, uint32_t *,
                      uint32_t *);
int ora_blend(const uint8_t *, int, int, const uint32_t *, int, int, int, uint8_t *, int64_t,
              int64_t);
int ora_set_threads(int);
int ora_texel_bytes(int, int);
int ora_nn_query_n(const void *, int, int, int, int, const uint8_t *, const void *, int64_t,
                   uint32_t *);
int ora_nn_sweep_n(const void *, int, int, int, int, const uint8_t *, const void *, int64_t,
                   uint32_t *);
int ora_stylize_n(const uint8_t *, const void *, int, int, int, int, const uint8_t *,
                  const void *, int, int, const uint32_t *, int, int, uint32_t, int, uint8_t *,
                  uint32_t *, uint32_t *);

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next32(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (uint32_t)(rng >> 16);
}

/* exact-size heap blocks, so any read past the end is caught */
static void *fill_random(size_t bytes) {
  uint8_t *p = (uint8_t *)malloc(bytes ? bytes : 1);
  for (size_t i = 0; i < bytes; ++i) p[i] = (uint8_t)next32();
  return p;
}

static int failures = 0;
#define EXPECT(call, want)                                                       \
  do {                                                                           \
    int rc_ = (call);                                                            \
    if (rc_ != (want)) {                                                         \
      fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__, __LINE__, \
              #call, rc_, (want));                                               \
      ++failures;                                                                \
    }                                                                            \
  } while (0)

static size_t texel_bytes(int fmt) { return fmt == 0 ? 2 : 4; }

/* One style (source guide, exemplar, weights and its table). */
typedef struct {
  int fmt, lut_bits, sw, sh;
  void *sg;
  uint8_t *srgb;
  uint8_t weights[4];
  uint32_t *lut;
  size_t bins;
} style_t;

static void style_make(style_t *S, int fmt, int lut_bits, int sw, int sh) {
  const int ch = fmt == 2 ? 3 : 2;
  S->fmt = fmt;
  S->lut_bits = lut_bits;
  S->sw = sw;
  S->sh = sh;
  S->bins = (size_t)1 << (ch * lut_bits);
  S->sg = fill_random((size_t)sw * sh * texel_bytes(fmt));
  S->srgb = (uint8_t *)fill_random((size_t)sw * sh * 3);
  memset(S->weights, 0, sizeof S->weights);
  if (fmt == 2) {
    S->weights[0] = 1 + next32() % 127;
    S->weights[1] = next32() % 128;
    S->weights[2] = 1 + next32() % 127;
  }
  S->lut = (uint32_t *)malloc(S->bins * 4);
  EXPECT(ora_lut_build_w(S->sg, fmt, sw, sh, lut_bits, fmt == 2 ? S->weights : NULL, S->lut), 0);
  int64_t q[5] = {0, (int64_t)S->bins - 1, (int64_t)S->bins / 2, 1, (int64_t)S->bins / 3};
  uint32_t qo[5], qs[5];
  EXPECT(ora_lut_query_w(S->sg, fmt, sw, sh, lut_bits, fmt == 2 ? S->weights : NULL, q, 5, qo),
         0);
  EXPECT(ora_lut_query_sweep_w(S->sg, fmt, sw, sh, lut_bits, fmt == 2 ? S->weights : NULL, q, 5,
                               qs),
         0);
}

static void style_free(style_t *S) {
  free(S->sg);
  free(S->srgb);
  free(S->lut);
}

static void one_case(const style_t *S, int w, int h, int levels, int finest, uint32_t t,
                     int radius, int use_hash, int nlabels) {
  const int fmt = S->fmt, lut_bits = S->lut_bits, sw = S->sw, sh = S->sh;
  const size_t bins = S->bins;
  void *sg = S->sg;
  uint8_t *srgb = S->srgb;
  const uint8_t *weights = S->weights;
  const uint32_t *lut = S->lut;
  void *tg = fill_random((size_t)w * h * texel_bytes(fmt));
  const int64_t nj = ora_jitter_len(w, h, levels, finest);
  if (nj < 0) {
    ++failures;
    fprintf(stderr, "jitter_len %dx%d L=%d f=%d failed\n", w, h, levels, finest);
    return;
  }
  uint32_t *jit = (uint32_t *)malloc((size_t)(nj ? nj : 1) * 4);
  if (use_hash)
    EXPECT(ora_jitter_hash(w, h, levels, finest, next32(), jit), 0);
  else
    EXPECT(ora_jitter_fill(w, h, levels, finest, next32(), next32() % 4, jit), 0);
  for (int l = 0; l < levels; ++l) {
    const int64_t probe[4][2] = {{0, 0}, {w - 1, h - 1}, {w / 2, 0}, {0, h - 1}};
    for (int k = 0; k < 4; ++k) {
      int64_t qx, qy;
      ora_nearest_seed(w, h, levels, finest, jit, l, probe[k][0], probe[k][1], &qx, &qy);
    }
  }
  uint8_t *out_rgb = (uint8_t *)malloc((size_t)w * h * 3);
  uint32_t *chunk = (uint32_t *)malloc((size_t)w * h * 4);
  uint32_t *nnf = (uint32_t *)malloc((size_t)w * h * 4);
  EXPECT(ora_stylize_w(srgb, sg, sw, sh, lut, fmt, lut_bits, fmt == 2 ? weights : NULL, tg, w, h,
                       jit, levels, finest, t, radius, out_rgb, chunk, nnf),
         0);
  /* the vote alone over two row bands of the frame (out_rgb is the whole
     frame: bands write their own rows), the second ending at the last row */
  EXPECT(ora_blend(srgb, sw, sh, nnf, w, h, radius, out_rgb, 0, h / 2), 0);
  EXPECT(ora_blend(srgb, sw, sh, nnf, w, h, radius, out_rgb, h / 2, h - h / 2), 0);
  if (nlabels > 0) {
    uint8_t *sl = (uint8_t *)malloc((size_t)sw * sh);
    uint8_t *tl = (uint8_t *)malloc((size_t)w * h);
    for (int i = 0; i < sw * sh; ++i) sl[i] = (uint8_t)(next32() % nlabels);
    /* target labels may exceed the source's: they select the last table */
    for (int i = 0; i < w * h; ++i) tl[i] = (uint8_t)(next32() % (nlabels + 1));
    uint32_t *luts = (uint32_t *)malloc(bins * 4 * (size_t)nlabels);
    EXPECT(ora_lut_build_labels_w(sg, sl, nlabels, fmt, sw, sh, lut_bits,
                                  fmt == 2 ? weights : NULL, luts),
           0);
    EXPECT(ora_stylize_seg_w(srgb, sg, sl, sw, sh, luts, nlabels, fmt, lut_bits,
                             fmt == 2 ? weights : NULL, tg, tl, w, h, jit, levels, finest, t,
                             radius, out_rgb, chunk, nnf),
           0);
    free(sl);
    free(tl);
    free(luts);
  }
  free(tg);
  free(jit);
  free(out_rgb);
  free(chunk);
  free(nnf);
}

int main(void) {
  ora_set_threads(1);
  const int shapes[][4] = {{19, 13, 37, 23}, {8, 8, 8, 8}, {5, 31, 3, 17},
                           {33, 7, 41, 1}, {1, 1, 9, 5}, {16, 16, 64, 40}};
  for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
    for (int fmt = 0; fmt < 3; ++fmt) {
      style_t S;
      /* coarse tables keep the ring searches short on these sparse
         sources; the full 8-bit table runs once on the densest source */
      const int lut_bits = (fmt == 0 && s == 5) ? 8 : fmt == 2 ? 3 : 5;
      style_make(&S, fmt, lut_bits, shapes[s][0], shapes[s][1]);
      for (int levels = 0; levels <= 3; ++levels) {
        const int finest = 1 << (next32() % 4);
        const int radius = (int)(next32() % 4);
        const uint32_t t = next32() % 3 == 0 ? 0u : next32() % 4000;
        one_case(&S, shapes[s][2], shapes[s][3], levels, finest, t, radius,
                 (levels + (int)s) & 1, (levels == 2) ? 3 : 0);
      }
      style_free(&S);
    }
  }
  /* guides of many channels: every depth and channel count, exact-size
     texel buffers, lookups and whole frames */
  for (int depth = 8; depth <= 16; depth += 8) {
    for (int ch = 2; ch <= 8; ++ch) {
      const int tb = ora_texel_bytes(depth, ch);
      const int sw = 3 + (int)(next32() % 20), sh = 1 + (int)(next32() % 12);
      const int w = 1 + (int)(next32() % 40), h = 1 + (int)(next32() % 24);
      uint8_t *sg = fill_random((size_t)sw * sh * tb);
      uint8_t *srgb = fill_random((size_t)sw * sh * 3);
      uint8_t *tg = fill_random((size_t)w * h * tb);
      uint8_t *wts = fill_random(8);
      for (int k = 0; k < 8; ++k) wts[k] &= 127;
      uint32_t *qo = (uint32_t *)malloc((size_t)w * h * 4);
      uint32_t *qs = (uint32_t *)malloc((size_t)w * h * 4);
      EXPECT(ora_nn_query_n(sg, depth, ch, sw, sh, wts, tg, (int64_t)w * h, qo), 0);
      EXPECT(ora_nn_sweep_n(sg, depth, ch, sw, sh, wts, tg, (int64_t)w * h, qs), 0);
      if (memcmp(qo, qs, (size_t)w * h * 4) != 0) {
        fprintf(stderr, "sweep differs from brute force (depth %d, %d channels)\n", depth, ch);
        ++failures;
      }
      const int levels = (int)(next32() % 4), finest = 1 << (next32() % 3);
      const int64_t nj = ora_jitter_len(w, h, levels, finest);
      uint32_t *jit = (uint32_t *)malloc((size_t)(nj > 0 ? nj : 1) * 4);
      EXPECT(ora_jitter_hash(w, h, levels, finest, next32(), jit), 0);
      uint8_t *out_rgb = (uint8_t *)malloc((size_t)w * h * 3);
      uint32_t *chunk = (uint32_t *)malloc((size_t)w * h * 4);
      uint32_t *nnf = (uint32_t *)malloc((size_t)w * h * 4);
      EXPECT(ora_stylize_n(srgb, sg, sw, sh, depth, ch, (ch & 1) ? wts : NULL, tg, w, h, jit,
                           levels, finest, next32() % 5000, (int)(next32() % 4), out_rgb, chunk,
                           nnf),
             0);
      free(sg); free(srgb); free(tg); free(wts); free(qo); free(qs); free(jit);
      free(out_rgb); free(chunk); free(nnf);
    }
  }
  if (ora_texel_bytes(8, 9) != 0 || ora_texel_bytes(10, 3) != 0) {
    fprintf(stderr, "bad many-channel layout accepted\n");
    ++failures;
  }
  /* invalid arguments are refused without touching memory */
  uint32_t dummy = 0;
  if (ora_lut_build(&dummy, 7, 1, 1, 8, &dummy) == 0) {
    fprintf(stderr, "bad format accepted\n");
    ++failures;
  }
  if (ora_blend((const uint8_t *)&dummy, 1, 1, &dummy, 1, 1, 17, (uint8_t *)&dummy, 0, 1) == 0) {
    fprintf(stderr, "radius 17 accepted\n");
    ++failures;
  }
  printf("oracle sanitizer driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
