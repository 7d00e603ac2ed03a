/*
 * styleblit_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU oracle for StyleBlit's per-pixel guided
 * chunk transfer (Sykora et al., "StyleBlit: Fast Example-Based Stylization
 * with Local Guidance", EGSR 2018): the guide-to-source lookup table of
 * Sec. 3.1, the seed hierarchy and per-pixel level loop of Sec. 3.2
 * (Algorithm 2, ParallelStyleBlit, with its SeedPoint and NearestSeed
 * functions), and the coordinate-transfer-plus-voting blend at the end of
 * Sec. 3.2.  It exists only to check the HIP library.  Only tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never does.  It shares no code with the HIP library.
 *
 * Readings of points the paper leaves open (all integer, so the result is
 * unique):
 *   - guide error and threshold: exact squared L2 over the two guide
 *     channels, accepted iff error < t (strict, as in both algorithms);
 *   - level spacings h_i = finest << (L-1-i), level 0 coarsest (the paper's
 *     2^l, l = L..1, is finest = 2);
 *   - RandomJitterTable: one integer jitter (jx, jy) in [0,h)^2 per cell and
 *     level, passed in as a table: defined by an integer hash of (cell,
 *     log2 h, seed) (ora_jitter_hash), drawn from Philox4x64-10
 *     (ora_jitter_fill), or all zero (seeds on the cell corners);
 *     SeedPoint(b) = h*b + j, the integer form of floor(h*(b + j/h));
 *   - seeds outside the target are not candidates; a level whose 3x3
 *     neighbourhood holds no in-image seed is skipped;
 *   - NearestSeed scans x outer, y inner over {-1,0,1} and keeps the first
 *     strict minimum of the squared distance;
 *   - the lookup table maps a (quantised) guide value to the source pixel
 *     whose guide is nearest to the bin centre, ties to the smallest raster
 *     index;
 *   - a transferred coordinate that falls outside the source rejects the
 *     level;
 *   - no level accepted: fall back to the pixel's own lookup (the spacing-1
 *     level, where SeedPoint(p) = p), accepted unconditionally;
 *   - voting: square (2r+1)^2 window of uniform weight over target pixels n;
 *     n votes with the source pixel NNF[n] + (p - n) when that lies in the
 *     source; per channel (sum + floor(k/2)) / k in integers.
 *
 * Segmentation guide (the extra guide of Sec. 4 that keeps chunks inside
 * semantic regions), read as a hard constraint:
 *   - a uint8 label per source pixel and per target pixel, labels
 *     0..nlabels-1 (a larger value selects table nlabels-1 and is compared
 *     as is);
 *   - one lookup table per label over the source pixels of that label
 *     (ties as above); a label with no source pixel uses the unconstrained
 *     table;
 *   - a seed q looks up u* in the table of its own label L_T[q];
 *   - a level is accepted only if, besides the error test, the transferred
 *     source pixel carries the pixel's label: L_S[v] == L_T[p];
 *   - the fallback is the pixel's own lookup in the table of its label.
 *
 * More than two guide channels (the additional guiding channels of Sec. 3.1,
 * for which the paper suggests a search tree; here the same exact argmin,
 * tabulated): fmt 2 holds three uint8 channels in 4 bytes per pixel (byte 3
 * ignored).  The error sums the three squared differences; the table has
 * (1 << lut_bits)^3 bins indexed c0 + (c1 << b) + (c2 << 2b) and is built by
 * brute force over every source pixel (the definition: nearest to the bin
 * centre, ties to the smallest raster index).  Optional integer channel
 * weights w0..w2 (0..127; the paper's strong or weak appearance guide) scale
 * each channel's squared difference, in the table's argmin and in the
 * error alike: e = sum_k w_k (a_k - b_k)^2.  Unit weights are the plain
 * case; two-channel formats take unit weights only.
 *
 * Guides of 2..8 channels of 8 or 16 bits (fmt 3 and 4, at the end of this
 * file) take the search the paper suggests literally, as an exact one: each
 * lookup is the nearest source pixel over the raw channel values (no
 * table, no quantisation), ties to the smallest raster index, with optional
 * channel weights 0..127.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ENOMEM (-2)

/* ------------------------------------------------------------------ guides */

/* Read the two guide channels of pixel `idx` (raster index). fmt 0: uint8,
 * fmt 1: uint16 (fmt 2 reads its first two channels here). */
static void guide_read(const void *g, int fmt, int64_t idx, int64_t *c0, int64_t *c1)
{
    if (fmt == 0) {
        const uint8_t *p = (const uint8_t *)g;
        *c0 = p[2 * idx];
        *c1 = p[2 * idx + 1];
    } else if (fmt == 1) {
        const uint16_t *p = (const uint16_t *)g;
        *c0 = p[2 * idx];
        *c1 = p[2 * idx + 1];
    } else {
        const uint8_t *p = (const uint8_t *)g;
        *c0 = p[4 * idx];
        *c1 = p[4 * idx + 1];
    }
}

/* Number of guide channels of a format. */
static int guide_channels(int fmt) { return fmt == 2 ? 3 : 2; }

/* Every channel of pixel `idx`: c[0..guide_channels(fmt)-1]. */
static void guide_read_all(const void *g, int fmt, int64_t idx, int64_t *c)
{
    guide_read(g, fmt, idx, &c[0], &c[1]);
    if (fmt == 2) c[2] = ((const uint8_t *)g)[4 * idx + 2];
}

static int guide_depth(int fmt) { return fmt == 1 ? 16 : 8; }

static int fmt_ok(int fmt) { return fmt == 0 || fmt == 1 || fmt == 2; }

/* Channel weights: NULL = unit; otherwise three values 0..127, and only for
 * three-channel guides (two-channel guides take unit weights).  Fills w[3]. */
static int weights_get(int fmt, const uint8_t *weights, int64_t *w)
{
    w[0] = w[1] = w[2] = 1;
    if (!weights) return ORA_OK;
    for (int k = 0; k < 3; ++k) {
        if (weights[k] > 127) return ORA_EINVAL;
        w[k] = weights[k];
    }
    if (fmt != 2 && (w[0] != 1 || w[1] != 1 || w[2] != 1)) return ORA_EINVAL;
    return ORA_OK;
}

/* Lookup-table bin of one guide channel value: drop the low bits. */
static int64_t lut_quantise(int64_t v, int fmt, int lut_bits)
{
    return v >> (guide_depth(fmt) - lut_bits);
}

/* Guide value at the centre of bin c of one channel. */
static int64_t lut_bin_centre(int64_t c, int fmt, int lut_bits)
{
    int s = guide_depth(fmt) - lut_bits;
    return s == 0 ? c : (c << s) + ((int64_t)1 << (s - 1));
}

/* ---------------------------------------------------- lookup table (Sec. 3.1)
 *
 * LUT[c] = argmin_u |centre(c) - G_S[u]|^2, ties to the smallest raster index
 * of u.  Computed by a ring search over a bucket grid equal to the LUT grid:
 * after the buckets at Chebyshev distance <= k around c have been visited,
 * every unvisited source pixel lies at squared distance >= LB(k+1) from the
 * centre, so the search may stop as soon as best < LB(k+1).  (Equality must
 * continue: a later ring may hold an equally near pixel with a smaller raster
 * index.)
 */
/* The table over the source pixels whose label is `want` (labels NULL: all
 * pixels).  Returns ORA_OK, or 1 when no source pixel qualifies (lut left
 * untouched). */
/* Three channels: every bin by brute force over every qualifying source
 * pixel, in raster order with a strict compare (so ties keep the smallest
 * raster index).  Returns 1 when no source pixel qualifies. */
static int lut_build3_filtered(const void *src_guide, const uint8_t *labels, int want, int sw,
                               int sh, int lut_bits, const int64_t *w, uint32_t *lut)
{
    const int64_t n = (int64_t)1 << lut_bits, npix = (int64_t)sw * sh;
    int64_t any = 0;
    for (int64_t i = 0; i < npix && !any; ++i) any = !labels || labels[i] == want;
    if (!any) return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < n * n * n; ++c) {
        const int64_t q[3] = {lut_bin_centre(c % n, 2, lut_bits),
                              lut_bin_centre((c / n) % n, 2, lut_bits),
                              lut_bin_centre(c / (n * n), 2, lut_bits)};
        uint64_t best_d = UINT64_MAX;
        int64_t best_i = -1;
        for (int64_t i = 0; i < npix; ++i) {
            if (labels && labels[i] != want) continue;
            int64_t g[3];
            guide_read_all(src_guide, 2, i, g);
            uint64_t d = 0;
            for (int k = 0; k < 3; ++k) d += (uint64_t)(w[k] * (q[k] - g[k]) * (q[k] - g[k]));
            if (d < best_d) {
                best_d = d;
                best_i = i;
            }
        }
        lut[c] = (uint32_t)(best_i % sw) | ((uint32_t)(best_i / sw) << 16);
    }
    return ORA_OK;
}

static int lut_build_filtered(const void *src_guide, const uint8_t *labels, int want, int fmt,
                              int sw, int sh, int lut_bits, const int64_t *wt, uint32_t *lut)
{
    if (!src_guide || !lut || sw < 1 || sh < 1 || !fmt_ok(fmt)) return ORA_EINVAL;
    if (fmt == 2) {
        if (lut_bits < 1 || lut_bits > 8) return ORA_EINVAL;
        return lut_build3_filtered(src_guide, labels, want, sw, sh, lut_bits, wt, lut);
    }
    if (lut_bits < 1 || lut_bits > guide_depth(fmt) || lut_bits > 12) return ORA_EINVAL;
    const int64_t n = (int64_t)1 << lut_bits;          /* bins per channel */
    const int64_t w = (int64_t)1 << (guide_depth(fmt) - lut_bits); /* bin width */
    const int64_t npix = (int64_t)sw * sh;

    /* counting sort of the source pixels into buckets, raster order kept */
    int64_t *start = (int64_t *)calloc((size_t)(n * n + 1), sizeof(int64_t));
    int64_t *list = (int64_t *)malloc((size_t)npix * sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc((size_t)(n * n) * sizeof(int64_t));
    if (!start || !list || !fill) { free(start); free(list); free(fill); return ORA_ENOMEM; }
    for (int64_t i = 0; i < npix; ++i) {
        if (labels && labels[i] != want) continue;
        int64_t g0, g1;
        guide_read(src_guide, fmt, i, &g0, &g1);
        int64_t b = lut_quantise(g1, fmt, lut_bits) * n + lut_quantise(g0, fmt, lut_bits);
        start[b + 1]++;
    }
    for (int64_t b = 0; b < n * n; ++b) start[b + 1] += start[b];
    if (start[n * n] == 0) { free(start); free(list); free(fill); return 1; }
    memcpy(fill, start, (size_t)(n * n) * sizeof(int64_t));
    for (int64_t i = 0; i < npix; ++i) {
        if (labels && labels[i] != want) continue;
        int64_t g0, g1;
        guide_read(src_guide, fmt, i, &g0, &g1);
        int64_t b = lut_quantise(g1, fmt, lut_bits) * n + lut_quantise(g0, fmt, lut_bits);
        list[fill[b]++] = i;
    }

    for (int64_t cy = 0; cy < n; ++cy) {
        for (int64_t cx = 0; cx < n; ++cx) {
            const int64_t qx = lut_bin_centre(cx, fmt, lut_bits);
            const int64_t qy = lut_bin_centre(cy, fmt, lut_bits);
            uint64_t best_d = UINT64_MAX;
            int64_t best_i = -1;
            for (int64_t k = 0;; ++k) {
                int any = 0;
                for (int64_t by = cy - k; by <= cy + k; ++by) {
                    if (by < 0 || by >= n) continue;
                    /* on the ring: full rows at the top and bottom, two
                     * columns in between */
                    int64_t step = (by == cy - k || by == cy + k) ? 1 : 2 * k;
                    if (step == 0) step = 1;
                    for (int64_t bx = cx - k; bx <= cx + k; bx += step) {
                        if (bx < 0 || bx >= n) continue;
                        any = 1;
                        int64_t b = by * n + bx;
                        for (int64_t e = start[b]; e < start[b + 1]; ++e) {
                            int64_t i = list[e], g0, g1;
                            guide_read(src_guide, fmt, i, &g0, &g1);
                            uint64_t d = (uint64_t)((qx - g0) * (qx - g0)) +
                                         (uint64_t)((qy - g1) * (qy - g1));
                            if (d < best_d || (d == best_d && i < best_i)) {
                                best_d = d;
                                best_i = i;
                            }
                        }
                    }
                }
                if (!any) break; /* the ring left the grid on every side */
                int64_t lb = (k + 1) * w - w / 2;
                if (best_i >= 0 && best_d < (uint64_t)(lb * lb)) break;
            }
            lut[cy * n + cx] = (uint32_t)(best_i % sw) | ((uint32_t)(best_i / sw) << 16);
        }
    }
    free(start);
    free(list);
    free(fill);
    return ORA_OK;
}

/* Threads of the OpenMP loops (timing only; results do not depend on it).
 * n <= 0 leaves the setting.  Returns the number now in effect. */
int ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* The table with channel weights (NULL: unit). */
int ora_lut_build_w(const void *src_guide, int fmt, int sw, int sh, int lut_bits,
                    const uint8_t *weights, uint32_t *lut)
{
    int64_t w[3];
    if (weights_get(fmt, weights, w)) return ORA_EINVAL;
    return lut_build_filtered(src_guide, NULL, 0, fmt, sw, sh, lut_bits, w, lut);
}

int ora_lut_build(const void *src_guide, int fmt, int sw, int sh, int lut_bits, uint32_t *lut)
{
    return ora_lut_build_w(src_guide, fmt, sw, sh, lut_bits, NULL, lut);
}

/* Selected bins of the table of any format, each by brute force over every
 * source pixel (the definition; for checking large tables by sampling):
 * out[k] = LUT[bins[k]]. */
int ora_lut_query_w(const void *src_guide, int fmt, int sw, int sh, int lut_bits,
                    const uint8_t *weights, const int64_t *bins, int64_t nbins, uint32_t *out)
{
    if (!src_guide || !bins || !out || sw < 1 || sh < 1 || !fmt_ok(fmt)) return ORA_EINVAL;
    int64_t w[3];
    if (weights_get(fmt, weights, w)) return ORA_EINVAL;
    if (lut_bits < 1 || lut_bits > guide_depth(fmt) || lut_bits > 12) return ORA_EINVAL;
    const int nc = guide_channels(fmt);
    const int64_t n = (int64_t)1 << lut_bits, npix = (int64_t)sw * sh;
    int64_t nb = 1;
    for (int k = 0; k < nc; ++k) nb *= n;
    for (int64_t j = 0; j < nbins; ++j)
        if (bins[j] < 0 || bins[j] >= nb) return ORA_EINVAL;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < nbins; ++j) {
        int64_t q[3], c = bins[j];
        for (int k = 0; k < nc; ++k, c /= n) q[k] = lut_bin_centre(c % n, fmt, lut_bits);
        uint64_t best_d = UINT64_MAX;
        int64_t best_i = -1;
        for (int64_t i = 0; i < npix; ++i) {
            int64_t g[3];
            guide_read_all(src_guide, fmt, i, g);
            uint64_t d = 0;
            for (int k = 0; k < nc; ++k) d += (uint64_t)(w[k] * (q[k] - g[k]) * (q[k] - g[k]));
            if (d < best_d) {
                best_d = d;
                best_i = i;
            }
        }
        out[j] = (uint32_t)(best_i % sw) | ((uint32_t)(best_i / sw) << 16);
    }
    return ORA_OK;
}

int ora_lut_query(const void *src_guide, int fmt, int sw, int sh, int lut_bits,
                  const int64_t *bins, int64_t nbins, uint32_t *out)
{
    return ora_lut_query_w(src_guide, fmt, sw, sh, lut_bits, NULL, bins, nbins, out);
}

/* The same entries as ora_lut_query_w, found faster for many bins: the
 * source pixels are grouped by their channel-0 value (raster order within a
 * group), and each query visits the groups outward from its centre's
 * channel-0 value, nearest first.  A group at channel-0 distance k holds
 * only pixels at (weighted) squared distance >= w0 k^2, so the walk stops
 * once that bound exceeds the best distance found (strictly: a pixel at
 * equal distance with a smaller raster index must still be seen).  Ties go
 * to the smallest raster index, as in the definition. */
int ora_lut_query_sweep_w(const void *src_guide, int fmt, int sw, int sh, int lut_bits,
                          const uint8_t *weights, const int64_t *bins, int64_t nbins,
                          uint32_t *out)
{
    if (!src_guide || !bins || !out || sw < 1 || sh < 1 || !fmt_ok(fmt)) return ORA_EINVAL;
    int64_t w[3];
    if (weights_get(fmt, weights, w)) return ORA_EINVAL;
    if (lut_bits < 1 || lut_bits > guide_depth(fmt) || lut_bits > 12) return ORA_EINVAL;
    const int nc = guide_channels(fmt);
    const int64_t n = (int64_t)1 << lut_bits, npix = (int64_t)sw * sh;
    const int64_t nv = (int64_t)1 << guide_depth(fmt); /* channel-0 values */
    int64_t nb = 1;
    for (int k = 0; k < nc; ++k) nb *= n;
    for (int64_t j = 0; j < nbins; ++j)
        if (bins[j] < 0 || bins[j] >= nb) return ORA_EINVAL;
    /* counting sort of the pixels by channel 0, raster order kept */
    int64_t *start = (int64_t *)calloc((size_t)(nv + 1), sizeof(int64_t));
    int64_t *order = (int64_t *)malloc((size_t)npix * sizeof(int64_t));
    if (!start || !order) { free(start); free(order); return ORA_ENOMEM; }
    for (int64_t i = 0; i < npix; ++i) {
        int64_t g[3];
        guide_read_all(src_guide, fmt, i, g);
        start[g[0] + 1]++;
    }
    for (int64_t v = 0; v < nv; ++v) start[v + 1] += start[v];
    {
        int64_t *fill = (int64_t *)malloc((size_t)nv * sizeof(int64_t));
        if (!fill) { free(start); free(order); return ORA_ENOMEM; }
        memcpy(fill, start, (size_t)nv * sizeof(int64_t));
        for (int64_t i = 0; i < npix; ++i) {
            int64_t g[3];
            guide_read_all(src_guide, fmt, i, g);
            order[fill[g[0]]++] = i;
        }
        free(fill);
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < nbins; ++j) {
        int64_t q[3], c = bins[j];
        for (int k = 0; k < nc; ++k, c /= n) q[k] = lut_bin_centre(c % n, fmt, lut_bits);
        uint64_t best_d = UINT64_MAX;
        int64_t best_i = -1;
        for (int64_t k = 0; k < nv; ++k) {
            const uint64_t lb = (uint64_t)(w[0] * k * k);
            if (best_i >= 0 && lb > best_d) break;
            for (int side = 0; side < (k == 0 ? 1 : 2); ++side) {
                const int64_t v = side == 0 ? q[0] - k : q[0] + k;
                if (v < 0 || v >= nv) continue;
                for (int64_t e = start[v]; e < start[v + 1]; ++e) {
                    const int64_t i = order[e];
                    int64_t g[3];
                    guide_read_all(src_guide, fmt, i, g);
                    uint64_t d = 0;
                    for (int m = 0; m < nc; ++m)
                        d += (uint64_t)(w[m] * (q[m] - g[m]) * (q[m] - g[m]));
                    if (d < best_d || (d == best_d && i < best_i)) {
                        best_d = d;
                        best_i = i;
                    }
                }
            }
        }
        out[j] = (uint32_t)(best_i % sw) | ((uint32_t)(best_i / sw) << 16);
    }
    free(start);
    free(order);
    return ORA_OK;
}

/* Per-label tables luts[l * bins + c] for labels l = 0..nlabels-1, from the
 * source pixels labelled l; a label without source pixels gets the
 * unconstrained table. */
int ora_lut_build_labels_w(const void *src_guide, const uint8_t *labels, int nlabels, int fmt,
                           int sw, int sh, int lut_bits, const uint8_t *weights, uint32_t *luts)
{
    if (!labels || !luts || nlabels < 1 || nlabels > 256) return ORA_EINVAL;
    int64_t w[3];
    if (weights_get(fmt, weights, w)) return ORA_EINVAL;
    if (!fmt_ok(fmt) || lut_bits < 1 || lut_bits > guide_depth(fmt) || lut_bits > 12)
        return ORA_EINVAL;
    const int64_t bins = (int64_t)1 << (guide_channels(fmt) * lut_bits);
    for (int l = 0; l < nlabels; ++l) {
        int rc = lut_build_filtered(src_guide, labels, l, fmt, sw, sh, lut_bits, w, luts + l * bins);
        if (rc == 1)
            rc = lut_build_filtered(src_guide, NULL, 0, fmt, sw, sh, lut_bits, w, luts + l * bins);
        if (rc != ORA_OK) return rc;
    }
    return ORA_OK;
}

int ora_lut_build_labels(const void *src_guide, const uint8_t *labels, int nlabels, int fmt, int sw,
                         int sh, int lut_bits, uint32_t *luts)
{
    return ora_lut_build_labels_w(src_guide, labels, nlabels, fmt, sw, sh, lut_bits, NULL, luts);
}

/* ------------------------------------------------ seed hierarchy (Sec. 3.2) */

typedef struct {
    int w, h;               /* target size */
    int levels, finest;
    const uint32_t *jitter; /* concatenated per-level tables */
} seeds_t;

static int64_t level_spacing(const seeds_t *S, int i) { return (int64_t)S->finest << (S->levels - 1 - i); }
static int64_t cells_x(const seeds_t *S, int i) { int64_t h = level_spacing(S, i); return (S->w + h - 1) / h; }
static int64_t cells_y(const seeds_t *S, int i) { int64_t h = level_spacing(S, i); return (S->h + h - 1) / h; }

static int64_t level_offset(const seeds_t *S, int i)
{
    int64_t off = 0;
    for (int k = 0; k < i; ++k) off += cells_x(S, k) * cells_y(S, k);
    return off;
}

/* Number of jitter entries for the whole hierarchy. */
int64_t ora_jitter_len(int w, int h, int levels, int finest)
{
    seeds_t S = {w, h, levels, finest, NULL};
    return level_offset(&S, levels);
}

/* ---------------------------------------- jitter from a counter-based RNG
 *
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011), written from its definition: ten rounds, each
 * multiplying words 0 and 2 of the counter by the two round constants and
 * mixing the halves of the 128-bit products with words 1 and 3 and the key,
 * which is bumped by the two Weyl constants between rounds.
 */
static void mul64_hilo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    const unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void ora_philox4x64(const uint64_t key_in[2], const uint64_t ctr_in[4], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t k0 = key_in[0], k1 = key_in[1];
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul64_hilo(M0, c0, &hi0, &lo0);
        mul64_hilo(M1, c2, &hi1, &lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* The jitter table of a W x H target drawn from Philox4x64-10 under key
 * (seed, stream): entry e (levels coarsest first, cells row-major) takes word
 * 0 of the block at counter (e, 0, 0, 0); jx = word mod h_i and jy = (word >>
 * 32) mod h_i for the level's spacing h_i (a power of two). */
int ora_jitter_fill(int w, int h, int levels, int finest, uint64_t seed, uint64_t stream,
                    uint32_t *out)
{
    if (w < 1 || h < 1 || levels < 0 || levels > 12 || finest < 1 || (finest & (finest - 1)))
        return ORA_EINVAL;
    if (!out && levels > 0) return ORA_EINVAL;
    seeds_t S = {w, h, levels, finest, NULL};
    const uint64_t key[2] = {seed, stream};
    for (int i = 0; i < levels; ++i) {
        const uint64_t hm = (uint64_t)level_spacing(&S, i) - 1;
        for (int64_t e = level_offset(&S, i); e < level_offset(&S, i + 1); ++e) {
            const uint64_t ctr[4] = {(uint64_t)e, 0, 0, 0};
            uint64_t r[4];
            ora_philox4x64(key, ctr, r);
            out[e] = (uint32_t)(r[0] & hm) | ((uint32_t)((r[0] >> 32) & hm) << 16);
        }
    }
    return ORA_OK;
}

/* ------------------------------------ jitter from an integer hash
 *
 * The paper leaves RandomJitterTable's contents open (Algorithm 2,
 * SeedPoint).  This reading defines them by a hash of (cell, level, seed), so
 * a frame's seeds follow from one 32-bit seed value with no table:
 *   mix(x):  x ^= x >> 16; x *= 0x9E3779B9; x ^= x >> 15; x *= 0x6A09E667;
 *            x ^= x >> 16   (uint32 arithmetic, wrapping)
 *   k = mix(mix(mix(mix(seed + 0xBB67AE85) ^ log2 h) ^ bx) ^ by)
 *   jx = k & (h - 1),  jy = (k >> 16) & (h - 1)
 * The multipliers are floor(2^32 / golden ratio) and the first 32 fraction
 * bits of sqrt(2); the additive constant is the first 32 fraction bits of
 * sqrt(3).  The level enters through log2 h, so one cell index at two levels
 * gets unrelated jitter.
 */
static uint32_t hash_mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x9E3779B9u;
    x ^= x >> 15;
    x *= 0x6A09E667u;
    x ^= x >> 16;
    return x;
}

uint32_t ora_jitter_hash_key(uint32_t seed, uint32_t log2h, uint32_t bx, uint32_t by)
{
    uint32_t k = hash_mix(seed + 0xBB67AE85u);
    k = hash_mix(k ^ log2h);
    k = hash_mix(k ^ bx);
    return hash_mix(k ^ by);
}

/* The jitter table that the hash defines for a W x H target: entry (level i,
 * cell b) = jx | jy << 16 with the level's spacing h_i, in the table layout
 * of ora_jitter_fill (levels coarsest first, cells row-major). */
int ora_jitter_hash(int w, int h, int levels, int finest, uint32_t seed, uint32_t *out)
{
    if (w < 1 || h < 1 || levels < 0 || levels > 12 || finest < 1 || (finest & (finest - 1)))
        return ORA_EINVAL;
    if (!out && levels > 0) return ORA_EINVAL;
    seeds_t S = {w, h, levels, finest, NULL};
    for (int i = 0; i < levels; ++i) {
        const int64_t sp = level_spacing(&S, i);
        uint32_t lg = 0;
        while (((int64_t)1 << lg) < sp) ++lg;
        const int64_t ncx = cells_x(&S, i), base = level_offset(&S, i);
        for (int64_t e = base; e < level_offset(&S, i + 1); ++e) {
            const int64_t bx = (e - base) % ncx, by = (e - base) / ncx;
            const uint32_t k = ora_jitter_hash_key(seed, lg, (uint32_t)bx, (uint32_t)by);
            out[e] = (k & (uint32_t)(sp - 1)) | (((k >> 16) & (uint32_t)(sp - 1)) << 16);
        }
    }
    return ORA_OK;
}

static int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

/* SeedPoint: the jittered seed of cell (bx, by) at level i.  Returns 0 when
 * the seed is not a candidate (cell outside the table, or seed outside the
 * target image). */
static int seed_point(const seeds_t *S, int i, int64_t bx, int64_t by, int64_t *sx, int64_t *sy)
{
    int64_t h = level_spacing(S, i), ncx = cells_x(S, i), ncy = cells_y(S, i);
    if (bx < 0 || by < 0 || bx >= ncx || by >= ncy) return 0;
    uint32_t j = S->jitter[level_offset(S, i) + by * ncx + bx];
    *sx = h * bx + (int64_t)(j & 0xFFFFu);
    *sy = h * by + (int64_t)(j >> 16);
    return *sx < S->w && *sy < S->h;
}

/* NearestSeed: among the seeds of the 3x3 cells around p's cell, the first
 * (x outer, y inner) with the strictly smallest distance to p. */
static int nearest_seed(const seeds_t *S, int i, int64_t px, int64_t py, int64_t *qx, int64_t *qy)
{
    int64_t h = level_spacing(S, i);
    int64_t bx = floor_div(px, h), by = floor_div(py, h);
    uint64_t best = UINT64_MAX;
    for (int dx = -1; dx <= 1; ++dx) {
        for (int dy = -1; dy <= 1; ++dy) {
            int64_t sx, sy;
            if (!seed_point(S, i, bx + dx, by + dy, &sx, &sy)) continue;
            uint64_t d = (uint64_t)((sx - px) * (sx - px) + (sy - py) * (sy - py));
            if (d < best) {
                best = d;
                *qx = sx;
                *qy = sy;
            }
        }
    }
    return best != UINT64_MAX;
}

int ora_seed_point(int w, int h, int levels, int finest, const uint32_t *jitter, int level,
                   int64_t bx, int64_t by, int64_t *sx, int64_t *sy)
{
    seeds_t S = {w, h, levels, finest, jitter};
    return seed_point(&S, level, bx, by, sx, sy);
}

int ora_nearest_seed(int w, int h, int levels, int finest, const uint32_t *jitter, int level,
                     int64_t px, int64_t py, int64_t *qx, int64_t *qy)
{
    seeds_t S = {w, h, levels, finest, jitter};
    return nearest_seed(&S, level, px, py, qx, qy);
}

/* ------------------------------------------ per-pixel level loop (Alg. 2) */

typedef struct {
    const void *src_guide;
    int sw, sh;
    const uint32_t *lut;    /* one table, or nlabels tables with labels */
    int fmt, lut_bits;
    const void *tgt_guide;
    seeds_t seeds;
    uint32_t threshold;
    const uint8_t *src_labels, *tgt_labels;  /* both NULL without segmentation */
    int nlabels;
    int64_t wt[3];          /* channel weights of the error (unit without weights) */
} assign_t;

/* The lookup of a guide value g[] in the table of `label` (ignored without
 * segmentation; values past the last table use the last one).  Bin index
 * c0 + c1 * n (+ c2 * n^2 with three channels). */
static uint32_t lut_lookup(const assign_t *A, const int64_t *g, int label)
{
    const int nc = guide_channels(A->fmt);
    const int64_t n = (int64_t)1 << A->lut_bits;
    int64_t bins = 1, c = 0;
    for (int k = 0; k < nc; ++k) {
        c += lut_quantise(g[k], A->fmt, A->lut_bits) * bins;
        bins *= n;
    }
    const uint32_t *t = A->lut;
    if (A->tgt_labels) t += (int64_t)(label < A->nlabels ? label : A->nlabels - 1) * bins;
    return t[c];
}

/* ParallelStyleBlit for one pixel, with colours replaced by coordinates:
 * returns the source coordinate (x | y << 16) and the chunk code
 * (level << 26) | (qy << 13) | qx. */
static void assign_pixel(const assign_t *A, int64_t px, int64_t py, uint32_t *nnf, uint32_t *chunk)
{
    const int W = A->seeds.w, nc = guide_channels(A->fmt);
    int64_t tg[3];
    guide_read_all(A->tgt_guide, A->fmt, py * W + px, tg);
    const int lp = A->tgt_labels ? A->tgt_labels[py * W + px] : 0;
    for (int i = 0; i < A->seeds.levels; ++i) {
        int64_t qx, qy;
        if (!nearest_seed(&A->seeds, i, px, py, &qx, &qy)) continue;
        int64_t qg[3];
        guide_read_all(A->tgt_guide, A->fmt, qy * W + qx, qg);
        const int lq = A->tgt_labels ? A->tgt_labels[qy * W + qx] : 0;
        uint32_t u = lut_lookup(A, qg, lq);
        int64_t vx = (int64_t)(u & 0xFFFFu) + (px - qx);
        int64_t vy = (int64_t)(u >> 16) + (py - qy);
        if (vx < 0 || vy < 0 || vx >= A->sw || vy >= A->sh) continue;
        /* segmentation: the source pixel must carry the pixel's label */
        if (A->tgt_labels && A->src_labels[vy * A->sw + vx] != lp) continue;
        int64_t sg[3];
        guide_read_all(A->src_guide, A->fmt, vy * A->sw + vx, sg);
        uint64_t e = 0;
        for (int k = 0; k < nc; ++k) e += (uint64_t)(A->wt[k] * (tg[k] - sg[k]) * (tg[k] - sg[k]));
        if (e < (uint64_t)A->threshold) {
            *nnf = (uint32_t)vx | ((uint32_t)vy << 16);
            *chunk = ((uint32_t)i << 26) | ((uint32_t)qy << 13) | (uint32_t)qx;
            return;
        }
    }
    *nnf = lut_lookup(A, tg, lp);
    *chunk = ((uint32_t)A->seeds.levels << 26) | ((uint32_t)py << 13) | (uint32_t)px;
}

static int check_common(int sw, int sh, int fmt, int lut_bits, int w, int h, int levels, int finest)
{
    if (sw < 1 || sh < 1 || sw > 8192 || sh > 8192) return ORA_EINVAL;
    if (w < 1 || h < 1 || w > 8192 || h > 8192) return ORA_EINVAL;
    if (!fmt_ok(fmt)) return ORA_EINVAL;
    if (lut_bits < 1 || lut_bits > guide_depth(fmt) || lut_bits > 12) return ORA_EINVAL;
    if (levels < 0 || levels > 12) return ORA_EINVAL;
    if (finest < 1 || (finest & (finest - 1)) != 0) return ORA_EINVAL;
    if (levels > 0 && ((int64_t)finest << (levels - 1)) > 8192) return ORA_EINVAL;
    return ORA_OK;
}

/* The level loop with channel weights (NULL: unit); the table must have
 * been built with the same weights. */
int ora_assign_w(const void *src_guide, int sw, int sh, const uint32_t *lut, int fmt, int lut_bits,
                 const uint8_t *weights, const void *tgt_guide, int w, int h,
                 const uint32_t *jitter, int levels, int finest, uint32_t threshold,
                 uint32_t *out_nnf, uint32_t *out_chunk, int64_t row0, int64_t rows)
{
    int rc = check_common(sw, sh, fmt, lut_bits, w, h, levels, finest);
    if (rc) return rc;
    if (!src_guide || !lut || !tgt_guide || !out_nnf || !out_chunk) return ORA_EINVAL;
    if (levels > 0 && !jitter) return ORA_EINVAL;
    if (rows < 0) rows = h;
    if (row0 < 0 || row0 + rows > h) return ORA_EINVAL;
    assign_t A = {src_guide, sw, sh, lut, fmt, lut_bits, tgt_guide, {w, h, levels, finest, jitter},
                  threshold, NULL, NULL, 0, {1, 1, 1}};
    if (weights_get(fmt, weights, A.wt)) return ORA_EINVAL;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t y = row0; y < row0 + rows; ++y)
        for (int64_t x = 0; x < w; ++x)
            assign_pixel(&A, x, y, &out_nnf[y * w + x], &out_chunk[y * w + x]);
    return ORA_OK;
}

int ora_assign(const void *src_guide, int sw, int sh, const uint32_t *lut, int fmt, int lut_bits,
               const void *tgt_guide, int w, int h, const uint32_t *jitter, int levels, int finest,
               uint32_t threshold, uint32_t *out_nnf, uint32_t *out_chunk, int64_t row0, int64_t rows)
{
    return ora_assign_w(src_guide, sw, sh, lut, fmt, lut_bits, NULL, tgt_guide, w, h, jitter,
                        levels, finest, threshold, out_nnf, out_chunk, row0, rows);
}

/* ------------------------------------------------ voting blend (Sec. 3.2) */

/* C_T[p] = average over target pixels n in the (2r+1)^2 window around p of
 * C_S[NNF[n] + (p - n)], counting only co-located pixels inside the source. */
int ora_blend(const uint8_t *src_rgb, int sw, int sh, const uint32_t *nnf, int w, int h, int radius,
              uint8_t *out_rgb, int64_t row0, int64_t rows)
{
    if (!src_rgb || !nnf || !out_rgb || radius < 0 || radius > 16) return ORA_EINVAL;
    if (sw < 1 || sh < 1 || w < 1 || h < 1) return ORA_EINVAL;
    if (rows < 0) rows = h;
    if (row0 < 0 || row0 + rows > h) return ORA_EINVAL;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t py = row0; py < row0 + rows; ++py) {
        for (int64_t px = 0; px < w; ++px) {
            uint64_t sum[3] = {0, 0, 0};
            uint64_t k = 0;
            for (int64_t ny = py - radius; ny <= py + radius; ++ny) {
                for (int64_t nx = px - radius; nx <= px + radius; ++nx) {
                    if (nx < 0 || ny < 0 || nx >= w || ny >= h) continue;
                    uint32_t v = nnf[ny * w + nx];
                    int64_t sx = (int64_t)(v & 0xFFFFu) + (px - nx);
                    int64_t sy = (int64_t)(v >> 16) + (py - ny);
                    if (sx < 0 || sy < 0 || sx >= sw || sy >= sh) continue;
                    const uint8_t *c = &src_rgb[3 * (sy * sw + sx)];
                    sum[0] += c[0];
                    sum[1] += c[1];
                    sum[2] += c[2];
                    k++;
                }
            }
            uint8_t *o = &out_rgb[3 * (py * w + px)];
            /* k >= 1 whenever NNF[p] itself lies in the source, which the
             * level loop guarantees; a foreign NNF without it yields 0. */
            for (int c = 0; c < 3; ++c) o[c] = k ? (uint8_t)((sum[c] + k / 2) / k) : 0;
        }
    }
    return ORA_OK;
}

/* ------------------------------------------------------------ whole path */

int ora_stylize_w(const uint8_t *src_rgb, const void *src_guide, int sw, int sh,
                  const uint32_t *lut, int fmt, int lut_bits, const uint8_t *weights,
                  const void *tgt_guide, int w, int h, const uint32_t *jitter, int levels,
                  int finest, uint32_t threshold, int radius, uint8_t *out_rgb,
                  uint32_t *out_chunk, uint32_t *out_nnf)
{
    if (!out_rgb || !out_chunk) return ORA_EINVAL;
    uint32_t *nnf = out_nnf ? out_nnf : (uint32_t *)malloc((size_t)w * h * sizeof(uint32_t));
    if (!nnf) return ORA_ENOMEM;
    int rc = ora_assign_w(src_guide, sw, sh, lut, fmt, lut_bits, weights, tgt_guide, w, h, jitter,
                          levels, finest, threshold, nnf, out_chunk, 0, -1);
    if (rc == ORA_OK) rc = ora_blend(src_rgb, sw, sh, nnf, w, h, radius, out_rgb, 0, -1);
    if (!out_nnf) free(nnf);
    return rc;
}

int ora_stylize(const uint8_t *src_rgb, const void *src_guide, int sw, int sh, const uint32_t *lut,
                int fmt, int lut_bits, const void *tgt_guide, int w, int h, const uint32_t *jitter,
                int levels, int finest, uint32_t threshold, int radius, uint8_t *out_rgb,
                uint32_t *out_chunk, uint32_t *out_nnf)
{
    return ora_stylize_w(src_rgb, src_guide, sw, sh, lut, fmt, lut_bits, NULL, tgt_guide, w, h,
                         jitter, levels, finest, threshold, radius, out_rgb, out_chunk, out_nnf);
}

/* ----------------------------------------------------- segmentation guide */

/* ora_assign with label maps: src_labels Sw*Sh, tgt_labels W*H, luts the
 * nlabels tables of ora_lut_build_labels. */
int ora_assign_seg_w(const void *src_guide, const uint8_t *src_labels, int sw, int sh,
                     const uint32_t *luts, int nlabels, int fmt, int lut_bits,
                     const uint8_t *weights, const void *tgt_guide, const uint8_t *tgt_labels,
                     int w, int h, const uint32_t *jitter, int levels, int finest,
                     uint32_t threshold, uint32_t *out_nnf, uint32_t *out_chunk)
{
    int rc = check_common(sw, sh, fmt, lut_bits, w, h, levels, finest);
    if (rc) return rc;
    if (!src_guide || !src_labels || !luts || !tgt_guide || !tgt_labels || !out_nnf || !out_chunk)
        return ORA_EINVAL;
    if (nlabels < 1 || nlabels > 256) return ORA_EINVAL;
    if (levels > 0 && !jitter) return ORA_EINVAL;
    assign_t A = {src_guide, sw, sh, luts, fmt, lut_bits, tgt_guide, {w, h, levels, finest, jitter},
                  threshold, src_labels, tgt_labels, nlabels, {1, 1, 1}};
    if (weights_get(fmt, weights, A.wt)) return ORA_EINVAL;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x)
            assign_pixel(&A, x, y, &out_nnf[y * w + x], &out_chunk[y * w + x]);
    return ORA_OK;
}

int ora_assign_seg(const void *src_guide, const uint8_t *src_labels, int sw, int sh,
                   const uint32_t *luts, int nlabels, int fmt, int lut_bits, const void *tgt_guide,
                   const uint8_t *tgt_labels, int w, int h, const uint32_t *jitter, int levels,
                   int finest, uint32_t threshold, uint32_t *out_nnf, uint32_t *out_chunk)
{
    return ora_assign_seg_w(src_guide, src_labels, sw, sh, luts, nlabels, fmt, lut_bits, NULL,
                            tgt_guide, tgt_labels, w, h, jitter, levels, finest, threshold,
                            out_nnf, out_chunk);
}

int ora_stylize_seg_w(const uint8_t *src_rgb, const void *src_guide, const uint8_t *src_labels,
                      int sw, int sh, const uint32_t *luts, int nlabels, int fmt, int lut_bits,
                      const uint8_t *weights, const void *tgt_guide, const uint8_t *tgt_labels,
                      int w, int h, const uint32_t *jitter, int levels, int finest,
                      uint32_t threshold, int radius, uint8_t *out_rgb, uint32_t *out_chunk,
                      uint32_t *out_nnf)
{
    if (!out_rgb || !out_chunk) return ORA_EINVAL;
    uint32_t *nnf = out_nnf ? out_nnf : (uint32_t *)malloc((size_t)w * h * sizeof(uint32_t));
    if (!nnf) return ORA_ENOMEM;
    int rc = ora_assign_seg_w(src_guide, src_labels, sw, sh, luts, nlabels, fmt, lut_bits, weights,
                              tgt_guide, tgt_labels, w, h, jitter, levels, finest, threshold, nnf,
                              out_chunk);
    if (rc == ORA_OK) rc = ora_blend(src_rgb, sw, sh, nnf, w, h, radius, out_rgb, 0, -1);
    if (!out_nnf) free(nnf);
    return rc;
}

int ora_stylize_seg(const uint8_t *src_rgb, const void *src_guide, const uint8_t *src_labels, int sw,
                    int sh, const uint32_t *luts, int nlabels, int fmt, int lut_bits,
                    const void *tgt_guide, const uint8_t *tgt_labels, int w, int h,
                    const uint32_t *jitter, int levels, int finest, uint32_t threshold, int radius,
                    uint8_t *out_rgb, uint32_t *out_chunk, uint32_t *out_nnf)
{
    if (!out_rgb || !out_chunk) return ORA_EINVAL;
    uint32_t *nnf = out_nnf ? out_nnf : (uint32_t *)malloc((size_t)w * h * sizeof(uint32_t));
    if (!nnf) return ORA_ENOMEM;
    int rc = ora_assign_seg(src_guide, src_labels, sw, sh, luts, nlabels, fmt, lut_bits, tgt_guide,
                            tgt_labels, w, h, jitter, levels, finest, threshold, nnf, out_chunk);
    if (rc == ORA_OK) rc = ora_blend(src_rgb, sw, sh, nnf, w, h, radius, out_rgb, 0, -1);
    if (!out_nnf) free(nnf);
    return rc;
}

/* ------------------------------------ guides of many channels, exact search
 *
 * The additional guiding channels of Sec. 3.1, where the paper suggests a
 * search tree instead of a table: a guide of C = 2..8 channels of depth 8
 * (fmt 3) or 16 bits (fmt 4).  Pixel i's channels are elements 0..C-1 of
 * its texel of S bytes, S the smallest of 4, 8 and 16 that holds C channels;
 * elements past C are ignored.  Read as an exact search with no
 * quantisation: the lookup of a guide value g is
 *     u*(g) = argmin over source pixels u of sum_k w_k (g_k - G_S[u]_k)^2,
 * ties to the smallest raster index, with integer weights w_k in 0..127
 * (NULL or all zero: unit).  The guide error of the level loop is the same
 * weighted sum, accepted iff it is < t; everything else (seeds, NearestSeed,
 * the fallback to the pixel's own lookup, voting) is the plain path's.
 */

/* Bytes per texel of a C-channel guide of the given depth; 0 if invalid. */
int ora_texel_bytes(int depth, int channels)
{
    if ((depth != 8 && depth != 16) || channels < 2 || channels > 8) return 0;
    const int bytes = channels * depth / 8;
    return bytes <= 4 ? 4 : bytes <= 8 ? 8 : 16;
}

typedef struct {
    const void *g;   /* texels */
    int depth, channels, stride;
} guide_n_t;

static int64_t chan_n(const guide_n_t *G, int64_t idx, int k)
{
    const uint8_t *p = (const uint8_t *)G->g + idx * G->stride;
    if (G->depth == 8) return p[k];
    uint16_t v;
    memcpy(&v, p + 2 * k, 2);
    return v;
}

/* Weights of a many-channel guide: NULL or all zero = unit; else 0..127. */
static int weights_get_n(const uint8_t *weights, int channels, int64_t *w)
{
    int any = 0;
    for (int k = 0; k < 8; ++k) w[k] = 1;
    if (!weights) return ORA_OK;
    for (int k = 0; k < channels; ++k) any |= weights[k] != 0;
    if (!any) return ORA_OK;
    for (int k = 0; k < channels; ++k) {
        if (weights[k] > 127) return ORA_EINVAL;
        w[k] = weights[k];
    }
    return ORA_OK;
}

/* sum_k w_k (a_k - b_k)^2 between texel ia of A and texel ib of B. */
static uint64_t dist_n(const guide_n_t *A, int64_t ia, const guide_n_t *B, int64_t ib,
                       const int64_t *w)
{
    uint64_t d = 0;
    for (int k = 0; k < A->channels; ++k) {
        const int64_t e = chan_n(A, ia, k) - chan_n(B, ib, k);
        d += (uint64_t)w[k] * (uint64_t)(e * e);
    }
    return d;
}

static int guide_n_make(const void *g, int depth, int channels, guide_n_t *G)
{
    G->g = g;
    G->depth = depth;
    G->channels = channels;
    G->stride = ora_texel_bytes(depth, channels);
    return g && G->stride ? ORA_OK : ORA_EINVAL;
}

static uint32_t pack_src(int64_t i, int sw)
{
    return (uint32_t)(i % sw) | ((uint32_t)(i / sw) << 16);
}

/* The lookup of every query texel by brute force over every source pixel in
 * raster order with a strict compare (the definition). */
int ora_nn_query_n(const void *src_guide, int depth, int channels, int sw, int sh,
                   const uint8_t *weights, const void *queries, int64_t nq, uint32_t *out)
{
    guide_n_t S, Q;
    int64_t w[8];
    if (sw < 1 || sh < 1 || !out || nq < 0) return ORA_EINVAL;
    if (guide_n_make(src_guide, depth, channels, &S) || guide_n_make(queries, depth, channels, &Q))
        return ORA_EINVAL;
    if (weights_get_n(weights, channels, w)) return ORA_EINVAL;
    const int64_t npix = (int64_t)sw * sh;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nq; ++j) {
        uint64_t best_d = UINT64_MAX;
        int64_t best_i = -1;
        for (int64_t i = 0; i < npix; ++i) {
            const uint64_t d = dist_n(&Q, j, &S, i, w);
            if (d < best_d) {
                best_d = d;
                best_i = i;
            }
        }
        out[j] = pack_src(best_i, sw);
    }
    return ORA_OK;
}

/* Source pixels grouped by their channel-0 value (raster order within a
 * group), for the sweep below. */
typedef struct {
    int64_t nv;       /* channel-0 values: 2^depth */
    int64_t *start;   /* nv + 1 group starts */
    int64_t *order;   /* raster indices by group */
} sweep_t;

static void sweep_free(sweep_t *T)
{
    free(T->start);
    free(T->order);
}

static int sweep_make(const guide_n_t *S, int64_t npix, sweep_t *T)
{
    T->nv = (int64_t)1 << S->depth;
    T->start = (int64_t *)calloc((size_t)(T->nv + 1), sizeof(int64_t));
    T->order = (int64_t *)malloc((size_t)npix * sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc((size_t)T->nv * sizeof(int64_t));
    if (!T->start || !T->order || !fill) {
        free(fill);
        sweep_free(T);
        return ORA_ENOMEM;
    }
    for (int64_t i = 0; i < npix; ++i) T->start[chan_n(S, i, 0) + 1]++;
    for (int64_t v = 0; v < T->nv; ++v) T->start[v + 1] += T->start[v];
    memcpy(fill, T->start, (size_t)T->nv * sizeof(int64_t));
    for (int64_t i = 0; i < npix; ++i) T->order[fill[chan_n(S, i, 0)]++] = i;
    free(fill);
    return ORA_OK;
}

/* The lookup of texel j of Q: the groups are visited outward from the
 * query's channel-0 value v0, at distance k = 0, 1, 2, ...; a group at
 * distance k holds only pixels at weighted squared distance >= w0 k^2, so the
 * walk stops once that bound exceeds the best distance (strictly: a pixel at
 * equal distance with a smaller raster index must still be seen).  Ties to
 * the smallest raster index, as in the definition. */
static uint32_t sweep_query(const guide_n_t *S, int sw, const sweep_t *T, const guide_n_t *Q,
                            int64_t j, const int64_t *w)
{
    const int64_t v0 = chan_n(Q, j, 0);
    uint64_t best_d = UINT64_MAX;
    int64_t best_i = -1;
    for (int64_t k = 0; k < T->nv; ++k) {
        if (best_i >= 0 && (uint64_t)w[0] * (uint64_t)(k * k) > best_d) break;
        for (int side = 0; side < (k == 0 ? 1 : 2); ++side) {
            const int64_t v = side == 0 ? v0 - k : v0 + k;
            if (v < 0 || v >= T->nv) continue;
            for (int64_t e = T->start[v]; e < T->start[v + 1]; ++e) {
                const int64_t i = T->order[e];
                const uint64_t d = dist_n(Q, j, S, i, w);
                if (d < best_d || (d == best_d && i < best_i)) {
                    best_d = d;
                    best_i = i;
                }
            }
        }
    }
    return pack_src(best_i, sw);
}

/* The same lookups as ora_nn_query_n, by the channel-0 sweep. */
int ora_nn_sweep_n(const void *src_guide, int depth, int channels, int sw, int sh,
                   const uint8_t *weights, const void *queries, int64_t nq, uint32_t *out)
{
    guide_n_t S, Q;
    sweep_t T;
    int64_t w[8];
    if (sw < 1 || sh < 1 || !out || nq < 0) return ORA_EINVAL;
    if (guide_n_make(src_guide, depth, channels, &S) || guide_n_make(queries, depth, channels, &Q))
        return ORA_EINVAL;
    if (weights_get_n(weights, channels, w)) return ORA_EINVAL;
    if (sweep_make(&S, (int64_t)sw * sh, &T)) return ORA_ENOMEM;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nq; ++j) out[j] = sweep_query(&S, sw, &T, &Q, j, w);
    sweep_free(&T);
    return ORA_OK;
}

/* The level loop (Algorithm 2) with a many-channel guide: as assign_pixel,
 * with u* the exact search above.  Each seed's lookup is a function of the
 * seed alone, so it is found once per seed (seed_u, per level and cell, in
 * the jitter table's order) and read by every pixel whose NearestSeed it is;
 * the fallback searches per pixel. */
int ora_assign_n(const void *src_guide, int sw, int sh, int depth, int channels,
                 const uint8_t *weights, const void *tgt_guide, int w, int h,
                 const uint32_t *jitter, int levels, int finest, uint32_t threshold,
                 uint32_t *out_nnf, uint32_t *out_chunk)
{
    guide_n_t S, T;
    int64_t wt[8];
    if (sw < 1 || sh < 1 || sw > 8192 || sh > 8192 || w < 1 || h < 1 || w > 8192 || h > 8192)
        return ORA_EINVAL;
    if (levels < 0 || levels > 12 || finest < 1 || (finest & (finest - 1)) != 0) return ORA_EINVAL;
    if (levels > 0 && ((int64_t)finest << (levels - 1)) > 8192) return ORA_EINVAL;
    if (levels > 0 && !jitter) return ORA_EINVAL;
    if (!out_nnf || !out_chunk) return ORA_EINVAL;
    if (guide_n_make(src_guide, depth, channels, &S) || guide_n_make(tgt_guide, depth, channels, &T))
        return ORA_EINVAL;
    if (weights_get_n(weights, channels, wt)) return ORA_EINVAL;
    const seeds_t sd = {w, h, levels, finest, jitter};
    sweep_t sweep;
    if (sweep_make(&S, (int64_t)sw * sh, &sweep)) return ORA_ENOMEM;
    const int64_t nseeds = levels > 0 ? level_offset(&sd, levels) : 0;
    uint32_t *seed_u = (uint32_t *)malloc((size_t)(nseeds > 0 ? nseeds : 1) * sizeof(uint32_t));
    if (!seed_u) {
        sweep_free(&sweep);
        return ORA_ENOMEM;
    }
    /* the lookup of every in-target seed */
    for (int i = 0; i < levels; ++i) {
        const int64_t ncx = cells_x(&sd, i), ncy = cells_y(&sd, i), base = level_offset(&sd, i);
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t c = 0; c < ncx * ncy; ++c) {
            int64_t sx, sy;
            seed_u[base + c] = 0;
            if (seed_point(&sd, i, c % ncx, c / ncx, &sx, &sy))
                seed_u[base + c] = sweep_query(&S, sw, &sweep, &T, sy * w + sx, wt);
        }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t py = 0; py < h; ++py) {
        for (int64_t px = 0; px < w; ++px) {
            const int64_t p = py * w + px;
            int done = 0;
            for (int i = 0; i < levels && !done; ++i) {
                int64_t qx, qy;
                if (!nearest_seed(&sd, i, px, py, &qx, &qy)) continue;
                const int64_t hsp = level_spacing(&sd, i);
                const int64_t cell = level_offset(&sd, i) + (qy / hsp) * cells_x(&sd, i) + qx / hsp;
                const uint32_t u = seed_u[cell];
                const int64_t vx = (int64_t)(u & 0xFFFFu) + (px - qx);
                const int64_t vy = (int64_t)(u >> 16) + (py - qy);
                if (vx < 0 || vy < 0 || vx >= sw || vy >= sh) continue;
                if (dist_n(&T, p, &S, vy * sw + vx, wt) < (uint64_t)threshold) {
                    out_nnf[p] = (uint32_t)vx | ((uint32_t)vy << 16);
                    out_chunk[p] = ((uint32_t)i << 26) | ((uint32_t)qy << 13) | (uint32_t)qx;
                    done = 1;
                }
            }
            if (!done) {
                out_nnf[p] = sweep_query(&S, sw, &sweep, &T, p, wt);
                out_chunk[p] = ((uint32_t)levels << 26) | ((uint32_t)py << 13) | (uint32_t)px;
            }
        }
    }
    free(seed_u);
    sweep_free(&sweep);
    return ORA_OK;
}

/* The whole path with a many-channel guide: ora_assign_n, then the vote. */
int ora_stylize_n(const uint8_t *src_rgb, const void *src_guide, int sw, int sh, int depth,
                  int channels, const uint8_t *weights, const void *tgt_guide, int w, int h,
                  const uint32_t *jitter, int levels, int finest, uint32_t threshold, int radius,
                  uint8_t *out_rgb, uint32_t *out_chunk, uint32_t *out_nnf)
{
    if (!out_rgb || !out_chunk || !out_nnf) return ORA_EINVAL;
    int rc = ora_assign_n(src_guide, sw, sh, depth, channels, weights, tgt_guide, w, h, jitter,
                          levels, finest, threshold, out_nnf, out_chunk);
    if (rc == ORA_OK) rc = ora_blend(src_rgb, sw, sh, out_nnf, w, h, radius, out_rgb, 0, -1);
    return rc;
}
