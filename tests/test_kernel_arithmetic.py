"""Integer identities the HIP kernels rely on, checked exhaustively over the
ranges where they are used (host arithmetic only, no GPU):

- the level loop stages seed record j (level j / 9, neighbour j % 9) with
  j / 9 = (57 j) >> 9 for j < 128 (two records per lane, 9 L <= 108), and
  splits neighbour k into x = (11 k) >> 5 = k / 3, y = k - 3 x for k < 9;
- each level's cell count per axis is ceil(n / 2^s) = ((n - 1) >> s) + 1
  for every side 1..8192 and log2 spacing 0..13, the form the level loop uses
  in place of the per-level table;
- pixel and texel indices fit the 24-bit multiplier: every factor is below
  2^24 and every product y * w + x below 2^32 for sides up to 8192 (plus the
  exemplar margin);
- the block level loop reads the record at slot (key & 15) of a level even
  when no neighbour holds a seed (key = INT32_MAX, slot 15): with records
  staged kRecStride apart that read stays inside the block's records for
  every hierarchy the block path runs (finest spacing >= 8, so at most
  log2(8192) - 2 levels)."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _define(path, pattern):
    with open(os.path.join(ROOT, path)) as f:
        return int(re.search(pattern, f.read()).group(1))


SB_MAX_SIDE = _define("include/styleblit.h", r"#define SB_MAX_SIDE (\d+)")
SB_MAX_LEVELS = _define("include/styleblit.h", r"#define SB_MAX_LEVELS (\d+)")
EX_MARGIN = _define("paper_1807_03249_amd/csrc/sb_internal.h", r"kExMargin = (\d+);")


def test_record_index_split():
    j = np.arange(128)
    assert np.array_equal((j * 57) >> 9, j // 9)
    assert 9 * SB_MAX_LEVELS <= 128
    k = np.arange(9)
    kx = (k * 11) >> 5
    assert np.array_equal(kx, k // 3)
    assert np.array_equal(k - 3 * kx, k % 3)


def test_cells_per_axis_by_shift():
    n = np.arange(1, SB_MAX_SIDE + 1)
    for s in range(0, SB_MAX_SIDE.bit_length()):
        assert np.array_equal(((n - 1) >> s) + 1, -(-n // (1 << s))), s


def test_index_products_fit_24_bit_multiplies():
    padded = SB_MAX_SIDE + 2 * EX_MARGIN + 2  # exemplar row with margins (and slack)
    assert padded < (1 << 24)
    assert (SB_MAX_SIDE - 1) * SB_MAX_SIDE + SB_MAX_SIDE - 1 < (1 << 26)
    # the vote's output byte offset 3 * (y * w + x) stays below 2^32
    assert 3 * (SB_MAX_SIDE * SB_MAX_SIDE) < (1 << 32)
    # signed offsets times the row length fit the signed 24-bit multiply
    assert SB_MAX_SIDE * padded < (1 << 31)


def _stylize_constant(name):
    return _define("paper_1807_03249_amd/csrc/stylize.hip", r"constexpr int32_t " + name +
                   r" = (\d+);")


def test_empty_neighbourhood_slot_stays_in_block_records():
    stride = _stylize_constant("kRecStride")
    wave_recs = SB_MAX_LEVELS * stride
    assert stride >= 9
    # the block path needs log2(finest) >= 3 and log2(finest) + L - 1 <= log2(SB_MAX_SIDE)
    max_levels = SB_MAX_SIDE.bit_length() - 1 - 3 + 1
    assert max_levels <= SB_MAX_LEVELS
    last_slot = stride * (max_levels - 1) + (0x7FFFFFFF & 15)
    assert last_slot < wave_recs
