"""The oracle's counter-based jitter generator (Philox4x64-10 from its
published definition) pinned against numpy's own Philox bit generator, and
the jitter tables drawn from it: entries recomputed from numpy's outputs,
values inside every cell, uniform per level."""
import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1


def numpy_block(key, counter):
    """numpy's Philox advances its 256-bit counter before each block: the
    block at counter c comes first from a generator started at c - 1."""
    c = sum(int(v) << (64 * i) for i, v in enumerate(counter))
    c = (c - 1) % (1 << 256)
    start = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    return np.random.Philox(key=np.asarray(key, dtype=np.uint64), counter=start).random_raw(4)


@pytest.mark.parametrize("key,counter", [
    ((0, 0), (0, 0, 0, 0)),
    ((1, 2), (1, 0, 0, 0)),
    ((0xFFFFFFFFFFFFFFFF, 7), (5, 0, 0, 0)),
    ((12345, 67890), (0, 1, 0, 0)),
    ((3, 4), (0xFFFFFFFFFFFFFFFF, 3, 9, 0)),
    ((0xDEADBEEF, 0xC0FFEE), (123456789, 0, 0, 0xFFFFFFFFFFFFFFFF)),
])
def test_philox_block_matches_numpy(key, counter):
    np.testing.assert_array_equal(oracle.philox4x64(key, counter), numpy_block(key, counter))


@pytest.mark.parametrize("w,h,levels,finest,seed,stream", [
    (64, 48, 3, 4, 1, 0), (97, 33, 4, 2, 2**63 + 5, 9), (200, 136, 4, 8, 77, 3), (5, 7, 1, 1, 0, 0)])
def test_jitter_fill_from_numpy_outputs(w, h, levels, finest, seed, stream):
    got = oracle.jitter_fill(w, h, levels, finest, seed, stream)
    assert got.size == oracle.jitter_len(w, h, levels, finest)
    e = 0
    for i in range(levels):
        sp = finest << (levels - 1 - i)
        n = ((w + sp - 1) // sp) * ((h + sp - 1) // sp)
        for _ in range(n):
            word = int(numpy_block((seed, stream), (e, 0, 0, 0))[0])
            want = (word & (sp - 1)) | (((word >> 32) & (sp - 1)) << 16)
            assert int(got[e]) == want, (i, e)
            e += 1
    assert e == got.size


def test_jitter_fill_is_uniform_and_inside_cells():
    w, h, levels, finest = 1920, 1080, 4, 8
    j = oracle.jitter_fill(w, h, levels, finest, 2024, 1)
    off = 0
    for i in range(levels):
        sp = finest << (levels - 1 - i)
        n = ((w + sp - 1) // sp) * ((h + sp - 1) // sp)
        jx = j[off:off + n] & 0xFFFF
        jy = j[off:off + n] >> 16
        assert jx.max() < sp and jy.max() < sp
        if n >= 20 * sp:  # chi-squared over sp bins, far beyond the 1e-6 tail
            for v in (jx, jy):
                cnt = np.bincount(v, minlength=sp)
                chi2 = ((cnt - n / sp) ** 2 / (n / sp)).sum()
                assert chi2 < sp + 10 * np.sqrt(2 * sp) + 30, (i, chi2)
        off += n
    assert not np.array_equal(j, oracle.jitter_fill(w, h, levels, finest, 2024, 2))
    assert not np.array_equal(j, oracle.jitter_fill(w, h, levels, finest, 2025, 1))
    np.testing.assert_array_equal(j, oracle.jitter_fill(w, h, levels, finest, 2024, 1))
