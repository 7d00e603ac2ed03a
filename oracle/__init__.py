"""CPU oracle for StyleBlit's guided chunk transfer -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes + numpy) to ``styleblit_oracle.c``, the plain C
implementation of the lookup table (Sec. 3.1), the seed hierarchy and
per-pixel level loop (Sec. 3.2, Algorithm 2) and the voting blend (end of
Sec. 3.2).  Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
CPU-baseline leg may import this package; the HIP library never does, and
nothing here imports the HIP library.

Parity pins (all in ``tests/test_oracle_*.py``, CPU only): brute-force
argmin for the lookup table, the closed form of identity UV guides, seed
positions against the jitter table read directly, hand-worked 8x8 cases
(``tests/golden/``), texture mapping as the threshold-0 special case and
the paper's invariants (identity guide reproduces the source, larger
threshold never picks a finer level, chunks are pure translations, every
accepted pixel has error below the threshold).  The segmentation-guide
variant (per-label tables, the label constraint in the level loop) is pinned
by its reduction to the plain path with one label, brute-force per-label
tables, a hand-worked case and its label invariants
(``tests/test_oracle_seg.py``).  The animation extension (Sec. 3.3) adds
no arithmetic of its own: a sequence is frames of the plain path with a
per-frame jitter table, and ``frame_change`` counts the pixels that changed
between two of them; ``tests/test_oracle_animation.py`` pins the paper's
statements about it (seeds that do not move leave a static target
unchanged, threshold 0 makes the result independent of the seeds, a larger
threshold changes more pixels) and checks the counts by brute force.
Three-channel guides (format 2, the additional guiding channels of
Sec. 3.1) are pinned in ``tests/test_oracle_channels.py``: the table against
an independent vectorised argmin and a full-coverage closed form, the
reduction to the two-channel path when the third channel is constant, an
adversarial third channel that alone decides acceptance, and the level
loop's invariants with the three-channel error.  Channel weights (the
strong or weak appearance guide) are pinned by a weighted vectorised argmin,
a zero weight that reduces the path to the first two channels, and uniform
weights that only rescale the threshold.  Guides of 2..8 channels of 8 or 16 bits
(formats 3 and 4, each lookup an exact nearest-pixel search, the search the
paper suggests for additional channels) are pinned in
``tests/test_oracle_search.py``: the lookup against the pinned two- and
three-channel tables, a closed form with ties at 16 bits, zero-weight
channel removal and channel permutations, the channel-0 sweep against brute
force; the level loop against the pinned two- and three-channel paths,
texture mapping at t = 0, a translation with a closed-form NNF, and its
invariants.  The counter-based jitter
generator (Philox4x64-10, from its published definition) is pinned block for
block against numpy's own Philox bit generator (``tests/test_oracle_rng.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "styleblit_oracle.c")
_LIB = os.path.join(_HERE, "libstyleblit_oracle.so")
_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build() -> str:
    """Compile the oracle with gcc (-O2, OpenMP over rows)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC],
                   check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    vp = ctypes.c_void_p
    i32 = ctypes.c_int
    lib.ora_lut_build.argtypes = [vp, i32, i32, i32, i32, _u32p]
    lib.ora_jitter_len.argtypes = [i32, i32, i32, i32]
    lib.ora_jitter_len.restype = ctypes.c_int64
    lib.ora_seed_point.argtypes = [i32, i32, i32, i32, _u32p, i32, ctypes.c_int64, ctypes.c_int64,
                                   _i64p, _i64p]
    lib.ora_nearest_seed.argtypes = [i32, i32, i32, i32, _u32p, i32, ctypes.c_int64,
                                     ctypes.c_int64, _i64p, _i64p]
    lib.ora_assign.argtypes = [vp, i32, i32, _u32p, i32, i32, vp, i32, i32, _u32p, i32, i32,
                               ctypes.c_uint32, _u32p, _u32p, ctypes.c_int64, ctypes.c_int64]
    lib.ora_blend.argtypes = [_u8p, i32, i32, _u32p, i32, i32, i32, _u8p, ctypes.c_int64,
                              ctypes.c_int64]
    lib.ora_stylize.argtypes = [_u8p, vp, i32, i32, _u32p, i32, i32, vp, i32, i32, _u32p, i32,
                                i32, ctypes.c_uint32, i32, _u8p, _u32p, _u32p]
    lib.ora_lut_build_labels.argtypes = [vp, _u8p, i32, i32, i32, i32, i32, _u32p]
    lib.ora_lut_query.argtypes = [vp, i32, i32, i32, i32, _i64p, ctypes.c_int64, _u32p]
    lib.ora_set_threads.argtypes = [i32]
    _u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.ora_philox4x64.argtypes = [_u64p, _u64p, _u64p]
    lib.ora_jitter_fill.argtypes = [i32, i32, i32, i32, ctypes.c_uint64, ctypes.c_uint64, _u32p]
    lib.ora_jitter_hash.argtypes = [i32, i32, i32, i32, ctypes.c_uint32, _u32p]
    lib.ora_jitter_hash_key.argtypes = [ctypes.c_uint32] * 4
    lib.ora_jitter_hash_key.restype = ctypes.c_uint32
    lib.ora_lut_build_w.argtypes = [vp, i32, i32, i32, i32, _u8p, _u32p]
    lib.ora_lut_query_w.argtypes = [vp, i32, i32, i32, i32, _u8p, _i64p, ctypes.c_int64, _u32p]
    lib.ora_lut_query_sweep_w.argtypes = [vp, i32, i32, i32, i32, _u8p, _i64p, ctypes.c_int64,
                                          _u32p]
    lib.ora_lut_build_labels_w.argtypes = [vp, _u8p, i32, i32, i32, i32, i32, _u8p, _u32p]
    lib.ora_assign_w.argtypes = [vp, i32, i32, _u32p, i32, i32, _u8p, vp, i32, i32, _u32p, i32,
                                 i32, ctypes.c_uint32, _u32p, _u32p, ctypes.c_int64,
                                 ctypes.c_int64]
    lib.ora_stylize_w.argtypes = [_u8p, vp, i32, i32, _u32p, i32, i32, _u8p, vp, i32, i32, _u32p,
                                  i32, i32, ctypes.c_uint32, i32, _u8p, _u32p, _u32p]
    lib.ora_stylize_seg_w.argtypes = [_u8p, vp, _u8p, i32, i32, _u32p, i32, i32, i32, _u8p, vp,
                                      _u8p, i32, i32, _u32p, i32, i32, ctypes.c_uint32, i32,
                                      _u8p, _u32p, _u32p]
    lib.ora_stylize_seg.argtypes = [_u8p, vp, _u8p, i32, i32, _u32p, i32, i32, i32, vp, _u8p,
                                    i32, i32, _u32p, i32, i32, ctypes.c_uint32, i32, _u8p, _u32p,
                                    _u32p]
    lib.ora_texel_bytes.argtypes = [i32, i32]
    lib.ora_nn_query_n.argtypes = [vp, i32, i32, i32, i32, _u8p, vp, ctypes.c_int64, _u32p]
    lib.ora_nn_sweep_n.argtypes = [vp, i32, i32, i32, i32, _u8p, vp, ctypes.c_int64, _u32p]
    lib.ora_assign_n.argtypes = [vp, i32, i32, i32, i32, _u8p, vp, i32, i32, _u32p, i32, i32,
                                 ctypes.c_uint32, _u32p, _u32p]
    lib.ora_stylize_n.argtypes = [_u8p, vp, i32, i32, i32, i32, _u8p, vp, i32, i32, _u32p, i32,
                                  i32, ctypes.c_uint32, i32, _u8p, _u32p, _u32p]
    _lib = lib
    return lib


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _guide(g: np.ndarray) -> Tuple[np.ndarray, int]:
    """Guide bytes and format: (rows, cols, 2) uint8 -> 0, (rows, cols, 2)
    uint16 -> 1, (rows, cols, 4) uint8 -> 2 (three channels, byte 3
    ignored)."""
    g = np.ascontiguousarray(g)
    if g.ndim == 3 and g.shape[2] == 4 and g.dtype == np.uint8:
        return g, 2
    if g.ndim != 3 or g.shape[2] != 2:
        raise ValueError("guide must be (rows, cols, 2), or (rows, cols, 4) uint8")
    if g.dtype == np.uint8:
        return g, 0
    if g.dtype == np.uint16:
        return g, 1
    raise ValueError("guide must be uint8 or uint16")


def _bins(fmt: int, lut_bits: int) -> int:
    return 1 << ((3 if fmt == 2 else 2) * lut_bits)


def _weights(weights):
    """Channel weights as a ctypes pointer (None: unit weights)."""
    if weights is None:
        return None, None
    w = np.ascontiguousarray(weights, dtype=np.uint8)
    if w.size != 3:
        raise ValueError("weights must hold three values")
    return w, _ptr(w, _u8p)


def _jit(jitter: Optional[np.ndarray], w: int, h: int, levels: int, finest: int,
         seed: Optional[int] = None) -> np.ndarray:
    """The jitter table a frame uses: ``jitter`` as given; else, with a
    ``seed``, the table the integer hash defines; else all zero (seeds on the
    cell corners)."""
    n = jitter_len(w, h, levels, finest)
    if jitter is None and seed is not None:
        return jitter_hash(w, h, levels, finest, seed) if n else np.zeros(1, np.uint32)
    if jitter is None:
        return np.zeros(max(n, 1), np.uint32)
    j = np.ascontiguousarray(jitter, dtype=np.uint32)
    if j.size != n:
        raise ValueError(f"jitter table has {j.size} entries, expected {n}")
    return j if n else np.zeros(1, np.uint32)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops (n <= 0: unchanged); returns the
    number in effect.  Timing only: results do not depend on it."""
    return int(_load().ora_set_threads(int(n)))


def philox4x64(key, counter) -> np.ndarray:
    """One Philox4x64-10 block: four uint64 words for a 2-word key and a
    4-word counter."""
    k = np.ascontiguousarray(key, dtype=np.uint64)
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    p = ctypes.POINTER(ctypes.c_uint64)
    _load().ora_philox4x64(k.ctypes.data_as(p), c.ctypes.data_as(p), out.ctypes.data_as(p))
    return out


def jitter_fill(w: int, h: int, levels: int, finest: int, seed: int, stream: int = 0) -> np.ndarray:
    """The jitter table drawn from Philox4x64-10 under key (seed, stream):
    entry e takes word 0 of block (e, 0, 0, 0), jx / jy from its low / high
    half modulo the level's spacing."""
    n = jitter_len(w, h, levels, finest)
    out = np.zeros(max(n, 1), np.uint32)
    _check(_load().ora_jitter_fill(w, h, levels, finest, seed, stream, _ptr(out, _u32p)),
           "jitter_fill")
    return out[:n]


def jitter_hash(w: int, h: int, levels: int, finest: int, seed: int) -> np.ndarray:
    """The jitter table defined by the integer hash of (cell, log2 h, seed)
    (the reading of RandomJitterTable used when a frame names a seed instead
    of passing a table)."""
    n = jitter_len(w, h, levels, finest)
    out = np.zeros(max(n, 1), np.uint32)
    _check(_load().ora_jitter_hash(w, h, levels, finest, int(seed) & 0xFFFFFFFF,
                                   _ptr(out, _u32p)), "jitter_hash")
    return out[:n]


def jitter_hash_key(seed: int, log2h: int, bx: int, by: int) -> int:
    """The 32-bit hash k of one cell (jx = k & (h-1), jy = (k >> 16) & (h-1))."""
    return int(_load().ora_jitter_hash_key(int(seed) & 0xFFFFFFFF, log2h, bx & 0xFFFFFFFF,
                                           by & 0xFFFFFFFF))


def jitter_len(w: int, h: int, levels: int, finest: int) -> int:
    return int(_load().ora_jitter_len(w, h, levels, finest))


def lut_build(src_guide: np.ndarray, lut_bits: int, weights=None) -> np.ndarray:
    """Exact lookup table, (2**lut_bits)**2 entries ((2**lut_bits)**3 for
    three-channel guides), entries x | y << 16.  ``weights``: three channel
    weights 0..127 of a three-channel guide (None: unit)."""
    g, fmt = _guide(src_guide)
    lut = np.zeros(_bins(fmt, lut_bits), np.uint32)
    w, wp = _weights(weights)
    _check(_load().ora_lut_build_w(g.ctypes.data, fmt, g.shape[1], g.shape[0], lut_bits, wp,
                                   _ptr(lut, _u32p)), "lut_build")
    return lut


def lut_query(src_guide: np.ndarray, lut_bits: int, bins, weights=None) -> np.ndarray:
    """Selected entries of the lookup table, each by brute force over every
    source pixel (for sampling tables too large to build here)."""
    g, fmt = _guide(src_guide)
    b = np.ascontiguousarray(bins, dtype=np.int64)
    out = np.zeros(b.size, np.uint32)
    w, wp = _weights(weights)
    _check(_load().ora_lut_query_w(g.ctypes.data, fmt, g.shape[1], g.shape[0], lut_bits, wp,
                                   _ptr(b, _i64p), b.size, _ptr(out, _u32p)), "lut_query")
    return out


def lut_query_sweep(src_guide: np.ndarray, lut_bits: int, bins, weights=None) -> np.ndarray:
    """The same entries as ``lut_query``, visiting the source pixels outward
    along channel 0 from each bin centre and stopping once that channel
    alone rules out every pixel not yet seen (for the many bins one large
    frame touches)."""
    g, fmt = _guide(src_guide)
    b = np.ascontiguousarray(bins, dtype=np.int64)
    out = np.zeros(b.size, np.uint32)
    w, wp = _weights(weights)
    _check(_load().ora_lut_query_sweep_w(g.ctypes.data, fmt, g.shape[1], g.shape[0], lut_bits,
                                         wp, _ptr(b, _i64p), b.size, _ptr(out, _u32p)),
           "lut_query_sweep")
    return out


def seed_point(w, h, levels, finest, jitter, level, bx, by, seed=None):
    """(valid, sx, sy) of cell (bx, by) at level `level` (``jitter`` None with a
    ``seed``: the hash-defined table)."""
    j = _jit(jitter, w, h, levels, finest, seed)
    sx, sy = ctypes.c_int64(), ctypes.c_int64()
    ok = _load().ora_seed_point(w, h, levels, finest, _ptr(j, _u32p), level, bx, by,
                                ctypes.byref(sx), ctypes.byref(sy))
    return bool(ok), sx.value, sy.value


def nearest_seed(w, h, levels, finest, jitter, level, px, py, seed=None):
    """(found, qx, qy) for pixel (px, py) at level `level`."""
    j = _jit(jitter, w, h, levels, finest, seed)
    qx, qy = ctypes.c_int64(-1), ctypes.c_int64(-1)
    ok = _load().ora_nearest_seed(w, h, levels, finest, _ptr(j, _u32p), level, px, py,
                                  ctypes.byref(qx), ctypes.byref(qy))
    return bool(ok), qx.value, qy.value


def assign(src_guide, lut, lut_bits, tgt_guide, jitter, levels, finest, threshold,
           rows: Optional[Tuple[int, int]] = None, weights=None, seed=None):
    """Per-pixel level loop only: returns (nnf, chunk), both uint32 (H, W).
    With ``rows=(row0, n)`` only those rows are computed (others stay 0)."""
    gs, fmt = _guide(src_guide)
    gt, fmt_t = _guide(tgt_guide)
    if fmt != fmt_t:
        raise ValueError("source and target guide formats differ")
    h, w = gt.shape[:2]
    j = _jit(jitter, w, h, levels, finest, seed)
    lut = np.ascontiguousarray(lut, dtype=np.uint32)
    if lut.size != _bins(fmt, lut_bits):
        raise ValueError("lookup table size does not match the guide format and lut_bits")
    nnf = np.zeros((h, w), np.uint32)
    chunk = np.zeros((h, w), np.uint32)
    r0, nr = rows if rows is not None else (0, -1)
    wt, wp = _weights(weights)
    _check(_load().ora_assign_w(gs.ctypes.data, gs.shape[1], gs.shape[0], _ptr(lut, _u32p), fmt,
                                lut_bits, wp, gt.ctypes.data, w, h, _ptr(j, _u32p), levels,
                                finest, threshold, _ptr(nnf, _u32p), _ptr(chunk, _u32p), r0, nr),
           "assign")
    return nnf, chunk


def blend(src_rgb: np.ndarray, nnf: np.ndarray, radius: int,
          rows: Optional[Tuple[int, int]] = None) -> np.ndarray:
    """Voting blend of an NNF (uint32 (H, W), x | y << 16) -> uint8 (H, W, 3)."""
    rgb = np.ascontiguousarray(src_rgb, dtype=np.uint8)
    nnf = np.ascontiguousarray(nnf, dtype=np.uint32)
    h, w = nnf.shape
    out = np.zeros((h, w, 3), np.uint8)
    r0, nr = rows if rows is not None else (0, -1)
    _check(_load().ora_blend(_ptr(rgb, _u8p), rgb.shape[1], rgb.shape[0], _ptr(nnf, _u32p), w, h,
                             radius, _ptr(out, _u8p), r0, nr), "blend")
    return out


def stylize(src_rgb, src_guide, lut, lut_bits, tgt_guide, jitter, levels, finest, threshold,
            radius, weights=None, seed=None):
    """The whole per-frame path: returns (rgb (H,W,3) uint8, chunk (H,W) uint32,
    nnf (H,W) uint32).  ``jitter``: the jitter table, or None for the table the
    integer hash of ``seed`` defines (None too: seeds on the cell corners).  ``weights``: channel weights of a three-channel guide
    (the table must be built with the same weights)."""
    gs, fmt = _guide(src_guide)
    gt, fmt_t = _guide(tgt_guide)
    if fmt != fmt_t:
        raise ValueError("source and target guide formats differ")
    rgb = np.ascontiguousarray(src_rgb, dtype=np.uint8)
    h, w = gt.shape[:2]
    j = _jit(jitter, w, h, levels, finest, seed)
    lut = np.ascontiguousarray(lut, dtype=np.uint32)
    if lut.size != _bins(fmt, lut_bits):
        raise ValueError("lookup table size does not match the guide format and lut_bits")
    out = np.zeros((h, w, 3), np.uint8)
    chunk = np.zeros((h, w), np.uint32)
    nnf = np.zeros((h, w), np.uint32)
    wt, wp = _weights(weights)
    _check(_load().ora_stylize_w(_ptr(rgb, _u8p), gs.ctypes.data, gs.shape[1], gs.shape[0],
                                 _ptr(lut, _u32p), fmt, lut_bits, wp, gt.ctypes.data, w, h,
                                 _ptr(j, _u32p), levels, finest, threshold, radius,
                                 _ptr(out, _u8p), _ptr(chunk, _u32p), _ptr(nnf, _u32p)),
           "stylize")
    return out, chunk, nnf


def _labels(lab: np.ndarray, shape) -> np.ndarray:
    lab = np.ascontiguousarray(lab, dtype=np.uint8)
    if lab.shape != tuple(shape):
        raise ValueError(f"label map has shape {lab.shape}, expected {tuple(shape)}")
    return lab


def lut_build_labels(src_guide: np.ndarray, src_labels: np.ndarray, nlabels: int,
                     lut_bits: int, weights=None) -> np.ndarray:
    """Per-label lookup tables (segmentation guide), shape (nlabels, bins):
    table l from the source pixels labelled l; a label without source pixels
    gets the unconstrained table."""
    g, fmt = _guide(src_guide)
    lab = _labels(src_labels, g.shape[:2])
    luts = np.zeros((nlabels, _bins(fmt, lut_bits)), np.uint32)
    w, wp = _weights(weights)
    _check(_load().ora_lut_build_labels_w(g.ctypes.data, _ptr(lab, _u8p), nlabels, fmt,
                                          g.shape[1], g.shape[0], lut_bits, wp,
                                          _ptr(luts, _u32p)), "lut_build_labels")
    return luts


def stylize_seg(src_rgb, src_guide, src_labels, luts, nlabels, lut_bits, tgt_guide, tgt_labels,
                jitter, levels, finest, threshold, radius, weights=None, seed=None):
    """The per-frame path with the segmentation guide as a hard constraint:
    returns (rgb, chunk, nnf) as ``stylize``."""
    gs, fmt = _guide(src_guide)
    gt, fmt_t = _guide(tgt_guide)
    if fmt != fmt_t:
        raise ValueError("source and target guide formats differ")
    ls = _labels(src_labels, gs.shape[:2])
    lt = _labels(tgt_labels, gt.shape[:2])
    rgb = np.ascontiguousarray(src_rgb, dtype=np.uint8)
    h, w = gt.shape[:2]
    j = _jit(jitter, w, h, levels, finest, seed)
    luts = np.ascontiguousarray(luts, dtype=np.uint32)
    if luts.size != nlabels * _bins(fmt, lut_bits):
        raise ValueError("luts must hold nlabels tables")
    out = np.zeros((h, w, 3), np.uint8)
    chunk = np.zeros((h, w), np.uint32)
    nnf = np.zeros((h, w), np.uint32)
    wt, wp = _weights(weights)
    _check(_load().ora_stylize_seg_w(_ptr(rgb, _u8p), gs.ctypes.data, _ptr(ls, _u8p),
                                     gs.shape[1], gs.shape[0], _ptr(luts, _u32p), nlabels, fmt,
                                     lut_bits, wp, gt.ctypes.data, _ptr(lt, _u8p), w, h,
                                     _ptr(j, _u32p), levels, finest, threshold, radius,
                                     _ptr(out, _u8p), _ptr(chunk, _u32p), _ptr(nnf, _u32p)),
           "stylize_seg")
    return out, chunk, nnf


def decode_chunk(chunk: np.ndarray):
    """(level, qx, qy) arrays from chunk codes (level << 26 | qy << 13 | qx)."""
    c = np.asarray(chunk, dtype=np.uint32)
    return (c >> 26).astype(np.int64), (c & 0x1FFF).astype(np.int64), ((c >> 13) & 0x1FFF).astype(np.int64)


def frame_change(chunk_a, chunk_b, nnf_a=None, nnf_b=None) -> Tuple[int, int]:
    """Frame-to-frame change of an animation (Sec. 3.3, extension to
    animation): (pixels whose chunk code differs, pixels whose source
    coordinate differs; 0 without NNF maps).  The definition, written out."""
    a = np.asarray(chunk_a).view(np.uint32).ravel()
    b = np.asarray(chunk_b).view(np.uint32).ravel()
    if a.shape != b.shape:
        raise ValueError("frames differ in size")
    code = int(np.count_nonzero(a != b))
    if nnf_a is None:
        return code, 0
    na = np.asarray(nnf_a).view(np.uint32).ravel()
    nb = np.asarray(nnf_b).view(np.uint32).ravel()
    if na.shape != a.shape or nb.shape != a.shape:
        raise ValueError("frames differ in size")
    return code, int(np.count_nonzero(na != nb))


# ----------------------------------------------- guides of many channels

def texel_bytes(depth: int, channels: int) -> int:
    """Bytes per texel of a ``channels``-channel guide of ``depth`` bits (4, 8
    or 16: the smallest that holds them); 0 if invalid."""
    return int(_load().ora_texel_bytes(depth, channels))


def _guide_n(g: np.ndarray, channels: int) -> Tuple[np.ndarray, int]:
    """Texels of a many-channel guide and its depth: (rows, cols, E) uint8
    or uint16 with E elements per texel, E * element bytes = the texel size
    of ``channels`` channels (elements past ``channels`` are ignored)."""
    g = np.ascontiguousarray(g)
    if g.ndim != 3 or g.dtype not in (np.uint8, np.uint16):
        raise ValueError("a many-channel guide is (rows, cols, elements) uint8 or uint16")
    depth = 8 * g.dtype.itemsize
    tb = texel_bytes(depth, channels)
    if tb == 0 or g.shape[2] * g.dtype.itemsize != tb:
        raise ValueError(f"{channels} channels of {depth} bits need {tb}-byte texels")
    return g, depth


def _weights_n(weights, channels: int):
    if weights is None:
        return None, None
    w = np.zeros(8, np.uint8)
    v = np.asarray(weights, dtype=np.int64).ravel()
    if v.size != channels or v.min() < 0 or v.max() > 255:
        raise ValueError(f"weights must hold {channels} values")
    w[:channels] = v
    return w, _ptr(w, _u8p)


def nn_query_n(src_guide, channels: int, queries, weights=None) -> np.ndarray:
    """Exact lookups of query texels ((..., E) in the guide's layout) by brute
    force over every source pixel: the argmin of sum_k w_k (q_k - G_S[u]_k)^2,
    ties to the smallest raster index.  Returns x | y << 16 per query."""
    gs, depth = _guide_n(src_guide, channels)
    q = np.ascontiguousarray(queries, dtype=gs.dtype).reshape(-1, gs.shape[2])
    out = np.zeros(q.shape[0], np.uint32)
    w, wp = _weights_n(weights, channels)
    _check(_load().ora_nn_query_n(gs.ctypes.data, depth, channels, gs.shape[1], gs.shape[0], wp,
                                 q.ctypes.data, q.shape[0], _ptr(out, _u32p)), "nn_query_n")
    return out


def nn_sweep_n(src_guide, channels: int, queries, weights=None) -> np.ndarray:
    """The same lookups as ``nn_query_n``, walking the source pixels outward
    along channel 0 with an exact stopping bound."""
    gs, depth = _guide_n(src_guide, channels)
    q = np.ascontiguousarray(queries, dtype=gs.dtype).reshape(-1, gs.shape[2])
    out = np.zeros(q.shape[0], np.uint32)
    w, wp = _weights_n(weights, channels)
    _check(_load().ora_nn_sweep_n(gs.ctypes.data, depth, channels, gs.shape[1], gs.shape[0], wp,
                                  q.ctypes.data, q.shape[0], _ptr(out, _u32p)), "nn_sweep_n")
    return out


def assign_n(src_guide, channels: int, tgt_guide, jitter, levels, finest, threshold,
             weights=None, seed=None):
    """Level loop with a many-channel guide (exact search lookups): returns
    (nnf, chunk), both uint32 (H, W)."""
    gs, depth = _guide_n(src_guide, channels)
    gt, depth_t = _guide_n(tgt_guide, channels)
    if depth != depth_t:
        raise ValueError("source and target guide depths differ")
    h, w = gt.shape[:2]
    j = _jit(jitter, w, h, levels, finest, seed)
    nnf = np.zeros((h, w), np.uint32)
    chunk = np.zeros((h, w), np.uint32)
    wt, wp = _weights_n(weights, channels)
    _check(_load().ora_assign_n(gs.ctypes.data, gs.shape[1], gs.shape[0], depth, channels, wp,
                                gt.ctypes.data, w, h, _ptr(j, _u32p), levels, finest, threshold,
                                _ptr(nnf, _u32p), _ptr(chunk, _u32p)), "assign_n")
    return nnf, chunk


def stylize_n(src_rgb, src_guide, channels: int, tgt_guide, jitter, levels, finest, threshold,
              radius, weights=None, seed=None):
    """The whole per-frame path with a many-channel guide: returns (rgb,
    chunk, nnf) as ``stylize``."""
    gs, depth = _guide_n(src_guide, channels)
    gt, depth_t = _guide_n(tgt_guide, channels)
    if depth != depth_t:
        raise ValueError("source and target guide depths differ")
    rgb = np.ascontiguousarray(src_rgb, dtype=np.uint8)
    h, w = gt.shape[:2]
    j = _jit(jitter, w, h, levels, finest, seed)
    out = np.zeros((h, w, 3), np.uint8)
    chunk = np.zeros((h, w), np.uint32)
    nnf = np.zeros((h, w), np.uint32)
    wt, wp = _weights_n(weights, channels)
    _check(_load().ora_stylize_n(_ptr(rgb, _u8p), gs.ctypes.data, gs.shape[1], gs.shape[0], depth,
                                 channels, wp, gt.ctypes.data, w, h, _ptr(j, _u32p), levels,
                                 finest, threshold, radius, _ptr(out, _u8p), _ptr(chunk, _u32p),
                                 _ptr(nnf, _u32p)), "stylize_n")
    return out, chunk, nnf
