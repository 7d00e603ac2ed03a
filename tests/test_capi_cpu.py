"""The C-ABI library loads and exports every function include/styleblit.h
declares; host-only entry points and argument validation (no compute calls,
no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "styleblit.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_1807_03249_amd as sb

    if not os.path.exists(sb.LIB_PATH):
        from paper_1807_03249_amd import build

        build.build()
    return sb.lib()


def test_exports_every_declared_symbol(L):
    import paper_1807_03249_amd as sb

    names = declared()
    assert len(names) >= 9
    out = subprocess.run(["nm", "-D", "--defined-only", sb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sb_[a-z0-9_]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert getattr(L, n) is not None


def test_host_helpers(L):
    import paper_1807_03249_amd as sb
    import oracle

    assert L.sb_version().startswith(b"styleblit")
    for w, h, lv, f in [(256, 256, 3, 8), (1920, 1080, 4, 8), (3840, 2160, 5, 8), (37, 5, 3, 1),
                        (1, 1, 0, 8), (8192, 3, 1, 8192)]:
        assert sb.jitter_len(w, h, lv, f) == oracle.jitter_len(w, h, lv, f)
    assert L.sb_jitter_len(0, 5, 1, 8) == -1
    assert L.sb_jitter_len(8193, 5, 1, 8) == -1
    assert L.sb_jitter_len(8, 8, 13, 1) == -1
    assert L.sb_jitter_len(8, 8, 2, 3) == -1          # finest not a power of two
    assert L.sb_jitter_len(8, 8, 3, 4096) == -1       # coarsest spacing 16384 > 8192
    assert sb.status_string(-1) == "invalid argument"


def test_workspace_sizes(L):
    import paper_1807_03249_amd as sb

    p = sb.params(4, 8, 32, 3)
    n = sb.workspace_bytes(1920, 1080, p)
    assert n >= 1920 * 1080 * 4 + sb.jitter_len(1920, 1080, 4, 8) * 8
    assert L.sb_workspace_bytes(1920, 1080, ctypes.byref(sb.params(4, 8, 32, 8))) == 0  # r > 7
    # 8-bit guides: the separable build's key grids, independent of the source size
    assert L.sb_lut_workspace_bytes(0, 512, 512, 8) == 256 * 256 * 8 + 256 * 256 * 4
    assert L.sb_lut_workspace_bytes(0, 7, 3, 8) == 256 * 256 * 8 + 256 * 256 * 4
    assert L.sb_lut_workspace_bytes(2, 512, 512, 8) == 2 * (128 << 20)
    assert L.sb_lut_workspace_bytes(2, 512, 512, 4) == (256 * 256 * 16 * 8 + (64 << 20))
    assert L.sb_lut_workspace_bytes(0, 512, 512, 9) == 0  # 9 bits from an 8-bit guide
    assert L.sb_lut_workspace_bytes(2, 512, 512, 9) == 0
    assert L.sb_lut_workspace_bytes(1, 512, 512, 13) == 0
    assert L.sb_lut_workspace_bytes(1, 512, 512, 11) >= 512 * 512 * 8
    assert L.sb_lut_workspace_bytes(3, 512, 512, 8) == 0  # no such format


def test_validation_rejects_before_launch(L):
    """Bad arguments return SB_EINVAL / SB_ENOMEM from host checks; nothing is
    enqueued, so this runs without a GPU."""
    import paper_1807_03249_amd as sb

    fake = 0x1000  # never dereferenced: validation fails first
    st = sb.SbStyle(fake, fake, fake, 512, 512, 0, 8)
    p = sb._with_table(sb.params(4, 8, 32, 3))  # the jitter table argument is read
    ws = sb.workspace_bytes(64, 64, p)

    def call(style=st, g=fake, w=64, h=64, j=fake, prm=p, rgb=fake, chunk=fake, wsb=ws):
        return L.sb_stylize(ctypes.byref(style) if style is not None else None, g, w, h, j,
                            ctypes.byref(prm) if prm is not None else None, rgb, chunk, None,
                            fake, wsb, None)

    assert call(g=None) == sb.SB_EINVAL
    assert call(rgb=None) == sb.SB_EINVAL
    assert call(chunk=None) == sb.SB_EINVAL
    assert call(j=None) == sb.SB_EINVAL  # SB_JITTER_TABLE without a table
    bad_mode = sb.params(4, 8, 32, 3)
    bad_mode.jitter = 3
    assert call(prm=bad_mode) == sb.SB_EINVAL
    assert L.sb_workspace_bytes(64, 64, ctypes.byref(bad_mode)) == 0
    assert call(prm=None) == sb.SB_EINVAL
    assert call(style=None) == sb.SB_EINVAL
    assert call(w=0) == sb.SB_EINVAL
    assert call(h=8193) == sb.SB_EINVAL
    assert call(prm=sb.params(13, 8, 32, 3)) == sb.SB_EINVAL
    assert call(prm=sb.params(2, 6, 32, 3)) == sb.SB_EINVAL
    assert call(prm=sb.params(2, 8, 32, -1)) == sb.SB_EINVAL
    assert call(prm=sb.params(2, 8, 32, 8)) == sb.SB_EINVAL
    assert call(style=sb.SbStyle(fake, fake, fake, 512, 512, 1, 13)) == sb.SB_EINVAL
    assert call(style=sb.SbStyle(fake, fake, fake, 512, 512, 0, 9)) == sb.SB_EINVAL
    assert call(style=sb.SbStyle(fake, fake, fake, 0, 512, 0, 8)) == sb.SB_EINVAL
    assert call(style=sb.SbStyle(None, fake, fake, 512, 512, 0, 8)) == sb.SB_EINVAL
    assert call(wsb=ws - 1) == sb.SB_ENOMEM
    assert L.sb_lut_build(fake, 0, 512, 512, 8, fake, fake, 10, None) == sb.SB_ENOMEM
    assert L.sb_lut_build(None, 0, 512, 512, 8, fake, fake, 1 << 30, None) == sb.SB_EINVAL
    assert L.sb_pack_exemplar(None, 4, 4, fake, None) == sb.SB_EINVAL


def test_tune_validation(L):
    """Unsupported kernel choices are refused on the host (no launch)."""
    import paper_1807_03249_amd as sb

    fake = 0x1000
    st = sb.SbStyle(fake, fake, fake, 512, 512, 0, 8)
    p = sb.params(4, 8, 32, 3)
    ws = sb.workspace_bytes(64, 64, p)

    def call(tune):
        return L.sb_stylize_ex(ctypes.byref(st), fake, 64, 64, fake, ctypes.byref(p), fake, fake,
                               None, fake, ws, ctypes.byref(sb.SbTune(*tune)), None)

    for bad in [(3, 16, 2), (1, 16, 2), (4, 12, 2), (4, 32, 2), (4, 16, 3), (4, 16, 1),
                (-4, 16, 2), (4, 16, 2, 3), (4, 16, 2, -1)]:
        assert call(bad) == sb.SB_EINVAL, bad
    ev = (ctypes.c_void_p * 4)()
    assert L.sb_stylize_timed(ctypes.byref(st), fake, 64, 64, fake, ctypes.byref(p), fake, fake,
                              None, fake, ws, None, ev, None) == sb.SB_EINVAL  # null events
    h = ctypes.c_void_p()
    assert L.sb_batch_create(fake, fake, 0, ctypes.byref(sb.SbTune(4, 16, 5)), 0, None,
                             ctypes.byref(h)) == sb.SB_EINVAL
    assert L.sb_batch_create(fake, fake, 0, None, 17, None, ctypes.byref(h)) == sb.SB_EINVAL
    assert L.sb_batch_create(fake, fake, 0, None, -1, None, ctypes.byref(h)) == sb.SB_EINVAL


def test_exemplar_layout(L):
    """The padded exemplar holds the source with an 8-texel margin and at
    least one voting tile of zero rows below it."""
    for sw, sh in [(512, 512), (1, 1), (17, 3), (8192, 8192)]:
        n = L.sb_exemplar_texels(sw, sh)
        P = sw + 16
        assert n % P == 0
        rows = n // P
        assert rows >= sh + 16 + 15
        # zero rows must cover a 64 x 16 tile laid out with this row length
        assert (rows - sh - 16) * P >= 15 * P + 64
    assert L.sb_exemplar_texels(0, 5) == 0
    assert L.sb_exemplar_texels(5, 8193) == 0


def test_segmentation_validation(L):
    """Label maps on one side only, bad label counts and missing tables are
    refused on the host."""
    import paper_1807_03249_amd as sb

    fake = 0x1000
    p = sb.params(4, 8, 32, 3)
    ws = sb.workspace_bytes(64, 64, p)

    def seg(style, labels=fake):
        return L.sb_stylize_seg(ctypes.byref(style), fake, labels, 64, 64, fake, ctypes.byref(p),
                                fake, fake, None, fake, ws, None, None)

    plain = sb.SbStyle(fake, fake, fake, 512, 512, 0, 8)
    labelled = sb.SbStyle(fake, fake, fake, 512, 512, 0, 8, fake, fake, 3)
    assert seg(plain) == sb.SB_EINVAL                       # style without labels
    assert seg(labelled, labels=None) == sb.SB_EINVAL       # frame without labels
    assert seg(sb.SbStyle(fake, fake, fake, 512, 512, 0, 8, None, fake, 3)) == sb.SB_EINVAL
    assert seg(sb.SbStyle(fake, fake, fake, 512, 512, 0, 8, fake, None, 3)) == sb.SB_EINVAL
    assert seg(sb.SbStyle(fake, fake, fake, 512, 512, 0, 8, fake, fake, 257)) == sb.SB_EINVAL
    assert seg(sb.SbStyle(fake, fake, fake, 512, 512, 0, 8, fake, fake, -1)) == sb.SB_EINVAL
    wsl = L.sb_lut_workspace_bytes(0, 512, 512, 8)
    assert L.sb_lut_build_labels(fake, fake, 0, 512, 512, 8, 0, fake, fake, fake, wsl,
                                 None) == sb.SB_EINVAL
    assert L.sb_lut_build_labels(fake, None, 0, 512, 512, 8, 2, fake, fake, fake, wsl,
                                 None) == sb.SB_EINVAL
    assert L.sb_lut_build_labels(fake, fake, 0, 512, 512, 8, 2, fake, fake, fake, wsl - 1,
                                 None) == sb.SB_ENOMEM


def test_channel_weight_validation(L):
    """Weights above 127, or non-unit weights on a two-channel guide, are
    refused on the host, for the table builds and for frames."""
    import paper_1807_03249_amd as sb

    fake = 0x1000
    u8x3 = (ctypes.c_uint8 * 3)
    ws3 = L.sb_lut_workspace_bytes(2, 64, 64, 4)
    ws2 = L.sb_lut_workspace_bytes(0, 64, 64, 4)
    assert L.sb_lut_build_w(fake, 2, 64, 64, 4, u8x3(1, 128, 1), fake, fake, ws3,
                            None) == sb.SB_EINVAL
    assert L.sb_lut_build_w(fake, 0, 64, 64, 4, u8x3(2, 1, 1), fake, fake, ws2,
                            None) == sb.SB_EINVAL
    assert L.sb_lut_build_labels_w(fake, fake, 2, 64, 64, 4, u8x3(200, 1, 1), 2, fake, fake,
                                   fake, ws3, None) == sb.SB_EINVAL
    # workspace checks still apply after valid weights
    assert L.sb_lut_build_w(fake, 2, 64, 64, 4, u8x3(3, 1, 7), fake, fake, ws3 - 1,
                            None) == sb.SB_ENOMEM
    p = sb.params(4, 8, 32, 3)
    ws = sb.workspace_bytes(64, 64, p)

    def frame(style):
        return L.sb_stylize(ctypes.byref(style), fake, 64, 64, fake, ctypes.byref(p), fake, fake,
                            None, fake, ws, None)

    w8 = ctypes.c_uint8 * 8
    assert frame(sb.SbStyle(fake, fake, fake, 64, 64, 0, 4, None, None, 0,
                            w8(2, 1, 1, 0))) == sb.SB_EINVAL
    assert frame(sb.SbStyle(fake, fake, fake, 64, 64, 2, 4, None, None, 0,
                            w8(1, 1, 128, 0))) == sb.SB_EINVAL


@pytest.mark.parametrize("fmt,channels,want", [
    (3, 2, 4), (3, 4, 4), (3, 5, 8), (3, 8, 8), (4, 2, 4), (4, 3, 8), (4, 4, 8), (4, 5, 16),
    (4, 8, 16), (3, 1, 0), (3, 9, 0), (2, 3, 0), (0, 2, 0), (5, 4, 0)])
def test_texel_bytes(L, fmt, channels, want):
    assert L.sb_texel_bytes(fmt, channels) == want


def test_search_format_validation(L):
    """Guides of many channels: sizes, the tree build and query, and frames
    of search-format styles refuse bad arguments before touching memory."""
    import paper_1807_03249_amd as sb

    fake = 0x1000
    U8XN, U16XN = sb.GUIDE_U8XN, sb.GUIDE_U16XN
    tb = L.sb_tree_bytes(U8XN, 5, 64, 48)
    wb = L.sb_tree_workspace_bytes(U8XN, 5, 64, 48)
    # at most 2n - 1 nodes of 8 B and two 8-byte box texels, n texels and keys
    n = 64 * 48
    assert tb >= 2 * n * 8 + 2 * n * 16 + n * 8 + n * 4
    assert wb >= 2 * n * (8 + 4)
    assert L.sb_tree_bytes(U8XN, 9, 64, 48) == 0 and L.sb_tree_bytes(U8XN, 5, 0, 48) == 0
    assert L.sb_tree_workspace_bytes(2, 3, 64, 48) == 0
    w8 = ctypes.c_uint8 * 8
    ok_w = w8(1, 2, 3, 4, 5)

    def build(fmt=U8XN, ch=5, w=ok_w, tree_bytes=tb, ws_bytes=wb, guide=fake, tree=fake,
              ws=fake):
        return L.sb_tree_build(guide, fmt, ch, 64, 48, w, tree, tree_bytes, ws, ws_bytes, None)

    assert build(fmt=2) == sb.SB_EINVAL
    assert build(ch=1) == sb.SB_EINVAL
    assert build(w=w8(1, 2, 128, 4, 5)) == sb.SB_EINVAL
    assert build(guide=None) == sb.SB_EINVAL and build(tree=None) == sb.SB_EINVAL
    assert build(ws=None) == sb.SB_EINVAL
    assert build(tree_bytes=tb - 1) == sb.SB_ENOMEM
    assert build(ws_bytes=wb - 1) == sb.SB_ENOMEM
    # a weight past the channel count is ignored
    assert build(fmt=U16XN, ch=2, w=w8(1, 1, 200), tree_bytes=0) == sb.SB_ENOMEM

    def style(fmt=U8XN, lut_bits=0, nlabels=0, channels=5, tree=fake, w=None):
        return sb.SbStyle(fake, fake, None, 64, 48, fmt, lut_bits, fake if nlabels else None,
                          fake if nlabels else None, nlabels, w or w8(), channels, tree)

    out = fake
    assert L.sb_tree_query(ctypes.byref(style(fmt=2)), fake, 4, out, None) == sb.SB_EINVAL
    assert L.sb_tree_query(ctypes.byref(style()), fake, -1, out, None) == sb.SB_EINVAL
    assert L.sb_tree_query(ctypes.byref(style(tree=None)), fake, 4, out, None) == sb.SB_EINVAL
    assert L.sb_tree_query(ctypes.byref(style(channels=9)), fake, 4, out, None) == sb.SB_EINVAL
    assert L.sb_tree_query(ctypes.byref(style()), fake, 0, out, None) == sb.SB_OK  # no work
    p = sb.params(4, 8, 32, 3)
    ws = sb.workspace_bytes(64, 48, p)

    def frame(st, labels=None):
        if labels is not None:
            return L.sb_stylize_seg(ctypes.byref(st), fake, labels, 64, 48, fake,
                                    ctypes.byref(p), fake, fake, None, fake, ws, None, None)
        return L.sb_stylize(ctypes.byref(st), fake, 64, 48, fake, ctypes.byref(p), fake, fake,
                            None, fake, ws, None)

    assert frame(style(lut_bits=8)) == sb.SB_EINVAL
    assert frame(style(nlabels=2)) == sb.SB_EINVAL
    assert frame(style(), labels=fake) == sb.SB_EINVAL
    assert frame(style(tree=None)) == sb.SB_EINVAL
    assert frame(style(channels=1)) == sb.SB_EINVAL
    assert frame(style(w=w8(1, 1, 1, 1, 255))) == sb.SB_EINVAL
    sp = ctypes.c_void_p()
    assert L.sb_style_create_n(fake, fake, 64, 48, U8XN, 9, None, None,
                               ctypes.byref(sp)) == sb.SB_EINVAL
    assert L.sb_style_create_n(fake, fake, 64, 48, 1, 4, None, None,
                               ctypes.byref(sp)) == sb.SB_EINVAL
    assert L.sb_style_create_n(None, fake, 64, 48, U8XN, 4, None, None,
                               ctypes.byref(sp)) == sb.SB_EINVAL
    assert not sp.value


def test_jitter_fill_validation(L):
    import paper_1807_03249_amd as sb

    assert L.sb_jitter_fill(0, 10, 3, 8, 1, 0, 0x1000, None) == sb.SB_EINVAL
    assert L.sb_jitter_fill(10, 10, 3, 6, 1, 0, 0x1000, None) == sb.SB_EINVAL  # finest not 2^k
    assert L.sb_jitter_fill(10, 10, 13, 1, 1, 0, 0x1000, None) == sb.SB_EINVAL
    assert L.sb_jitter_fill(10, 10, 3, 8, 1, 0, None, None) == sb.SB_EINVAL
    assert L.sb_jitter_fill(10, 10, 0, 8, 1, 0, None, None) == sb.SB_OK  # no levels: no work


def test_style_create_validation(L):
    """sb_style_create refuses bad arguments before allocating anything;
    sb_style_destroy(NULL) is a no-op."""
    import paper_1807_03249_amd as sb

    fake = 0x1000
    out = ctypes.c_void_p()
    assert L.sb_style_create(None, fake, 64, 64, 0, 8, None, ctypes.byref(out)) == sb.SB_EINVAL
    assert L.sb_style_create(fake, None, 64, 64, 0, 8, None, ctypes.byref(out)) == sb.SB_EINVAL
    assert L.sb_style_create(fake, fake, 64, 64, 0, 8, None, None) == sb.SB_EINVAL
    assert L.sb_style_create(fake, fake, 0, 64, 0, 8, None, ctypes.byref(out)) == sb.SB_EINVAL
    assert L.sb_style_create(fake, fake, 64, 8193, 0, 8, None, ctypes.byref(out)) == sb.SB_EINVAL
    assert L.sb_style_create(fake, fake, 64, 64, 0, 9, None, ctypes.byref(out)) == sb.SB_EINVAL
    assert L.sb_style_create(fake, fake, 64, 64, 1, 13, None, ctypes.byref(out)) == sb.SB_EINVAL
    assert L.sb_style_create(fake, fake, 64, 64, 3, 8, None, ctypes.byref(out)) == sb.SB_EINVAL
    assert out.value is None
    assert L.sb_style_destroy(None) == sb.SB_OK


def test_params_layout_and_jitter_modes(L):
    """sb_params as the header lays it out (seed and jitter mode after the
    radius); the binding's params() picks the hash with a seed and the cell
    corners without one."""
    import paper_1807_03249_amd as sb

    assert ctypes.sizeof(sb.SbParams) == 24
    assert sb.SbParams.seed.offset == 16 and sb.SbParams.jitter.offset == 20
    assert (sb.JITTER_HASH, sb.JITTER_NONE, sb.JITTER_TABLE) == (0, 1, 2)
    h = sb.params(4, 8, 32, 3, seed=2**32 + 5)
    assert h.jitter == sb.JITTER_HASH and h.seed == 5
    assert sb.params(4, 8, 32, 3).jitter == sb.JITTER_NONE
    assert sb._with_table(h).jitter == sb.JITTER_TABLE


def test_noalloc_rejects_frames_beyond_the_static_scratch(L):
    """sb_stylize_noalloc refuses, before any device call, a frame whose
    workspace exceeds the static scratch; the limit is what the header says."""
    import paper_1807_03249_amd as sb

    cap = sb.noalloc_scratch_bytes()
    assert cap == 41943040
    p = sb.params(5, 8, 4096, 3, seed=1)
    assert sb.workspace_bytes(3840, 2160, p) <= cap  # a 4K UHD frame fits
    fake = ctypes.c_void_p(0x1000)
    st = sb.SbStyle(fake, fake, fake, 512, 512, 0, 8)
    big = sb.params(4, 8, 32, 3, seed=1)
    assert sb.workspace_bytes(8192, 8192, big) > cap
    rc = L.sb_stylize_noalloc(ctypes.byref(st), fake, 8192, 8192, None, ctypes.byref(big),
                              fake, fake, None, None)
    assert rc == sb.SB_ENOMEM
    msg = L.sb_last_hip_error().decode()
    assert "8192x8192" in msg and str(cap) in msg
    # invalid arguments stay SB_EINVAL (radius 8 has no workspace size at all)
    bad = sb.params(4, 8, 32, 8, seed=1)
    assert L.sb_stylize_noalloc(ctypes.byref(st), fake, 64, 64, None, ctypes.byref(bad),
                                fake, fake, None, None) == sb.SB_EINVAL
    assert L.sb_stylize_noalloc(ctypes.byref(st), None, 64, 64, None, ctypes.byref(big),
                                fake, fake, None, None) == sb.SB_EINVAL
