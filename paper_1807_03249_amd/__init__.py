"""MI355X (gfx950) StyleBlit: Python binding of ``libstyleblit.so``.

Argument marshalling only: every step of the path runs in the HIP kernels
behind the C ABI declared in ``include/styleblit.h``.  PyTorch supplies device
memory (tensors) and the current HIP stream.  There is no CPU fallback: if
the library is not built or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

# STYLEBLIT_LIB names another build of the same library (e.g. to compare two
# builds in one process); by default the in-tree build is loaded
LIB_PATH = os.environ.get("STYLEBLIT_LIB") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libstyleblit.so")

GUIDE_U8X2 = 0
GUIDE_U16X2 = 1
GUIDE_U8X3 = 2  # three uint8 channels in 4 bytes per pixel (byte 3 ignored)
GUIDE_U8XN = 3  # 2..8 uint8 channels in 4- or 8-byte texels, exact search lookups
GUIDE_U16XN = 4  # 2..8 uint16 channels in 4-, 8- or 16-byte texels, exact search lookups
MAX_CHANNELS = 8
MAX_SIDE = 8192
MAX_LEVELS = 12
MAX_RADIUS = 7
MAX_LUT_BITS = 12

SB_OK, SB_EINVAL, SB_ENOMEM, SB_EHIP, SB_EBUDGET = 0, -1, -2, -3, -4


class StyleBlitError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})" + (f": {detail}" if detail else ""))


class SbStyle(ctypes.Structure):
    _fields_ = [("rgba", ctypes.c_void_p), ("guide", ctypes.c_void_p), ("lut", ctypes.c_void_p),
                ("sw", ctypes.c_int32), ("sh", ctypes.c_int32), ("fmt", ctypes.c_int32),
                ("lut_bits", ctypes.c_int32), ("labels", ctypes.c_void_p),
                ("label_luts", ctypes.c_void_p), ("nlabels", ctypes.c_int32),
                ("weights", ctypes.c_uint8 * 8), ("channels", ctypes.c_int32),
                ("tree", ctypes.c_void_p)]


class SbTune(ctypes.Structure):
    _fields_ = [("blend_ppt", ctypes.c_int32), ("blend_rows", ctypes.c_int32),
                ("level_group", ctypes.c_int32), ("level_ppt", ctypes.c_int32),
                ("blend_split", ctypes.c_int32)]


# every kernel choice (blend_ppt, blend_rows, level_group, level_ppt, blend_split); all
# compute the same bits, (0, 0, 0, 0, 0) is the library default
TUNES = [(ppt, rows, grp, lpx, split) for ppt in (4, 2) for rows in (16, 8) for grp in (2, 4)
         for lpx in (1, 2, 4) for split in (2, 1)]


def tune_struct(tune) -> Optional[SbTune]:
    """SbTune from a (blend_ppt, blend_rows, level_group, level_ppt,
    blend_split) tuple (None stays None; a shorter tuple leaves the rest at
    their defaults)."""
    if tune is None:
        return None
    if isinstance(tune, SbTune):
        return tune
    vals = [int(v) for v in tune] + [0] * (5 - len(tune))
    return SbTune(*vals)


JITTER_HASH, JITTER_NONE, JITTER_TABLE = 0, 1, 2


class SbParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("finest", ctypes.c_int32),
                ("threshold", ctypes.c_uint32), ("radius", ctypes.c_int32),
                ("seed", ctypes.c_uint32), ("jitter", ctypes.c_int32)]


class SbFrame(ctypes.Structure):
    _fields_ = [("style", ctypes.POINTER(SbStyle)), ("tgt_guide", ctypes.c_void_p),
                ("jitter", ctypes.c_void_p), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("params", SbParams), ("out_rgb", ctypes.c_void_p), ("out_chunk", ctypes.c_void_p),
                ("out_nnf", ctypes.c_void_p), ("tgt_labels", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded C-ABI library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1807_03249_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    L.sb_version.restype = ctypes.c_char_p
    L.sb_status_string.restype = ctypes.c_char_p
    L.sb_status_string.argtypes = [ctypes.c_int]
    L.sb_last_hip_error.restype = ctypes.c_char_p
    L.sb_jitter_len.restype = ctypes.c_int64
    L.sb_jitter_len.argtypes = [i32, i32, i32, i32]
    L.sb_exemplar_texels.restype = sz
    L.sb_exemplar_texels.argtypes = [i32, i32]
    L.sb_pack_exemplar.argtypes = [vp, i32, i32, vp, vp]
    L.sb_lut_workspace_bytes.restype = sz
    L.sb_lut_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.sb_lut_build.argtypes = [vp, i32, i32, i32, i32, vp, vp, sz, vp]
    L.sb_workspace_bytes.restype = sz
    L.sb_workspace_bytes.argtypes = [i32, i32, ctypes.POINTER(SbParams)]
    L.sb_stylize.argtypes = [ctypes.POINTER(SbStyle), vp, i32, i32, vp, ctypes.POINTER(SbParams),
                             vp, vp, vp, vp, sz, vp]
    L.sb_stylize_ex.argtypes = [ctypes.POINTER(SbStyle), vp, i32, i32, vp,
                                ctypes.POINTER(SbParams), vp, vp, vp, vp, sz,
                                ctypes.POINTER(SbTune), vp]
    L.sb_lut_build_labels.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, sz, vp]
    L.sb_lut_build_w.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, sz, vp]
    L.sb_lut_build_labels_w.argtypes = [vp, vp, i32, i32, i32, i32, vp, i32, vp, vp, vp, sz, vp]
    L.sb_stylize_seg.argtypes = [ctypes.POINTER(SbStyle), vp, vp, i32, i32, vp,
                                 ctypes.POINTER(SbParams), vp, vp, vp, vp, sz,
                                 ctypes.POINTER(SbTune), vp]
    L.sb_stylize_timed.argtypes = [ctypes.POINTER(SbStyle), vp, i32, i32, vp,
                                   ctypes.POINTER(SbParams), vp, vp, vp, vp, sz,
                                   ctypes.POINTER(SbTune), ctypes.POINTER(vp), vp]
    L.sb_timing_events_create.argtypes = [ctypes.POINTER(vp)]
    L.sb_timing_events_destroy.argtypes = [ctypes.POINTER(vp)]
    L.sb_event_elapsed_ms.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_float)]
    L.sb_batch_max_frames.restype = ctypes.c_int32
    L.sb_batch_desc_bytes.restype = sz
    L.sb_batch_workspace_bytes.restype = sz
    L.sb_batch_workspace_bytes.argtypes = [ctypes.POINTER(SbFrame), i32]
    L.sb_batch_create.argtypes = [vp, vp, i32, ctypes.POINTER(SbTune), i32, vp,
                                  ctypes.POINTER(ctypes.c_void_p)]
    L.sb_batch_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(SbFrame), i32, vp, sz, vp]
    L.sb_batch_destroy.argtypes = [ctypes.c_void_p]
    L.sb_stylize_frames.argtypes = [ctypes.POINTER(SbFrame), i32, vp, sz,
                                    ctypes.POINTER(SbTune), vp]
    L.sb_jitter_fill.argtypes = [i32, i32, i32, i32, ctypes.c_uint64, ctypes.c_uint64, vp, vp]
    L.sb_style_create.argtypes = [vp, vp, i32, i32, i32, i32, vp, ctypes.POINTER(vp)]
    L.sb_style_create_n.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, ctypes.POINTER(vp)]
    L.sb_texel_bytes.restype = i32
    L.sb_texel_bytes.argtypes = [i32, i32]
    L.sb_tree_bytes.restype = sz
    L.sb_tree_bytes.argtypes = [i32, i32, i32, i32]
    L.sb_tree_workspace_bytes.restype = sz
    L.sb_tree_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.sb_tree_build.argtypes = [vp, i32, i32, i32, i32, vp, vp, sz, vp, sz, vp]
    L.sb_tree_query.argtypes = [ctypes.POINTER(SbStyle), vp, ctypes.c_int64, vp, vp]
    L.sb_style_destroy.argtypes = [vp]
    L.sb_stylize_noalloc.argtypes = [ctypes.POINTER(SbStyle), vp, i32, i32, vp,
                                     ctypes.POINTER(SbParams), vp, vp, vp, vp]
    L.sb_noalloc_scratch_bytes.restype = sz
    L.sb_change_workspace_bytes.restype = sz
    L.sb_frame_change.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, vp, sz, vp]
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().sb_status_string(status).decode()


def _check(rc: int, where: str):
    if rc != SB_OK:
        detail = lib().sb_last_hip_error().decode() if rc == SB_EHIP else ""
        raise StyleBlitError(rc, where, detail)


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("StyleBlit needs a HIP device; none is visible")
    return torch


def _stream(torch) -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(torch, a, dtype=None):
    """Device tensor (contiguous) from a numpy array or tensor."""
    if isinstance(a, torch.Tensor):
        t = a
    else:
        t = torch.from_numpy(a)
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.to("cuda", non_blocking=False).contiguous()


def jitter_len(w: int, h: int, levels: int, finest: int) -> int:
    n = lib().sb_jitter_len(w, h, levels, finest)
    if n < 0:
        raise StyleBlitError(SB_EINVAL, "jitter_len")
    return int(n)


def params(levels: int, finest: int, threshold: int, radius: int,
           seed: Optional[int] = None) -> SbParams:
    """Frame parameters.  ``seed``: the seeds' jitter is the integer hash of
    (cell, level, seed) computed in the kernels (SB_JITTER_HASH); None puts
    the seeds on the cell corners (SB_JITTER_NONE) unless a jitter table is
    passed to the call, which then selects SB_JITTER_TABLE."""
    if seed is None:
        return SbParams(int(levels), int(finest), int(threshold), int(radius), 0, JITTER_NONE)
    return SbParams(int(levels), int(finest), int(threshold), int(radius),
                    int(seed) & 0xFFFFFFFF, JITTER_HASH)


def _with_table(p: SbParams) -> SbParams:
    """A copy of p that reads its jitter from the table passed beside it."""
    return SbParams(p.levels, p.finest, p.threshold, p.radius, p.seed, JITTER_TABLE)


def _jitter_arg(torch, jitter, p: SbParams, w: int, h: int):
    """(params, jitter tensor or None) for a call: a given table selects
    SB_JITTER_TABLE; without one, p's hash or corner mode needs no table."""
    if jitter is None:
        if p.jitter == JITTER_TABLE:
            raise ValueError("SB_JITTER_TABLE needs a jitter table")
        return p, None
    nj = jitter_len(w, h, p.levels, p.finest)
    j = jitter
    if not isinstance(j, torch.Tensor):
        j = j.view("int32") if str(j.dtype) == "uint32" else j
    j = _dev(torch, j)
    if j.numel() < nj or j.element_size() != 4:
        raise ValueError(f"jitter table needs {nj} 32-bit entries, got {j.numel()}")
    if j.numel() == 0:
        j = torch.zeros(1, dtype=torch.int32, device="cuda")
    return _with_table(p), j


def _guide_fmt(torch, g) -> int:
    """Format of a (rows, cols, channels) guide tensor: two uint8 channels,
    two uint16 channels, or (rows, cols, 4) uint8 holding three channels."""
    if g.dim() == 3 and g.shape[2] == 4 and g.dtype == torch.uint8:
        return GUIDE_U8X3
    if g.dim() != 3 or g.shape[2] != 2:
        raise TypeError("guide must be (rows, cols, 2), or (rows, cols, 4) uint8")
    if g.dtype == torch.uint8:
        return GUIDE_U8X2
    if g.dtype in (torch.uint16, torch.int16):
        return GUIDE_U16X2
    raise TypeError("guides are uint8 or uint16 with two channels")


def _search_fmt(torch, g, channels: int) -> int:
    """Format of a many-channel guide tensor (rows, cols, elements): uint8
    (GUIDE_U8XN) or uint16 / int16 bits (GUIDE_U16XN), whose texels
    (elements x element bytes) are the texel size of ``channels`` channels."""
    if g.dim() != 3:
        raise TypeError("a many-channel guide is (rows, cols, elements)")
    if g.dtype == torch.uint8:
        fmt = GUIDE_U8XN
    elif g.dtype in (torch.uint16, torch.int16):
        fmt = GUIDE_U16XN
    else:
        raise TypeError("many-channel guides are uint8 or uint16")
    tb = int(lib().sb_texel_bytes(fmt, int(channels)))
    if tb == 0 or g.shape[2] * g.element_size() != tb:
        raise TypeError(f"{channels} channels of this depth need {tb}-byte texels")
    return fmt


def _check_guide(torch, g, style) -> None:
    """A target guide must have its style's format (and channel count)."""
    if style.fmt in (GUIDE_U8XN, GUIDE_U16XN):
        if _search_fmt(torch, g, style.channels) != style.fmt:
            raise TypeError("target guide format differs from the style's guide format")
    elif _guide_fmt(torch, g) != style.fmt:
        raise TypeError("target guide format differs from the style's guide format")


def table_entries(fmt: int, lut_bits: int) -> int:
    """Entries of one lookup table: (2**lut_bits)**channels."""
    return 1 << ((3 if fmt == GUIDE_U8X3 else 2) * lut_bits)


class Style:
    """A device-resident style: RGBA-packed exemplar, its guide and the lookup
    table built from it on the GPU (Sec. 3.1).  With ``labels`` (uint8
    (rows, cols), values below ``nlabels``) the style also carries the
    segmentation guide: its label map and one lookup table per label.
    ``weights`` (three values 0..127, three-channel guides only) weight the
    channels' squared differences in the table and in the error test (the
    strong or weak appearance guide); None means unit weights.

    With ``channels`` (2..8) the guide holds that many channels of uint8 or
    uint16 in the texel layout of ``sb_texel_bytes`` ((rows, cols, elements)),
    looked up by the exact search on a k-d tree built on the GPU instead of a
    table (``lut_bits`` is then 0); ``weights`` then hold ``channels`` values."""

    def __init__(self, rgb, guide, lut_bits: int = 0, labels=None,
                 nlabels: Optional[int] = None, weights=None, channels: Optional[int] = None):
        torch = _torch()
        self.rgb = _dev(torch, rgb)
        if self.rgb.dtype != torch.uint8 or self.rgb.dim() != 3 or self.rgb.shape[2] != 3:
            raise TypeError("exemplar must be uint8 (rows, cols, 3)")
        g = guide
        if not isinstance(g, torch.Tensor) and getattr(g, "dtype", None) is not None and str(g.dtype) == "uint16":
            g = g.view("int16")  # torch.from_numpy has no uint16 on every build; same bits
        self.guide = _dev(torch, g)
        self.channels = int(channels) if channels is not None else 0
        self.fmt = (_search_fmt(torch, self.guide, self.channels) if channels is not None
                    else _guide_fmt(torch, self.guide))
        self.sh, self.sw = int(self.rgb.shape[0]), int(self.rgb.shape[1])
        if tuple(self.guide.shape[:2]) != (self.sh, self.sw):
            raise ValueError("exemplar and guide sizes differ")
        self.lut_bits = int(lut_bits)
        L = lib()
        # every temporary below is allocated on, and used by, torch's current
        # stream, so the caching allocator never hands it to other work early
        s = _stream(torch)
        # padded RGBA exemplar (zero margins, alpha 1 inside), see sb_exemplar_texels
        self.rgba = torch.empty(int(L.sb_exemplar_texels(self.sw, self.sh)), dtype=torch.int32,
                                device="cuda")
        _check(L.sb_pack_exemplar(self.rgb.data_ptr(), self.sw, self.sh, self.rgba.data_ptr(), s),
               "sb_pack_exemplar")
        self.labels = self.label_luts = self.lut = self.tree = None
        self.nlabels = 0
        if channels is not None:
            self._init_search(torch, L, s, weights, labels)
            return
        wsb = L.sb_lut_workspace_bytes(self.fmt, self.sw, self.sh, self.lut_bits)
        if wsb == 0:
            raise StyleBlitError(SB_EINVAL, "sb_lut_workspace_bytes")
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        self.lut = torch.empty(table_entries(self.fmt, self.lut_bits), dtype=torch.int32,
                               device="cuda")
        if weights is not None and len(weights) != 3:
            raise ValueError("weights must hold three values")
        self.weights = (ctypes.c_uint8 * 8)(*([int(v) for v in weights] + [0] * 5)
                                            if weights is not None else (0,) * 8)
        _check(L.sb_lut_build_w(self.guide.data_ptr(), self.fmt, self.sw, self.sh, self.lut_bits,
                                self.weights, self.lut.data_ptr(), ws.data_ptr(), wsb, s),
               "sb_lut_build_w")
        self._ws = ws  # keep alive until the enqueued build has run
        if labels is not None:
            self.labels = _dev(torch, labels, torch.uint8)
            if tuple(self.labels.shape) != (self.sh, self.sw):
                raise ValueError("label map and exemplar sizes differ")
            self.nlabels = int(nlabels if nlabels is not None else int(self.labels.max()) + 1)
            self.label_luts = torch.empty((self.nlabels, table_entries(self.fmt, self.lut_bits)),
                                          dtype=torch.int32, device="cuda")
            _check(L.sb_lut_build_labels_w(self.guide.data_ptr(), self.labels.data_ptr(),
                                           self.fmt, self.sw, self.sh, self.lut_bits,
                                           self.weights, self.nlabels, self.lut.data_ptr(),
                                           self.label_luts.data_ptr(), ws.data_ptr(), wsb, s),
                   "sb_lut_build_labels_w")
        self.c = SbStyle(self.rgba.data_ptr(), self.guide.data_ptr(), self.lut.data_ptr(),
                         self.sw, self.sh, self.fmt, self.lut_bits,
                         self.labels.data_ptr() if self.labels is not None else None,
                         self.label_luts.data_ptr() if self.label_luts is not None else None,
                         self.nlabels, self.weights)

    def _init_search(self, torch, L, s, weights, labels):
        if labels is not None:
            raise ValueError("many-channel guides take no labels")
        if int(self.lut_bits) != 0:
            raise ValueError("many-channel guides have no table: lut_bits must be 0")
        if weights is not None and len(weights) != self.channels:
            raise ValueError(f"weights must hold {self.channels} values")
        w = [int(v) for v in weights] if weights is not None else []
        self.weights = (ctypes.c_uint8 * 8)(*(w + [0] * (8 - len(w))))
        tb = int(L.sb_tree_bytes(self.fmt, self.channels, self.sw, self.sh))
        wsb = int(L.sb_tree_workspace_bytes(self.fmt, self.channels, self.sw, self.sh))
        if tb == 0 or wsb == 0:
            raise StyleBlitError(SB_EINVAL, "sb_tree_bytes")
        self.tree = torch.empty(tb, dtype=torch.uint8, device="cuda")
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        # synchronises the stream: the workspace is idle when this returns
        _check(L.sb_tree_build(self.guide.data_ptr(), self.fmt, self.channels, self.sw, self.sh,
                               self.weights, self.tree.data_ptr(), tb, ws.data_ptr(), wsb, s),
               "sb_tree_build")
        self.c = SbStyle(self.rgba.data_ptr(), self.guide.data_ptr(), None, self.sw, self.sh,
                         self.fmt, 0, None, None, 0, self.weights, self.channels,
                         self.tree.data_ptr())

    def query(self, texels):
        """Exact lookups of guide texels ((..., elements) in this style's
        layout, on the device) through the search tree: x | y << 16 per texel
        as int32 bits (sb_tree_query)."""
        torch = _torch()
        if self.tree is None:
            raise ValueError("query needs a many-channel style")
        if not isinstance(texels, torch.Tensor) and str(getattr(texels, "dtype", "")) == "uint16":
            texels = texels.view("int16")  # same bits; not every torch build takes uint16
        q = _dev(torch, texels)
        tb = int(lib().sb_texel_bytes(self.fmt, self.channels))
        if (q.numel() * q.element_size()) % tb != 0:
            raise ValueError(f"query texels must be whole {tb}-byte texels")
        n = q.numel() * q.element_size() // tb
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(lib().sb_tree_query(ctypes.byref(self.c), q.data_ptr(), n, out.data_ptr(),
                                   _stream(torch)), "sb_tree_query")
        return out

    def resident_bytes(self) -> int:
        if self.tree is not None:
            return (self.rgba.numel() * 4 + self.guide.numel() * self.guide.element_size()
                    + self.tree.numel())
        n = (self.rgba.numel() * 4 + self.guide.numel() * self.guide.element_size()
             + self.lut.numel() * 4)
        if self.labels is not None:
            n += self.labels.numel() + self.label_luts.numel() * 4
        return n


def workspace_bytes(w: int, h: int, p: SbParams) -> int:
    n = lib().sb_workspace_bytes(w, h, ctypes.byref(p))
    if n == 0:
        raise StyleBlitError(SB_EINVAL, "sb_workspace_bytes")
    return int(n)


def stylize(style: Style, tgt_guide, jitter, p: SbParams, out_rgb=None, out_chunk=None,
            want_nnf: bool = False, workspace=None, tune=None, events=None,
            tgt_labels=None):
    """Stylise one frame.  ``tgt_guide`` (H, W, 2) or (H, W, 4), or a many-channel
    style's texel layout (H, W, elements), and ``jitter`` (uint32 as int32
    bits) may be numpy arrays or device tensors.  Returns
    ``(rgb (H,W,3) uint8, chunk (H,W) int32-bits[, nnf])`` as device tensors;
    the work is enqueued on torch's current stream, the stream every
    temporary here is allocated on.  ``tune`` is a (blend_ppt, blend_rows,
    level_group, level_ppt, blend_split) choice (None = defaults); with
    ``events`` (a TimingEvents) the passes are bracketed by its events
    (sb_stylize_timed).  With ``tgt_labels`` (uint8 (H, W)) the frame runs
    with the segmentation guide (sb_stylize_seg; the style must carry labels)."""
    torch = _torch()
    g = tgt_guide
    if not isinstance(g, torch.Tensor) and str(getattr(g, "dtype", "")) == "uint16":
        g = g.view("int16")
    g = _dev(torch, g)
    _check_guide(torch, g, style)
    h, w = int(g.shape[0]), int(g.shape[1])
    p, j = _jitter_arg(torch, jitter, p, w, h)
    jp = j.data_ptr() if j is not None else None
    if out_rgb is None:
        out_rgb = torch.empty((h, w, 3), dtype=torch.uint8, device="cuda")
    if out_chunk is None:
        out_chunk = torch.empty((h, w), dtype=torch.int32, device="cuda")
    if out_rgb.numel() != h * w * 3 or out_rgb.dtype != torch.uint8 or out_chunk.numel() != h * w \
            or out_chunk.element_size() != 4:
        raise ValueError("output tensors do not match the frame size")
    if not (out_rgb.is_cuda and out_chunk.is_cuda and out_rgb.is_contiguous()
            and out_chunk.is_contiguous()):
        raise ValueError("output tensors must be contiguous device tensors")
    nnf = torch.empty((h, w), dtype=torch.int32, device="cuda") if want_nnf else None
    wsb = workspace_bytes(w, h, p)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    s = _stream(torch)
    tn = tune_struct(tune)
    tp = ctypes.byref(tn) if tn is not None else None
    nnf_p = nnf.data_ptr() if nnf is not None else None
    if tgt_labels is not None:
        if events is not None:
            raise ValueError("timed runs take no label maps")
        lt = _dev(torch, tgt_labels, torch.uint8)
        if tuple(lt.shape) != (h, w):
            raise ValueError("target label map and guide sizes differ")
        _check(lib().sb_stylize_seg(ctypes.byref(style.c), g.data_ptr(), lt.data_ptr(), w, h,
                                    jp, ctypes.byref(p), out_rgb.data_ptr(),
                                    out_chunk.data_ptr(), nnf_p, workspace.data_ptr(), wsb, tp, s),
               "sb_stylize_seg")
    elif events is not None:
        _check(lib().sb_stylize_timed(ctypes.byref(style.c), g.data_ptr(), w, h, jp,
                                      ctypes.byref(p), out_rgb.data_ptr(), out_chunk.data_ptr(),
                                      nnf_p, workspace.data_ptr(), wsb, tp, events.handles, s),
               "sb_stylize_timed")
    elif tn is None:
        _check(lib().sb_stylize(ctypes.byref(style.c), g.data_ptr(), w, h, jp,
                                ctypes.byref(p), out_rgb.data_ptr(), out_chunk.data_ptr(),
                                nnf_p, workspace.data_ptr(), wsb, s), "sb_stylize")
    else:
        _check(lib().sb_stylize_ex(ctypes.byref(style.c), g.data_ptr(), w, h, jp,
                                   ctypes.byref(p), out_rgb.data_ptr(), out_chunk.data_ptr(),
                                   nnf_p, workspace.data_ptr(), wsb, tp, s), "sb_stylize_ex")
    if want_nnf:
        return out_rgb, out_chunk, nnf
    return out_rgb, out_chunk


class FramePlan:
    """One frame's sb_stylize_ex call with its arguments checked and
    marshalled once (device tensors for guide, outputs and workspace), so a
    loop over many frames pays only the C call per launch.  ``launch()``
    enqueues the frame on torch's current stream (or on ``stream``, a raw
    stream handle); the tensors must stay alive while the plan is used."""

    def __init__(self, style: Style, tgt_guide, jitter, p: SbParams, out_rgb, out_chunk,
                 workspace, tune=None):
        torch = _torch()
        for t in (tgt_guide, out_rgb, out_chunk, workspace):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
                raise ValueError("FramePlan takes contiguous device tensors only")
        _check_guide(torch, tgt_guide, style)
        h, w = int(tgt_guide.shape[0]), int(tgt_guide.shape[1])
        if out_rgb.numel() != h * w * 3 or out_rgb.dtype != torch.uint8 \
                or out_chunk.numel() != h * w or out_chunk.element_size() != 4:
            raise ValueError("output tensors do not match the frame size")
        self.params, self.jitter = _jitter_arg(torch, jitter, p, w, h)
        wsb = workspace_bytes(w, h, self.params)
        if workspace.numel() < wsb:
            raise ValueError(f"workspace needs {wsb} bytes")
        self.tune = tune_struct(tune)
        self._keep = (style, tgt_guide, out_rgb, out_chunk, workspace)
        self._fn = lib().sb_stylize_ex
        self._args = (ctypes.byref(style.c), tgt_guide.data_ptr(), w, h,
                      self.jitter.data_ptr() if self.jitter is not None else None,
                      ctypes.byref(self.params), out_rgb.data_ptr(), out_chunk.data_ptr(), None,
                      workspace.data_ptr(), workspace.numel(),
                      ctypes.byref(self.tune) if self.tune is not None else None)
        self._torch = torch

    def launch(self, stream=None):
        s = self._torch.cuda.current_stream().cuda_stream if stream is None else stream
        rc = self._fn(*self._args, s)
        if rc != SB_OK:
            _check(rc, "sb_stylize_ex")


def stylize_noalloc(style: Style, tgt_guide, jitter, p: SbParams, out_rgb, out_chunk,
                    out_nnf=None):
    """Stylise one frame through sb_stylize_noalloc (no workspace: the
    library's static scratch).  ``tgt_guide``, ``jitter`` and the outputs must
    already be contiguous device tensors (nothing is allocated here either);
    the work is enqueued on torch's current stream."""
    torch = _torch()
    for t in (tgt_guide, out_rgb, out_chunk) + ((out_nnf,) if out_nnf is not None else ()):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise ValueError("stylize_noalloc takes contiguous device tensors only")
    _check_guide(torch, tgt_guide, style)
    h, w = int(tgt_guide.shape[0]), int(tgt_guide.shape[1])
    if out_rgb.numel() != h * w * 3 or out_rgb.dtype != torch.uint8 or out_chunk.numel() != h * w \
            or out_chunk.element_size() != 4:
        raise ValueError("output tensors do not match the frame size")
    if out_nnf is not None and (out_nnf.numel() != h * w or out_nnf.element_size() != 4):
        raise ValueError("nnf tensor does not match the frame size")
    jp = None
    if jitter is not None:
        if not isinstance(jitter, torch.Tensor) or not jitter.is_cuda or jitter.element_size() != 4:
            raise ValueError("stylize_noalloc takes a device jitter table")
        p = _with_table(p)
        jp = jitter.data_ptr()
    _check(lib().sb_stylize_noalloc(ctypes.byref(style.c), tgt_guide.data_ptr(), w, h, jp,
                                    ctypes.byref(p), out_rgb.data_ptr(), out_chunk.data_ptr(),
                                    out_nnf.data_ptr() if out_nnf is not None else None,
                                    _stream(torch)), "sb_stylize_noalloc")
    return out_rgb, out_chunk


def noalloc_scratch_bytes() -> int:
    """Size of the static scratch behind sb_stylize_noalloc (bytes)."""
    return int(lib().sb_noalloc_scratch_bytes())


def jitter_fill(w: int, h: int, levels: int, finest: int, seed: int, stream_id: int = 0,
                out=None):
    """A jitter table drawn on the device (sb_jitter_fill: Philox4x64-10
    under key (seed, stream_id)), as an int32 device tensor, enqueued on the
    current stream."""
    torch = _torch()
    n = jitter_len(w, h, levels, finest)
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    elif out.numel() < n or out.element_size() != 4 or not out.is_cuda:
        raise ValueError(f"jitter table needs {n} 32-bit device entries")
    _check(lib().sb_jitter_fill(w, h, levels, finest, seed, stream_id, out.data_ptr(),
                                _stream(torch)), "sb_jitter_fill")
    return out


def frame_change(chunk_a, chunk_b, nnf_a=None, nnf_b=None, counts=None, workspace=None):
    """Pixels that changed between two frames of a sequence (sb_frame_change):
    a device int64 tensor [chunk codes that differ, source coordinates that
    differ] (the second 0 without NNF maps), enqueued on the current stream."""
    torch = _torch()
    L = lib()
    maps = [chunk_a, chunk_b] + ([nnf_a, nnf_b] if nnf_a is not None else [])
    for m in maps:
        if not isinstance(m, torch.Tensor) or not m.is_cuda or m.element_size() != 4 \
                or not m.is_contiguous():
            raise TypeError("change maps must be contiguous 32-bit device tensors")
        if m.numel() != chunk_a.numel():
            raise ValueError("change maps must have the same number of pixels")
    if (nnf_a is None) != (nnf_b is None):
        raise ValueError("give both NNF maps or neither")
    if counts is None:
        counts = torch.empty(2, dtype=torch.int64, device="cuda")
    if workspace is None:
        workspace = torch.empty(L.sb_change_workspace_bytes(), dtype=torch.uint8, device="cuda")
    _check(L.sb_frame_change(chunk_a.data_ptr(), chunk_b.data_ptr(),
                             nnf_a.data_ptr() if nnf_a is not None else None,
                             nnf_b.data_ptr() if nnf_b is not None else None, chunk_a.numel(),
                             counts.data_ptr(), workspace.data_ptr(), workspace.numel(),
                             _stream(torch)), "sb_frame_change")
    return counts


class TimingEvents:
    """Four fence-free timing events (sb_timing_events_create) for one
    stylize(..., events=...) call; ``pass_ms()`` after the work completed
    gives the seed, level-loop and voting pass durations in milliseconds."""

    def __init__(self):
        self.handles = (ctypes.c_void_p * 4)()
        _check(lib().sb_timing_events_create(self.handles), "sb_timing_events_create")

    def elapsed_ms(self, i: int, j: int) -> float:
        ms = ctypes.c_float()
        _check(lib().sb_event_elapsed_ms(self.handles[i], self.handles[j], ctypes.byref(ms)),
               "sb_event_elapsed_ms")
        return float(ms.value)

    def pass_ms(self):
        return [self.elapsed_ms(0, 1), self.elapsed_ms(1, 2), self.elapsed_ms(2, 3)]

    def close(self):
        if self.handles is not None:
            _check(lib().sb_timing_events_destroy(self.handles), "sb_timing_events_destroy")
            self.handles = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FrameJob:
    """One frame of a batch: device tensors for the target guide, jitter and
    outputs (allocated here when not given)."""

    def __init__(self, style: Style, tgt_guide, jitter, p: SbParams, out_rgb=None, out_chunk=None,
                 out_nnf=None, tgt_labels=None):
        torch = _torch()
        g = tgt_guide
        if not isinstance(g, torch.Tensor) and str(getattr(g, "dtype", "")) == "uint16":
            g = g.view("int16")
        self.style = style
        self.guide = _dev(torch, g)
        _check_guide(torch, self.guide, style)
        self.h, self.w = int(self.guide.shape[0]), int(self.guide.shape[1])
        self.params, self.jitter = _jitter_arg(torch, jitter, p, self.w, self.h)
        self.out_rgb = out_rgb if out_rgb is not None else torch.empty(
            (self.h, self.w, 3), dtype=torch.uint8, device="cuda")
        self.out_chunk = out_chunk if out_chunk is not None else torch.empty(
            (self.h, self.w), dtype=torch.int32, device="cuda")
        self.out_nnf = out_nnf
        self.tgt_labels = None if tgt_labels is None else _dev(torch, tgt_labels, torch.uint8)

    def c(self) -> SbFrame:
        return SbFrame(ctypes.pointer(self.style.c), self.guide.data_ptr(),
                       self.jitter.data_ptr() if self.jitter is not None else None,
                       self.w, self.h, self.params, self.out_rgb.data_ptr(),
                       self.out_chunk.data_ptr(),
                       self.out_nnf.data_ptr() if self.out_nnf is not None else None,
                       self.tgt_labels.data_ptr() if self.tgt_labels is not None else None)


def stylize_frames(jobs, workspace=None, tune=None):
    """The frames of ``jobs`` (FrameJob) one after another, each through the
    per-frame kernels (sb_stylize_frames: one C call, no batching), on
    torch's current stream.  ``workspace`` must hold the largest frame's
    workspace (allocated here when not given)."""
    torch = _torch()
    arr = (SbFrame * len(jobs))(*[j.c() for j in jobs])
    wsb = max(workspace_bytes(j.w, j.h, j.params) for j in jobs)
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    tn = tune_struct(tune)
    _check(lib().sb_stylize_frames(arr, len(jobs), workspace.data_ptr(), workspace.numel(),
                                   ctypes.byref(tn) if tn is not None else None, _stream(torch)),
           "sb_stylize_frames")
    return jobs


class Batch:
    """A batch plan: many frames per launch.  With ``use_graph`` the launch
    is one replay of a hipGraph captured once (descriptor upload + the
    persistent kernels) on the plan's own stream.  ``tune`` and
    ``blocks_per_cu`` fix the kernel choice and persistent grid."""

    def __init__(self, use_graph: bool = True, tune=None, blocks_per_cu: int = 0):
        torch = _torch()
        L = lib()
        nb = L.sb_batch_desc_bytes()
        self.desc_dev = torch.empty(nb, dtype=torch.uint8, device="cuda")
        self.desc_host = torch.empty(nb, dtype=torch.uint8).pin_memory()
        self.capture_stream = torch.cuda.Stream()
        self.tune = tune_struct(tune)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(L.sb_batch_create(self.desc_dev.data_ptr(), self.desc_host.data_ptr(),
                                 1 if use_graph else 0,
                                 ctypes.byref(self.tune) if self.tune is not None else None,
                                 int(blocks_per_cu), self.capture_stream.cuda_stream,
                                 ctypes.byref(h)), "sb_batch_create")
        self.handle = h
        self.max_frames = L.sb_batch_max_frames()
        self._ws = None
        self._keep = [None, None]
        self._k = 0

    def workspace_bytes(self, jobs) -> int:
        arr = (SbFrame * len(jobs))(*[j.c() for j in jobs])
        n = lib().sb_batch_workspace_bytes(arr, len(jobs))
        if n == 0:
            raise StyleBlitError(SB_EINVAL, "sb_batch_workspace_bytes")
        return int(n)

    def run(self, jobs, workspace=None):
        """Enqueue the batch on torch's current stream (where the workspace
        is allocated too)."""
        torch = _torch()
        arr = (SbFrame * len(jobs))(*[j.c() for j in jobs])
        wsb = lib().sb_batch_workspace_bytes(arr, len(jobs))
        if wsb == 0:
            raise StyleBlitError(SB_EINVAL, "sb_batch_workspace_bytes")
        if workspace is None:
            workspace = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        s = _stream(torch)
        _check(lib().sb_batch_run(self.handle, arr, len(jobs), workspace.data_ptr(), wsb, s),
               "sb_batch_run")
        # keep this run's tensors alive until its descriptor half is reused
        self._keep[self._k] = (jobs, workspace)
        self._k ^= 1
        return jobs

    def close(self):
        if self.handle:
            _check(lib().sb_batch_destroy(self.handle), "sb_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
