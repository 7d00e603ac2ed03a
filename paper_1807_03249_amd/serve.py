"""Serving: a request trace through the library's native request loop
(``sb_serve_run``), with HBM-budget admission and continuous batching over
several streams, or the plain per-request path for comparison.

Everything timing-critical runs in C++ (one host thread polling arrivals and
events); this module only marshals the trace and the buffers."""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from . import (JITTER_TABLE, SB_OK, SbParams, SbStyle, SbTune, Style, StyleBlitError, _check,
               _dev, _torch, _with_table, lib, tune_struct, workspace_bytes)


class SbServeConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("plain", ctypes.c_int32),
                ("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("desc_dev", ctypes.c_void_p), ("desc_host", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes_per_slot", ctypes.c_size_t),
                ("tune", SbTune), ("blocks_per_cu", ctypes.c_int32)]


class SbRequest(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("style", ctypes.POINTER(SbStyle)),
                ("tgt_guide", ctypes.c_void_p), ("jitter", ctypes.c_void_p),
                ("w", ctypes.c_int32), ("h", ctypes.c_int32), ("params", SbParams),
                ("out_rgb", ctypes.c_void_p), ("out_chunk", ctypes.c_void_p),
                ("out_nnf", ctypes.c_void_p), ("session", ctypes.c_int32),
                ("tgt_labels", ctypes.c_void_p)]


class SbRequestResult(ctypes.Structure):
    _fields_ = [("admitted_s", ctypes.c_double), ("launched_s", ctypes.c_double),
                ("completed_s", ctypes.c_double), ("batch", ctypes.c_int32),
                ("slot", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("status", ctypes.c_int32)]


def _bind():
    L = lib()
    if getattr(L, "_serve_bound", False):
        return L
    L.sb_frame_bytes.restype = ctypes.c_size_t
    L.sb_frame_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.sb_serve_run.argtypes = [ctypes.POINTER(SbServeConfig), ctypes.POINTER(SbRequest),
                               ctypes.c_int32, ctypes.POINTER(SbRequestResult)]
    L._serve_bound = True
    return L


class Request:
    """One request: a resident style, a device-resident target guide, a
    jitter table (a device int32 tensor, which selects SB_JITTER_TABLE) or
    None (the params' hash seed, or seeds on the cell corners), the frame
    parameters and (optionally) output tensors.
    ``session`` >= 0 marks a frame of an animated sequence: frames of one
    session complete in arrival order.  ``tgt_labels`` (uint8 (H, W) device
    tensor) runs the frame with the segmentation guide."""

    def __init__(self, arrival_s: float, style: Style, guide, jitter, p: SbParams,
                 out_rgb=None, out_chunk=None, out_nnf=None, session: int = -1,
                 tgt_labels=None):
        self.arrival_s = float(arrival_s)
        self.style = style
        self.guide = guide
        self.jitter = jitter
        if jitter is not None:
            p = _with_table(p)
        elif p.jitter == JITTER_TABLE:
            raise ValueError("SB_JITTER_TABLE needs a jitter table")
        self.params = p
        self.out_rgb = out_rgb
        self.out_chunk = out_chunk
        self.out_nnf = out_nnf
        self.session = int(session)
        self.tgt_labels = tgt_labels

    @property
    def h(self):
        return int(self.guide.shape[0])

    @property
    def w(self):
        return int(self.guide.shape[1])


def _check_request(torch, i: int, r: Request):
    """Shapes and types of a request's device tensors (the C loop checks
    sizes and parameters, not what the pointers hold)."""
    h, w = r.h, r.w

    def need(t, shape, dtype, what):
        if t is None:
            return
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"request {i}: {what} must be a contiguous device tensor")
        if tuple(t.shape) != shape or t.dtype != dtype:
            raise ValueError(f"request {i}: {what} must be {dtype} of shape {shape}")

    need(r.out_rgb, (h, w, 3), torch.uint8, "out_rgb")
    need(r.out_chunk, (h, w), torch.int32, "out_chunk")
    need(r.out_nnf, (h, w), torch.int32, "out_nnf")
    need(r.tgt_labels, (h, w), torch.uint8, "tgt_labels")


def run(requests: Sequence[Request], slots: int = 4, max_batch: int = 16,
        budget_bytes: int = 1 << 30, use_graph: bool = True, plain: bool = False, tune=None,
        blocks_per_cu: int = 0):
    """Run the trace in real time.  Returns a dict of numpy arrays (arrival,
    admitted, launched, completed times in seconds, batch ids and sizes,
    status) plus latency percentiles and throughput.  ``tune`` and
    ``blocks_per_cu`` fix the kernel choice (as for a batch plan)."""
    torch = _torch()
    L = _bind()
    n = len(requests)
    reqs = (SbRequest * n)()
    max_ws = 0
    for i, r in enumerate(requests):
        _check_request(torch, i, r)
        reqs[i] = SbRequest(r.arrival_s, ctypes.pointer(r.style.c), r.guide.data_ptr(),
                            r.jitter.data_ptr() if r.jitter is not None else None,
                            r.w, r.h, r.params,
                            r.out_rgb.data_ptr() if r.out_rgb is not None else None,
                            r.out_chunk.data_ptr() if r.out_chunk is not None else None,
                            r.out_nnf.data_ptr() if r.out_nnf is not None else None,
                            r.session,
                            r.tgt_labels.data_ptr() if r.tgt_labels is not None else None)
        max_ws = max(max_ws, workspace_bytes(r.w, r.h, r.params))
    nslots = 1 if plain else slots
    mb = 1 if plain else max_batch
    per_slot = (max_ws + 256) * mb
    arena = torch.empty(int(budget_bytes), dtype=torch.uint8, device="cuda")
    ws = torch.empty(per_slot * nslots, dtype=torch.uint8, device="cuda")
    db = L.sb_batch_desc_bytes()
    desc_dev = torch.empty(db * nslots, dtype=torch.uint8, device="cuda")
    desc_host = torch.empty(db * nslots, dtype=torch.uint8).pin_memory()
    cfg = SbServeConfig(nslots, mb, 1 if use_graph else 0, 1 if plain else 0, arena.data_ptr(),
                        int(budget_bytes), desc_dev.data_ptr(), desc_host.data_ptr(),
                        ws.data_ptr(), per_slot, tune_struct(tune) or SbTune(0, 0, 0, 0),
                        int(blocks_per_cu))
    res = (SbRequestResult * n)()
    torch.cuda.synchronize()
    _check(L.sb_serve_run(ctypes.byref(cfg), reqs, n, res), "sb_serve_run")
    torch.cuda.synchronize()
    arrival = np.array([r.arrival_s for r in requests])
    out = {
        "arrival": arrival,
        "admitted": np.array([x.admitted_s for x in res]),
        "launched": np.array([x.launched_s for x in res]),
        "completed": np.array([x.completed_s for x in res]),
        "batch": np.array([x.batch for x in res]),
        "batch_size": np.array([x.batch_size for x in res]),
        "status": np.array([x.status for x in res]),
        "slot": np.array([x.slot for x in res]),
        "session": np.array([r.session for r in requests]),
    }
    out["latency"] = out["completed"] - arrival
    return out


def summarize(out, discard_frac: float = 0.05, pixels: Optional[np.ndarray] = None):
    """p50/p90/p99/max latency (ms) over the trace minus its first
    ``discard_frac``, throughput (requests/s and Mpixel/s if ``pixels``)."""
    n = len(out["latency"])
    k = int(n * discard_frac)
    ok = out["status"][k:] == SB_OK
    lat = out["latency"][k:][ok] * 1e3
    span = out["completed"][k:].max() - out["arrival"][k]
    s = {
        "requests": int(ok.sum()),
        "p50_ms": float(np.percentile(lat, 50)),
        "p90_ms": float(np.percentile(lat, 90)),
        "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()),
        "req_per_s": float(ok.sum() / span),
        "mean_batch": float(out["batch_size"][k:][ok].mean()),
    }
    if pixels is not None:
        s["mpixel_per_s"] = float(pixels[k:][ok].sum() / span / 1e6)
    return s
