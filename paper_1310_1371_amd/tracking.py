"""Linking detected rings into trajectories on the GPU, and depth from radius: a thin
binding of the rd_link* entry points (argument marshalling only; every step runs in the
HIP kernel).  The tracker (prediction from the last velocity, or from the polynomial through
the last three detections, gate, greedy matching in (cost, track id, detection index) order,
memory for missed frames) is defined where the entry points are declared, in
ridge_detect.h."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import native as N

MAX_DETECTIONS = 4096
MAX_ACTIVE = 6144
MODELS = {"velocity": 0, "acceleration": 1}


class Linker:
    """Tracks over a sequence of frames; each `link` call continues where the last one
    stopped.  Detections are float32 (x, y, r) rows, e.g. the (cx, cy, r) of detected
    rings."""

    def __init__(self, gate: float, memory: int, depth=(8.0, 0.0, 72.0), max_tracks: int = 1 << 20,
                 max_frames: int = 256, stream: torch.cuda.Stream | None = None, model: str = "velocity"):
        if not torch.cuda.is_available():
            raise RuntimeError("the linker needs a HIP device")
        if model not in MODELS:
            raise ValueError(f"model must be one of {list(MODELS)}")
        self._lib = N.lib()
        self.params = N.RdLinkParams(float(gate), int(memory), float(depth[0]), float(depth[1]), float(depth[2]),
                                     MODELS[model])
        self.stream = stream or torch.cuda.current_stream()
        self.max_frames = int(max_frames)
        h = ctypes.c_void_p()
        N.check(self._lib.rd_linker_create(ctypes.byref(self.params), int(max_tracks), self.max_frames,
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                "rd_linker_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rd_linker_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def reset(self):
        N.check(self._lib.rd_linker_reset(self._h), "rd_linker_reset")

    def _info_raw(self):
        """(tracks, active, frame) without raising on a recorded overflow."""
        nt, na, fr = N._i32(), N._i32(), N._i32()
        self._lib.rd_linker_info(self._h, ctypes.byref(nt), ctypes.byref(na), ctypes.byref(fr))
        return nt.value, na.value, fr.value

    def info(self) -> dict:
        nt, na, fr = N._i32(), N._i32(), N._i32()
        st = self._lib.rd_linker_info(self._h, ctypes.byref(nt), ctypes.byref(na), ctypes.byref(fr))
        N.check(st, "rd_linker_info")
        return {"tracks": nt.value, "active": na.value, "frame": fr.value}

    def link(self, det: torch.Tensor, offsets, want_depth: bool = True, strict: bool = True):
        """det: float32 (n, 3) device tensor, frames back to back; offsets: nframes + 1 prefix
        offsets (host).  Returns (ids int32, z float32 or None), device tensors of length n.
        With strict=False an overflow does not raise: the call returns (ids, z, status), ids
        being -1 where no track could be given."""
        offs = np.ascontiguousarray(offsets, dtype=np.int32)
        nframes = len(offs) - 1
        det = det.contiguous()
        if det.dtype != torch.float32 or det.dim() != 2 or det.shape[1] != 3 or not det.is_cuda:
            raise ValueError("det must be a float32 (n, 3) device tensor")
        if nframes < 1 or int(offs[-1]) != det.shape[0]:
            raise ValueError("offsets must end at the number of detections")
        ids = torch.empty(det.shape[0], dtype=torch.int32, device=det.device)
        z = torch.empty(det.shape[0], dtype=torch.float32, device=det.device) if want_depth else None
        with torch.cuda.stream(self.stream):
            st = self._lib.rd_link(self._h, ctypes.c_void_p(det.data_ptr()),
                                   offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nframes,
                                   ctypes.c_void_p(ids.data_ptr()),
                                   ctypes.c_void_p(z.data_ptr()) if z is not None else None)
        if not strict and st == N.RD_E_OVERFLOW:
            return ids, z, st
        N.check(st, "rd_link")
        return (ids, z) if strict else (ids, z, st)
