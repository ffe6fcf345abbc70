"""Python front end of the ridge-directed Hough library.

PyTorch provides device memory and the stream; every step of the method runs in the HIP
kernels behind the C ABI.  Frames may be numpy arrays (copied in by the library) or CUDA
tensors (used in place).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import native as N

RING_DTYPE = np.dtype([("cx", np.float32), ("cy", np.float32), ("r", np.float32), ("score", np.float32),
                       ("a", np.int32), ("b", np.int32), ("r_bin", np.int32), ("n_fit", np.int32),
                       ("fit_ok", np.int32)])
assert RING_DTYPE.itemsize == ctypes.sizeof(N.RdRing)


def _frame_struct(frame):
    """rd_frame for a 2D uint16/float32 numpy array or CUDA tensor (kept alive by caller)."""
    if isinstance(frame, torch.Tensor):
        if frame.dim() != 2:
            raise ValueError("frame must be 2D")
        if frame.dtype == torch.uint16:
            dt, esz = N.RD_U16, 2
        elif frame.dtype == torch.float32:
            dt, esz = N.RD_F32, 4
        else:
            raise TypeError(f"unsupported frame dtype {frame.dtype}")
        if frame.stride(1) != 1:
            raise ValueError("frame rows must be contiguous")
        on_dev = 1 if frame.is_cuda else 0
        return N.RdFrame(frame.shape[1], frame.shape[0], frame.stride(0) * esz, dt, on_dev, frame.data_ptr())
    arr = np.asarray(frame)
    if arr.ndim != 2:
        raise ValueError("frame must be 2D")
    if arr.dtype == np.uint16:
        dt = N.RD_U16
    elif arr.dtype == np.float32:
        dt = N.RD_F32
    else:
        raise TypeError(f"unsupported frame dtype {arr.dtype}")
    if arr.strides[1] != arr.itemsize:
        raise ValueError("frame rows must be contiguous")
    return N.RdFrame(arr.shape[1], arr.shape[0], arr.strides[0], dt, 0, arr.ctypes.data)


def rings_to_numpy(buf, n: int) -> np.ndarray:
    out = np.frombuffer(buf, dtype=RING_DTYPE, count=n).copy() if n else np.zeros(0, RING_DTYPE)
    return out


class Detector:
    """One library context on one GPU, ordered on a torch stream."""

    def __init__(self, max_width: int = 2048, max_height: int = 2048, max_peaks: int = 65536,
                 max_frames: int = 1, max_batch_pixels: int = 0, device: int = 0, stream=None):
        self._lib = N.lib()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        info = N.RdCreateInfo(device, max_width, max_height, max_peaks, max_frames, max_batch_pixels,
                              ctypes.c_void_p(self.stream.cuda_stream))
        h = ctypes.c_void_p()
        N.check(self._lib.rd_create(ctypes.byref(info), ctypes.byref(h)), "rd_create")
        self._h = h
        self.max_peaks = max_peaks
        self._rings = (N.RdRing * max_peaks)()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -------------------------------------------------------------------- full pipeline
    def detect(self, frame, params: dict) -> np.ndarray:
        fr = _frame_struct(frame)
        p = N.make_params(params)
        n = ctypes.c_int32()
        st = self._lib.rd_detect(self._h, ctypes.byref(fr), ctypes.byref(p), self._rings, self.max_peaks,
                                 ctypes.byref(n))
        N.check(st, "rd_detect")
        return rings_to_numpy(self._rings, n.value)

    def detect_from_ridges(self, xy: torch.Tensor, q: torch.Tensor, width: int, height: int,
                           params: dict) -> np.ndarray:
        xy, q = self._ridge_tensors(xy, q)
        p = N.make_params(params)
        n = ctypes.c_int32()
        st = self._lib.rd_detect_ridges(self._h, xy.data_ptr(), q.data_ptr(), xy.shape[0], width, height,
                                        ctypes.byref(p), self._rings, self.max_peaks, ctypes.byref(n))
        N.check(st, "rd_detect_ridges")
        return rings_to_numpy(self._rings, n.value)

    # -------------------------------------------------------------------- batches
    def _frame_array(self, frames):
        n = len(frames)
        arr = (N.RdFrame * n)()
        for i, f in enumerate(frames):
            arr[i] = _frame_struct(f)
        return arr

    def detect_batch(self, frames, params: dict, capacity_per_frame: int | None = None) -> list:
        """Rings of every frame of a list (numpy arrays or CUDA tensors of one dtype), one launch
        sequence for the whole batch.  Returns a list of RING_DTYPE arrays."""
        n = len(frames)
        arr = self._frame_array(frames)
        cap = capacity_per_frame or self.max_peaks
        out = (N.RdRing * (n * cap))()
        offs = (ctypes.c_int64 * n)(*[i * cap for i in range(n)])
        caps = (ctypes.c_int32 * n)(*([cap] * n))
        counts = (ctypes.c_int32 * n)()
        p = N.make_params(params)
        st = self._lib.rd_detect_batch(self._h, arr, n, ctypes.byref(p), out, offs, caps, counts)
        N.check(st, "rd_detect_batch")
        buf = np.frombuffer(out, dtype=RING_DTYPE)
        return [buf[i * cap:i * cap + counts[i]].copy() for i in range(n)]

    def set_tuning(self, stencil_tile: int = 0, vote_lds_kb: int = 52, use_graph: bool = True):
        t = N.RdTuning(stencil_tile, vote_lds_kb, 1 if use_graph else 0)
        N.check(self._lib.rd_set_tuning(self._h, ctypes.byref(t)), "rd_set_tuning")

    def get_tuning(self) -> dict:
        t = N.RdTuning()
        N.check(self._lib.rd_get_tuning(self._h, ctypes.byref(t)), "rd_get_tuning")
        return dict(stencil_tile=t.stencil_tile, vote_lds_kb=t.vote_lds_kb, use_graph=bool(t.use_graph))

    def autotune(self, frames, params: dict, reps: int = 3) -> dict:
        arr = self._frame_array(frames)
        p = N.make_params(params)
        t = N.RdTuning()
        N.check(self._lib.rd_autotune(self._h, arr, len(frames), ctypes.byref(p), reps, ctypes.byref(t)),
                "rd_autotune")
        return dict(stencil_tile=t.stencil_tile, vote_lds_kb=t.vote_lds_kb, use_graph=bool(t.use_graph))

    def stats(self) -> dict:
        """Counters of the last call: ridges, votes, hotspots, taps, strong voxels, peaks."""
        v = (ctypes.c_int64 * 6)()
        N.check(self._lib.rd_read_stats(self._h, v), "rd_read_stats")
        return dict(zip(("ridges", "votes", "hotspots", "taps", "strong", "peaks"), list(v)))

    # -------------------------------------------------------------------- kernel timing
    def enable_timing(self, on: bool = True):
        N.check(self._lib.rd_enable_timing(self._h, 1 if on else 0), "rd_enable_timing")

    def read_timing(self, reset: bool = False):
        """{stage: (total ms, launches)} for 'ridge', 'vote', 'fit' kernels."""
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        N.check(self._lib.rd_read_timing(self._h, ms, n, 1 if reset else 0), "rd_read_timing")
        return {name: (ms[i], n[i]) for i, name in enumerate(("ridge", "vote", "fit"))}

    # -------------------------------------------------------------------- stage outputs
    def curvature(self, frame, params: dict):
        """k_- (float32 [H, W]) and direction codes (int16 [H, W, 2]) as CUDA tensors."""
        fr = _frame_struct(frame)
        H, W = fr.height, fr.width
        k = torch.empty((H, W), dtype=torch.float32, device=f"cuda:{self.device}")
        q = torch.empty((H, W, 2), dtype=torch.int16, device=f"cuda:{self.device}")
        p = N.make_params(params)
        N.check(self._lib.rd_stage_curvature(self._h, ctypes.byref(fr), ctypes.byref(p), k.data_ptr(),
                                             q.data_ptr()), "rd_stage_curvature")
        return k, q

    def ridges(self, frame, params: dict, capacity: int | None = None):
        """Ridge list as CUDA tensors: xy int32 [n, 2], q int16 [n, 2], k float32 [n]."""
        fr = _frame_struct(frame)
        if capacity is None:
            capacity = fr.width * fr.height
        dev = f"cuda:{self.device}"
        xy = torch.empty((capacity, 2), dtype=torch.int32, device=dev)
        q = torch.empty((capacity, 2), dtype=torch.int16, device=dev)
        k = torch.empty((capacity,), dtype=torch.float32, device=dev)
        p = N.make_params(params)
        n = ctypes.c_int64()
        N.check(self._lib.rd_stage_ridges(self._h, ctypes.byref(fr), ctypes.byref(p), xy.data_ptr(),
                                          q.data_ptr(), k.data_ptr(), capacity, ctypes.byref(n)),
                "rd_stage_ridges")
        m = n.value
        return xy[:m], q[:m], k[:m]

    def accumulate(self, xy: torch.Tensor, q: torch.Tensor, width: int, height: int, params: dict,
                   scores: bool = True):
        """Dense vote accumulator (int32 view of uint32, [L, H, W]) and integer scores (int64 view of
        uint64, [L, H, W]) from a given ridge list."""
        xy, q = self._ridge_tensors(xy, q)
        L = int(params["r_max"]) - int(params["r_min"]) + 3
        dev = f"cuda:{self.device}"
        acc = torch.empty((L, height, width), dtype=torch.int32, device=dev)
        sc = torch.empty((L, height, width), dtype=torch.int64, device=dev) if scores else None
        p = N.make_params(params)
        N.check(self._lib.rd_stage_accumulate(self._h, xy.data_ptr(), q.data_ptr(), xy.shape[0], width, height,
                                              ctypes.byref(p), acc.data_ptr(),
                                              sc.data_ptr() if sc is not None else None),
                "rd_stage_accumulate")
        return acc, sc

    def _ridge_tensors(self, xy, q):
        dev = f"cuda:{self.device}"
        xy = torch.as_tensor(xy).to(device=dev, dtype=torch.int32).contiguous().reshape(-1, 2)
        q = torch.as_tensor(q).to(device=dev, dtype=torch.int16).contiguous().reshape(-1, 2)
        if xy.shape[0] != q.shape[0]:
            raise ValueError("xy and q must have the same length")
        if xy.shape[0] == 0:
            xy = torch.zeros((1, 2), dtype=torch.int32, device=dev)[:0]
            q = torch.zeros((1, 2), dtype=torch.int16, device=dev)[:0]
        return xy, q


def validate_params(params: dict) -> int:
    """Host-only parameter check (no GPU needed); returns an rd_status code."""
    p = N.make_params(params)
    return N.lib().rd_validate_params(ctypes.byref(p))
