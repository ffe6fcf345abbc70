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


def _copy_rings(raw: np.ndarray, first: int, n: int) -> np.ndarray:
    """Rings first .. first + n - 1 of a byte view of a ring buffer, as a new RING_DTYPE array.
    Copied as bytes: numpy copies a structured array field by field (~8 us for 200 rings)."""
    sz = RING_DTYPE.itemsize
    return raw[first * sz:(first + n) * sz].copy().view(RING_DTYPE)


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
        self.default_tuning = self.get_tuning()
        self.max_peaks = max_peaks
        self._rings = (N.RdRing * max_peaks)()
        self._rings_raw = np.frombuffer(self._rings, dtype=np.uint8)   # shares self._rings
        self._batch_buf = None
        self._batch_meta = None          # (frames, capacity, offsets, capacities) of the last batch

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
        return _copy_rings(self._rings_raw, 0, n.value)

    def detect_from_ridges(self, xy: torch.Tensor, q: torch.Tensor, width: int, height: int,
                           params: dict) -> np.ndarray:
        xy, q = self._ridge_tensors(xy, q)
        p = N.make_params(params)
        n = ctypes.c_int32()
        st = self._lib.rd_detect_ridges(self._h, xy.data_ptr(), q.data_ptr(), xy.shape[0], width, height,
                                        ctypes.byref(p), self._rings, self.max_peaks, ctypes.byref(n))
        N.check(st, "rd_detect_ridges")
        return _copy_rings(self._rings_raw, 0, n.value)

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
        # one uninitialised host buffer, kept across calls: only the rings found are written
        if self._batch_buf is None or self._batch_buf.shape[0] < n * cap:
            self._batch_buf = np.empty(n * cap, dtype=RING_DTYPE)
        buf = self._batch_buf
        out = ctypes.cast(buf.ctypes.data, ctypes.POINTER(N.RdRing))
        if self._batch_meta is None or self._batch_meta[:2] != (n, cap):
            self._batch_meta = (n, cap, (ctypes.c_int64 * n)(*[i * cap for i in range(n)]),
                                (ctypes.c_int32 * n)(*([cap] * n)))
        offs, caps = self._batch_meta[2], self._batch_meta[3]
        counts = (ctypes.c_int32 * n)()
        p = N.make_params(params)
        st = self._lib.rd_detect_batch(self._h, arr, n, ctypes.byref(p), out, offs, caps, counts)
        N.check(st, "rd_detect_batch")
        raw = buf.view(np.uint8)
        return [_copy_rings(raw, i * cap, counts[i]) for i in range(n)]

    # -------------------------------------------------------------------- encoded ridge streams
    def encode_ridges(self, frames, params: dict, out: torch.Tensor | None = None):
        """Steps 1-2 on a list of frames, their ridges as encoded streams: (uint8 CUDA tensor
        holding the streams, int64 numpy offsets of n + 1).  `out` (uint8 CUDA tensor) is reused
        when it is large enough."""
        n = len(frames)
        arr = self._frame_array(frames)
        p = N.make_params(params)
        offs = np.zeros(n + 1, dtype=np.int64)
        if out is None:
            px = sum(int(f.shape[0]) * int(f.shape[1]) for f in frames)
            out = torch.empty(px + 64 * n + 1024, dtype=torch.uint8, device=self._dev())
        po = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        st = self._lib.rd_encode_ridges(self._h, arr, n, ctypes.byref(p), out.data_ptr(), out.numel(), po)
        if st == N.RD_E_TRUNCATED:
            out = torch.empty(int(offs[n]), dtype=torch.uint8, device=self._dev())
            st = self._lib.rd_encode_ridges(self._h, arr, n, ctypes.byref(p), out.data_ptr(), out.numel(), po)
        N.check(st, "rd_encode_ridges")
        return out, offs

    def detect_encoded(self, enc, offsets, params: dict, capacity_per_frame: int | None = None) -> list:
        """Rings of every encoded stream (a uint8 numpy array in host memory or a uint8 CUDA
        tensor, with its n + 1 offsets).  Returns a list of RING_DTYPE arrays."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        n = len(offsets) - 1
        if isinstance(enc, torch.Tensor):
            on_dev, ptr = (1 if enc.is_cuda else 0), enc.data_ptr()
        else:
            enc = np.ascontiguousarray(enc, dtype=np.uint8)
            on_dev, ptr = 0, enc.ctypes.data
        cap = capacity_per_frame or self.max_peaks
        buf = np.empty(n * cap, dtype=RING_DTYPE)
        out = ctypes.cast(buf.ctypes.data, ctypes.POINTER(N.RdRing))
        oo = (ctypes.c_int64 * n)(*[i * cap for i in range(n)])
        cc = (ctypes.c_int32 * n)(*([cap] * n))
        counts = (ctypes.c_int32 * n)()
        p = N.make_params(params)
        st = self._lib.rd_detect_encoded(self._h, ptr, on_dev, offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                         n, ctypes.byref(p), out, oo, cc, counts)
        N.check(st, "rd_detect_encoded")
        raw = buf.view(np.uint8)
        return [_copy_rings(raw, i * cap, counts[i]) for i in range(n)]

    def set_tuning(self, stencil_tile: int = 0, vote_lds_kb: int = None, use_graph: bool = True):
        """Launch choices (no result depends on them); vote_lds_kb None keeps the largest."""
        if vote_lds_kb is None:
            vote_lds_kb = self.default_tuning["vote_lds_kb"]
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
    PHASES = ("tile set-up", "ridge staging", "item sort", "votes and hotspot listing", "scores",
              "above-threshold list", "3x3x3 test and peaks", "next chunk clear and weights")

    def profile_vote_phases(self, frame, params: dict) -> dict:
        """One detection with the phase-timed vote kernel: shader clocks per phase summed over
        the workgroups, their lifetimes, the tiles, the longest and shortest lifetime."""
        fr = _frame_struct(frame)
        p = N.make_params(params)
        n = len(self.PHASES)
        c = (ctypes.c_uint64 * (n + 4))()
        N.check(self._lib.rd_profile_vote_phases(self._h, ctypes.byref(fr), ctypes.byref(p), c),
                "rd_profile_vote_phases")
        return {"phases": dict(zip(self.PHASES, [int(v) for v in c[:n]])), "lifetime_sum": int(c[n]),
                "tiles": int(c[n + 1]), "lifetime_max": int(c[n + 2]), "lifetime_min": int(c[n + 3])}

    def profile_vote_tiles(self, frame, params: dict):
        """One detection with the phase-timed vote kernel, per vote tile: an int64 [n, 4] array of
        (workgroup, queue position, clock at start, clock at end); only end - start compares
        across workgroups."""
        import numpy as np
        fr = _frame_struct(frame)
        p = N.make_params(params)
        n = ctypes.c_int32(0)
        self._lib.rd_profile_vote_tiles(self._h, ctypes.byref(fr), ctypes.byref(p), None, 0, ctypes.byref(n))
        rec = np.zeros((max(n.value, 1), 4), dtype=np.uint64)
        N.check(self._lib.rd_profile_vote_tiles(self._h, ctypes.byref(fr), ctypes.byref(p),
                                                rec.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n)),
                "rd_profile_vote_tiles")
        return rec[:n.value].astype(np.int64)

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
        L = N.n_levels(params)
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


    # -------------------------------------------------------------------- differentiable path
    def _dev(self):
        return f"cuda:{self.device}"

    def soft_ridges(self, frame, params: dict, capacity: int | None = None):
        """Ridge set (int32 [n, 2]) and the Hessian (Ixx, Iyy, Ixy) at each ridge (float64 [n, 3])."""
        fr = _frame_struct(frame)
        if capacity is None:
            capacity = fr.width * fr.height
        xy = torch.empty((capacity, 2), dtype=torch.int32, device=self._dev())
        hess = torch.empty((capacity, 3), dtype=torch.float64, device=self._dev())
        p = N.make_params(params)
        n = ctypes.c_int64()
        N.check(self._lib.rd_soft_ridges(self._h, ctypes.byref(fr), ctypes.byref(p), xy.data_ptr(), hess.data_ptr(),
                                         capacity, ctypes.byref(n)), "rd_soft_ridges")
        return xy[:n.value], hess[:n.value]

    def _soft_inputs(self, xy, hess):
        xy = torch.as_tensor(xy).to(device=self._dev(), dtype=torch.int32).contiguous().reshape(-1, 2)
        hess = torch.as_tensor(hess).to(device=self._dev(), dtype=torch.float64).contiguous().reshape(-1, 3)
        if xy.shape[0] != hess.shape[0]:
            raise ValueError("xy and hess must have the same length")
        return xy, hess

    def soft_forward(self, xy, hess, width: int, height: int, params: dict) -> torch.Tensor:
        """Soft accumulator, float32 [L, H, W] with L = r_max - r_min + 3."""
        xy, hess = self._soft_inputs(xy, hess)
        L = int(params["r_max"]) - int(params["r_min"]) + 3
        acc = torch.empty((L, height, width), dtype=torch.float32, device=self._dev())
        p = N.make_params(params)
        N.check(self._lib.rd_soft_forward(self._h, xy.data_ptr(), hess.data_ptr(), xy.shape[0], width, height,
                                          ctypes.byref(p), acc.data_ptr()), "rd_soft_forward")
        return acc

    def soft_backward(self, xy, hess, width: int, height: int, params: dict, grad_acc: torch.Tensor,
                      count_isotropic: bool = False):
        """d/d(Ixx, Iyy, Ixy) per ridge (float64 [n, 3]) from dL/dA~; with count_isotropic also the
        number of near-isotropic ridges whose eigenvector term was dropped."""
        xy, hess = self._soft_inputs(xy, hess)
        L = int(params["r_max"]) - int(params["r_min"]) + 3
        g = grad_acc.to(device=self._dev(), dtype=torch.float32).contiguous()
        if tuple(g.shape) != (L, height, width):
            raise ValueError(f"grad_acc must have shape {(L, height, width)}")
        out = torch.empty((xy.shape[0], 3), dtype=torch.float64, device=self._dev())
        p = N.make_params(params)
        n_iso = ctypes.c_int64()
        N.check(self._lib.rd_soft_backward(self._h, xy.data_ptr(), hess.data_ptr(), xy.shape[0], width, height,
                                           ctypes.byref(p), g.data_ptr(), out.data_ptr(),
                                           ctypes.byref(n_iso) if count_isotropic else None),
                "rd_soft_backward")
        return (out, n_iso.value) if count_isotropic else out

    def hessian_backward(self, xy, grad_hess, width: int, height: int, params: dict,
                         grad_img: torch.Tensor | None = None) -> torch.Tensor:
        """Adds the image gradient of per-ridge Hessian gradients into grad_img (float32 [H, W],
        zeros if None) and returns it."""
        xy, grad_hess = self._soft_inputs(xy, grad_hess)
        if grad_img is None:
            grad_img = torch.zeros((height, width), dtype=torch.float32, device=self._dev())
        if grad_img.dtype != torch.float32 or not grad_img.is_contiguous() or tuple(grad_img.shape) != (height, width):
            raise ValueError("grad_img must be a contiguous float32 [H, W] tensor")
        p = N.make_params(params)
        N.check(self._lib.rd_hessian_backward(self._h, xy.data_ptr(), grad_hess.data_ptr(), xy.shape[0], width,
                                              height, ctypes.byref(p), grad_img.data_ptr()), "rd_hessian_backward")
        return grad_img

    # ---- the differentiable calls over a batch of frames (one library call each)
    def soft_ridges_batch(self, frames, params: dict, capacity: int | None = None):
        """Ridge sets of several device frames as one list: xy int32 [N, 2], hess float64
        [N, 3], and the frames' offsets into it (numpy int64 [nframes + 1])."""
        arr = self._frame_array(frames)
        n = len(frames)
        if capacity is None:
            capacity = sum(int(a.width) * int(a.height) for a in arr) // 4
        xy = torch.empty((capacity, 2), dtype=torch.int32, device=self._dev())
        hess = torch.empty((capacity, 3), dtype=torch.float64, device=self._dev())
        offs = np.zeros(n + 1, dtype=np.int64)
        p = N.make_params(params)
        N.check(self._lib.rd_soft_ridges_batch(self._h, arr, n, ctypes.byref(p), xy.data_ptr(), hess.data_ptr(),
                                               capacity, offs.ctypes.data), "rd_soft_ridges_batch")
        return xy[:int(offs[-1])], hess[:int(offs[-1])], offs

    @staticmethod
    def _sizes(sizes):
        w = np.ascontiguousarray([int(s[0]) for s in sizes], dtype=np.int32)
        h = np.ascontiguousarray([int(s[1]) for s in sizes], dtype=np.int32)
        return w, h

    def soft_forward_batch(self, xy, hess, offsets, sizes, params: dict) -> torch.Tensor:
        """Soft accumulators of a batch (sizes: (width, height) per frame), back to back as one
        float32 tensor; [nframes, L, H, W] when every frame has one size."""
        xy, hess = self._soft_inputs(xy, hess)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        w, h = self._sizes(sizes)
        L = int(params["r_max"]) - int(params["r_min"]) + 3
        acc = torch.empty(int((L * w.astype(np.int64) * h).sum()), dtype=torch.float32, device=self._dev())
        p = N.make_params(params)
        N.check(self._lib.rd_soft_forward_batch(self._h, xy.data_ptr(), hess.data_ptr(), offs.ctypes.data,
                                                w.ctypes.data, h.ctypes.data, len(w), ctypes.byref(p),
                                                acc.data_ptr()), "rd_soft_forward_batch")
        if (w == w[0]).all() and (h == h[0]).all():
            acc = acc.view(len(w), L, int(h[0]), int(w[0]))
        return acc

    def soft_backward_batch(self, xy, hess, offsets, sizes, params: dict, grad_acc: torch.Tensor) -> torch.Tensor:
        """d/d(Ixx, Iyy, Ixy) per ridge of a batch from the accumulators' gradients (laid out as
        soft_forward_batch returns them)."""
        xy, hess = self._soft_inputs(xy, hess)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        w, h = self._sizes(sizes)
        L = int(params["r_max"]) - int(params["r_min"]) + 3
        g = grad_acc.to(device=self._dev(), dtype=torch.float32).contiguous()
        if g.numel() != int((L * w.astype(np.int64) * h).sum()):
            raise ValueError("grad_acc does not match the batch's accumulators")
        out = torch.empty((xy.shape[0], 3), dtype=torch.float64, device=self._dev())
        p = N.make_params(params)
        N.check(self._lib.rd_soft_backward_batch(self._h, xy.data_ptr(), hess.data_ptr(), offs.ctypes.data,
                                                 w.ctypes.data, h.ctypes.data, len(w), ctypes.byref(p),
                                                 g.data_ptr(), out.data_ptr(), None), "rd_soft_backward_batch")
        return out

    def hessian_backward_batch(self, xy, grad_hess, offsets, sizes, params: dict,
                               grad_img: torch.Tensor | None = None) -> torch.Tensor:
        """Adds each frame's image gradient of its ridges' Hessian gradients into grad_img (the
        frames' float32 planes back to back; zeros if None) and returns it."""
        xy, grad_hess = self._soft_inputs(xy, grad_hess)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        w, h = self._sizes(sizes)
        npx = int((w.astype(np.int64) * h).sum())
        if grad_img is None:
            grad_img = torch.zeros(npx, dtype=torch.float32, device=self._dev())
        if grad_img.dtype != torch.float32 or not grad_img.is_contiguous() or grad_img.numel() != npx:
            raise ValueError("grad_img must be a contiguous float32 tensor of the batch's pixels")
        p = N.make_params(params)
        N.check(self._lib.rd_hessian_backward_batch(self._h, xy.data_ptr(), grad_hess.data_ptr(), offs.ctypes.data,
                                                    w.ctypes.data, h.ctypes.data, len(w), ctypes.byref(p),
                                                    grad_img.data_ptr()), "rd_hessian_backward_batch")
        return grad_img

    def _frame_of(self, frame_of, m):
        fo = torch.as_tensor(frame_of).to(device=self._dev(), dtype=torch.int32).contiguous().reshape(-1)
        if fo.shape[0] != m:
            raise ValueError("frame_of must have one entry per ring")
        return fo

    def fit_loss_batch(self, frames, theta, theta0, frame_of, s: float):
        """Ring fit loss (float64 [m]) and (A, B) (float64 [m, 2]) of rings on up to 64 frames."""
        arr = self._frame_array(frames)
        theta, theta0 = self._thetas(theta), self._thetas(theta0)
        m = theta.shape[0]
        fo = self._frame_of(frame_of, m)
        loss = torch.empty((m,), dtype=torch.float64, device=self._dev())
        ab = torch.empty((m, 2), dtype=torch.float64, device=self._dev())
        N.check(self._lib.rd_fit_loss_batch(self._h, arr, len(frames), fo.data_ptr(), theta.data_ptr(),
                                            theta0.data_ptr(), m, float(s), loss.data_ptr(), ab.data_ptr()),
                "rd_fit_loss_batch")
        return loss, ab

    def fit_loss_backward_batch(self, frames, theta, theta0, frame_of, s: float, grad_loss,
                                grad_img: torch.Tensor | None = None):
        """(grad_img with d/dI added to the frames' planes back to back, or None; d/dtheta
        float64 [m, 3]) of sum_j grad_loss[j] L_j over up to 64 frames."""
        arr = self._frame_array(frames)
        theta, theta0 = self._thetas(theta), self._thetas(theta0)
        m = theta.shape[0]
        fo = self._frame_of(frame_of, m)
        gl = torch.as_tensor(grad_loss).to(device=self._dev(), dtype=torch.float64).contiguous().reshape(-1)
        if gl.shape[0] != m:
            raise ValueError("grad_loss must have one entry per ring")
        npx = sum(int(a.width) * int(a.height) for a in arr)
        if grad_img is not None and (grad_img.dtype != torch.float32 or not grad_img.is_contiguous()
                                     or grad_img.numel() != npx):
            raise ValueError("grad_img must be a contiguous float32 tensor of the batch's pixels")
        gt = torch.empty((m, 3), dtype=torch.float64, device=self._dev())
        N.check(self._lib.rd_fit_loss_backward_batch(self._h, arr, len(frames), fo.data_ptr(), theta.data_ptr(),
                                                     theta0.data_ptr(), m, float(s), gl.data_ptr(),
                                                     grad_img.data_ptr() if grad_img is not None else None,
                                                     gt.data_ptr()), "rd_fit_loss_backward_batch")
        return grad_img, gt

    def _thetas(self, theta):
        return torch.as_tensor(theta).to(device=self._dev(), dtype=torch.float64).contiguous().reshape(-1, 3)

    def fit_loss(self, frame, theta, theta0, s: float):
        """Ring fit loss per ring (float64 [m]) and (A, B) per ring (float64 [m, 2])."""
        fr = _frame_struct(frame)
        theta, theta0 = self._thetas(theta), self._thetas(theta0)
        m = theta.shape[0]
        loss = torch.empty((m,), dtype=torch.float64, device=self._dev())
        ab = torch.empty((m, 2), dtype=torch.float64, device=self._dev())
        N.check(self._lib.rd_fit_loss(self._h, ctypes.byref(fr), theta.data_ptr(), theta0.data_ptr(), m, float(s),
                                      loss.data_ptr(), ab.data_ptr()), "rd_fit_loss")
        return loss, ab

    def fit_loss_backward(self, frame, theta, theta0, s: float, grad_loss, grad_img: torch.Tensor | None = None):
        """(grad_img with d/dI added, or None; d/dtheta float64 [m, 3]) of sum_j grad_loss[j] L_j."""
        fr = _frame_struct(frame)
        theta, theta0 = self._thetas(theta), self._thetas(theta0)
        m = theta.shape[0]
        gl = torch.as_tensor(grad_loss).to(device=self._dev(), dtype=torch.float64).contiguous().reshape(-1)
        if gl.shape[0] != m:
            raise ValueError("grad_loss must have one entry per ring")
        if grad_img is not None and (grad_img.dtype != torch.float32 or not grad_img.is_contiguous()
                                     or tuple(grad_img.shape) != (fr.height, fr.width)):
            raise ValueError("grad_img must be a contiguous float32 [H, W] tensor")
        gt = torch.empty((m, 3), dtype=torch.float64, device=self._dev())
        N.check(self._lib.rd_fit_loss_backward(self._h, ctypes.byref(fr), theta.data_ptr(), theta0.data_ptr(), m,
                                               float(s), gl.data_ptr(),
                                               grad_img.data_ptr() if grad_img is not None else None,
                                               gt.data_ptr()), "rd_fit_loss_backward")
        return grad_img, gt

    def refine(self, frames, theta0, s: float, iters: int = 20, frame_of=None, tol: float = 0.0,
               return_steps: bool = False):
        """Levenberg-Marquardt refinement: (theta float64 [m, 3], loss float64 [m]), plus the
        steps taken (int32 [m]) with return_steps.  frames is one device frame or a list of up
        to 64; frame_of gives each ring's frame index; a step whose update is within tol
        pixels in every component is a ring's last (tol = 0: `iters` steps)."""
        if not isinstance(frames, (list, tuple)):
            frames = [frames]
        arr = (N.RdFrame * len(frames))(*[_frame_struct(f) for f in frames])
        theta0 = self._thetas(theta0)
        m = theta0.shape[0]
        fo = None
        if frame_of is not None:
            fo = torch.as_tensor(frame_of).to(device=self._dev(), dtype=torch.int32).contiguous().reshape(-1)
            if fo.shape[0] != m:
                raise ValueError("frame_of must have one entry per ring")
        theta = torch.empty((m, 3), dtype=torch.float64, device=self._dev())
        loss = torch.empty((m,), dtype=torch.float64, device=self._dev())
        steps = torch.empty((m,), dtype=torch.int32, device=self._dev()) if return_steps else None
        N.check(self._lib.rd_refine(self._h, arr, len(frames), fo.data_ptr() if fo is not None else None,
                                    theta0.data_ptr(), m, float(s), int(iters), float(tol), theta.data_ptr(),
                                    loss.data_ptr(), steps.data_ptr() if steps is not None else None),
                "rd_refine")
        return (theta, loss, steps) if return_steps else (theta, loss)


def validate_params(params: dict) -> int:
    """Host-only parameter check (no GPU needed); returns an rd_status code."""
    p = N.make_params(params)
    return N.lib().rd_validate_params(ctypes.byref(p))
