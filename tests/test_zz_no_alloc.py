"""rd_detect_noalloc (no context, scratch in a static device array) against rd_detect on the
same frames: two calls in a row, the second on a smaller frame, must give the same ring list
byte for byte (same kernels, same tuning); truncation and the size limit behave as declared."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1310_1371_amd import native as N
from paper_1310_1371_amd import synth
from paper_1310_1371_amd.detector import RING_DTYPE, Detector, _frame_struct

pytestmark = pytest.mark.gpu


def _noalloc(frame: torch.Tensor, params: dict, capacity: int):
    lib = N.lib()
    fr = _frame_struct(frame)
    p = N.make_params(params)
    out = torch.zeros(max(capacity, 1) * RING_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    n = ctypes.c_int32(-1)
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.rd_detect_noalloc(ctypes.byref(fr), ctypes.byref(p), ctypes.c_void_p(stream), out.data_ptr(),
                               capacity, ctypes.byref(n))
    rings = out.cpu().numpy()[:min(n.value, capacity) * RING_DTYPE.itemsize].view(RING_DTYPE)
    return st, n.value, rings


def test_noalloc_matches_detect_on_two_calls_second_smaller():
    big = synth.config2()            # 1024 x 1024 u16, 200 rings, radii 5-70
    small = synth.config1()          # 256 x 256 f32, 8 rings, radii 8-40
    with Detector(max_width=1024, max_height=1024, max_peaks=8192) as det:
        for f in (big, small):
            img = torch.from_numpy(f.image).cuda()
            ref = det.detect(img, f.params)
            print(f"noalloc vs rd_detect: {f.image.shape} {f.image.dtype}, {len(ref)} rings", flush=True)
            st, n, got = _noalloc(img, f.params, 8192)
            assert st == N.RD_OK, N.status_string(st)
            assert n == len(ref) and n > 0
            assert got.tobytes() == ref.tobytes()


def test_noalloc_truncation_and_limits():
    f = synth.config1()
    img = torch.from_numpy(f.image).cuda()
    st, n, full = _noalloc(img, f.params, 8192)
    assert st == N.RD_OK and n >= 2
    st, n2, part = _noalloc(img, f.params, 1)
    assert st == N.RD_E_TRUNCATED and n2 == n
    assert part.tobytes() == full[:1].tobytes()
    big = torch.zeros((1025, 64), dtype=torch.uint16, device="cuda")
    st, _, _ = _noalloc(big, synth.PARAMS_C2, 16)
    assert st == N.RD_E_TOO_LARGE
    host = torch.from_numpy(f.image)             # a host frame is not accepted
    st, _, _ = _noalloc(host, f.params, 16)
    assert st == N.RD_E_INVALID
