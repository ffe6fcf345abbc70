"""The float32 variant of steps 1-2 (rd_params.curvature_fp32 = 1: float32 filters after the
tile mean is taken out of the input) against the float64 oracle: k_- within 1e-5 of max|k_-|,
direction codes within one unit (up to the sign, which names the same axis), ridge sets
within 0.01 % of the oracle's, rings within 0.05 px; batches equal per-frame calls; the
differentiable entry points refuse it."""
import sys

import numpy as np
import pytest
import torch

from oracle import ridge_hough as O
from paper_1310_1371_amd import native as N
from paper_1310_1371_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def det():
    from paper_1310_1371_amd.detector import Detector
    d = Detector(max_width=2048, max_height=2048, max_peaks=65536, max_frames=8, max_batch_pixels=8 * 1024 * 1024)
    yield d
    d.close()


def _fp32(p):
    return dict(p, curvature_fp32=1)


def _stream_frame():
    return synth.Stream(seed=4).frame(0)


FRAMES = {
    "c1_256_f32": synth.config1,
    "ragged_300x170_u16": lambda: synth.config2(seed=21, W=300, H=170, n_rings=12),
    "c2_1024_u16": synth.config2,
    "c5_2048_u16": _stream_frame,
}


def _code_diff(q, qx_ref, qy_ref):
    """Largest component difference of two codes, up to the sign of the code."""
    same = np.maximum(np.abs(q[..., 0] - qx_ref), np.abs(q[..., 1] - qy_ref))
    flip = np.maximum(np.abs(q[..., 0] + qx_ref), np.abs(q[..., 1] + qy_ref))
    return np.minimum(same, flip)


@pytest.mark.parametrize("name", ["c1_256_f32", "ragged_300x170_u16", "c2_1024_u16"])
def test_fp32_curvature(det, name):
    say(f"[fp32] curvature {name}")
    f = FRAMES[name]()
    p = f.params
    k_ref, qx_ref, qy_ref = O.curvature(f.image.astype(np.float64), O.f32(p["sigma_smooth"]))
    k, q = det.curvature(torch.from_numpy(f.image).cuda(), _fp32(p))
    k = k.cpu().numpy().astype(np.float64)
    q = q.cpu().numpy().astype(np.int64)
    err = np.abs(k - k_ref)
    kmax = np.abs(k_ref).max()
    say(f"  max |dk| {err.max():.3e} = {err.max() / kmax:.2e} max|k|")
    assert err.max() <= 1e-5 * kmax
    # a Hessian error dH turns X_- by about dH / d (d: half the eigengap), so a code is held
    # to one unit (2^-14 rad) only where d >= 2^14 dH, with dH taken as the largest k_- error
    Ixx, Iyy, Ixy = O.hessian(f.image.astype(np.float64), O.f32(p["sigma_smooth"]))
    resolved = np.hypot(0.5 * (Ixx - Iyy), Ixy) > 16384.0 * err.max()
    dq = _code_diff(q, qx_ref, qy_ref)
    far = int(((dq > 1) & resolved).sum())
    say(f"  codes more than one unit off where resolved ({int(resolved.sum())} px): {far}")
    assert far <= max(1, 1e-5 * k.size)


@pytest.mark.parametrize("name", ["ragged_300x170_u16", "c2_1024_u16", "c5_2048_u16"])
def test_fp32_ridge_sets(det, name):
    say(f"[fp32] ridges {name}")
    f = FRAMES[name]()
    p = f.params
    xs, ys, qx, qy, _ = O.ridges(f.image, p)
    xy, q, _ = det.ridges(torch.from_numpy(f.image).cuda(), _fp32(p))
    xy, q = xy.cpu().numpy().astype(np.int64), q.cpu().numpy().astype(np.int64)
    ref = {(int(x), int(y)): (int(a), int(b)) for x, y, a, b in zip(xs, ys, qx, qy)}
    got = {(int(x), int(y)): (int(a), int(b)) for (x, y), (a, b) in zip(xy, q)}
    sym = set(ref) ^ set(got)
    say(f"  oracle {len(ref)} gpu {len(got)} mismatched {len(sym)} ({100.0 * len(sym) / len(ref):.4f} %)")
    assert len(sym) <= 1e-4 * len(ref)
    common = set(ref) & set(got)
    a = np.array([ref[key] for key in common])
    b = np.array([got[key] for key in common])
    assert _code_diff(b[:, None, :], a[:, 0:1], a[:, 1:2]).max() <= 1


def test_fp32_rings_c2(det):
    say("[fp32] rings c2 1024x1024 u16")
    f = synth.config2()
    ref = O.detect(f.image, f.params)
    got = det.detect(torch.from_numpy(f.image).cuda(), _fp32(f.params))
    kr = {(int(r["a"]), int(r["b"]), int(r["r_bin"])): r for r in ref}
    kg = {(int(r["a"]), int(r["b"]), int(r["r_bin"])): r for r in got}
    unmatched = len(set(kr) ^ set(kg))
    say(f"  oracle {len(ref)} gpu {len(got)} unmatched {unmatched}")
    assert unmatched <= max(1, 0.01 * len(ref))
    for key in set(kr) & set(kg):
        for fld in ("cx", "cy", "r"):
            assert abs(float(kr[key][fld]) - float(kg[key][fld])) <= 0.05


def test_fp32_batch_equals_per_frame(det):
    say("[fp32] uneven batch against per-frame calls")
    fs = [synth.config2(seed=300 + i, W=w, H=h, n_rings=n) for i, (w, h, n) in
          enumerate([(512, 512, 50), (1024, 768, 150), (300, 170, 12), (640, 480, 80)])]
    p = _fp32(fs[0].params)
    frames = [torch.from_numpy(f.image).cuda() for f in fs]
    batch = det.detect_batch(frames, p)
    for i, fr in enumerate(frames):
        assert det.detect(fr, p).tobytes() == batch[i].tobytes(), i


def test_fp32_refused_by_the_differentiable_path(det):
    f = synth.config1()
    with pytest.raises(N.RdError) as e:
        det.soft_ridges(torch.from_numpy(f.image).cuda(), _fp32(f.params))
    assert e.value.status == N.RD_E_INVALID
