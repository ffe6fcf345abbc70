"""The workloads at their full sizes, in the launch configurations bench.py times: batch
equals per-frame (bit-exact, a property at any size), and oracle checks on sampled outputs the
oracle can compute one by one.

  c2 batch  64 x 1024^2 u16 frames, 200 rings each (seeds 1000..1063)
  c3        64 u16 frames of uneven sizes, 50-800 rings each (seed 2)
  c4        1024^2 f32, 300 rings: soft accumulator, adjoint, ring loss, refinement
  c5        one 32-frame launch of the 2048^2 u16 stream, 1000 rings, radii 8-80
"""
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import torch

from oracle import ridge_hough as O
from oracle import soft as S
from paper_1310_1371_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pool_map(fn, items):
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(fn, items))


@pytest.fixture(scope="module")
def det():
    from paper_1310_1371_amd.detector import Detector
    d = Detector(max_width=2048, max_height=2048, max_peaks=16384, max_frames=64,
                 max_batch_pixels=64 * 2048 * 1088)
    yield d
    d.close()


def _key(r):
    return (int(r["a"]), int(r["b"]), int(r["r_bin"]))


def _oracle_match(ref, got):
    kr = {_key(r): r for r in ref}
    kg = {_key(r): r for r in got}
    for k in set(kr) & set(kg):
        a, b = kr[k], kg[k]
        assert abs(a["cx"] - b["cx"]) <= 0.05 and abs(a["cy"] - b["cy"]) <= 0.05 and abs(a["r"] - b["r"]) <= 0.05
    return len(set(kr) ^ set(kg))


def _batch_vs_plain(det, frames, params):
    batch = det.detect_batch(frames, params)
    for i, fr in enumerate(frames):
        one = det.detect(fr, params)
        assert one.tobytes() == batch[i].tobytes(), i
    return batch


def test_c2_batch_of_64(det):
    say("[full] c2 batch of 64 1024^2 frames")
    fs = pool_map(synth.config2, [1000 + i for i in range(64)])
    frames = [torch.from_numpy(f.image).cuda() for f in fs]
    batch = _batch_vs_plain(det, frames, fs[0].params)
    for i in (0, 37):
        ref = O.detect(fs[i].image, fs[i].params)
        unmatched = _oracle_match(ref, batch[i])
        say(f"  frame {i}: oracle {len(ref)}, gpu {len(batch[i])}, unmatched {unmatched}")
        assert unmatched <= max(1, 0.01 * len(ref))


def test_c3_uneven_batch_of_64(det):
    say("[full] c3 uneven batch of 64")
    fs = pool_map(synth.config3_frame, synth.config3_plan(2, 64))
    frames = [torch.from_numpy(f.image).cuda() for f in fs]
    batch = _batch_vs_plain(det, frames, fs[0].params)
    sizes = [f.image.shape for f in fs]
    for shape in ((512, 512), (768, 1024)):
        i = sizes.index(shape)
        ref = O.detect(fs[i].image, fs[i].params)
        unmatched = _oracle_match(ref, batch[i])
        say(f"  frame {i} {shape}: oracle {len(ref)}, gpu {len(batch[i])}, unmatched {unmatched}")
        assert unmatched <= max(1, 0.01 * len(ref))


def test_c4_differentiable_full_frame(det):
    f = synth.config4(seed=3, n_frames=1)[0]
    p = f.params
    img = torch.from_numpy(f.image).cuda()
    H, W = f.image.shape
    xy, hess = det.soft_ridges(img, p)
    say(f"[full] c4 1024^2 f32: {xy.shape[0]} ridges")
    xs, ys = xy[:, 0].cpu().numpy(), xy[:, 1].cpu().numpy()
    h = hess.cpu().numpy()
    geo = S.geometry_from_hessian(h[:, 0], h[:, 1], h[:, 2])
    r_lo, r_hi = S.levels(p)
    acc = det.soft_forward(xy, hess, W, H, p).cpu().numpy()
    ref = S.soft_accumulator(geo, xs, ys, W, H, r_lo, r_hi)
    tol = 2e-6 * np.abs(ref) + 1e-7 * np.abs(ref).max()
    assert np.all(np.abs(acc - ref) <= tol)
    del acc, ref
    G = np.random.default_rng(3).normal(size=(r_hi - r_lo + 1, H, W)).astype(np.float32)
    gw, gux, guy = S.soft_accumulator_vjp(G.astype(np.float64), geo, xs, ys, W, H, r_lo, r_hi)
    dxx, dyy, dxy, _ = S.eigen_vjp(geo, -gw, gux, guy)
    ref_g = np.stack([dxx, dyy, dxy], 1)
    got_g = det.soft_backward(xy, hess, W, H, p, torch.from_numpy(G).cuda()).cpu().numpy()
    assert np.all(np.abs(got_g - ref_g) <= 1e-9 * np.abs(ref_g) + 1e-10 * np.abs(ref_g).max())
    # refinement of every detected ring, 50 of them checked against the oracle
    rings = det.detect(img, p)
    th0 = np.stack([rings["cx"], rings["cy"], rings["r"]], 1).astype(np.float64)
    th, loss = det.refine(img, th0, 1.5, iters=20)
    th = th.cpu().numpy()
    for j in np.random.default_rng(0).choice(len(th0), 50, replace=False):
        ref_th, _ = S.refine(f.image, th0[j], 1.5, iters=20)
        assert np.abs(th[j] - ref_th).max() <= 1e-6, j


def _crop_scores(xs, ys, qx, qy, W, H, a, b, r, p):
    """Oracle S_int on levels r-1..r+1 of the 3x3 box around (a, b), from the votes of every
    ridge computed on a crop that holds the smoothing window of the box."""
    K = max(O.level_radius(l, p) for l in (r - 1, r, r + 1))
    x0, x1 = max(a - 1 - K, 0), min(a + 2 + K, W)
    y0, y1 = max(b - 1 - K, 0), min(b + 2 + K, H)
    A = O.vote(xs - x0, ys - y0, qx, qy, x1 - x0, y1 - y0, r - 1, r + 1)
    # votes that land in the crop but off the frame cannot occur: the crop lies in the frame
    out = np.zeros((3, 3, 3), dtype=np.int64)
    for li, l in enumerate((r - 1, r, r + 1)):
        Sl = O.smooth_level_int(A[li], O.hotspots(A[li], int(p["vote_threshold"])), l, p)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yy, xx = b + dy - y0, a + dx - x0
                if 0 <= yy < Sl.shape[0] and 0 <= xx < Sl.shape[1] and 0 <= b + dy < H and 0 <= a + dx < W:
                    out[li, dy + 1, dx + 1] = Sl[yy, xx]
                else:
                    out[li, dy + 1, dx + 1] = -1
    return out


def _is_peak(box, r, p):
    """The 3x3x3 rule on a box of integer scores (-1: outside the frame)."""
    sv = int(box[1, 1, 1])
    if sv <= O.score_threshold(r, p):
        return False
    for dl in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dl, dy, dx) == (0, 0, 0):
                    continue
                su = int(box[dl + 1, dy + 1, dx + 1])
                if su < 0:
                    continue
                lhs, rhs = sv * (r + dl), su * r
                if (dl, dy, dx) < (0, 0, 0):
                    if not lhs > rhs:
                        return False
                elif not lhs >= rhs:
                    return False
    return True


def test_c5_stream_launch(det):
    st = synth.Stream(seed=4)
    fs = pool_map(st.frame, list(range(32)))
    p = fs[0].params
    say("[full] c5: one 32-frame launch of 2048^2 frames")
    frames = [torch.from_numpy(f.image).cuda() for f in fs]
    batch = _batch_vs_plain(det, frames, p)
    say(f"  rings per frame: {[len(b) for b in batch[:4]]} ...")
    # frame 0: the ridge set at full size, then sampled peaks and fits one by one
    f = fs[0]
    H, W = f.image.shape
    xs, ys, qx, qy, _ = O.ridges(f.image, p)
    xy_g, q_g, _ = det.ridges(frames[0], p)
    sg = set(map(tuple, xy_g.cpu().numpy().tolist()))
    so = set(zip(xs.tolist(), ys.tolist()))
    diff = len(sg ^ so)
    say(f"  ridges: oracle {len(so)}, gpu {len(sg)}, symmetric difference {diff}")
    assert diff <= max(1, 1e-4 * len(so))
    rings = batch[0]
    pp = dict(O.DEFAULTS, **p)
    for j in np.random.default_rng(5).choice(len(rings), 24, replace=False):
        a, b, r = int(rings["a"][j]), int(rings["b"][j]), int(rings["r_bin"][j])
        box = _crop_scores(xs, ys, qx, qy, W, H, a, b, r, pp)
        assert _is_peak(box, r, pp), (a, b, r)
        s_ref = box[1, 1, 1] / (r * O.S_SCALE)
        assert abs(float(rings["score"][j]) - s_ref) <= 1e-6 * s_ref
        fit = O.fit_rings(xs, ys, np.array([a]), np.array([b]), np.array([r]), np.array([box[1, 1, 1]]), pp)[0]
        assert int(fit["fit_ok"]) == int(rings["fit_ok"][j])
        for fld in ("cx", "cy", "r"):
            assert abs(float(fit[fld]) - float(rings[fld][j])) <= 0.05
