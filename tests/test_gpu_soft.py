"""Parity of the differentiable path (HIP kernels through the C ABI) with the FP64 oracle:
ridge Hessians, soft accumulator and its adjoint, Hessian adjoint with reflect-101 fold-back,
ring fit loss and its gradient, Levenberg-Marquardt refinement, and the autograd wrappers."""
import sys

import numpy as np
import pytest
import torch

from oracle import ridge_hough as O
from oracle import soft as S
from paper_1310_1371_amd import synth
from paper_1310_1371_amd import native as N

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def det():
    from paper_1310_1371_amd.detector import Detector
    d = Detector(max_width=1024, max_height=1024, max_peaks=16384)
    yield d
    d.close()


def _oracle_hess(img, params):
    p = dict(O.DEFAULTS, **params)
    return O.hessian(np.asarray(img, dtype=np.float64), O.f32(p["sigma_smooth"]))


def _ridges_and_hess(img, params):
    xs, ys, _, _, _ = O.ridges(img, params)
    Ixx, Iyy, Ixy = _oracle_hess(img, params)
    hess = np.stack([Ixx[ys, xs], Iyy[ys, xs], Ixy[ys, xs]], 1)
    return xs, ys, hess


def _close(got, ref, rtol, atol_rel, what):
    """|got - ref| <= rtol |ref| + atol_rel max|ref| elementwise; returns the worst ratio."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    tol = rtol * np.abs(ref) + atol_rel * max(np.abs(ref).max(), 1e-300)
    bad = np.abs(got - ref) > tol
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} off, worst {np.abs(got - ref)[bad].max():.3e}"
    return float((np.abs(got - ref) / np.maximum(tol, 1e-300)).max())


# ------------------------------------------------------------------------- ridges + Hessian

@pytest.mark.parametrize("case", ["c1", "ragged_u16"])
def test_soft_ridges_and_hessian(det, case):
    say(f"[soft] ridges + Hessian {case}")
    if case == "c1":
        f = synth.config1()
    else:
        f = synth.config2(seed=5, W=300, H=170, n_rings=12)
    img = torch.from_numpy(f.image).cuda()
    xy, hess = det.soft_ridges(img, f.params)
    xy_plain, _, _ = det.ridges(img, f.params)
    assert torch.equal(xy, xy_plain)
    xy = xy.cpu().numpy()
    Ixx, Iyy, Ixy = _oracle_hess(f.image, f.params)
    ref = np.stack([Ixx[xy[:, 1], xy[:, 0]], Iyy[xy[:, 1], xy[:, 0]], Ixy[xy[:, 1], xy[:, 0]]], 1)
    _close(hess.cpu().numpy(), ref, 1e-9, 1e-11, "hessian")


# ------------------------------------------------------------------------- soft accumulator

def _soft_case(name):
    if name == "c1":
        f = synth.config1()
        return f.image, f.params
    if name == "ragged":
        f = synth.config2(seed=6, W=300, H=170, n_rings=12)
        return f.image, dict(f.params, r_min=5, r_max=40)
    if name == "min_frame":
        f = synth.single_ring(32, 32, 15.0, 16.0, 9.3)
        return f.image, dict(f.params, r_min=4, r_max=20)
    if name == "max_radius":
        f = synth.config1(seed=2)
        return f.image, dict(f.params, r_min=90, r_max=126)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["c1", "ragged", "min_frame", "max_radius"])
def test_soft_forward_matches_oracle(det, name):
    img, params = _soft_case(name)
    H, W = img.shape
    xs, ys, hess = _ridges_and_hess(img, params)
    say(f"[soft] forward {name}: {W}x{H}, {len(xs)} ridges")
    r_lo, r_hi = S.levels(params)
    geo = S.geometry_from_hessian(hess[:, 0], hess[:, 1], hess[:, 2])
    ref = S.soft_accumulator(geo, xs, ys, W, H, r_lo, r_hi)
    xy = np.stack([xs, ys], 1)
    got = det.soft_forward(xy, hess, W, H, params).cpu().numpy()
    assert got.shape == ref.shape
    # w beta per splat rounded once to float32, sums of positive terms in float32
    _close(got, ref, 2e-6, 1e-7, "soft accumulator")


def test_soft_forward_empty_and_errors(det):
    from paper_1310_1371_amd import native as N
    say("[soft] empty ridge list, off-frame ridge")
    params = dict(synth.PARAMS_C1, r_min=5, r_max=9)
    acc = det.soft_forward(np.zeros((0, 2), np.int32), np.zeros((0, 3)), 64, 48, params)
    assert acc.shape == (7, 48, 64) and not acc.any()
    with pytest.raises(N.RdError) as e:
        det.soft_forward(np.array([[64, 3]], np.int32), np.array([[-1.0, 0.0, 0.0]]), 64, 48, params)
    assert e.value.status == N.RD_E_INVALID


@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_soft_backward_matches_oracle(det, name):
    img, params = _soft_case(name)
    H, W = img.shape
    xs, ys, hess = _ridges_and_hess(img, params)
    say(f"[soft] backward {name}: {len(xs)} ridges")
    r_lo, r_hi = S.levels(params)
    G = np.random.default_rng(7).normal(size=(r_hi - r_lo + 1, H, W)).astype(np.float32)
    geo = S.geometry_from_hessian(hess[:, 0], hess[:, 1], hess[:, 2])
    gw, gux, guy = S.soft_accumulator_vjp(G.astype(np.float64), geo, xs, ys, W, H, r_lo, r_hi)
    dxx, dyy, dxy, dropped = S.eigen_vjp(geo, -gw, gux, guy)
    ref = np.stack([dxx, dyy, dxy], 1)
    got, n_iso = det.soft_backward(np.stack([xs, ys], 1), hess, W, H, params, torch.from_numpy(G).cuda(),
                                   count_isotropic=True)
    assert n_iso == dropped
    # float64 sums of the same float32 inputs: only the summation order differs
    _close(got.cpu().numpy(), ref, 1e-9, 1e-10, "soft backward")


@pytest.mark.parametrize("shape", [(48, 40), (300, 170)])
def test_hessian_backward_matches_oracle(det, shape):
    W, H = shape
    say(f"[soft] Hessian adjoint {W}x{H}")
    rng = np.random.default_rng(W)
    yy, xx = np.mgrid[0:H, 0:W]
    border = (np.minimum(np.minimum(xx, W - 1 - xx), np.minimum(yy, H - 1 - yy)) <= 9).ravel()
    pick = np.flatnonzero(border | (rng.random(W * H) < 0.05))
    xs, ys = xx.ravel()[pick], yy.ravel()[pick]
    gh = rng.normal(size=(len(xs), 3))
    params = dict(synth.PARAMS_C1)
    planes = [np.zeros((H, W)) for _ in range(3)]
    for c in range(3):
        planes[c][ys, xs] = gh[:, c]
    ref = S.hessian_adjoint(*planes, O.f32(params["sigma_smooth"]))
    base = torch.full((H, W), 0.5, dtype=torch.float32, device="cuda")
    got = det.hessian_backward(np.stack([xs, ys], 1), gh, W, H, params, base.clone())
    # float32 planes between the passes; the call adds into the given buffer
    _close(got.cpu().numpy() - 0.5, ref, 1e-5, 2e-6, "hessian adjoint")


# ------------------------------------------------------------------------- ring fit

@pytest.fixture(scope="module")
def c4_frame():
    return synth.config4(seed=3, n_frames=1, W=512, H=512, n_rings=80)[0]


def _perturbed(f, n, seed=0, sd=0.3):
    rng = np.random.default_rng(seed)
    th0 = np.stack([f.cx[:n], f.cy[:n], f.R[:n]], 1)
    return th0 + rng.normal(0, sd, th0.shape), th0


def test_fit_loss_matches_oracle(det, c4_frame):
    f = c4_frame
    th, th0 = _perturbed(f, 60)
    say(f"[fit] loss and gradient, {len(th)} rings on 512^2 f32")
    img = torch.from_numpy(f.image).cuda()
    loss, ab = det.fit_loss(img, th, th0, 1.5)
    gl = np.random.default_rng(1).uniform(0.5, 2.0, len(th))
    gimg, gth = det.fit_loss_backward(img, th, th0, 1.5, gl, torch.zeros_like(img))
    ref_l = np.array([S.fit_loss(f.image, a, b, 1.5)[0] for a, b in zip(th, th0)])
    ref_ab = np.array([S.fit_loss(f.image, a, b, 1.5)[1:] for a, b in zip(th, th0)])
    _close(loss.cpu().numpy(), ref_l, 1e-10, 0, "loss")
    _close(ab.cpu().numpy(), ref_ab, 1e-9, 1e-12, "A, B")
    ref_gi = np.zeros(f.image.shape)
    ref_gt = np.zeros_like(th)
    for j, (a, b) in enumerate(zip(th, th0)):
        xs, ys, dv, dt = S.fit_loss_grad(f.image, a, b, 1.5)
        np.add.at(ref_gi, (ys, xs), gl[j] * dv)
        ref_gt[j] = gl[j] * dt
    _close(gth.cpu().numpy(), ref_gt, 1e-8, 1e-10, "dL/dtheta")
    _close(gimg.cpu().numpy(), ref_gi, 1e-6, 1e-7, "dL/dI")


def test_fit_loss_u16_frame(det):
    f = synth.config2(seed=8, W=300, H=170, n_rings=12)
    th, th0 = _perturbed(f, len(f.R), seed=2)
    say("[fit] u16 frame")
    loss, ab = det.fit_loss(torch.from_numpy(f.image).cuda(), th, th0, 1.5)
    ref = np.array([S.fit_loss(f.image, a, b, 1.5)[0] for a, b in zip(th, th0)])
    _close(loss.cpu().numpy(), ref, 1e-10, 0, "u16 loss")


def test_refine_matches_oracle(det, c4_frame):
    f = c4_frame
    _, th0 = _perturbed(f, 40)
    th0 = th0 + np.random.default_rng(3).normal(0, 0.5, th0.shape)
    say(f"[fit] refine {len(th0)} rings, 20 steps")
    th, loss = det.refine(torch.from_numpy(f.image).cuda(), th0, 1.5, iters=20)
    th = th.cpu().numpy()
    for j in range(len(th0)):
        ref_th, ref_l = S.refine(f.image, th0[j], 1.5, iters=20)
        assert np.abs(th[j] - ref_th).max() <= 1e-6, (j, th[j], ref_th)
        assert abs(loss[j].item() - ref_l) <= 1e-9 * ref_l


def test_refine_tol_matches_oracle(det, c4_frame):
    # the convergence stop: rings, losses and step counts against the oracle's.  The kernel
    # takes the loss as sum I^2 - A sum I g - B sum I, whose rounding (about 1e-13 here) hides
    # the loss change of steps below about 2e-8 px, so the tolerance sits well above that
    f = c4_frame
    _, th0 = _perturbed(f, 40)
    th0 = th0 + np.random.default_rng(3).normal(0, 0.5, th0.shape)
    say(f"[fit] refine {len(th0)} rings, tol 1e-6")
    th, loss, steps = det.refine(torch.from_numpy(f.image).cuda(), th0, 1.5, iters=20, tol=1e-6, return_steps=True)
    th, steps = th.cpu().numpy(), steps.cpu().numpy()
    for j in range(len(th0)):
        ref_th, ref_l, ref_n = S.refine(f.image, th0[j], 1.5, iters=20, tol=1e-6, return_steps=True)
        assert steps[j] == ref_n, (j, steps[j], ref_n)
        assert np.abs(th[j] - ref_th).max() <= 1e-6, (j, th[j], ref_th)
        assert abs(loss[j].item() - ref_l) <= 1e-9 * ref_l
    say(f"  steps: mean {steps.mean():.2f}, max {steps.max()}")
    assert steps.max() < 20


def test_refine_tol_limits(det, c4_frame):
    f = c4_frame
    img = torch.from_numpy(f.image).cuda()
    _, th0 = _perturbed(f, 12)
    th0 = th0 + 0.4
    # tol = 0 runs every step; an infinite tol stops after the first, equal to iters = 1
    _, _, n0 = det.refine(img, th0, 1.5, iters=9, tol=0.0, return_steps=True)
    assert (n0.cpu().numpy() == 9).all()
    t1, l1 = det.refine(img, th0, 1.5, iters=1)
    ti, li, ni = det.refine(img, th0, 1.5, iters=20, tol=float("inf"), return_steps=True)
    assert (ni.cpu().numpy() == 1).all() and torch.equal(t1, ti) and torch.equal(l1, li)
    for bad in (-1e-9, float("nan")):
        with pytest.raises(N.RdError) as e:
            det.refine(img, th0, 1.5, iters=5, tol=bad)
        assert e.value.status == N.RD_E_INVALID


def test_refine_noise_free_ring_converges(det):
    theta = np.array([40.3, 37.6, 20.45])
    img = S.render_ring(96, 96, theta, 1.5, 1.0, 0.2).astype(np.float32)
    say("[fit] refine noise-free ring")
    starts = theta + np.array([[0.8, -0.6, 0.7], [-1.0, 0.5, -0.8], [0.3, 0.9, 1.2]])
    th, loss = det.refine(torch.from_numpy(img).cuda(), starts, 1.5, iters=20)
    th = th.cpu().numpy()
    # the image is float32 (profile rounded to ~6e-8); the fit runs in float64
    assert np.abs(th - theta).max() <= 1e-3
    for j, st in enumerate(starts):
        ref, _ = S.refine(img, st, 1.5, iters=20)
        assert np.abs(th[j] - ref).max() <= 1e-6


def test_refine_batch_of_frames(det):
    fs = synth.config4(seed=4, n_frames=3, W=256, H=256, n_rings=10)
    say("[fit] refine over 3 frames with a frame index")
    imgs = [torch.from_numpy(f.image).cuda() for f in fs]
    th0 = np.concatenate([np.stack([f.cx, f.cy, f.R], 1) + 0.4 for f in fs])
    fo = np.concatenate([np.full(len(f.R), i) for i, f in enumerate(fs)]).astype(np.int32)
    th, loss = det.refine(imgs, th0, 1.5, iters=20, frame_of=fo)
    k = 0
    for i, f in enumerate(fs):
        t1, l1 = det.refine(imgs[i], th0[k:k + len(f.R)], 1.5, iters=20)
        assert torch.equal(th[k:k + len(f.R)], t1) and torch.equal(loss[k:k + len(f.R)], l1)
        k += len(f.R)
    bad = fo.copy()
    bad[0] = 7
    th2, _ = det.refine(imgs, th0, 1.5, iters=2, frame_of=bad)
    assert torch.isnan(th2[0]).all() and not torch.isnan(th2[1:]).any()


# ------------------------------------------------------------------------- autograd

def test_autograd_check_objective(det):
    """L = sum_j L_j + <G, A~> through both autograd functions against the oracle gradient."""
    from paper_1310_1371_amd.autograd import ring_fit_loss, soft_accumulator
    W = H = 96
    truth = [(30.3, 40.6, 14.4), (70.2, 61.7, 18.3), (85.0, 10.0, 12.0)]
    img = np.full((H, W), 0.2)
    for t in truth:
        img = img + S.render_ring(W, H, t, 1.5, 1.0, 0.0)
    img = (img + np.random.default_rng(9).normal(0, 0.05, img.shape)).astype(np.float32)
    params = dict(O.DEFAULTS, r_min=8, r_max=22, k_threshold=-0.02)
    r_lo, r_hi = S.levels(params)
    G = np.random.default_rng(10).normal(size=(r_hi - r_lo + 1, H, W)).astype(np.float32)
    th0 = np.array(truth)
    th = th0 + np.array([0.2, -0.3, 0.25])
    say("[autograd] check objective on 96x96")

    image = torch.from_numpy(img).cuda().requires_grad_(True)
    theta = torch.from_numpy(th).cuda().requires_grad_(True)
    acc = soft_accumulator(image, det, params)
    loss = ring_fit_loss(image, theta, torch.from_numpy(th0).cuda(), det, 1.5)
    total = loss.sum() + (torch.from_numpy(G).cuda() * acc).sum().double()
    total.backward()

    xs, ys, _, _, _ = O.ridges(img, params)
    ref_dI, ref_dth, _ = S.objective_grad(img.astype(np.float64), params, xs, ys, list(th), list(th0), 1.5,
                                          G.astype(np.float64))
    ref_L = S.objective(img.astype(np.float64), params, xs, ys, list(th), list(th0), 1.5, G.astype(np.float64))
    assert abs(total.item() - ref_L) <= 1e-5 * abs(ref_L) + 1e-4
    _close(theta.grad.cpu().numpy(), ref_dth, 1e-8, 1e-10, "dL/dtheta")
    _close(image.grad.cpu().numpy(), ref_dI, 1e-4, 1e-5, "dL/dI")


def test_large_window_streams_from_the_frame(det):
    """A ring whose window holds more pixels than the per-ring list (r ~ 100 px, about 8200
    pixels) is fitted by walking its bounding box on every pass: same results."""
    theta = np.array([128.4, 127.7, 100.3])
    rng = np.random.default_rng(5)
    img = (S.render_ring(256, 256, theta, 1.5, 1.0, 0.2) + rng.normal(0, 0.05, (256, 256))).astype(np.float32)
    th0 = theta + np.array([[0.5, -0.4, 0.6]])
    assert len(S.ring_window(th0[0], 1.5, 256, 256)[0]) > 6144
    say("[fit] large window")
    t = torch.from_numpy(img).cuda()
    th, loss = det.refine(t, th0, 1.5, iters=20)
    ref_th, ref_l = S.refine(img, th0[0], 1.5, iters=20)
    assert np.abs(th.cpu().numpy()[0] - ref_th).max() <= 1e-6
    assert abs(loss[0].item() - ref_l) <= 1e-9 * ref_l
    l2, ab = det.fit_loss(t, th0 + 0.2, th0, 1.5)
    assert abs(l2[0].item() - S.fit_loss(img, th0[0] + 0.2, th0[0], 1.5)[0]) <= 1e-10 * l2[0].item()
