"""The differentiable calls over a batch of frames against the same calls frame by frame:
ridges, Hessians, ridge Hessian gradients and ring losses bit for bit; soft accumulators and
image gradients to float32 rounding (their float32 sums run in an order set by atomics: the
soft binning's slots, the gradient planes' adds, which varies from call to call); uneven
frame sizes; the batched autograd functions against the per-frame ones."""
import sys

import numpy as np
import pytest
import torch

from paper_1310_1371_amd import native as N
from paper_1310_1371_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def det():
    from paper_1310_1371_amd.detector import Detector
    d = Detector(max_width=1024, max_height=1024, max_peaks=16384, max_frames=8, max_batch_pixels=8 * 1024 * 1024)
    yield d
    d.close()


@pytest.fixture(scope="module")
def uneven():
    fs = [synth.config4(seed=40 + i, n_frames=1, W=w, H=h, n_rings=n)[0]
          for i, (w, h, n) in enumerate([(256, 256, 10), (384, 200, 12), (300, 300, 14)])]
    return fs


def _close(a, b, rtol, what):
    a, b = a.double().cpu(), b.double().cpu()
    scale = b.abs().max().item() or 1.0
    err = (a - b).abs().max().item()
    say(f"  {what}: max |diff| {err:.3e} (max |ref| {scale:.3e})")
    assert err <= rtol * scale, what


def test_soft_batch_equals_per_frame(det, uneven):
    say("[soft batch] ridges, accumulators, Hessian and image gradients over 3 uneven frames")
    fs = uneven
    p = dict(fs[0].params)
    imgs = [torch.from_numpy(f.image).cuda() for f in fs]
    sizes = [(f.image.shape[1], f.image.shape[0]) for f in fs]
    xy, hess, offs = det.soft_ridges_batch(imgs, p)
    L = p["r_max"] - p["r_min"] + 3
    acc = det.soft_forward_batch(xy, hess, offs, sizes, p)
    rng = np.random.default_rng(7)
    G = torch.from_numpy(rng.normal(size=acc.numel()).astype(np.float32)).cuda()
    gh = det.soft_backward_batch(xy, hess, offs, sizes, p, G)
    gi = det.hessian_backward_batch(xy, gh, offs, sizes, p)
    a0 = g0 = 0
    for i, (img, (w, h)) in enumerate(zip(imgs, sizes)):
        xy1, hess1 = det.soft_ridges(img, p)
        o0, o1 = int(offs[i]), int(offs[i + 1])
        assert torch.equal(xy[o0:o1], xy1) and torch.equal(hess[o0:o1], hess1), i
        acc1 = det.soft_forward(xy1, hess1, w, h, p)
        n_acc = L * w * h
        _close(acc[a0:a0 + n_acc].view(L, h, w), acc1, 2e-6, f"frame {i} soft accumulator")
        G1 = G[a0:a0 + n_acc].view(L, h, w)
        gh1 = det.soft_backward(xy1, hess1, w, h, p, G1)
        assert torch.equal(gh[o0:o1], gh1), i
        gi1 = det.hessian_backward(xy1, gh1, w, h, p)
        _close(gi[g0:g0 + w * h].view(h, w), gi1, 1e-6, f"frame {i} image gradient")
        a0 += n_acc
        g0 += w * h


def test_fit_loss_batch_equals_per_frame(det, uneven):
    say("[soft batch] ring losses and their gradients over 3 uneven frames")
    fs = uneven
    imgs = [torch.from_numpy(f.image).cuda() for f in fs]
    th0 = np.concatenate([np.stack([f.cx, f.cy, f.R], 1) for f in fs])
    th = th0 + np.random.default_rng(2).normal(0, 0.3, th0.shape)
    fo = np.concatenate([np.full(len(f.R), i) for i, f in enumerate(fs)]).astype(np.int32)
    loss, ab = det.fit_loss_batch(imgs, th, th0, fo, 1.5)
    gl = torch.from_numpy(np.random.default_rng(3).normal(size=len(th))).cuda()
    npx = sum(f.image.size for f in fs)
    gimg = torch.zeros(npx, dtype=torch.float32, device="cuda")
    gimg, gt = det.fit_loss_backward_batch(imgs, th, th0, fo, 1.5, gl, gimg)
    k = g0 = 0
    for i, (f, img) in enumerate(zip(fs, imgs)):
        m = len(f.R)
        l1, ab1 = det.fit_loss(img, th[k:k + m], th0[k:k + m], 1.5)
        assert torch.equal(loss[k:k + m], l1) and torch.equal(ab[k:k + m], ab1), i
        g1 = torch.zeros(f.image.shape, dtype=torch.float32, device="cuda")
        g1, gt1 = det.fit_loss_backward(img, th[k:k + m], th0[k:k + m], 1.5, gl[k:k + m], g1)
        assert torch.equal(gt[k:k + m], gt1), i
        _close(gimg[g0:g0 + f.image.size].view(f.image.shape), g1, 1e-6, f"frame {i} image gradient")
        k += m
        g0 += f.image.size
    bad = fo.copy()
    bad[0] = 9
    l2, _ = det.fit_loss_batch(imgs, th, th0, bad, 1.5)
    assert torch.isnan(l2[0]) and not torch.isnan(l2[1:]).any()


def test_autograd_batch_equals_per_frame(det):
    from paper_1310_1371_amd.autograd import (ring_fit_loss, ring_fit_loss_batch, soft_accumulator,
                                              soft_accumulator_batch)
    say("[soft batch] autograd over 4 c4-like frames against per-frame autograd")
    fs = synth.config4(seed=9, n_frames=4, W=512, H=512, n_rings=40)
    p = dict(fs[0].params)
    X = torch.stack([torch.from_numpy(f.image) for f in fs]).cuda()
    th0 = torch.from_numpy(np.concatenate([np.stack([f.cx, f.cy, f.R], 1) for f in fs])).cuda()
    fo = torch.from_numpy(np.concatenate([np.full(len(f.R), i) for i, f in enumerate(fs)]).astype(np.int32)).cuda()
    L = p["r_max"] - p["r_min"] + 3
    G = torch.from_numpy(np.random.default_rng(4).normal(size=(4, L, 512, 512)).astype(np.float32)).cuda()
    xb = X.clone().requires_grad_(True)
    tb = (th0 + 0.2).clone().requires_grad_(True)
    acc = soft_accumulator_batch(xb, det, p)
    loss = ring_fit_loss_batch(xb, tb, th0, fo, det, 1.5)
    torch.autograd.backward([loss.sum(), acc], [None, G])
    k = 0
    for i in range(4):
        x1 = X[i].clone().requires_grad_(True)
        m = len(fs[i].R)
        t1 = (th0[k:k + m] + 0.2).clone().requires_grad_(True)
        a1 = soft_accumulator(x1, det, p)
        l1 = ring_fit_loss(x1, t1, th0[k:k + m], det, 1.5)
        torch.autograd.backward([l1.sum(), a1], [None, G[i]])
        _close(acc[i], a1, 2e-6, f"frame {i} soft accumulator")
        assert torch.equal(loss[k:k + m], l1), i
        assert torch.equal(tb.grad[k:k + m], t1.grad), i
        _close(xb.grad[i], x1.grad, 1e-6, f"frame {i} image gradient")
        k += m


def test_batch_arguments_are_checked(det, uneven):
    fs = uneven
    p = dict(fs[0].params)
    imgs = [torch.from_numpy(f.image).cuda() for f in fs]
    xy, hess, offs = det.soft_ridges_batch(imgs, p)
    bad = offs.copy()
    bad[1] = bad[2] + 1                     # offsets must not decrease
    with pytest.raises(N.RdError) as e:
        det.soft_forward_batch(xy, hess, bad, [(f.image.shape[1], f.image.shape[0]) for f in fs], p)
    assert e.value.status == N.RD_E_INVALID
    with pytest.raises(N.RdError) as e:
        det.soft_ridges_batch(imgs, p, capacity=10)
    assert e.value.status == N.RD_E_TRUNCATED
