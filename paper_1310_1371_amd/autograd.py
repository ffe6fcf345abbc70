"""torch.autograd wrappers of the differentiable extension.  Forward and backward both run in
the library's HIP kernels (soft accumulator and its adjoint, eigen and Hessian adjoints,
ring-profile loss and its gradient); torch only holds the tensors.

    acc = soft_accumulator(image, det, params)        # float32 [L, H, W], differentiable in image
    loss = ring_fit_loss(image, theta, theta0, det, s)  # float64 [m], differentiable in image, theta

and over a batch of frames of one size, one library call per step instead of one per frame:

    acc = soft_accumulator_batch(images, det, params)                # [F, L, H, W] from [F, H, W]
    loss = ring_fit_loss_batch(images, theta, theta0, frame_of, det, s)

The ridge set of the soft accumulator is taken from the image at forward time and held fixed
(ridge selection is a threshold, not differentiable).
"""
from __future__ import annotations

import torch


class SoftAccumulator(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image, det, params):
        if image.dtype != torch.float32 or not image.is_cuda or image.dim() != 2:
            raise TypeError("image must be a 2D float32 CUDA tensor")
        img = image.detach()
        H, W = img.shape
        xy, hess = det.soft_ridges(img, params)
        acc = det.soft_forward(xy, hess, W, H, params)
        ctx.save_for_backward(xy, hess)
        ctx.det, ctx.params, ctx.shape = det, params, (H, W)
        return acc

    @staticmethod
    def backward(ctx, grad_acc):
        xy, hess = ctx.saved_tensors
        H, W = ctx.shape
        grad_img = None
        if ctx.needs_input_grad[0]:
            gh = ctx.det.soft_backward(xy, hess, W, H, ctx.params, grad_acc)
            grad_img = ctx.det.hessian_backward(xy, gh, W, H, ctx.params)
        return grad_img, None, None


class RingFitLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image, theta, theta0, det, s):
        if image.dim() != 2 or not image.is_cuda:
            raise TypeError("image must be a 2D CUDA tensor")
        img = image.detach()
        loss, _ = det.fit_loss(img, theta.detach(), theta0, s)
        ctx.save_for_backward(img, theta.detach(), theta0)
        ctx.det, ctx.s = det, s
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        img, theta, theta0 = ctx.saved_tensors
        grad_img = None
        if ctx.needs_input_grad[0]:
            if img.dtype != torch.float32:
                raise TypeError("image gradients need a float32 image")
            grad_img = torch.zeros(img.shape, dtype=torch.float32, device=img.device)
        grad_img, grad_theta = ctx.det.fit_loss_backward(img, theta, theta0, ctx.s, grad_loss, grad_img)
        return grad_img, grad_theta.to(theta.dtype), None, None, None


class SoftAccumulatorBatch(torch.autograd.Function):
    @staticmethod
    def forward(ctx, images, det, params):
        if images.dtype != torch.float32 or not images.is_cuda or images.dim() != 3:
            raise TypeError("images must be a 3D float32 CUDA tensor [F, H, W]")
        imgs = images.detach().contiguous()
        F, H, W = imgs.shape
        xy, hess, offs = det.soft_ridges_batch(list(imgs), params)
        acc = det.soft_forward_batch(xy, hess, offs, [(W, H)] * F, params)
        ctx.save_for_backward(xy, hess)
        ctx.det, ctx.params, ctx.shape, ctx.offs = det, params, (F, H, W), offs
        return acc

    @staticmethod
    def backward(ctx, grad_acc):
        xy, hess = ctx.saved_tensors
        F, H, W = ctx.shape
        grad_img = None
        if ctx.needs_input_grad[0]:
            sizes = [(W, H)] * F
            gh = ctx.det.soft_backward_batch(xy, hess, ctx.offs, sizes, ctx.params, grad_acc)
            grad_img = ctx.det.hessian_backward_batch(xy, gh, ctx.offs, sizes, ctx.params).view(F, H, W)
        return grad_img, None, None


class RingFitLossBatch(torch.autograd.Function):
    @staticmethod
    def forward(ctx, images, theta, theta0, frame_of, det, s):
        if images.dim() != 3 or not images.is_cuda:
            raise TypeError("images must be a 3D CUDA tensor [F, H, W]")
        imgs = images.detach().contiguous()
        frames = list(imgs)
        loss, _ = det.fit_loss_batch(frames, theta.detach(), theta0, frame_of, s)
        ctx.save_for_backward(imgs, theta.detach(), theta0, torch.as_tensor(frame_of))
        ctx.det, ctx.s = det, s
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        imgs, theta, theta0, frame_of = ctx.saved_tensors
        grad_img = None
        if ctx.needs_input_grad[0]:
            if imgs.dtype != torch.float32:
                raise TypeError("image gradients need float32 images")
            grad_img = torch.zeros(imgs.shape, dtype=torch.float32, device=imgs.device)
        grad_img, grad_theta = ctx.det.fit_loss_backward_batch(list(imgs), theta, theta0, frame_of, ctx.s,
                                                               grad_loss, grad_img)
        return grad_img, grad_theta.to(theta.dtype), None, None, None, None


def soft_accumulator(image, det, params):
    return SoftAccumulator.apply(image, det, params)


def ring_fit_loss(image, theta, theta0, det, s: float):
    return RingFitLoss.apply(image, theta, theta0, det, s)


def soft_accumulator_batch(images, det, params):
    return SoftAccumulatorBatch.apply(images, det, params)


def ring_fit_loss_batch(images, theta, theta0, frame_of, det, s: float):
    return RingFitLossBatch.apply(images, theta, theta0, frame_of, det, s)
