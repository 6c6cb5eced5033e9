"""Torch-facing API: render options, a Renderer that owns the library context
and acceleration structure, and the autograd.Function whose forward and
backward call the C ABI.  PyTorch provides device memory and the stream; all
arithmetic runs in librgx.so."""
from __future__ import annotations

import dataclasses

import torch

from . import lib

PARAM_KEYS = ("means", "log_scales", "quats", "density", "sh")


@dataclasses.dataclass
class RenderOptions:
    """Mirror of rgx_render_opts.  Defaults: the paper's real-scene adaptive
    sampling constants (Sec. 4.2) and its uniform synthetic step."""
    adaptive: bool = False
    dt: float = 0.0025
    dt_min: float = 0.005
    dt_max: float = 0.02
    beta: float = 1024.0
    n_s: int = 8
    t_eps: float = 1e-4
    ess: int = 1
    brute_force: bool = False
    ray_order: int = 1
    tile_w: int = 8
    tile_h: int = 8
    persistent: bool = False
    window_segments: int = 1
    bg: tuple = (0.0, 0.0, 0.0)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def n_rays(cams) -> int:
    return sum(int(c.width) * int(c.height) for c in cams)


class Renderer:
    """Owns an rgx context and acceleration structure on one device."""

    def __init__(self, device: int = 0, sigma_eps: float = 0.01, morton_bits: int = 21):
        self.ctx = lib.Context(device)
        self.bvh = lib.BVH(self.ctx)
        self.sigma_eps = sigma_eps
        self.morton_bits = morton_bits
        self._key = None

    def build(self, params: dict, sh_degree: int, force: bool = False):
        key = tuple((params[k].data_ptr(), params[k]._version) for k in PARAM_KEYS)
        if force or key != self._key:
            for k in PARAM_KEYS:
                t = params[k]
                if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                    raise ValueError(f"{k} must be a contiguous float32 device tensor")
            self.bvh.build(params["means"], params["log_scales"], params["quats"],
                           params["density"], params["sh"], sh_degree, self.sigma_eps,
                           self.morton_bits, _stream())
            self._key = key
        return self

    def forward(self, cams, opts: RenderOptions, stats: bool = False):
        R = n_rays(cams)
        dev = torch.device("cuda", self.ctx.device)
        rgb = torch.empty((R, 3), device=dev, dtype=torch.float32)
        T = torch.empty((R,), device=dev, dtype=torch.float32)
        st = torch.zeros((R, lib.NSTAT), device=dev, dtype=torch.int32) if stats else None
        lib.render_forward(self.ctx, self.bvh, cams, opts, rgb, T, st, _stream())
        return (rgb, T, st) if stats else (rgb, T)

    def backward(self, cams, opts: RenderOptions, rgb, T, grad_rgb, grad_T, params: dict,
                 densify=None, densify_views=None):
        """Parameter gradients; with `densify` / `densify_views` ([n] float32 /
        int32 device tensors) also adds the densification statistic of each
        view (per-view mean-gradient norms weighted by distance / focal)."""
        grads = {k: torch.empty_like(params[k]) for k in PARAM_KEYS}
        lib.render_backward(self.ctx, self.bvh, cams, opts, rgb, T, grad_rgb.contiguous(),
                            None if grad_T is None else grad_T.contiguous(), grads, False,
                            _stream(), densify, densify_views)
        return grads

    def close(self):
        self.bvh.close()
        self.ctx.close()


class RayMarchFunction(torch.autograd.Function):
    """(means, log_scales, quats, density, sh) -> (rgb [R,3], T [R]).

    The forward (re)builds the acceleration structure when a parameter tensor
    changed (data pointer or version), then renders; the backward re-traverses
    the same segments and returns gradients for the five parameter tensors."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, density, sh, renderer: Renderer, cams,
                opts: RenderOptions, sh_degree: int):
        params = dict(means=means, log_scales=log_scales, quats=quats, density=density, sh=sh)
        renderer.build(params, sh_degree)
        rgb, T = renderer.forward(cams, opts)
        ctx.renderer, ctx.cams, ctx.opts = renderer, cams, opts
        ctx.save_for_backward(means, log_scales, quats, density, sh, rgb, T)
        return rgb, T

    @staticmethod
    def backward(ctx, grad_rgb, grad_T):
        means, log_scales, quats, density, sh, rgb, T = ctx.saved_tensors
        params = dict(means=means, log_scales=log_scales, quats=quats, density=density, sh=sh)
        if grad_rgb is None:
            grad_rgb = torch.zeros_like(rgb)
        g = ctx.renderer.backward(ctx.cams, ctx.opts, rgb, T, grad_rgb, grad_T, params)
        return g["means"], g["log_scales"], g["quats"], g["density"], g["sh"], None, None, None, None


def render(params: dict, sh_degree: int, renderer: Renderer, cams, opts: RenderOptions):
    return RayMarchFunction.apply(params["means"], params["log_scales"], params["quats"],
                                  params["density"], params["sh"], renderer, cams, opts, sh_degree)


class TrainStep:
    """One training step of the ray marcher as a replayable HIP graph.

    The step rebuilds the acceleration structure from the current parameter
    values, renders every view in one batched launch, evaluates `loss_fn`
    on (rgb, T), back-propagates through RayMarchFunction and applies
    p -= lr * grad in place.  It is captured once (after warm-up calls that
    size every buffer, so nothing is allocated inside the graph) and replayed
    with a single launch per step.  All library work is kernels on the
    capturing stream; accumulators and work queues are cleared by kernels,
    never by memset nodes."""

    def __init__(self, renderer: Renderer, params: dict, sh_degree: int, cams,
                 opts: RenderOptions, loss_fn, lr: float = 0.0, warmup: int = 2):
        self.renderer, self.params, self.deg = renderer, params, sh_degree
        self.cams, self.opts, self.loss_fn, self.lr = cams, opts, loss_fn, lr
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self._step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.loss, self.rgb, self.T = self._step()
        self.grads = {k: params[k].grad for k in PARAM_KEYS}

    def _step(self):
        for p in self.params.values():
            p.grad = None
        self.renderer.build(self.params, self.deg, force=True)
        rgb, T = render(self.params, self.deg, self.renderer, self.cams, self.opts)
        loss = self.loss_fn(rgb, T)
        loss.backward()
        if self.lr:
            with torch.no_grad():
                for p in self.params.values():
                    p.add_(p.grad, alpha=-self.lr)
        return loss.detach(), rgb.detach(), T.detach()

    def replay(self):
        self.graph.replay()
        return self.loss


class IsotropicLossFunction(torch.autograd.Function):
    """Isotropic scale loss (library kernel): mean over Gaussians of
    max(r, r0) - r0, r the AABB/ellipsoid volume-ratio bound of the scales."""

    @staticmethod
    def forward(ctx, log_scales, renderer: Renderer, r0: float):
        ls = log_scales.contiguous()
        loss = torch.empty((), device=ls.device, dtype=torch.float32)
        grad = torch.empty_like(ls)
        lib.isotropic_loss(renderer.ctx, ls, r0, loss, grad, False, _stream())
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g, None, None


def isotropic_loss(log_scales, renderer: Renderer, r0: float = 10.0):
    return IsotropicLossFunction.apply(log_scales, renderer, r0)
