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
    no_record: bool = False
    no_sample_record: bool = False


def _keys(params: dict):
    """The parameter tensors of a scene: the five of every scene, and the
    spherical-Gaussian lobes when present."""
    return PARAM_KEYS + (("sg",) if params.get("sg") is not None else ())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def n_rays(cams) -> int:
    return sum(int(c.width) * int(c.height) for c in cams)


class _Lease:
    """Marks a pooled forward state busy while an autograd graph holds it;
    releases it when that graph (and so this object) is freed."""

    def __init__(self, st):
        self.st = st
        st.busy = True

    def __del__(self):
        self.st.busy = False


class Renderer:
    """Owns an rgx context and acceleration structure on one device, and a
    pool of forward states for RayMarchFunction."""

    def __init__(self, device: int = 0, sigma_eps: float = 0.01, morton_bits: int = 21):
        self.ctx = lib.Context(device)
        self.bvh = lib.BVH(self.ctx)
        self.sigma_eps = sigma_eps
        self.morton_bits = morton_bits
        self._key = None
        self.serial = 0            # bumped by every build of the structure
        self._pool = []

    def build(self, params: dict, sh_degree: int, force: bool = False):
        """(Re)builds the structure when a parameter tensor changed.  params
        may hold "sg" [n, n_sg, 7] spherical-Gaussian colour lobes."""
        keys = _keys(params)
        key = tuple((params[k].data_ptr(), params[k]._version) for k in keys)
        if force or key != self._key:
            for k in keys:
                t = params[k]
                if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
                    raise ValueError(f"{k} must be a contiguous float32 device tensor")
            self.bvh.build(params["means"], params["log_scales"], params["quats"],
                           params["density"], params["sh"], sh_degree, self.sigma_eps,
                           self.morton_bits, _stream(), sg=params.get("sg"))
            self._key = key
            self.serial += 1
        return self

    def new_state(self) -> lib.ForwardState:
        """A forward state of this renderer's context (caller-owned)."""
        st = lib.ForwardState(self.ctx)
        st.busy = False
        return st

    def acquire_state(self) -> lib.ForwardState:
        for st in self._pool:
            if not st.busy:
                return st
        st = self.new_state()
        self._pool.append(st)
        return st

    def forward(self, cams, opts: RenderOptions, stats: bool = False, state=None):
        """(rgb [R,3], T [R]) and, with stats, the per-ray counters [R, NSTAT].
        With `state` (a ForwardState) the forward records what the matching
        backward needs into it."""
        R = n_rays(cams)
        dev = torch.device("cuda", self.ctx.device)
        rgb = torch.empty((R, 3), device=dev, dtype=torch.float32)
        T = torch.empty((R,), device=dev, dtype=torch.float32)
        st = torch.zeros((R, lib.NSTAT), device=dev, dtype=torch.int32) if stats else None
        lib.render_forward(self.ctx, self.bvh, cams, opts, rgb, T, st, _stream(), state)
        return (rgb, T, st) if stats else (rgb, T)

    def backward(self, state, rgb, T, grad_rgb, grad_T, params: dict, densify=None,
                 densify_views=None):
        """Parameter gradients of the forward recorded in `state`; with
        `densify` / `densify_views` ([n] float32 / int32 device tensors) also
        adds the densification statistic of each view (per-view
        mean-gradient norms weighted by distance / focal)."""
        grads = {k: torch.empty_like(params[k]) for k in _keys(params)}
        lib.render_backward(self.ctx, self.bvh, state, rgb, T, grad_rgb.contiguous(),
                            None if grad_T is None else grad_T.contiguous(), grads, False,
                            _stream(), densify, densify_views)
        return grads

    def false_positives(self, cam, pix, t_end):
        """Whole-ray AABB false-positive counts of one view's listed pixels
        over [t_near, t_end] (int32 device tensor)."""
        dev = torch.device("cuda", self.ctx.device)
        pix = pix.to(device=dev, dtype=torch.int32).contiguous()
        count = torch.empty(pix.shape, device=dev, dtype=torch.int32)
        lib.false_positives(self.ctx, self.bvh, cam, pix, t_end.contiguous(), count, _stream())
        return count

    def check_errors(self):
        """Raises if a kernel of this context set its error flag."""
        f = self.ctx.error_flags(_stream())
        if f:
            raise lib.RgxError(f"device error flag {f}: results of this context are invalid")

    def close(self):
        for st in self._pool:
            st.close()
        self._pool = []
        self.bvh.close()
        self.ctx.close()


class RayMarchFunction(torch.autograd.Function):
    """(means, log_scales, quats, density, sh) -> (rgb [R,3], T [R]).

    The forward (re)builds the acceleration structure when a parameter tensor
    changed (data pointer or version), then renders into a forward state (the
    caller's, or one leased from the renderer's pool for as long as the
    autograd graph lives); the backward replays that state.  If the renderer
    rebuilt its structure since (another parameter set rendered in between),
    the backward rebuilds it from the saved parameters and renders the
    forward again before differentiating: the build is deterministic, so the
    gradients are those of the original forward."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, density, sh, sg, renderer: Renderer, cams,
                opts: RenderOptions, sh_degree: int, state):
        params = dict(means=means, log_scales=log_scales, quats=quats, density=density, sh=sh,
                      sg=sg)
        renderer.build(params, sh_degree)
        if state is None:
            state = renderer.acquire_state()
            ctx.lease = _Lease(state)
        rgb, T = renderer.forward(cams, opts, state=state)
        ctx.renderer, ctx.cams, ctx.opts, ctx.deg = renderer, cams, opts, sh_degree
        ctx.state, ctx.serial = state, renderer.serial
        ctx.state_gen = getattr(state, "gen", 0) + 1
        state.gen = ctx.state_gen
        ctx.save_for_backward(means, log_scales, quats, density, sh, sg, rgb, T)
        return rgb, T

    @staticmethod
    def backward(ctx, grad_rgb, grad_T):
        means, log_scales, quats, density, sh, sg, rgb, T = ctx.saved_tensors
        params = dict(means=means, log_scales=log_scales, quats=quats, density=density, sh=sh,
                      sg=sg)
        r, st = ctx.renderer, ctx.state
        if grad_rgb is None:
            grad_rgb = torch.zeros_like(rgb)
        if r.serial != ctx.serial or getattr(st, "gen", 0) != ctx.state_gen:
            # the structure or the state moved on: rebuild and render again
            r.build(params, ctx.deg, force=True)
            rgb, T = r.forward(ctx.cams, ctx.opts, state=st)
            ctx.serial = r.serial
            st.gen = getattr(st, "gen", 0) + 1
            ctx.state_gen = st.gen
        g = r.backward(st, rgb, T, grad_rgb, grad_T, params)
        return (g["means"], g["log_scales"], g["quats"], g["density"], g["sh"], g.get("sg"), None,
                None, None, None, None)


def render(params: dict, sh_degree: int, renderer: Renderer, cams, opts: RenderOptions,
           state=None):
    """Differentiable render of the views.  Without autograd (no_grad, or no
    parameter requiring gradients) the forward records nothing."""
    if not (torch.is_grad_enabled() and any(params[k].requires_grad for k in _keys(params))):
        renderer.build(params, sh_degree)
        return renderer.forward(cams, opts)
    return RayMarchFunction.apply(params["means"], params["log_scales"], params["quats"],
                                  params["density"], params["sh"], params.get("sg"), renderer,
                                  cams, opts, sh_degree, state)


class Adam:
    """Adam over the five parameter tensors through the library kernel
    (rgx_adam_step).  The step counter and the moments live on the device,
    so the update can be captured into a graph."""

    # learning rates per parameter tensor (the paper defers its training
    # hyperparameters to RayGauss; these follow common Gaussian-splatting
    # practice for the same parameterisation)
    DEFAULT_LR = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, density=5e-2, sh=2.5e-3)

    def __init__(self, renderer: Renderer, params: dict, lr: dict | None = None,
                 betas=(0.9, 0.999), eps: float = 1e-15):
        self.renderer, self.params = renderer, params
        self.lr = dict(self.DEFAULT_LR if lr is None else lr)
        self.betas, self.eps = betas, eps
        self.m = {k: torch.zeros_like(params[k]) for k in PARAM_KEYS}
        self.v = {k: torch.zeros_like(params[k]) for k in PARAM_KEYS}
        self.t = torch.zeros((), dtype=torch.int32, device=params["means"].device)

    @torch.no_grad()
    def step(self):
        groups = [(self.params[k], self.params[k].grad, self.m[k], self.v[k], self.lr[k])
                  for k in PARAM_KEYS if self.params[k].grad is not None]
        lib.adam_step(self.renderer.ctx, groups, self.t, self.betas[0], self.betas[1], self.eps,
                      _stream())


class TrainStep:
    """One training step of the ray marcher as a replayable HIP graph.

    The step rebuilds the acceleration structure from the current parameter
    values, renders every view in one batched launch, evaluates `loss_fn`
    on (rgb, T) (plus iso_weight times the isotropic scale loss when given),
    back-propagates through RayMarchFunction and updates the parameters in
    place: an Adam step when `optimizer` is given, else p -= lr * grad.  It is captured once (after warm-up calls that
    size every buffer, so nothing is allocated inside the graph) and replayed
    with a single launch per step.  All library work is kernels on the
    capturing stream; accumulators and work queues are cleared by kernels,
    never by memset nodes."""

    def __init__(self, renderer: Renderer, params: dict, sh_degree: int, cams,
                 opts: RenderOptions, loss_fn, lr: float = 0.0, warmup: int = 2,
                 optimizer: Adam | None = None, iso_weight: float = 0.0, iso_r0: float = 10.0):
        self.renderer, self.params, self.deg = renderer, params, sh_degree
        self.cams, self.opts, self.loss_fn, self.lr = cams, opts, loss_fn, lr
        self.optimizer, self.iso_weight, self.iso_r0 = optimizer, iso_weight, iso_r0
        self.state = renderer.new_state()      # captured with the step: never shared
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self._step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        renderer.check_errors()     # a device error flag would make the captured step invalid
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.loss, self.rgb, self.T = self._step()
        self.grads = {k: params[k].grad for k in PARAM_KEYS}

    def _step(self):
        for p in self.params.values():
            p.grad = None
        self.renderer.build(self.params, self.deg, force=True)
        rgb, T = render(self.params, self.deg, self.renderer, self.cams, self.opts, self.state)
        loss = self.loss_fn(rgb, T)
        if self.iso_weight:
            loss = loss + self.iso_weight * isotropic_loss(self.params["log_scales"], self.renderer,
                                                           self.iso_r0)
        loss.backward()
        if self.optimizer is not None:
            self.optimizer.step()
        elif self.lr:
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
