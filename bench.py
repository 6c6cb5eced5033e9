"""Benchmark of the Gaussian ray-marching hot path on one MI355X.

One step = one training step of the 1M-Gaussian scene over 4 views at
1024x768: acceleration-structure rebuild (preprocess, Morton keys, radix sort,
Z-order pack, LBVH), forward ray marching with empty-space skipping and
adaptive sampling, L2 loss against a random target, backward (gradients of
means, log-scales, quaternions, densities and SH degree 3), and a plain SGD
update of the parameters.  Inputs are seeded synthetic arrays already resident
in device memory when timing starts.

Prints one JSON line: value = whole-step rays per second (Mrays/s), with the
forward-only rate, the time of a 1920x1080 forward frame, the dominant
kernel's achieved algorithmic bandwidth against the HBM peak, and the FP64 CPU
oracle timed on a bounded pixel sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
RECORD_BYTES = {0: 4 * (11 + 3), 1: 4 * (11 + 12), 2: 4 * (11 + 27), 3: 4 * (11 + 48)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000, help="Gaussians (workload: 1M)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=17)
    ap.add_argument("--persistent", type=int, default=1)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device copy of this size first (HBM counter calibration)")
    ap.add_argument("--tile", default="8x8")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--workload", type=int, default=3,
                    help="3: 1M-Gaussian training step (default); 5: 5M Gaussians, 16 mixed "
                         "views, persistent + graph-captured step vs 16 plain launches")
    return ap.parse_args()


def source_hash():
    """Hash of the library sources: HBM counter figures stored under
    profiles/ are used only while it matches."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2509_07782_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU (the HIP library is the only compute path)")
    from paper_2509_07782_amd import inputs, lib
    from paper_2509_07782_amd.render import RenderOptions, Renderer, render

    lib.load()
    if args.workload == 5:
        return batched_workload(args)
    if args.copy_probe_mb:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale between counter units and bytes moved
        nbytes = args.copy_probe_mb << 20
        src = torch.ones(nbytes // 4, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes read and written")
        del src, dst
    t0 = time.time()
    scene = inputs.config_scene(3, n=args.n)
    cams = inputs.config_cameras(3)
    R = sum(c.width * c.height for c in cams)
    log(f"scene {args.n} Gaussians, {len(cams)} views, {R} rays ({time.time() - t0:.1f}s to draw)")
    tw, th = (int(v) for v in args.tile.split("x"))
    opts = RenderOptions(adaptive=True, dt_min=0.005, dt_max=0.02, beta=1024.0, n_s=8,
                         t_eps=1e-4, ess=1, ray_order=1, tile_w=tw, tile_h=th,
                         persistent=bool(args.persistent))
    keys = ("means", "log_scales", "quats", "density", "sh")
    params = {k: torch.from_numpy(scene[k]).cuda().requires_grad_(True) for k in keys}
    target = torch.from_numpy(inputs.target_image(3, R)).cuda()
    renderer = Renderer(0)
    deg = scene["sh_degree"]
    lr = 1e-5
    def step():
        for p in params.values():
            p.grad = None
        renderer._key = None                      # parameters changed: rebuild
        rgb, T = render(params, deg, renderer, cams, opts)
        loss = ((rgb - target) ** 2).mean()
        loss.backward()
        with torch.no_grad():
            for p in params.values():
                p.add_(p.grad, alpha=-lr)
        return loss

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    # the library brackets each of its launches with HIP events on the stream
    # it launches on (torch's current stream here)
    renderer.ctx.set_kernel_timing(True)
    t_start = time.perf_counter()
    for i in range(args.steps):
        loss = step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    log(f"timed {args.steps} steps: {t_total:.3f}s, loss {float(loss):.5f}")
    ms_step = 1000.0 * t_total / args.steps
    kt = renderer.ctx.kernel_times()
    renderer.ctx.set_kernel_timing(False)
    kern_ms = {k: ms / n for k, (ms, n) in kt.items() if n}
    kern_launches = {k: n for k, (ms, n) in kt.items() if n}
    if renderer.ctx.error_flags() != 0:
        raise SystemExit("device error flag set during the benchmark")

    # forward-only rate and the 1920x1080 frame (structure already built)
    with torch.no_grad():
        renderer.build({k: v.detach() for k, v in params.items()}, deg, force=True)
        for _ in range(2):
            renderer.forward(cams, opts)
        torch.cuda.synchronize()
        nrep = max(3, args.steps)
        t1 = time.perf_counter()
        for _ in range(nrep):
            renderer.forward(cams, opts)
        torch.cuda.synchronize()
        fwd_ms = 1000.0 * (time.perf_counter() - t1) / nrep
        hd = [inputs.hd_camera()]
        renderer.forward(hd, opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(nrep):
            renderer.forward(hd, opts)
        torch.cuda.synchronize()
        hd_ms = 1000.0 * (time.perf_counter() - t1) / nrep
        # algorithmic traffic: distinct (ray, Gaussian) pairs Q from the stats pass
        rgb, T, st = renderer.forward(cams, opts, stats=True)
        torch.cuda.synchronize()
        st = st.cpu().numpy().astype(np.int64)
        Q = int(st[:, 0].sum())
        P = int(st[:, 1].sum())
        samples = int(st[:, 2].sum())
        box_only = int(st[:, 5].sum())
    g_touched = int((params["density"].grad != 0).sum().item()) if params["density"].grad is not None else 0
    rec = RECORD_BYTES[deg]
    fwd_bytes = Q * rec + R * 16
    bwd_bytes = Q * rec + R * 32 + g_touched * rec
    dom = "backward" if kern_ms.get("backward", 0) >= kern_ms.get("forward", 0) else "forward"
    dom_bytes = bwd_bytes if dom == "backward" else fwd_bytes
    achieved = dom_bytes / (kern_ms[dom] * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("source_hash") == source_hash() and dom in t.get("by_role", {}):
            traffic = t["by_role"][dom]["bytes_per_launch"]
    out = {
        "metric": "Mrays/s fwd and fwd+bwd at 1M Gaussians; ms per 1920x1080 frame",
        "value": R / (ms_step * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.n} Gaussians (32-cluster mixture, SH degree 3), 4 views "
                               "1024x768, training step: BVH rebuild + forward + L2 loss + "
                               "backward + SGD",
                   "gaussians": args.n, "views": len(cams), "width": 1024, "height": 768,
                   "sampling": "adaptive (dt_min 0.005, dt_max 0.02, beta 1024, N_s 8), "
                               "closest-hit skipping, T_eps 1e-4",
                   "tile": args.tile, "persistent": bool(args.persistent)},
        "fwd_mrays_s": R / (fwd_ms * 1e-3) / 1e6,
        "ms_forward_4views": fwd_ms,
        "ms_per_1920x1080_frame": hd_ms,
        "kernel_ms": kern_ms,
        "kernel_launches_timed": kern_launches,
        "per_ray": {"Q": Q / R, "P": P / R, "samples": samples / R, "box_only": box_only / R},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": dom_bytes},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, cams, opts, args.cpu_stride)
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as fh:
            fh.write(line + "\n")


def batched_workload(args):
    """5M Gaussians (outdoor layout), 16 views of mixed size: one persistent
    launch over all views inside a graph-captured training step, against the
    plain forward of the same views launched one by one."""
    import torch
    from paper_2509_07782_amd import inputs
    from paper_2509_07782_amd.render import RenderOptions, Renderer, TrainStep
    scene = inputs.config_scene(5)
    cams = inputs.config_cameras(5)
    R = sum(c.width * c.height for c in cams)
    keys = ("means", "log_scales", "quats", "density", "sh")
    params = {k: torch.from_numpy(scene[k]).cuda().requires_grad_(True) for k in keys}
    target = torch.from_numpy(inputs.target_image(5, R)).cuda()
    r = Renderer(0)
    batched = RenderOptions(adaptive=True, t_eps=1e-4, ess=1, persistent=True)
    plain = RenderOptions(adaptive=True, t_eps=1e-4, ess=1, persistent=False)
    step = TrainStep(r, params, scene["sh_degree"], cams, batched,
                     lambda c, t: ((c - target) ** 2).mean(), lr=1e-5)
    for _ in range(args.warmup):
        step.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step.replay()
    torch.cuda.synchronize()
    ms_graph = 1000 * (time.perf_counter() - t0) / args.steps
    with torch.no_grad():
        r.build({k: v.detach() for k, v in params.items()}, scene["sh_degree"], force=True)
        a = r.forward(cams, batched)
        outs = [r.forward([c], plain) for c in cams]
        identical = bool(torch.equal(a[0], torch.cat([o[0] for o in outs])))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for c in cams:
                r.forward([c], plain)
        torch.cuda.synchronize()
        ms_plain = 1000 * (time.perf_counter() - t0) / args.steps
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r.forward(cams, batched)
        torch.cuda.synchronize()
        ms_batched_fwd = 1000 * (time.perf_counter() - t0) / args.steps
    out = {"metric": "Mrays/s batched fwd+bwd (graph) vs plain forward, 5M Gaussians, 16 views",
           "value": R / (ms_graph * 1e-3) / 1e6, "unit": "Mrays/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_graph,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "5M Gaussians (outdoor layout), 16 views 256..1920 x 256..1080, "
                                  "graph-captured training step (build + forward + L2 + backward + SGD)",
                      "rays": R},
           "plain_forward_16_launches_mrays_s": R / (ms_plain * 1e-3) / 1e6,
           "batched_forward_mrays_s": R / (ms_batched_fwd * 1e-3) / 1e6,
           "batched_equals_plain_bitwise": identical}
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as fh:
            fh.write(line + "\n")


def cpu_baseline(scene, cams, opts, stride):
    """The FP64 oracle (forward and adjoint of the L2 loss) on every
    stride-th pixel of every view, in the same rays-per-second unit."""
    import oracle
    o = oracle.Opts(adaptive=opts.adaptive, dt=opts.dt, dt_min=opts.dt_min, dt_max=opts.dt_max,
                    beta=opts.beta, n_s=opts.n_s, t_eps=opts.t_eps, ess=opts.ess,
                    bg=tuple(opts.bg), sigma_eps=0.01)
    from paper_2509_07782_amd import inputs
    nr = 0
    t0 = time.perf_counter()
    for cam in cams:
        pix = inputs.pixel_subset(cam, stride)
        rgb, T, _, _ = oracle.render(scene, cam, o, pix)
        gC = np.ones_like(rgb) * 1e-3
        oracle.backward(scene, cam, o, pix, gC, None)
        nr += len(pix)
    dt = time.perf_counter() - t0
    return {"value": nr / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": dt,
            "sample": f"every {stride}th pixel on both axes of the 4 views ({nr} rays), "
                      "forward + adjoint"}


if __name__ == "__main__":
    main()
