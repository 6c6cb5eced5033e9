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
    ap.add_argument("--no-side", action="store_true",
                    help="skip the bounded side measurements of the other workloads")
    ap.add_argument("--side-reps", type=int, default=3)
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
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1"}))
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
    log(f"timed {args.steps} steps: {t_total:.3f}s, loss {float(loss.detach()):.5f}")
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
    valu = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("source_hash") == source_hash() and dom in t.get("by_role", {}):
            role = t["by_role"][dom]
            traffic = role["bytes_per_launch"]
            if "valu_insts_per_launch" in role:
                # VALU issue against the chip's: 1024 SIMDs, one wave64 VALU
                # instruction per 4 cycles each, at the 2.4 GHz peak clock;
                # the counter run's busy cycles give the clock the kernel
                # actually ran at
                ins = role["valu_insts_per_launch"]
                peak = 1024 * 2.4e9 / 4
                valu = {"bound": "alu", "kernel": dom, "unit": "wave64 VALU instructions/s",
                        "achieved": ins / (kern_ms[dom] * 1e-3), "peak": peak,
                        "frac": ins / (kern_ms[dom] * 1e-3) / peak,
                        "clock_ghz": role["busy_cycles_per_launch"] / (kern_ms[dom] * 1e-3) / 1e9,
                        "source": "rocprofv3 SQ_INSTS_VALU, SQ_BUSY_CYCLES (profiles/)"}
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
        "roofline_alu": valu,
        # both march kernels against the same roofline (the object above is
        # the dominant one's)
        "roofline_by_kernel": {
            k: {"ms": kern_ms[k], "algorithmic_bytes": b, "achieved": b / (kern_ms[k] * 1e-3) / 1e9,
                "frac": b / (kern_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
            for k, b in (("forward", fwd_bytes), ("backward", bwd_bytes)) if kern_ms.get(k)},
    }
    if not args.no_side:
        # free the headline workload's buffers before the larger scenes
        del params, target
        renderer.close()
        torch.cuda.empty_cache()
        out["side"] = side_measurements(args.side_reps)
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


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return 1000.0 * (time.perf_counter() - t0) / reps


def side_measurements(reps):
    """Bounded measurements of the other workloads (each a few repetitions,
    inputs resident in device memory before timing):
    - 100k Gaussians, 800x800: forward Mrays/s with tiles in Morton order
      against scanline ray order (Sec. 3.3 ray coherence);
    - 3M Gaussians, outdoor layout, 4 views 1297x840: forward and
      forward+backward Mrays/s;
    - 1M Gaussians, 4 views 1024x768: the training workload with Adam and
      the isotropic scale loss (weight 2.5e-4, r0 10, Sec. 4.2), rebuild every
      step, graph-captured: steps/s;
    - 5M Gaussians, 16 views of mixed size: the graph-captured training step
      over one persistent launch (autotuned knobs), against the plain forward
      of the 16 views launched one by one; and one GPU's share of that step
      with the views sharded over 8 GPUs (2 views, forward + backward on the
      whole scene) with the size of the gradient buffer to be summed."""
    import torch
    from paper_2509_07782_amd import autotune, inputs
    from paper_2509_07782_amd.render import Adam, RenderOptions, Renderer, TrainStep
    keys = ("means", "log_scales", "quats", "density", "sh")
    out = {}
    adaptive = dict(adaptive=True, dt_min=0.005, dt_max=0.02, beta=1024.0, n_s=8, t_eps=1e-4, ess=1)

    # ray order on the 100k scene
    t0 = time.time()
    sc = inputs.config_scene(2)
    cams = inputs.config_cameras(2)
    r = Renderer(0)
    r.build({k: torch.from_numpy(sc[k]).cuda() for k in keys}, sc["sh_degree"])
    R = sum(c.width * c.height for c in cams)
    res = {}
    for name, order in (("morton_tiles", 1), ("scanline", 0)):
        o = RenderOptions(**adaptive, ray_order=order, persistent=True)
        res[name] = R / (_timed(lambda: r.forward(cams, o), reps) * 1e-3) / 1e6
    out["config2_fwd_mrays_s"] = res
    r.check_errors()
    r.close()
    log(f"side: ray order done ({time.time() - t0:.1f}s)")

    # outdoor layout, forward and forward + backward
    t0 = time.time()
    sc = inputs.config_scene(4)
    cams = inputs.config_cameras(4)
    r = Renderer(0)
    params = {k: torch.from_numpy(sc[k]).cuda() for k in keys}
    r.build(params, sc["sh_degree"])
    R = sum(c.width * c.height for c in cams)
    o = RenderOptions(**adaptive, persistent=True)
    st = r.new_state()
    gC = torch.full((R, 3), 1e-3, device="cuda")
    ms_f = _timed(lambda: r.forward(cams, o), reps)

    def fwd_bwd():
        rgb, T = r.forward(cams, o, state=st)
        r.backward(st, rgb, T, gC, None, params)
    ms_fb = _timed(fwd_bwd, reps)
    _, _, stats = r.forward(cams, o, stats=True, state=st)
    tot = st.totals()
    out["config4"] = {"fwd_mrays_s": R / (ms_f * 1e-3) / 1e6,
                      "fwd_bwd_mrays_s": R / (ms_fb * 1e-3) / 1e6,
                      "ms_fwd": ms_f, "ms_fwd_bwd": ms_fb,
                      "per_ray": {k: tot[k] / tot["rays"] for k in ("Q", "P", "samples", "segments",
                                                                   "closest", "box_only")},
                      "chunked_segments": tot["chunked"]}
    r.check_errors()
    st.close()
    r.close()
    del params, gC
    torch.cuda.empty_cache()
    log(f"side: outdoor done ({time.time() - t0:.1f}s)")

    # training workload with Adam, per-step rebuild, isotropic loss
    t0 = time.time()
    sc = inputs.config_scene(3)
    cams = inputs.config_cameras(3)
    R = sum(c.width * c.height for c in cams)
    target = torch.from_numpy(inputs.target_image(3, R)).cuda()
    r = Renderer(0)
    p = {k: torch.from_numpy(sc[k]).cuda().requires_grad_(True) for k in keys}
    step = TrainStep(r, p, sc["sh_degree"], cams, RenderOptions(**adaptive, persistent=True),
                     lambda c, t: ((c - target) ** 2).mean(), optimizer=Adam(r, p),
                     iso_weight=2.5e-4, iso_r0=10.0)
    ms_t = _timed(step.replay, max(reps, 3))
    out["train_adam"] = {"steps_per_s": 1000.0 / ms_t, "ms_per_step": ms_t,
                         "mrays_s": R / (ms_t * 1e-3) / 1e6,
                         "workload": "1M Gaussians, 4 views 1024x768, rebuild + forward + L2 + "
                                     "2.5e-4 isotropic loss + backward + Adam, graph-captured"}
    r.check_errors()
    del step, p, target
    r.close()
    torch.cuda.empty_cache()
    log(f"side: training done ({time.time() - t0:.1f}s)")

    # batched persistent graph step against plain launches, 5M / 16 views
    t0 = time.time()
    sc = inputs.config_scene(5)
    cams = inputs.config_cameras(5)
    R = sum(c.width * c.height for c in cams)
    target = torch.from_numpy(inputs.target_image(5, R)).cuda()
    r = Renderer(0)
    p = {k: torch.from_numpy(sc[k]).cuda().requires_grad_(True) for k in keys}
    r.build({k: v.detach() for k, v in p.items()}, sc["sh_degree"])
    base = RenderOptions(**adaptive, persistent=True)
    # knobs tuned for the persistent launch on a quarter of the views (the
    # candidates' images are checked bit for bit against the reference)
    import tempfile
    tuned, table = autotune.tune(r, cams[:4], base, reps=1, persistent=True,
                                 cache_path=os.path.join(tempfile.gettempdir(), "rgx_autotune.json"))
    plain = RenderOptions(**adaptive, persistent=False)
    ms_plain = _timed(lambda: [r.forward([c], plain) for c in cams], reps)
    ms_base_fwd = _timed(lambda: r.forward(cams, base), reps)
    ms_tuned_fwd = _timed(lambda: r.forward(cams, tuned), reps)
    step = TrainStep(r, p, sc["sh_degree"], cams, tuned, lambda c, t: ((c - target) ** 2).mean(),
                     lr=0.0)
    ms_graph = _timed(step.replay, reps)
    r.check_errors()
    # one GPU's share of the step when the 16 views are sharded over 8 GPUs
    # (2 views, the full 5M scene and structure): forward + backward; the
    # gradient buffer is what the one collective of that layout would sum
    share = cams[:2]
    Rs = sum(c.width * c.height for c in share)
    pd = {k: v.detach() for k, v in p.items()}
    gC = torch.full((Rs, 3), 1e-3, device="cuda")
    st = r.new_state()

    def share_step():
        rgb, T = r.forward(share, tuned, state=st)
        r.backward(st, rgb, T, gC, None, pd)

    ms_share = _timed(share_step, reps)
    st.close()
    r.check_errors()
    n5 = int(sc["means"].shape[0])
    out["workload5_share_of_8"] = {
        "views": len(share), "rays": Rs, "ms_fwd_bwd": ms_share,
        "fwd_bwd_mrays_s": Rs / (ms_share * 1e-3) / 1e6,
        "gradient_buffer_bytes": n5 * 4 * (3 + 3 + 4 + 1 + 3 * (sc["sh_degree"] + 1) ** 2)}
    out["workload5"] = {"rays": R,
                        "graph_fwd_bwd_step_mrays_s": R / (ms_graph * 1e-3) / 1e6,
                        "batched_fwd_mrays_s": R / (ms_tuned_fwd * 1e-3) / 1e6,
                        "batched_fwd_fixed_knobs_mrays_s": R / (ms_base_fwd * 1e-3) / 1e6,
                        "plain_fwd_16_launches_mrays_s": R / (ms_plain * 1e-3) / 1e6,
                        "autotuned_knobs": {k: getattr(tuned, k) for k in
                                            ("tile_w", "tile_h", "persistent", "window_segments")}}
    r.check_errors()
    del step, p, target
    r.close()
    torch.cuda.empty_cache()
    log(f"side: workload 5 done ({time.time() - t0:.1f}s)")
    return out


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
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": nr / dt / 1e6, "unit": "Mrays/s", "cores": oracle.num_threads(),
            "host_cpu": model, "host_cpus_online": os.cpu_count(),
            "kind": "oracle", "seconds": dt,
            "sample": f"every {stride}th pixel on both axes of the 4 views ({nr} rays), "
                      "forward + adjoint"}


if __name__ == "__main__":
    main()
