"""Benchmark of the linear-primitive rasterizer on one GPU.

Default workload: forward + backward megapixels/s on 1,000,000 octahedra at
1920x1080 (one view, plain launches).  One step = the whole hot path over
one synthetic batch: preprocess (primitive build, ray-space projection,
bounds, SH colour, tile counts and their prefix sum), binning and the radix
sort, the forward compositing, the rasterization backward and the
preprocessing backward.  Inputs and the loss gradient dL/dC are resident in
HBM before the timed region.  The line also carries the batched-views
comparison (500,000 octahedra, 16 views of mixed resolution: one
graph-captured multi-view step against 16 per-view plain launches) unless
--no-batched is given, and a short run of the optimisation step loop (20
replays, see below) unless --no-steploop is given.

--workload batched runs only the batched-views comparison.

--workload copy times a plain device copy of known size (the calibration
of the HBM byte counters).

--workload steploop times the optimisation loop instead: 3,000,000
octahedra, per step a batch of 8 random 1920x1080 views (from a pool of
batches whose targets were rendered once from a perturbed copy of the
scene), forward + backward + the L1 loss gradient (--loss l1_ssim: the
paper's L1 + SSIM) + fused Adam captured in one graph and replayed on each
batch's poses.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3        # MI355X FP32 vector peak
PEAK_HBM_GBS = 8000.0
# Algorithmic cost per unit of the compositing kernels (per evaluated /
# intersected pixel-primitive pair), octahedra / tetrahedra.
F_FWD = {0: 108.0, 1: 60.0}
F_BWD_EXTRA = {0: 112.0, 1: 112.0}
ADAM_BYTES_PER_PARAM = 28       # read p, g, m, v; write p, m, v (float32)
STAGES = ("preprocess", "bin_sort", "render_fwd", "raster_bwd", "preprocess_bwd")


def _src_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(workload_key, kernel_key, src_file):
    """HBM bytes per launch measured by rocprofv3 counters for this workload
    and kernel, if the record on file was taken on the current kernel
    source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        rec = json.load(f).get(f"{workload_key}/{kernel_key}")
    if not rec or rec.get("source_sha256_16") != _src_hash(src_file):
        return None
    return rec.get("bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, cams, grad, band_rows, threads):
    """The FP64 oracle (as it stands) on the headline workload, wall time:
    on all host threads the whole frame, forward (preprocess, sort,
    compositing) and forward + backward; on one thread the preprocess and
    sort of every primitive, then a band of rows composited and
    back-propagated, the band's times scaled by the frame's rows (which also
    scales the backward's fixed per-call cost: conservative for the CPU)."""
    import numpy as np

    import oracle
    cam = cams[0]
    hw = cam.width * cam.height
    mp = hw / 1e6
    band_rows = max(1, min(band_rows if band_rows > 0 else 216, cam.height))
    j0 = cam.height // 2 - band_rows // 2
    j1 = j0 + band_rows
    g_band = np.zeros_like(grad, dtype=np.float64)
    for c in range(3):
        g_band[c * hw: (c + 1) * hw].reshape(cam.height, cam.width)[j0:j1] = \
            grad[c * hw: (c + 1) * hw].reshape(cam.height, cam.width)[j0:j1]

    def setup():
        t0 = time.perf_counter()
        O = oracle.OracleScene(scene, cams, tile=16)
        O.sort()
        return O, time.perf_counter() - t0

    # all threads, whole frame
    oracle.set_threads(threads)
    O, t_setup = setup()
    t0 = time.perf_counter()
    O.render()
    t_render = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.backward(grad.astype(np.float64))
    t_bwd = time.perf_counter() - t0
    cores = oracle.num_threads()
    del O
    all_fwd = mp / (t_setup + t_render)
    all_fb = mp / (t_setup + t_render + t_bwd)
    # one thread, a band of rows
    oracle.set_threads(1)
    O, t1_setup = setup()
    t0 = time.perf_counter()
    O.render_band(j0, j1)
    t1_render = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.backward(g_band)
    t1_bwd = time.perf_counter() - t0
    del O
    oracle.set_threads(threads)
    scale = cam.height / band_rows
    one_fwd_t = t1_setup + t1_render * scale
    one_fb_t = one_fwd_t + t1_bwd * scale
    wall = t_setup + t_render + t_bwd + t1_setup + t1_render + t1_bwd
    return {"value": round(all_fb, 4), "unit": "megapixels/s", "cores": cores, "kind": "oracle",
            "timing": "wall time", "cpu_model": _cpu_model(),
            "fwd_megapixels_per_s": {"all_cores": round(all_fwd, 4), "one_core": round(mp / one_fwd_t, 4)},
            "fwd_bwd_megapixels_per_s": {"all_cores": round(all_fb, 4), "one_core": round(mp / one_fb_t, 4)},
            "sample": f"{cores} threads: the whole frame once (all {scene.n} primitives preprocessed and sorted "
                      f"{t_setup:.1f} s, composited {t_render:.1f} s, back-propagated {t_bwd:.1f} s); 1 thread: "
                      f"preprocess and sort {t1_setup:.1f} s, rows {j0}-{j1 - 1} ({band_rows} of {cam.height}) "
                      f"composited {t1_render:.1f} s and back-propagated {t1_bwd:.1f} s, both scaled to the frame; "
                      f"{wall:.1f} s wall"}


class Staged:
    """The five stages of one fwd + bwd step as plain launches, each
    bracketed by events on the stream the library launches on."""

    def __init__(self, rast, prims, bg, grad, grads=None):
        self.rast, self.prims, self.bg, self.grad = rast, prims, bg, grad
        rast.preprocess(prims, sync_count=True)
        self.outs = rast.alloc_outputs()
        self.grads = grads if grads is not None else rast.alloc_grads(prims)

    def run(self, ev=None):
        from paper_2501_16312_amd import linprim as L
        r, p = self.rast, self.prims

        def mark(k):
            if ev is not None:
                ev[k].record()
        mark(0)
        L.linprim_preprocess(p, r.cams_c, r.tune, r.view_ws)
        mark(1)
        r.bin_sort(p)
        mark(2)
        rgb, T, last = r.render(p, self.bg, out=self.outs)
        mark(3)
        L.linprim_raster_bwd(p, r.cams_c, r.tune, self.bg, r.view_ws, r.pair_ws, r.max_pairs, T, last, self.grad)
        mark(4)
        L.linprim_preprocess_bwd(p, r.cams_c, r.tune, r.view_ws, r.pair_ws, r.max_pairs, self.grads)
        mark(5)

    def time_plain(self, steps):
        """Wall time of `steps` steps with no events between the stages."""
        import torch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.run()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def time_stages(self, steps):
        import numpy as np
        import torch
        events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            self.run(events[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stage_ms = {s: float(np.median([events[k][i].elapsed_time(events[k][i + 1]) for k in range(steps)]))
                    for i, s in enumerate(STAGES)}
        return wall, stage_ms

    def counts(self):
        import torch
        cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
        self.rast.render(self.prims, self.bg, out=self.outs, counters=cnt)
        torch.cuda.synchronize()
        return tuple(int(x) for x in cnt.cpu())


def roofline_of(kind, stage_ms, counts, workload_key):
    iterated, evaluated, intersected = counts
    fwd_flop = evaluated * F_FWD[kind]
    bwd_flop = evaluated * F_FWD[kind] + intersected * F_BWD_EXTRA[kind]
    dominant = max(("render_fwd", "raster_bwd"), key=lambda s: stage_ms[s])
    flop = fwd_flop if dominant == "render_fwd" else bwd_flop
    achieved = flop / (stage_ms[dominant] * 1e-3) / 1e12
    src = os.path.join(ROOT, "paper_2501_16312_amd", "csrc", "k_render.hip")
    return {"bound": "alu", "kernel": dominant, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": _traffic(workload_key, dominant, src)}


def batched_comparison(args, log):
    """500k octahedra, 16 views of mixed resolution: one graph-captured
    multi-view step (autotuned launch shape) against the same views as 16
    per-view plain launch sequences whose gradients are summed."""
    import numpy as np
    import torch

    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd import scenes
    from paper_2501_16312_amd.autotune import autotune
    from paper_2501_16312_amd.graph import CapturedStep, split_views
    from paper_2501_16312_amd.render import Rasterizer

    scene, cams = scenes.config3()
    prims = L.Prims.from_scene(scene)
    grad = torch.as_tensor(scenes.image_gradient(cams, seed=2), device="cuda")
    mp = sum(c.width * c.height for c in cams) / 1e6
    tuned = autotune(prims, cams, grad, None)
    tile, digit, radix = tuned["tile"], tuned["sort_digit_bits"], tuned["radix_sort"]
    log(f"batched: autotuned tile {tile}, radix sort {radix}, digit {digit} ({tuned['table']})")

    rast = Rasterizer(scene.kind, scene.n, cams, tile=tile, sort_digit_bits=digit, headroom=1.05, radix_sort=radix)
    cap = CapturedStep(rast, prims, None, grad_rgb=grad, headroom=1.05)
    for _ in range(args.warmup):
        cap.replay()
    torch.cuda.synchronize()
    reps = max(args.batched_steps, 1)
    t0 = time.perf_counter()
    for _ in range(reps):
        cap.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / reps
    cap.check()

    per = []
    for c, g in zip(cams, split_views(grad, cams)):
        r = Rasterizer(scene.kind, scene.n, [c], tile=tile, sort_digit_bits=digit, headroom=1.05, radix_sort=radix)
        per.append(Staged(r, prims, None, g))
    acc = {k: torch.empty_like(v) for k, v in per[0].grads.items()}

    def per_view_step():
        for i, s in enumerate(per):
            s.run()
            for k in acc:
                if i == 0:
                    acc[k].copy_(s.grads[k])
                else:
                    acc[k].add_(s.grads[k])

    for _ in range(args.warmup):
        per_view_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        per_view_step()
    torch.cuda.synchronize()
    per_ms = (time.perf_counter() - t0) * 1e3 / reps
    for s in per:
        if s.rast.status()[1]:
            raise RuntimeError("pair capacity overflow in a per-view step")
    # the two paths must agree (sums over views in a different order)
    rel = max(float((acc[k] - cap.grads[k]).abs().max() / (cap.grads[k].abs().max() + 1e-30)) for k in acc)
    img = float((torch.cat([s.outs[0] for s in per]) - cap.outs[0]).abs().max())
    return {"workload": f"500,000 room-scale octahedra, 16 views on a circle of radius 8, "
                        f"{'/'.join(sorted({f'{c.width}x{c.height}' for c in cams}))}, {mp:.2f} MP per step",
            "megapixels": round(mp, 3), "tile": tile, "radix_sort": radix, "sort_digit_bits": digit,
            "graph_ms": round(graph_ms, 3),
            "per_view_ms": round(per_ms, 3),
            "speedup": round(per_ms / graph_ms, 3), "batched_megapixels_per_s": round(mp / (graph_ms * 1e-3), 1),
            "per_view_megapixels_per_s": round(mp / (per_ms * 1e-3), 1), "max_image_diff": img,
            "max_grad_rel_diff": rel, "autotune_ms": {k: round(v, 3) for k, v in tuned["table"].items()}}


def single(args, log):
    import torch

    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd import scenes
    from paper_2501_16312_amd.render import Rasterizer

    scene, cams = scenes.config2()
    cam = cams[0]
    grad_np = scenes.image_gradient(cams, seed=1)
    prims = L.Prims.from_scene(scene)
    grad = torch.as_tensor(grad_np, device="cuda")

    def measure(exact):
        rast = Rasterizer(scene.kind, scene.n, cams, tile=args.tile, sort_digit_bits=args.digit, headroom=1.05,
                          radix_sort=args.radix_sort, exact=exact)
        st = Staged(rast, prims, (0.0, 0.0, 0.0), grad)
        log(f"{'exact rays: ' if exact else ''}pairs {rast.n_pairs}, capacity {rast.max_pairs}")
        for _ in range(args.warmup):
            st.run()
        # the timed steps carry no instrumentation; a second pass with events
        # around each stage gives the stage times
        wall = st.time_plain(args.steps)
        _, stage_ms = st.time_stages(args.steps)
        n_pairs, overflow = rast.status()
        if overflow:
            raise RuntimeError("pair capacity overflow in the timed region")
        ms = wall * 1e3 / args.steps
        log("stage ms (median): " + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items()))
        counts = st.counts()
        log(f"iterated {counts[0]}, evaluated {counts[1]}, intersected {counts[2]}")
        del st, rast
        torch.cuda.empty_cache()
        return ms, stage_ms, counts, n_pairs

    ms_per_step, stage_ms, counts, n_pairs = measure(args.exact)
    value = cam.width * cam.height / 1e6 / (ms_per_step / 1e3)
    roofline = roofline_of(scene.kind, stage_ms, counts, f"octa1M_1080p_tile{args.tile}") if not args.exact else None

    exact = None
    if not args.exact and not args.no_exact:
        # the variant without the ray-space approximation on the same workload
        e_ms, e_stage, e_counts, e_pairs = measure(True)
        exact = {"megapixels_per_s": round(cam.width * cam.height / 1e6 / (e_ms / 1e3), 3),
                 "ms_per_step": round(e_ms, 4), "pairs": int(e_pairs),
                 "stage_ms": {k: round(v, 4) for k, v in e_stage.items()},
                 "pair_counts": {"iterated": e_counts[0], "evaluated": e_counts[1], "intersected": e_counts[2]},
                 "render_ms_ratio_to_ray_space": round((e_stage["render_fwd"] + e_stage["raster_bwd"]) /
                                                       (stage_ms["render_fwd"] + stage_ms["raster_bwd"]), 3)}
        log(f"exact rays: {exact['megapixels_per_s']} MP/s, render time x{exact['render_ms_ratio_to_ray_space']}")

    batched = None
    if not args.no_batched:
        log("batched views ...")
        batched = batched_comparison(args, log)
        log(f"batched: {batched['graph_ms']} ms vs per-view {batched['per_view_ms']} ms, "
            f"speedup {batched['speedup']}")
        torch.cuda.empty_cache()
    steploop_leg = None
    if not args.no_steploop:
        # the optimisation step loop, short: 20 replays on 2 batches of views
        log("step loop ...")
        import copy
        a2 = copy.copy(args)
        a2.steps, a2.warmup, a2.view_batches = args.steploop_steps, 3, 2
        sl = steploop(a2, log)
        steploop_leg = {"workload": sl["config"]["workload"], "steps": a2.steps, "warmup": a2.warmup,
                        "steps_per_s": sl["value"], "ms_per_step": sl["ms_per_step"],
                        "megapixels_per_s": sl["megapixels_per_s"], "peak_hbm_gb": sl["peak_hbm_gb"],
                        "device_memory_in_use_gb": sl["device_memory_in_use_gb"],
                        "loss": sl["loss"], "pairs_last": sl["config"]["pairs_last"], "params": sl["config"]["params"]}
        log(f"step loop: {sl['value']} steps/s, peak HBM {sl['peak_hbm_gb']} GB")
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        cpu = cpu_baseline(scene, cams, grad_np, args.band_rows, threads=min(os.cpu_count() or 1, 16))
    return {
        "metric": "fwd+bwd megapixels/s at 1M octahedra 1080p" + (", exact rays" if args.exact else ""),
        "value": round(value, 3), "unit": "megapixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1,000,000 octahedra (256-component room-scale mixture, extent 20), one "
                               "1920x1080 view, 60 deg vertical fov, forward + backward", "tile": args.tile,
                   "sort": f"radix{args.digit}" if args.radix_sort else "per-tile", "pairs": int(n_pairs)},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "pair_counts": {"iterated": counts[0], "evaluated": counts[1], "intersected": counts[2]},
        "roofline": roofline,
        "batched": batched,
        "exact_rays": exact,
        "steploop": steploop_leg,
        "cpu_baseline": cpu,
    }


def steploop(args, log):
    """Optimisation loop: fwd + bwd + loss + Adam, one graph replayed per step
    on a new batch of 8 random 1080p views (a pool of batches whose targets
    are rendered once, up front, from a perturbed copy of the scene)."""
    import numpy as np
    import torch

    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd import scenes
    from paper_2501_16312_amd.graph import CapturedStep
    from paper_2501_16312_amd.render import Rasterizer

    torch.cuda.reset_peak_memory_stats()
    scene = scenes.config4()
    pool = [scenes.random_views(b, n_views=8) for b in range(args.view_batches)]
    rng = np.random.default_rng(99)
    pert = scene.copy()
    med_d = float(np.median(scene.dists))
    pert.means = (pert.means + rng.normal(0.0, 0.01 * med_d, size=pert.means.shape)).astype(np.float32)
    pert.sh = (pert.sh + rng.normal(0.0, 0.05, size=pert.sh.shape)).astype(np.float32)
    logit = np.log(pert.opacity) - np.log1p(-pert.opacity)
    pert.opacity = (1.0 / (1.0 + np.exp(-(logit + rng.normal(0.0, 0.2, size=logit.shape))))).astype(np.float32)
    pp = L.Prims.from_scene(pert)
    targets, max_pairs = [], 0
    for cams in pool:
        tr = Rasterizer(scene.kind, scene.n, cams, tile=args.tile, sort_digit_bits=args.digit,
                        radix_sort=args.radix_sort)
        targets.append(tr.forward(pp, None)[0].clone())
        max_pairs = max(max_pairs, tr.n_pairs)
        del tr
    del pp
    torch.cuda.empty_cache()

    prims = L.Prims.from_scene(scene)
    grads = {k: torch.zeros_like(getattr(prims, k)) for k in ("means", "quats", "dists", "opacity", "sh")}
    centres = np.concatenate([np.stack([-(c.world_to_cam[:, :3].T @ c.world_to_cam[:, 3]) for c in cams])
                              for cams in pool]).astype(np.float64)
    extent = float(np.linalg.norm(centres - centres.mean(0), axis=1).max())
    lrs = {"means": 1.6e-4 * extent, "quats": 1e-3, "dists": 1e-4 / 2.6 * extent, "opacity": 2.5e-2,
           "sh": 2.5e-3}
    bounds = {"dists": (1e-5, math.inf), "opacity": (0.0, 1.0)}
    groups = []
    for k, g in grads.items():
        lo, hi = bounds.get(k, (-math.inf, math.inf))
        grp = {"param": getattr(prims, k), "grad": g, "exp_avg": torch.zeros_like(g),
               "exp_avg_sq": torch.zeros_like(g), "lr": lrs[k], "lo": lo, "hi": hi}
        if k == "sh":
            grp.update(period=3 * (scene.sh_degree + 1) ** 2, head=3, lr_tail=1.25e-4)
        groups.append(grp)
    n_params = sum(g.numel() for g in grads.values())
    rast = Rasterizer(scene.kind, scene.n, pool[0], tile=args.tile, sort_digit_bits=args.digit,
                      radix_sort=args.radix_sort,
                      views_resident=True, headroom=1.3)
    rast.reserve_pairs(max_pairs)
    target = targets[0].clone()
    cap = CapturedStep(rast, prims, None, target=target, l1_scale=1.0 / target.numel(),
                       adam={"groups": groups, "beta1": 0.9, "beta2": 0.999, "eps": 1e-15}, headroom=1.3,
                       grads=grads, loss=args.loss)
    log(f"pair capacity {rast.max_pairs} (largest batch {max_pairs}), {n_params} parameters")

    def step(k):
        b = k % len(pool)
        rast.set_views(pool[b])
        target.copy_(targets[b])
        cap.replay()

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    loss0 = cap.loss()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k)
        if (k + 1) % 25 == 0:
            torch.cuda.synchronize()
            log(f"step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_pairs = cap.check()
    loss1 = cap.loss()
    peak = torch.cuda.max_memory_allocated()
    free, total = torch.cuda.mem_get_info()          # hipMemGetInfo: everything on the device

    # one instrumented eager step on the final parameters for the roofline,
    # and the Adam kernel timed alone
    st = Staged(rast, prims, None, cap.grad_rgb, grads=grads)
    st.run()
    _, stage_ms = st.time_stages(3)
    counts = st.counts()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sb = [{**g, "param": g["param"].clone(), "exp_avg": g["exp_avg"].clone(),
           "exp_avg_sq": g["exp_avg_sq"].clone()} for g in groups]
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        L.linprim_adam_step(sb, 0.9, 0.999, 1e-15, 10)
    e1.record()
    e1.synchronize()
    adam_ms = e0.elapsed_time(e1) / 5
    adam_gbs = n_params * ADAM_BYTES_PER_PARAM / (adam_ms * 1e-3) / 1e9
    mp = sum(c.width * c.height for c in pool[0]) / 1e6
    ms = wall * 1e3 / args.steps
    loss_name = "L1 + 0.2 (1 - SSIM) per view" if args.loss == "l1_ssim" else "mean L1"
    loss_ms = None
    if args.loss == "l1_ssim":
        # the fused loss kernels timed alone on the last batch
        e0l, e1l = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0l.record()
        for _ in range(5):
            L.linprim_loss_grad(cap.outs[0], target, rast.cams_c, cap.loss_ws, cap.grad_rgb)
        e1l.record()
        e1l.synchronize()
        loss_ms = round(e0l.elapsed_time(e1l) / 5, 4)
    return {
        "metric": "optimisation steps/s at 3M octahedra, 8 x 1080p views",
        "value": round(1e3 / ms, 3), "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"3,000,000 room-scale octahedra (extent 40); per step a batch of 8 random "
                               f"1920x1080 views from a pool of {len(pool)}, {loss_name} to targets rendered "
                               f"from a perturbed copy; fwd + bwd + loss + fused Adam in one graph",
                   "loss": args.loss,
                   "tile": args.tile, "sort": f"radix{args.digit}" if args.radix_sort else "per-tile",
                   "pairs_last": int(n_pairs),
                   "params": n_params},
        "megapixels_per_s": round(mp / (ms * 1e-3), 1),
        "peak_hbm_gb": round(peak / 1e9, 3),
        "device_memory_in_use_gb": round((total - free) / 1e9, 3),
        "loss": {"before": loss0, "after": loss1, "kernel_ms": loss_ms},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "adam": {"ms": round(adam_ms, 4), "achieved_gbs": round(adam_gbs, 1), "peak_gbs": PEAK_HBM_GBS,
                 "frac": round(adam_gbs / PEAK_HBM_GBS, 4), "bytes_per_param": ADAM_BYTES_PER_PARAM},
        "roofline": roofline_of(scene.kind, stage_ms, counts, "steploop_3M_8views"),
        "cpu_baseline": None,
    }


def batched(args, log):
    """The batched-views comparison on its own (500k octahedra, 16 views)."""
    b = batched_comparison(args, log)
    mp = b["megapixels"]
    return {"metric": "batched vs per-view speedup, 500k octahedra x 16 views", "value": b["speedup"],
            "unit": "x", "n_gpus": 1, "steps": max(args.batched_steps, 1), "warmup": args.warmup,
            "ms_per_step": b["graph_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic", "config": {"workload": b["workload"], "megapixels": mp},
            "batched": b}


def copy_calibration(args, log):
    """A plain device-to-device copy of known size: the reference against
    which the HBM byte counters (FETCH_SIZE, WRITE_SIZE) are scaled."""
    import torch
    nbytes = args.copy_mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    return {"metric": "device copy GB/s (read + write)", "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"copy of {args.copy_mib} MiB", "bytes_read": nbytes, "bytes_written": nbytes}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("single", "batched", "steploop", "copy"), default="single")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--view-batches", type=int, default=4)
    ap.add_argument("--loss", choices=("l1_ssim", "l1"), default="l1",
                    help="step-loop loss: mean L1 (default) or 3DGS's L1 + SSIM")
    ap.add_argument("--tile", type=int, default=8)
    ap.add_argument("--digit", type=int, default=8)
    ap.add_argument("--radix-sort", action="store_true", help="global LSD radix sort instead of the per-tile sort")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--exact", action="store_true", help="time the variant without the ray-space approximation")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact-rays comparison of the default run")
    ap.add_argument("--batched-steps", type=int, default=10)
    ap.add_argument("--no-steploop", action="store_true", help="skip the short step-loop leg of the default run")
    ap.add_argument("--steploop-steps", type=int, default=20)
    ap.add_argument("--band-rows", type=int, default=216, help="rows of the one-thread oracle sample")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus N>1 is not supported (the "
                                   "library has no multi-GPU path)"}), flush=True)
        sys.exit(2)
    if args.steps is None:
        args.steps = 100 if args.workload == "steploop" else 20

    import torch
    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    torch.cuda.set_device(0)
    run = {"single": single, "batched": batched, "steploop": steploop, "copy": copy_calibration}[args.workload]
    out = run(args, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
