"""Benchmark: forward + backward megapixels/s of the linear-primitive
rasterizer on 1,000,000 octahedra at 1920x1080 (one view).

One step = the whole hot path over one synthetic batch: preprocess
(primitive build, ray-space projection, bounds, SH colour, tile counts and
their prefix sum), binning and the radix sort, the forward compositing, the
rasterization backward and the preprocessing backward.  Inputs and the
loss gradient dL/dC are resident in HBM before the timed region.

Prints one JSON line (see the design doc for the roofline and baseline recipe).
"""
import argparse
import hashlib
import json
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


def _src_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(kernel_key, src_file):
    """HBM bytes per launch measured by rocprofv3 counters, if the summary
    on record was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        rec = json.load(f).get(kernel_key)
    if not rec or rec.get("source_sha256_16") != _src_hash(src_file):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(scene, cams, grad, band_rows, threads):
    """FP64 oracle on a bounded sample: every primitive preprocessed and
    sorted, then a band of image rows composited and back-propagated;
    extrapolated to the whole frame."""
    import numpy as np

    import oracle
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    cam = cams[0]
    t0 = time.perf_counter()
    O = oracle.OracleScene(scene, cams, tile=16)
    O.sort()
    t_setup = time.perf_counter() - t0
    j0 = cam.height // 2 - band_rows // 2
    j1 = j0 + band_rows
    t1 = time.perf_counter()
    O.render_band(j0, j1)
    g = np.zeros_like(grad, dtype=np.float64)
    hw = cam.width * cam.height
    for c in range(3):
        sl = grad[c * hw: (c + 1) * hw].reshape(cam.height, cam.width)
        g[c * hw: (c + 1) * hw].reshape(cam.height, cam.width)[j0:j1] = sl[j0:j1]
    O.backward(g)
    t_band = time.perf_counter() - t1
    frac = band_rows / cam.height
    t_full = t_setup + t_band / frac
    mp = cam.width * cam.height / 1e6
    return {"value": mp / t_full, "unit": "megapixels/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"all {scene.n} primitives preprocessed and sorted ({t_setup:.1f} s), rows {j0}-{j1 - 1} "
                      f"({band_rows} of {cam.height}) composited and back-propagated ({t_band:.1f} s); "
                      f"frame time extrapolated by row fraction"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tile", type=int, default=8)
    ap.add_argument("--digit", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--band-rows", type=int, default=24)
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus N>1 is not supported (the multi-GPU "
                                   "design is described in DESIGN.md)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd import scenes
    from paper_2501_16312_amd.render import Rasterizer

    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    torch.cuda.set_device(0)
    scene, cams = scenes.config2()
    cam = cams[0]
    grad_np = scenes.image_gradient(cams, seed=1)
    prims = L.Prims.from_scene(scene)
    grad = torch.as_tensor(grad_np, device="cuda")
    bg = (0.0, 0.0, 0.0)
    rast = Rasterizer(scene.kind, scene.n, cams, tile=args.tile, sort_digit_bits=args.digit, headroom=1.05)
    rast.preprocess(prims, sync_count=True)
    outs = rast.alloc_outputs()
    grads = rast.alloc_grads(prims)
    log(f"pairs {rast.n_pairs}, capacity {rast.max_pairs}")

    stages = ("preprocess", "bin_sort", "render_fwd", "raster_bwd", "preprocess_bwd")

    def step(ev=None):
        def mark(k):
            if ev is not None:
                ev[k].record()
        mark(0)
        L.linprim_preprocess(prims, rast.cams_c, rast.tune, rast.view_ws)
        mark(1)
        rast.bin_sort(prims)
        mark(2)
        rgb, T, last = rast.render(prims, bg, out=outs)
        mark(3)
        L.linprim_raster_bwd(prims, rast.cams_c, rast.tune, bg, rast.view_ws, rast.pair_ws, rast.max_pairs, T, last,
                             grad)
        mark(4)
        L.linprim_preprocess_bwd(prims, rast.cams_c, rast.tune, rast.view_ws, rast.pair_ws, rast.max_pairs, grads)
        mark(5)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_pairs, overflow = rast.status()
    if overflow:
        raise RuntimeError("pair capacity overflow in the timed region")
    stage_ms = {s: float(np.median([events[k][i].elapsed_time(events[k][i + 1]) for k in range(args.steps)]))
                for i, s in enumerate(stages)}
    ms_per_step = wall * 1e3 / args.steps
    mp = cam.width * cam.height / 1e6
    value = mp / (ms_per_step / 1e3)
    log("stage ms (median): " + ", ".join(f"{k} {v:.3f}" for k, v in stage_ms.items()))

    # pair counts of the compositing kernels (GPU counters; the oracle's
    # counts for this workload are recorded in profiles/ when available)
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
    rast.render(prims, bg, out=outs, counters=cnt)
    torch.cuda.synchronize()
    iterated, evaluated, intersected = (int(x) for x in cnt.cpu())
    log(f"iterated {iterated}, evaluated {evaluated}, intersected {intersected}")
    kind = scene.kind
    fwd_flop = evaluated * F_FWD[kind]
    bwd_flop = evaluated * F_FWD[kind] + intersected * F_BWD_EXTRA[kind]
    dominant = max(("render_fwd", "raster_bwd"), key=lambda s: stage_ms[s])
    flop = fwd_flop if dominant == "render_fwd" else bwd_flop
    achieved = flop / (stage_ms[dominant] * 1e-3) / 1e12
    src = os.path.join(ROOT, "paper_2501_16312_amd", "csrc", "k_render.hip")
    roofline = {"bound": "alu", "kernel": dominant, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": _traffic(dominant, src)}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        cpu = cpu_baseline(scene, cams, grad_np, args.band_rows, threads=os.cpu_count() or 1)
    out = {
        "metric": "fwd+bwd megapixels/s at 1M octahedra 1080p",
        "value": round(value, 3), "unit": "megapixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1,000,000 octahedra (256-component room-scale mixture, extent 20), one "
                               "1920x1080 view, 60 deg vertical fov, forward + backward", "tile": args.tile,
                   "sort_digit_bits": args.digit, "pairs": int(n_pairs)},
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "pair_counts": {"iterated": iterated, "evaluated": evaluated, "intersected": intersected},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
