"""Shared helpers of the GPU parity tests: run the HIP path through the C
ABI, run the oracle on the same seeded inputs, and compare at the stated
tolerances."""
import numpy as np
import torch

from paper_2501_16312_amd import linprim as L
from paper_2501_16312_amd.render import Rasterizer

IMG_TOL = 1e-5          # absolute, per colour channel and transmittance
GRAD_TOL = 1e-3         # relative, with a floor of 1e-2 x rms of the tensor


def gpu_forward(scene, cams, tile=16, bg=(0.0, 0.0, 0.0), digit=8, counters=False, radix=False, exact=False,
                antialias=False):
    torch.cuda.synchronize()
    prims = L.Prims.from_scene(scene)
    rast = Rasterizer(scene.kind, scene.n, cams, tile=tile, sort_digit_bits=digit, radix_sort=radix, exact=exact,
                      antialias=antialias)
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda") if counters else None
    rgb, T, last = rast.forward(prims, bg, counters=cnt)
    torch.cuda.synchronize()
    out = {"rgb": rgb.cpu().numpy().astype(np.float64), "T": T.cpu().numpy().astype(np.float64),
           "last": last.cpu().numpy().astype(np.int64), "rast": rast, "prims": prims,
           "_T": T, "_last": last, "n_pairs": rast.n_pairs}
    if counters:
        out["counts"] = cnt.cpu().numpy()
    return out


def gpu_backward(fwd, grad_rgb, bg=(0.0, 0.0, 0.0)):
    g = torch.as_tensor(np.ascontiguousarray(grad_rgb, dtype=np.float32), device="cuda")
    grads = fwd["rast"].backward(fwd["prims"], bg, fwd["_T"], fwd["_last"], g)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()}
    K = fwd["prims"].sh.shape[1]
    out["sh"] = out["sh"].reshape(-1, K, 3)
    return out


def compare_images(gpu, ref, label=""):
    """Returns (max error on well-conditioned pixels, max error overall,
    fraction of ill-conditioned pixels)."""
    npx = ref["T"].size
    ill = (ref["ill"] & 1).astype(bool)
    rgb_err = np.abs(gpu["rgb"] - ref["rgb"]).reshape(-1, npx) if False else None
    # rgb is packed view by view as [3,H,W]; per-pixel error = max over channels
    err = np.zeros(npx)
    off_rgb, off_px = 0, 0
    for c in ref.get("cams", []):
        hw = c.width * c.height
        e = np.abs(gpu["rgb"][off_rgb: off_rgb + 3 * hw] - ref["rgb"][off_rgb: off_rgb + 3 * hw]).reshape(3, hw)
        err[off_px: off_px + hw] = e.max(0)
        off_rgb += 3 * hw
        off_px += hw
    errT = np.abs(gpu["T"] - ref["T"])
    good = ~ill
    worst_good = max(err[good].max(initial=0.0), errT[good].max(initial=0.0))
    worst_all = max(err.max(initial=0.0), errT.max(initial=0.0))
    print(f"[{label}] image max err (well-conditioned) {worst_good:.3e}, overall {worst_all:.3e}, "
          f"ill-conditioned {ill.mean() * 100:.4f}% of {npx} px")
    return worst_good, worst_all, ill.mean()


def grad_errors(gpu, ref, mask_ok, label=""):
    """Per-tensor worst relative error on primitives not flagged ill."""
    worst = {}
    for k in ("means", "quats", "dists", "opacity", "sh"):
        a = gpu[k]
        b = ref[k]
        if k == "sh":
            b = b[:, : a.shape[1]]
        a = a.reshape(a.shape[0], -1)[mask_ok]
        b = b.reshape(b.shape[0], -1)[mask_ok]
        if b.size == 0:
            worst[k] = 0.0
            continue
        rms = float(np.sqrt(np.mean(b ** 2))) + 1e-30
        denom = np.maximum(np.abs(b), 1e-2 * rms)
        worst[k] = float((np.abs(a - b) / denom).max())
    print(f"[{label}] gradient worst rel err: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    return worst
