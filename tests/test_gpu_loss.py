"""The fused L1 + SSIM loss gradient (Sec. 3.4 "Optimization") vs the FP64
oracle, through the C ABI (MI355X only): gradients within 1e-3 relative
(floor 1e-2 x rms), loss value within 1e-5 relative."""
import sys

import numpy as np
import pytest
import torch

from oracle import loss as LOSS
from paper_2501_16312_amd import linprim as L
from paper_2501_16312_amd import scenes
from tests import gpu_common as GC

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cams(sizes):
    return [scenes.make_camera(np.eye(3, 4, dtype=np.float32), w, h) for w, h in sizes]


def _run(rgb, target, sizes, lam=0.2):
    cams_c = L.cameras(_cams(sizes))
    ws = torch.empty(L.linprim_loss_workspace_size(cams_c), dtype=torch.uint8, device="cuda")
    x = torch.as_tensor(rgb.astype(np.float32), device="cuda")
    y = torch.as_tensor(target.astype(np.float32), device="cuda")
    g = torch.empty_like(x)
    L.linprim_loss_grad(x, y, cams_c, ws, g, lam)
    val = L.linprim_loss_value(ws, cams_c, lam)
    return val, g.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("sizes", [[(96, 70)], [(33, 17), (64, 64), (7, 5)]])
def test_loss_parity(sizes):
    _say(f"loss sizes={sizes}")
    rng = np.random.default_rng(len(sizes))
    n = sum(3 * w * h for w, h in sizes)
    # smooth-ish images plus noise: a render and a perturbed target
    rgb = np.clip(rng.uniform(0.2, 0.8, size=n) + 0.05 * rng.normal(size=n), 0, 1)
    target = np.clip(rgb + 0.1 * rng.normal(size=n), 0, 1)
    val, g = _run(rgb, target, sizes)
    ref_val, ref_g = LOSS.loss_and_grad(rgb.astype(np.float32), target.astype(np.float32), sizes)
    _say(f"  loss gpu {val:.9f} oracle {ref_val:.9f}")
    assert abs(val - ref_val) <= 1e-5 * abs(ref_val)
    rms = float(np.sqrt(np.mean(ref_g ** 2)))
    err = np.abs(g - ref_g) / np.maximum(np.abs(ref_g), 1e-2 * rms)
    _say(f"  gradient worst rel err {err.max():.2e}")
    assert err.max() <= GC.GRAD_TOL


def test_ssim_only_and_identical_images():
    _say("loss ssim-only / identical")
    sizes = [(50, 40)]
    rng = np.random.default_rng(9)
    n = 3 * 50 * 40
    rgb = rng.uniform(size=n)
    target = np.clip(rgb + 0.2 * rng.normal(size=n), 0, 1)
    val, g = _run(rgb, target, sizes, lam=1.0)
    ref_val, ref_g = LOSS.loss_and_grad(rgb.astype(np.float32), target.astype(np.float32), sizes, lam=1.0)
    assert abs(val - ref_val) <= 1e-5 * abs(ref_val)
    rms = float(np.sqrt(np.mean(ref_g ** 2)))
    assert (np.abs(g - ref_g) / np.maximum(np.abs(ref_g), 1e-2 * rms)).max() <= GC.GRAD_TOL
    val, g = _run(rgb, rgb, sizes)
    assert abs(val) < 1e-6 and np.abs(g).max() < 1e-9
