"""FP64 CPU oracle of the photometric loss (Sec. 3.4 "Optimization": the
loss of 3DGS, an L1 term and an SSIM term).  TEST INFRASTRUCTURE ONLY: only
the test-suite may import it.  Shares no code with the HIP path.

Readings (the paper defers to 3DGS for the formulation):
  * per view, L_v = (1 - lam) * mean |C - T| + lam * (1 - SSIM(C, T)) with
    lam = 0.2, means over the 3 channels and all pixels; a batch of views
    sums its L_v;
  * SSIM (Wang et al., 2004) per channel: Gaussian window of 11 x 11 taps,
    standard deviation 1.5, normalised to sum 1; local statistics by
    correlation with zero padding at the image border ("same" size);
    C1 = 0.01^2, C2 = 0.03^2 (dynamic range 1);
      s = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
    with s_x^2 = G*(x^2) - mu_x^2, s_xy = G*(x y) - mu_x mu_y; SSIM is the
    mean of s over channels and pixels.
The gradient with respect to C follows the chain through the five local
statistics; the window is symmetric, so the adjoint of each correlation is
the same correlation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import signal

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WINDOW = 11
SIGMA = 1.5
LAMBDA = 0.2


def gaussian_window():
    r = np.arange(WINDOW, dtype=np.float64) - WINDOW // 2
    g = np.exp(-(r * r) / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def _blur(img, w):
    return signal.correlate2d(img, w, mode="same", boundary="fill", fillvalue=0.0)


def ssim_map(x, y):
    """Per-pixel SSIM of two single-channel images (float64)."""
    w = gaussian_window()
    mx, my = _blur(x, w), _blur(y, w)
    sxx = _blur(x * x, w) - mx * mx
    syy = _blur(y * y, w) - my * my
    sxy = _blur(x * y, w) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def ssim_grad(x, y):
    """dS/dx of S = sum of ssim_map(x, y) over the pixels."""
    w = gaussian_window()
    mx, my = _blur(x, w), _blur(y, w)
    exx, eyy, exy = _blur(x * x, w), _blur(y * y, w), _blur(x * y, w)
    a = 2 * mx * my + C1
    b = 2 * (exy - mx * my) + C2
    c = mx * mx + my * my + C1
    d = (exx - mx * mx) + (eyy - my * my) + C2
    s = a * b / (c * d)
    # partial derivatives of s with respect to mu_x, E[x^2], E[x y]
    ds_dmx = 2 * my * (b - a) / (c * d) - 2 * mx * s / c + 2 * mx * s / d
    ds_dexx = -s / d
    ds_dexy = 2 * a / (c * d)
    return _blur(ds_dmx, w) + 2 * x * _blur(ds_dexx, w) + y * _blur(ds_dexy, w)


def loss_and_grad(rgb, target, sizes, lam=LAMBDA):
    """rgb, target: packed view-major images (each view [3,H,W], float);
    sizes: [(W, H), ...].  Returns (L, dL/drgb) in float64."""
    c = np.asarray(rgb, np.float64)
    t = np.asarray(target, np.float64)
    g = np.zeros_like(c)
    total = 0.0
    off = 0
    for (W, H) in sizes:
        n = 3 * W * H
        cv = c[off:off + n].reshape(3, H, W)
        tv = t[off:off + n].reshape(3, H, W)
        diff = cv - tv
        l1 = np.abs(diff).mean()
        ssim = np.mean([ssim_map(cv[k], tv[k]).mean() for k in range(3)])
        total += (1 - lam) * l1 + lam * (1 - ssim)
        gv = (1 - lam) * np.sign(diff) / n
        for k in range(3):
            gv[k] -= lam * ssim_grad(cv[k], tv[k]) / n
        g[off:off + n] = gv.reshape(-1)
        off += n
    return total, g
