"""FP64 CPU oracle of the optimisation step around the rasterizer (test
infrastructure; only the test-suite, ``__graft_entry__.smoke()`` and
``bench.py``'s cpu_baseline leg use it).

Sec. 3.4 trains with an L1 photometric loss and Adam.  Both are written out
here from their definitions, element by element, in float64:

* L1: L = scale * sum_i |C_i - T_i|, dL/dC_i = scale * sign(C_i - T_i)
  (sign(0) = 0, the subgradient every autograd system picks).
* Adam (Kingma & Ba, Algorithm 1): m = b1 m + (1 - b1) g,
  v = b2 v + (1 - b2) g^2, m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t),
  p = p - lr m_hat / (sqrt(v_hat) + eps); then the projection of p onto
  [lo, hi] that keeps distances positive and opacities inside [0, 1].

Shares no code with the HIP path.
"""
from __future__ import annotations

import numpy as np


def l1_grad(rgb, target, scale: float):
    """Returns (dL/dC as float64 array, L)."""
    c = np.asarray(rgb, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    d = c - t
    return scale * np.sign(d), float(scale * np.abs(d).sum())


def adam_step(param, grad, exp_avg, exp_avg_sq, step: int, lr: float, beta1: float, beta2: float, eps: float,
              lo: float = -np.inf, hi: float = np.inf):
    """One Adam update at step t = `step` (>= 1); `lr` is a scalar or one rate
    per element.  Returns new (param, exp_avg, exp_avg_sq) as float64 arrays;
    inputs are not modified."""
    p = np.array(param, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(exp_avg, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(exp_avg_sq, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    p = p - lr * m_hat / (np.sqrt(v_hat) + eps)
    p = np.minimum(np.maximum(p, lo), hi)
    return p, m, v
