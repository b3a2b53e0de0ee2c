"""Pins of the oracle's LinPrim-MCMC population steps (Sec. 3.4
"LinPrim-MCMC", after GS-MCMC).

* N stacked copies with the relocated opacity composite to the original
  opacity (transmittance product).
* The relocated size keeps the line integral of the composited opacity of
  a Gaussian profile (numerical quadrature, independent of the nested
  binomial sum).
* Sampling: exact extreme draws, never a dead primitive, frequencies
  proportional to the opacities.
* A hand-built relocation and the noise step's closed form.
No GPU needed."""
import math

import numpy as np
import pytest

from oracle import mcmc as MC


@pytest.mark.parametrize("alpha,n", [(0.3, 2), (0.9, 3), (0.05, 7), (0.999, 5), (0.6, 51)])
def test_relocated_opacity_composites_to_the_original(alpha, n):
    a_new = 1.0 - (1.0 - alpha) ** (1.0 / n)
    assert abs((1.0 - (1.0 - a_new) ** n) - alpha) < 1e-14


@pytest.mark.parametrize("alpha,n", [(0.3, 2), (0.9, 3), (0.05, 7), (0.7, 12)])
def test_relocated_scale_keeps_the_line_integral(alpha, n):
    a_new = 1.0 - (1.0 - alpha) ** (1.0 / n)
    coeff = MC.relocation_scale(alpha, a_new, n)
    s_old = 1.0
    s_new = coeff * s_old
    x = np.linspace(-40, 40, 400001)
    g_old = np.exp(-0.5 * (x / s_old) ** 2)
    g_new = np.exp(-0.5 * (x / s_new) ** 2)
    lhs = np.trapezoid(1.0 - (1.0 - a_new * g_new) ** n, x)
    rhs = np.trapezoid(alpha * g_old, x)
    assert abs(lhs - rhs) < 1e-9 * rhs, (lhs, rhs, coeff)


def test_sampling_extremes_and_dead():
    op = np.array([0.001, 0.5, 0.004, 0.25, 0.005, 0.75, 0.0], np.float32)
    w = MC.weights(op)
    assert list(np.nonzero(w)[0]) == [1, 3, 5]                 # 0.005 and below are dead
    assert MC.sample(w, [0])[0] == 1                            # first live primitive
    assert MC.sample(w, [2 ** 32 - 1])[0] == 5                  # last live primitive
    total = int(w.sum())
    # a draw just below / at the first boundary
    b = int(w[1])
    r_lo = (b * 2 ** 32) // total - 1                           # t < b
    assert MC.sample(w, [r_lo])[0] == 1
    r_hi = -(-(b * 2 ** 32) // total)                           # ceil: t >= b
    assert MC.sample(w, [r_hi])[0] == 3


def test_sampling_frequencies():
    rng = np.random.default_rng(0)
    op = np.array([0.1, 0.2, 0.3, 0.4], np.float32)
    r = rng.integers(0, 2 ** 32, size=200000, dtype=np.uint64)
    idx = MC.sample(MC.weights(op), r)
    freq = np.bincount(idx, minlength=4) / len(r)
    np.testing.assert_allclose(freq, op / op.sum(), atol=4e-3)


def test_relocation_by_hand():
    op = np.array([0.6, 0.002, 0.3, 0.001, 0.9], np.float32)
    n = len(op)
    params = {"means": np.arange(n * 3, dtype=np.float32).reshape(n, 3),
              "quats": np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)),
              "dists": np.tile(np.array([0.1, 0.2, 0.3], np.float32), (n, 1)),
              "opacity": op, "sh": np.zeros((n, 4, 3), np.float32)}
    moments = {("m", k): np.ones_like(v) for k, v in params.items()}
    w = MC.weights(op)
    total = int(w.sum())
    # two dead (1, 3); draws chosen to land on primitive 4 twice
    r = int(((int(w[0]) + int(w[2])) * 2 ** 32) // total) + 10
    p, m, nd = MC.relocate(params, moments, [r, r])
    assert nd == 2
    # primitive 4 sampled twice -> becomes 3 primitives: itself and slots 1, 3
    a_new = 1.0 - (1.0 - float(op[4])) ** (1.0 / 3)
    assert abs(p["opacity"][4] - a_new) < 1e-15
    coeff = MC.relocation_scale(float(op[4]), a_new, 3)
    np.testing.assert_allclose(p["dists"][4], params["dists"][4].astype(np.float64) * coeff, rtol=1e-15)
    for j in (1, 3):
        for k in params:
            np.testing.assert_array_equal(p[k][j], p[k][4])
    for key in m:
        assert np.all(m[key][[1, 3, 4]] == 0) and np.all(m[key][[0, 2]] == 1)
    np.testing.assert_array_equal(p["opacity"][[0, 2]], op[[0, 2]].astype(np.float64))


def test_noise_closed_form():
    params = {"means": np.zeros((2, 3), np.float32),
              "quats": np.array([[1, 0, 0, 0], [1, 0, 0, 0]], np.float32),
              "dists": np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0]], np.float32),
              "opacity": np.array([0.9, 0.002], np.float32)}
    eps = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, 0.5]])
    mu = MC.noise(params, eps, lr_means=1e-4, noise_lr=5e5)
    assert np.abs(mu[0]).max() < 1e-30                           # opaque: the gate is closed
    gate = 1.0 / (1.0 + math.exp(-100.0 * ((1.0 - float(np.float32(0.002))) - 0.995)))
    ref = 5e5 * 1e-4 * gate * (np.array([1.0, 2.0, 3.0]) / 2.6) ** 2 * eps[1]
    np.testing.assert_allclose(mu[1], ref, rtol=1e-12)


def test_growth_step_appends_updated_sources():
    op = np.array([0.4, 0.001, 0.8], np.float32)
    n = len(op)
    params = {"means": np.arange(n * 3, dtype=np.float32).reshape(n, 3),
              "quats": np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)),
              "dists": np.full((n, 3), 0.2, np.float32), "opacity": op}
    moments = {("m", k): np.ones_like(v) for k, v in params.items()}
    w = MC.weights(op)
    r_last = 2 ** 32 - 1                        # the last live primitive (2)
    p, m = MC.add(params, moments, 2, [r_last, 0])  # draws: primitive 2, then primitive 0
    assert p["means"].shape[0] == 5
    assert list(np.nonzero(w)[0]) == [0, 2]
    for row, s in ((3, 2), (4, 0)):
        for k in params:
            np.testing.assert_array_equal(p[k][row], p[k][s])
    a0 = 1.0 - (1.0 - float(op[0])) ** 0.5       # each source drawn once: one of 2 copies
    assert abs(p["opacity"][0] - a0) < 1e-15 and p["opacity"][1] == float(op[1])
    for key in m:
        assert np.all(m[key][[0, 2, 3, 4]] == 0) and np.all(m[key][1] == 1)
