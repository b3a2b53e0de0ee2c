"""Pins of the oracle's analytic backward pass (Sec. 3.4, App. E).

Three independent references: central differences of the oracle's own
forward in double precision, autograd of an independent PyTorch float64
renderer, and closed-form gradients of a single axis-aligned octahedron.
"""
import math

import numpy as np
import pytest
import torch

from paper_2501_16312_amd import scenes
from tests import helpers as H
from tests import torch_reference as TR

OCTA, TETRA = scenes.OCTAHEDRON, scenes.TETRAHEDRON
FIELDS = ("means", "quats", "dists", "opacity", "sh")


def _small_scene(kind, n, seed, W=32, H_=32):
    rng = np.random.default_rng(seed)
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(n, seed=seed, box=0.35, dmin=0.15, dmax=0.4)
    sc.means[:, 2] += 0.0
    sc.opacity[:] = rng.uniform(0.3, 0.9, size=n).astype(np.float32)
    cam = scenes.look_at((0.2, -0.1, -2.5), (0, 0, 0), W, H_)
    return sc, cam


def _loss64(oracle_mod, sc, cam, p64, g, bg):
    O = oracle_mod.OracleScene(sc, [cam], tile=16, inputs64=p64)
    return float(np.dot(O.render(bg=bg)["rgb"], g))


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_backward_matches_torch_autograd(oracle_mod, kind):
    """P10: analytic FP64 backward vs autograd of an independent renderer."""
    sc, cam = _small_scene(kind, 8, seed=21 + kind)
    bg = np.array([0.2, 0.1, 0.3])
    rng = np.random.default_rng(5)
    g = rng.normal(size=3 * cam.width * cam.height)
    O = oracle_mod.OracleScene(sc, [cam], tile=16)
    r = O.render(bg=bg)
    params = {k: torch.tensor(getattr(sc, k).astype(np.float64), requires_grad=True) for k in FIELDS}
    img = TR.render(kind, params, cam, bg)
    np.testing.assert_allclose(img.detach().numpy().reshape(-1), r["rgb"], atol=1e-11)
    (img.reshape(-1) * torch.tensor(g)).sum().backward()
    ob = O.backward(g, bg=bg)
    assert not (ob["ill_bits"] & 1).any()      # no discrete decision near a switch
    for k in FIELDS:
        ref = params[k].grad.numpy()
        got = ob[k]
        scale = np.abs(ref).max() + 1e-12
        np.testing.assert_allclose(got, ref, rtol=1e-7, atol=1e-9 * scale, err_msg=k)
    assert np.abs(ob["means"]).max() > 0 and np.abs(ob["quats"]).max() > 0


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_backward_matches_central_differences(oracle_mod, kind):
    """P10: analytic FP64 backward vs central differences of the forward."""
    sc, cam = _small_scene(kind, 6, seed=31 + kind, W=40, H_=32)
    bg = np.array([0.3, 0.2, 0.1])
    rng = np.random.default_rng(9)
    g = rng.normal(size=3 * cam.width * cam.height)
    O = oracle_mod.OracleScene(sc, [cam], tile=8)
    ob = O.backward(g, bg=bg)
    base = {k: getattr(sc, k).astype(np.float64) for k in FIELDS}
    h = 1e-6
    checked = 0
    for field in FIELDS:
        arr = base[field]
        flat_idx = rng.choice(arr.size, size=min(arr.size, 12), replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, arr.shape)
            if field == "sh" and idx[1] >= 16:
                continue
            plus = {k: v.copy() for k, v in base.items()}
            minus = {k: v.copy() for k, v in base.items()}
            plus[field][idx] += h
            minus[field][idx] -= h
            fd = (_loss64(oracle_mod, sc, cam, plus, g, bg) - _loss64(oracle_mod, sc, cam, minus, g, bg)) / (2 * h)
            an = ob[field][idx]
            if field == "dists" and np.sum(base["dists"][idx[0]] == base["dists"][idx[0]].min()) == 1 \
                    and idx[1] == int(np.argmin(base["dists"][idx[0]])):
                # the analytic gradient holds min(d) of Eq. 1 constant (App. G);
                # central differences also move sigma through it: add
                # dL/dsigma * dsigma/dmin, with dL/dsigma = dL/dalpha / dsigma/dalpha
                al = base["opacity"][idx[0]]
                dmin = base["dists"][idx[0]].min()
                sigma = -math.log(1 - 0.99 * al) / (2 * dmin)
                dL_dsigma = ob["opacity"][idx[0]] / (0.99 / ((1 - 0.99 * al) * 2 * dmin))
                an = an + dL_dsigma * (-sigma / dmin)
            assert abs(an - fd) <= 1e-5 * max(abs(fd), 1e-3), (field, idx, an, fd)
            checked += 1
    assert checked >= 40


def test_single_octahedron_closed_form_gradients(oracle_mod):
    """P2 derivatives: o = 1 - (1 - 0.99 alpha)^(chord / 2 min d) with the
    rhombus chord 2c(1 - |X|/A - |Y|/B), A = f a / D, B = f b / D."""
    W = H_ = 32
    cam = H.origin_camera(W, H_)
    f = float(cam.fx)
    a, b, c, D, alpha = 0.3, 0.25, 0.2, 2.0, 0.6
    sc = H.prims(OCTA, [0, 0, D], [1, 0, 0, 0], [a, b, c], alpha, rgb=(0.9, 0.4, 0.2))
    a32, b32, c32, al32 = (float(np.float32(v)) for v in (a, b, c, alpha))
    A, B = f * a32 / D, f * b32 / D
    O = oracle_mod.OracleScene(sc, [cam])
    i, j = 17, 15
    X, Y = i + 0.5 - W / 2, j + 0.5 - H_ / 2
    g = np.zeros(3 * W * H_)
    g[j * W + i] = 1.0                                  # dL/dC_red at one pixel
    ob = O.backward(g)
    rgb_r = H.rgb_of(sc)[0]
    chord = 2 * c32 * (1 - abs(X) / A - abs(Y) / B)
    assert chord > 0
    sigma = -math.log(1 - 0.99 * al32) / (2 * c32)
    o = 1 - math.exp(-sigma * chord)
    do_dalpha = (1 - o) * chord * 0.99 / ((1 - 0.99 * al32) * 2 * c32)
    do_dchord = sigma * (1 - o)
    assert abs(ob["opacity"][0] - rgb_r * do_dalpha) < 1e-12
    # depth half-axis c: the chord scales with c; min d held constant in sigma
    assert abs(ob["dists"][0, 2] - rgb_r * do_dchord * 2 * (1 - abs(X) / A - abs(Y) / B)) < 1e-10
    # lateral half-axis a: chord depends on A = f a / D
    assert abs(ob["dists"][0, 0] - rgb_r * do_dchord * 2 * c32 * abs(X) / (A * a32)) < 1e-10
    assert abs(ob["dists"][0, 1] - rgb_r * do_dchord * 2 * c32 * abs(Y) / (B * b32)) < 1e-10
    # colour: dC/drgb = T o with T = 1; degree-0 SH coefficient gets Y_00
    assert abs(ob["sh"][0, 0, 0] - o * H.SH_C0) < 1e-12
    assert ob["sh"][0, 0, 1] == 0.0
