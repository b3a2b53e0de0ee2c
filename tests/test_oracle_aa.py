"""Pins of the oracle's 2D anti-aliasing filter (appendix "Anti-Aliasing";
filter size 0.1 pixel in App. G): corners on the tiling box move outward
parallel to the screen, an octahedron's axis vector by half the size.

Closed forms: the rhombus of an axis-aligned octahedron on the optical axis
(its half-extents grow by 0.05 pixel), and the square pyramid chord of a
tetrahedron seen along a 2-fold axis (every corner lies on the box; its
half-extent grows by the same 0.05 pixel).  The same tetrahedron also pins the
ray-space tetrahedron chord without the filter.  Plus: the two chord
formulations, brute force against the tiled walk, and the analytic backward
against central differences.  No GPU needed.
"""
import math

import numpy as np
import pytest

from paper_2501_16312_amd import scenes
from tests import helpers as H

OCTA, TETRA = scenes.OCTAHEDRON, scenes.TETRAHEDRON
FIELDS = ("means", "quats", "dists", "opacity", "sh")


def _f32(v):
    return float(np.float32(v))


@pytest.mark.parametrize("aa", [False, True])
def test_rhombus_with_filter(oracle_mod, aa):
    W = H_ = 40
    cam = H.origin_camera(W, H_)
    f = _f32(cam.fx)
    a, b, c, D, alpha = 0.375, 0.25, 0.5, 1.5, 0.6
    sc = H.prims(OCTA, [0, 0, D], [1, 0, 0, 0], [a, b, c], alpha, rgb=(0.9, 0.3, 0.1))
    O = oracle_mod.OracleScene(sc, [cam], antialias=aa)
    A, B = f * a / D, f * b / D
    if aa:
        A, B = A + 0.05, B + 0.05
    n_in = 0
    for j in range(H_):
        for i in range(W):
            X, Y = i + 0.5 - W / 2, j + 0.5 - H_ / 2
            ref = 2 * c * max(0.0, 1 - abs(X) / A - abs(Y) / B)
            got = O.chord(0, 0, i + 0.5, j + 0.5)
            assert abs(got - ref) < 1e-12, (i, j, got, ref)
            assert abs(O.chord(0, 0, i + 0.5, j + 0.5, "clip") - ref) < 1e-12
            n_in += ref > 0
    assert n_in > 50
    # image: Eq. 1 density from the world distances (the filter leaves it)
    img = O.render()["rgb"]
    sigma = -math.log(1 - 0.99 * _f32(alpha)) / (2 * min(a, b, c))
    red = H.rgb_of(sc)[0]
    for (i, j) in [(20, 20), (22, 19), (17, 21)]:
        X, Y = i + 0.5 - W / 2, j + 0.5 - H_ / 2
        ch = 2 * c * max(0.0, 1 - abs(X) / A - abs(Y) / B)
        assert abs(img[j * W + i] - red * min(0.99, 1 - math.exp(-sigma * ch))) < 1e-12


@pytest.mark.parametrize("aa", [False, True])
def test_tetrahedron_square_pyramid(oracle_mod, aa):
    """Regular tetrahedron (identity rotation, all distances d) on the axis at
    depth D: its ray-space corners are (+-s, +-s, +-h) with s = f d / (sqrt3 D),
    h = d / sqrt3, two edges crossing at right angles seen along z, and the
    chord is 2 h max(0, 1 - max(|X|, |Y|) / s); the filter puts every corner
    on the box and makes s -> s + 0.05 (the box grows by 0.1 per axis, as an
    octahedron's does)."""
    W = H_ = 48
    cam = H.origin_camera(W, H_)
    f = _f32(cam.fx)
    d, D = 0.5, 2.0
    sc = H.prims(TETRA, [0, 0, D], [1, 0, 0, 0], [d, d, d, d], 0.5)
    O = oracle_mod.OracleScene(sc, [cam], antialias=aa)
    s = f * d / (math.sqrt(3) * D) + (0.05 if aa else 0.0)
    h = d / math.sqrt(3)
    n_in = 0
    for j in range(H_):
        for i in range(W):
            X, Y = i + 0.5 - W / 2, j + 0.5 - H_ / 2
            ref = 2 * h * max(0.0, 1 - max(abs(X), abs(Y)) / s)
            got = O.chord(0, 0, i + 0.5, j + 0.5)
            assert abs(got - ref) < 1e-12, (i, j, got, ref)
            n_in += ref > 0
    assert n_in > 100


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_filter_two_formulations_and_brute_force(oracle_mod, kind):
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(50, seed=61 + kind, box=0.8, dmin=0.02, dmax=0.2)
    cam = scenes.look_at((0.2, -0.2, -3.0), (0, 0, 0), 56, 40)
    O = oracle_mod.OracleScene(sc, [cam], tile=8, antialias=True)
    r1, r2, r3 = O.render(mode="tiled"), O.render(mode="clip"), O.render(mode="brute")
    np.testing.assert_allclose(r1["rgb"], r2["rgb"], atol=1e-12)
    assert np.array_equal(r1["rgb"], r3["rgb"])
    plain = oracle_mod.OracleScene(sc, [cam], tile=8).render()
    assert np.abs(plain["rgb"] - r1["rgb"]).max() > 1e-4       # the filter changes the image
    # every primitive's rectangle grows or stays (corners only move outward)
    pa = O.prep()
    pp = oracle_mod.OracleScene(sc, [cam], tile=8).prep()
    both = pa["valid"] & pp["valid"]
    assert np.all(pa["rect"][both, :2] <= pp["rect"][both, :2])
    assert np.all(pa["rect"][both, 2:] >= pp["rect"][both, 2:])
    assert np.all(pa["valid"] >= pp["valid"])


def test_filter_rejected_without_ray_space(oracle_mod):
    sc = H.prims(OCTA, [0, 0, 2.0], [1, 0, 0, 0], [0.2, 0.2, 0.2], 0.5)
    with pytest.raises(ValueError):
        oracle_mod.OracleScene(sc, [H.origin_camera(16, 16)], exact=True, antialias=True)


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_filter_backward_matches_central_differences(oracle_mod, kind):
    rng = np.random.default_rng(70 + kind)
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(6, seed=71 + kind, box=0.35, dmin=0.1, dmax=0.3)
    sc.opacity[:] = rng.uniform(0.3, 0.9, size=sc.n).astype(np.float32)
    cam = scenes.look_at((0.2, -0.1, -2.5), (0, 0, 0), 40, 32)
    bg = np.array([0.3, 0.2, 0.1])
    g = rng.normal(size=3 * cam.width * cam.height)
    ob = oracle_mod.OracleScene(sc, [cam], tile=8, antialias=True).backward(g, bg=bg)
    base = {k: getattr(sc, k).astype(np.float64) for k in FIELDS}

    def loss(p64):
        O = oracle_mod.OracleScene(sc, [cam], tile=16, inputs64=p64, antialias=True)
        return float(np.dot(O.render(bg=bg)["rgb"], g))

    h = 1e-6
    checked = 0
    for field in ("means", "quats", "dists", "opacity"):
        arr = base[field]
        for fi in rng.choice(arr.size, size=min(arr.size, 10), replace=False):
            idx = np.unravel_index(fi, arr.shape)
            if field == "dists" and idx[1] == int(np.argmin(base["dists"][idx[0]])):
                continue          # min(d) of Eq. 1 is held constant in the analytic gradient
            plus = {k: v.copy() for k, v in base.items()}
            minus = {k: v.copy() for k, v in base.items()}
            plus[field][idx] += h
            minus[field][idx] -= h
            fd = (loss(plus) - loss(minus)) / (2 * h)
            an = ob[field][idx]
            assert abs(an - fd) <= 1e-5 * max(abs(fd), 1e-3), (field, idx, an, fd)
            checked += 1
    assert checked >= 25
