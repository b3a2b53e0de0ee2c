"""Pins of the oracle's adaptive population control (Sec. 3.4 "Adaptive
Population Control"; App. G).

* The view-space positional gradient: moving the principal point cx by h
  translates every ray-space primitive by h pixels (the Jacobian does not
  depend on cx), so the sum over primitives of dL/d(centre x) equals the
  derivative of the loss with respect to cx (central differences), and
  likewise for y.
* The screen radius of an axis-aligned octahedron on the axis is its
  rhombus half-extent f max(a, b) / D.
* The densification rules, case by case on hand-built statistics: expected
  outputs written from the paper's text, not from the implementation.
No GPU needed.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import population as POP
from paper_2501_16312_amd import scenes
from tests import helpers as H

OCTA, TETRA = scenes.OCTAHEDRON, scenes.TETRAHEDRON


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_screen_gradient_is_derivative_in_principal_point(oracle_mod, kind):
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(12, seed=101 + kind, box=0.4, dmin=0.1, dmax=0.3)
    sc.opacity[:] = 0.6
    cam = scenes.look_at((0.2, -0.1, -2.5), (0, 0, 0), 40, 32)
    bg = np.array([0.2, 0.3, 0.1])
    g = np.random.default_rng(3).normal(size=3 * cam.width * cam.height)
    O = oracle_mod.OracleScene(sc, [cam], tile=8)
    O.backward(g, bg=bg)
    st = O.stats()
    total = st["sgrad"][0].sum(0)
    h = 2.0 ** -14     # exact in float32 at these magnitudes; small enough not to straddle a kink

    def loss(dx, dy):
        c = dataclasses.replace(cam, cx=float(np.float32(cam.cx)) + dx, cy=float(np.float32(cam.cy)) + dy)
        return float(np.dot(oracle_mod.OracleScene(sc, [c], tile=8).render(bg=bg)["rgb"], g))

    fdx = (loss(h, 0) - loss(-h, 0)) / (2 * h)
    fdy = (loss(0, h) - loss(0, -h)) / (2 * h)
    assert abs(total[0] - fdx) <= 1e-4 * max(abs(fdx), 1e-2), (total[0], fdx)
    assert abs(total[1] - fdy) <= 1e-4 * max(abs(fdy), 1e-2), (total[1], fdy)
    assert st["visible"][0].sum() >= 8


def test_screen_radius_of_axis_octahedron(oracle_mod):
    cam = H.origin_camera(64, 64)
    f = float(np.float32(cam.fx))
    a, b, c, D = 0.375, 0.25, 0.5, 2.0
    sc = H.prims(OCTA, [0, 0, D], [1, 0, 0, 0], [a, b, c], 0.5)
    O = oracle_mod.OracleScene(sc, [cam])
    O.backward(np.zeros(3 * 64 * 64))
    assert abs(O.stats()["radius"][0, 0] - f * max(a, b) / D) < 1e-12


def test_accumulated_statistics_over_views(oracle_mod):
    sc = scenes.uniform_octahedra(40, seed=7, box=0.5, dmin=0.05, dmax=0.2)
    cams = [scenes.look_at((0, 0, -3.0), (0, 0, 0), 48, 40), scenes.look_at((3.0, 0.2, 0.0), (0, 0, 0), 32, 32)]
    O = oracle_mod.OracleScene(sc, cams, tile=8)
    g = scenes.image_gradient(cams, seed=2).astype(np.float64)
    O.backward(g)
    acc, cnt, rad = np.zeros(sc.n), np.zeros(sc.n), np.zeros(sc.n)
    POP.accumulate_stats(O, acc, cnt, rad)
    vis = np.stack([O.prep(v)["valid"] for v in range(2)])
    assert np.array_equal(cnt, vis.sum(0))
    assert np.all(acc[cnt == 0] == 0) and np.all(acc[cnt > 0] >= 0) and acc.max() > 0
    POP.accumulate_stats(O, acc, cnt, rad)          # a second step adds again
    assert np.array_equal(cnt, 2 * vis.sum(0))


def _case_arrays(kind):
    """Nine primitives, one rule each (extent 10, threshold 1.5e-4)."""
    nd = 3 if kind == OCTA else 4
    n = 9
    s = 2.0 if kind == OCTA else math.sqrt(2.0)            # size = s * max d
    sizes = np.array([0.02, 0.5, 0.3, 0.3, 6.0, 0.3, 0.02, 0.3, 4.4])
    # 0.02 < 0.1 (1% of 10): clone; 6 > 4 (40%): too large; 4.4 > 4 but 4.4 / 1.2 < 4
    dmax = sizes / s
    dists = np.repeat(dmax[:, None], nd, 1).astype(np.float32)
    dists[:, 0] *= 0.5                                      # not all equal: max d still dmax
    opacity = np.array([0.5, 0.5, 0.5, 0.01, 0.5, 0.5, 0.01, 0.5, 0.5], np.float32)
    acc = np.array([4e-4, 4e-4, 1e-4, 0, 0, 0, 4e-4, 0, 4e-4], np.float32)
    cnt = np.array([2, 2, 2, 2, 2, 2, 2, 0, 2], np.int32)
    rad = np.array([1, 1, 1, 1, 1, 25, 1, 0, 1], np.float32)
    return n, dists, opacity, acc, cnt, rad


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_densification_rules_case_by_case(kind):
    n, dists, opacity, acc, cnt, rad = _case_arrays(kind)
    d = POP.decide(kind, dists, opacity, acc, cnt, rad, extent=10.0)
    # 0: high gradient, small -> kept and cloned
    # 1: high gradient, large -> replaced by two children
    # 2: mean gradient 5e-5 below the threshold -> kept
    # 3: transparent -> removed
    # 4: larger than 40% of the scene -> removed
    # 5: screen radius 25 px -> removed
    # 6: high gradient, small, transparent -> removed with its clone
    # 7: never seen -> kept
    # 8: high gradient, larger than 40% of the scene: the original goes, its
    #    children (size / 1.2 = 3.67 < 4) stay
    assert d["keep"].tolist() == [True, False, True, False, False, False, False, True, False]
    assert d["split"].tolist() == [False, True, False, False, False, False, False, False, True]
    assert d["clone"].tolist() == [True, False, False, False, False, False, False, False, False]


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_densify_outputs(kind):
    n, dists, opacity, acc, cnt, rad = _case_arrays(kind)
    rng = np.random.default_rng(5)
    K = 16
    params = {"means": rng.normal(size=(n, 3)).astype(np.float32),
              "quats": rng.normal(size=(n, 4)).astype(np.float32),
              "dists": dists, "opacity": opacity,
              "sh": rng.normal(size=(n, K, 3)).astype(np.float32)}
    moments = {(w, k): rng.normal(size=params[k].shape).astype(np.float32)
               for w in ("m", "v") for k in params}
    normals = rng.normal(size=(n, 2, 3)).astype(np.float32)
    stats = {"grad_accum": acc, "count": cnt, "max_radius": rad}
    newp, newm = POP.densify(kind, params, moments, stats, 10.0, normals)
    # order: 0, clone of 0, children of 1 (two), 2, 7, children of 8 (two)
    src = [0, 0, 1, 1, 2, 7, 8, 8]
    assert newp["means"].shape[0] == len(src)
    for k in ("quats", "opacity", "sh"):
        np.testing.assert_array_equal(newp[k], params[k][src].astype(np.float64))
    kept = [0, 4, 5]                                       # rows that are originals
    new = [1, 2, 3, 6, 7]
    for k in params:
        np.testing.assert_array_equal(newm[("m", k)][kept], moments[("m", k)][[0, 2, 7]].astype(np.float64))
        assert np.all(newm[("m", k)][new] == 0) and np.all(newm[("v", k)][new] == 0)
    np.testing.assert_array_equal(newp["means"][[0, 1, 4, 5]], params["means"][[0, 0, 2, 7]].astype(np.float64))
    for row, (i, j) in zip([2, 3, 6, 7], [(1, 0), (1, 1), (8, 0), (8, 1)]):
        d64 = params["dists"][i].astype(np.float64)
        np.testing.assert_allclose(newp["dists"][row], d64 / 1.2, rtol=1e-15)
        off = newp["means"][row] - params["means"][i].astype(np.float64)
        z = normals[i, j].astype(np.float64)
        if kind == OCTA:
            # the offset in the primitive's own frame is d * z
            R = H.quat_to_matrix(params["quats"][i].astype(np.float64))
            np.testing.assert_allclose(R.T @ off, d64 * z, rtol=1e-12, atol=1e-14)
        else:
            np.testing.assert_allclose(off, d64.max() / 2 * z, rtol=1e-12, atol=1e-14)
