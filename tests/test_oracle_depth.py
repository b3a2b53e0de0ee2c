"""Pins of the oracle's depth map (appendix "Depth and Surface
Reconstruction"): the depth of the first primitive along the ray at which
the cumulative opacity exceeds 0.5, read as that primitive's centre camera
depth (the float32 sort key); 0 where the opacity never exceeds 0.5.

References: the textbook transmittance product on primitives stacked along
the axis, and invariants on a random scene (a depth exists exactly where the
final transmittance is below 0.5, and it is the depth of a primitive in the
pixel's list).  No GPU needed.
"""
import math

import numpy as np

from paper_2501_16312_amd import scenes
from tests import helpers as H

OCTA = scenes.OCTAHEDRON


def _stack(alphas, depths, c=0.25):
    return H.prims(OCTA, [[0, 0, z] for z in depths], [1, 0, 0, 0], [1.0, 1.0, c], alphas)


def _expected_depth(cam, alphas, depths, X, Y, c=0.25):
    f = float(np.float32(cam.fx))
    c32 = float(np.float32(c))
    T = 1.0
    for k in range(len(depths)):
        A = f / float(np.float32(depths[k]))
        delta = 2 * c32 * max(0.0, 1 - abs(X) / A - abs(Y) / A)
        sigma = -math.log(1 - 0.99 * float(np.float32(alphas[k]))) / (2 * c32)
        o = min(0.99, 1 - math.exp(-sigma * delta))
        before, T = T, T * (1 - o)
        if before >= 0.5 > T:
            return float(np.float32(depths[k]))
        if T <= 1e-3:
            break
    return 0.0


def test_depth_of_stacked_primitives(oracle_mod):
    W = H_ = 16
    cam = H.origin_camera(W, H_)
    depths = [2.0, 2.6, 3.2, 3.8, 4.4]
    for alphas, want_k in [([0.2, 0.3, 0.9, 0.9, 0.9], 2), ([0.9, 0.2, 0.2, 0.2, 0.2], 0),
                           ([0.1, 0.1, 0.1, 0.1, 0.1], None)]:
        sc = _stack(alphas, depths)
        d = oracle_mod.OracleScene(sc, [cam]).render_depth()
        i = j = 8
        ref = _expected_depth(cam, alphas, depths, i + 0.5 - W / 2, j + 0.5 - H_ / 2)
        got = d["depth"][j * W + i]
        assert got == ref, (alphas, got, ref)
        if want_k is None:
            assert got == 0.0
        else:
            assert got == float(np.float32(depths[want_k]))


def test_depth_invariants_on_a_random_scene(oracle_mod):
    sc = scenes.uniform_octahedra(1500, seed=91, dmin=0.05, dmax=0.25)
    cam = scenes.look_at((0.2, 0.1, -3.0), (0, 0, 0), 64, 48)
    O = oracle_mod.OracleScene(sc, [cam], tile=8)
    r = O.render()
    d = O.render_depth()
    has = d["depth"] > 0
    assert np.array_equal(has, r["T"] < 0.5)
    assert 0.2 < has.mean() < 0.95
    keys = O.prep()["key"].view(np.float32).astype(np.float64)
    valid = O.prep()["valid"]
    assert np.all(np.isin(d["depth"][has], keys[valid]))
