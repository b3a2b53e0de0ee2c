"""Pins of the oracle's depth map (appendix "Depth and Surface
Reconstruction"): the distance along the pixel's viewing ray to the first
primitive at which the cumulative opacity exceeds 0.5, i.e. to that
primitive's entry hit; 0 where the opacity never exceeds 0.5.

References: closed forms for axis-aligned octahedra stacked along the
optical axis, in ray space (the rhombus chord of Sec. 3.2, centred on the
centre's depth) and along the true pixel ray (a line entering the L1 ball),
with the textbook transmittance product deciding which primitive crosses
0.5; and invariants on a random scene (a depth exists exactly where the
final transmittance is below 0.5, and it lies inside the depth range of a
primitive that covers the pixel).  No GPU needed.
"""
import math

import numpy as np

from paper_2501_16312_amd import scenes
from tests import helpers as H

OCTA = scenes.OCTAHEDRON


def _stack(alphas, depths, c=0.25):
    return H.prims(OCTA, [[0, 0, z] for z in depths], [1, 0, 0, 0], [1.0, 1.0, c], alphas)


def _crossing(alphas, chords, c32):
    """Index of the primitive at which 1 - T first exceeds 0.5, or None."""
    T = 1.0
    for k, delta in enumerate(chords):
        sigma = -math.log(1 - 0.99 * float(np.float32(alphas[k]))) / (2 * c32)
        o = min(0.99, 1 - math.exp(-sigma * delta))
        before, T = T, T * (1 - o)
        if before >= 0.5 > T:
            return k
        if T <= 1e-3:
            break
    return None


def _expected_ray_space(cam, alphas, depths, X, Y, c=0.25):
    """Ray space: at the centre J = diag(f/D, f/D, 1), the footprint is the
    rhombus |X|/A + |Y|/A <= 1 (A = f/D for half-axes 1) and the chord
    2c (1 - |X|/A - |Y|/A) is centred on the ray-space depth D, so the entry
    lies half a chord in front of it."""
    f = float(np.float32(cam.fx))
    c32 = float(np.float32(c))
    chords = []
    for z in depths:
        A = f / float(np.float32(z))
        chords.append(2 * c32 * max(0.0, 1 - abs(X) / A - abs(Y) / A))
    k = _crossing(alphas, chords, c32)
    return 0.0 if k is None else float(np.float32(depths[k])) - chords[k] / 2, k


def _expected_exact(cam, alphas, depths, X, Y, c=0.25):
    """Exact rays: the ray t (X/f, Y/f, 1) enters |x| + |y| + |z - D|/c <= 1
    through its front face at t = (D/c - 1) / (1/c - (|X| + |Y|)/f) and
    leaves through the back face at t = (D/c + 1) / (1/c + (|X| + |Y|)/f);
    the chord and the entry distance are those parameters times |(X/f, Y/f, 1)|."""
    f = float(np.float32(cam.fx))
    c32 = float(np.float32(c))
    s = (abs(X) + abs(Y)) / f
    nD = math.sqrt((X / f) ** 2 + (Y / f) ** 2 + 1.0)
    t_in, t_out = [], []
    for z in depths:
        D = float(np.float32(z))
        t_in.append((D / c32 - 1) / (1 / c32 - s))
        t_out.append((D / c32 + 1) / (1 / c32 + s))
    chords = [(b - a) * nD for a, b in zip(t_in, t_out)]
    k = _crossing(alphas, chords, c32)
    return 0.0 if k is None else t_in[k] * nD, k


def test_depth_of_stacked_primitives(oracle_mod):
    W = H_ = 16
    cam = H.origin_camera(W, H_)
    depths = [2.0, 2.6, 3.2, 3.8, 4.4]
    for alphas, want_k in [([0.2, 0.3, 0.9, 0.9, 0.9], 2), ([0.9, 0.2, 0.2, 0.2, 0.2], 0),
                           ([0.1, 0.1, 0.1, 0.1, 0.1], None)]:
        sc = _stack(alphas, depths)
        for exact, expect in ((False, _expected_ray_space), (True, _expected_exact)):
            d = oracle_mod.OracleScene(sc, [cam], exact=exact).render_depth()
            for i, j in ((8, 8), (7, 8), (9, 8)):
                ref, k = expect(cam, alphas, depths, i + 0.5 - W / 2, j + 0.5 - H_ / 2)
                got = d["depth"][j * W + i]
                assert k == want_k
                assert abs(got - ref) <= 1e-12 * max(ref, 1.0), (alphas, exact, i, j, got, ref)
                if want_k is None:
                    assert got == 0.0
                else:
                    # in front of the centre, behind the front corner
                    assert float(np.float32(depths[want_k])) - 0.25 - 1e-6 < got < float(np.float32(depths[want_k]))


def test_depth_invariants_on_a_random_scene(oracle_mod):
    sc = scenes.uniform_octahedra(1500, seed=91, dmin=0.05, dmax=0.25)
    cam = scenes.look_at((0.2, 0.1, -3.0), (0, 0, 0), 64, 48)
    O = oracle_mod.OracleScene(sc, [cam], tile=8)
    r = O.render()
    d = O.render_depth()
    has = d["depth"] > 0
    assert np.array_equal(has, r["T"] < 0.5)
    assert 0.2 < has.mean() < 0.95
    p = O.prep()
    # ray-space depth range of each primitive: centre depth +/- the largest
    # depth component of its three axis vectors
    zc = p["c"][:, 2]
    ext = np.abs(p["a"][:, :3, 2]).max(1)
    rect = p["rect"]
    for q in np.nonzero(has)[0][::7]:
        i, j = q % cam.width, q // cam.width
        cover = p["valid"] & (rect[:, 0] <= i) & (i <= rect[:, 2]) & (rect[:, 1] <= j) & (j <= rect[:, 3])
        z = d["depth"][q]
        assert np.any(cover & (zc - ext - 1e-9 <= z) & (z <= zc + ext + 1e-9)), q
