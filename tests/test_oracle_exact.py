"""Pins of the oracle's exact variant (the appendix on the ray-space
approximation): pixel rays from the camera centre meet the camera-space
primitive, with no affine ray space.

References other than the oracle itself: a closed form for an axis-aligned
octahedron on the optical axis (and its exact ratio to the ray-space closed
form), point-membership sampling along the ray, the independent clipping
formulation, brute force against the tiled walk, central differences of
single hits and of whole renders, autograd of the independent PyTorch
renderer, and the convergence of the ray-space chord to the exact one as
primitives shrink.  No GPU needed.
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


def _ray(cam, px, py):
    """Pixel ray direction with the camera's float32 intrinsics (what the
    renderers receive)."""
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    return np.array([(px - cx) / fx, (py - cy) / fy, 1.0])


def test_ray_hit_gradient_matches_central_differences(oracle_mod):
    """dt/dV_j = w_j n / (n . D) against central differences of the hit."""
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(40):
        V = rng.normal(size=(3, 3)) * 0.3 + np.array([0.0, 0.0, 5.0])
        w = rng.dirichlet(np.ones(3))
        target = w @ V
        D = target / target[2]
        r = oracle_mod.mtia_ray(V, D)
        assert r["hit"]
        assert abs(r["t"] - target[2]) < 1e-12
        h = 1e-7
        for j in range(3):
            for k in range(3):
                Vp, Vm = V.copy(), V.copy()
                Vp[j, k] += h
                Vm[j, k] -= h
                tp, tm = oracle_mod.mtia_ray(Vp, D), oracle_mod.mtia_ray(Vm, D)
                if not (tp["hit"] and tm["hit"]):
                    continue
                fd = (tp["t"] - tm["t"]) / (2 * h)
                assert abs(r["dV"][j, k] - fd) < 1e-6 * max(1.0, abs(fd)), (j, k)
                checked += 1
    assert checked > 300


def test_ray_hit_misses_outside_triangle(oracle_mod):
    V = np.array([[0.0, 0.0, 4.0], [1.0, 0.0, 4.0], [0.0, 1.0, 4.0]])
    assert oracle_mod.mtia_ray(V, [-0.05, 0.1, 1.0])["hit"] is False        # (-0.2, 0.4, 4): outside
    hit = oracle_mod.mtia_ray(V, [0.05, 0.05, 1.0])                          # (0.2, 0.2, 4): inside
    assert hit["hit"] and abs(hit["t"] - 4.0) < 1e-15
    assert abs(hit["u"] - 0.2) < 1e-15 and abs(hit["v"] - 0.2) < 1e-15
    assert oracle_mod.mtia_ray(V, [0.2, 0.2, 1.0])["hit"] is False          # (0.8, 0.8): u + v > 1
    edge = oracle_mod.mtia_ray(V, [0.125, 0.125, 1.0])                       # (0.5, 0.5): on the edge
    assert edge["hit"]


def _axis_octa_closed_form(cam, a, b, c, D, px, py):
    """Chord of |x|/a + |y|/b + |z - D|/c <= 1 along t r: with
    k = |r_x|/a + |r_y|/b the segment is t in [(D-c)/(1+... )], length
    2 c |r| (1 - k D) / (1 - (k c)^2) when k D <= 1, else 0."""
    r = _ray(cam, px, py)
    k = abs(r[0]) / a + abs(r[1]) / b
    if k * D >= 1.0:
        return 0.0
    return 2.0 * c * np.linalg.norm(r) * (1.0 - k * D) / (1.0 - (k * c) ** 2)


def test_axis_octahedron_closed_form(oracle_mod):
    W = H_ = 48
    cam = H.origin_camera(W, H_)
    a, b, c, D, alpha = 0.375, 0.25, 0.5, 1.5, 0.75     # float32-exact values
    sc = H.prims(OCTA, [0, 0, D], [1, 0, 0, 0], [a, b, c], alpha, rgb=(0.7, 0.4, 0.2))
    ex = oracle_mod.OracleScene(sc, [cam], exact=True)
    rs = oracle_mod.OracleScene(sc, [cam])
    n_in = 0
    for j in range(H_):
        for i in range(W):
            px, py = i + 0.5, j + 0.5
            ref = _axis_octa_closed_form(cam, a, b, c, D, px, py)
            got = ex.chord(0, 0, px, py)
            assert abs(got - ref) < 1e-12, (i, j, got, ref)
            assert abs(ex.chord(0, 0, px, py, method="clip") - ref) < 1e-12
            if ref > 0:
                n_in += 1
                # relation to the ray-space rhombus 2c(1 - |X|/A - |Y|/B):
                # exact = ray space * |r| / (1 - (k c)^2)
                r = _ray(cam, px, py)
                k = abs(r[0]) / a + abs(r[1]) / b
                assert abs(got - rs.chord(0, 0, px, py) * np.linalg.norm(r) / (1 - (k * c) ** 2)) < 1e-12
    assert n_in > 100
    # the rendered opacity follows Eq. 1 with the exact chord
    out = ex.render()
    sigma = -math.log(1 - 0.99 * alpha) / (2 * min(a, b, c))
    rgb = H.rgb_of(sc)
    for (i, j) in [(24, 24), (20, 27), (30, 18)]:
        ch = _axis_octa_closed_form(cam, a, b, c, D, i + 0.5, j + 0.5)
        o = min(0.99, 1 - math.exp(-sigma * ch))
        assert abs(out["rgb"][j * W + i] - o * rgb[0]) < 1e-12


def _inside_octa(x, mu, R, d):
    loc = (x - mu) @ R                       # rows: local coordinates R^T (x - mu)
    return np.abs(loc / d).sum(-1) <= 1.0


def _inside_tetra(x, corners):
    E = (corners[1:] - corners[0]).T
    lam = np.linalg.solve(E, (x - corners[0]).T).T
    return (lam >= 0).all(-1) & (lam.sum(-1) <= 1.0)


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_chord_by_membership_sampling(oracle_mod, kind):
    """Count sample points of the pixel ray inside the primitive (membership
    tested in the primitive's own frame) against the oracle's chord."""
    W, H_ = 40, 32
    cam = H.origin_camera(W, H_)
    rng = np.random.default_rng(11 + kind)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    R = H.quat_to_matrix(q)
    mu = np.array([0.1, -0.05, 1.2])
    d = np.array([0.3, 0.22, 0.35]) if kind == OCTA else np.array([0.4, 0.3, 0.35, 0.45])
    sc = H.prims(kind, mu, q, d, 0.5)
    mu32 = sc.means[0].astype(np.float64)
    R32 = H.quat_to_matrix(sc.quats[0].astype(np.float64))
    d32 = sc.dists[0].astype(np.float64)
    O = oracle_mod.OracleScene(sc, [cam], exact=True)
    if kind == TETRA:
        corners = mu32 + (R32 @ (TR.TET_DIRS * d32[:, None]).T).T
    ts = np.linspace(0.4, 2.0, 320001)
    dt = ts[1] - ts[0]
    checked = 0
    for (i, j) in [(22, 14), (20, 15), (24, 13), (22, 12), (19, 16), (23, 16)]:
        r = _ray(cam, i + 0.5, j + 0.5)
        pts = ts[:, None] * r[None, :]
        inside = _inside_octa(pts, mu32, R32, d32) if kind == OCTA else _inside_tetra(pts, corners)
        est = inside.sum() * dt * np.linalg.norm(r)
        got = O.chord(0, 0, i + 0.5, j + 0.5)
        assert abs(got - est) <= 2.5 * dt * np.linalg.norm(r), (i, j, got, est)
        checked += got > 0
    assert checked >= 4
    del R


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_two_formulations_agree(oracle_mod, kind):
    """Per-face ray hits against slab / barycentric clipping of the line."""
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(24, seed=5 + kind, box=0.8, dmin=0.1, dmax=0.45)
    cam = scenes.look_at((0.3, 0.2, -3.0), (0, 0, 0), 48, 40)
    O = oracle_mod.OracleScene(sc, [cam], exact=True)
    p = O.prep()
    n_cmp = 0
    for n in np.nonzero(p["valid"])[0]:
        i0, j0, i1, j1 = p["rect"][n]
        for j in range(j0, j1 + 1):
            for i in range(i0, i1 + 1):
                a = O.chord(0, int(n), i + 0.5, j + 0.5, "mtia")
                b = O.chord(0, int(n), i + 0.5, j + 0.5, "clip")
                assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (n, i, j, a, b)
                n_cmp += a > 0
    assert n_cmp > 150
    # the whole render through either formulation
    r1, r2 = O.render(mode="tiled"), O.render(mode="clip")
    np.testing.assert_allclose(r1["rgb"], r2["rgb"], atol=1e-12)


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_footprint_inside_rectangle(oracle_mod, kind):
    """Every pixel whose ray meets the primitive lies in its pixel rectangle
    (bounding box of the perspective-projected corners)."""
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(12, seed=9 + kind, box=0.6, dmin=0.1, dmax=0.35)
    cam = scenes.look_at((0.0, 0.0, -2.5), (0, 0, 0), 40, 40)
    O = oracle_mod.OracleScene(sc, [cam], exact=True)
    p = O.prep()
    hits = 0
    for n in np.nonzero(p["valid"])[0]:
        i0, j0, i1, j1 = p["rect"][n]
        for j in range(cam.height):
            for i in range(cam.width):
                if O.chord(0, int(n), i + 0.5, j + 0.5, "clip") > 0:
                    hits += 1
                    assert i0 <= i <= i1 and j0 <= j <= j1, (n, i, j)
    assert hits > 60


def test_corner_behind_near_plane_is_culled(oracle_mod):
    """A primitive whose corner crosses the near plane keeps its ray-space
    footprint but is culled without ray space (no projection there)."""
    cam = H.origin_camera(32, 32)
    sc = H.prims(OCTA, [[0.0, 0.0, 0.5], [0.0, 0.0, 2.0]], [1, 0, 0, 0], [[0.1, 0.1, 0.4], [0.1, 0.1, 0.1]], 0.5)
    ex = oracle_mod.OracleScene(sc, [cam], exact=True).prep()
    rs = oracle_mod.OracleScene(sc, [cam]).prep()
    assert rs["valid"][0] and not ex["valid"][0]       # corner z = 0.1 < near 0.2
    assert rs["valid"][1] and ex["valid"][1]


@pytest.mark.parametrize("kind", [OCTA, TETRA])
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_brute_force_equals_tiled(oracle_mod, kind, tile):
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(60, seed=13 + kind, box=0.9, dmin=0.05, dmax=0.25)
    cam = scenes.look_at((0.2, -0.3, -3.0), (0, 0, 0), 56, 40)
    O = oracle_mod.OracleScene(sc, [cam], tile=tile, exact=True)
    a, b = O.render(mode="tiled"), O.render(mode="brute")
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["T"], b["T"])


def test_ray_space_converges_to_exact_for_small_primitives(oracle_mod):
    """The affine ray-space map is the first-order expansion of the exact
    projection at the centre: chord differences shrink with the size."""
    cam = H.origin_camera(512, 512)
    q = np.array([0.9, 0.2, -0.3, 0.25])
    errs = []
    for s in (0.4, 0.1, 0.025):
        sc = H.prims(OCTA, [0.9, -0.6, 3.0], q, [s, 0.8 * s, 1.2 * s], 0.5)
        ex = oracle_mod.OracleScene(sc, [cam], exact=True)
        rs = oracle_mod.OracleScene(sc, [cam])
        c = rs.prep()["c"][0]
        rad = cam.fx * s / 3.0
        worst = 0.0
        for (u, v) in [(0.3, 0.1), (-0.2, 0.25), (0.1, -0.35), (0.0, 0.0)]:
            px, py = c[0] + u * rad, c[1] + v * rad
            e, r = ex.chord(0, 0, px, py), rs.chord(0, 0, px, py)
            assert e > 0 and r > 0
            worst = max(worst, abs(e - r) / e)
        errs.append(worst)
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], errs
    assert errs[2] < 0.02, errs


def _small_scene(kind, n, seed, W=32, H_=32):
    rng = np.random.default_rng(seed)
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(n, seed=seed, box=0.35, dmin=0.15, dmax=0.4)
    sc.opacity[:] = rng.uniform(0.3, 0.9, size=n).astype(np.float32)
    cam = scenes.look_at((0.2, -0.1, -2.5), (0, 0, 0), W, H_)
    return sc, cam


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_backward_matches_torch_autograd(oracle_mod, kind):
    """Analytic FP64 backward of the exact variant vs autograd of the
    independent renderer's exact mode."""
    sc, cam = _small_scene(kind, 8, seed=41 + kind)
    bg = np.array([0.2, 0.1, 0.3])
    g = np.random.default_rng(6).normal(size=3 * cam.width * cam.height)
    O = oracle_mod.OracleScene(sc, [cam], tile=16, exact=True)
    r = O.render(bg=bg)
    params = {k: torch.tensor(getattr(sc, k).astype(np.float64), requires_grad=True) for k in FIELDS}
    img = TR.render(kind, params, cam, bg, exact=True)
    np.testing.assert_allclose(img.detach().numpy().reshape(-1), r["rgb"], atol=1e-11)
    (img.reshape(-1) * torch.tensor(g)).sum().backward()
    ob = O.backward(g, bg=bg)
    assert not (ob["ill_bits"] & 1).any()      # no discrete decision near a switch
    for k in FIELDS:
        ref = params[k].grad.numpy()
        scale = np.abs(ref).max() + 1e-12
        np.testing.assert_allclose(ob[k], ref, rtol=1e-7, atol=1e-9 * scale, err_msg=k)
    assert np.abs(ob["means"]).max() > 0 and np.abs(ob["quats"]).max() > 0


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_backward_matches_central_differences(oracle_mod, kind):
    sc, cam = _small_scene(kind, 6, seed=51 + kind, W=40, H_=32)
    bg = np.array([0.3, 0.2, 0.1])
    rng = np.random.default_rng(10)
    g = rng.normal(size=3 * cam.width * cam.height)
    ob = oracle_mod.OracleScene(sc, [cam], tile=8, exact=True).backward(g, bg=bg)
    base = {k: getattr(sc, k).astype(np.float64) for k in FIELDS}

    def loss(p64):
        O = oracle_mod.OracleScene(sc, [cam], tile=16, inputs64=p64, exact=True)
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
