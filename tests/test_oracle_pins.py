"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms of single primitives, invariants, textbook products, an independent
chord formulation, brute force, and library routines.  No GPU needed.
"""
import math

import numpy as np
import pytest
import scipy.special as sps

from paper_2501_16312_amd import scenes
from tests import helpers as H

OCTA, TETRA = scenes.OCTAHEDRON, scenes.TETRAHEDRON


# ---------------------------------------------------------------- SH (P11)
def _sphere_quadrature(nt=48, nph=96):
    xg, wg = np.polynomial.legendre.leggauss(nt)          # cos(theta) nodes
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    ct, p = np.meshgrid(xg, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(p), st * np.sin(p), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nph, 2 * np.pi / nph)[None, :]).reshape(-1)
    return dirs, w


def test_sh_orthonormal(oracle_mod):
    dirs, w = _sphere_quadrature()
    Y = np.stack([oracle_mod.sh_basis(3, d) for d in dirs])
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_matches_scipy_real_basis(oracle_mod):
    """Real SH with the Condon-Shortley phase: Y_lm = sqrt2 Re Y_l^m (m>0),
    sqrt2 Im Y_l^|m| (m<0), Y_l^0 (m=0), from scipy's complex harmonics."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        theta = math.acos(d[2])
        phi = math.atan2(d[1], d[0])
        Y = oracle_mod.sh_basis(3, d)
        k = 0
        for l in range(4):
            for m in range(-l, l + 1):
                c = sps.sph_harm_y(l, abs(m), theta, phi)
                ref = c.real if m == 0 else (math.sqrt(2) * (c.real if m > 0 else c.imag))
                assert abs(Y[k] - ref) < 1e-12, (l, m)
                k += 1


def test_sh_degree_truncation(oracle_mod):
    d = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    full = oracle_mod.sh_basis(3, d)
    for deg in range(4):
        Y = oracle_mod.sh_basis(deg, d)
        K = (deg + 1) ** 2
        np.testing.assert_array_equal(Y[:K], full[:K])
        assert np.all(Y[K:] == 0)


# -------------------------------------------------- MTIA and App. E (P9)
def test_mtia_depth_gradient_matches_central_differences(oracle_mod):
    rng = np.random.default_rng(1)
    checked = 0
    while checked < 200:
        V = rng.normal(size=(3, 3)) * np.array([10.0, 10.0, 1.0])
        w = rng.dirichlet([1, 1, 1])
        r = w @ V[:, :2]
        res = oracle_mod.mtia(V, r[0], r[1])
        if not res["hit"] or min(w) < 0.05:
            continue
        assert abs(res["t"] - w @ V[:, 2]) < 1e-9 * (1 + np.abs(V[:, 2]).max())
        h = 1e-6
        for j in range(3):
            for k in range(3):
                Vp, Vm = V.copy(), V.copy()
                Vp[j, k] += h
                Vm[j, k] -= h
                fd = (oracle_mod.mtia(Vp, *r)["t"] - oracle_mod.mtia(Vm, *r)["t"]) / (2 * h)
                assert abs(res["dV"][j, k] - fd) < 1e-6 * (1 + abs(fd)), (j, k)
        checked += 1


def test_mtia_inclusive_edges_and_misses(oracle_mod):
    V = np.array([[0.0, 0.0, 1.0], [4.0, 0.0, 2.0], [0.0, 4.0, 3.0]])
    assert oracle_mod.mtia(V, 0.0, 0.0)["hit"]            # vertex
    assert oracle_mod.mtia(V, 2.0, 2.0)["hit"]            # hypotenuse
    assert not oracle_mod.mtia(V, 2.0, 2.0001)["hit"]
    assert not oracle_mod.mtia(V, -0.001, 1.0)["hit"]
    Vd = np.array([[0.0, 0.0, 1.0], [1.0, 1.0, 2.0], [2.0, 2.0, 3.0]])   # degenerate in xy
    assert not oracle_mod.mtia(Vd, 1.0, 1.0)["hit"]


# --------------------------------------------------------- closed forms
def test_rhombus_closed_form(oracle_mod):
    """P2: axis-aligned octahedron on the optical axis (App. E geometry)."""
    W = H_ = 64
    cam = H.origin_camera(W, H_)
    f = float(cam.fx)
    a, b, c, D, alpha = 0.3, 0.2, 0.25, 2.0, 0.7
    sc = H.prims(OCTA, [0, 0, D], [1, 0, 0, 0], [a, b, c], alpha)
    O = oracle_mod.OracleScene(sc, [cam], tile=16)
    A, B = f * float(np.float32(a)) / D, f * float(np.float32(b)) / D
    cz = float(np.float32(c))
    rgb = H.rgb_of(sc)
    r = O.render()
    img = r["rgb"].reshape(3, H_, W)
    sigma = -math.log(1 - 0.99 * float(np.float32(alpha))) / (2 * float(np.float32(b)))
    worst = 0.0
    for j in range(H_):
        for i in range(W):
            X, Y = i + 0.5 - W / 2, j + 0.5 - H_ / 2
            delta = 2 * cz * max(0.0, 1 - abs(X) / A - abs(Y) / B)
            got = O.chord(0, 0, i + 0.5, j + 0.5)
            worst = max(worst, abs(got - delta))
            o = min(0.99, 1 - math.exp(-sigma * delta))
            np.testing.assert_allclose(img[:, j, i], rgb * o, atol=1e-12)
    assert worst < 1e-12


def test_eq1_design_point(oracle_mod):
    """P1: a chord of twice the smallest distance gives opacity 0.99 alpha."""
    cam = H.origin_camera(32, 32)
    for alpha in (0.1, 0.5, 0.9):
        # depth half-axis c is the smallest distance; at the principal point
        # the chord is 2c(1 - |X|/A - |Y|/B); with huge A, B it tends to 2c.
        sc = H.prims(OCTA, [0, 0, 3.0], [1, 0, 0, 0], [400.0, 400.0, 0.05], alpha, rgb=(1, 1, 1))
        O = oracle_mod.OracleScene(sc, [cam])
        r = O.render()
        img = r["rgb"].reshape(3, 32, 32)
        f = float(cam.fx)
        A = f * 400.0 / 3.0
        delta = 2 * float(np.float32(0.05)) * (1 - 1.0 / A)   # |X| = |Y| = 0.5
        ratio = delta / (2 * float(np.float32(0.05)))
        expected = 1 - (1 - 0.99 * float(np.float32(alpha))) ** ratio
        assert abs(img[0, 16, 16] - expected * H.rgb_of(sc)[0]) < 1e-12
        assert abs(expected - 0.99 * alpha) < 2e-3 * alpha + 1e-6


def _hexagon_setup(D=2.0, a=0.3):
    n_hat = np.ones(3) / math.sqrt(3.0)
    R = H.rotation_taking(n_hat, [0, 0, 1])          # local (1,1,1) -> camera z
    q = H.rotation_to_quat(R)
    return R, q, D, a


def _hexagon_chord(p0, a):
    """Chord of |x|_1 <= a along (1,1,1)/sqrt3 through p0 (sum p0 = 0).

    With u = s/sqrt3, f(u) = sum_k |p_k + u| is u - 2 p_min between the
    middle and the smallest breakpoint and 2 p_max - u between the largest
    and the middle one, 3|u| outside; solving f = a on each side gives
    u_hi = min(a/3, a + 2 p_min), u_lo = max(-a/3, 2 p_max - a).  Inside
    the inner hexagon (max |p_k| <= a/3) this is the plateau 2a/sqrt3."""
    hi = min(a / 3.0, a + 2.0 * p0.min())
    lo = max(-a / 3.0, 2.0 * p0.max() - a)
    return math.sqrt(3.0) * max(0.0, hi - lo)


def test_hexagon_formula_by_line_sampling():
    """The hexagon chord formula itself, by brute-force sampling of |x|_1 <= a."""
    rng = np.random.default_rng(3)
    a = 0.3
    n_hat = np.ones(3) / math.sqrt(3)
    s = np.linspace(-1, 1, 400001)
    for _ in range(40):
        p = rng.normal(size=3) * 0.15
        p -= p.dot(n_hat) * n_hat
        inside = np.abs(p[None, :] + s[:, None] * n_hat[None, :]).sum(1) <= a
        approx = inside.sum() * (s[1] - s[0])
        assert abs(approx - _hexagon_chord(p, a)) < 2e-5


def test_hexagon_closed_form(oracle_mod):
    """P3: regular octahedron with a 3-fold axis along the view."""
    W = H_ = 64
    cam = H.origin_camera(W, H_)
    f = float(cam.fx)
    R, q, D, a = _hexagon_setup()
    q32 = np.asarray(q, np.float32)
    Rq = H.quat_to_matrix(q32.astype(np.float64))  # the rotation the float32 quaternion encodes
    a32 = float(np.float32(a))
    sc = H.prims(OCTA, [0, 0, D], q32, [a, a, a], 0.5)
    O = oracle_mod.OracleScene(sc, [cam])
    worst = 0.0
    plateau = 0
    for j in range(H_):
        for i in range(W):
            X, Y = i + 0.5 - W / 2, j + 0.5 - H_ / 2
            # the viewing line in the octahedron frame: p0 + s n_loc, with
            # p0 orthogonal to n_loc (= (1,1,1)/sqrt3 up to float32 rounding)
            p0 = Rq.T @ np.array([X * D / f, Y * D / f, 0.0])
            n_loc = Rq.T @ np.array([0, 0, 1.0])
            expect = _hexagon_chord_general(p0, n_loc, a32)
            ideal = _hexagon_chord(p0, a32)
            assert abs(expect - ideal) < 1e-6
            got = O.chord(0, 0, i + 0.5, j + 0.5)
            worst = max(worst, abs(got - expect))
            plateau += abs(got - 2 * a32 / math.sqrt(3)) < 1e-12
    assert worst < 1e-9
    assert plateau > 10
    # footprint area: sqrt(3) (f a / D)^2 pixels
    r = O.render(mode="tiled")
    hit = (r["T"] < 1.0).sum()
    assert abs(hit - math.sqrt(3) * (f * a32 / D) ** 2) < 0.05 * hit
    # plateau opacity 1 - (1 - 0.99 alpha)^(1/sqrt 3)
    sigma = -math.log(1 - 0.99 * 0.5) / (2 * a32)
    o_plateau = 1 - math.exp(-sigma * 2 * a32 / math.sqrt(3))
    assert abs(o_plateau - (1 - (1 - 0.99 * 0.5) ** (1 / math.sqrt(3)))) < 1e-15
    assert abs(o_plateau - 0.3259452) < 1e-7


def _hexagon_chord_general(p0, n_loc, a):
    """Chord of |x|_1 <= a along direction n_loc through p0 (exact, by
    breakpoints), used when the float32 quaternion is not exactly the ideal
    3-fold rotation."""
    # along x(s) = p0 + s n, f(s) = sum |p0_k + s n_k| is convex piecewise linear
    bps = sorted(-p0[k] / n_loc[k] for k in range(3) if n_loc[k] != 0)
    f = lambda s: np.abs(p0 + s * n_loc).sum()
    cand = [(f(s), s) for s in bps]
    fmin, smin = min(cand)
    if fmin > a:
        return 0.0
    slope_inf = np.abs(n_loc).sum()

    def walk(direction):
        s0, f0 = smin, fmin
        pts = [s for s in bps if (s - smin) * direction > 0]
        pts.sort(key=lambda s: direction * s)
        for s1 in pts:
            f1 = f(s1)
            if f1 > a:
                return s0 + (a - f0) * (s1 - s0) / (f1 - f0)
            s0, f0 = s1, f1
        return s0 + direction * (a - f0) / slope_inf

    return walk(+1) - walk(-1)


def test_volume_invariant(oracle_mod):
    """P4: summing the chord over pixels integrates the ray-space volume,
    |det J| times the world volume, for any rotation and both types."""
    rng = np.random.default_rng(5)
    W, H_ = 256, 256
    cam = H.origin_camera(W, H_)
    for kind in (OCTA, TETRA):
        for _ in range(3):
            q = rng.normal(size=4)
            mu = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), 3.0])
            nd = 3 if kind == OCTA else 4
            d = rng.uniform(0.4, 0.7, size=nd)
            sc = H.prims(kind, mu, q, d, 0.5)
            O = oracle_mod.OracleScene(sc, [cam])
            total = 0.0
            p = O.prep()
            i0, j0, i1, j1 = p["rect"][0]
            for j in range(j0, j1 + 1):
                for i in range(i0, i1 + 1):
                    total += O.chord(0, 0, i + 0.5, j + 0.5)
            mu64 = sc.means[0].astype(np.float64)
            J = H.ewa_jacobian_fd(cam, mu64)
            Rq = H.quat_to_matrix(sc.quats[0].astype(np.float64))
            d64 = sc.dists[0].astype(np.float64)
            if kind == OCTA:
                vol = 4.0 / 3.0 * np.prod(d64)
            else:
                B = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]) / math.sqrt(3)
                V = (Rq @ (B * d64[:, None]).T).T
                vol = abs(np.linalg.det(np.stack([V[1] - V[0], V[2] - V[0], V[3] - V[0]]))) / 6
            expect = abs(np.linalg.det(J)) * vol
            assert abs(total - expect) < 2e-3 * expect, (kind, total, expect)


def test_transmittance_product_and_termination(oracle_mod):
    """P5: primitives stacked on the axis composite as the textbook product
    C = sum rgb_k o_k prod_{j<k}(1-o_j), stopping after T <= 1e-3."""
    W = H_ = 16
    cam = H.origin_camera(W, H_)
    f = float(cam.fx)
    depths = [2.0, 2.6, 3.2, 3.8, 4.4, 5.0, 5.6]
    alphas = [0.9, 0.8, 0.95, 0.9, 0.99, 0.9, 0.9]
    cols = [(0.9, 0.1, 0.1), (0.1, 0.9, 0.1), (0.1, 0.1, 0.9), (0.5, 0.5, 0.5), (0.2, 0.7, 0.4),
            (0.6, 0.3, 0.9), (0.3, 0.3, 0.3)]
    n = len(depths)
    sc = H.prims(OCTA, [[0, 0, z] for z in depths], [1, 0, 0, 0], [1.0, 1.0, 0.25], alphas)
    sc.sh[:] = H.sh_for_rgb(cols[0], n)
    for k in range(n):
        sc.sh[k] = H.sh_for_rgb(cols[k])[0]
    bg = np.array([0.2, 0.3, 0.4])
    O = oracle_mod.OracleScene(sc, [cam], tile=16)
    r = O.render(bg=bg)
    img = r["rgb"].reshape(3, H_, W)
    i = j = 8
    X = Y = 0.5
    T, C, last_k = 1.0, np.zeros(3), None
    c32 = float(np.float32(0.25))
    for k in range(n):
        A = f / float(np.float32(depths[k]))
        delta = 2 * c32 * (1 - X / A - Y / A)
        sigma = -math.log(1 - 0.99 * float(np.float32(alphas[k]))) / (2 * c32)
        o = min(0.99, 1 - math.exp(-sigma * delta))
        rgb_k = H.rgb_of(sc, k)
        C += T * o * rgb_k
        T *= 1 - o
        last_k = k
        if T <= 1e-3:
            break
    assert last_k < n - 1, "the stack must terminate early for this test"
    C += T * bg
    np.testing.assert_allclose(img[:, j, i], C, atol=1e-12)
    assert abs(r["T"][j * W + i] - T) < 1e-15
    assert r["last"][j * W + i] == last_k + 1          # one tile: list starts at 0
    assert r["counts"][0, 0] > 0


def test_opaque_full_screen(oracle_mod):
    """P6: alpha = 1 and a chord of at least twice the smallest distance at
    every pixel clamp the opacity to 0.99: C = 0.99 rgb + 0.01 bg everywhere."""
    W = H_ = 32
    cam = H.origin_camera(W, H_)
    sc = H.prims(OCTA, [0, 0, 1.0], [1, 0, 0, 0], [1.5, 1.5, 15.0], 1.0, rgb=(0.7, 0.2, 0.9))
    bg = np.array([0.1, 0.6, 0.3])
    r = oracle_mod.OracleScene(sc, [cam]).render(bg=bg)
    img = r["rgb"].reshape(3, -1)
    rgb = H.rgb_of(sc)
    expect = 0.99 * rgb + 0.01 * bg
    np.testing.assert_allclose(img, np.repeat(expect[:, None], W * H_, 1), atol=1e-12)
    assert abs(img.sum() - W * H_ * expect.sum()) < 1e-9


# ------------------------------------------- independent formulations
@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_mtia_chord_equals_clipping_chord(oracle_mod, kind):
    """P7: per-face MTIA and L1-ball / barycentric clipping give one chord."""
    rng = np.random.default_rng(11)
    sc = (scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra)(64, seed=2, dmin=0.1,
                                                                                   dmax=0.4)
    cam = H.origin_camera(96, 96)
    sc.means[:, 2] += 3.0
    O = oracle_mod.OracleScene(sc, [cam])
    p = O.prep()
    hits = 0
    for n in np.nonzero(p["valid"])[0]:
        i0, j0, i1, j1 = p["rect"][n]
        for _ in range(30):
            px, py = rng.uniform(i0, i1 + 1), rng.uniform(j0, j1 + 1)
            a = O.chord(0, n, px, py, "mtia")
            b = O.chord(0, n, px, py, "clip")
            scale = 2 * sc.dists[n].max()
            assert abs(a - b) < 1e-9 * scale, (n, px, py, a, b)
            hits += a > 0
    assert hits > 500


@pytest.mark.parametrize("kind", [OCTA, TETRA])
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_brute_force_equals_tiled(oracle_mod, kind, tile):
    """P8: the tiled pipeline reaches exactly the per-pixel definition."""
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(400, seed=4, dmin=0.03, dmax=0.2)
    cam = scenes.look_at((0.3, -0.2, -3.5), (0, 0, 0), 80, 56)
    O = oracle_mod.OracleScene(sc, [cam], tile=tile)
    bg = np.array([0.3, 0.1, 0.2])
    a = O.render(bg=bg, mode="tiled")
    b = O.render(bg=bg, mode="brute")
    np.testing.assert_array_equal(a["rgb"], b["rgb"])
    np.testing.assert_array_equal(a["T"], b["T"])
    assert (a["T"] < 1).mean() > 0.1


def test_image_independent_of_tile_size(oracle_mod):
    sc = scenes.uniform_octahedra(300, seed=6)
    cam = scenes.look_at((0, 0, -3), (0, 0, 0), 72, 40)
    imgs = [oracle_mod.OracleScene(sc, [cam], tile=t).render()["rgb"] for t in (8, 16, 32)]
    np.testing.assert_array_equal(imgs[0], imgs[1])
    np.testing.assert_array_equal(imgs[0], imgs[2])


# ------------------------------------------------------- sort (P12)
def test_sort_matches_python_stable_sort(oracle_mod):
    sc = scenes.uniform_octahedra(500, seed=8, dmin=0.05, dmax=0.3)
    cams = [scenes.look_at((0, 0, -3), (0, 0, 0), 64, 48), scenes.look_at((3, 0, 0), (0, 0, 0), 40, 40)]
    tile = 8
    O = oracle_mod.OracleScene(sc, cams, tile=tile)
    s = O.sort()
    pairs = []
    base = 0
    for v, cam in enumerate(cams):
        p = O.prep(v)
        tx = (cam.width + tile - 1) // tile
        ty = (cam.height + tile - 1) // tile
        for n in range(sc.n):
            if not p["valid"][n]:
                continue
            i0, j0, i1, j1 = p["rect"][n]
            for y in range(j0 // tile, j1 // tile + 1):
                for x in range(i0 // tile, i1 // tile + 1):
                    pairs.append((((base + y * tx + x) << 32) | int(p["key"][n]), n))
        base += tx * ty
    pairs.sort(key=lambda kv: kv[0])                 # Python's sort is stable
    np.testing.assert_array_equal(s["keys"], np.array([k for k, _ in pairs], np.uint64))
    np.testing.assert_array_equal(s["values"], np.array([v for _, v in pairs], np.uint32))
    tiles = (s["keys"] >> np.uint64(32)).astype(np.int64)
    for t in range(base):
        idx = np.nonzero(tiles == t)[0]
        if idx.size:
            assert s["ranges"][t, 0] == idx[0] and s["ranges"][t, 1] == idx[-1] + 1
        else:
            assert s["ranges"][t, 0] == s["ranges"][t, 1]


def test_depth_key_is_float32_camera_z(oracle_mod):
    sc = scenes.uniform_octahedra(200, seed=9)
    cam = scenes.look_at((1.0, 0.5, -3), (0, 0, 0), 64, 64)
    O = oracle_mod.OracleScene(sc, [cam])
    p = O.prep()
    Rw = cam.world_to_cam.astype(np.float64)
    m = sc.means.astype(np.float64)
    z = ((Rw[2, 0] * m[:, 0] + Rw[2, 1] * m[:, 1]) + Rw[2, 2] * m[:, 2]) + Rw[2, 3]
    keys = z.astype(np.float32).view(np.uint32)
    v = p["valid"]
    np.testing.assert_array_equal(p["key"][v], keys[v])
    np.testing.assert_allclose(p["tc"][v, 2], z[v], rtol=0, atol=0)


def test_rectangle_is_pixel_centres_in_projected_box(oracle_mod):
    """The pixel rectangle holds exactly the pixel centres inside the box of
    the corners mapped by the EWA map linearised at the centre."""
    sc = scenes.uniform_octahedra(150, seed=12, dmin=0.05, dmax=0.3)
    cam = scenes.look_at((0.4, 0.2, -3), (0, 0, 0), 100, 70)
    O = oracle_mod.OracleScene(sc, [cam])
    p = O.prep()
    Rw = cam.world_to_cam[:, :3].astype(np.float64)
    t = cam.world_to_cam[:, 3].astype(np.float64)
    for n in range(sc.n):
        mu = sc.means[n].astype(np.float64)
        tc = Rw @ mu + t
        if tc[2] <= 0.2:
            assert not p["valid"][n]
            continue
        J = H.ewa_jacobian_fd(cam, tc)
        R = H.quat_to_matrix(sc.quats[n].astype(np.float64))
        d = sc.dists[n].astype(np.float64)
        offs = [R[:, k] * d[k] * s for k in range(3) for s in (1, -1)]
        pts = np.array([H.ewa_map(cam, tc) + J @ (Rw @ o) for o in offs])
        xs = np.arange(cam.width) + 0.5
        ys = np.arange(cam.height) + 0.5
        inx = np.nonzero((xs >= pts[:, 0].min() - 1e-7) & (xs <= pts[:, 0].max() + 1e-7))[0]
        iny = np.nonzero((ys >= pts[:, 1].min() - 1e-7) & (ys <= pts[:, 1].max() + 1e-7))[0]
        if inx.size == 0 or iny.size == 0:
            assert not p["valid"][n]
            continue
        assert p["valid"][n]
        assert tuple(p["rect"][n]) == (inx[0], iny[0], inx[-1], iny[-1]), n


def test_culling_of_degenerate_primitives(oracle_mod):
    cam = H.origin_camera(32, 32)
    sc = H.prims(OCTA, [[0, 0, 2], [0, 0, 0.1], [0, 0, 2], [0, 0, 2], [0, 0, 2], [0, 0, 2]],
                 [1, 0, 0, 0], [0.1, 0.1, 0.1], 0.5)
    sc.quats[2] = 0.0                        # zero quaternion
    sc.dists[3, 1] = 0.0                     # non-positive distance
    sc.means[4, 0] = np.nan                  # non-finite centre
    sc.means[5, 0] = 100.0                   # entirely off screen
    p = oracle_mod.OracleScene(sc, [cam]).prep()
    assert list(p["valid"]) == [True, False, False, False, False, False]
