"""HIP path with the 2D anti-aliasing filter (appendix "Anti-Aliasing")
vs the FP64 oracle's filtered ray-space model, through the C ABI (MI355X
only).  Same bars as the unfiltered path."""
import sys

import numpy as np
import pytest

from paper_2501_16312_amd import scenes
from tests import gpu_common as GC

pytestmark = pytest.mark.gpu

OCTA, TETRA = scenes.OCTAHEDRON, scenes.TETRAHEDRON


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


def _scene(kind, n, seed, dmax=0.2):
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    # small primitives too: the filter matters most where a primitive covers few pixels
    return gen(n, seed=seed, dmin=0.005, dmax=dmax)


def _cams():
    return [scenes.look_at((0.2, 0.1, -3.0), (0, 0, 0), 88, 61),
            scenes.look_at((2.8, 0.5, 0.6), (0, 0, 0), 45, 37)]


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_aa_binning_bit_exact(oracle_mod, kind):
    _say(f"aa binning kind={kind}")
    sc = _scene(kind, 800, seed=81)
    cams = _cams()
    g = GC.gpu_forward(sc, cams, tile=8, antialias=True)
    dbg = g["rast"].debug_arrays(g["prims"])
    O = oracle_mod.OracleScene(sc, cams, tile=8, antialias=True)
    grown = 0
    for v in range(len(cams)):
        p = O.prep(v)
        pay = dbg["payload"][v * sc.n:(v + 1) * sc.n].numpy()
        rect = pay[:, :4].view(np.int32)
        assert np.array_equal(rect[p["valid"]], p["rect"][p["valid"]])
        assert np.all(dbg["tiles"][v * sc.n:(v + 1) * sc.n].numpy()[~p["valid"]] == 0)   # culled
        keys = dbg["depth_keys"][v * sc.n:(v + 1) * sc.n].numpy().view(np.uint32)
        assert np.array_equal(keys[p["valid"]], p["key"][p["valid"]])
        plain = oracle_mod.OracleScene(sc, [cams[v]], tile=8).prep()
        grown += int((p["valid"] & ~plain["valid"]).sum() + (p["tiles"] > plain["tiles"]).sum())
    s = O.sort()
    assert g["n_pairs"] == len(s["keys"])
    assert np.array_equal(dbg["keys"].numpy().view(np.uint64), s["keys"])
    assert np.array_equal(dbg["values"].numpy().view(np.uint32), s["values"])
    _say(f"  primitives whose footprint the filter grows into more tiles or into view: {grown}")
    assert grown > 0


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_aa_forward_parity(oracle_mod, kind):
    _say(f"aa forward kind={kind}")
    sc = _scene(kind, 900, seed=83)
    cams = _cams()
    bg = (0.1, 0.2, 0.3)
    g = GC.gpu_forward(sc, cams, tile=16, bg=bg, antialias=True)
    r = oracle_mod.OracleScene(sc, cams, tile=16, antialias=True).render(bg=np.asarray(bg))
    r["cams"] = cams
    GC.compare_images(g, r, f"aa kind={kind}")
    GC.compare_last(g, r, f"aa kind={kind}")
    plain = GC.gpu_forward(sc, cams, tile=16, bg=bg)
    assert np.abs(plain["rgb"] - g["rgb"]).max() > 1e-3


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_aa_backward_parity(oracle_mod, kind):
    _say(f"aa backward kind={kind}")
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(500, seed=85, dmin=0.01, dmax=0.12)
    cams = _cams()
    bg = (0.3, 0.1, 0.2)
    grad = scenes.image_gradient(cams, seed=8)
    g = GC.gpu_forward(sc, cams, tile=8, bg=bg, antialias=True)
    gg = GC.gpu_backward(g, grad, bg)
    rb = oracle_mod.OracleScene(sc, cams, tile=8, antialias=True).backward(grad.astype(np.float64),
                                                                            bg=np.asarray(bg))
    ok = ~rb["ill"]
    _say(f"  prims ill {rb['ill'].mean() * 100:.2f}%")
    w = GC.grad_errors(gg, rb, ok, f"aa kind={kind}")
    for k, v in w.items():
        assert v <= GC.GRAD_TOL, k


def test_aa_with_exact_rays_rejected():
    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd.render import Rasterizer
    with pytest.raises(L.LinPrimError):
        Rasterizer(OCTA, 10, _cams(), tile=8, exact=True, antialias=True)
