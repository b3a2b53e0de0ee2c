"""Depth map of the forward pass (appendix "Depth and Surface
Reconstruction") vs the FP64 oracle, through the C ABI (MI355X only).

The depth is the distance along the pixel ray to the entry of the first
primitive at which cumulative opacity exceeds 0.5.  Which pixels have a
depth is compared exactly, and the distance within 1e-5 relative (a float32
plane evaluation), on every pixel the oracle does not flag (a step ending
within 1e-6 of 0.5, or a value-ill pixel)."""
import sys

import numpy as np
import pytest
import torch

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


DEPTH_TOL = 1e-5   # relative, floor 1 world unit


def _check_depth(depth, ref, ok, label):
    got = depth.astype(np.float64)
    assert np.array_equal(got[ok] > 0, ref[ok] > 0)
    err = np.abs(got - ref) / np.maximum(ref, 1.0)
    _say(f"  [{label}] depth max rel err {err[ok].max(initial=0.0):.3e} (all pixels {err.max(initial=0.0):.3e})")
    assert err[ok].max(initial=0.0) <= DEPTH_TOL


def _gpu_depth(sc, cams, tile, bg, exact=False):
    g = GC.gpu_forward(sc, cams, tile=tile, bg=bg, exact=exact)
    rast, prims = g["rast"], g["prims"]
    depth = torch.full((rast.n_pixels,), -1.0, dtype=torch.float32, device="cuda")
    rgb, T, last = rast.render(prims, bg, depth=depth)
    torch.cuda.synchronize()
    return g, depth.cpu().numpy(), rgb.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("kind", [OCTA, TETRA])
@pytest.mark.parametrize("tile", [8, 16])
def test_depth_parity(oracle_mod, kind, tile, exact):
    _say(f"depth kind={kind} tile={tile} exact={exact}")
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(1500, seed=95 + kind, dmin=0.05, dmax=0.25)
    cams = [scenes.look_at((0.2, 0.1, -3.0), (0, 0, 0), 88, 61), scenes.look_at((2.8, 0.5, 0.6), (0, 0, 0), 45, 37)]
    bg = (0.1, 0.2, 0.3)
    g, depth, rgb, T = _gpu_depth(sc, cams, tile, bg, exact)
    # the depth output leaves the image untouched
    assert np.array_equal(rgb, g["rgb"]) and np.array_equal(T, g["T"])
    d = oracle_mod.OracleScene(sc, cams, tile=tile, exact=exact).render_depth(bg=np.asarray(bg))
    ok = ~d["ill"]
    has = d["depth"] > 0
    _say(f"  covered {has.mean() * 100:.1f}%, flagged {(~ok).mean() * 100:.3f}%")
    assert has.mean() > 0.2 and ok.mean() > 0.999
    _check_depth(depth, d["depth"], ok, f"kind={kind} tile={tile} exact={exact}")
    assert np.all(depth >= 0)


def test_depth_config0(oracle_mod):
    _say("depth config0")
    sc, cams = scenes.config0()
    g, depth, _, _ = _gpu_depth(sc, cams, 16, (0.0, 0.0, 0.0))
    d = oracle_mod.OracleScene(sc, cams, tile=16).render_depth()
    ok = ~d["ill"]
    _check_depth(depth, d["depth"], ok, "config0")
    assert (d["depth"] > 0).mean() > 0.04
