"""Fixtures under tests/golden: the paper's stated constants (behaviourally
checked against the oracle) and a regression record of the oracle itself."""
import json
import math
import os

import numpy as np

from paper_2501_16312_amd import scenes
from tests import helpers as H

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_paper_constants_in_behaviour(oracle_mod):
    C = _load("paper_constants.json")
    # Eq. 1 scale: a chord equal to twice the smallest distance at alpha gives
    # 1 - (1 - 0.99 alpha) (principal point pixel of a very wide primitive).
    cam = H.origin_camera(32, 32)
    sc = H.prims(0, [0, 0, 3.0], [1, 0, 0, 0], [1e4, 1e4, 0.05], 0.5, rgb=(1, 1, 1))
    img = oracle_mod.OracleScene(sc, [cam]).render()["rgb"].reshape(3, 32, 32)
    k = C["density_alpha_scale"]["value"]
    assert abs(img[0, 16, 16] / H.rgb_of(sc)[0] - k * 0.5) < 1e-5
    # termination at cumulative opacity 0.999: two opaque layers (o = 0.99
    # each) bring T to 1e-4 and the third layer is never blended
    stop = 1.0 - C["termination_cumulative_opacity"]["value"]
    # (each layer is far wider than the 8x8 view and ten times deeper than
    # wide, so its chord exceeds twice its smallest distance at every pixel)
    cam = H.origin_camera(8, 8)
    sc = H.prims(0, [[0, 0, 2.0], [0, 0, 3.0], [0, 0, 4.0]], [1, 0, 0, 0], [20.0, 20.0, 200.0], 1.0)
    r = oracle_mod.OracleScene(sc, [cam]).render()
    assert r["T"].max() <= stop and abs(r["T"][0] - 1e-4) < 1e-12
    assert np.all(r["last"] == 2)
    # tile size used by the paper's measurements is accepted and bins 16 px
    O = oracle_mod.OracleScene(scenes.uniform_octahedra(50, seed=1), [scenes.look_at((0, 0, -3), (0, 0, 0), 64, 32)],
                               tile=C["tile_size_px"]["value"])
    assert O.sort()["ranges"].shape[0] == (64 // 16) * (32 // 16)
    assert C["sh_coefficients_per_primitive"]["value"] == 16 * 3


def test_oracle_regression_config0(oracle_mod):
    G = _load("oracle_config0.json")
    sc, cams = scenes.config0()
    O = oracle_mod.OracleScene(sc, cams, tile=16)
    r = O.render()
    pix = np.array(G["pixels"])
    rgb = np.stack([r["rgb"][c * 16384 + pix] for c in range(3)], 1)
    np.testing.assert_allclose(rgb, np.array(G["rgb"]), rtol=0, atol=1e-13)
    np.testing.assert_allclose(r["T"][pix], np.array(G["T"]), rtol=0, atol=1e-13)
    assert [int(x) for x in r["counts"][0][:4]] == G["counts"]
    assert math.isclose(r["rgb"].sum(), G["image_sum"], rel_tol=1e-12)
    g = scenes.image_gradient(cams, seed=1).astype(np.float64)
    b = O.backward(g)
    prims = np.array(G["prims"])
    np.testing.assert_allclose(b["means"][prims], np.array(G["grad_means"]), rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(b["opacity"][prims], np.array(G["grad_opacity"]), rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(b["sh"][prims, 0], np.array(G["grad_sh00"]), rtol=1e-10, atol=1e-13)
