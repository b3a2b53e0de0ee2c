"""Adaptive population control on the GPU (Sec. 3.4; App. G) vs the
oracle, through the C ABI (MI355X only).

Statistics: counts exact, radii to float32 rounding, accumulated gradient
norms within the gradient tolerance on primitives the oracle does not flag.
Densify / prune: the decisions are taken in float32 on both sides from the
same arrays, so the row count and every copied row are exact; split
children's positions and distances within 1e-6 relative."""
import sys

import numpy as np
import pytest
import torch

from oracle import population as POP
from paper_2501_16312_amd import linprim as L
from paper_2501_16312_amd import scenes
from paper_2501_16312_amd.population import PopulationControl
from tests import gpu_common as GC

pytestmark = pytest.mark.gpu

OCTA, TETRA = scenes.OCTAHEDRON, scenes.TETRAHEDRON
FIELDS = ("means", "quats", "dists", "opacity", "sh")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


@pytest.mark.parametrize("kind,tile", [(OCTA, 8), (TETRA, 8), (OCTA, 16), (TETRA, 32)])
def test_stats_parity(oracle_mod, kind, tile):
    """Densification statistics; with 16- and 32-pixel tiles each tile holds
    several 8x8 groups, whose gradient records the slot backward sums."""
    _say(f"stats kind={kind} tile={tile}")
    gen = scenes.uniform_octahedra if kind == OCTA else scenes.uniform_tetrahedra
    sc = gen(600, seed=111 + kind, dmin=0.02, dmax=0.15)
    cams = [scenes.look_at((0.2, 0.1, -3.0), (0, 0, 0), 88, 61), scenes.look_at((2.8, 0.5, 0.6), (0, 0, 0), 45, 37)]
    grad = scenes.image_gradient(cams, seed=12)
    g = GC.gpu_forward(sc, cams, tile=tile)
    GC.gpu_backward(g, grad)
    pc = PopulationControl(kind, sc.sh_degree, sc.n)
    pc.accumulate(g["rast"], g["prims"])
    pc.accumulate(g["rast"], g["prims"])             # a second step adds again
    torch.cuda.synchronize()
    O = oracle_mod.OracleScene(sc, cams, tile=tile)
    rb = O.backward(grad.astype(np.float64))
    acc, cnt, rad = np.zeros(sc.n), np.zeros(sc.n), np.zeros(sc.n)
    POP.accumulate_stats(O, acc, cnt, rad)
    POP.accumulate_stats(O, acc, cnt, rad)
    assert np.array_equal(pc.count.cpu().numpy(), cnt.astype(np.int32))
    np.testing.assert_allclose(pc.max_radius.cpu().numpy(), rad, rtol=1e-6)
    ok = ~rb["ill"]
    a = pc.grad_accum.cpu().numpy().astype(np.float64)
    rms = float(np.sqrt(np.mean(acc[ok] ** 2)))
    err = np.abs(a - acc)[ok] / np.maximum(np.abs(acc[ok]), 1e-2 * rms)
    _say(f"  worst rel err {err.max():.2e} over {ok.sum()} primitives, visible {int((cnt > 0).sum())}")
    assert err.max() <= GC.GRAD_TOL
    assert (cnt > 0).sum() > 100
    assert ok[cnt > 0].mean() >= 0.95


def _random_state(kind, n, seed, K=16):
    rng = np.random.default_rng(seed)
    nd = 3 if kind == OCTA else 4
    params = {"means": rng.normal(size=(n, 3)).astype(np.float32),
              "quats": rng.normal(size=(n, 4)).astype(np.float32),
              "dists": np.exp(rng.uniform(np.log(0.01), np.log(3.0), size=(n, nd))).astype(np.float32),
              "opacity": rng.uniform(0.0, 0.2, size=n).astype(np.float32),
              "sh": rng.normal(size=(n, K, 3)).astype(np.float32)}
    moments = {(w, k): rng.normal(size=params[k].shape).astype(np.float32) for w in ("m", "v") for k in params}
    stats = {"grad_accum": rng.uniform(0, 1.2e-3, size=n).astype(np.float32),
             "count": rng.integers(0, 5, size=n).astype(np.int32),
             "max_radius": rng.uniform(0, 40, size=n).astype(np.float32)}
    normals = rng.normal(size=(n, 2, 3)).astype(np.float32)
    return params, moments, stats, normals


def _run_gpu(kind, params, moments, stats, normals, extent):
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    P = {k: dev(params[k]) for k in FIELDS}
    M = {k: dev(moments[("m", k)]) for k in FIELDS}
    V = {k: dev(moments[("v", k)]) for k in FIELDS}
    pc = PopulationControl(kind, 3, params["means"].shape[0])
    pc.grad_accum.copy_(dev(stats["grad_accum"]))
    pc.count.copy_(dev(stats["count"]))
    pc.max_radius.copy_(dev(stats["max_radius"]))
    newp, newm, newv = pc.densify(P, extent, M, V, normals=dev(normals))
    torch.cuda.synchronize()
    assert pc.n == newp["means"].shape[0] and int(pc.count.sum()) == 0
    return ({k: v.cpu().numpy() for k, v in newp.items()}, {k: v.cpu().numpy() for k, v in newm.items()},
            {k: v.cpu().numpy() for k, v in newv.items()})


def _compare(kind, params, moments, stats, normals, extent):
    gp, gm, gv = _run_gpu(kind, params, moments, stats, normals, extent)
    op, om = POP.densify(kind, params, moments, stats, extent, normals)
    n_out = op["means"].shape[0]
    assert gp["means"].shape[0] == n_out
    d = POP.decide(kind, params["dists"], params["opacity"], stats["grad_accum"], stats["count"],
                   stats["max_radius"], extent)
    _say(f"  n {params['means'].shape[0]} -> {n_out}: kept {d['keep'].sum()}, split {d['split'].sum()}, "
         f"cloned {d['clone'].sum()}")
    for k in ("quats", "opacity", "sh"):
        assert np.array_equal(gp[k].astype(np.float64), op[k]), k
    for k in FIELDS:
        assert np.array_equal(gm[k].astype(np.float64), om[("m", k)]), k
        assert np.array_equal(gv[k].astype(np.float64), om[("v", k)]), k
    for k in ("means", "dists"):
        np.testing.assert_allclose(gp[k], op[k], rtol=1e-6, atol=1e-6, err_msg=k)
    return d


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_densify_random_parity(kind):
    _say(f"densify random kind={kind}")
    params, moments, stats, normals = _random_state(kind, 20000, seed=7 + kind)
    d = _compare(kind, params, moments, stats, normals, extent=10.0)
    for k in ("keep", "split", "clone"):
        assert d[k].sum() > 100, k
    assert (~(d["keep"] | d["split"])).sum() > 100          # some removed


def test_densify_edge_cases():
    _say("densify edges")
    # nothing to do, everything removed, and a single primitive
    params, moments, stats, normals = _random_state(OCTA, 50, seed=3)
    stats["grad_accum"][:] = 0
    params["opacity"][:] = 0.5
    params["dists"][:] = 0.1
    stats["max_radius"][:] = 1
    _compare(OCTA, params, moments, stats, normals, extent=10.0)   # all kept, unchanged
    params["opacity"][:] = 0.0
    _compare(OCTA, params, moments, stats, normals, extent=10.0)   # all removed
    params, moments, stats, normals = _random_state(TETRA, 1, seed=4)
    _compare(TETRA, params, moments, stats, normals, extent=10.0)
