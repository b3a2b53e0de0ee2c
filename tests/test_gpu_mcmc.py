"""LinPrim-MCMC's relocation and noise steps on the GPU vs the oracle,
through the C ABI (MI355X only).  The draws are integer decisions taken
from the same 32-bit random numbers on both sides, so the sources and the
relocated slots are exact; updated opacities and distances within 1e-6
relative; the noise within 1e-5 relative."""
import sys

import numpy as np
import pytest
import torch

from oracle import mcmc as MC
from paper_2501_16312_amd import linprim as L
from paper_2501_16312_amd.population import MCMC

pytestmark = pytest.mark.gpu
FIELDS = ("means", "quats", "dists", "opacity", "sh")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _state(n, seed, dead_frac=0.1):
    rng = np.random.default_rng(seed)
    op = rng.uniform(0.006, 1.0, size=n).astype(np.float32)
    op[rng.random(n) < dead_frac] = rng.uniform(0, 0.005, size=1).astype(np.float32)[0]
    params = {"means": rng.normal(size=(n, 3)).astype(np.float32),
              "quats": rng.normal(size=(n, 4)).astype(np.float32),
              "dists": np.exp(rng.uniform(-4, -1, size=(n, 3))).astype(np.float32),
              "opacity": op, "sh": rng.normal(size=(n, 16, 3)).astype(np.float32)}
    moments = {(w, k): rng.normal(size=params[k].shape).astype(np.float32) for w in ("m", "v") for k in params}
    r = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    return params, moments, r


def _gpu_relocate(params, moments, r):
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    P = {k: dev(params[k]) for k in FIELDS}
    M = {k: dev(moments[("m", k)]) for k in FIELDS}
    V = {k: dev(moments[("v", k)]) for k in FIELDS}
    mc = MCMC(params["means"].shape[0])
    mc.relocate(P, M, V, rand_u32=dev(r.view(np.int32)))
    nd = mc.dead_count()
    torch.cuda.synchronize()
    return ({k: v.cpu().numpy() for k, v in P.items()}, {k: v.cpu().numpy() for k, v in M.items()},
            {k: v.cpu().numpy() for k, v in V.items()}, nd)


@pytest.mark.parametrize("n", [20000, 3])
def test_relocate_parity(n):
    _say(f"mcmc relocate n={n}")
    params, moments, r = _state(n, seed=n)
    gp, gm, gv, nd = _gpu_relocate(params, moments, r)
    op, om, ond = MC.relocate(params, moments, r)
    assert nd == ond
    _say(f"  dead {nd}")
    for k in ("means", "quats", "sh"):
        assert np.array_equal(gp[k].astype(np.float64), op[k]), k
    for k in ("dists", "opacity"):
        np.testing.assert_allclose(gp[k], op[k], rtol=1e-6, err_msg=k)
    for k in FIELDS:
        assert np.array_equal(gm[k].astype(np.float64), om[("m", k)]), k
        assert np.array_equal(gv[k].astype(np.float64), om[("v", k)]), k


def test_relocate_edges():
    _say("mcmc edges")
    params, moments, r = _state(100, seed=5, dead_frac=0.0)
    gp, _, _, nd = _gpu_relocate(params, moments, r)
    assert nd == 0 and np.array_equal(gp["opacity"], params["opacity"])
    params["opacity"][:] = 0.001                                   # nothing alive: nothing moves
    gp, _, _, nd = _gpu_relocate(params, moments, r)
    assert nd == 100 and np.array_equal(gp["means"], params["means"])


def test_noise_parity():
    _say("mcmc noise")
    params, _, _ = _state(5000, seed=9, dead_frac=0.3)
    rng = np.random.default_rng(10)
    eps = rng.normal(size=(5000, 3)).astype(np.float32)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    P = {k: dev(params[k]) for k in FIELDS}
    MCMC(5000).noise(P, 1e-4, normals=dev(eps))
    torch.cuda.synchronize()
    ref = MC.noise(params, eps, lr_means=float(np.float32(1e-4)))
    got = P["means"].cpu().numpy().astype(np.float64)
    moved = np.abs(ref - params["means"]).max(1) > 1e-6
    assert moved.sum() > 100
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-6)


def test_tetrahedra_rejected():
    st = L.state({k: torch.zeros((1, 4 if k in ("quats", "dists") else 3), device="cuda") for k in FIELDS})
    ws = torch.empty(L.linprim_mcmc_workspace_size(1), dtype=torch.uint8, device="cuda")
    with pytest.raises(L.LinPrimError):
        L.linprim_mcmc_relocate(L.TETRAHEDRON, 3, 1, st, torch.zeros(1, dtype=torch.int32, device="cuda"), ws)


def test_add_parity():
    _say("mcmc add")
    n, n_add = 8000, 400
    params, moments, r = _state(n, seed=21)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    P = {k: dev(params[k]) for k in FIELDS}
    M = {k: dev(moments[("m", k)]) for k in FIELDS}
    V = {k: dev(moments[("v", k)]) for k in FIELDS}
    mc = MCMC(n)
    newp, newm, newv = mc.add(P, n_add, M, V, rand_u32=dev(r[:n_add].view(np.int32)))
    torch.cuda.synchronize()
    op, om = MC.add(params, moments, n_add, r[:n_add])
    assert mc.n == n + n_add and newp["means"].shape[0] == n + n_add
    for k in ("means", "quats", "sh"):
        assert np.array_equal(newp[k].cpu().numpy().astype(np.float64), op[k]), k
    for k in ("dists", "opacity"):
        np.testing.assert_allclose(newp[k].cpu().numpy(), op[k], rtol=1e-6, err_msg=k)
    for k in FIELDS:
        assert np.array_equal(newm[k].cpu().numpy().astype(np.float64), om[("m", k)]), k
        assert np.array_equal(newv[k].cpu().numpy().astype(np.float64), om[("v", k)]), k
