"""The allocation-free densify entry point (linprim_densify_noalloc) against
the plan + apply pair with a caller workspace, through the C ABI: identical
outputs on two calls in a row, the second with fewer primitives, and the
size checks (MI355X only)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2501_16312_amd import linprim as L
from paper_2501_16312_amd import scenes

pytestmark = pytest.mark.gpu

OCTA, TETRA = scenes.OCTAHEDRON, scenes.TETRAHEDRON
FIELDS = L.FIELDS


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _random_state(kind, n, seed, K=16):
    rng = np.random.default_rng(seed)
    nd = 3 if kind == OCTA else 4
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    params = {"means": rng.normal(size=(n, 3)), "quats": rng.normal(size=(n, 4)),
              "dists": np.exp(rng.uniform(np.log(0.01), np.log(3.0), size=(n, nd))),
              "opacity": rng.uniform(0.0, 0.2, size=n), "sh": rng.normal(size=(n, K, 3))}
    params = {k: dev(v.astype(np.float32)) for k, v in params.items()}
    m = {k: dev(rng.normal(size=tuple(v.shape)).astype(np.float32)) for k, v in params.items()}
    v = {k: dev(rng.uniform(0, 1, size=tuple(t.shape)).astype(np.float32)) for k, t in params.items()}
    stats = {"grad_accum": dev(rng.uniform(0, 1.2e-3, size=n).astype(np.float32)),
             "count": dev(rng.integers(0, 5, size=n).astype(np.int32)),
             "max_radius": dev(rng.uniform(0, 40, size=n).astype(np.float32))}
    normals = dev(rng.normal(size=(n, 2, 3)).astype(np.float32))
    return params, m, v, stats, normals


def _outputs(params, rows):
    new = {k: torch.full((rows,) + tuple(params[k].shape[1:]), -5.0, dtype=torch.float32, device="cuda")
           for k in FIELDS}
    return new, {k: torch.full_like(t, -6.0) for k, t in new.items()}, {k: torch.full_like(t, -7.0)
                                                                        for k, t in new.items()}


def _with_workspace(kind, n, params, m, v, stats, normals, dp):
    ws = torch.empty(max(L.linprim_densify_workspace_size(n), 1), dtype=torch.uint8, device="cuda")
    n_out = L.linprim_densify_plan(kind, params["dists"], params["opacity"], stats["grad_accum"], stats["count"],
                                   stats["max_radius"], dp, ws)
    new, nm, nv = _outputs(params, n_out)
    L.linprim_densify_apply(kind, 3, n, L.state(params, m, v), normals, stats["grad_accum"], stats["count"],
                            stats["max_radius"], dp, ws, L.state(new, nm, nv), n_out)
    torch.cuda.synchronize()
    return n_out, new, nm, nv


def _no_alloc(kind, n, params, m, v, stats, normals, dp):
    rows = 3 * n
    new, nm, nv = _outputs(params, rows)
    n_out = L.linprim_densify_noalloc(kind, 3, n, L.state(params, m, v), normals, stats["grad_accum"],
                                      stats["count"], stats["max_radius"], dp, L.state(new, nm, nv), rows)
    torch.cuda.synchronize()
    return n_out, new, nm, nv


@pytest.mark.parametrize("kind", [OCTA, TETRA])
def test_noalloc_matches_workspace_entry_points(kind):
    dp = L.densify_params(10.0)
    for call, n in enumerate((20000, 1500)):           # the second call is smaller
        _say(f"densify without allocation kind={kind} call={call} n={n}")
        params, m, v, stats, normals = _random_state(kind, n, seed=31 + 10 * call + kind)
        a = _with_workspace(kind, n, params, m, v, stats, normals, dp)
        b = _no_alloc(kind, n, params, m, v, stats, normals, dp)
        assert a[0] == b[0] and a[0] > n // 2, (a[0], b[0])
        n_out = a[0]
        for ta, tb in zip(a[1:], b[1:]):
            for k in FIELDS:
                assert torch.equal(ta[k], tb[k][:n_out]), (call, k)
                assert torch.all(tb[k][n_out:] == tb[k][n_out:].flatten()[0]).item()   # rows past n_out untouched


def test_noalloc_size_checks():
    _say("densify without allocation: size checks")
    dp = L.densify_params(10.0)
    params, m, v, stats, normals = _random_state(OCTA, 256, seed=5)
    params["opacity"].fill_(0.5)
    stats["grad_accum"].fill_(1.0)
    stats["count"].fill_(1)
    stats["max_radius"].fill_(1.0)
    params["dists"].fill_(0.01)                          # all cloned: 512 rows after the pass
    new, nm, nv = _outputs(params, 300)
    lib = L.load()
    out = ctypes.c_int64(0)
    src, dst = L.state(params, m, v), L.state(new, nm, nv)
    rc = lib.linprim_densify_noalloc(OCTA, 3, 256, ctypes.byref(src), L._ptr(normals), L._ptr(stats["grad_accum"]),
                                     L._ptr(stats["count"]), L._ptr(stats["max_radius"]), ctypes.byref(dp),
                                     ctypes.byref(dst), 300, ctypes.byref(out), None)
    torch.cuda.synchronize()
    assert rc == L.ERR_WORKSPACE and out.value == 512
    assert torch.all(new["means"] == -5.0).item()     # dst untouched
    # more primitives than the scratch covers: rejected before any work
    rc = lib.linprim_densify_noalloc(OCTA, 3, L.NOALLOC_MAX_PRIMS + 1, ctypes.byref(src), L._ptr(normals),
                                     L._ptr(stats["grad_accum"]), L._ptr(stats["count"]),
                                     L._ptr(stats["max_radius"]), ctypes.byref(dp), ctypes.byref(dst), 300,
                                     ctypes.byref(out), None)
    assert rc == L.ERR_WORKSPACE
