"""Adaptive population control over the C ABI (Sec. 3.4 "Adaptive
Population Control"; thresholds in App. G): statistics accumulated after
every backward pass, and a densify / prune pass that returns new parameter
and Adam-moment tensors.  Argument marshalling only; the work runs in
csrc/k_population.hip and the statistics come from the preprocessing
backward kernels."""
from __future__ import annotations

from typing import Optional

import torch

from . import linprim as L


class PopulationControl:
    def __init__(self, kind: int, sh_degree: int, n: int, device: str = "cuda", **thresholds):
        self.kind, self.sh_degree = int(kind), int(sh_degree)
        self.device = torch.device(device)
        self.thresholds = thresholds
        self.reset(n)

    def reset(self, n: int):
        self.n = int(n)
        self.grad_accum = torch.zeros(self.n, dtype=torch.float32, device=self.device)
        self.count = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        self.max_radius = torch.zeros(self.n, dtype=torch.float32, device=self.device)

    def accumulate(self, rast, prims: L.Prims):
        """After rast.backward(...) on these primitives."""
        L.linprim_accumulate_stats(prims, rast.cams_c, rast.tune, rast.view_ws, self.grad_accum, self.count,
                                   self.max_radius)

    def densify(self, params: dict, extent: float, exp_avg: Optional[dict] = None,
                exp_avg_sq: Optional[dict] = None, normals: Optional[torch.Tensor] = None,
                generator: Optional[torch.Generator] = None):
        """Returns (params, exp_avg, exp_avg_sq) after the pass (new tensors;
        moments None if none were given) and resets the statistics."""
        dp = L.densify_params(extent, **self.thresholds)
        n = self.n
        ws = torch.empty(max(L.linprim_densify_workspace_size(n), 1), dtype=torch.uint8, device=self.device)
        n_out = L.linprim_densify_plan(self.kind, params["dists"], params["opacity"], self.grad_accum, self.count,
                                       self.max_radius, dp, ws)
        if normals is None:
            normals = torch.randn((n, 2, 3), generator=generator, dtype=torch.float32, device=self.device)
        new = {k: torch.empty((n_out,) + tuple(params[k].shape[1:]), dtype=torch.float32, device=self.device)
               for k in L.FIELDS}
        m_new = v_new = None
        if exp_avg is not None:
            m_new = {k: torch.empty_like(new[k]) for k in L.FIELDS}
            v_new = {k: torch.empty_like(new[k]) for k in L.FIELDS}
        L.linprim_densify_apply(self.kind, self.sh_degree, n, L.state(params, exp_avg, exp_avg_sq),
                                normals.contiguous(), self.grad_accum, self.count, self.max_radius, dp, ws,
                                L.state(new, m_new, v_new), n_out)
        self.reset(n_out)
        return new, m_new, v_new


class MCMC:
    """LinPrim-MCMC's population steps (Sec. 3.4): relocation of dead
    octahedra and the opacity-gated position noise, in place."""

    def __init__(self, n: int, sh_degree: int = 3, device: str = "cuda"):
        self.n, self.sh_degree = int(n), int(sh_degree)
        self.device = torch.device(device)
        self.ws = torch.empty(max(L.linprim_mcmc_workspace_size(self.n), 1), dtype=torch.uint8, device=self.device)

    def relocate(self, params: dict, exp_avg: Optional[dict] = None, exp_avg_sq: Optional[dict] = None,
                 rand_u32: Optional[torch.Tensor] = None, generator: Optional[torch.Generator] = None) -> None:
        if rand_u32 is None:
            r = torch.randint(0, 2 ** 32, (self.n,), generator=generator, dtype=torch.int64, device=self.device)
            rand_u32 = r.to(torch.int32)                 # same 32 bits
        L.linprim_mcmc_relocate(L.OCTAHEDRON, self.sh_degree, self.n, L.state(params, exp_avg, exp_avg_sq),
                                rand_u32, self.ws)

    def add(self, params: dict, n_add: int, exp_avg: Optional[dict] = None, exp_avg_sq: Optional[dict] = None,
            rand_u32: Optional[torch.Tensor] = None, generator: Optional[torch.Generator] = None):
        """Returns new (params, exp_avg, exp_avg_sq) with n_add more rows,
        copies of sources drawn by opacity (GS-MCMC's growth step)."""
        n_add = int(min(max(n_add, 0), self.n))
        grow = lambda t: torch.cat([t, torch.empty((n_add,) + tuple(t.shape[1:]), dtype=t.dtype,
                                                   device=t.device)]) if t is not None else None
        newp = {k: grow(v) for k, v in params.items()}
        newm = {k: grow(v) for k, v in exp_avg.items()} if exp_avg is not None else None
        newv = {k: grow(v) for k, v in exp_avg_sq.items()} if exp_avg_sq is not None else None
        if rand_u32 is None:
            r = torch.randint(0, 2 ** 32, (max(n_add, 1),), generator=generator, dtype=torch.int64,
                              device=self.device)
            rand_u32 = r.to(torch.int32)
        L.linprim_mcmc_add(L.OCTAHEDRON, self.sh_degree, self.n, n_add, L.state(newp, newm, newv), rand_u32,
                           self.ws)
        self.n += n_add
        self.ws = torch.empty(max(L.linprim_mcmc_workspace_size(self.n), 1), dtype=torch.uint8, device=self.device)
        return newp, newm, newv

    def dead_count(self) -> int:
        return L.linprim_mcmc_dead_count(self.ws, self.n)

    def noise(self, params: dict, lr_means: float, noise_lr: float = 5e5, normals: Optional[torch.Tensor] = None,
              generator: Optional[torch.Generator] = None) -> None:
        if normals is None:
            normals = torch.randn((self.n, 3), generator=generator, dtype=torch.float32, device=self.device)
        L.linprim_mcmc_noise(L.OCTAHEDRON, self.n, L.state(params), normals.contiguous(), lr_means, noise_lr)
