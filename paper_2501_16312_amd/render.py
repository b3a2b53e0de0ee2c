"""Rasterizer object and autograd Function over the C ABI.

Owns the two device workspaces (torch uint8 tensors) and sequences the
entry points: preprocess -> pair_count (the one host sync, to size the pair
workspace) -> bin_sort -> render_fwd, and render_bwd for gradients.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import linprim as L


class Rasterizer:
    def __init__(self, kind: int, n: int, cams: Sequence, tile: int = 16, sort_digit_bits: int = 8,
                 device: str = "cuda", headroom: float = 1.0, views_resident: bool = False,
                 radix_sort: bool = False, exact: bool = False, antialias: bool = False):
        """views_resident: the camera poses live in the view workspace and
        are replaced with set_views() (same image sizes), so that a captured
        graph can be replayed on new poses.  radix_sort: order the pairs with
        the global LSD radix sort (sort_digit_bits per pass) instead of the
        per-tile sort.  exact: render without the ray-space approximation
        (pixel rays meet the camera-space primitives).  antialias: the 2D
        anti-aliasing filter of the ray-space model."""
        self.kind = int(kind)
        self.n = int(n)
        self.cams = list(cams)
        self.cams_c = L.cameras(self.cams)
        self.views_resident = bool(views_resident)
        flags = ((L.FLAG_VIEWS_RESIDENT if views_resident else 0) | (L.FLAG_RADIX_SORT if radix_sort else 0)
                 | (L.FLAG_EXACT_RAYS if exact else 0) | (L.FLAG_ANTIALIAS if antialias else 0))
        self.exact = bool(exact)
        self.tune = L.tuning(tile, sort_digit_bits, flags)
        self.device = torch.device(device)
        self.headroom = float(headroom)
        size = L.linprim_view_workspace_size(self.kind, self.n, self.cams_c, self.tune)
        if size == 0:
            raise L.LinPrimError("invalid rasterizer configuration")
        self.view_ws = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.pair_ws = torch.empty(0, dtype=torch.uint8, device=self.device)
        self.max_pairs = 0
        self.n_pixels = sum(c.width * c.height for c in self.cams)
        self.n_pairs = 0
        # bumped by every preprocess: the workspaces then hold another
        # render's lists, which a pending backward of an earlier render
        # must not read
        self.generation = 0
        if self.views_resident:
            L.linprim_upload_views(self.cams_c, self.tune, self.view_ws, self.n, self.kind)

    def set_views(self, cams: Sequence):
        """New camera poses for a views_resident rasterizer (enqueued on the
        current stream; image sizes must match the original ones)."""
        if not self.views_resident:
            raise L.LinPrimError("set_views needs a views_resident rasterizer")
        cams = list(cams)
        if [(c.width, c.height) for c in cams] != [(c.width, c.height) for c in self.cams]:
            raise L.LinPrimError("set_views: image sizes must stay the same")
        self.cams = cams
        self.cams_c = L.cameras(cams)
        L.linprim_upload_views(self.cams_c, self.tune, self.view_ws, self.n, self.kind)

    def reserve_pairs(self, n_pairs: int):
        if n_pairs <= self.max_pairs and self.pair_ws.numel() > 0:
            return
        cap = max(int(n_pairs * self.headroom), n_pairs, 1)
        size = L.linprim_pair_workspace_size(cap, self.cams_c, self.tune)
        if size == 0:
            raise L.LinPrimError(f"pair capacity {cap} not supported")
        self.pair_ws = torch.empty(size, dtype=torch.uint8, device=self.device)
        self.max_pairs = cap

    # -- forward
    def preprocess(self, prims: L.Prims, sync_count: bool = True) -> int:
        self.generation += 1
        L.linprim_preprocess(prims, self.cams_c, self.tune, self.view_ws)
        if sync_count:
            self.n_pairs = L.linprim_pair_count(self.view_ws)
            self.reserve_pairs(self.n_pairs)
        return self.n_pairs

    def bin_sort(self, prims: L.Prims):
        L.linprim_bin_sort(prims, self.cams_c, self.tune, self.view_ws, self.pair_ws, self.max_pairs)

    def alloc_outputs(self):
        rgb = torch.empty(3 * self.n_pixels, dtype=torch.float32, device=self.device)
        T = torch.empty(self.n_pixels, dtype=torch.float32, device=self.device)
        last = torch.empty(self.n_pixels, dtype=torch.int32, device=self.device)
        return rgb, T, last

    def render(self, prims: L.Prims, bg=None, out=None, counters: Optional[torch.Tensor] = None,
               depth: Optional[torch.Tensor] = None):
        """depth: optional float32 [n_pixels] tensor that receives the depth
        map (distance along the pixel ray to the entry of the primitive at
        which cumulative opacity first exceeds 0.5, 0 elsewhere)."""
        rgb, T, last = out if out is not None else self.alloc_outputs()
        L.linprim_render_fwd(prims, self.cams_c, self.tune, bg, self.view_ws, self.pair_ws, self.max_pairs, rgb,
                             T, last, counters=counters, out_depth=depth)
        return rgb, T, last

    def forward(self, prims: L.Prims, bg=None, counters: Optional[torch.Tensor] = None):
        self.preprocess(prims)
        self.bin_sort(prims)
        return self.render(prims, bg, counters=counters)

    # -- backward
    def alloc_grads(self, prims: L.Prims) -> dict:
        z = lambda t: torch.empty_like(t)
        return {"means": z(prims.means), "quats": z(prims.quats), "dists": z(prims.dists),
                "opacity": z(prims.opacity), "sh": z(prims.sh)}

    def backward(self, prims: L.Prims, bg, T, last, grad_rgb, grads: Optional[dict] = None) -> dict:
        g = grads if grads is not None else self.alloc_grads(prims)
        L.linprim_render_bwd(prims, self.cams_c, self.tune, bg, self.view_ws, self.pair_ws, self.max_pairs, T, last,
                             grad_rgb.contiguous(), g)
        return g

    def status(self):
        return L.linprim_read_status(self.view_ws)

    def debug_arrays(self, prims: L.Prims) -> dict:
        """Copies of the workspace arrays (payload records, depth keys, tile
        counts, offsets, sorted keys/values, tile ranges) as CPU tensors."""
        ptr = L.linprim_debug_pointers(prims, self.cams_c, self.tune, self.view_ws, self.pair_ws, self.max_pairs)
        vn = self.n * len(self.cams)
        vbase, pbase = self.view_ws.data_ptr(), self.pair_ws.data_ptr()
        n_tiles = sum(((c.width + self.tune.tile - 1) // self.tune.tile) * ((c.height + self.tune.tile - 1)
                                                                           // self.tune.tile) for c in self.cams)

        def take(ws, base, addr, count, dtype, itemsize):
            off = addr - base
            return ws[off: off + count * itemsize].view(dtype).cpu().clone()

        return {
            "payload": take(self.view_ws, vbase, ptr["payload"], vn * 32, torch.float32, 4).reshape(vn, 32),
            "depth_keys": take(self.view_ws, vbase, ptr["depth_keys"], vn, torch.int32, 4),
            "tiles": take(self.view_ws, vbase, ptr["tiles"], vn, torch.int32, 4),
            "offsets": take(self.view_ws, vbase, ptr["offsets"], vn, torch.int32, 4),
            "keys": take(self.pair_ws, pbase, ptr["keys"], self.n_pairs, torch.int64, 8),
            "values": take(self.pair_ws, pbase, ptr["values"], self.n_pairs, torch.int32, 4),
            "ranges": take(self.view_ws, vbase, ptr["ranges"], 2 * n_tiles, torch.int32, 4).reshape(n_tiles, 2),
        }


class LinPrimRender(torch.autograd.Function):
    """Differentiable render of all views (Sec. 3.4 backpropagation with the
    hand-written backward of App. E): returns the packed image (view-major,
    each [3,H,W]).  The forward keeps only the final transmittance and the
    last blended list position per pixel; the backward recomputes the rest
    from the rasterizer's workspaces, so one rasterizer serves one pending
    backward at a time: running it forward again before this backward raises
    instead of returning another render's gradients."""

    @staticmethod
    def forward(ctx, rast: Rasterizer, kind: int, sh_degree: int, bg, means, quats, dists, opacity, sh):
        prims = L.Prims(kind, means.detach(), quats.detach(), dists.detach(), opacity.detach(), sh.detach(),
                        sh_degree)
        rgb, T, last = rast.forward(prims, bg)
        ctx.rast, ctx.prims, ctx.bg = rast, prims, bg
        ctx.generation = rast.generation
        ctx.save_for_backward(T, last)
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        if ctx.rast.generation != ctx.generation:
            raise L.LinPrimError("the rasterizer has rendered again since this forward; use one rasterizer per "
                                 "pending backward")
        T, last = ctx.saved_tensors
        g = ctx.rast.backward(ctx.prims, ctx.bg, T, last, grad_rgb)
        return None, None, None, None, g["means"], g["quats"], g["dists"], g["opacity"], g["sh"]


def render(rast: Rasterizer, kind: int, means, quats, dists, opacity, sh, sh_degree: int = 3, bg=None):
    return LinPrimRender.apply(rast, kind, sh_degree, bg, means, quats, dists, opacity, sh)
