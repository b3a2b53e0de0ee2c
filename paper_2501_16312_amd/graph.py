"""Graph-captured steps: the whole forward + backward (and optionally the loss
gradient and the Adam update) of all views recorded once into a HIP
graph and replayed, with no host work or synchronisation inside a step.

The pair count is data-dependent; the pair workspace is sized once, with
headroom, from an eager step, and every kernel reads the live count from
the device.  If a replay needs more pairs than the capacity, the render
stages leave their outputs untouched, the loss-gradient and Adam kernels
skip their work (the parameters do not change), and a sticky device flag
records it: check() raises after any number of replays if one of them
overflowed, and the step can be rebuilt with a larger capacity.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import linprim as L
from .render import Rasterizer


class CapturedStep:
    """fwd + bwd over every view of `rast`, captured in one graph.

    grad_rgb: a fixed dL/dC buffer, or None with `target` given, in which
    case the step computes the loss gradient itself: loss="l1" gives
    scale * sign(C - target); loss="l1_ssim" gives the gradient of 3DGS's
    per-view (1 - lam) L1 + lam (1 - SSIM) summed over the views (Sec. 3.4
    "Optimization"), lam = ssim_lambda.
    adam: optional dict (groups, beta1, beta2, eps) -- the update then runs
    inside the graph, reading its bias corrections from a device buffer; its
    groups' "grad" tensors must be the ones in `grads`.
    grads: optional caller-owned gradient buffers (means, quats, dists,
    opacity, sh), overwritten by every replay.
    """

    def __init__(self, rast: Rasterizer, prims: L.Prims, bg=None, grad_rgb: Optional[torch.Tensor] = None,
                 target: Optional[torch.Tensor] = None, l1_scale: Optional[float] = None,
                 adam: Optional[dict] = None, headroom: float = 1.25, grads: Optional[dict] = None,
                 loss: str = "l1", ssim_lambda: float = L.SSIM_LAMBDA):
        self.rast, self.prims, self.bg = rast, prims, bg
        rast.headroom = max(rast.headroom, headroom)
        rast.preprocess(prims, sync_count=True)          # sizes the pair workspace
        self.outs = rast.alloc_outputs()
        self.grads = grads if grads is not None else rast.alloc_grads(prims)
        self.target = target
        self.loss_kind = "l1"
        if grad_rgb is None:
            if target is None:
                raise ValueError("need grad_rgb or target")
            if loss not in ("l1", "l1_ssim"):
                raise ValueError(f"unknown loss {loss}")
            self.loss_kind = loss
            self.ssim_lambda = float(ssim_lambda)
            self.grad_rgb = torch.empty_like(self.outs[0])
            self.partial = torch.zeros((self.outs[0].numel() + 1023) // 1024, device=self.outs[0].device)
            self.l1_scale = float(l1_scale if l1_scale is not None else 1.0 / self.outs[0].numel())
            if loss == "l1_ssim":
                self.loss_ws = torch.empty(L.linprim_loss_workspace_size(rast.cams_c), dtype=torch.uint8,
                                           device=self.outs[0].device)
        else:
            self.grad_rgb = grad_rgb.contiguous()
        self.adam = adam
        # guard[0]: this replay overflowed its pair capacity; guard[1]: some
        # replay did (only the host clears it)
        self.guard = torch.zeros(2, dtype=torch.int32, device=self.outs[0].device)
        if adam is not None:
            self.bias_corr = torch.ones(2, dtype=torch.float32, device=self.outs[0].device)
            self.step_count = 0
        self._record_eager()            # one eager pass (also warms the kernels)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._enqueue()

    def _enqueue(self):
        r, p = self.rast, self.prims
        rgb, T, last = self.outs
        L.linprim_preprocess(p, r.cams_c, r.tune, r.view_ws)
        r.bin_sort(p)
        L.linprim_step_guard(p, r.cams_c, r.tune, r.view_ws, self.guard)
        r.render(p, self.bg, out=self.outs)
        if self.target is not None:
            if self.loss_kind == "l1_ssim":
                L.linprim_loss_grad(rgb, self.target, r.cams_c, self.loss_ws, self.grad_rgb, self.ssim_lambda,
                                    skip=self.guard)
            else:
                L.linprim_l1_grad(rgb, self.target, self.l1_scale, self.grad_rgb, self.partial, skip=self.guard)
        L.linprim_raster_bwd(p, r.cams_c, r.tune, self.bg, r.view_ws, r.pair_ws, r.max_pairs, T, last, self.grad_rgb)
        L.linprim_preprocess_bwd(p, r.cams_c, r.tune, r.view_ws, r.pair_ws, r.max_pairs, self.grads)
        if self.adam is not None:
            a = self.adam
            L.linprim_adam_step_dev(a["groups"], a["beta1"], a["beta2"], a["eps"], self.bias_corr, skip=self.guard)

    def _record_eager(self):
        if self.adam is None:
            self._enqueue()
        else:
            # no parameter update in the warm-up pass
            saved, self.adam = self.adam, None
            self._enqueue()
            self.adam = saved

    def replay(self):
        if self.adam is not None:
            self.step_count += 1
            bc = L.adam_bias_corrections(self.adam["beta1"], self.adam["beta2"], self.step_count)
            self.bias_corr.copy_(torch.tensor([float(bc[0]), float(bc[1])], dtype=torch.float32), non_blocking=False)
        self.graph.replay()

    def loss(self) -> float:
        """Loss of the last replay (host sync; for logging only)."""
        if self.loss_kind == "l1_ssim":
            return L.linprim_loss_value(self.loss_ws, self.rast.cams_c, self.ssim_lambda)
        return float(self.partial.sum().item())

    def check(self):
        """Raises if any replay since construction (or the last clear())
        overflowed its pair capacity; returns the last replay's pair count.
        Host sync."""
        n, overflow = self.rast.status()
        if overflow or int(self.guard[1].item()):
            raise L.LinPrimError(f"pair capacity {self.rast.max_pairs} exceeded ({n} needed by the last replay); "
                                 "those steps changed nothing; rebuild the step")
        return n

    def clear(self):
        """Forget earlier overflows (enqueued on the current stream)."""
        self.guard.zero_()


class PlainStep:
    """The same fwd + bwd with plain (uncaptured) launches."""

    def __init__(self, rast: Rasterizer, prims: L.Prims, bg, grad_rgb: torch.Tensor):
        self.rast, self.prims, self.bg = rast, prims, bg
        rast.preprocess(prims, sync_count=True)
        self.outs = rast.alloc_outputs()
        self.grads = rast.alloc_grads(prims)
        self.grad_rgb = grad_rgb.contiguous()

    def run(self):
        r, p = self.rast, self.prims
        rgb, T, last = self.outs
        L.linprim_preprocess(p, r.cams_c, r.tune, r.view_ws)
        r.bin_sort(p)
        r.render(p, self.bg, out=self.outs)
        L.linprim_raster_bwd(p, r.cams_c, r.tune, self.bg, r.view_ws, r.pair_ws, r.max_pairs, T, last, self.grad_rgb)
        L.linprim_preprocess_bwd(p, r.cams_c, r.tune, r.view_ws, r.pair_ws, r.max_pairs, self.grads)


def split_views(grad_rgb: torch.Tensor, cams: Sequence) -> list:
    """Views of a packed per-view buffer ([3,H,W] per view)."""
    out, off = [], 0
    for c in cams:
        n = 3 * c.width * c.height
        out.append(grad_rgb[off: off + n])
        off += n
    return out
