"""ctypes binding of liblinprim.so, the gfx950 rasterizer for transparent
octahedra and tetrahedra (LinPrim, arXiv 2501.16312).

Argument marshalling only: every function here has the name of the C entry
point it calls and passes torch device pointers and the current HIP stream
through.  Nothing is computed on the host; if the library is missing the
import fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblinprim.so")

OCTAHEDRON = 0
TETRAHEDRON = 1

OK = 0
ERR_INVALID_ARG = -1
ERR_WORKSPACE = -2
ERR_PAIR_OVERFLOW = -3
ERR_HIP = -4
ERR_DEVICE = -5
# largest primitive count of linprim_densify_noalloc (its scratch is static)
NOALLOC_MAX_PRIMS = 8388608

FLAG_COUNTERS = 1
FLAG_VIEWS_RESIDENT = 2
FLAG_RADIX_SORT = 4
FLAG_EXACT_RAYS = 8
FLAG_ANTIALIAS = 16


class linprim_prims(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("sh_degree", ctypes.c_int32), ("n", ctypes.c_int64),
                ("means", ctypes.c_void_p), ("quats", ctypes.c_void_p), ("dists", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class linprim_camera(ctypes.Structure):
    _fields_ = [("world_to_cam", ctypes.c_float * 12), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("near_z", ctypes.c_float), ("reserved", ctypes.c_int32)]


class linprim_tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("sort_digit_bits", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class linprim_adam_group(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("exp_avg", ctypes.c_void_p),
                ("exp_avg_sq", ctypes.c_void_p), ("numel", ctypes.c_int64), ("lr", ctypes.c_float),
                ("lo", ctypes.c_float), ("hi", ctypes.c_float), ("period", ctypes.c_int32),
                ("lr_tail", ctypes.c_float), ("head", ctypes.c_int32)]


class linprim_densify_params(ctypes.Structure):
    _fields_ = [("grad_threshold", ctypes.c_float), ("min_opacity", ctypes.c_float),
                ("max_size_frac", ctypes.c_float), ("max_screen_radius", ctypes.c_float),
                ("clone_size_frac", ctypes.c_float), ("split_shrink", ctypes.c_float),
                ("extent", ctypes.c_float), ("reserved", ctypes.c_int32)]


class linprim_state(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("quats", ctypes.c_void_p), ("dists", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("exp_avg", ctypes.c_void_p * 5),
                ("exp_avg_sq", ctypes.c_void_p * 5)]


EXPORTS = ("linprim_view_workspace_size", "linprim_pair_workspace_size", "linprim_preprocess",
           "linprim_pair_count", "linprim_bin_sort", "linprim_render_fwd", "linprim_render_fwd_counted",
           "linprim_render_fwd_depth",
           "linprim_render_bwd", "linprim_raster_bwd", "linprim_preprocess_bwd", "linprim_read_status",
           "linprim_strerror", "linprim_debug_pointers", "linprim_upload_views", "linprim_l1_grad",
           "linprim_adam_step", "linprim_adam_step_dev", "linprim_step_guard", "linprim_accumulate_stats",
           "linprim_densify_workspace_size", "linprim_densify_plan", "linprim_densify_apply",
           "linprim_densify_noalloc",
           "linprim_loss_workspace_size", "linprim_loss_grad", "linprim_loss_value",
           "linprim_mcmc_workspace_size", "linprim_mcmc_relocate", "linprim_mcmc_dead_count",
           "linprim_mcmc_noise", "linprim_mcmc_add")

_lib = None


class LinPrimError(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Loads liblinprim.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LinPrimError(f"{path} is missing: build it with paper_2501_16312_amd/build.py "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    pr, cm, tu = ctypes.POINTER(linprim_prims), ctypes.POINTER(linprim_camera), ctypes.POINTER(linprim_tuning)
    lib.linprim_view_workspace_size.restype = SZ
    lib.linprim_view_workspace_size.argtypes = [I32, I64, cm, I32, tu]
    lib.linprim_pair_workspace_size.restype = SZ
    lib.linprim_pair_workspace_size.argtypes = [I64, cm, I32, tu]
    lib.linprim_preprocess.argtypes = [pr, cm, I32, tu, P, SZ, P]
    lib.linprim_pair_count.argtypes = [P, ctypes.POINTER(I64), P]
    lib.linprim_upload_views.argtypes = [cm, I32, tu, P, SZ, I64, I32, P]
    lib.linprim_l1_grad.argtypes = [P, P, I64, ctypes.c_float, P, P, P, P]
    lib.linprim_adam_step.argtypes = [ctypes.POINTER(linprim_adam_group), I32, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, I32, P]
    lib.linprim_adam_step_dev.argtypes = [ctypes.POINTER(linprim_adam_group), I32, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, P, P, P]
    lib.linprim_step_guard.argtypes = [pr, cm, I32, tu, P, SZ, P, P]
    lib.linprim_bin_sort.argtypes = [pr, cm, I32, tu, P, SZ, P, SZ, I64, P]
    lib.linprim_render_fwd.argtypes = [pr, cm, I32, tu, ctypes.POINTER(ctypes.c_float), P, SZ, P, SZ, I64,
                                       P, P, P, P]
    lib.linprim_render_fwd_counted.argtypes = [pr, cm, I32, tu, ctypes.POINTER(ctypes.c_float), P, SZ, P, SZ,
                                               I64, P, P, P, P, P]
    lib.linprim_render_fwd_depth.argtypes = [pr, cm, I32, tu, ctypes.POINTER(ctypes.c_float), P, SZ, P, SZ,
                                             I64, P, P, P, P, P]
    lib.linprim_render_bwd.argtypes = [pr, cm, I32, tu, ctypes.POINTER(ctypes.c_float), P, SZ, P, SZ, I64,
                                       P, P, P, P, P, P, P, P, P]
    lib.linprim_raster_bwd.argtypes = [pr, cm, I32, tu, ctypes.POINTER(ctypes.c_float), P, SZ, P, SZ, I64,
                                       P, P, P, P]
    lib.linprim_preprocess_bwd.argtypes = [pr, cm, I32, tu, P, SZ, P, SZ, I64, P, P, P, P, P, P]
    lib.linprim_read_status.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I32), P]
    dpp, stp = ctypes.POINTER(linprim_densify_params), ctypes.POINTER(linprim_state)
    lib.linprim_accumulate_stats.argtypes = [pr, cm, I32, tu, P, SZ, P, P, P, P]
    lib.linprim_densify_workspace_size.restype = SZ
    lib.linprim_densify_workspace_size.argtypes = [I64]
    lib.linprim_densify_plan.argtypes = [I32, I64, P, P, P, P, P, dpp, P, SZ, ctypes.POINTER(I64), P]
    lib.linprim_densify_apply.argtypes = [I32, I32, I64, stp, P, P, P, P, dpp, P, SZ, stp, I64, P]
    lib.linprim_mcmc_workspace_size.restype = SZ
    lib.linprim_mcmc_workspace_size.argtypes = [I64]
    lib.linprim_mcmc_relocate.argtypes = [I32, I32, I64, stp, P, P, SZ, P]
    lib.linprim_mcmc_dead_count.argtypes = [P, SZ, I64, ctypes.POINTER(I64), P]
    lib.linprim_mcmc_add.argtypes = [I32, I32, I64, I64, stp, P, P, SZ, P]
    lib.linprim_mcmc_noise.argtypes = [I32, I64, stp, P, ctypes.c_float, ctypes.c_float, P]
    lib.linprim_loss_workspace_size.restype = SZ
    lib.linprim_loss_workspace_size.argtypes = [cm, I32]
    lib.linprim_loss_grad.argtypes = [P, P, cm, I32, ctypes.c_float, P, SZ, P, P, P]
    lib.linprim_densify_noalloc.argtypes = [I32, I32, I64, ctypes.POINTER(linprim_state), P, P, P, P,
                                            ctypes.POINTER(linprim_densify_params), ctypes.POINTER(linprim_state),
                                            I64, ctypes.POINTER(I64), P]
    lib.linprim_loss_value.argtypes = [P, SZ, cm, I32, ctypes.c_float, ctypes.POINTER(ctypes.c_double), P]
    lib.linprim_strerror.restype = ctypes.c_char_p
    lib.linprim_strerror.argtypes = [ctypes.c_int]
    lib.linprim_debug_pointers.argtypes = [pr, cm, I32, tu, P, P, I64] + [ctypes.POINTER(P)] * 9
    for f in (lib.linprim_preprocess, lib.linprim_pair_count, lib.linprim_bin_sort, lib.linprim_render_fwd,
              lib.linprim_render_fwd_counted, lib.linprim_render_fwd_depth, lib.linprim_render_bwd,
              lib.linprim_raster_bwd,
              lib.linprim_preprocess_bwd, lib.linprim_read_status, lib.linprim_upload_views,
              lib.linprim_l1_grad, lib.linprim_adam_step, lib.linprim_adam_step_dev, lib.linprim_step_guard,
              lib.linprim_debug_pointers, lib.linprim_accumulate_stats, lib.linprim_densify_plan,
              lib.linprim_densify_apply, lib.linprim_densify_noalloc, lib.linprim_loss_grad, lib.linprim_loss_value,
              lib.linprim_mcmc_relocate, lib.linprim_mcmc_dead_count, lib.linprim_mcmc_noise,
              lib.linprim_mcmc_add):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != OK:
        msg = load().linprim_strerror(rc).decode()
        raise LinPrimError(f"{what} failed: {msg} ({rc})")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ structs
class Prims:
    """Primitive features as float32 CUDA tensors (the C struct keeps raw
    pointers, so this object keeps the tensors alive)."""

    def __init__(self, kind: int, means, quats, dists, opacity, sh, sh_degree: int = 3):
        self.kind = int(kind)
        self.sh_degree = int(sh_degree)
        self.means = means.contiguous()
        self.quats = quats.contiguous()
        self.dists = dists.contiguous()
        self.opacity = opacity.contiguous()
        self.sh = sh.contiguous()
        for t in (self.means, self.quats, self.dists, self.opacity, self.sh):
            if t.dtype != torch.float32 or not t.is_cuda:
                raise LinPrimError("primitive tensors must be float32 on the GPU")
        if self.kind not in (OCTAHEDRON, TETRAHEDRON):
            raise LinPrimError(f"unknown primitive type {self.kind}")
        if not 0 <= self.sh_degree <= 3:
            raise LinPrimError(f"sh_degree must be 0..3, got {self.sh_degree}")
        n = int(self.means.shape[0]) if self.means.dim() == 2 else -1
        nd = 3 if self.kind == OCTAHEDRON else 4
        K = (self.sh_degree + 1) ** 2
        want = {"means": (n, 3), "quats": (n, 4), "dists": (n, nd), "opacity": (n,)}
        for name, shape in want.items():
            if tuple(getattr(self, name).shape) != shape:
                raise LinPrimError(f"{name} has shape {tuple(getattr(self, name).shape)}, expected {shape}")
        if tuple(self.sh.shape) not in ((n, K, 3), (n, 3 * K)):
            raise LinPrimError(f"sh has shape {tuple(self.sh.shape)}, expected ({n}, {K}, 3) for degree "
                               f"{self.sh_degree}")

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        K = (scene.sh_degree + 1) ** 2
        f = lambda a: torch.as_tensor(a, dtype=torch.float32, device=device).contiguous()
        return cls(scene.kind, f(scene.means), f(scene.quats), f(scene.dists), f(scene.opacity),
                   f(scene.sh[:, :K]), scene.sh_degree)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def c(self) -> linprim_prims:
        return linprim_prims(self.kind, self.sh_degree, self.n, self.means.data_ptr(), self.quats.data_ptr(),
                             self.dists.data_ptr(), self.opacity.data_ptr(), self.sh.data_ptr())


def cameras(cams: Sequence) -> ctypes.Array:
    """ctypes array of linprim_camera from scene cameras (world_to_cam, fx,
    fy, cx, cy, width, height, near)."""
    arr = (linprim_camera * len(cams))()
    for k, c in enumerate(cams):
        w = c.world_to_cam.astype("float32").reshape(-1)
        for i in range(12):
            arr[k].world_to_cam[i] = float(w[i])
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[k].width, arr[k].height = int(c.width), int(c.height)
        arr[k].near_z = float(c.near)
        arr[k].reserved = 0
    return arr


def tuning(tile: int = 16, sort_digit_bits: int = 8, flags: int = 0) -> linprim_tuning:
    return linprim_tuning(int(tile), int(sort_digit_bits), int(flags), 0)


# --------------------------------------------------------------- entry points
def linprim_view_workspace_size(kind: int, n: int, cams, tune) -> int:
    return int(load().linprim_view_workspace_size(kind, n, cams, len(cams), ctypes.byref(tune)))


def linprim_pair_workspace_size(max_pairs: int, cams, tune) -> int:
    return int(load().linprim_pair_workspace_size(max_pairs, cams, len(cams), ctypes.byref(tune)))


def linprim_preprocess(prims: Prims, cams, tune, view_ws: torch.Tensor, stream=None):
    p = prims.c()
    _check(load().linprim_preprocess(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _ptr(view_ws),
                                     view_ws.numel(), _stream(stream)), "linprim_preprocess")


def linprim_upload_views(cams, tune, view_ws, n: int, kind: int, stream=None):
    _check(load().linprim_upload_views(cams, len(cams), ctypes.byref(tune), _ptr(view_ws), view_ws.numel(), n, kind,
                                       _stream(stream)), "linprim_upload_views")


def linprim_l1_grad(rgb, target, scale: float, grad, partial, skip=None, stream=None):
    _check(load().linprim_l1_grad(_ptr(rgb), _ptr(target), rgb.numel(), float(scale), _ptr(grad), _ptr(partial),
                                  _ptr(skip), _stream(stream)), "linprim_l1_grad")


def _adam_groups(groups: list):
    arr = (linprim_adam_group * len(groups))()
    for k, g in enumerate(groups):
        arr[k].param = g["param"].data_ptr()
        arr[k].grad = g["grad"].data_ptr()
        arr[k].exp_avg = g["exp_avg"].data_ptr()
        arr[k].exp_avg_sq = g["exp_avg_sq"].data_ptr()
        arr[k].numel = g["param"].numel()
        arr[k].lr = float(g["lr"])
        arr[k].lo = float(g.get("lo", float("-inf")))
        arr[k].hi = float(g.get("hi", float("inf")))
        arr[k].period = int(g.get("period", 0))
        arr[k].lr_tail = float(g.get("lr_tail", g["lr"]))
        arr[k].head = int(g.get("head", 0))
    return arr


def linprim_adam_step(groups: list, beta1: float, beta2: float, eps: float, step: int, stream=None):
    """groups: list of dicts param, grad, exp_avg, exp_avg_sq (CUDA float32
    tensors of equal size), lr, and optional lo / hi projection bounds and
    period / head / lr_tail (a second rate for positions i % period >= head)."""
    arr = _adam_groups(groups)
    _check(load().linprim_adam_step(arr, len(groups), float(beta1), float(beta2), float(eps), int(step),
                                    _stream(stream)), "linprim_adam_step")


def adam_bias_corrections(beta1: float, beta2: float, step: int):
    """(1 - beta1^t, 1 - beta2^t) as float32, formed exactly as
    linprim_adam_step forms them (the float32 betas widened to double, the
    power and difference in double, one rounding to float32), so that a
    linprim_adam_step_dev fed these values updates bit-identically."""
    b1 = float(np.float32(beta1))
    b2 = float(np.float32(beta2))
    return np.float32(1.0 - b1 ** int(step)), np.float32(1.0 - b2 ** int(step))


def linprim_adam_step_dev(groups: list, beta1: float, beta2: float, eps: float, bias_corr, skip=None,
                          stream=None):
    arr = _adam_groups(groups)
    _check(load().linprim_adam_step_dev(arr, len(groups), float(beta1), float(beta2), float(eps), _ptr(bias_corr),
                                        _ptr(skip), _stream(stream)), "linprim_adam_step_dev")


def linprim_step_guard(prims: Prims, cams, tune, view_ws, guard, stream=None):
    p = prims.c()
    _check(load().linprim_step_guard(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _ptr(view_ws),
                                     view_ws.numel(), _ptr(guard), _stream(stream)), "linprim_step_guard")


def linprim_pair_count(view_ws: torch.Tensor, stream=None) -> int:
    out = ctypes.c_int64(0)
    _check(load().linprim_pair_count(_ptr(view_ws), ctypes.byref(out), _stream(stream)), "linprim_pair_count")
    return int(out.value)


def linprim_bin_sort(prims: Prims, cams, tune, view_ws, pair_ws, max_pairs: int, stream=None):
    p = prims.c()
    _check(load().linprim_bin_sort(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _ptr(view_ws),
                                   view_ws.numel(), _ptr(pair_ws), pair_ws.numel(), max_pairs, _stream(stream)),
           "linprim_bin_sort")


def _bg(bg):
    b = [0.0, 0.0, 0.0] if bg is None else [float(x) for x in bg]
    return (ctypes.c_float * 3)(*b)


def linprim_render_fwd(prims: Prims, cams, tune, bg, view_ws, pair_ws, max_pairs, out_rgb, out_T, out_last,
                       stream=None, counters: Optional[torch.Tensor] = None,
                       out_depth: Optional[torch.Tensor] = None):
    p = prims.c()
    lib = load()
    if out_depth is not None:
        if counters is not None:
            raise LinPrimError("counters and the depth map are separate entry points")
        rc = lib.linprim_render_fwd_depth(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _bg(bg),
                                          _ptr(view_ws), view_ws.numel(), _ptr(pair_ws), pair_ws.numel(), max_pairs,
                                          _ptr(out_rgb), _ptr(out_T), _ptr(out_last), _ptr(out_depth),
                                          _stream(stream))
    elif counters is None:
        rc = lib.linprim_render_fwd(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _bg(bg), _ptr(view_ws),
                                    view_ws.numel(), _ptr(pair_ws), pair_ws.numel(), max_pairs, _ptr(out_rgb),
                                    _ptr(out_T), _ptr(out_last), _stream(stream))
    else:
        rc = lib.linprim_render_fwd_counted(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _bg(bg),
                                            _ptr(view_ws), view_ws.numel(), _ptr(pair_ws), pair_ws.numel(),
                                            max_pairs, _ptr(out_rgb), _ptr(out_T), _ptr(out_last), _ptr(counters),
                                            _stream(stream))
    _check(rc, "linprim_render_fwd")


def linprim_render_bwd(prims: Prims, cams, tune, bg, view_ws, pair_ws, max_pairs, out_T, out_last, grad_rgb,
                       grads: dict, stream=None):
    p = prims.c()
    _check(load().linprim_render_bwd(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _bg(bg), _ptr(view_ws),
                                     view_ws.numel(), _ptr(pair_ws), pair_ws.numel(), max_pairs, _ptr(out_T),
                                     _ptr(out_last), _ptr(grad_rgb), _ptr(grads["means"]), _ptr(grads["quats"]),
                                     _ptr(grads["dists"]), _ptr(grads["opacity"]), _ptr(grads["sh"]),
                                     _stream(stream)), "linprim_render_bwd")


def linprim_raster_bwd(prims: Prims, cams, tune, bg, view_ws, pair_ws, max_pairs, out_T, out_last, grad_rgb,
                       stream=None):
    p = prims.c()
    _check(load().linprim_raster_bwd(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _bg(bg), _ptr(view_ws),
                                     view_ws.numel(), _ptr(pair_ws), pair_ws.numel(), max_pairs, _ptr(out_T),
                                     _ptr(out_last), _ptr(grad_rgb), _stream(stream)), "linprim_raster_bwd")


def linprim_preprocess_bwd(prims: Prims, cams, tune, view_ws, pair_ws, max_pairs, grads: dict, stream=None):
    p = prims.c()
    _check(load().linprim_preprocess_bwd(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _ptr(view_ws),
                                         view_ws.numel(), _ptr(pair_ws), pair_ws.numel(), max_pairs,
                                         _ptr(grads["means"]), _ptr(grads["quats"]), _ptr(grads["dists"]),
                                         _ptr(grads["opacity"]), _ptr(grads["sh"]), _stream(stream)),
           "linprim_preprocess_bwd")


def linprim_read_status(view_ws, stream=None):
    n = ctypes.c_int64(0)
    ov = ctypes.c_int32(0)
    _check(load().linprim_read_status(_ptr(view_ws), ctypes.byref(n), ctypes.byref(ov), _stream(stream)),
           "linprim_read_status")
    return int(n.value), bool(ov.value)


def linprim_debug_pointers(prims: Prims, cams, tune, view_ws, pair_ws, max_pairs) -> dict:
    p = prims.c()
    outs = [ctypes.c_void_p() for _ in range(9)]
    _check(load().linprim_debug_pointers(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _ptr(view_ws),
                                         _ptr(pair_ws), max_pairs, *[ctypes.byref(o) for o in outs]),
           "linprim_debug_pointers")
    names = ("payload", "depth_keys", "tiles", "offsets", "keys", "values", "ranges", "order_fwd", "order_bwd")
    return {k: int(o.value or 0) for k, o in zip(names, outs)}


# ---------------------------------------------------------------------------
# Adaptive population control.
# ---------------------------------------------------------------------------
FIELDS = ("means", "quats", "dists", "opacity", "sh")


def densify_params(extent: float, grad_threshold: float = 1.5e-4, min_opacity: float = 0.025,
                   max_size_frac: float = 0.4, max_screen_radius: float = 20.0, clone_size_frac: float = 0.01,
                   split_shrink: float = 1.2) -> linprim_densify_params:
    """App. G's thresholds by default."""
    return linprim_densify_params(grad_threshold, min_opacity, max_size_frac, max_screen_radius, clone_size_frac,
                                  split_shrink, float(extent), 0)


def state(params: dict, exp_avg: Optional[dict] = None, exp_avg_sq: Optional[dict] = None) -> linprim_state:
    st = linprim_state()
    for k in FIELDS:
        setattr(st, k, params[k].data_ptr() if params[k].numel() else None)
    for f, k in enumerate(FIELDS):
        st.exp_avg[f] = exp_avg[k].data_ptr() if exp_avg is not None and exp_avg[k].numel() else None
        st.exp_avg_sq[f] = exp_avg_sq[k].data_ptr() if exp_avg_sq is not None and exp_avg_sq[k].numel() else None
    return st


def linprim_accumulate_stats(prims: Prims, cams, tune, view_ws, grad_accum, count, max_radius, stream=None):
    p = prims.c()
    _check(load().linprim_accumulate_stats(ctypes.byref(p), cams, len(cams), ctypes.byref(tune), _ptr(view_ws),
                                           view_ws.numel(), _ptr(grad_accum), _ptr(count), _ptr(max_radius),
                                           _stream(stream)), "linprim_accumulate_stats")


def linprim_densify_workspace_size(n: int) -> int:
    return int(load().linprim_densify_workspace_size(int(n)))


def linprim_densify_plan(kind: int, dists, opacity, grad_accum, count, max_radius, dp: linprim_densify_params,
                         ws, stream=None) -> int:
    out = ctypes.c_int64(0)
    _check(load().linprim_densify_plan(int(kind), int(opacity.numel()), _ptr(dists), _ptr(opacity),
                                       _ptr(grad_accum), _ptr(count), _ptr(max_radius), ctypes.byref(dp), _ptr(ws),
                                       ws.numel(), ctypes.byref(out), _stream(stream)), "linprim_densify_plan")
    return int(out.value)


def linprim_densify_apply(kind: int, sh_degree: int, n: int, src: linprim_state, normals, grad_accum, count,
                          max_radius, dp: linprim_densify_params, ws, dst: linprim_state, n_out: int, stream=None):
    _check(load().linprim_densify_apply(int(kind), int(sh_degree), int(n), ctypes.byref(src), _ptr(normals),
                                        _ptr(grad_accum), _ptr(count), _ptr(max_radius), ctypes.byref(dp), _ptr(ws),
                                        ws.numel(), ctypes.byref(dst), int(n_out), _stream(stream)),
           "linprim_densify_apply")


def linprim_densify_noalloc(kind: int, sh_degree: int, n: int, src: linprim_state, normals, grad_accum, count,
                            max_radius, dp: linprim_densify_params, dst: linprim_state, dst_rows: int,
                            stream=None) -> int:
    """Plan and apply in one call with the library's own scratch (no
    workspace); returns the number of primitives written to dst."""
    out = ctypes.c_int64(0)
    _check(load().linprim_densify_noalloc(int(kind), int(sh_degree), int(n), ctypes.byref(src), _ptr(normals),
                                          _ptr(grad_accum), _ptr(count), _ptr(max_radius), ctypes.byref(dp),
                                          ctypes.byref(dst), int(dst_rows), ctypes.byref(out), _stream(stream)),
           "linprim_densify_noalloc")
    return int(out.value)


# ---------------------------------------------------------------------------
# Photometric loss (3DGS's L1 + SSIM).
# ---------------------------------------------------------------------------
SSIM_LAMBDA = 0.2


def linprim_loss_workspace_size(cams) -> int:
    return int(load().linprim_loss_workspace_size(cams, len(cams)))


def linprim_loss_grad(rgb, target, cams, ws, grad, lam: float = SSIM_LAMBDA, skip=None, stream=None):
    _check(load().linprim_loss_grad(_ptr(rgb), _ptr(target), cams, len(cams), float(lam), _ptr(ws), ws.numel(),
                                    _ptr(grad), _ptr(skip), _stream(stream)), "linprim_loss_grad")


def linprim_loss_value(ws, cams, lam: float = SSIM_LAMBDA, stream=None) -> float:
    out = ctypes.c_double(0.0)
    _check(load().linprim_loss_value(_ptr(ws), ws.numel(), cams, len(cams), float(lam), ctypes.byref(out),
                                     _stream(stream)), "linprim_loss_value")
    return float(out.value)


# ---------------------------------------------------------------------------
# LinPrim-MCMC population steps.
# ---------------------------------------------------------------------------
def linprim_mcmc_workspace_size(n: int) -> int:
    return int(load().linprim_mcmc_workspace_size(int(n)))


def linprim_mcmc_relocate(kind: int, sh_degree: int, n: int, st: linprim_state, rand_u32, ws, stream=None):
    _check(load().linprim_mcmc_relocate(int(kind), int(sh_degree), int(n), ctypes.byref(st), _ptr(rand_u32),
                                        _ptr(ws), ws.numel(), _stream(stream)), "linprim_mcmc_relocate")


def linprim_mcmc_add(kind: int, sh_degree: int, n: int, n_add: int, st: linprim_state, rand_u32, ws, stream=None):
    _check(load().linprim_mcmc_add(int(kind), int(sh_degree), int(n), int(n_add), ctypes.byref(st), _ptr(rand_u32),
                                   _ptr(ws), ws.numel(), _stream(stream)), "linprim_mcmc_add")


def linprim_mcmc_dead_count(ws, n: int, stream=None) -> int:
    out = ctypes.c_int64(0)
    _check(load().linprim_mcmc_dead_count(_ptr(ws), ws.numel(), int(n), ctypes.byref(out), _stream(stream)),
           "linprim_mcmc_dead_count")
    return int(out.value)


def linprim_mcmc_noise(kind: int, n: int, st: linprim_state, normals, lr_means: float, noise_lr: float = 5e5,
                       stream=None):
    _check(load().linprim_mcmc_noise(int(kind), int(n), ctypes.byref(st), _ptr(normals), float(lr_means),
                                     float(noise_lr), _stream(stream)), "linprim_mcmc_noise")
