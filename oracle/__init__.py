"""FP64 CPU oracle for the linear-primitive rasterizer (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It loads ``liblinprim_oracle.so``,
compiled from ``linprim_oracle.c`` by :func:`build`, and shares no code with
the HIP implementation.  Inputs are the float32 scene arrays, widened to
float64 exactly once here, so both implementations start from the same
numbers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "linprim_oracle.c")
_LIB = os.path.join(_HERE, "liblinprim_oracle.so")

OCTAHEDRON = 0
TETRAHEDRON = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (double precision, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    I64 = ctypes.c_int64
    lib.orc_new.restype = P
    lib.orc_new.argtypes = [ctypes.c_int, ctypes.c_int, I64, D, D, D, D, D]
    lib.orc_free.argtypes = [P]
    lib.orc_set_views.argtypes = [P, ctypes.c_int, D, ctypes.c_int]
    lib.orc_preprocess.argtypes = [P]
    lib.orc_get_prep.argtypes = [P, ctypes.c_int] + [ctypes.c_void_p] * 9
    lib.orc_sort.argtypes = [P]
    lib.orc_num_pairs.restype = I64
    lib.orc_num_pairs.argtypes = [P]
    lib.orc_num_tiles.restype = I64
    lib.orc_num_tiles.argtypes = [P]
    lib.orc_get_sort.argtypes = [P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_render.argtypes = [P, ctypes.c_int] + [ctypes.c_void_p] * 7
    lib.orc_render_band.argtypes = [P, ctypes.c_int] + [ctypes.c_void_p] * 7 + [ctypes.c_int, ctypes.c_int]
    lib.orc_render_pixels.argtypes = [P, ctypes.c_int, I64] + [ctypes.c_void_p] * 7
    lib.orc_chord.restype = ctypes.c_double
    lib.orc_chord.argtypes = [P, ctypes.c_int, I64, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.orc_mtia.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    lib.orc_mtia_ray.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_set_exact.argtypes = [P, ctypes.c_int]
    lib.orc_set_antialias.argtypes = [P, ctypes.c_int]
    lib.orc_render_depth.argtypes = [P] + [ctypes.c_void_p] * 3
    lib.orc_get_stats.argtypes = [P] + [ctypes.c_void_p] * 3
    lib.orc_sh_basis.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.orc_backward.argtypes = [P] + [ctypes.c_void_p] * 8
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel regions from now on."""
    _load().orc_set_threads(int(n))


def sh_basis(deg: int, direction) -> np.ndarray:
    d = _f64(direction).reshape(3)
    out = np.zeros(16)
    _load().orc_sh_basis(int(deg), _ptr(d), _ptr(out))
    return out


def mtia(corners, rx: float, ry: float) -> dict:
    """Moeller-Trumbore for a +z ray through (rx, ry) and its App. E gradient."""
    V = _f64(corners).reshape(9)
    out = np.zeros(14)
    _load().orc_mtia(_ptr(V), float(rx), float(ry), _ptr(out))
    return {"hit": bool(out[0]), "t": out[1], "u": out[2], "v": out[3], "det": out[4],
            "dV": out[5:].reshape(3, 3)}


def mtia_ray(corners, direction) -> dict:
    """Moeller-Trumbore for the ray t * direction from the origin (exact
    variant) and the derivatives of t with respect to the corners."""
    V = _f64(corners).reshape(9)
    D = _f64(direction).reshape(3)
    out = np.zeros(14)
    _load().orc_mtia_ray(_ptr(V), _ptr(D), _ptr(out))
    return {"hit": bool(out[0]), "t": out[1], "u": out[2], "v": out[3], "det": out[4],
            "dV": out[5:].reshape(3, 3)}


def camera_rows(cams) -> np.ndarray:
    return np.stack([c.as_row() for c in cams]).astype(np.float64)


class OracleScene:
    """One scene and a set of views, rendered in double precision.

    ``exact`` selects the variant without the ray-space approximation: pixel
    rays from the camera centre meet the camera-space primitives.
    ``antialias`` applies the 2D anti-aliasing filter (ray space only)."""

    def __init__(self, scene, cams, tile: int = 16, inputs64: Optional[dict] = None, exact: bool = False,
                 antialias: bool = False):
        if exact and antialias:
            raise ValueError("the anti-aliasing filter belongs to the ray-space model")
        lib = _load()
        self.kind = int(scene.kind)
        self.n = int(scene.n)
        self.sh_degree = int(scene.sh_degree)
        src = inputs64 or {}
        # float32 -> float64 exactly once; the caller may pass float64 inputs
        # directly (finite-difference tests).
        self._m = _f64(src.get("means", scene.means))
        self._q = _f64(src.get("quats", scene.quats))
        self._d = _f64(src.get("dists", scene.dists))
        self._o = _f64(src.get("opacity", scene.opacity))
        sh = _f64(src.get("sh", scene.sh)).reshape(self.n, -1, 3)
        sh48 = np.zeros((self.n, 16, 3))
        sh48[:, : sh.shape[1]] = sh
        self._sh = np.ascontiguousarray(sh48)
        D = ctypes.POINTER(ctypes.c_double)
        self.h = lib.orc_new(self.kind, self.sh_degree, self.n,
                             self._m.ctypes.data_as(D), self._q.ctypes.data_as(D),
                             self._d.ctypes.data_as(D), self._o.ctypes.data_as(D),
                             self._sh.ctypes.data_as(D))
        if not self.h:
            raise ValueError("oracle rejected the scene")
        self.cams = list(cams)
        self.tile = int(tile)
        rows = camera_rows(self.cams)
        if lib.orc_set_views(self.h, len(self.cams), rows.ctypes.data_as(D), self.tile) != 0:
            raise ValueError("oracle rejected the cameras")
        self._sorted = False
        self.exact = bool(exact)
        lib.orc_set_exact(self.h, 1 if self.exact else 0)
        self.antialias = bool(antialias)
        lib.orc_set_antialias(self.h, 1 if self.antialias else 0)
        lib.orc_preprocess(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self.h = None

    @property
    def nd(self) -> int:
        return 3 if self.kind == OCTAHEDRON else 4

    def prep(self, v: int = 0) -> dict:
        n = self.n
        out = {"rect": np.zeros((n, 4), np.int32), "tiles": np.zeros(n, np.int64),
               "key": np.zeros(n, np.uint32), "tc": np.zeros((n, 3)), "c": np.zeros((n, 3)),
               "a": np.zeros((n, 4, 3)), "sigma": np.zeros(n), "rgb": np.zeros((n, 3)),
               "raw": np.zeros((n, 3))}
        _load().orc_get_prep(self.h, v, *[_ptr(out[k]) for k in
                                          ("rect", "tiles", "key", "tc", "c", "a", "sigma", "rgb", "raw")])
        out["valid"] = out["rect"][:, 0] >= 0
        return out

    def sort(self) -> dict:
        lib = _load()
        lib.orc_sort(self.h)
        self._sorted = True
        npairs = int(lib.orc_num_pairs(self.h))
        ntiles = int(lib.orc_num_tiles(self.h))
        keys = np.zeros(max(npairs, 1), np.uint64)
        vals = np.zeros(max(npairs, 1), np.uint32)
        ranges = np.zeros((ntiles, 2), np.int64)
        lib.orc_get_sort(self.h, _ptr(keys), _ptr(vals), _ptr(ranges))
        return {"keys": keys[:npairs], "values": vals[:npairs], "ranges": ranges}

    def _ensure_sorted(self):
        if not self._sorted:
            _load().orc_sort(self.h)
            self._sorted = True

    def _bg(self, bg) -> np.ndarray:
        b = _f64(np.zeros(3) if bg is None else bg)
        if b.size == 3:
            b = np.tile(b, len(self.cams))
        return np.ascontiguousarray(b.reshape(-1))

    def render(self, bg=None, mode: str = "tiled") -> dict:
        """mode: 'tiled' (paper pipeline), 'brute' (plain definition), 'clip'
        (tiled, independent chord formulation)."""
        m = {"tiled": 0, "brute": 1, "clip": 2}[mode]
        if m != 1:
            self._ensure_sorted()
        npx = sum(c.width * c.height for c in self.cams)
        rgb = np.zeros(3 * npx)
        T = np.zeros(npx)
        last = np.zeros(npx, np.int64)
        ill = np.zeros(npx, np.uint8)
        cond = np.zeros(npx)
        counts = np.zeros((len(self.cams), 6), np.int64)
        b = self._bg(bg)
        rc = _load().orc_render(self.h, m, _ptr(b), _ptr(rgb), _ptr(T), _ptr(last), _ptr(ill),
                                _ptr(cond), _ptr(counts))
        if rc != 0:
            raise RuntimeError("oracle render failed")
        return {"rgb": rgb, "T": T, "last": last, "ill": ill, "cond": cond, "counts": counts}

    def render_depth(self, bg=None) -> dict:
        """Depth map (centre camera z of the primitive at which cumulative
        opacity first exceeds 0.5; 0 where it never does), packed like T."""
        self._ensure_sorted()
        npx = sum(c.width * c.height for c in self.cams)
        depth = np.zeros(npx)
        ill = np.zeros(npx, np.uint8)
        b = self._bg(bg)
        if _load().orc_render_depth(self.h, _ptr(b), _ptr(depth), _ptr(ill)) != 0:
            raise RuntimeError("oracle depth render failed")
        return {"depth": depth, "ill": ill.astype(bool)}

    def stats(self) -> dict:
        """Screen-space statistics of the last backward(): per view and
        primitive, sgrad [V,n,2] = dL/d(projected centre, pixels) with the
        ray-space offsets held fixed, radius [V,n] (half the larger side of
        the projected box, pixels) and visible [V,n] (touches a tile)."""
        V, n = len(self.cams), self.n
        sg = np.zeros((V, n, 2))
        rad = np.zeros((V, n))
        vis = np.zeros((V, n), np.uint8)
        if _load().orc_get_stats(self.h, _ptr(sg), _ptr(rad), _ptr(vis)) != 0:
            raise RuntimeError("call backward() first")
        return {"sgrad": sg, "radius": rad, "visible": vis.astype(bool)}

    def render_band(self, j0: int, j1: int, bg=None) -> dict:
        """Tiled render of the rows [j0, j1) of every view only (others zero)."""
        self._ensure_sorted()
        npx = sum(c.width * c.height for c in self.cams)
        rgb = np.zeros(3 * npx)
        T = np.zeros(npx)
        last = np.zeros(npx, np.int64)
        ill = np.zeros(npx, np.uint8)
        cond = np.zeros(npx)
        counts = np.zeros((len(self.cams), 6), np.int64)
        b = self._bg(bg)
        rc = _load().orc_render_band(self.h, 0, _ptr(b), _ptr(rgb), _ptr(T), _ptr(last), _ptr(ill),
                                     _ptr(cond), _ptr(counts), int(j0), int(j1))
        if rc != 0:
            raise RuntimeError("oracle render failed")
        return {"rgb": rgb, "T": T, "last": last, "ill": ill, "cond": cond, "counts": counts}

    def render_pixels(self, v: int, pix: np.ndarray, bg=None) -> dict:
        pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 2)
        q = pix.shape[0]
        rgb = np.zeros((q, 3))
        T = np.zeros(q)
        ill = np.zeros(q, np.uint8)
        ev = np.zeros(q, np.int64)
        cond = np.zeros(q)
        b = _f64(np.zeros(3) if bg is None else bg).reshape(3)
        _load().orc_render_pixels(self.h, v, q, _ptr(pix), _ptr(b), _ptr(rgb), _ptr(T), _ptr(ill),
                                  _ptr(ev), _ptr(cond))
        return {"rgb": rgb, "T": T, "ill": ill, "evaluated": ev, "cond": cond}

    def chord(self, v: int, n: int, px: float, py: float, method: str = "mtia") -> float:
        return float(_load().orc_chord(self.h, v, n, px, py, 0 if method == "mtia" else 1))

    def backward(self, grad_rgb, bg=None) -> dict:
        self._ensure_sorted()
        g = _f64(grad_rgb).reshape(-1)
        n = self.n
        out = {"means": np.zeros((n, 3)), "quats": np.zeros((n, 4)), "dists": np.zeros((n, self.nd)),
               "opacity": np.zeros(n), "sh": np.zeros((n, 16, 3)), "ill": np.zeros(n, np.uint8)}
        b = self._bg(bg)
        rc = _load().orc_backward(self.h, _ptr(b), _ptr(g), *[_ptr(out[k]) for k in
                                                            ("means", "quats", "dists", "opacity", "sh", "ill")])
        if rc != 0:
            raise RuntimeError("oracle backward failed")
        out["sh"] = out["sh"][:, : (self.sh_degree + 1) ** 2]
        # bit 0: a discrete decision of a step may differ in float32; bit 1:
        # the float32 error estimate of the opacity or SH gradient is too large
        out["ill_bits"] = out["ill"]
        out["ill"] = out["ill"] != 0
        return out


def render(scene, cams, bg=None, tile: int = 16, mode: str = "tiled", exact: bool = False) -> dict:
    return OracleScene(scene, cams, tile, exact=exact).render(bg, mode)
