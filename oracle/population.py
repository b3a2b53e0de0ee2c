"""Plain CPU oracle of the adaptive population control (Sec. 3.4 "Adaptive
Population Control"; thresholds in App. G).  TEST INFRASTRUCTURE ONLY: only
the test-suite may import it.  Shares no code with the HIP path.

Statistics (accumulated over the views of each step, as in 3DGS, whose
scheme the paper mirrors): for every view in which a primitive touches a
tile, add the norm of its view-space positional gradient, i.e. dL/d(ray-space
centre x, y) with the offsets held fixed, expressed per unit of normalised
device coordinates (pixels x W/2, y H/2), count the view, and keep the
largest screen radius (half the larger side of the projected box, pixels).

Densification and pruning, every decision taken in float32 (the precision
of the arrays) in the order the paper lists them:
  * size of a primitive: octahedron 2 max d (its longest axis), tetrahedron
    sqrt(2) max d (sqrt 2 times the distance to the furthest corner);
  * candidates: mean positional gradient (sum / count) above the threshold;
  * a candidate smaller than 1% of the scene extent is cloned (same
    features, zero Adam moments); a larger one is replaced by two children
    whose distances are divided by 1.2, placed at mu + R (d * z) for an
    octahedron (standard deviations equal to its distances along its own
    axes, then rotated) or mu + (max d / 2) z for a tetrahedron, z a standard
    normal 3-vector per child (passed in), zero Adam moments;
  * removed: opacity below the minimum, size above 40% of the extent, or
    (originals only, whose statistics exist) a screen radius above 20 px.
Output order: for each input primitive in index order, its survivor (the
original, or its two children), then its clone.
"""
from __future__ import annotations

import math

import numpy as np

OCTAHEDRON, TETRAHEDRON = 0, 1


def accumulate_stats(oscene, grad_accum, count, max_radius):
    """Adds the statistics of the last ``oscene.backward`` (all its views)
    to the float64 arrays grad_accum [n], count [n], max_radius [n]."""
    st = oscene.stats()
    for v, cam in enumerate(oscene.cams):
        vis = st["visible"][v]
        g = st["sgrad"][v] * np.array([cam.width / 2.0, cam.height / 2.0])
        norm = np.sqrt((g * g).sum(1))
        grad_accum[vis] += norm[vis]
        count[vis] += 1
        max_radius[vis] = np.maximum(max_radius[vis], st["radius"][v][vis])


def primitive_size(kind, dists):
    """float32 size: longest axis 2 max d (octahedron), sqrt(2) max d (tetrahedron)."""
    dm = np.max(np.asarray(dists, np.float32), axis=1)
    return (np.float32(2.0) * dm) if kind == OCTAHEDRON else (np.float32(math.sqrt(2.0)) * dm)


def quat_matrix(q):
    q = np.asarray(q, np.float64)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def decide(kind, dists, opacity, grad_accum, count, max_radius, extent, grad_threshold=1.5e-4,
           min_opacity=0.025, max_size_frac=0.4, max_radius_px=20.0, clone_size_frac=0.01, shrink=1.2):
    """Per-primitive decisions (float32 arithmetic): returns dict of boolean
    arrays keep, split (two children kept), clone (clone kept)."""
    f32 = np.float32
    acc = np.asarray(grad_accum, f32)
    cnt = np.asarray(count, np.int32)
    avg = np.where(cnt > 0, acc / np.maximum(cnt, 1).astype(f32), f32(0.0)).astype(f32)
    size = primitive_size(kind, dists)
    op = np.asarray(opacity, f32)
    ext = f32(extent)
    max_size = f32(max_size_frac) * ext
    cand = avg > f32(grad_threshold)
    small = size < f32(clone_size_frac) * ext
    clone = cand & small
    split = cand & ~small
    transparent = op < f32(min_opacity)
    keep_orig = ~split & ~transparent & ~(size > max_size) & ~(np.asarray(max_radius, f32) > f32(max_radius_px))
    child_size = size / f32(shrink)
    keep_children = split & ~transparent & ~(child_size > max_size)
    keep_clone = clone & ~transparent & ~(size > max_size)
    return {"keep": keep_orig, "split": keep_children, "clone": keep_clone}


def densify(kind, params: dict, moments: dict, stats: dict, extent: float, normals, **thresholds):
    """params / moments: dict of float arrays keyed means, quats, dists,
    opacity, sh (moments: ('m', key) and ('v', key)); stats: grad_accum,
    count, max_radius; normals [n, 2, 3] standard normal draws for the two
    children.  Returns (new params, new moments) as float64 arrays."""
    d = decide(kind, params["dists"], params["opacity"], stats["grad_accum"], stats["count"],
               stats["max_radius"], extent, **thresholds)
    shrink = float(thresholds.get("shrink", 1.2))
    keys = ("means", "quats", "dists", "opacity", "sh")
    out = {k: [] for k in keys}
    mout = {(w, k): [] for w in ("m", "v") for k in keys}
    n = params["means"].shape[0]
    for i in range(n):
        src = {k: np.asarray(params[k][i], np.float64) for k in keys}
        zero = {k: np.zeros_like(src[k]) for k in keys}
        emitted = []
        if d["keep"][i]:
            emitted.append((src, {w: {k: np.asarray(moments[(w, k)][i], np.float64) for k in keys}
                                  for w in ("m", "v")}))
        if d["split"][i]:
            dist = src["dists"]
            for j in range(2):
                z = np.asarray(normals[i, j], np.float64)
                if kind == OCTAHEDRON:
                    off = quat_matrix(src["quats"]) @ (dist * z)
                else:
                    off = (dist.max() / 2.0) * z
                child = dict(src)
                child["means"] = src["means"] + off
                child["dists"] = dist / shrink
                emitted.append((child, {"m": zero, "v": zero}))
        if d["clone"][i]:
            emitted.append((dict(src), {"m": zero, "v": zero}))
        for p, m in emitted:
            for k in keys:
                out[k].append(p[k])
                for w in ("m", "v"):
                    mout[(w, k)].append(m[w][k])
    shapes = {k: params[k].shape[1:] for k in keys}
    newp = {k: (np.array(out[k]) if out[k] else np.zeros((0,) + shapes[k])) for k in keys}
    newm = {wk: (np.array(v) if v else np.zeros((0,) + shapes[wk[1]])) for wk, v in mout.items()}
    return newp, newm
