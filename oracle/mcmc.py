"""Plain CPU oracle of LinPrim-MCMC's population steps (Sec. 3.4
"LinPrim-MCMC"): the relocation and noise steps of GS-MCMC (Kheradmand et
al., 2024) applied to octahedra treated as Gaussians with the same
features and standard deviations d / 2.6.  TEST INFRASTRUCTURE ONLY: only
the test-suite may import it.  Shares no code with the HIP path.

Readings (GS-MCMC's published algorithm, restated):
  * dead: opacity <= 0.005;
  * sampling with replacement, probability proportional to opacity among
    the live primitives.  To make the integer decision exact and
    reproducible, weights are w_i = floor(alpha_i 2^32) (exact from float32)
    summed in 64-bit integers, and a 32-bit random r picks the first index
    whose inclusive prefix exceeds floor(total r / 2^32);
  * a source sampled c times becomes N = min(c + 1, 51) primitives: its
    opacity becomes 1 - (1 - alpha)^(1/N) (clamped to [0.005, 1 - 2^-23]),
    so that N stacked copies have the original opacity, and its distances
    are scaled by alpha / sum_{i=1}^{N} sum_{k=0}^{i-1} C(i-1, k) (-1)^k
    alpha_new^(k+1) / sqrt(k+1), which keeps the line integral of the
    composited opacity of a Gaussian profile; the k-th dead primitive (in
    index order) becomes a copy of the k-th sample after this update; the
    Adam moments of sources and relocated primitives are reset to zero;
  * noise: mu += noise_lr * lr_mu * s(1 - alpha) * R S^2 R^T eps with S =
    diag(d / 2.6), s(x) = 1 / (1 + exp(-100 (x - 0.995))), eps standard
    normal (passed in).
"""
from __future__ import annotations

import math

import numpy as np

MIN_OPACITY = 0.005
N_MAX = 51
SCALE_DIV = 2.6


def weights(opacity):
    a = np.asarray(opacity, np.float32)
    w = np.floor(a.astype(np.float64) * 2.0 ** 32).astype(np.uint64)
    w[a <= np.float32(MIN_OPACITY)] = 0
    return w


def sample(w, r_u32):
    """Indices drawn with probability w_i / sum(w) from 32-bit randoms."""
    prefix = np.cumsum(w.astype(object))          # exact integers
    total = int(prefix[-1]) if len(prefix) else 0
    out = []
    for r in np.asarray(r_u32, np.uint64):
        t = (total * int(r)) >> 32
        lo, hi = 0, len(prefix) - 1
        while lo < hi:                            # first prefix > t
            mid = (lo + hi) // 2
            if int(prefix[mid]) > t:
                hi = mid
            else:
                lo = mid + 1
        out.append(lo)
    return np.array(out, np.int64)


def relocation_scale(alpha_old, alpha_new, n):
    denom = 0.0
    for i in range(1, n + 1):
        for k in range(i):
            denom += math.comb(i - 1, k) * (-1.0) ** k * alpha_new ** (k + 1) / math.sqrt(k + 1)
    return alpha_old / denom


def relocate(params: dict, moments: dict, r_u32):
    """In-place on float64 copies; returns (params, moments, n_dead)."""
    p = {k: np.array(v, np.float64) for k, v in params.items()}
    m = {k: np.array(v, np.float64) for k, v in moments.items()}
    op32 = np.asarray(params["opacity"], np.float32)
    dead = np.nonzero(op32 <= np.float32(MIN_OPACITY))[0]
    if len(dead) == 0 or weights(op32).sum() == 0:
        return p, m, len(dead)
    src = sample(weights(op32), np.asarray(r_u32)[: len(dead)])
    counts = np.bincount(src, minlength=len(op32))
    for s in np.nonzero(counts)[0]:
        n = min(int(counts[s]) + 1, N_MAX)
        a = float(op32[s])
        a_new = 1.0 - (1.0 - a) ** (1.0 / n)
        a_new = min(max(a_new, MIN_OPACITY), 1.0 - 2.0 ** -23)
        p["dists"][s] = p["dists"][s] * relocation_scale(a, a_new, n)
        p["opacity"][s] = a_new
        for key in m:
            m[key][s] = 0.0
    for j, s in zip(dead, src):
        for k in p:
            p[k][j] = p[k][s]
        for key in m:
            m[key][j] = 0.0
    return p, m, len(dead)


def add(params: dict, moments: dict, n_add: int, r_u32):
    """GS-MCMC's growth step: n_add sources drawn as in relocate (among all
    current rows), the same source update, copies appended.  Returns float64
    (params, moments) with n + n_add rows."""
    p = {k: np.array(v, np.float64) for k, v in params.items()}
    m = {k: np.array(v, np.float64) for k, v in moments.items()}
    op32 = np.asarray(params["opacity"], np.float32)
    w = weights(op32)
    if n_add == 0 or w.sum() == 0:
        return p, m
    src = sample(w, np.asarray(r_u32)[:n_add])
    counts = np.bincount(src, minlength=len(op32))
    for s in np.nonzero(counts)[0]:
        nn = min(int(counts[s]) + 1, N_MAX)
        a = float(op32[s])
        a_new = min(max(1.0 - (1.0 - a) ** (1.0 / nn), MIN_OPACITY), 1.0 - 2.0 ** -23)
        p["dists"][s] = p["dists"][s] * relocation_scale(a, a_new, nn)
        p["opacity"][s] = a_new
        for key in m:
            m[key][s] = 0.0
    for k in p:
        p[k] = np.concatenate([p[k], p[k][src]])
    for key in m:
        m[key] = np.concatenate([m[key], np.zeros((n_add,) + m[key].shape[1:])])
    return p, m


def quat_matrix(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(np.asarray(q, np.float64))
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def noise(params: dict, normals, lr_means: float, noise_lr: float = 5e5):
    """Returns the new means (float64)."""
    mu = np.array(params["means"], np.float64)
    for i in range(mu.shape[0]):
        a = float(np.float32(params["opacity"][i]))
        gate = 1.0 / (1.0 + math.exp(-100.0 * ((1.0 - a) - 0.995)))
        R = quat_matrix(params["quats"][i])
        S2 = np.diag((np.asarray(params["dists"][i], np.float64) / SCALE_DIV) ** 2)
        cov = R @ S2 @ R.T
        mu[i] += noise_lr * lr_means * gate * (cov @ np.asarray(normals[i], np.float64))
    return mu
