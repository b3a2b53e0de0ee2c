"""Independent differentiable renderer in PyTorch float64 (tests only).

A third implementation of the forward definition, written with different
formulations from both the oracle and the HIP path, so that autograd gives
reference gradients for tiny scenes:

  * rotation: normalise q, then the textbook unit-quaternion matrix;
  * ray-space Jacobian: autograd Jacobian of the EWA map
    t -> (fx x/z + cx, fy y/z + cy, |t|) at the centre;
  * chord: octahedron as the intersection of the four slabs
    |sigma . M^-1 (X - c)| <= 1; tetrahedron by barycentric clipping;
  * SH: real harmonics from the associated-Legendre recurrence in spherical
    coordinates (not the Cartesian polynomials).

No pixel rectangle is needed: the footprint lies inside it, so the chord is
zero wherever the rectangle test would reject the pixel.

``exact=True`` renders the variant without ray space: the same slab and
barycentric clipping along the camera-space pixel ray t D,
D = ((px - cx)/fx, (py - cy)/fy, 1), with the chord t-interval scaled by |D|;
primitives with a corner at or in front of the near plane are skipped.
"""
import math

import numpy as np
import torch

T_STOP = 1e-3
O_MAX = 0.99


def _quat_matrix(q):
    q = q / q.norm(dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def _legendre(lmax, ct):
    """Associated Legendre P_l^m(ct) with the Condon-Shortley phase, m >= 0."""
    st = torch.sqrt(torch.clamp(1 - ct * ct, min=0.0))
    P = {(0, 0): torch.ones_like(ct)}
    for m in range(1, lmax + 1):
        P[(m, m)] = -(2 * m - 1) * st * P[(m - 1, m - 1)]
    for m in range(0, lmax):
        P[(m + 1, m)] = (2 * m + 1) * ct * P[(m, m)]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * ct * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def real_sh(lmax, dirs):
    """[..., (lmax+1)^2] real SH: sqrt2 K P cos(m phi) for m>0, sqrt2 K P sin(|m| phi)
    for m<0 (K the complex normalisation, P with the Condon-Shortley phase)."""
    x, y, z = dirs.unbind(-1)
    ct = z / dirs.norm(dim=-1)
    phi = torch.atan2(y, x)
    P = _legendre(lmax, ct)
    out = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                out.append(K * P[(l, 0)])
            elif m > 0:
                out.append(math.sqrt(2) * K * P[(l, am)] * torch.cos(am * phi))
            else:
                out.append(math.sqrt(2) * K * P[(l, am)] * torch.sin(am * phi))
    return torch.stack(out, -1)


TET_DIRS = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64) / math.sqrt(3.0)
SLABS = torch.tensor([[1, 1, 1], [1, 1, -1], [1, -1, 1], [-1, 1, 1]], dtype=torch.float64)


def render(kind, params, cam, bg, sh_degree=3, exact=False):
    """params: dict of float64 tensors means [N,3], quats [N,4], dists [N,k],
    opacity [N], sh [N,K,3].  Returns the image [3,H,W]."""
    means, quats, dists, opac, sh = (params[k] for k in ("means", "quats", "dists", "opacity", "sh"))
    n = means.shape[0]
    W, H = cam.width, cam.height
    Rw = torch.tensor(cam.world_to_cam[:, :3].astype(np.float64))
    tw = torch.tensor(cam.world_to_cam[:, 3].astype(np.float64))
    fx, fy, cx, cy = (float(v) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    R = _quat_matrix(quats)
    if kind == 0:
        offs = (R * dists[:, None, :]).transpose(1, 2)          # [N,3 axes,3]
    else:
        B = torch.tensor(TET_DIRS)
        offs = torch.einsum("nrc,ic,ni->nir", R, B, dists)     # [N,4,3]
    tc = means @ Rw.T + tw

    def ewa(t):
        return torch.stack([fx * t[0] / t[2] + cx, fy * t[1] / t[2] + cy, t.norm()])

    J = torch.stack([torch.autograd.functional.jacobian(ewa, tc[i], create_graph=True) for i in range(n)])
    c = torch.stack([ewa(tc[i]) for i in range(n)])
    a = torch.einsum("nrc,nkc->nkr", J, offs @ Rw.T)              # ray-space offsets

    # colour from SH along the viewing direction
    campos = -(Rw.T @ tw)
    dirs = means - campos
    Y = real_sh(sh_degree, dirs)
    rgb = torch.clamp(torch.einsum("nk,nkc->nc", Y, sh[:, : Y.shape[1]]) + 0.5, min=0.0)
    dmin = dists.min(dim=1).values.detach()
    sigma = -torch.log(1 - 0.99 * opac) / (2 * dmin)

    ii, jj = torch.meshgrid(torch.arange(W, dtype=torch.float64) + 0.5,
                            torch.arange(H, dtype=torch.float64) + 0.5, indexing="xy")
    pix = torch.stack([ii.reshape(-1), jj.reshape(-1)], -1)        # [P,2]
    P = pix.shape[0]
    deltas = []
    offc = offs @ Rw.T                                            # camera-space offsets
    near32 = float(np.float32(cam.near))
    culled = set()
    if exact:
        D = torch.stack([(pix[:, 0] - cx) / fx, (pix[:, 1] - cy) / fy,
                         torch.ones(P, dtype=torch.float64)], -1)   # [P,3]
        Dn = D.norm(dim=1)
        for k in range(n):
            if kind == 0:
                corners = torch.cat([tc[k] + offc[k], tc[k] - offc[k]], 0)
            else:
                corners = tc[k] + offc[k]
            if bool((corners[:, 2] <= near32).any()):
                culled.add(k)
            if kind == 0:
                Minv = torch.linalg.inv(offc[k].T)
                s0 = Minv @ (-tc[k])                          # local coords of the camera centre
                m = D @ Minv.T                                # [P,3] local direction
                num = SLABS @ s0                              # [4]
                den = m @ SLABS.T                             # [P,4]
                e1 = (-1 - num) / den
                e2 = (1 - num) / den
                lo = torch.minimum(e1, e2).max(dim=1).values
                hi = torch.maximum(e1, e2).min(dim=1).values
            else:
                E = torch.stack([offc[k, 1] - offc[k, 0], offc[k, 2] - offc[k, 0], offc[k, 3] - offc[k, 0]], 1)
                Einv = torch.linalg.inv(E)
                l0 = Einv @ (-tc[k] - offc[k, 0])             # lambda_1..3 at t = 0
                l1 = D @ Einv.T                               # [P,3]
                L0 = torch.cat([(1 - l0.sum()).reshape(1), l0])
                L1 = torch.cat([-l1.sum(1, keepdim=True), l1], 1)
                big = torch.tensor(1e30, dtype=torch.float64)
                roots = -L0 / L1
                lo = torch.where(L1 > 0, roots, -big).max(dim=1).values
                hi = torch.where(L1 < 0, roots, big).min(dim=1).values
            deltas.append(torch.relu(hi - lo) * Dn)
    for k in range(n if not exact else 0):
        rel = torch.cat([pix - c[k, :2], torch.zeros(P, 1, dtype=torch.float64)], 1)   # X - c at z = c_z
        if kind == 0:
            M = a[k].T                                        # columns = axis offsets
            Minv = torch.linalg.inv(M)
            s0 = rel @ Minv.T                                 # [P,3]
            m = Minv[:, 2]
            num = s0 @ SLABS.T                                # [P,4]
            den = SLABS @ m                                   # [4]
            e1 = (-1 - num) / den
            e2 = (1 - num) / den
            lo = torch.minimum(e1, e2).max(dim=1).values
            hi = torch.maximum(e1, e2).min(dim=1).values
        else:
            E = torch.stack([a[k, 1] - a[k, 0], a[k, 2] - a[k, 0], a[k, 3] - a[k, 0]], 1)
            Einv = torch.linalg.inv(E)
            l0 = (rel - a[k, 0]) @ Einv.T                     # lambda_1..3 at z' = 0
            l1 = Einv[:, 2]
            L0 = torch.cat([1 - l0.sum(1, keepdim=True), l0], 1)
            L1 = torch.cat([-l1.sum().reshape(1), l1])
            big = torch.tensor(1e30, dtype=torch.float64)
            roots = -L0 / L1
            lo = torch.where(L1 > 0, roots, -big).max(dim=1).values
            hi = torch.where(L1 < 0, roots, big).min(dim=1).values
        deltas.append(torch.relu(hi - lo))
    keys = tc[:, 2].detach().numpy().astype(np.float32).view(np.uint32)
    order = sorted(range(n), key=lambda k: (int(keys[k]), k))
    T = torch.ones(P, dtype=torch.float64)
    alive = torch.ones(P, dtype=torch.bool)
    C = torch.zeros(3, P, dtype=torch.float64)
    for k in order:
        if tc[k, 2].item() <= near32 or k in culled:
            continue
        o = torch.minimum(1 - torch.exp(-sigma[k] * deltas[k]), torch.tensor(O_MAX, dtype=torch.float64))
        o = torch.where(alive, o, torch.zeros_like(o))
        C = C + (T * o)[None, :] * rgb[k][:, None]
        T = T * (1 - o)
        alive = alive & (T.detach() > T_STOP)
    C = C + T[None, :] * torch.as_tensor(bg, dtype=torch.float64)[:, None]
    return C.reshape(3, H, W)
