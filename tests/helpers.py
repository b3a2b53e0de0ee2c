"""Small scene builders shared by the tests (no rendering arithmetic here)."""
import math

import numpy as np

from paper_2501_16312_amd import scenes

SH_C0 = 0.5 / math.sqrt(math.pi)  # Y_00 of the real orthonormal SH basis


def sh_for_rgb(rgb, n=1):
    """Degree-0 SH coefficients that give a view-independent colour ``rgb``."""
    sh = np.zeros((n, 16, 3), np.float32)
    sh[:, 0, :] = (np.asarray(rgb, np.float64) - 0.5) / SH_C0
    return sh


def rgb_of(scene, n=0):
    """View-independent colour of a degree-0 primitive built by sh_for_rgb."""
    return scene.sh[n, 0].astype(np.float64) * SH_C0 + 0.5


def prims(kind, means, quats, dists, opacity, rgb=(0.8, 0.5, 0.3), sh=None, sh_degree=3):
    means = np.atleast_2d(np.asarray(means, np.float32))
    n = means.shape[0]
    quats = np.broadcast_to(np.asarray(quats, np.float32), (n, 4)).copy()
    nd = 3 if kind == scenes.OCTAHEDRON else 4
    dists = np.broadcast_to(np.asarray(dists, np.float32), (n, nd)).copy()
    opacity = np.broadcast_to(np.asarray(opacity, np.float32), (n,)).copy()
    if sh is None:
        rgb = np.broadcast_to(np.asarray(rgb, np.float64), (n, 3))
        sh = np.zeros((n, 16, 3), np.float32)
        sh[:, 0, :] = (rgb - 0.5) / SH_C0
    return scenes.Scene(kind, means, quats, dists, opacity, np.asarray(sh, np.float32), sh_degree)


def origin_camera(W, H, vfov=60.0):
    """Camera at the world origin looking down +z (world axes = camera axes)."""
    w2c = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], np.float32)
    return scenes.make_camera(w2c, W, H, vfov)


def rotation_to_quat(R):
    """(w,x,y,z) of a rotation matrix (Shepperd's method)."""
    R = np.asarray(R, np.float64)
    tr = np.trace(R)
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        return np.array([0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s])
    i = int(np.argmax(np.diag(R)))
    if i == 0:
        s = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        return np.array([(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s])
    if i == 1:
        s = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        return np.array([(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s])
    s = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
    return np.array([(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s])


def rotation_taking(a, b):
    """Rotation matrix taking unit vector a to unit vector b (Rodrigues)."""
    a = np.asarray(a, np.float64) / np.linalg.norm(a)
    b = np.asarray(b, np.float64) / np.linalg.norm(b)
    v = np.cross(a, b)
    c = float(np.dot(a, b))
    if np.linalg.norm(v) < 1e-15:
        return np.eye(3) if c > 0 else -np.eye(3)
    K = np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])
    return np.eye(3) + K + K @ K * (1.0 / (1.0 + c))


def quat_to_matrix(q):
    """Rotation of the normalised quaternion (w,x,y,z), textbook form."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def ewa_map(cam, t):
    """Ray-space map of a camera-space point: (fx x/z + cx, fy y/z + cy, |t|)."""
    x, y, z = t
    return np.array([cam.fx * x / z + cam.cx, cam.fy * y / z + cam.cy, math.sqrt(x * x + y * y + z * z)],
                    np.float64)


def ewa_jacobian_fd(cam, t, h=1e-6):
    """Jacobian of ewa_map by central differences (independent of any renderer)."""
    J = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (ewa_map(cam, t + e) - ewa_map(cam, t - e)) / (2 * h)
    return J
