"""Pins of the oracle's photometric loss (Sec. 3.4 "Optimization": 3DGS's
L1 + SSIM).  References: SSIM of an image with itself, the closed form on
constant images away from the border, the definition evaluated by explicit
windowed sums at sampled pixels (no correlation routine), and central
differences of the whole loss.  No GPU needed."""
import math

import numpy as np

from oracle import loss as LOSS


def test_window_is_a_normalised_gaussian():
    w = LOSS.gaussian_window()
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    r = np.arange(11) - 5
    ratio = w[5, 6] / w[5, 5]
    assert abs(ratio - math.exp(-1 / (2 * 1.5 ** 2))) < 1e-14
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])
    assert r.sum() == 0


def test_identical_images():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(3, 20, 24))
    for k in range(3):
        np.testing.assert_allclose(LOSS.ssim_map(x[k], x[k]), 1.0, atol=1e-12)
        np.testing.assert_allclose(LOSS.ssim_grad(x[k], x[k]), 0.0, atol=1e-9)
    L, g = LOSS.loss_and_grad(x.reshape(-1), x.reshape(-1), [(24, 20)])
    assert abs(L) < 1e-12 and np.abs(g).max() < 1e-9


def test_constant_images_away_from_the_border():
    a, b = 0.3, 0.7
    x = np.full((30, 30), a)
    y = np.full((30, 30), b)
    s = LOSS.ssim_map(x, y)
    ref = (2 * a * b + LOSS.C1) / (a * a + b * b + LOSS.C1)      # the variances vanish
    np.testing.assert_allclose(s[5:-5, 5:-5], ref, rtol=1e-12)
    assert abs(s[0, 0] - ref) > 1e-3                             # zero padding reaches the corner


def test_map_equals_windowed_sums():
    """Local statistics summed explicitly over the 11 x 11 window (zero
    outside the image) at sampled pixels, including the border."""
    rng = np.random.default_rng(1)
    x, y = rng.uniform(size=(17, 23)), rng.uniform(size=(17, 23))
    s = LOSS.ssim_map(x, y)
    sigma = 1.5
    taps = [math.exp(-(r * r) / (2 * sigma * sigma)) for r in range(-5, 6)]
    tot = sum(taps)
    taps = [t / tot for t in taps]
    H, W = x.shape
    for (i, j) in [(0, 0), (3, 7), (8, 11), (16, 22), (10, 0), (0, 15)]:
        mx = my = exx = eyy = exy = 0.0
        for di in range(-5, 6):
            for dj in range(-5, 6):
                p, q = i + di, j + dj
                if 0 <= p < H and 0 <= q < W:
                    wt = taps[di + 5] * taps[dj + 5]
                    mx += wt * x[p, q]
                    my += wt * y[p, q]
                    exx += wt * x[p, q] ** 2
                    eyy += wt * y[p, q] ** 2
                    exy += wt * x[p, q] * y[p, q]
        sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
        ref = ((2 * mx * my + LOSS.C1) * (2 * sxy + LOSS.C2)) / ((mx * mx + my * my + LOSS.C1) *
                                                                   (sxx + syy + LOSS.C2))
        assert abs(s[i, j] - ref) < 1e-13, (i, j)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    sizes = [(14, 11), (9, 13)]
    n = sum(3 * w * h for w, h in sizes)
    c = rng.uniform(0.1, 0.9, size=n)
    t = rng.uniform(0.1, 0.9, size=n)
    L, g = LOSS.loss_and_grad(c, t, sizes)
    h = 1e-6
    for idx in rng.choice(n, size=40, replace=False):
        cp, cm = c.copy(), c.copy()
        cp[idx] += h
        cm[idx] -= h
        fd = (LOSS.loss_and_grad(cp, t, sizes)[0] - LOSS.loss_and_grad(cm, t, sizes)[0]) / (2 * h)
        assert abs(g[idx] - fd) <= 1e-6 * max(abs(fd), 1e-3), (idx, g[idx], fd)
