"""Pins of the optimisation-step oracle (L1 gradient and Adam, Sec. 3.4)
against a library routine and closed forms.  No GPU needed."""
import math

import numpy as np
import torch

from oracle import optim as O


def test_adam_matches_torch_optim_fp64():
    """Several consecutive steps equal torch.optim.Adam (float64, plain loop)."""
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=257)
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-15, foreach=False)
    mine = (p0.copy(), np.zeros(257), np.zeros(257))
    for t in range(1, 6):
        g = rng.normal(size=257) * (10.0 ** rng.uniform(-4, 1, size=257))
        p.grad = torch.tensor(g)
        opt.step()
        mine = O.adam_step(mine[0], g, mine[1], mine[2], t, 3e-3, 0.9, 0.999, 1e-15)
        np.testing.assert_allclose(mine[0], p.detach().numpy(), rtol=1e-13, atol=1e-15)
        st = opt.state[p]
        # torch forms m by lerp, a different rounding of the same sum
        np.testing.assert_allclose(mine[1], st["exp_avg"].numpy(), rtol=1e-12, atol=0)
        np.testing.assert_allclose(mine[2], st["exp_avg_sq"].numpy(), rtol=1e-12, atol=0)


def test_adam_first_step_is_signed_lr():
    """At t = 1 with eps -> 0 the bias-corrected step is exactly lr * sign(g)."""
    g = np.array([3.0, -1e-3, 7e5, -2.5])
    p, m, v = O.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01, 0.9, 0.999, 0.0)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


def test_adam_projection_bounds():
    p, _, _ = O.adam_step(np.array([0.001, 0.999, 0.5]), np.array([1.0, -1.0, 0.0]), np.zeros(3), np.zeros(3), 1,
                          0.1, 0.9, 0.999, 1e-15, lo=0.0, hi=1.0)
    assert p[0] == 0.0 and p[1] == 1.0 and p[2] == 0.5


def test_l1_grad_matches_autograd():
    rng = np.random.default_rng(2)
    c = rng.random(1001)
    t = rng.random(1001)
    t[::7] = c[::7]                       # exact ties: sign(0) = 0
    g, loss = O.l1_grad(c, t, 0.25)
    ct = torch.tensor(c, requires_grad=True)
    lt = 0.25 * (ct - torch.tensor(t)).abs().sum()
    lt.backward()
    np.testing.assert_array_equal(g, ct.grad.numpy())
    assert math.isclose(loss, float(lt), rel_tol=1e-14)
