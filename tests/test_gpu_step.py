"""GPU tests of the optimisation step (Sec. 3.4): the L1 loss gradient and
the fused Adam kernel against the FP64 oracle, and the graph-captured
fwd + bwd (+ Adam) step against the same launches made eagerly."""
import sys

import numpy as np
import pytest

from paper_2501_16312_amd import scenes
from tests import gpu_common as GC

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("count", [0, 3, 1027, 3 * 128 * 128 + 1])
def test_l1_grad_parity(torch_cuda, count):
    from oracle import optim as O
    from paper_2501_16312_amd import linprim as L
    torch = torch_cuda
    _say(f"l1_grad count={count}")
    rng = np.random.default_rng(count)
    c = rng.random(count).astype(np.float32)
    t = rng.random(count).astype(np.float32)
    t[::5] = c[::5]                                   # exact ties -> zero gradient
    scale = 2.0 ** -7
    blocks = max((count + 1023) // 1024, 1)
    dc, dt = torch.tensor(c, device="cuda"), torch.tensor(t, device="cuda")
    grad = torch.full((count,), 7.0, device="cuda")
    partial = torch.zeros(blocks, device="cuda")
    L.linprim_l1_grad(dc, dt, scale, grad, partial)
    torch.cuda.synchronize()
    g_ref, loss_ref = O.l1_grad(c, t, scale)
    np.testing.assert_array_equal(grad.cpu().numpy().astype(np.float64), g_ref)   # bit-exact
    loss = float(partial.double().sum())
    assert abs(loss - loss_ref) <= 1e-5 * max(abs(loss_ref), 1e-30) + 1e-12


def _groups(torch, rng, sizes, bounds):
    """Five ragged groups; group 1's arrays start one float past a 16-byte
    boundary (the scalar path), group 4 is an SH-like [n][16][3] array with
    the degree-0 / higher-degree learning-rate split."""
    gs = []
    for k, ((n, (lo, hi)), lr) in enumerate(zip(zip(sizes, bounds), (1.6e-4, 1e-3, 5e-2, 2.5e-3, 2.5e-3))):
        p = rng.uniform(0.0, 1.0, n).astype(np.float32) if lo == 0.0 else rng.normal(size=n).astype(np.float32)
        off = 1 if k == 1 else 0

        def buf(init=None):
            b = torch.zeros(n + off, device="cuda")
            if init is not None:
                b[off:] = torch.tensor(init, device="cuda")
            return b[off:]
        g = {"param": buf(p), "grad": buf(), "exp_avg": buf(), "exp_avg_sq": buf(), "lr": lr, "lo": lo, "hi": hi}
        if k == 4:
            g.update(period=48, head=3, lr_tail=1.25e-4)
        gs.append(g)
    return gs


def _lr_array(g, n):
    if g.get("period", 0) > 0:
        pos = np.arange(n) % g["period"]
        return np.where(pos >= g["head"], g["lr_tail"], g["lr"])
    return g["lr"]


def test_adam_parity(torch_cuda):
    """Three steps over five ragged groups, with and without projection bounds,
    aligned and unaligned, with a two-rate group, against the FP64 oracle;
    the device-side bias correction variant gives bit-identical results."""
    from oracle import optim as O
    from paper_2501_16312_amd import linprim as L
    torch = torch_cuda
    rng = np.random.default_rng(11)
    sizes = [3 * 1001, 4 * 1001, 3 * 1001, 1001, 48 * 1001]
    bounds = [(-np.inf, np.inf), (-np.inf, np.inf), (1e-4, np.inf), (0.0, 1.0), (-np.inf, np.inf)]
    b1, b2, eps = 0.9, 0.999, 1e-15
    ga = _groups(torch, rng, sizes, bounds)
    gb = [{k: (v.clone() if torch.is_tensor(v) else v) for k, v in g.items()} for g in ga]
    ref = [(g["param"].cpu().numpy().astype(np.float64), np.zeros(n), np.zeros(n)) for g, n in zip(ga, sizes)]
    bc = torch.empty(2, device="cuda")
    for step in range(1, 4):
        _say(f"adam step {step}")
        for g, h in zip(ga, gb):
            gr = torch.tensor(rng.normal(size=g["param"].numel()) * 10.0 ** rng.uniform(-6, 1), dtype=torch.float32,
                              device="cuda")
            g["grad"].copy_(gr)
            h["grad"].copy_(gr)
        L.linprim_adam_step(ga, b1, b2, eps, step)
        bcs = L.adam_bias_corrections(b1, b2, step)
        bc.copy_(torch.tensor([float(bcs[0]), float(bcs[1])], dtype=torch.float32))
        L.linprim_adam_step_dev(gb, b1, b2, eps, bc)
        torch.cuda.synchronize()
        for k, (g, h, n) in enumerate(zip(ga, gb, sizes)):
            assert torch.equal(g["param"], h["param"]) and torch.equal(g["exp_avg_sq"], h["exp_avg_sq"])
            lr = _lr_array(g, n)
            # the kernel receives float32 betas and eps: the oracle gets the same numbers
            f1, f2, fe = (float(np.float32(x)) for x in (b1, b2, eps))
            p, m, v = O.adam_step(ref[k][0], g["grad"].cpu().numpy(), ref[k][1], ref[k][2], step, lr, f1, f2,
                                  fe, *(float(np.float32(b)) for b in bounds[k]))
            # FP32 kernel vs FP64 oracle: m, v to float32 rounding; the update
            # lr * m_hat / sqrt(v_hat) is O(lr), so p to a few ulp plus lr * 1e-5
            gp = g["param"].cpu().numpy().astype(np.float64)
            gr64 = g["grad"].cpu().numpy().astype(np.float64)
            m_scale = f1 * np.abs(ref[k][1]) + (1 - f1) * np.abs(gr64)     # m may cancel; v cannot
            assert np.all(np.abs(g["exp_avg"].cpu().numpy() - m) <= 1e-6 * m_scale)
            np.testing.assert_allclose(g["exp_avg_sq"].cpu().numpy(), v, rtol=1e-6, atol=0)
            assert np.all(np.abs(gp - p) <= 4 * np.spacing(np.abs(p).astype(np.float32)) + lr * 1e-5)
            # the bounds reach the kernel as float32
            assert np.all(gp >= np.float32(bounds[k][0])) and np.all(gp <= np.float32(bounds[k][1]))
            ref[k] = (gp, g["exp_avg"].cpu().numpy().astype(np.float64), g["exp_avg_sq"].cpu().numpy().astype(np.float64))


def _small_scene(n=1500, seed=21):
    """Octahedra in [-1,1]^3 seen from distance 4 on an uneven 200x136 image
    (ragged last tile row and column at tiles 8 and 16)."""
    sc = scenes.uniform_octahedra(n, seed=seed, dmin=0.03, dmax=0.2)
    cams = [scenes.look_at((0.3, -0.2, -4.0), (0.0, 0.0, 0.0), 200, 136)]
    return sc, cams


@pytest.mark.parametrize("tile", [8, 16])
def test_graph_replay_matches_eager(torch_cuda, tile):
    """Replays of the captured step equal the eager step bit for bit, with
    unrelated eager work and synchronisations between the replays."""
    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd.graph import CapturedStep, PlainStep
    from paper_2501_16312_amd.render import Rasterizer
    torch = torch_cuda
    _say(f"graph replay tile={tile}")
    sc, cams = _small_scene()
    prims = L.Prims.from_scene(sc)
    npx = sum(c.width * c.height for c in cams)
    grad = torch.tensor(scenes.image_gradient(cams, seed=4), device="cuda")
    bg = (0.1, 0.2, 0.3)
    eager = PlainStep(Rasterizer(sc.kind, sc.n, cams, tile=tile), prims, bg, grad)
    eager.run()
    torch.cuda.synchronize()
    cap = CapturedStep(Rasterizer(sc.kind, sc.n, cams, tile=tile), prims, bg, grad_rgb=grad)
    for r in range(3):
        for t in list(cap.outs) + list(cap.grads.values()):
            t.fill_(0)
        junk = torch.randn(1 << 20, device="cuda")
        junk = (junk * 2).sum()
        torch.cuda.synchronize()
        cap.replay()
        torch.cuda.synchronize()
        assert cap.check() == eager.rast.n_pairs
        for a, b in zip(cap.outs, eager.outs):
            assert torch.equal(a, b), f"replay {r}: image differs"
        for k in eager.grads:
            assert torch.equal(cap.grads[k], eager.grads[k]), f"replay {r}: grad {k} differs"
    assert npx == cap.outs[1].numel()


@pytest.mark.parametrize("loss", ["l1", "l1_ssim"])
def test_captured_training_step_matches_eager(torch_cuda, loss):
    """Loss gradient + Adam inside the graph: three replays follow the eager
    sequence (fwd, loss gradient, bwd, Adam) step for step, bit for bit,
    for the mean L1 and for 3DGS's L1 + SSIM."""
    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd.graph import CapturedStep
    from paper_2501_16312_amd.render import Rasterizer
    torch = torch_cuda
    sc, cams = _small_scene(1200, seed=8)
    target_scene = sc.copy()
    target_scene.means = target_scene.means + np.float32(0.01)
    tp = L.Prims.from_scene(target_scene)
    tr = Rasterizer(sc.kind, sc.n, cams, tile=16)
    target = tr.forward(tp, None)[0].clone()

    def make(prims):
        grads = {k: torch.zeros_like(getattr(prims, k)) for k in ("means", "quats", "dists", "opacity", "sh")}
        lrs = {"means": 1.6e-4, "quats": 1e-3, "dists": 5e-3, "opacity": 2.5e-2, "sh": 2.5e-3}
        bounds = {"dists": (1e-4, np.inf), "opacity": (0.0, 1.0)}
        groups = [{"param": getattr(prims, k), "grad": grads[k], "exp_avg": torch.zeros_like(grads[k]),
                   "exp_avg_sq": torch.zeros_like(grads[k]), "lr": lrs[k],
                   "lo": bounds.get(k, (-np.inf, np.inf))[0], "hi": bounds.get(k, (-np.inf, np.inf))[1]}
                  for k in grads]
        return grads, groups

    pa = L.Prims.from_scene(sc)
    pb = L.Prims.from_scene(sc)
    ga, groups_a = make(pa)
    gb, groups_b = make(pb)
    scale = 1.0 / target.numel()
    b1, b2, eps = 0.9, 0.999, 1e-15
    # eager reference
    ra = Rasterizer(sc.kind, sc.n, cams, tile=16, headroom=1.5)
    ra.preprocess(pa)
    outs = ra.alloc_outputs()
    g_rgb = torch.empty_like(outs[0])
    part = torch.zeros((outs[0].numel() + 1023) // 1024, device="cuda")
    lws = torch.empty(L.linprim_loss_workspace_size(ra.cams_c), dtype=torch.uint8, device="cuda")
    # captured
    cap = CapturedStep(Rasterizer(sc.kind, sc.n, cams, tile=16), pb, None, target=target, l1_scale=scale,
                       adam={"groups": groups_b, "beta1": b1, "beta2": b2, "eps": eps}, headroom=1.5, grads=gb,
                       loss=loss)
    for step in range(1, 4):
        _say(f"captured training step {step}")
        L.linprim_preprocess(pa, ra.cams_c, ra.tune, ra.view_ws)
        ra.bin_sort(pa)
        ra.render(pa, None, out=outs)
        if loss == "l1_ssim":
            L.linprim_loss_grad(outs[0], target, ra.cams_c, lws, g_rgb)
        else:
            L.linprim_l1_grad(outs[0], target, scale, g_rgb, part)
        L.linprim_raster_bwd(pa, ra.cams_c, ra.tune, None, ra.view_ws, ra.pair_ws, ra.max_pairs, outs[1], outs[2],
                             g_rgb)
        L.linprim_preprocess_bwd(pa, ra.cams_c, ra.tune, ra.view_ws, ra.pair_ws, ra.max_pairs, ga)
        L.linprim_adam_step(groups_a, b1, b2, eps, step)
        cap.replay()
        torch.cuda.synchronize()
        cap.check()
        assert torch.equal(outs[0], cap.outs[0]), f"step {step}: image differs"
        for k in ("means", "quats", "dists", "opacity", "sh"):
            assert torch.equal(getattr(pa, k), getattr(pb, k)), f"step {step}: {k} differs"
        eager_loss = L.linprim_loss_value(lws, ra.cams_c) if loss == "l1_ssim" else float(part.sum())
        assert eager_loss == cap.loss() and eager_loss > 0


def test_graph_replay_new_views(torch_cuda):
    """A graph captured on one set of camera poses, replayed after
    set_views() with another, equals eager launches on the new poses."""
    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd.graph import CapturedStep, PlainStep
    from paper_2501_16312_amd.render import Rasterizer
    torch = torch_cuda
    sc, _ = _small_scene(1300, seed=5)
    pos_a = [(0.3, -0.2, -4.0), (4.0, 0.5, 0.2)]
    pos_b = [(-0.5, 0.4, -3.5), (3.0, -1.0, 2.0)]
    cams_a = [scenes.look_at(p, (0.0, 0.0, 0.0), w, h) for p, (w, h) in zip(pos_a, [(120, 88), (64, 100)])]
    cams_b = [scenes.look_at(p, (0.0, 0.0, 0.0), w, h) for p, (w, h) in zip(pos_b, [(120, 88), (64, 100)])]
    prims = L.Prims.from_scene(sc)
    grad = torch.tensor(scenes.image_gradient(cams_a, seed=12), device="cuda")
    rast = Rasterizer(sc.kind, sc.n, cams_a, tile=8, views_resident=True, headroom=3.0)
    cap = CapturedStep(rast, prims, None, grad_rgb=grad, headroom=3.0)
    for r, cams in enumerate([cams_b, cams_a, cams_b]):
        _say(f"replay on new views {r}")
        rast.set_views(cams)
        cap.replay()
        torch.cuda.synchronize()
        cap.check()
        eager = PlainStep(Rasterizer(sc.kind, sc.n, cams, tile=8), prims, None, grad)
        eager.run()
        torch.cuda.synchronize()
        for a, b in zip(cap.outs, eager.outs):
            assert torch.equal(a, b), f"replay {r}: image differs"
        for k in eager.grads:
            assert torch.equal(cap.grads[k], eager.grads[k]), f"replay {r}: grad {k} differs"


@pytest.mark.parametrize("loss", ["l1", "l1_ssim"])
def test_captured_step_overflow_changes_nothing(torch_cuda, loss):
    """A replay whose (tile, primitive) pairs exceed the pair capacity leaves
    the parameters and the Adam moments unchanged; check() reports it after
    later, valid replays too (the flag is sticky) until clear()."""
    from paper_2501_16312_amd import linprim as L
    from paper_2501_16312_amd.graph import CapturedStep
    from paper_2501_16312_amd.render import Rasterizer
    torch = torch_cuda
    _say(f"captured step overflow loss={loss}")
    sc, cams = _small_scene(1200, seed=8)
    near = [scenes.look_at((0.15, -0.1, -2.0), (0.0, 0.0, 0.0), cams[0].width, cams[0].height)]
    target_scene = sc.copy()
    target_scene.means = target_scene.means + np.float32(0.01)
    target = Rasterizer(sc.kind, sc.n, cams, tile=16).forward(L.Prims.from_scene(target_scene), None)[0].clone()
    probe = Rasterizer(sc.kind, sc.n, near, tile=16)
    probe.forward(L.Prims.from_scene(sc), None)
    prims = L.Prims.from_scene(sc)
    grads = {k: torch.zeros_like(getattr(prims, k)) for k in ("means", "quats", "dists", "opacity", "sh")}
    groups = [{"param": getattr(prims, k), "grad": grads[k], "exp_avg": torch.zeros_like(grads[k]),
               "exp_avg_sq": torch.zeros_like(grads[k]), "lr": 1e-3} for k in grads]
    rast = Rasterizer(sc.kind, sc.n, cams, tile=16, views_resident=True)
    cap = CapturedStep(rast, prims, None, target=target, l1_scale=1.0 / target.numel(),
                       adam={"groups": groups, "beta1": 0.9, "beta2": 0.999, "eps": 1e-15}, headroom=1.2,
                       grads=grads, loss=loss)
    # (the updates move the primitives, so the pair count drifts a little
    # from step to step: the capacity keeps 20% headroom)
    assert probe.n_pairs > rast.max_pairs, (probe.n_pairs, rast.max_pairs)

    def snapshot():
        return [t.clone() for g in groups for t in (g["param"], g["exp_avg"], g["exp_avg_sq"])]

    cap.replay()
    torch.cuda.synchronize()
    cap.check()
    before = snapshot()
    rast.set_views(near)
    cap.replay()
    torch.cuda.synchronize()
    after = snapshot()
    assert all(torch.equal(a, b) for a, b in zip(before, after)), "an overflowed step changed the parameters"
    with pytest.raises(L.LinPrimError):
        cap.check()
    rast.set_views(cams)
    cap.replay()
    torch.cuda.synchronize()
    assert not torch.equal(prims.means, before[0]), "the valid step after the overflow did not update"
    with pytest.raises(L.LinPrimError):
        cap.check()                      # sticky
    cap.clear()
    cap.replay()
    torch.cuda.synchronize()
    cap.check()
