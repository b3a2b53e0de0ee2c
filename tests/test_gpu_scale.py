"""Prefix paths taken only at large sizes (GPU).

* More than 8192 scan blocks (32M (view, primitive) slots): a single block
  turns the block totals into prefixes before the block-local scans.  The
  pair offsets must equal the exclusive prefix sum of the tile counts and
  the pair count their sum (the definition of the scan, Sec. 3.2 "Global
  Sorting and Tiling").
* More than 256 blocks of tiles in the render orders: images of 40 full-HD
  views rendered in one call equal those rendered one view at a time (the
  orders only schedule waves), the sorted pairs equal the oracle's, and both
  render orders are the documented permutations of the tiles (as with one
  view, where every block computes its own prefix)."""
import numpy as np
import pytest
import torch

from paper_2501_16312_amd import linprim as L
from paper_2501_16312_amd import scenes
from paper_2501_16312_amd.render import Rasterizer

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _ws_view(ws, base, addr, count, dtype, itemsize):
    off = addr - base
    return ws[off: off + count * itemsize].view(dtype)


# list-length classes of the backward order (longest first) and the forward
# order's parts (lists of more than 128 pairs, of more than 72, the others)
ORDER_BOUNDS = np.array([192, 128, 96, 72, 56, 48, 40, 32, 26, 20, 16, 12, 8, 4, 0])


def _check_orders(rast, prims):
    """Both render orders against their definitions, from the tile ranges:
    stable sorts of the tiles by class (backward) and by heaviness (forward)."""
    ptr = L.linprim_debug_pointers(prims, rast.cams_c, rast.tune, rast.view_ws, rast.pair_ws, rast.max_pairs)
    base = rast.view_ws.data_ptr()
    tile = rast.tune.tile
    nt = int(sum(((c.width + tile - 1) // tile) * ((c.height + tile - 1) // tile)
                 for c in rast.cams))
    rg = _ws_view(rast.view_ws, base, ptr["ranges"], 2 * nt, torch.int32, 4).cpu().numpy().view(np.uint32)
    length = (rg[1::2].astype(np.int64) - rg[0::2]).astype(np.int64)
    fwd = _ws_view(rast.view_ws, base, ptr["order_fwd"], nt, torch.int32, 4).cpu().numpy().view(np.uint32)
    bwd = _ws_view(rast.view_ws, base, ptr["order_bwd"], nt, torch.int32, 4).cpu().numpy().view(np.uint32)
    cls = (length[:, None] <= ORDER_BOUNDS[None, :]).sum(1)
    tiles = np.arange(nt)
    assert np.array_equal(bwd, tiles[np.lexsort((tiles, cls))])
    part = (length <= 128).astype(np.int64) + (length <= 72).astype(np.int64)
    assert np.array_equal(fwd, tiles[np.lexsort((tiles, part))])
    _say(f"  orders of {nt} tiles: {int((length > 128).sum())} and {int((length > 72).sum())} lists of more than "
         f"128 and 72 pairs, "
         f"{len(np.unique(cls))} length classes")


def test_scan_beyond_direct_blocks():
    n, views = 1_100_000, 32                    # 35.2M slots -> 8594 scan blocks
    _say(f"scan prefix path: {n} x {views} slots")
    sc = scenes.uniform_octahedra(n, seed=5, box=1.0, dmin=0.002, dmax=0.01)
    cams = [scenes.look_at((3 * np.cos(a), 0.4, 3 * np.sin(a)), (0, 0, 0), 64, 48)
            for a in np.linspace(0, 2 * np.pi, views, endpoint=False)]
    prims = L.Prims.from_scene(sc)
    rast = Rasterizer(sc.kind, sc.n, cams, tile=8)
    n_pairs = rast.preprocess(prims, sync_count=True)
    torch.cuda.synchronize()
    ptr = L.linprim_debug_pointers(prims, rast.cams_c, rast.tune, rast.view_ws, rast.pair_ws, rast.max_pairs)
    base = rast.view_ws.data_ptr()
    vn = n * views
    tiles = _ws_view(rast.view_ws, base, ptr["tiles"], vn, torch.int32, 4).to(torch.int64)
    offs = _ws_view(rast.view_ws, base, ptr["offsets"], vn, torch.int32, 4).to(torch.int64) & 0xFFFFFFFF
    ref = torch.cumsum(tiles, 0) - tiles
    _say(f"  pairs {n_pairs}, visible slots {int((tiles > 0).sum())}")
    assert n_pairs == int(tiles.sum())
    assert torch.equal(offs, ref)
    assert int((tiles > 0).sum()) > 100_000


def test_render_order_beyond_direct_blocks(oracle_mod):
    _say("render order prefix path: 40 x 1920x1080")
    sc = scenes.uniform_octahedra(2000, seed=8, box=1.0, dmin=0.01, dmax=0.08)
    cams = [scenes.look_at((3 * np.cos(a), 0.3, 3 * np.sin(a)), (0, 0, 0), 1920, 1080)
            for a in np.linspace(0, 2 * np.pi, 40, endpoint=False)]
    n_tiles = sum(((c.width + 7) // 8) * ((c.height + 7) // 8) for c in cams)
    assert n_tiles > 256 * 4096          # more than 256 blocks of the largest size (4096 tiles)
    prims = L.Prims.from_scene(sc)
    rast = Rasterizer(sc.kind, sc.n, cams, tile=8)
    rgb, _, _ = rast.forward(prims, (0.1, 0.2, 0.3))
    torch.cuda.synchronize()
    ptr = L.linprim_debug_pointers(prims, rast.cams_c, rast.tune, rast.view_ws, rast.pair_ws, rast.max_pairs)
    pb = rast.pair_ws.data_ptr()
    keys = _ws_view(rast.pair_ws, pb, ptr["keys"], rast.n_pairs, torch.int64, 8).cpu().numpy().view(np.uint64)
    vals = _ws_view(rast.pair_ws, pb, ptr["values"], rast.n_pairs, torch.int32, 4).cpu().numpy().view(np.uint32)
    s = oracle_mod.OracleScene(sc, cams, tile=8).sort()
    _say(f"  pairs {rast.n_pairs}")
    assert np.array_equal(keys, s["keys"])
    assert np.array_equal(vals, s["values"])
    _check_orders(rast, prims)
    # images do not depend on the order in which waves take the tiles
    for k in range(0, len(cams), 13):
        one = Rasterizer(sc.kind, sc.n, [cams[k]], tile=8)
        rgb1, _, _ = one.forward(prims, (0.1, 0.2, 0.3))
        start = 3 * sum(c.width * c.height for c in cams[:k])
        assert torch.equal(rgb[start: start + rgb1.numel()], rgb1)


@pytest.mark.parametrize("n_views", [1, 3])
def test_render_orders_one_view(n_views):
    """Full-HD views whose tiles fit in at most 256 blocks, so that every
    block sums the class counts itself: one view (127 blocks of 256 tiles)
    and three (190 blocks of 512, taken in two rounds), with list lengths from
    0 to several hundred."""
    _say(f"render orders, {n_views} 1920x1080 view(s)")
    sc = scenes.uniform_octahedra(300_000, seed=11, box=1.0, dmin=0.004, dmax=0.05)
    cams = [scenes.look_at((2.2 * np.sin(a), 0.2, 2.2 * np.cos(a)), (0, 0, 0), 1920, 1080)
            for a in np.linspace(0, 2 * np.pi, n_views, endpoint=False)]
    prims = L.Prims.from_scene(sc)
    rast = Rasterizer(sc.kind, sc.n, cams, tile=8)
    rast.forward(prims, (0.0, 0.0, 0.0))
    torch.cuda.synchronize()
    _check_orders(rast, prims)


@pytest.mark.parametrize("n_views", [8, 9])
def test_views_by_value_and_stored(n_views):
    """Up to 8 views travel by value with the preprocessing launch (its first
    block stores them for the later kernels), more are stored by their own
    launch first: on both sides of the limit, a multi-view render equals the
    views rendered one at a time (one view always goes by value)."""
    _say(f"views by value / stored: {n_views} views")
    sc = scenes.uniform_octahedra(20_000, seed=21, box=1.0, dmin=0.005, dmax=0.05)
    cams = [scenes.look_at((2.5 * np.cos(a), 0.4, 2.5 * np.sin(a)), (0, 0, 0), 160 + 8 * k, 96 + 4 * k)
            for k, a in enumerate(np.linspace(0, 2 * np.pi, n_views, endpoint=False))]
    prims = L.Prims.from_scene(sc)
    rast = Rasterizer(sc.kind, sc.n, cams, tile=8)
    rgb, T, last = rast.forward(prims, (0.1, 0.2, 0.3))
    start = 0
    for k, cam in enumerate(cams):
        one = Rasterizer(sc.kind, sc.n, [cam], tile=8)
        rgb1, T1, last1 = one.forward(prims, (0.1, 0.2, 0.3))
        npx = cam.width * cam.height
        assert torch.equal(rgb[3 * start: 3 * (start + npx)], rgb1)
        assert torch.equal(T[start: start + npx], T1)
        start += npx
