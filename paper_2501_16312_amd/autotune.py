"""Autotuner for the rasterizer's launch configuration.

Times the full forward + backward step for each candidate -- screen tile
edge in {8, 16, 32} and the pair sort (per-tile sort, or the global LSD
radix sort with its digit width) -- on the caller's own primitives, cameras
and loss gradient, and keeps the fastest.  Results are cached in memory
and, optionally, in a JSON file, keyed by device, primitive type,
primitive-count bucket and the list of image sizes.

The list walk of the render kernels is batched 64 entries at a time (one
wavefront), so there is no separate batch-depth knob to tune.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional, Sequence

import torch

from . import linprim as L
from .graph import PlainStep
from .render import Rasterizer

# (tile, radix sort?, digit bits)
DEFAULT_CANDIDATES = ((8, False, 8), (16, False, 8), (32, False, 8), (8, True, 8), (16, True, 7))

_memo: dict = {}


def cache_key(kind: int, n: int, cams: Sequence) -> str:
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    bucket = int(math.log2(max(n, 1)))
    sizes = ",".join(f"{c.width}x{c.height}" for c in cams)
    return f"{dev}|{kind}|2^{bucket}|{sizes}"


def _time_config(prims: L.Prims, cams, tile: int, radix: bool, digit: int, grad, bg, reps: int) -> float:
    rast = Rasterizer(prims.kind, prims.n, cams, tile=tile, sort_digit_bits=digit, headroom=1.05, radix_sort=radix)
    step = PlainStep(rast, prims, bg, grad)
    step.run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        step.run()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    del step, rast
    torch.cuda.empty_cache()
    times.sort()
    return times[len(times) // 2]


def autotune(prims: L.Prims, cams: Sequence, grad_rgb: torch.Tensor, bg=None, candidates=DEFAULT_CANDIDATES,
             reps: int = 3, cache_file: Optional[str] = None) -> dict:
    """Returns {"tile": t, "radix_sort": r, "sort_digit_bits": d, "ms": best, "table": {...}}."""
    key = cache_key(prims.kind, prims.n, cams)
    if key in _memo:
        return _memo[key]
    if cache_file and os.path.exists(cache_file):
        with open(cache_file) as f:
            disk = json.load(f)
        if key in disk:
            _memo[key] = disk[key]
            return disk[key]
    table, conf = {}, {}
    for tile, radix, digit in candidates:
        name = f"{tile}/{'radix' + str(digit) if radix else 'tiles'}"
        table[name] = _time_config(prims, cams, tile, radix, digit, grad_rgb, bg, reps)
        conf[name] = (tile, radix, digit)
    best = min(table, key=table.get)
    tile, radix, digit = conf[best]
    res = {"tile": tile, "radix_sort": radix, "sort_digit_bits": digit, "ms": table[best], "table": table}
    _memo[key] = res
    if cache_file:
        disk = {}
        if os.path.exists(cache_file):
            with open(cache_file) as f:
                disk = json.load(f)
        disk[key] = res
        with open(cache_file, "w") as f:
            json.dump(disk, f, indent=1)
    return res
