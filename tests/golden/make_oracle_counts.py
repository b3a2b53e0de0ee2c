"""Writes oracle_counts.json: the FP64 oracle's pixel-primitive pair counts
(frustum primitives, tile-list length, iterated / evaluated / intersected
pairs) for the measured workloads, the quantities of the paper's Table 7
(App. A), and the oracle's conditioning flags on them.  Calls only the oracle and the seeded scene generator.  The
roofline of the compositing kernels uses these counts as its work units."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2501_16312_amd import scenes  # noqa: E402


def counts(config, tile):
    sc, cams = scenes.CONFIGS[config]()
    O = oracle.OracleScene(sc, cams, tile=tile)
    s = O.sort()
    r = O.render()
    it, ev, hit, fr, amb_hit, amb_term = (int(x) for x in r["counts"].sum(0))
    return {"frustum": fr, "tile_list": int(len(s["keys"])), "iterated": it, "evaluated": ev,
            "intersected": hit, "pixels": int(sum(c.width * c.height for c in cams)),
            # conditioning flags of the parity contract
            "value_flag_pixels": int((r["ill"] & 1).sum()),
            "termination_ambiguous_pixels": amb_term,
            "float32_estimate_above_tolerance_pixels": int(((r["ill"] & 16) != 0).sum()),
            "hit_ambiguous_pairs": amb_hit,
            "float32_value_error_estimate_max": float(r["cond"].max()),
            "float32_value_error_estimate_median_covered": float(np.median(r["cond"][r["T"] < 1]))}


def main():
    out = {"_about": "FP64 oracle pair counts per workload and tile size (written by make_oracle_counts.py)"}
    for config in (0, 1, 2):
        for tile in (8, 16, 32):
            t = time.time()
            out[f"config{config}_tile{tile}"] = counts(config, tile)
            print(config, tile, out[f"config{config}_tile{tile}"], f"{time.time() - t:.1f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_counts.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
