"""Writes oracle_config0.json: a regression fixture of the FP64 oracle on the
1,024-octahedron 128x128 workload (seed 0).  Calls only the oracle and the
seeded scene generator; rerun only when a change to the oracle's arithmetic
is justified by a passage of the paper."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2501_16312_amd import scenes  # noqa: E402


def main():
    sc, cams = scenes.config0()
    O = oracle.OracleScene(sc, cams, tile=16)
    r = O.render()
    g = scenes.image_gradient(cams, seed=1).astype(np.float64)
    b = O.backward(g)
    rng = np.random.default_rng(123)
    pix = rng.choice(128 * 128, size=48, replace=False)
    prims = rng.choice(sc.n, size=24, replace=False)
    out = {
        "workload": "1,024 octahedra (seed 0), 128x128, 16x16 tiles, black background; dL/dC ~ N(0,1) seed 1",
        "pixels": [int(p) for p in pix],
        "rgb": [[float(r["rgb"][c * 16384 + p]) for c in range(3)] for p in pix],
        "T": [float(r["T"][p]) for p in pix],
        "counts": [int(x) for x in r["counts"][0][:4]],
        "image_sum": float(r["rgb"].sum()),
        "prims": [int(n) for n in prims],
        "grad_means": [[float(x) for x in b["means"][n]] for n in prims],
        "grad_opacity": [float(b["opacity"][n]) for n in prims],
        "grad_sh00": [[float(x) for x in b["sh"][n, 0]] for n in prims],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_config0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
