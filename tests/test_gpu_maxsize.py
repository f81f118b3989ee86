"""Parity at the largest grid the library accepts: 1024 x 1024 x 511 nodes in
FP32 storage (535,822,336 nodes; one field of 4-byte values is 2,143,289,344
bytes, just under the 2^31-byte reach of the kernels' 32-bit offsets; about
139 GB of device memory).  The z extent is odd, so the last tile layer is
ragged.  The next size up is rejected before anything is allocated
(test_abi).

A droplet whose interface crosses all three pairs of periodic faces is
translated for 3 steps.  The GPU fields are compared with the FP64 CPU
reference on windows around sample nodes: on the interface where it crosses
the faces, at the grid's corners (where periodic neighbours lie farthest
apart in memory) and in the bulk.  Bound: FP32 storage 2e-5 of each field's
scale over the compared blocks (P: at least rho_heavy T max|u|).
"""
import gc
import json
import os

import numpy as np
import pytest

from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W

from _window import cone, inner_block, ref_block, window_reference

pytestmark = pytest.mark.gpu

T_LATTICE = 1.0 / 3.0
OUT = os.environ.get("PULBM_RESULTS_DIR",
                     os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "results"))


def _samples(cfg, center, R):
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    cx, cy, cz = (int(round(v)) for v in center)
    wrap = lambda v, n: int(round(v)) % n  # noqa: E731
    return [(wrap(cx + R, nx), cy, cz), (wrap(cx - R, nx), cy, cz),
            (cx, wrap(cy - R, ny), cz), (cx, wrap(cy + R, ny), cz),
            (cx, cy, wrap(cz + R, nz)), (cx, cy, wrap(cz - R, nz)),
            (0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny - 1, 0), (nx - 1, 0, nz - 1),
            (nx // 2, ny // 2, nz // 2), (nx // 5, (4 * ny) // 5, nz // 5)]


def _compare(cfg, refs, got):
    scale = [1.0, 0.0, 0.0]
    for ref, axes, pos in refs:
        w = ref_block(ref, axes, pos, 2)
        for k in (1, 2):
            scale[k] = max(scale[k], float(np.abs(w[k]).max()))
    scale[1] = max(scale[1], cfg["rho_heavy"] * T_LATTICE * scale[2])
    worst = [0.0, 0.0, 0.0]
    for ref, axes, pos in refs:
        g, w = inner_block(got, ref, axes, pos, 2)
        for k in range(3):
            worst[k] = max(worst[k], float(np.abs(g[k] - w[k]).max() / scale[k]))
    return worst


def test_max_grid_fp32_droplet_across_faces():
    R = 40.0
    cfg, f, center = W.config_droplet_max_grid("fp32", R=R)
    wrap = lambda v, n: int(round(v)) % n  # noqa: E731
    centers = _samples(cfg, center, R)
    steps = 3
    refs = [window_reference(cfg, f, c, steps, cone(steps) + 2) for c in centers]
    c = B.Case(cfg)
    try:
        c.init_fields(*f)
        c.step(steps)
        d = c.diagnostics()
        got = c.read_fields()
    finally:
        c.close()
    del f
    gc.collect()
    assert d["nonfinite"] == 0
    worst = _compare(cfg, refs, got)
    rec = {"case": "droplet_max_grid_1024x1024x511", "store": "fp32", "steps": steps, "samples": len(centers),
           "max_rel": dict(zip(("phi", "P", "u"), (float(f"{e:.3e}") for e in worst)))}
    print(json.dumps(rec), flush=True)
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "fullsize.jsonl"), "a") as fh:
        fh.write(json.dumps(rec) + "\n")
    assert max(worst) < 2e-5, rec
