"""Full-size parity: the workloads at their real sizes, in the launch
configuration the benchmark times, against the FP64 CPU reference on seeded
sample nodes.

The reference value at a sample comes from the reference run on a window
around it (tests/_window.py; the window principle itself is pinned on the CPU
by test_oracle_window.py).  Each sample compares the 5^3 block around the
node, scaled by the largest reference magnitude of the field over the
compared blocks (phi: 1; P: also at least rho_heavy T max|u|, the pressure
that a velocity divergence of the flow's own size makes in the heavy phase,
through which the storage rounding of u* reaches P).  Bounds: FP32 storage
2e-5; FP16 shifted storage 1e-3 on phi and P and 2e-3 on u.
"""
import json
import os

import numpy as np
import pytest

from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W

from _window import cone, inner_block, ref_block, sample_centers, window_reference

pytestmark = pytest.mark.gpu

T_LATTICE = 1.0 / 3.0
# per-case records of the GPU runs (one JSON line each)
OUT = os.environ.get("PULBM_RESULTS_DIR",
                     os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "results"))


def _run_gpu(cfg, f, steps):
    c = B.Case(cfg)
    c.init_fields(*f)
    c.step(steps)
    out = c.read_fields()
    d = c.diagnostics()
    c.close()
    assert d["nonfinite"] == 0
    return out


def _check(tag, cfg, f, steps, stores, nsamp, seed, extra=()):
    centers = sample_centers(cfg, f, nsamp, seed) + list(extra)
    refs = [window_reference(cfg, f, c, steps, cone(steps) + 2) for c in centers]
    # field scales from the compared blocks only: outside the dependency cone
    # the window's own edge makes its values meaningless
    scale = [1.0, 0.0, 0.0]
    for ref, axes, pos in refs:
        w = ref_block(ref, axes, pos, 2)
        for k in (1, 2):
            scale[k] = max(scale[k], float(np.abs(w[k]).max()))
    # pressure scale of the flow: the rounding of the stored populations
    # reaches P through (rho - rho_light) T div u*
    scale[1] = max(scale[1], cfg["rho_heavy"] * T_LATTICE * scale[2])
    for store, tol in stores:
        got = _run_gpu(dict(cfg, store=store), f, steps)
        worst = [0.0, 0.0, 0.0]
        for ref, axes, pos in refs:
            g, w = inner_block(got, ref, axes, pos, 2)
            for k in range(3):
                worst[k] = max(worst[k], float(np.abs(g[k] - w[k]).max() / max(scale[k], 1e-300)))
        rec = {"case": tag, "store": store, "steps": steps, "samples": len(centers),
               "max_rel": dict(zip(("phi", "P", "u"), (float(f"{e:.3e}") for e in worst)))}
        print(json.dumps(rec), flush=True)
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, "fullsize.jsonl"), "a") as fh:
            fh.write(json.dumps(rec) + "\n")
        tphi, tP, tu = tol
        assert worst[0] < tphi and worst[1] < tP and worst[2] < tu, rec
        del got


FP32 = (2e-5, 2e-5, 2e-5)
FP16 = (1e-3, 1e-3, 2e-3)


def test_galilean_droplet_128_fp32():
    cfg, f, _ = W.config_galilean_droplet_3d(128)
    _check("galilean_droplet_128", cfg, f, 3, [("fp32", FP32), ("fp16", FP16)], 12, 11)


def test_rising_bubble_256_walls_z():
    cfg, f, _ = W.config_rising_bubble_3d(256, store="fp32")
    _check("rising_bubble_256", cfg, f, 2, [("fp32", FP32), ("fp16", FP16)], 12, 12)


def test_dam_break_512x256x256_all_walls():
    cfg, f, _ = W.config_dam_break_3d()
    _check("dam_break_512x256x256", cfg, f, 2, [("fp16", FP16), ("fp32", FP32)], 12, 13)


def test_dam_break_block_585x182x182_open_top():
    """The dam break against a block in the container of Sec. III: samples
    also at the block's face, top edge and corner, next to the floor beside
    it, and at the open top."""
    cfg, f, _ = W.config_dam_break_block(store="fp16")
    (bx0, by0, _), (bx1, by1, bz1) = cfg["block"]
    nz = cfg["nz"]
    extra = [(bx1, (by0 + by1) // 2, bz1 // 2), (bx1, by0 + 3, bz1), (bx0 - 1, by0 - 1, bz1),
             (bx1 + 1, by1, 0), (300, 91, nz - 1), (450, 20, nz - 1), (438, 100, 99)]
    _check("dam_break_block_585x182x182", cfg, f, 2, [("fp16", FP16), ("fp32", FP32)], 8, 14, extra)

