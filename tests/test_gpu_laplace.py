"""Laplace's law on the GPU at the sizes of Sec. III.A: 2D static droplets of
radius R = 8, 12, 16, 20, 24 in 5R periodic boxes, density ratio 1000, FP64
storage, with the paper's first viscosity set and with set 2's water
viscosity under set 1's air viscosity.  dP = mean P(phi > 0.99) - mean
P(phi < 0.01), averaged over steps 4000-8000: the largest droplet's pressure
jump swings by several percent over the first 4000 steps before it settles.
Bounds: each dP within 5% of sigma / R for R >= 12, the fitted slope of dP
against 1/R within 5% of sigma (the paper reports agreement without a
number; the CPU reference test uses the same bounds).

Set 2 itself (air viscosity 5.56e-3) diverges under this reading: the light
phase needs an air viscosity of about 0.025 or more next to a density-ratio-
1000 interface.  It is not run here.
"""
import json
import os

import numpy as np
import pytest

from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W

pytestmark = pytest.mark.gpu

OUT = os.environ.get("PULBM_RESULTS_DIR",
                     os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "results"))
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_cases.json")))


@pytest.mark.parametrize("sigma", [1e-2, 1e-3])
@pytest.mark.parametrize("nus", ["set1", "set2_water_set1_air"])
def test_laplace_law_paper_radii(sigma, nus):
    lap = GOLD["laplace"]
    nu_air = lap["nu_set1"]["air"]
    nu_water = lap["nu_set1"]["water"] if nus == "set1" else lap["nu_set2"]["water"]
    inv_r, dps = [], []
    for R in lap["R"]:
        n = lap["domain_factor"] * R
        cfg = W.base_case(2, n, n, sigma=sigma, nu_heavy=nu_water, nu_light=nu_air,
                          W=GOLD["common"]["W"], M=GOLD["common"]["M"], store="fp64")
        c = B.Case(cfg)
        try:
            c.init_fields(*W.droplet(cfg, float(R), center=(n / 2, n / 2, 0)))
            c.step(4000)
            acc = []
            for _ in range(40):
                c.step(100)
                phi, P, _ = c.read_fields()
                acc.append(P[phi > 0.99].mean() - P[phi < 0.01].mean())
            assert c.diagnostics()["nonfinite"] == 0
        finally:
            c.close()
        dps.append(float(np.mean(acc)))
        inv_r.append(1.0 / R)
    slope = float(np.polyfit(inv_r, dps, 1)[0])
    rec = {"sigma": sigma, "viscosities": nus, "R": lap["R"],
           "dP_over_laplace": [round(d * R / sigma, 4) for d, R in zip(dps, lap["R"])],
           "slope_over_sigma": round(slope / sigma, 4)}
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "laplace.jsonl"), "a") as f:
        f.write(json.dumps(rec) + "\n")
    for d, R in zip(dps, lap["R"]):
        if R >= 12:
            assert abs(d - sigma / R) < 0.05 * sigma / R, rec
    assert abs(slope - sigma) < 0.05 * sigma, rec
