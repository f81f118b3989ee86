"""Head-on binary collision of water droplets in air (Sec. III) at the
paper's Re = 1715 and We = 58.4, in lattice units that keep Re, We and the
air / water viscosity ratio (D3Q19 for both lattices, the paper's 3D
lattice), on a reduced grid:

- FP64 parity with the CPU reference over the first steps of the approach
  (1e-10 relative, or 3x the reference's own spread under a 1e-15
  perturbation of phi0, whichever is larger);
- FP32 and FP16 runs through the collision (3 time units D / U; U D = 3.84,
  nu_water = 2.2e-3, the smallest viscosity at which the step runs this
  collision): the two droplets merge into one, spread into a disc wider than a droplet, no
  value turns non-finite, and phi's mass holds.  The experiment's images are
  not available here, so the run is self-consistency only.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2512_01027_amd import analysis as A
from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W

pytestmark = pytest.mark.gpu

# per-case records of the GPU runs (one JSON line each)
OUT = os.environ.get("PULBM_RESULTS_DIR",
                     os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "results"))
# off the grid's mirror planes, where the interface normal of an exactly
# vanishing gradient would follow rounding
SMALL = dict(D=32.0, U=0.12, grid=(96, 64, 64), offset=(0.37, 0.29, 0.61))


@pytest.mark.parametrize("store,tol,marks", [("fp64", 1e-10, (1, 6, 23)), ("fp32", 2e-5, (1, 2, 3))])
def test_head_on_parity(store, tol, marks):
    """FP32 is compared over the first 6 steps: from step ~7 the approaching
    droplets compress the water to phi = 1 + 1e-3, across the kink of the
    clamped density at phi = 1 (R2) and the delta-theta ramp of width 1e-4
    below it, where FP32 rounding of phi moves the result by 1e-3 within a few
    steps (before that FP32 stays at 5e-7 of the reference)."""
    cfg, f, _ = W.config_head_on_collision(store=store, **SMALL)
    g = B.Case(cfg)
    g.init_fields(*f)
    o = oracle.OracleCase(dict(cfg, store="fp64"))
    o.init_fields(*f)
    rng = np.random.Generator(np.random.PCG64(23))
    p = oracle.OracleCase(dict(cfg, store="fp64"))
    p.init_fields(f[0] * (1.0 + 1e-15 * rng.standard_normal(f[0].shape)), f[1], f[2])
    for s in marks:
        g.step(s)
        o.step(s)
        p.step(s)
        got, ref, per = g.read_fields(), o.read_fields(), p.read_fields()
        scale = [1.0, max(np.abs(ref[1] - ref[1].mean()).max(), 1e-12), max(np.abs(ref[2]).max(), 1e-12)]
        for k, name in enumerate(("phi", "P", "u")):
            err = np.abs(got[k] - ref[k]).max() / scale[k]
            env = np.abs(per[k] - ref[k]).max() / scale[k]
            print(f"{store} +{s} {name} gpu {err:.2e} envelope {env:.2e}", flush=True)
            assert err <= max(tol, 3.0 * env), (store, s, name, err, env)


@pytest.mark.parametrize("store", ["fp32", "fp16"])
def test_head_on_droplets_merge_and_spread(store):
    cfg, f, unit = W.config_head_on_collision(store=store, **SMALL)
    R = SMALL["D"] / 2
    c = B.Case(cfg)
    c.init_fields(*f)
    m0 = c.diagnostics()["phi_sum"]
    c.step(20)  # still approaching: the 8-node gap closes after ~67 steps
    assert A.droplet_count(c.read_fields()[0]) == 2
    series = []
    for k in range(1, 7):
        c.step(unit // 2 - (20 if k == 1 else 0))
        phi, P, u = c.read_fields()
        d = c.diagnostics(allow_diverged=True)
        r, L = A.collision_extent(phi, axis_yz=(32.29, 32.61))
        series.append({"t": k / 2, "droplets": A.droplet_count(phi), "disc_radius_over_R": round(r / R, 3),
                       "length_over_D": round(L / SMALL["D"], 3),
                       "air_speed_over_U": round(A.max_air_speed(phi, u) / SMALL["U"], 3),
                       "nonfinite": d["nonfinite"], "mass_drift": abs(d["phi_sum"] - m0) / m0})
        print(json.dumps(series[-1]), flush=True)
        assert d["nonfinite"] == 0
    c.close()
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "head_on.jsonl"), "a") as fh:
        fh.write(json.dumps({"store": store, **SMALL, "series": series}) + "\n")
    assert any(s["droplets"] == 1 for s in series)
    assert max(s["disc_radius_over_R"] for s in series) > 1.3
    assert all(s["mass_drift"] < 1e-5 for s in series)
