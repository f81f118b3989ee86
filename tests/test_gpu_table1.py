"""The 2D rising bubble of Sec. III.D, Table I cases 1 (density ratio 10,
We = 10) and 2 (ratio 1000, We = 125), at full size (200 x 400).

- FP64 parity with the CPU reference after 100 steps (1e-10 relative, or
  the reference's own spread under a 1e-15 perturbation);
- a longer GPU run in FP32 (0.2 time units of sqrt(2R/g), ~17k steps) with
  the benchmark's diagnostics: phi mass kept to 1e-6, the bubble rises
  (centroid and rise velocity up), circularity at most 1.  The benchmark's reference
  values are not available here, so the long run is self-consistency only.
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


@pytest.mark.parametrize("case", [1, 2])
def test_table1_fp64_parity(case):
    """FP64 against the reference after 100 steps, within 1e-10 relative or 3x
    the reference's own spread under a 1e-15 relative perturbation of phi0,
    whichever is larger.  In these closed boxes gravity compresses phi to
    1 +- 1e-6 in the bulk, on the delta-theta ramp F((1 - phi) / D) of slope
    1e4 (Sec. II), and the reference itself moves by ~2e-7 under such a
    perturbation within tens of steps."""
    cfg, f, _ = W.config_table1_bubble(case, "fp64")
    steps = 100
    g = B.Case(cfg)
    g.init_fields(*f)
    g.step(steps)
    o = oracle.OracleCase(cfg)
    o.init_fields(*f)
    o.step(steps)
    rng = np.random.Generator(np.random.PCG64(21))
    p = oracle.OracleCase(cfg)
    p.init_fields(f[0] * (1.0 + 1e-15 * rng.standard_normal(f[0].shape)), f[1], f[2])
    p.step(steps)
    got, ref, per = g.read_fields(), o.read_fields(), p.read_fields()
    scale = [1.0, max(np.abs(ref[1] - ref[1].mean()).max(), 1e-12), max(np.abs(ref[2]).max(), 1e-12)]
    rec = {"test": f"table1_case{case}_fp64_parity", "steps": steps}
    ok = []
    for k, name in enumerate(("phi", "P", "u")):
        err = np.abs(got[k] - ref[k]).max() / scale[k]
        env = np.abs(per[k] - ref[k]).max() / scale[k]
        print(name, f"gpu {err:.2e} envelope {env:.2e}", flush=True)
        rec[f"{name}_err"], rec[f"{name}_envelope"] = float(f"{err:.3e}"), float(f"{env:.3e}")
        ok.append((name, err, env))
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "parity.jsonl"), "a") as fh:
        fh.write(json.dumps(rec) + "\n")
    for name, err, env in ok:
        assert err <= max(1e-10, 3.0 * env), (name, err, env)


@pytest.mark.parametrize("case", [1, 2])
def test_table1_bubble_rises(case):
    cfg, f, unit = W.config_table1_bubble(case, "fp32")
    c = B.Case(cfg)
    c.init_fields(*f)
    m0 = c.diagnostics()["phi_sum"]  # phi as stored (FP32), step 0
    y0 = A.centroid(f[0][0])[1]
    steps = int(0.2 * unit)
    c.step(steps)
    phi, P, u = c.read_fields()
    d = c.diagnostics()
    yc = A.centroid(phi[0])[1]
    vy = A.rise_velocity(phi[0], u[:, 0])[1]
    circ = A.circularity(phi[0])
    rec = {"case": case, "steps": steps, "t": 0.2, "centroid_y": yc, "rise_velocity": vy,
           "rise_velocity_over_Ug": vy / np.sqrt(2 * 50.0 * 1.36e-8), "circularity": circ,
           "phi_mass_drift": abs(d["phi_sum"] - m0) / m0}
    print(json.dumps(rec), flush=True)
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "table1.jsonl"), "a") as fh:
        fh.write(json.dumps(rec) + "\n")
    assert d["nonfinite"] == 0
    # the remaining drift is the rounding of one stored population per node
    # and step (1.2e-7 over these 17k steps); before the rest population was
    # taken as the mass balance, the FP32 weights (sum 1 + 7.5e-9 on D2Q9) gave
    # 1.3e-4
    assert rec["phi_mass_drift"] < 1e-6
    assert yc > y0 and vy > 0
    assert circ <= 1.0 + 5e-3
