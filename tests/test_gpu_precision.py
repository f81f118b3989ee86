"""Storage precision layer: FP32, FP16 and BF16 distributions against the FP64
CPU reference on the same seeded inputs.

Errors (relative L2, reported for every mode):
    phi     ||phi - phi_ref|| / ||phi_ref||
    u       ||u - u_ref|| / ||u_ref||
    P       ||dP - dP_ref|| / ||dP_ref||, dP = P - mean(P) (the level of P is
            arbitrary in a periodic box, Sec. I)
    P_flow  ||dP - dP_ref|| / (sqrt(N) * max(max|dP_ref|, rho_heavy T max|u_ref|))
The pressure of the heavy phase contains (rho - rho_light) T times the
divergence of the streamed velocity u* (Sec. II, pressure reconstruction), so
the rounding of the stored populations reaches P multiplied by
rho_heavy T = 333 at density ratio 1000.  P_flow measures the error against
the pressure scale of the flow itself; P against the (possibly much smaller)
pressure variation.  Gates per mode, each raised to 3x the spread of the reference itself (the
reference run from phi0 perturbed by 1e-10 relative, far below FP32
rounding): with noise in phi the delta-theta switches of Sec. II (the sign
of lap(phi), the ramps of width D = 1e-4) make the discrete map
discontinuous, and no arithmetic can stay closer to the reference than the
method's own response to such a perturbation.
    FP32  phi, u, P_flow <= 1e-5
    FP16  phi, u, P_flow <= 1e-3, and P <= 1e-3 on the rising bubbles (the
          slow, buoyancy-driven flows of the FP16 workloads)
    BF16  phi, u, P_flow <= 3e-2 (8-bit mantissa: reported, loosely gated)
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W

pytestmark = pytest.mark.gpu

T_LATTICE = 1.0 / 3.0
# per-case records of the GPU runs (one JSON line each)
OUT = os.environ.get("PULBM_RESULTS_DIR",
                     os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "results"))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def errors(gpu, ref, rho_heavy):
    (pg, Pg, ug), (pr, Pr, ur) = gpu, ref
    dPg, dPr = Pg - Pg.mean(), Pr - Pr.mean()
    pscale = max(np.abs(dPr).max(), rho_heavy * T_LATTICE * np.sqrt((ur ** 2).sum(0)).max())
    return {"phi": rel_l2(pg, pr), "u": rel_l2(ug, ur), "P": rel_l2(dPg, dPr),
            "P_flow": float(np.linalg.norm(dPg - dPr) / (np.sqrt(dPr.size) * pscale))}


def _cases():
    n = 32
    drop = W.base_case(3, n, n, n, sigma=0.005, nu_heavy=0.05, nu_light=0.05, W=4.0)
    # off the grid's symmetry points: where the tails of periodic images meet
    # on a mirror plane, grad phi vanishes exactly with phi away from 0 and the
    # interface normal is set by rounding (see the DESIGN notes on epsilon)
    fd = W.droplet(drop, 8.0, center=(15.3, 16.6, 15.8), u0=(0.05, 0.02, 0.0))
    bub = W.base_case(3, n, n, n, wall=(0, 0, 1), gravity=(0.0, 0.0, -1e-5), sigma=0.01, nu_heavy=0.02,
                      nu_light=0.2, W=5.0)
    phi, P, u = W.droplet(bub, 8.0, center=(15.4, 16.7, 10.3), heavy_inside=False)
    fb = (W.add_noise(phi, 1e-3, 1), P, u)
    d2 = W.base_case(2, 96, 80, wall=(0, 1, 0), gravity=(0.0, -1e-5, 0.0), sigma=0.01, nu_heavy=0.02,
                     nu_light=0.2, W=5.0)
    phi, P, u = W.droplet(d2, 16.0, center=(47.6, 26.3, 0.0), heavy_inside=False)
    f2 = (W.add_noise(phi, 1e-3, 1), P, u)
    return {"galilean_droplet_3d": (drop, fd), "rising_bubble_3d": (bub, fb), "rising_bubble_2d": (d2, f2)}


_REF = {}


def _reference(name, steps, perturb=0.0):
    key = (name, steps, perturb)
    if key not in _REF:
        cfg, f = _cases()[name]
        phi = f[0]
        if perturb:
            rng = np.random.Generator(np.random.PCG64(17))
            phi = phi * (1.0 + perturb * rng.standard_normal(phi.shape))
        o = oracle.OracleCase(dict(cfg, store="fp64"))
        o.init_fields(phi, f[1], f[2])
        o.step(steps)
        _REF[key] = o.read_fields()
    return _REF[key]


def _envelope(name, steps):
    cfg, _ = _cases()[name]
    return errors(_reference(name, steps, 1e-10), _reference(name, steps), cfg["rho_heavy"])


BOUNDS = {"fp32": 1e-5, "fp16": 1e-3, "bf16": 3e-2}


def _gate(name, store, e, env):
    b = {k: max(BOUNDS[store], 3.0 * env[k]) for k in env}
    keys = ["phi", "u", "P_flow"]
    if store == "fp16" and name.startswith("rising_bubble"):
        keys.append("P")
    return all(e[k] <= b[k] for k in keys), b


@pytest.mark.parametrize("store", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("name", ["galilean_droplet_3d", "rising_bubble_3d", "rising_bubble_2d"])
def test_storage_precision_l2(name, store):
    steps = 200
    cfg, f = _cases()[name]
    ref = _reference(name, steps)
    c = B.Case(dict(cfg, store=store))
    c.init_fields(*f)
    c.step(steps)
    got = c.read_fields()
    d = c.diagnostics()
    e = errors(got, ref, cfg["rho_heavy"])
    env = _envelope(name, steps)
    ok, bound = _gate(name, store, e, env)
    rec = {"case": name, "store": store, "steps": steps, **{k: float(f"{v:.3e}") for k, v in e.items()},
           "envelope": {k: float(f"{v:.2e}") for k, v in env.items()}}
    print(json.dumps(rec), flush=True)
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "precision_l2.jsonl"), "a") as fh:
        fh.write(json.dumps(rec) + "\n")
    assert d["nonfinite"] == 0
    assert ok, (rec, bound)
