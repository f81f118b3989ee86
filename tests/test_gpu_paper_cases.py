"""The paper's own fully parameterised validation cases, at its own settings,
run in FP64 on the GPU through the C ABI:

- the moving droplet of Sec. III.A (R = 16 in an 80 x 80 periodic box,
  u_x = 0.025, viscosity set 1, sigma = 1e-3, density ratio 1000) to the
  paper's snapshots at 32,000 and 33,600 steps: the droplet "remains
  circular" (circularity >= 0.99, the paper's claim), and its centroid is
  within 0.2% of the distance travelled (800 and 840 nodes) of the static
  droplet of the same age moved by u t; the relative L2 difference of phi
  from that moved droplet is recorded (a lag of a fraction of a node over
  ten box lengths gives several per cent) and held below 10%; the first 100
  steps against the CPU reference;
- the two-layer Poiseuille flow of Sec. I / III.B in a channel of width 100
  (water on one half, air on the other, g = 5e-7 along the channel, set 1,
  sigma = 1e-3) run to its steady state: within 1% of the diffuse-interface
  steady solution of d/dx(rho nu du/dx) = -rho g and within 10% of the
  sharp-interface analytic profile (the diffuse-interface solution itself is
  7.6% from the sharp one at W = 4: on the air side next to the interface
  the mixture is still viscous water); the first 100 steps against the CPU
  reference.

Each test writes one JSON line of its figures to the results directory.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2512_01027_amd import analysis as A
from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W
from test_oracle_physics import GOLD, _diffuse_poiseuille

pytestmark = pytest.mark.gpu

OUT = os.environ.get("PULBM_RESULTS_DIR",
                     os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "results"))


def _record(name, rec):
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "paper_cases.jsonl"), "a") as f:
        f.write(json.dumps({"test": name, **rec}) + "\n")


def _prefix_parity(cfg, f, steps=100):
    """GPU against the reference after `steps` steps: 1e-10 relative, or 3x
    the reference's own spread under a 1e-15 relative perturbation of phi0
    (the interface normal's epsilon amplifies rounding where grad phi ~ 0).
    P is measured against the flow's pressure scale, max(|P - mean P|,
    rho_heavy T max|u|): where P hardly varies (the channel), the heavy
    phase's pressure carries rho_heavy T times the velocity's rounding."""
    g = B.Case(cfg)
    g.init_fields(*f)
    g.step(steps)
    o = oracle.OracleCase(cfg)
    o.init_fields(*f)
    o.step(steps)
    rng = np.random.Generator(np.random.PCG64(31))
    p = oracle.OracleCase(cfg)
    p.init_fields(f[0] * (1.0 + 1e-15 * rng.standard_normal(f[0].shape)), f[1], f[2])
    p.step(steps)
    got, ref, per = g.read_fields(), o.read_fields(), p.read_fields()
    out = {}
    pflow = cfg["rho_heavy"] / 3.0 * np.sqrt((ref[2] ** 2).sum(axis=0)).max()
    for k, name in enumerate(("phi", "P", "u")):
        scale = max(np.abs(ref[k] - (ref[k].mean() if k == 1 else 0.0)).max(), pflow if k == 1 else 0.0, 1e-12)
        err = float(np.abs(got[k] - ref[k]).max() / scale)
        env = float(np.abs(per[k] - ref[k]).max() / scale)
        out[name] = {"err": err, "envelope": env}
        assert err <= max(1e-10, 3.0 * env), (name, err, env)
    return out


def test_moving_droplet_paper_settings():
    mc = GOLD["moving_droplet"]
    n, R, ux = mc["L"], float(mc["R"]), mc["ux"]
    nu = GOLD["laplace"]["nu_set1"]
    cfg = W.base_case(2, n, n, sigma=GOLD["poiseuille"]["sigma"], nu_heavy=nu["water"], nu_light=nu["air"],
                      store="fp64")
    c = (n / 2.0, n / 2.0, 0.0)
    fm = W.droplet(cfg, R, center=c, u0=(ux, 0.0))
    fs = W.droplet(cfg, R, center=c)
    parity = _prefix_parity(cfg, fm)
    mv = B.Case(cfg)
    mv.init_fields(*fm)
    st = B.Case(cfg)
    st.init_fields(*fs)
    rec = {"parity_100_steps": parity, "snapshots": []}
    done = 0
    for steps in mc["steps"]:
        mv.step(steps - done)
        st.step(steps - done)
        done = steps
        pm, _, um = mv.read_fields()
        ps, _, _ = st.read_fields()
        shift = int(round(ux * steps)) % n
        # the moving droplet brought back by u t (whole nodes), so that the
        # box edge does not cut it, against the static one
        back = np.roll(pm, -shift, axis=-1)
        drift = float(np.linalg.norm(back - ps) / np.linalg.norm(ps))
        circ = float(A.circularity(1.0 - back[0]))
        cx = A.centroid(1.0 - back[0])[0]
        sx = A.centroid(1.0 - ps[0])[0]
        d = mv.diagnostics()
        rec["snapshots"].append({"step": steps, "shift": shift, "drift_vs_static": drift, "circularity": circ,
                                 "centroid_x_error": float(cx - sx),
                                 "ux_range": [float(um[0].min()), float(um[0].max())],
                                 "phi_mass_rel_drift": float((d["phi_sum"] - fm[0].sum()) / fm[0].sum())})
        print(rec["snapshots"][-1], flush=True)
        assert d["nonfinite"] == 0
        assert circ >= 0.99
        assert abs(rec["snapshots"][-1]["centroid_x_error"]) < 0.002 * ux * steps
        assert drift < 0.10
    _record("moving_droplet_paper_settings", rec)


def _sharp_poiseuille(width, h, g, nu_w, nu_a, rho_w, rho_a, xs):
    """Steady two-layer channel flow with a sharp interface: walls half a link
    outside the first and last node (at -1/2 and width - 1/2), water in
    [-1/2, h], air in [h, width - 1/2]; u'' = -g / nu in each layer, u = 0 at
    the walls, u and rho nu u' continuous at the interface."""
    x0, x1 = -0.5, width - 0.5
    # water: u = -g (x - x0)^2 / (2 nu_w) + a (x - x0); air: u = -g (x - x1)^2 / (2 nu_a) + b (x - x1)
    hw, ha = h - x0, h - x1
    M = np.array([[hw, -ha], [rho_w * nu_w, -rho_a * nu_a]])
    rhs = np.array([g * hw * hw / (2 * nu_w) - g * ha * ha / (2 * nu_a),
                    rho_w * nu_w * (g * hw / nu_w) - rho_a * nu_a * (g * ha / nu_a)])
    a, b = np.linalg.solve(M, rhs)
    return np.where(xs <= h, -g * (xs - x0) ** 2 / (2 * nu_w) + a * (xs - x0),
                    -g * (xs - x1) ** 2 / (2 * nu_a) + b * (xs - x1))


def test_two_layer_poiseuille_width_100():
    pc = GOLD["poiseuille"]
    width = pc["width"]
    cfg = W.base_case(2, width, 4, wall=(1, 0, 0), gravity=(0.0, pc["g"], 0.0), sigma=pc["sigma"],
                      nu_heavy=pc["nu_water"], nu_light=pc["nu_air"], store="fp64")
    xi = (width - 1) / 2.0
    f = W.slab(cfg, -1e9, xi, axis=0)
    parity = _prefix_parity(cfg, f)
    c = B.Case(cfg)
    c.init_fields(*f)
    # the water layer's slowest mode decays at nu_w (pi / width)^2 per step
    # (about 1.1e-5): 900k steps leave 6e-5 of the start
    steps = 900_000
    c.step(steps)
    phi, P, u = c.read_fields()
    assert c.diagnostics()["nonfinite"] == 0
    prof = u[1, 0, 1, :]
    xs = np.arange(width, dtype=float)
    diffuse = _diffuse_poiseuille(lambda x: 0.5 + 0.5 * np.tanh(2 * (xi - x) / cfg["W"]),
                                  cfg["rho_heavy"], cfg["rho_light"], pc["nu_water"], pc["nu_air"],
                                  pc["g"], -0.5, width - 0.5, xs)
    sharp = _sharp_poiseuille(width, xi, pc["g"], pc["nu_water"], pc["nu_air"], cfg["rho_heavy"],
                              cfg["rho_light"], xs)
    e_diff = float(np.linalg.norm(prof - diffuse) / np.linalg.norm(diffuse))
    e_sharp = float(np.linalg.norm(prof - sharp) / np.linalg.norm(sharp))
    ux_max = float(np.abs(u[0]).max())
    rec = {"parity_100_steps": parity, "steps": steps, "rel_l2_vs_diffuse": e_diff, "rel_l2_vs_sharp": e_sharp,
           "u_peak": float(prof.max()), "ux_max": ux_max}
    print(rec, flush=True)
    _record("two_layer_poiseuille_width_100", rec)
    assert ux_max < 1e-3 * np.abs(diffuse).max()
    assert e_diff < 0.01
    assert e_sharp < 0.10
