"""Closed-form physics of the paper's validation cases, checked on the CPU
reference (the paper prints no result values; these are the analytic targets
its figures compare against, Sec. III, plus two textbook limits).

* flat interface: the tanh profile is stationary (Eq. AC_eq);
* Laplace's law dP = sigma / R for a 2D static droplet (Sec. III.A);
* Galilean invariance: a droplet translated with U equals the static droplet
  shifted by U t (Sec. III.A);
* shear-wave decay exp(-nu k^2 t) from the momentum equation (Eq. mom_eq);
* two-layer Poiseuille flow against the diffuse-interface steady solution of
  d/dx(rho nu du/dx) = -rho g (Sec. I / III.B);
* hydrostatic rest in a closed box under gravity (walls);
* the delta-theta correction removes a shallow "dense bubble" dip (Sec. II).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2512_01027_amd import workloads as W

T = 1.0 / 3.0
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_cases.json")))


def _run(cfg, fields, steps):
    oc = oracle.OracleCase(cfg)
    oc.init_fields(*fields)
    oc.step(steps)
    return oc


def test_flat_interface_is_stationary():
    cfg = W.base_case(2, 64, 8, nu_heavy=0.1, nu_light=0.1, sigma=0.01)
    phi0, P, u = W.slab(cfg, 16.0, 48.0, axis=0)
    oc = _run(cfg, (phi0, P, u), 2000)
    phi_a, _, _ = oc.read_fields()
    oc.step(1000)
    phi, Pr, ur = oc.read_fields()
    # the discrete profile settles within O(W^-2) of the tanh and then stays put
    assert np.abs(phi - phi0).max() < 1e-2
    assert np.abs(phi - phi_a).max() < 1e-7
    # interface positions (phi = 1/2 crossings) unchanged to 0.05 lattice units
    prof = phi[0, 4]
    xs = [i + (0.5 - prof[i]) / (prof[i + 1] - prof[i]) for i in range(63)
          if (prof[i] - 0.5) * (prof[i + 1] - 0.5) < 0]
    assert len(xs) == 2 and abs(xs[0] - 16.0) < 0.05 and abs(xs[1] - 48.0) < 0.05
    # no pressure jump between the bulk phases of a flat interface (up to the
    # discrete profile's O(1%) of sigma/W), no flow beyond spurious currents
    jump = Pr[phi > 0.99].mean() - Pr[phi < 0.01].mean()
    assert abs(jump) < 0.02 * cfg["sigma"] / cfg["W"]
    assert np.abs(ur).max() < 1e-6


@pytest.mark.parametrize("sigma,collision", [(1e-2, "filter"), (1e-3, "filter"), (1e-2, "bgk")])
def test_laplace_law_2d(sigma, collision):
    """Static droplets R = 10, 12, 14 in 5R periodic boxes with the paper's
    first viscosity set (the BGK collision: nu = 0.1 in both fluids, where it
    is stable at this density ratio); dP averaged over steps 2000-4000 (the
    droplet's slow pressure oscillation)."""
    lap = GOLD["laplace"]
    nus = lap["nu_set1"] if collision == "filter" else {"water": 0.1, "air": 0.1}
    inv_r, dps = [], []
    for R in (10, 12, 14):
        n = lap["domain_factor"] * R
        cfg = W.base_case(2, n, n, sigma=sigma, nu_heavy=nus["water"], nu_light=nus["air"],
                          W=GOLD["common"]["W"], M=GOLD["common"]["M"], collision=collision)
        fields = W.droplet(cfg, float(R), center=(n / 2, n / 2, 0))
        oc = _run(cfg, fields, 2000)
        acc = []
        for _ in range(20):
            oc.step(100)
            phi, P, u = oc.read_fields()
            acc.append(P[phi > 0.99].mean() - P[phi < 0.01].mean())
        assert oc.diagnostics()["nonfinite"] == 0
        dps.append(float(np.mean(acc)))
        inv_r.append(1.0 / R)
        assert abs(dps[-1] - sigma / R) < 0.05 * sigma / R
    slope = np.polyfit(inv_r, dps, 1)[0]
    assert abs(slope - sigma) < 0.05 * sigma


@pytest.mark.parametrize("collision", ["filter", "bgk"])
@pytest.mark.parametrize("phase,nu", [(0.0, 0.1), (0.0, 0.011), (1.0, 0.05)])
def test_shear_wave_decay(phase, nu, collision):
    """Decay rate nu k^2 of a shear wave, for the filter collision and for
    the BGK collision of Eq. BGK_LBeq_hydroeq (both relax with tau_mix)."""
    ny = 64
    cfg = W.base_case(2, 4, ny, nu_heavy=nu, nu_light=nu, collision=collision)
    fields = W.shear_wave(cfg, amp=1e-4, heavy=bool(phase))
    oc = oracle.OracleCase(cfg)
    oc.init_fields(*fields)
    y = np.arange(ny)
    s = np.sin(2 * math.pi * y / ny)
    amps, ts = [], []
    oc.step(100)
    for k in range(6):
        _, _, u = oc.read_fields()
        amps.append((u[0, 0, :, 0] * s).sum() / (s * s).sum())
        ts.append(100 + 300 * k)
        oc.step(300)
    rate = -np.polyfit(ts, np.log(amps), 1)[0]
    kk = 2 * math.pi / ny
    assert abs(rate - nu * kk * kk) < 0.01 * nu * kk * kk


@pytest.mark.parametrize("q_hydro", [27, 19])
def test_shear_wave_decay_3d(q_hydro):
    """Decay rate nu k^2 of a 3D shear wave on either hydrodynamic lattice
    (D3Q27, or D3Q19 as in the paper's 3D runs), heavy phase, nu = 0.05."""
    ny, nu = 32, 0.05
    cfg = W.base_case(3, 4, ny, 4, nu_heavy=nu, nu_light=nu, q_hydro=q_hydro)
    oc = oracle.OracleCase(cfg)
    oc.init_fields(*W.shear_wave(cfg, amp=1e-4, heavy=True))
    s = np.sin(2 * math.pi * np.arange(ny) / ny)
    amps, ts = [], []
    oc.step(50)
    for k in range(5):
        _, _, u = oc.read_fields()
        amps.append((u[0, :, :, :].mean(axis=(0, 2)) * s).sum() / (s * s).sum())
        ts.append(50 + 100 * k)
        oc.step(100)
    rate = -np.polyfit(ts, np.log(amps), 1)[0]
    kk = 2 * math.pi / ny
    assert abs(rate - nu * kk * kk) < 0.01 * nu * kk * kk


def test_filter_collision_is_more_robust_than_bgk():
    """Sec. II adopts the filter collision for robustness: at density ratio
    1000 and nu = 0.03 the BGK collision diverges within 2000 steps on a
    static droplet while the filter collision stays finite."""
    n, R = 50, 10.0
    out = {}
    for collision in ("filter", "bgk"):
        cfg = W.base_case(2, n, n, sigma=0.01, nu_heavy=0.03, nu_light=0.03, collision=collision)
        oc = _run(cfg, W.droplet(cfg, R, center=(n / 2, n / 2, 0)), 2000)
        out[collision] = oc.diagnostics()["nonfinite"]
    assert out["filter"] == 0 and out["bgk"] > 0


def test_galilean_invariance_translated_droplet():
    """Moving droplet = static droplet shifted by U t, with U t a lattice vector."""
    n, R = 48, 10.0
    cfg = W.base_case(2, n, n, sigma=0.01, nu_heavy=0.05, nu_light=0.05)
    U = (0.02, 0.01)
    t = 2400  # U t = (48, 24): a whole number of nodes
    still = _run(cfg, W.droplet(cfg, R, center=(24, 24, 0)), t)
    moving = _run(cfg, W.droplet(cfg, R, center=(24, 24, 0), u0=U), t)
    ps, Ps, us = still.read_fields()
    pm, Pm, um = moving.read_fields()
    shift = lambda q: np.roll(q, shift=(24, 0), axis=(-2, -1))  # noqa: E731
    err = np.linalg.norm(pm - shift(ps)) / np.linalg.norm(ps)
    assert err < 0.02
    # the moving droplet keeps its mass centre on the translated path
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    w = pm[0]
    ang = 2 * math.pi / n
    cx = (math.atan2((w * np.sin(ang * xx)).sum(), (w * np.cos(ang * xx)).sum()) / ang) % n
    cy = (math.atan2((w * np.sin(ang * yy)).sum(), (w * np.cos(ang * yy)).sum()) / ang) % n
    wrap = lambda d: (d + n / 2) % n - n / 2  # noqa: E731
    assert abs(wrap(cx - 24.0)) < 0.25 and abs(wrap(cy - 48.0)) < 0.25
    # velocity stays close to U everywhere
    assert np.abs(um[0] - U[0]).max() < 0.1 * U[0]
    assert np.abs(um[1] - U[1]).max() < 0.1 * U[0]


def test_moving_droplet_paper_settings_one_transit():
    """Sec. III.A's moving droplet at the paper's own settings: R = 16 in an
    80 x 80 periodic box, u_x = 0.025 everywhere, viscosity set 1, sigma =
    1e-3, density ratio 1000.  After 3200 steps (u t = 80, one box length) the
    droplet is back where it started: it matches the static droplet of the
    same age within 2% (relative L2 of phi), stays circular (>= 0.99) and its
    centroid is back at the start.  The full 33,600 steps run on the GPU."""
    from paper_2512_01027_amd import analysis as A

    mc = GOLD["moving_droplet"]
    n, R = mc["L"], float(mc["R"])
    nu = GOLD["laplace"]["nu_set1"]
    cfg = W.base_case(2, n, n, sigma=GOLD["poiseuille"]["sigma"], nu_heavy=nu["water"], nu_light=nu["air"])
    c = (n / 2.0, n / 2.0, 0.0)
    steps = int(round(n / mc["ux"]))
    still = _run(cfg, W.droplet(cfg, R, center=c), steps)
    moving = _run(cfg, W.droplet(cfg, R, center=c, u0=(mc["ux"], 0.0)), steps)
    ps, _, _ = still.read_fields()
    pm, _, um = moving.read_fields()
    assert np.linalg.norm(pm - ps) / np.linalg.norm(ps) < 0.02
    # the droplet is the heavy fluid: its indicator is phi itself
    assert A.circularity(1.0 - pm[0]) >= 0.99
    cx, cy = A.centroid(1.0 - pm[0])
    sx, sy = A.centroid(1.0 - ps[0])
    assert abs(cx - sx) < 0.25 and abs(cy - sy) < 0.25
    assert np.abs(um[0] - mc["ux"]).max() < 0.01 * mc["ux"]


def _diffuse_poiseuille(phi_of_x, rho_w, rho_a, nu_w, nu_a, g, lo, hi, xs):
    """Steady u(x) of d/dx(rho nu du/dx) = -rho g, u(lo) = u(hi) = 0, with rho
    and nu linear in phi (the model's mixing rules)."""
    from scipy.integrate import cumulative_trapezoid

    fine = np.linspace(lo, hi, 40001)
    ph = np.clip(phi_of_x(fine), 0, 1)
    rho = rho_a + ph * (rho_w - rho_a)
    nu = nu_a + ph * (nu_w - nu_a)
    A = -g * cumulative_trapezoid(rho, fine, initial=0.0)
    I1 = cumulative_trapezoid(A / (rho * nu), fine, initial=0.0)
    I2 = cumulative_trapezoid(1.0 / (rho * nu), fine, initial=0.0)
    C = -I1[-1] / I2[-1]
    u = I1 + C * I2
    return np.interp(xs, fine, u)


def test_two_layer_poiseuille():
    pc = GOLD["poiseuille"]
    width = 40  # the paper uses 100; 40 keeps the CPU run short
    cfg = W.base_case(2, width, 4, wall=(1, 0, 0), gravity=(0.0, pc["g"], 0.0),
                      sigma=pc["sigma"], nu_heavy=pc["nu_water"], nu_light=pc["nu_air"])
    xi = (width - 1) / 2.0
    phi0, P, u = W.slab(cfg, -1e9, xi, axis=0)
    oc = _run(cfg, (phi0, P, u), 80000)
    phi, Pr, ur = oc.read_fields()
    prof = ur[1, 0, 1, :]
    xs = np.arange(width, dtype=float)
    ref = _diffuse_poiseuille(lambda x: 0.5 + 0.5 * np.tanh(2 * (xi - x) / cfg["W"]),
                              cfg["rho_heavy"], cfg["rho_light"], pc["nu_water"], pc["nu_air"],
                              pc["g"], -0.5, width - 0.5, xs)
    assert np.abs(ur[0]).max() < 1e-3 * np.abs(ref).max()
    assert np.linalg.norm(prof - ref) / np.linalg.norm(ref) < 0.01


@pytest.mark.parametrize("phase", [0.0, 1.0])
def test_hydrostatic_closed_box(phase):
    g = 1e-5
    cfg = W.base_case(2, 12, 24, wall=(1, 1, 0), gravity=(0.0, -g, 0.0), nu_heavy=0.1,
                      nu_light=0.1)
    shape = (1, 24, 12)
    oc = _run(cfg, (np.full(shape, phase), np.zeros(shape), np.zeros((2,) + shape)), 3000)
    phi, P, u = oc.read_fields()
    rho = cfg["rho_heavy"] if phase else cfg["rho_light"]
    assert np.abs(u).max() < 1e-8
    dPdy = np.diff(P[0], axis=0)
    assert np.abs(dPdy + rho * g).max() < 1e-6 * rho * g
    assert np.abs(np.diff(P[0], axis=1)).max() < 1e-6 * rho * g


def test_delta_theta_removes_dense_bubble():
    """A shallow dip (phi down to 0.9) in the heavy phase: with the correction
    on, the dip is smoothed out several times faster (Sec. II, the text after
    the delta-theta definition)."""
    n = 32
    out = {}
    for dt in (0, 1):
        cfg = W.base_case(2, n, n, delta_theta=dt, nu_heavy=0.1, nu_light=0.1)
        x, y = np.meshgrid(np.arange(n), np.arange(n))
        r2 = (x - 16.0) ** 2 + (y - 16.0) ** 2
        phi = (1.0 - 0.1 * np.exp(-r2 / 16.0))[None]
        oc = _run(cfg, (phi, np.zeros_like(phi), np.zeros((2,) + phi.shape)), 200)
        ph, _, _ = oc.read_fields()
        out[dt] = 1.0 - ph.min()
    assert out[1] < 0.5 * out[0]
