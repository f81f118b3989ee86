"""Exact invariants of the coupled step, checked on the CPU reference.

Each test pins part of the reference against a property the method must have
whatever its implementation (no retyped formula):

* phi-mass conservation (sum of h is conserved by BGK + streaming +
  bounce-back), periodic and walled;
* uniform states, including uniform translation, are fixed points;
* single phase, periodic: sum u and sum P are conserved; with gravity sum u
  grows by exactly N g per step (telescoping sums of the central stencils);
* absolute-pressure invariance (the paper's motivation, Sec. I): P0 -> P0 + c
  shifts P by c and leaves phi, u unchanged;
* the literal P/u reconstruction equals its compact form, derived from
  (1 + omega) rho_ref / rho = 1 when omega_max = rho_water / rho_air;
* lattice symmetry: transposing the input transposes the output;
* restart: state save / restore reproduces the run bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2512_01027_amd import workloads as W

T = 1.0 / 3.0


def _droplet_case(dim=2, wall=(0, 0, 0), n=24, grav=(0.0, 0.0, 0.0), seed=3):
    cfg = W.base_case(dim, n, n + 4, n - 2 if dim == 3 else 1, wall=wall, gravity=grav,
                      nu_heavy=0.05, nu_light=0.15, sigma=0.01)
    if dim == 3:
        cfg.update(nx=14, ny=16, nz=12)
    phi, P, u = W.droplet(cfg, 4.5 if dim == 3 else 7.0)
    phi = np.clip(phi + W.random_smooth(cfg, seed, amp=0.02), 0, 1)
    for a in range(dim):
        u[a] += W.random_smooth(cfg, seed + 10 + a, amp=0.01)
    P += W.random_smooth(cfg, seed + 20, amp=1e-3)
    return cfg, (phi, P, u)


@pytest.mark.parametrize("dim,wall", [(2, (0, 0, 0)), (2, (1, 1, 0)), (3, (0, 0, 0)),
                                      (3, (1, 0, 1))])
def test_phi_mass_conserved(dim, wall):
    grav = (0.0, -1e-5, 0.0) if dim == 2 else (0.0, 0.0, -1e-5)
    cfg, f = _droplet_case(dim, wall, grav=grav)
    oc = oracle.OracleCase(cfg)
    oc.init_fields(*f)
    m0 = oc.diagnostics()["phi_sum"]
    assert abs(m0 - f[0].sum()) < 1e-12 * m0
    oc.step(60 if dim == 3 else 300)
    d = oc.diagnostics()
    assert d["nonfinite"] == 0
    assert abs(d["phi_sum"] - m0) < 1e-12 * m0


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("phi0", [0.0, 1.0, 0.37])
def test_uniform_translation_is_fixed_point(dim, phi0):
    cfg = W.base_case(dim, 6, 5, 4 if dim == 3 else 1, nu_heavy=0.02, nu_light=0.2)
    shape = (cfg["nz"], cfg["ny"], cfg["nx"])
    U = [0.04, -0.03, 0.02][:dim]
    phi = np.full(shape, phi0)
    P = np.full(shape, 0.123)
    u = np.stack([np.full(shape, U[a]) for a in range(dim)])
    oc = oracle.OracleCase(cfg)
    oc.init_fields(phi, P, u)
    oc.step(40)
    ph, Pr, ur = oc.read_fields()
    assert np.abs(ph - phi0).max() < 1e-14
    assert np.abs(Pr - 0.123).max() < 1e-13
    for a in range(dim):
        assert np.abs(ur[a] - U[a]).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_single_phase_momentum_and_pressure_sums(dim):
    """phi = 0 stays exactly 0 (its advective flux phi u vanishes), so this is a
    true single-phase run.  (phi = 1 is not invariant: the conservative
    advection div(phi u) turns any compressible u into phi != 1.)"""
    phase = 0.0
    n = (10, 9, 8)
    cfg = W.base_case(dim, n[0], n[1], n[2] if dim == 3 else 1, nu_heavy=0.03, nu_light=0.3)
    shape = (cfg["nz"], cfg["ny"], cfg["nx"])
    N = int(np.prod(shape))
    phi = np.full(shape, phase)
    u = np.stack([W.random_smooth(cfg, 40 + a, amp=0.02) for a in range(dim)])
    P = W.random_smooth(cfg, 50, amp=0.01) + 0.2
    oc = oracle.OracleCase(cfg)
    oc.init_fields(phi, P, u)
    _, P0r, u0r = oc.read_fields()
    oc.step(25)
    _, P1, u1 = oc.read_fields()
    assert abs(P1.sum() - P0r.sum()) < 1e-12 * N
    for a in range(dim):
        assert abs(u1[a].sum() - u0r[a].sum()) < 1e-13 * N
    # with gravity: sum u grows by N g per step
    g = [2e-5, -1e-5, 3e-5][:dim] + [0.0] * (3 - dim)
    cfg2 = dict(cfg, gravity=tuple(g))
    oc = oracle.OracleCase(cfg2)
    oc.init_fields(phi, P, u)
    _, _, ua = oc.read_fields()
    oc.step(10)
    _, _, ub = oc.read_fields()
    for a in range(dim):
        assert abs((ub[a].sum() - ua[a].sum()) - 10 * N * g[a]) < 1e-12 * N


@pytest.mark.parametrize("dim", [2, 3])
def test_absolute_pressure_invariance(dim):
    cfg, (phi, P, u) = _droplet_case(dim)
    a = oracle.OracleCase(cfg)
    a.init_fields(phi, P, u)
    b = oracle.OracleCase(cfg)
    b.init_fields(phi, P + 1.0, u)
    a.step(30)
    b.step(30)
    pa, Pa, ua = a.read_fields()
    pb, Pb, ub = b.read_fields()
    assert np.abs(pa - pb).max() < 1e-12
    assert np.abs(ua - ub).max() < 1e-12
    assert np.abs((Pb - Pa) - 1.0).max() < 1e-12


def _shift(q, c):
    """q(x + c) on a periodic grid (nz, ny, nx)."""
    return np.roll(q, shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2))


@pytest.mark.parametrize("dim", [2, 3])
def test_reconstruction_matches_compact_form(dim):
    """P = P* + sum_i w_i [P*(x - c_i) - P*(x)] - (rho - rho_ref) T D.u*, with
    P* = rho_ref T sum g, u = u* - D P / rho, u* = sum g c: the paper's K_i /
    omega form collapses to this when omega_max = rho_water / rho_air, because
    (1 + omega) rho_ref / rho = 1 and sum_i w_i c_i q(x - c_i) = -T D q."""
    cfg, f = _droplet_case(dim)
    oc = oracle.OracleCase(cfg)
    oc.init_fields(*f)
    oc.step(7)
    h, g, Pl, _ = oc.get_state()
    cg, wg = oracle.lattice(dim, cfg["q_hydro"])
    ra, rw = cfg["rho_light"], cfg["rho_heavy"]
    phi = h.sum(0)
    rho = ra + np.clip(phi, 0, 1) * (rw - ra)

    def D(q):
        out = np.zeros((3,) + q.shape)
        for i, c in enumerate(cg):
            d = _shift(q, c) - _shift(q, -c)
            for a in range(3):
                out[a] += wg[i] * c[a] * d
        return out / (2 * T)

    # P first: u* = sum g c at x - c_i in the omega term, K from P* = rho_ref T sum g
    J = np.stack([np.tensordot(cg[:, a], g, axes=(0, 0)) for a in range(dim)])
    Ps = ra * T * g.sum(0)
    Lsum = sum(wg[i] * (_shift(Ps, -c) - Ps) for i, c in enumerate(cg))
    divJ = sum(D(J[a])[a] for a in range(dim))
    P = Ps + Lsum - (rho - ra) * T * divJ
    # then u with K of the new P
    DP = D(P)
    u = np.stack([J[a] - DP[a] / rho for a in range(dim)])
    ph, Pr, ur = oc.read_fields()
    assert np.abs(ph - phi).max() < 1e-15
    assert np.abs(ur - u).max() < 1e-13
    assert np.abs(Pr - P).max() < 1e-12 * max(1.0, np.abs(P).max())


def test_lattice_symmetry_2d_transpose():
    cfg = W.base_case(2, 20, 20, nu_heavy=0.05, nu_light=0.15, gravity=(1e-5, -2e-5, 0.0))
    phi, P, u = W.droplet(cfg, 6.0, center=(8.3, 11.1, 0))
    phi = np.clip(phi + W.random_smooth(cfg, 9, amp=0.02), 0, 1)
    u[0] += W.random_smooth(cfg, 10, amp=0.01)
    u[1] += W.random_smooth(cfg, 11, amp=0.01)
    a = oracle.OracleCase(cfg)
    a.init_fields(phi, P, u)
    a.step(30)
    pa, Pa, ua = a.read_fields()
    cfgT = dict(cfg, gravity=(-2e-5, 1e-5, 0.0))
    tr = lambda q: np.ascontiguousarray(np.swapaxes(q, -1, -2))  # noqa: E731
    b = oracle.OracleCase(cfgT)
    b.init_fields(tr(phi), tr(P), np.stack([tr(u[1]), tr(u[0])]))
    b.step(30)
    pb, Pb, ub = b.read_fields()
    assert np.abs(tr(pb) - pa).max() < 1e-13
    assert np.abs(tr(Pb) - Pa).max() < 1e-13
    assert np.abs(tr(ub[1]) - ua[0]).max() < 1e-13
    assert np.abs(tr(ub[0]) - ua[1]).max() < 1e-13


def test_lattice_symmetry_3d_axis_cycle_with_walls():
    cfg = W.base_case(3, 10, 10, 10, wall=(0, 0, 1), nu_heavy=0.05, nu_light=0.15,
                      gravity=(0.0, 0.0, -1e-5))
    phi, P, u = W.droplet(cfg, 3.5, center=(4.2, 5.3, 4.7))
    for a in range(3):
        u[a] += W.random_smooth(cfg, 20 + a, amp=0.01)
    a = oracle.OracleCase(cfg)
    a.init_fields(phi, P, u)
    a.step(12)
    pa, Pa, ua = a.read_fields()
    # relabel axes (x, y, z) -> (z, x, y): arrays (nz, ny, nx) -> transpose
    perm = lambda q: np.ascontiguousarray(np.transpose(q, (2, 0, 1)))  # noqa: E731
    cfgP = dict(cfg, wall=(0, 1, 0), gravity=(0.0, -1e-5, 0.0))
    b = oracle.OracleCase(cfgP)
    # new (x', y', z') = (y, z, x): new u components (u'_x, u'_y, u'_z) = (u_y, u_z, u_x)
    b.init_fields(perm(phi), perm(P), np.stack([perm(u[1]), perm(u[2]), perm(u[0])]))
    b.step(12)
    pb, Pb, ub = b.read_fields()
    assert np.abs(pb - perm(pa)).max() < 1e-13
    assert np.abs(Pb - perm(Pa)).max() < 1e-12
    assert np.abs(ub[0] - perm(ua[1])).max() < 1e-13
    assert np.abs(ub[1] - perm(ua[2])).max() < 1e-13
    assert np.abs(ub[2] - perm(ua[0])).max() < 1e-13


def test_restart_is_bitwise():
    cfg, f = _droplet_case(2, wall=(0, 1, 0), grav=(0.0, -1e-5, 0.0))
    a = oracle.OracleCase(cfg)
    a.init_fields(*f)
    a.step(40)
    b = oracle.OracleCase(cfg)
    b.init_fields(*f)
    b.step(15)
    st = b.get_state()
    c = oracle.OracleCase(cfg)
    c.set_state(*st)
    c.step(25)
    ra_ = a.read_fields()
    rc_ = c.read_fields()
    for x, y in zip(ra_, rc_):
        assert np.array_equal(x, y)
