"""The CPU reference pinned by brute force: a second FP64 implementation of the
whole step (``oracle/twin.py``: NumPy whole-grid arrays, ghost-padded fields,
streaming by rolls) reproduces it on tiny grids, periodic and walled, in 2D and
3D, with both hydrodynamic collisions, over 20 steps; and the reference's
conservation diagnostics equal plain NumPy sums of the fields it reads back.

Error measure: max |twin - reference| over the grid, relative to the largest
|reference| value the field takes over the run (the step's transients decay
the fields by 20x in 20 steps, and rounding differences of the early, larger
values are what remains), at most 1e-12.
"""
import numpy as np
import pytest

import oracle
from oracle.twin import Twin
from paper_2512_01027_amd import workloads as W

TOL = 1e-12


def _fields(cfg, seed=3):
    dim = cfg["dim"]
    phi, P, u = W.droplet(cfg, 0.3 * min(cfg["nx"], cfg["ny"]))
    phi = np.clip(phi + W.random_smooth(cfg, seed, amp=0.03), 0, 1)
    for a in range(dim):
        u[a] += W.random_smooth(cfg, seed + 10 + a, amp=0.01)
    P += W.random_smooth(cfg, seed + 20, amp=1e-3)
    return phi, P, u


CASES = {
    "2d_periodic": dict(dim=2, nx=12, ny=10),
    "2d_walls": dict(dim=2, nx=12, ny=10, wall=(1, 1, 0), gravity=(1e-5, -2e-5, 0.0)),
    "2d_channel": dict(dim=2, nx=12, ny=10, wall=(1, 0, 0), gravity=(0.0, 3e-5, 0.0)),
    "3d_periodic": dict(dim=3, nx=8, ny=6, nz=5),
    "3d_walls_xz": dict(dim=3, nx=8, ny=6, nz=5, wall=(1, 0, 1), gravity=(0.0, 1e-5, -2e-5)),
    "3d_d3q19_all_walls": dict(dim=3, nx=8, ny=6, nz=5, q_hydro=19, wall=(1, 1, 1),
                               gravity=(1e-6, 1e-5, -2e-5)),
}


@pytest.mark.parametrize("collision", ["filter", "bgk"])
@pytest.mark.parametrize("case", list(CASES))
def test_twin_reproduces_reference(case, collision):
    kw = dict(CASES[case])
    dim, nx, ny = kw.pop("dim"), kw.pop("nx"), kw.pop("ny")
    nz = kw.pop("nz", 1)
    cfg = W.base_case(dim, nx, ny, nz, nu_heavy=0.05, nu_light=0.15, sigma=0.01, collision=collision, **kw)
    f = _fields(cfg)
    ref = oracle.OracleCase(cfg)
    ref.init_fields(*f)
    tw = Twin(cfg)
    tw.init_fields(*f)
    scale = [0.0, 0.0, 0.0]
    worst = [0.0, 0.0, 0.0]
    for s in (0, 1, 4, 15):  # read at steps 0, 1, 5, 20
        ref.step(s)
        tw.step(s)
        a, b = ref.read_fields(), tw.read_fields()
        for k in range(3):
            scale[k] = max(scale[k], np.abs(a[k]).max())
            worst[k] = max(worst[k], np.abs(a[k] - b[k]).max())
    rel = [w / max(sc, 1e-30) for w, sc in zip(worst, scale)]
    print(case, collision, "phi %.1e P %.1e u %.1e" % tuple(rel))
    assert max(rel) < TOL, rel


def test_twin_catches_a_planted_slip():
    """The comparison has teeth: a twin whose filter collision drops the
    trace part of Phi_i (a plausible slip) departs from the reference at once."""
    cfg = W.base_case(2, 12, 10, nu_heavy=0.05, nu_light=0.15, sigma=0.01)
    f = _fields(cfg)
    ref = oracle.OracleCase(cfg)
    ref.init_fields(*f)
    tw = Twin(cfg)
    tw.init_fields(*f)
    T = 1.0 / 3.0
    orig = tw.equilibria

    def slipped_step():
        phi, _, P, u = tw.moments(tw.h, tw.g)
        heq, geq, F, rho, tau = orig(phi, P, u)
        hs = tw.h - (tw.h - heq) / tw.tau_phi
        ne = tw.g - geq
        gs = np.empty_like(tw.g)
        for i, (ci, wi) in enumerate(zip(tw.cG, tw.wG)):
            pp = sum(wi / (2 * T * T) * ci[a] * ci[b] * np.tensordot((tw.cG[:, a] * tw.cG[:, b]).astype(float),
                                                                      ne, axes=1)
                     for a in range(2) for b in range(2))
            gs[i] = geq[i] + (1.0 - 1.0 / tau) * pp
        tw.h = tw._stream(hs, tw.cH, tw.oppH, None, rho)
        tw.g = tw._stream(gs, tw.cG, tw.oppG, F, rho)

    slipped_step()
    ref.step(1)
    a, b = ref.read_fields(), tw.read_fields()
    assert np.abs(a[2] - b[2]).max() / np.abs(a[2]).max() > 1e-6


@pytest.mark.parametrize("dim,wall", [(2, (0, 0, 0)), (2, (1, 1, 0)), (3, (1, 0, 1))])
def test_diagnostics_equal_numpy_sums(dim, wall):
    """phi_sum, u_sum, rhou_sum (rho from phi clamped to [0, 1], reading R2)
    and umax of the reference equal NumPy sums of the fields it reads back,
    including a state whose phi over- and undershoots [0, 1]."""
    cfg = W.base_case(dim, 14, 12, 6 if dim == 3 else 1, wall=wall, nu_heavy=0.05, nu_light=0.15, sigma=0.01,
                      gravity=(0.0, -1e-5, 0.0) if dim == 2 else (0.0, 0.0, -1e-5))
    f = _fields(cfg, seed=7)
    oc = oracle.OracleCase(cfg)
    oc.init_fields(*f)
    oc.step(7)
    h, g, Pl, st = oc.get_state()
    # push phi outside [0, 1] at some nodes through the rest population
    h = h.copy()
    h[0].flat[::5] += 0.03
    h[0].flat[2::7] -= 0.04
    oc.set_state(h, g, Pl, st)
    phi, P, u = oc.read_fields()
    assert phi.max() > 1.0 or phi.min() < 0.0
    d = oc.diagnostics()
    rho = cfg["rho_light"] + np.clip(phi, 0, 1) * (cfg["rho_heavy"] - cfg["rho_light"])
    assert d["phi_sum"] == pytest.approx(phi.sum(), rel=1e-13, abs=1e-13)
    for a in range(dim):
        assert d["u_sum"][a] == pytest.approx(u[a].sum(), rel=1e-12, abs=1e-15)
        assert d["rhou_sum"][a] == pytest.approx((rho * u[a]).sum(), rel=1e-12, abs=1e-13)
    assert d["umax"] == pytest.approx(np.sqrt((u ** 2).sum(axis=0)).max(), rel=1e-14)
    assert d["nonfinite"] == 0
    # the unclamped density would give a different momentum sum here
    rho_raw = cfg["rho_light"] + phi * (cfg["rho_heavy"] - cfg["rho_light"])
    assert abs((rho_raw * u[0]).sum() - d["rhou_sum"][0]) > 1e-9 * np.abs(rho * u[0]).sum()


def test_diagnostics_count_nonfinite_nodes():
    """A NaN population at one node: the nodes whose phi, P or u read back
    non-finite are counted, no more and no fewer."""
    cfg = W.base_case(2, 14, 12, nu_heavy=0.05, nu_light=0.15, sigma=0.01)
    oc = oracle.OracleCase(cfg)
    oc.init_fields(*_fields(cfg))
    oc.step(3)
    h, g, Pl, st = oc.get_state()
    g = g.copy()
    g[4, 0, 5, 6] = np.nan
    oc.set_state(h, g, Pl, st)
    phi, P, u = oc.read_fields()
    bad = ~np.isfinite(phi) | ~np.isfinite(P) | ~np.isfinite(u).all(axis=0)
    d = oc.diagnostics()
    assert bad.sum() > 1
    assert d["nonfinite"] == int(bad.sum())
