"""The linear stability analysis of the reconstruction readings
(``oracle/stability.py``), pinned against closed forms and against the CPU
reference itself, and the stability table it gives.

* closed forms at small k: shear waves decay at nu k^2, sound travels at
  sqrt(T) (the paper keeps the sound speed sqrt(T), Sec. I) in the light and
  the heavy fluid;
* the CPU reference's own standing sound wave (single fluid, periodic 64 x 4,
  light and heavy) oscillates at the analysis's frequency and decays at its
  rate, and its speed is sqrt(T) within 0.5%;
* the table: the adopted reading ("pstar") is stable in both fluids at every
  viscosity down to 1e-3; K_i of the previous step's pressure ("plag") is
  unstable in the light fluid below about 5e-3; the readings that take the
  omega term or both formulas from the previous step are unstable already at
  1e-2.
"""
import numpy as np
import pytest

import oracle
from oracle import stability as S
from paper_2512_01027_amd import workloads as W

T = 1.0 / 3.0


def _physical(modes):
    return [m for m in modes if m[0] < 10.0]


@pytest.mark.parametrize("rho", [1.0, 1000.0])
@pytest.mark.parametrize("nu", [0.1, 0.01])
def test_small_k_shear_and_sound(rho, nu):
    modes = _physical(S.small_k_modes(2, 9, nu, rho, 1.0, 1000.0, kmag=0.02))
    shear = [m for m in modes if abs(m[1]) < 1e-6]
    sound = [m for m in modes if abs(m[1]) > 0.1]
    assert len(shear) == 1 and len(sound) == 2
    assert shear[0][0] == pytest.approx(nu, rel=1e-3)
    for rate, speed in sound:
        assert abs(speed) == pytest.approx(np.sqrt(T), rel=1e-3)


@pytest.mark.parametrize("phi0,rho", [(0.0, 1.0), (1.0, 1000.0)])
def test_reference_sound_wave_matches_analysis(phi0, rho):
    n, nu = 64, 0.05
    k = 2 * np.pi / n
    cfg = W.base_case(2, n, 4, nu_heavy=nu, nu_light=nu, sigma=0.01)
    x = np.arange(n)
    phi = np.full((1, 4, n), phi0)
    P = 1e-6 * np.cos(k * x)[None, None, :] * np.ones((1, 4, n))
    oc = oracle.OracleCase(cfg)
    oc.init_fields(phi, P, np.zeros((2, 1, 4, n)))
    amp = []
    for _ in range(400):
        p = oc.read_fields()[1][0, 0]
        amp.append(2.0 / n * (p * np.exp(-1j * k * x)).sum().real)
        oc.step(1)
    amp = np.array(amp)
    # the analysis's two sound eigenvalues at this k: a standing wave is
    # their sum, A lambda^t + conj(A) conj(lambda)^t
    ev = np.linalg.eigvals(S.amplification((k, 0.0), 2, 9, nu, rho, 1.0, 1000.0))
    snd = [e for e in ev if np.angle(e) > 0.01 and abs(e) > 0.99]
    lam = min(snd, key=lambda e: np.angle(e))
    # fit A by least squares over the record and compare the whole series
    t = np.arange(len(amp))
    basis = np.stack([(lam ** t).real, -(lam ** t).imag], axis=1)
    coef, *_ = np.linalg.lstsq(basis, amp, rcond=None)
    model = basis @ coef
    assert np.abs(model - amp).max() < 2e-3 * np.abs(amp).max()
    assert np.angle(lam) / k == pytest.approx(np.sqrt(T), rel=5e-3)


@pytest.mark.parametrize("rho", [1.0, 1000.0])
@pytest.mark.parametrize("nu", [1e-1, 1e-2, 5.56e-3, 3.3e-3, 1e-3])
def test_adopted_reading_is_stable(nu, rho):
    r, _ = S.spectral_radius(2, 9, nu, rho, 1.0, 1000.0, "pstar", nk=17)
    assert r < 1.0 + 1e-9


def test_rejected_readings_are_unstable():
    assert S.spectral_radius(2, 9, 5.56e-3, 1.0, 1.0, 1000.0, "plag", nk=17)[0] < 1.0 + 1e-9
    assert S.spectral_radius(2, 9, 3.3e-3, 1.0, 1.0, 1000.0, "plag", nk=17)[0] > 1.005
    assert S.spectral_radius(2, 9, 1e-2, 1000.0, 1.0, 1000.0, "ulag", nk=17)[0] > 1.01
    for reading in ("lag_both", "u_first"):
        assert S.spectral_radius(2, 9, 1e-2, 1.0, 1.0, 1000.0, reading, nk=17)[0] > 1.01
