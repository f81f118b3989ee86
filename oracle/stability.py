"""Linear stability of the hydrodynamic step in one fluid at rest (von Neumann
analysis), for the readings of the pressure / velocity reconstruction weighed
in ``twin.py`` (R1).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

A single fluid of density rho at rest is a fixed point of the step.  About it
the step is linear and shift-invariant, so each Fourier mode exp(i k.x)
evolves on its own: the populations g_i, and for readings that use them the
previous step's P and u, are multiplied by an amplification matrix A(k) per
step.  The step is stable when no eigenvalue of A(k) exceeds 1 in modulus for
any k.  The matrix is built from the step's operations in Sec. II, linearised
(no force, no density gradient: phi is uniform):

  P* = rho_ref T sum g,  u* = sum g c
  K_i = w_i / (T rho) [P(x - c_i) - P(x)],  omega = (rho - rho_ref) / rho_ref
  P = rho_ref T sum (g_i + (1 + omega) K_i) + omega rho_ref sum w_i c_i . u(x - c_i)
  u = sum (g_i + K_i) c_i
  g^eq_i = P / (rho_ref T) delta_i0 + w_i c_i . u / T + B (w_i - delta_i0) div u / T
  filter: g*_i = g^eq_i + (1 - 1/tau) w_i / (2 T^2) (c_i c_i - T I) : Pi
  BGK:    g*_i = g_i - (g_i - g^eq_i) / tau
  stream: g_i(x + c_i) = g*_i(x)

with the isotropic central differences of Sec. II for div u, and the time
level of P and u inside the reconstruction set by the reading.  In Fourier
space a shift by d multiplies by exp(i k.d), the gradient stencil becomes
i s(k) with s_a = sum_i w_i c_ia sin(k.c_i) / T.

Closed forms the analysis reproduces at small k (pinned by tests): sound
waves travel at sqrt(T) in either fluid and decay at (2 nu / 3 + lambda_b / 3)
k^2 per step (the bulk and shear viscosities of the target momentum equation,
Sec. I); shear waves decay at nu k^2.
"""
from __future__ import annotations

import numpy as np

from .twin import T, velocity_set


def amplification(k, dim, q, nu, rho, rho_ref, rho_heavy, reading="pstar", collision="filter",
                  lambda_b=1.0 / 6.0):
    """Amplification matrix A(k) of one step.  State vector: g_0..g_{q-1},
    then the previous step's P and u (always carried; readings that do not
    use them leave those columns zero)."""
    c, w = velocity_set(dim, q)
    c = c[:, :dim].astype(float)
    k = np.asarray(k, dtype=float)[:dim]
    kc = c @ k
    s = (w[:, None] * c * np.sin(kc)[:, None]).sum(axis=0) / T       # D -> i s
    half_lap = (w * (np.exp(-1j * kc) - 1.0)).sum()                     # sum w [q(x-c) - q(x)]
    shift_m = np.exp(-1j * kc)                                          # value at x - c_i
    tau = nu / T + 0.5
    B = (2.0 / 3.0) * (nu - lambda_b) + T / 2.0
    omega_max = rho_heavy / rho_ref
    omega = (rho - rho_ref) / (rho_heavy - rho_ref) * (omega_max - 1.0)
    rest = int(np.nonzero((c == 0).all(axis=1))[0][0])
    n = q + 1 + dim

    def omega_term(v):
        # omega rho_ref sum_i w_i c_i . v(x - c_i)
        return omega * rho_ref * (w[:, None] * c * shift_m[:, None] * v[None, :]).sum()

    def k_sum(Pv):
        # rho_ref T (1 + omega) sum_i K_i
        return rho_ref * T * (1.0 + omega) * (w / (T * rho) * (shift_m - 1.0)).sum() * Pv

    def k_vel(Pv):
        # sum_i K_i c_i
        return (w[:, None] * c * (shift_m[:, None] - 1.0)).sum(axis=0) * Pv / (T * rho)

    def apply(x):
        g, Plag, ulag = x[:q], x[q], x[q + 1:]
        gs_ = g.sum()
        Ps = rho_ref * T * gs_
        us = (g[:, None] * c).sum(axis=0)
        if reading == "pstar":
            P = rho_ref * T * gs_ + k_sum(Ps) + omega_term(us)
            u = us + k_vel(P)
        elif reading == "plag":
            P = rho_ref * T * gs_ + k_sum(Plag) + omega_term(us)
            u = us + k_vel(P)
        elif reading == "ulag":
            P = rho_ref * T * gs_ + k_sum(Ps) + omega_term(ulag)
            u = us + k_vel(P)
        elif reading == "lag_both":
            P = rho_ref * T * gs_ + k_sum(Plag) + omega_term(ulag)
            u = us + k_vel(Plag)
        elif reading == "u_first":
            u = us + k_vel(Plag)
            P = rho_ref * T * gs_ + k_sum(Plag) + omega_term(u)
        else:
            raise ValueError(reading)
        div = 1j * (s * u).sum()
        geq = w * (c @ u) / T + B * w * div / T
        geq[rest] += P / (rho_ref * T) - B * div / T
        if collision == "bgk":
            gstar = g - (g - geq) / tau
        else:
            ne = g - geq
            Pi = (c[:, :, None] * c[:, None, :] * ne[:, None, None]).sum(axis=0)
            proj = (c[:, :, None] * c[:, None, :] - T * np.eye(dim)[None]) * Pi[None]
            gstar = geq + (1.0 - 1.0 / tau) * w / (2 * T * T) * proj.sum(axis=(1, 2))
        out = np.empty(n, dtype=complex)
        out[:q] = np.exp(-1j * kc) * gstar
        out[q] = P
        out[q + 1:] = u
        return out

    A = np.empty((n, n), dtype=complex)
    for j in range(n):
        e = np.zeros(n, dtype=complex)
        e[j] = 1.0
        A[:, j] = apply(e)
    return A


def spectral_radius(dim, q, nu, rho, rho_ref, rho_heavy, reading="pstar", collision="filter", nk=33):
    """max over a grid of wave vectors in [0, pi]^dim of the largest
    |eigenvalue| of A(k); returns (radius, k at the maximum)."""
    ks = np.linspace(0.0, np.pi, nk)
    best, kbest = 0.0, None
    grids = np.meshgrid(*([ks] * dim), indexing="ij")
    for kv in zip(*(g.ravel() for g in grids)):
        ev = np.linalg.eigvals(amplification(kv, dim, q, nu, rho, rho_ref, rho_heavy, reading, collision))
        r = np.abs(ev).max()
        if r > best:
            best, kbest = r, kv
    return best, kbest


def small_k_modes(dim, q, nu, rho, rho_ref, rho_heavy, kmag=0.05, reading="pstar", collision="filter"):
    """Eigenvalues of A(k) along x at |k| = kmag, as (decay rate, phase speed)
    per mode: rate = -ln|lambda| / k^2, speed = arg(lambda) / k."""
    k = np.zeros(dim)
    k[0] = kmag
    ev = np.linalg.eigvals(amplification(k, dim, q, nu, rho, rho_ref, rho_heavy, reading, collision))
    ev = ev[np.abs(ev) > 1e-8]
    return [(-np.log(np.abs(e)) / kmag ** 2, np.angle(e) / kmag) for e in ev]


if __name__ == "__main__":
    # the table of the readings in one fluid (light: rho = rho_ref, heavy:
    # rho = rho_heavy), D2Q9, density ratio 1000
    for reading in ("pstar", "plag", "ulag", "lag_both", "u_first"):
        for phase, rho in (("light", 1.0), ("heavy", 1000.0)):
            row = []
            for nu in (1e-1, 1e-2, 5.56e-3, 3.3e-3, 1e-3, 3.67e-4):
                r, _ = spectral_radius(2, 9, nu, rho, 1.0, 1000.0, reading, nk=25)
                row.append(f"{r:.4f}")
            print(reading, phase, " ".join(row))
