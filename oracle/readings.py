"""The static-droplet Laplace test of Sec. III.A under each reading of the
pressure / velocity reconstruction (R1) and viscosity set, on the NumPy twin.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

    python -m oracle.readings [--R 8] [--steps 3000] [--sets 1,2] [--leave-out]

Sec. III.A runs a droplet of radius R in a periodic box of 5R at density
ratio 1000, M = 0.166, W = 4, with sigma = 1e-2 or 1e-3 and two viscosity
sets (air, water): set 1 = (1.67e-1, 1.10e-2), set 2 = (5.56e-3, 3.67e-4).
Each run prints whether it stayed finite (max |u| < 0.5), the step by which
it diverged otherwise, and the pressure jump against sigma / R.  With
--leave-out the adopted reading is also run at set 2 with single terms of the
method dropped (diagnostic builds, not readings).
"""
from __future__ import annotations

import argparse
import time
import warnings

import numpy as np

from .twin import READINGS, Twin

SETS = {1: (1.67e-1, 1.10e-2), 2: (5.56e-3, 3.67e-4)}


def laplace_case(R, sigma, nu_air, nu_water):
    """Case dictionary and initial fields of the static droplet (tanh
    profile, P = 0, u = 0) in a periodic box of 5R."""
    n = int(round(5 * R))
    cfg = {"dim": 2, "nx": n, "ny": n, "nz": 1, "q_hydro": 9, "q_phase": 9, "wall": (0, 0, 0),
           "rho_heavy": 1000.0, "rho_light": 1.0, "nu_heavy": nu_water, "nu_light": nu_air,
           "sigma": sigma, "W": 4.0, "M": 0.166, "lambda_bulk": 1.0 / 6.0, "gravity": (0.0, 0.0, 0.0),
           "delta_theta": 1, "collision": "filter"}
    y, x = np.meshgrid(np.arange(n) + 0.0, np.arange(n) + 0.0, indexing="ij")
    c = (n - 1) / 2.0
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2)
    phi = (0.5 + 0.5 * np.tanh(2.0 * (R - r) / 4.0))[None]
    return cfg, (phi, np.zeros_like(phi), np.zeros((2,) + phi.shape))


def run(R, sigma, nu_air, nu_water, steps, reading="pstar", leave_out=(), every=50):
    """(diverged_at or None, dP / (sigma / R), max |u|) of one run."""
    cfg, f = laplace_case(R, sigma, nu_air, nu_water)
    t = Twin(cfg, reading, leave_out)
    t.init_fields(*f)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        for s in range(0, steps, every):
            t.step(min(every, steps - s))
            phi, P, u = t.read_fields()
            umax = float(np.sqrt((u ** 2).sum(axis=0)).max())
            if not np.isfinite(umax) or umax > 0.5:
                return s + every, float("nan"), umax
    dP = P[phi > 0.99].mean() - P[phi < 0.01].mean()
    return None, float(dP / (sigma / R)), umax


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--R", type=float, default=8.0)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--sigma", type=float, default=1e-2)
    ap.add_argument("--sets", default="1,2")
    ap.add_argument("--leave-out", action="store_true")
    a = ap.parse_args(argv)
    print(f"static droplet R = {a.R}, box {int(round(5 * a.R))}^2, sigma = {a.sigma}, {a.steps} steps")
    print("set | reading | result | dP / (sigma/R) | max |u|")
    for k in (int(v) for v in a.sets.split(",")):
        for reading in READINGS:
            t0 = time.time()
            div, dp, um = run(a.R, a.sigma, *SETS[k], a.steps, reading)
            res = f"diverged by step {div}" if div else "finite"
            print(f"{k} | {reading} | {res} | {dp:.4f} | {um:.2e}  ({time.time() - t0:.0f} s)", flush=True)
    if a.leave_out:
        for terms in (("stress_density",), ("bulk",), ("omega",)):
            div, dp, um = run(a.R, a.sigma, *SETS[2], a.steps, "pstar", terms)
            res = f"diverged by step {div}" if div else "finite"
            print(f"2 | pstar without {'+'.join(terms)} | {res} | {dp:.4f} | {um:.2e}", flush=True)


if __name__ == "__main__":
    main()
