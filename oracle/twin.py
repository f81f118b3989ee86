"""NumPy twin of the coupled step (Otomo et al., arXiv 2512.01027, Sec. II).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  A second plain FP64
implementation of the same step, written from the paper independently of
``pulbm_oracle.c`` and in a different form: whole-grid array operations
instead of node-by-node loops, neighbour values from ghost-padded copies of a
field instead of per-link index resolution, and streaming by rolling whole
population arrays.  It shares no code with the C reference; tests hold the two
together (``tests/test_oracle_twin.py``), which catches an index, sign or
transposition slip in either one.

Scope: 2D (D2Q9 / D2Q9) and 3D (D3Q27 or D3Q19 hydro, D3Q19 phase field),
periodic axes or no-slip walls at both ends of an axis, the filter or the BGK
hydrodynamic collision, gravity.  (The solid block and the open top are
pinned by their own tests of the C reference.)

The readings of the points the paper leaves open are those of the C
reference: R2 (rho, tau, omega from phi clamped to [0, 1]), R7 (every stencil
on the hydro lattice), R8 (F_ext = rho g), R11 (halfway bounce-back with the
force part of a reflected population kept; ghost values: phi and rho even,
u odd, u* odd in its flow part and even in its body-force part, P
extrapolated hydrostatically).  For the time level of the pressure and
velocity reconstruction (R1) the twin also carries the alternatives that were
weighed against the adopted one (``reading``), so that they can be run side
by side on the same inputs:

  "pstar"    (adopted) P from K_i of the pressure the streamed populations
             carry, P* = rho_ref T sum g, and the omega term of the velocity
             they carry, u* = sum g c, at x - c_i; then u = sum (g_i + K_i) c_i
             with K_i of the new P.
  "plag"     as "pstar", but K_i of the pressure of the previous step.
  "ulag"     as "pstar", but the omega term of the previous step's
             reconstructed velocity at x - c_i.
  "lag_both" P and u both from the previous step's P and u: K_i of the
             previous P in both formulas, the omega term of the previous u.
  "u_first"  u first, from K_i of the previous P; then P from K_i of the
             previous P and the omega term of that new u.

``leave_out`` names terms of the method to drop, for diagnostic runs only
(never a reading): "stress_density" (the w_i c_l sigma_lm d_m rho / (rho^2 T)
term of g^eq), "bulk" (B = 0), "omega" (the omega term of the pressure).
"""
from __future__ import annotations

import itertools

import numpy as np

T = 1.0 / 3.0
EPS = 1.0e-10
GAMMA, PHI_N, PHI_M, D_DT = -22.5, 0.8, 0.2, 1.0e-4
READINGS = ("pstar", "plag", "ulag", "lag_both", "u_first")

# weights of the velocity sets of Sec. II by squared speed |c|^2 = 0, 1, 2, 3
_WEIGHTS = {(2, 9): (4 / 9, 1 / 9, 1 / 36, 0.0), (3, 19): (1 / 3, 1 / 18, 1 / 36, 0.0),
            (3, 27): (8 / 27, 2 / 27, 1 / 54, 1 / 216)}


def velocity_set(dim, q):
    """(c[q, 3] int, w[q]) with the rest direction first, then by speed."""
    wt = _WEIGHTS[(dim, q)]
    cs = []
    for c in itertools.product((-1, 0, 1), repeat=dim):
        n2 = sum(x * x for x in c)
        if wt[n2] > 0.0:
            cs.append((n2, tuple(c) + (0,) * (3 - dim)))
    cs.sort()
    c = np.array([v for _, v in cs], dtype=np.int64)
    w = np.array([wt[n2] for n2, _ in cs])
    assert len(c) == q
    return c, w


class Twin:
    """One case, held as whole-grid arrays (z, y, x)."""

    def __init__(self, cfg: dict, reading: str = "pstar", leave_out=()):
        if reading not in READINGS:
            raise ValueError(f"unknown reading {reading!r}")
        unknown = set(leave_out) - {"stress_density", "bulk", "omega"}
        if unknown:
            raise ValueError(f"unknown terms {sorted(unknown)}")
        self.leave_out = frozenset(leave_out)
        if cfg.get("block") or any(int(w) == 2 for w in cfg.get("wall", (0, 0, 0))):
            raise ValueError("the twin covers periodic axes and no-slip walls only")
        self.reading = reading
        self.dim = int(cfg["dim"])
        self.n = (int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1)))
        self.shape = (self.n[2], self.n[1], self.n[0])
        qg = int(cfg.get("q_hydro", 9 if self.dim == 2 else 27))
        qh = int(cfg.get("q_phase", 9 if self.dim == 2 else 19))
        self.cG, self.wG = velocity_set(self.dim, qg)
        self.cH, self.wH = velocity_set(self.dim, qh)
        self.oppG = self._opposites(self.cG)
        self.oppH = self._opposites(self.cH)
        self.wall = [int(w) for w in (list(cfg.get("wall", (0, 0, 0))) + [0, 0, 0])[:3]]
        self.grav = np.array([float(v) for v in (list(cfg.get("gravity", (0.0, 0.0, 0.0))) + [0, 0, 0])[:3]])
        self.ra, self.rw = float(cfg["rho_light"]), float(cfg["rho_heavy"])
        self.tau_a = float(cfg["nu_light"]) / T + 0.5
        self.tau_w = float(cfg["nu_heavy"]) / T + 0.5
        self.M = float(cfg.get("M", 0.166))
        self.W = float(cfg["W"])
        self.sigma = float(cfg["sigma"])
        self.lam = float(cfg.get("lambda_bulk", 1.0 / 6.0))
        self.delta_theta = int(cfg.get("delta_theta", 1))
        self.bgk = cfg.get("collision", "filter") in ("bgk", 1)
        self.tau_phi = self.M / T + 0.5
        self.omega_max = self.rw / self.ra
        self._ghost_tables()
        self.step_count = 0

    # ------------------------------------------------------------ geometry

    @staticmethod
    def _opposites(c):
        return np.array([int(np.nonzero((c == -ci).all(axis=1))[0][0]) for ci in c])

    def _ghost_tables(self):
        """Crossing count and wall offset of every cell of the one-cell ghost
        frame (component a lives on array axis 2 - a)."""
        shp = tuple(s + 2 for s in self.shape)
        self.kpad = np.zeros(shp, dtype=np.int64)
        self.offpad = np.zeros((3,) + shp)
        for a in range(3):
            if not self.wall[a]:
                continue
            ax = 2 - a
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[ax], hi[ax] = 0, shp[ax] - 1
            self.kpad[tuple(lo)] += 1
            self.kpad[tuple(hi)] += 1
            self.offpad[a][tuple(lo)] = -1.0
            self.offpad[a][tuple(hi)] = 1.0
        self.gopad = np.tensordot(self.grav, self.offpad, axes=1)  # g . (ghost - mirror)

    def _pad(self, f):
        out = f
        for a in range(3):
            ax = 2 - a
            width = [(0, 0)] * 3
            width[ax] = (1, 1)
            out = np.pad(out, width, mode="edge" if self.wall[a] else "wrap")
        return out

    def _at(self, fpad, d):
        """Values of a padded field at x + d for every node x."""
        nz, ny, nx = self.shape
        return fpad[1 + d[2]:1 + d[2] + nz, 1 + d[1]:1 + d[1] + ny, 1 + d[0]:1 + d[0] + nx]

    def even(self, f, d):
        return self._at(self._pad(f), d)

    def odd(self, f, d):
        s = np.where(self._at(self.kpad, d) % 2 == 1, -1.0, 1.0)
        return s * self._at(self._pad(f), d)

    def ustar(self, Ja, a, d):
        v = self._at(self._pad(Ja), d)
        return np.where(self._at(self.kpad, d) % 2 == 1, -v + 2.0 * self.grav[a], v)

    def pres(self, P, d, rho):
        return self._at(self._pad(P), d) + rho * self._at(self.gopad, d)

    # ------------------------------------------------------------ physics

    def props(self, phi):
        pc = np.clip(phi, 0.0, 1.0)
        return self.ra + pc * (self.rw - self.ra), self.tau_a + pc * (self.tau_w - self.tau_a)

    def stencil(self, f, kind):
        """Central gradient and Laplacian on the hydro lattice (Sec. II)."""
        at = self.even if kind == "even" else self.odd
        grad = np.zeros((3,) + self.shape)
        lap = np.zeros(self.shape)
        for ci, wi in zip(self.cG, self.wG):
            fp, fm = at(f, ci), at(f, -ci)
            for a in range(self.dim):
                grad[a] += (fp - fm) * ci[a] * wi
            lap += (fp - f) * wi
        return grad / (2.0 * T), 2.0 * lap / T

    def _k_terms(self, P, rho):
        """K_i = w_i / (T rho) [P(x - c_i) - P(x)] for every direction."""
        return [wi / (T * rho) * (self.pres(P, -ci, rho) - P) for ci, wi in zip(self.cG, self.wG)]

    def _omega_sum(self, vel, kind):
        """sum_i w_i c_i . v(x - c_i) for the velocity field vel[3]."""
        s = np.zeros(self.shape)
        for ci, wi in zip(self.cG, self.wG):
            for a in range(self.dim):
                if ci[a]:
                    v = self.ustar(vel[a], a, -ci) if kind == "ustar" else self.odd(vel[a], -ci)
                    s += wi * ci[a] * v
        return s

    def moments(self, h, g):
        """phi, rho, P, u of the state (the state is not changed)."""
        phi = h.sum(axis=0)
        rho, _ = self.props(phi)
        J = np.zeros((3,) + self.shape)
        for a in range(self.dim):
            J[a] = np.tensordot(self.cG[:, a].astype(float), g, axes=1)
        gsum = g.sum(axis=0)
        Ps = self.ra * T * gsum
        omega = (rho - self.ra) / (self.rw - self.ra) * (self.omega_max - 1.0)
        r = self.reading
        P_in_K = Ps if r in ("pstar", "ulag") else self.Plag
        K = self._k_terms(P_in_K, rho)
        u = np.zeros((3,) + self.shape)
        if r == "u_first":
            for ci, Ki in zip(self.cG, K):
                for a in range(self.dim):
                    u[a] += Ki * ci[a]
            u[: self.dim] += J[: self.dim]
            om = self._omega_sum(u, "u")
        elif r in ("ulag", "lag_both"):
            om = self._omega_sum(self.ulag, "u")
        else:
            om = self._omega_sum(J, "ustar")
        if "omega" in self.leave_out:
            om = 0.0
        P = self.ra * T * (gsum + (1.0 + omega) * sum(K)) + omega * self.ra * om
        if r != "u_first":
            Ku = K if r == "lag_both" else self._k_terms(P, rho)
            for ci, Ki in zip(self.cG, Ku):
                for a in range(self.dim):
                    u[a] += Ki * ci[a]
            u[: self.dim] += J[: self.dim]
        return phi, rho, P, u

    def equilibria(self, phi, P, u):
        """h^eq (with delta theta) and g^eq of Sec. II, plus F, rho, tau."""
        dim = self.dim
        rho, tau = self.props(phi)
        gphi, lphi = self.stencil(phi, "even")
        grho, _ = self.stencil(rho, "even")
        G = np.zeros((3, 3) + self.shape)  # G[a, b] = d u_a / d x_b
        for a in range(dim):
            gr, _ = self.stencil(u[a], "odd")
            G[a] = gr
        gnorm = np.sqrt((gphi[:dim] ** 2).sum(axis=0))
        n = gphi / (gnorm + EPS)
        theta = (self.M / T) * (1.0 - 4.0 * (phi - 0.5) ** 2) / self.W
        if self.delta_theta:
            s = lphi / (np.abs(lphi) + EPS)
            ramp = lambda v: np.clip(v, 0.0, 1.0)  # noqa: E731
            Y1 = np.minimum(ramp((phi - PHI_N) / D_DT), ramp(-(phi - 1.0) / D_DT))
            Y2 = np.minimum(ramp(phi / D_DT), ramp(-(phi - PHI_M) / D_DT))
            theta = theta + GAMMA * (self.M / (T * self.W)) * gnorm * ((1.0 + s) * Y1 + (1.0 - s) * Y2)
        u2 = (u[:dim] ** 2).sum(axis=0)
        heq = np.empty((len(self.cH),) + self.shape)
        for j, (cj, wj) in enumerate(zip(self.cH, self.wH)):
            cu = sum(cj[a] * u[a] for a in range(dim))
            cn = sum(cj[a] * n[a] for a in range(dim))
            gam = wj * (1.0 + cu / T + cu * cu / (2 * T * T) - u2 / (2 * T))
            heq[j] = phi * gam + theta * wj * cn
        nu = T * (tau - 0.5)
        mu = (48.0 * self.sigma / self.W) * phi * (phi - 1.0) * (phi - 0.5) - 1.5 * self.sigma * self.W * lphi
        F = np.zeros((3,) + self.shape)
        for a in range(dim):
            F[a] = rho * self.grav[a] + mu * gphi[a]
        div = sum(G[a, a] for a in range(dim))
        sig = np.zeros((3, 3) + self.shape)
        for a in range(dim):
            for b in range(dim):
                sig[a, b] = rho * nu * (G[a, b] + G[b, a])
            sig[a, a] += rho * (2.0 / 3.0) * (self.lam - nu) * div
        B = 0.0 if "bulk" in self.leave_out else (2.0 / 3.0) * (nu - self.lam) + T / 2.0
        geq = np.empty((len(self.cG),) + self.shape)
        for i, (ci, wi) in enumerate(zip(self.cG, self.wG)):
            rest = 1.0 if not ci.any() else 0.0
            cu = sum(ci[a] * u[a] for a in range(dim))
            cF = sum(ci[a] * F[a] for a in range(dim))
            csd = 0.0 if "stress_density" in self.leave_out else sum(
                ci[l] * sig[l, m] * grho[m] for l in range(dim) for m in range(dim))
            gam = wi * (1.0 + cu / T + cu * cu / (2 * T * T) - u2 / (2 * T))
            geq[i] = (P / (self.ra * T) * rest + gam - wi + wi * cF / (rho * T)
                      + B * (wi - rest) / T * div + wi * csd / (rho * rho * T))
        return heq, geq, F, rho, tau

    # ------------------------------------------------------------ the step

    def init_fields(self, phi, P, u):
        phi = np.asarray(phi, dtype=np.float64).reshape(self.shape)
        P = np.asarray(P, dtype=np.float64).reshape(self.shape)
        uu = np.zeros((3,) + self.shape)
        uu[: self.dim] = np.asarray(u, dtype=np.float64).reshape((self.dim,) + self.shape)
        self.h, self.g, _, _, _ = self.equilibria(phi, P, uu)
        self.Plag = P.copy()
        self.ulag = uu.copy()
        self.step_count = 0

    def step(self, nsteps=1):
        for _ in range(int(nsteps)):
            phi, _, P, u = self.moments(self.h, self.g)
            heq, geq, F, rho, tau = self.equilibria(phi, P, u)
            hs = self.h - (self.h - heq) / self.tau_phi
            if self.bgk:
                gs = self.g - (self.g - geq) / tau
            else:
                ne = self.g - geq
                Pi = np.zeros((3, 3) + self.shape)
                for a in range(self.dim):
                    for b in range(self.dim):
                        Pi[a, b] = np.tensordot((self.cG[:, a] * self.cG[:, b]).astype(float), ne, axes=1)
                gs = np.empty_like(self.g)
                for i, (ci, wi) in enumerate(zip(self.cG, self.wG)):
                    phipi = sum(wi / (2 * T * T) * (ci[a] * ci[b] - (T if a == b else 0.0)) * Pi[a, b]
                                for a in range(self.dim) for b in range(self.dim))
                    gs[i] = geq[i] + (1.0 - 1.0 / tau) * phipi
            self.h = self._stream(hs, self.cH, self.oppH, None, rho)
            self.g = self._stream(gs, self.cG, self.oppG, F, rho)
            self.Plag, self.ulag = P, u
            self.step_count += 1

    def _stream(self, fs, c, opp, F, rho):
        """Push to x + c_i (periodic wrap); a population whose link leaves
        through a wall comes back into the opposite slot of its own node,
        for g less twice the force part of its equilibrium."""
        out = np.empty_like(fs)
        for i, ci in enumerate(c):
            j = opp[i]
            moved = np.roll(fs[i], shift=(ci[2], ci[1], ci[0]), axis=(0, 1, 2))
            back = fs[j]
            if F is not None:
                cj, wj = c[j], (self.wG[j])
                back = back - 2.0 * wj * sum(cj[a] * F[a] for a in range(self.dim)) / (rho * T)
            # node y receives along c_i from y - c_i, unless that link of y's
            # own population j (c_j = -c_i) leaves the box
            leaving = self._leaves(c[j])
            out[i] = np.where(leaving, back, moved)
        return out

    def _leaves(self, cj):
        m = np.zeros(self.shape, dtype=bool)
        for a in range(3):
            if self.wall[a] and cj[a]:
                ax = 2 - a
                sl = [slice(None)] * 3
                sl[ax] = 0 if cj[a] < 0 else self.shape[ax] - 1
                m[tuple(sl)] = True
        return m

    def read_fields(self):
        phi, _, P, u = self.moments(self.h, self.g)
        return phi, P, u[: self.dim].copy()
