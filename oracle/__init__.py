"""Plain FP64 CPU reference ("the oracle") of the coupled phase-field + P-u
lattice Boltzmann step (Otomo et al., arXiv 2512.01027, Sec. II).

TEST INFRASTRUCTURE ONLY.  Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_2512_01027_amd``) never imports it, and this package never
imports the product.  The two share no code; only the seeded input generators
(``paper_2512_01027_amd.workloads``, which holds none of the method's
arithmetic) feed both.

This module is a thin ctypes binding of ``liboracle.so`` built from
``pulbm_oracle.c`` (see ``build.py``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")


class Params(C.Structure):
    """Mirror of ``pulbm_oracle_params`` (oracle/pulbm_oracle.h)."""

    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("q_hydro", C.c_int32), ("q_phase", C.c_int32),
        ("wall", C.c_int32 * 3), ("delta_theta", C.c_int32), ("collision", C.c_int32),
        ("rho_heavy", C.c_double), ("rho_light", C.c_double),
        ("nu_heavy", C.c_double), ("nu_light", C.c_double),
        ("sigma", C.c_double), ("W", C.c_double), ("M", C.c_double),
        ("lambda_bulk", C.c_double), ("gravity", C.c_double * 3),
        ("block_lo", C.c_int32 * 3), ("block_hi", C.c_int32 * 3), ("p_top", C.c_double),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("phi_sum", C.c_double), ("u_sum", C.c_double * 3), ("rhou_sum", C.c_double * 3),
        ("umax", C.c_double), ("nonfinite", C.c_int64), ("step", C.c_int64),
    ]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b

        _b.build()
    lib = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    lib.pulbm_oracle_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
    lib.pulbm_oracle_destroy.argtypes = [vp]
    lib.pulbm_oracle_destroy.restype = None
    lib.pulbm_oracle_init_fields.argtypes = [vp, dp, dp, dp]
    lib.pulbm_oracle_step.argtypes = [vp, C.c_int64]
    lib.pulbm_oracle_read_fields.argtypes = [vp, dp, dp, dp]
    lib.pulbm_oracle_diagnostics.argtypes = [vp, C.POINTER(Diag)]
    lib.pulbm_oracle_get_state.argtypes = [vp, dp, dp, dp, C.POINTER(C.c_int64)]
    lib.pulbm_oracle_set_state.argtypes = [vp, dp, dp, dp, C.c_int64]
    lib.pulbm_oracle_lattice.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int32), dp]
    lib.pulbm_oracle_node_eq.argtypes = [C.POINTER(Params), C.c_double, C.c_double, dp, dp,
                                         C.c_double, dp, dp, dp, dp]
    lib.pulbm_oracle_stencil.argtypes = [vp, dp, dp, dp]
    lib.pulbm_oracle_num_threads.argtypes = []
    lib.pulbm_oracle_set_num_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(cfg: dict) -> Params:
    """Build the oracle's parameter struct from a plain case dictionary."""
    p = Params()
    p.dim = int(cfg["dim"])
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1))
    p.q_hydro = int(cfg.get("q_hydro", 9 if p.dim == 2 else 27))
    p.q_phase = int(cfg.get("q_phase", 9 if p.dim == 2 else 19))
    w = list(cfg.get("wall", (0, 0, 0))) + [0, 0, 0]
    for a in range(3):
        p.wall[a] = int(w[a])
    p.delta_theta = int(cfg.get("delta_theta", 1))
    p.collision = {"filter": 0, "bgk": 1}[cfg.get("collision", "filter")]
    p.rho_heavy = float(cfg["rho_heavy"])
    p.rho_light = float(cfg["rho_light"])
    p.nu_heavy = float(cfg["nu_heavy"])
    p.nu_light = float(cfg["nu_light"])
    p.sigma = float(cfg["sigma"])
    p.W = float(cfg["W"])
    p.M = float(cfg.get("M", 0.166))
    p.lambda_bulk = float(cfg.get("lambda_bulk", 1.0 / 6.0))
    gv = list(cfg.get("gravity", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
    for a in range(3):
        p.gravity[a] = float(gv[a])
    # solid block: ((lo_x, lo_y, lo_z), (hi_x, hi_y, hi_z)), nodes lo <= x < hi
    blk = cfg.get("block")
    for a in range(3):
        p.block_lo[a] = int(blk[0][a]) if blk else 0
        p.block_hi[a] = int(blk[1][a]) if blk else 0
    p.p_top = float(cfg.get("p_top", 0.0))
    return p


class OracleCase:
    """One simulation case held by the FP64 CPU reference."""

    def __init__(self, cfg: dict):
        self.lib = load()
        self.cfg = dict(cfg)
        self.params = make_params(cfg)
        self.dim = self.params.dim
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.N = self.params.nx * self.params.ny * self.params.nz
        h = C.c_void_p()
        rc = self.lib.pulbm_oracle_create(C.byref(self.params), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle rejected the case parameters (rc={rc})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.pulbm_oracle_destroy(h)
            self._h = None

    def init_fields(self, phi, P, u):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        assert phi.size == self.N and P.size == self.N and u.size == self.dim * self.N
        rc = self.lib.pulbm_oracle_init_fields(self._h, _dp(phi), _dp(P), _dp(u))
        if rc:
            raise RuntimeError(f"oracle init_fields failed ({rc})")

    def step(self, n: int):
        rc = self.lib.pulbm_oracle_step(self._h, int(n))
        if rc:
            raise RuntimeError(f"oracle step failed ({rc})")

    def read_fields(self):
        phi = np.empty(self.N)
        P = np.empty(self.N)
        u = np.empty(self.dim * self.N)
        rc = self.lib.pulbm_oracle_read_fields(self._h, _dp(phi), _dp(P), _dp(u))
        if rc:
            raise RuntimeError(f"oracle read_fields failed ({rc})")
        return (phi.reshape(self.shape), P.reshape(self.shape),
                u.reshape((self.dim,) + self.shape))

    def diagnostics(self) -> dict:
        d = Diag()
        rc = self.lib.pulbm_oracle_diagnostics(self._h, C.byref(d))
        if rc:
            raise RuntimeError(f"oracle diagnostics failed ({rc})")
        return {"phi_sum": d.phi_sum, "u_sum": list(d.u_sum)[: self.dim],
                "rhou_sum": list(d.rhou_sum)[: self.dim], "umax": d.umax,
                "nonfinite": d.nonfinite, "step": d.step}

    def get_state(self):
        qh, qg = self.params.q_phase, self.params.q_hydro
        h = np.empty(qh * self.N)
        g = np.empty(qg * self.N)
        Pl = np.empty(self.N)
        st = C.c_int64()
        self.lib.pulbm_oracle_get_state(self._h, _dp(h), _dp(g), _dp(Pl), C.byref(st))
        return (h.reshape((qh,) + self.shape), g.reshape((qg,) + self.shape),
                Pl.reshape(self.shape), st.value)

    def set_state(self, h, g, Plag, step):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (h, g, Plag)]
        rc = self.lib.pulbm_oracle_set_state(self._h, *[_dp(a) for a in arrs], int(step))
        if rc:
            raise RuntimeError("oracle set_state failed")

    def stencil(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        grad = np.empty(3 * self.N)
        lap = np.empty(self.N)
        self.lib.pulbm_oracle_stencil(self._h, _dp(q), _dp(grad), _dp(lap))
        return grad.reshape((3,) + self.shape), lap.reshape(self.shape)


def lattice(dim: int, q: int):
    """(c[q,3], w[q]) of a velocity set, in the oracle's own direction order."""
    lib = load()
    c = np.zeros(3 * q, dtype=np.int32)
    w = np.zeros(q)
    if lib.pulbm_oracle_lattice(dim, q, c.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w)):
        raise ValueError("unknown lattice")
    return c.reshape(q, 3), w


def node_eq(cfg: dict, phi, P, u, gradphi, lapphi, gradrho, G):
    """Equilibria h^eq, g^eq at one node for given local values and gradients."""
    lib = load()
    p = make_params(cfg)
    v3 = lambda a: np.ascontiguousarray(list(a) + [0.0] * (3 - len(a)), dtype=np.float64)  # noqa: E731
    u, gp, gr = v3(u), v3(gradphi), v3(gradrho)
    Gm = np.zeros(9)
    Garr = np.asarray(G, dtype=np.float64)
    d = Garr.shape[0]
    Gm.reshape(3, 3)[:d, :d] = Garr
    heq = np.zeros(p.q_phase)
    geq = np.zeros(p.q_hydro)
    rc = lib.pulbm_oracle_node_eq(C.byref(p), float(phi), float(P), _dp(u), _dp(gp),
                                  float(lapphi), _dp(gr), _dp(Gm), _dp(heq), _dp(geq))
    if rc:
        raise ValueError("oracle rejected parameters")
    return heq, geq


def num_threads() -> int:
    return int(load().pulbm_oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the reference's node loops (its results do not depend on it)."""
    if load().pulbm_oracle_set_num_threads(int(n)):
        raise ValueError("thread count must be >= 1")
