"""ctypes binding of libpulbm.so (include/pulbm.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch, when a
GPU is visible, provides the device arena (a uint8 tensor) and the stream; no
computation goes through it.  There is no CPU fallback: if the library is
missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpulbm.so")

OK, EINVAL, ENOMEM, EDEVICE, EDIVERGED, ESTATE, EAGAIN = 0, -1, -2, -3, -4, -5, -6
STORES = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}
COLLISIONS = {"filter": 0, "bgk": 1}

EXPORTS = [
    "pulbm_required_bytes", "pulbm_create", "pulbm_init_fields", "pulbm_step", "pulbm_step_timed",
    "pulbm_read_fields", "pulbm_diagnostics", "pulbm_checkpoint_bytes", "pulbm_checkpoint",
    "pulbm_restore", "pulbm_sync", "pulbm_steps_done", "pulbm_destroy", "pulbm_last_error",
    "pulbm_batch_create", "pulbm_batch_admit", "pulbm_batch_advance", "pulbm_batch_poll",
    "pulbm_batch_take", "pulbm_batch_usage", "pulbm_batch_destroy", "pulbm_stream_copy",
    "pulbm_read_fields_noalloc", "pulbm_set_tile_order",
]


class PulbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pulbm error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    """Mirror of ``pulbm_params``."""

    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("q_hydro", C.c_int32), ("q_phase", C.c_int32), ("wall", C.c_int32 * 3),
        ("delta_theta", C.c_int32), ("store", C.c_int32), ("collision", C.c_int32),
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
    """Load libpulbm.so (built in place by ``build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2512_01027_amd/build.py "
                           "(there is no fallback path)")
    # PyTorch ships its own HIP runtime under the same soname; load it first so
    # that the library, the arena and the streams all use one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover
        pass
    lib = C.CDLL(LIB_PATH)
    vp, dp, i32, i64, sz = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64, C.c_size_t
    pp = C.POINTER(Params)
    sig = {
        "pulbm_required_bytes": [pp, C.POINTER(sz)],
        "pulbm_create": [pp, vp, sz, vp, C.POINTER(vp)],
        "pulbm_init_fields": [vp, dp, dp, dp],
        "pulbm_step": [vp, i64],
        "pulbm_step_timed": [vp, i64, dp],
        "pulbm_read_fields": [vp, dp, dp, dp],
        "pulbm_read_fields_noalloc": [vp, dp, dp, dp],
        "pulbm_diagnostics": [vp, C.POINTER(Diag)],
        "pulbm_checkpoint_bytes": [vp, C.POINTER(sz)],
        "pulbm_checkpoint": [vp, vp, sz],
        "pulbm_restore": [vp, vp, sz],
        "pulbm_sync": [vp],
        "pulbm_steps_done": [vp],
        "pulbm_set_tile_order": [vp, i32],
        "pulbm_destroy": [vp],
        "pulbm_last_error": [],
        "pulbm_batch_create": [sz, i32, i32, vp, C.POINTER(vp)],
        "pulbm_batch_admit": [vp, pp, dp, dp, dp, i64, C.POINTER(i32)],
        "pulbm_batch_advance": [vp, i32],
        "pulbm_batch_poll": [vp, C.POINTER(i32), i32, C.POINTER(i32)],
        "pulbm_batch_take": [vp, i32, dp, dp, dp],
        "pulbm_batch_usage": [vp, C.POINTER(sz), C.POINTER(i32)],
        "pulbm_batch_destroy": [vp],
        "pulbm_stream_copy": [vp, vp, sz, i32, i32, vp, dp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.pulbm_steps_done.restype = C.c_int64
    lib.pulbm_destroy.restype = None
    lib.pulbm_batch_destroy.restype = None
    lib.pulbm_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise PulbmError(rc, load().pulbm_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(cfg: dict) -> Params:
    """Parameter struct from a plain case dictionary (see ``workloads``)."""
    p = Params()
    p.dim = int(cfg["dim"])
    p.nx, p.ny, p.nz = int(cfg["nx"]), int(cfg["ny"]), int(cfg.get("nz", 1))
    p.q_hydro = int(cfg.get("q_hydro", 9 if p.dim == 2 else 27))
    p.q_phase = int(cfg.get("q_phase", 9 if p.dim == 2 else 19))
    w = list(cfg.get("wall", (0, 0, 0))) + [0, 0, 0]
    for a in range(3):
        p.wall[a] = int(w[a])
    p.delta_theta = int(cfg.get("delta_theta", 1))
    st = cfg.get("store", "fp64")
    p.store = STORES[st] if isinstance(st, str) else int(st)
    coll = cfg.get("collision", "filter")
    p.collision = COLLISIONS[coll] if isinstance(coll, str) else int(coll)
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
    # solid block ((lo_x, lo_y, lo_z), (hi_x, hi_y, hi_z)): nodes lo <= x < hi
    blk = cfg.get("block")
    for a in range(3):
        p.block_lo[a] = int(blk[0][a]) if blk else 0
        p.block_hi[a] = int(blk[1][a]) if blk else 0
    p.p_top = float(cfg.get("p_top", 0.0))
    return p


def _torch_stream_and_arena(nbytes):
    """Device arena and stream from PyTorch, if a GPU is visible."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        return None, None, None
    if not torch.cuda.is_available():
        return None, None, None
    arena = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
    addr = arena.data_ptr()
    pad = (-addr) % 256
    return arena, addr + pad, torch.cuda.current_stream().cuda_stream


class Case:
    """One simulation case on the GPU."""

    def __init__(self, cfg: dict, use_torch_arena: bool = True):
        self.lib = load()
        self.cfg = dict(cfg)
        self.params = make_params(cfg)
        self.dim = self.params.dim
        self.shape = (self.params.nz, self.params.ny, self.params.nx)
        self.N = self.params.nx * self.params.ny * self.params.nz
        nb = C.c_size_t()
        _check(self.lib.pulbm_required_bytes(C.byref(self.params), C.byref(nb)))
        self.bytes = nb.value
        self._arena = None
        addr, stream = None, None
        if use_torch_arena:
            self._arena, addr, stream = _torch_stream_and_arena(self.bytes)
        h = C.c_void_p()
        _check(self.lib.pulbm_create(C.byref(self.params), addr, self.bytes + 0, stream, C.byref(h)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.pulbm_destroy(h)
        self._h = None
        self._arena = None

    def __del__(self):
        self.close()

    def init_fields(self, phi, P, u):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        if phi.size != self.N or P.size != self.N or u.size != self.dim * self.N:
            raise ValueError("field sizes do not match the grid")
        _check(self.lib.pulbm_init_fields(self._h, _dp(phi), _dp(P), _dp(u)))

    def step(self, n: int):
        _check(self.lib.pulbm_step(self._h, int(n)))

    def step_timed(self, n: int):
        """GPU milliseconds of the moments, pressure, velocity and collide kernels."""
        ms = np.zeros(4)
        _check(self.lib.pulbm_step_timed(self._h, int(n), _dp(ms)))
        return ms

    def sync(self):
        _check(self.lib.pulbm_sync(self._h))

    @property
    def steps_done(self) -> int:
        return int(self.lib.pulbm_steps_done(self._h))

    def set_tile_order(self, order: int):
        """0: the usual tile order; 1: reversed (a race check, see pulbm.h)."""
        _check(self.lib.pulbm_set_tile_order(self._h, int(order)))

    def read_fields(self):
        phi = np.empty(self.N)
        P = np.empty(self.N)
        u = np.empty(self.dim * self.N)
        _check(self.lib.pulbm_read_fields(self._h, _dp(phi), _dp(P), _dp(u)))
        return (phi.reshape(self.shape), P.reshape(self.shape),
                u.reshape((self.dim,) + self.shape))

    def read_fields_noalloc(self, phi=None, P=None, u=None):
        """As read_fields, through the allocation-free entry point; the
        caller may pass the output arrays (FP64, C-contiguous)."""
        phi = np.empty(self.N) if phi is None else phi
        P = np.empty(self.N) if P is None else P
        u = np.empty(self.dim * self.N) if u is None else u
        for a, n in ((phi, self.N), (P, self.N), (u, self.dim * self.N)):
            if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"] or a.size != n:
                raise ValueError("output arrays must be C-contiguous FP64 of the case's sizes")
        _check(self.lib.pulbm_read_fields_noalloc(self._h, _dp(phi), _dp(P), _dp(u)))
        return (phi.reshape(self.shape), P.reshape(self.shape),
                u.reshape((self.dim,) + self.shape))

    def diagnostics(self, allow_diverged: bool = False) -> dict:
        d = Diag()
        rc = self.lib.pulbm_diagnostics(self._h, C.byref(d))
        if rc != OK and not (allow_diverged and rc == EDIVERGED):
            _check(rc)
        return {"phi_sum": d.phi_sum, "u_sum": list(d.u_sum)[: self.dim],
                "rhou_sum": list(d.rhou_sum)[: self.dim], "umax": d.umax,
                "nonfinite": d.nonfinite, "step": d.step}

    def checkpoint(self) -> bytes:
        nb = C.c_size_t()
        _check(self.lib.pulbm_checkpoint_bytes(self._h, C.byref(nb)))
        buf = C.create_string_buffer(nb.value)
        _check(self.lib.pulbm_checkpoint(self._h, buf, nb.value))
        return buf.raw

    def restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self.lib.pulbm_restore(self._h, buf, len(blob)))


def stream_copy(dst_ptr: int, src_ptr: int, nbytes: int, mode: int, reps: int, stream=None) -> float:
    """Average milliseconds of a device-to-device streaming copy (bandwidth
    probe; see pulbm_stream_copy)."""
    ms = C.c_double()
    _check(load().pulbm_stream_copy(dst_ptr, src_ptr, int(nbytes), int(mode), int(reps), stream, C.byref(ms)))
    return ms.value


class Batch:
    """Serving batch: many resident cases advanced together (see pulbm.h)."""

    def __init__(self, hbm_budget: int, store="fp16", max_slots: int = 64):
        self.lib = load()
        st = STORES[store] if isinstance(store, str) else int(store)
        stream = None
        try:
            import torch

            if torch.cuda.is_available():
                self._torch_stream = torch.cuda.Stream()
                stream = self._torch_stream.cuda_stream
        except ImportError:  # pragma: no cover
            pass
        h = C.c_void_p()
        _check(self.lib.pulbm_batch_create(int(hbm_budget), st, int(max_slots), stream, C.byref(h)))
        self._h = h
        self.shapes = {}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.lib.pulbm_batch_destroy(h)
        self._h = None

    def __del__(self):
        self.close()

    def admit(self, cfg: dict, phi, P, u, nsteps: int):
        """Slot id, or None if the batch has no room right now."""
        p = make_params(cfg)
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (phi, P, u)]
        slot = C.c_int32()
        rc = self.lib.pulbm_batch_admit(self._h, C.byref(p), *[_dp(a) for a in arrs], int(nsteps),
                                        C.byref(slot))
        if rc == EAGAIN:
            return None
        _check(rc)
        self.shapes[slot.value] = (p.dim, (p.nz, p.ny, p.nx))
        return slot.value

    def advance(self, k: int):
        _check(self.lib.pulbm_batch_advance(self._h, int(k)))

    def poll(self, cap: int = 4096):
        out = (C.c_int32 * cap)()
        n = C.c_int32()
        _check(self.lib.pulbm_batch_poll(self._h, out, cap, C.byref(n)))
        return [out[i] for i in range(min(n.value, cap))]

    def take(self, slot: int):
        dim, shape = self.shapes.pop(slot)
        N = int(np.prod(shape))
        phi, P, u = np.empty(N), np.empty(N), np.empty(dim * N)
        _check(self.lib.pulbm_batch_take(self._h, int(slot), _dp(phi), _dp(P), _dp(u)))
        return phi.reshape(shape), P.reshape(shape), u.reshape((dim,) + shape)

    def usage(self):
        used = C.c_size_t()
        act = C.c_int32()
        _check(self.lib.pulbm_batch_usage(self._h, C.byref(used), C.byref(act)))
        return used.value, act.value
