"""The C ABI of libpulbm.so, checked without a GPU.

- every function declared in include/pulbm.h is exported by the built library
  (and nothing else under the pulbm_ prefix), and the ctypes binding wraps
  exactly that set;
- the ctypes mirrors of pulbm_params / pulbm_diag have the C layout (a small C
  program built here with gcc prints sizeof / offsetof);
- host-only calls (parameter validation, arena sizing, NULL handles, the
  thread-local error message) behave as the header documents.  None of these
  calls reaches the HIP runtime.
"""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess
import threading

import pytest

from paper_2512_01027_amd import binding as B
from paper_2512_01027_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pulbm.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return set(re.findall(r"\b(pulbm_[a-z_0-9]+)\s*\(", txt))


def _exported():
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    return {ln.split()[-1] for ln in out.splitlines() if " T " in ln and ln.split()[-1].startswith("pulbm_")}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libpulbm.so is not built (run __graft_entry__.build())")
    return B.load()


def test_header_matches_exports_and_binding(lib):
    decl = _declared()
    assert len(decl) == 24
    assert decl == _exported()
    assert decl == set(B.EXPORTS)
    for name in decl:
        assert getattr(lib, name) is not None


def test_struct_layout_matches_c(tmp_path):
    fields_p = [f for f, _ in B.Params._fields_]
    fields_d = [f for f, _ in B.Diag._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pulbm.h"', "int main(void){",
             'printf("P %zu\\n", sizeof(pulbm_params));', 'printf("D %zu\\n", sizeof(pulbm_diag));']
    lines += [f'printf("p.{f} %zu\\n", offsetof(pulbm_params, {f}));' for f in fields_p]
    lines += [f'printf("d.{f} %zu\\n", offsetof(pulbm_diag, {f}));' for f in fields_d]
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                     check=True).stdout.splitlines())
    assert int(got["P"]) == C.sizeof(B.Params)
    assert int(got["D"]) == C.sizeof(B.Diag)
    for f in fields_p:
        assert int(got[f"p.{f}"]) == getattr(B.Params, f).offset, f
    for f in fields_d:
        assert int(got[f"d.{f}"]) == getattr(B.Diag, f).offset, f


def _req(lib, p):
    n = C.c_size_t(0)
    rc = lib.pulbm_required_bytes(C.byref(p), C.byref(n))
    return rc, n.value


def test_required_bytes_scales_with_store(lib):
    cfg, _, _ = W.config_galilean_droplet_3d(32)
    N = 32 ** 3
    sizes = {}
    for store in ("fp64", "fp32", "fp16", "bf16"):
        rc, nb = _req(lib, B.make_params(dict(cfg, store=store)))
        assert rc == B.OK, lib.pulbm_last_error()
        sizes[store] = nb
    # 46 populations per node at the storage width, at least
    assert sizes["fp64"] >= 46 * 8 * N
    assert sizes["fp32"] >= 46 * 4 * N
    assert sizes["fp16"] >= 46 * 2 * N
    assert sizes["fp16"] == sizes["bf16"]
    assert sizes["fp64"] > sizes["fp32"] > sizes["fp16"]
    # the arena is not wildly larger than the state: populations plus a few
    # per-node auxiliary fields
    assert sizes["fp32"] < (46 + 40) * 4 * N


@pytest.mark.parametrize("change,msg", [
    (dict(nz=2), "nz = 1"),                   # 2D with nz != 1
    (dict(nx=0), ""),                         # empty grid
    (dict(q_hydro=27), ""),                   # wrong lattice for 2D
    (dict(collision=2), "collision"),
    (dict(store=7), ""),
    (dict(nu_light=0.0), "viscosities"),
    (dict(rho_light=2000.0), "densities"),
    (dict(W=0.0), "W"),
    (dict(delta_theta=2), "delta_theta"),
    (dict(gravity=(0.0, float("nan"), 0.0)), "gravity"),
])
def test_invalid_params_rejected(lib, change, msg):
    cfg, _, _ = W.config_static_droplet_2d()
    p = B.make_params(cfg)
    for k, v in change.items():
        if k == "gravity":
            for a in range(3):
                p.gravity[a] = v[a]
        else:
            setattr(p, k, v)
    rc, _ = _req(lib, p)
    assert rc == B.EINVAL
    err = lib.pulbm_last_error().decode()
    assert err and msg in err


def test_grid_size_limit(lib):
    """Field byte offsets are 32-bit: N x widest element must stay below 2^31."""
    cfg, _, _ = W.config_galilean_droplet_3d(32)
    ok = [("fp64", 1024, 512, 511), ("fp32", 1024, 1024, 511), ("fp16", 1024, 1024, 511)]
    bad = [("fp64", 1024, 512, 512), ("fp32", 1024, 1024, 512), ("bf16", 2048, 1024, 1024)]
    for store, nx, ny, nz in ok:
        rc, nb = _req(lib, B.make_params(dict(cfg, store=store, nx=nx, ny=ny, nz=nz)))
        assert rc == B.OK and nb > 0
    for store, nx, ny, nz in bad:
        rc, _ = _req(lib, B.make_params(dict(cfg, store=store, nx=nx, ny=ny, nz=nz)))
        assert rc == B.EINVAL
        assert "too large" in lib.pulbm_last_error().decode()


def test_null_handles(lib):
    assert lib.pulbm_required_bytes(None, None) == B.EINVAL
    assert lib.pulbm_step(None, 1) == B.EINVAL
    assert lib.pulbm_steps_done(None) == -1
    assert lib.pulbm_set_tile_order(None, 1) == B.EINVAL
    lib.pulbm_destroy(None)
    lib.pulbm_batch_destroy(None)
    assert lib.pulbm_batch_create(0, 2, 4, None, None) == B.EINVAL
    out = C.c_void_p()
    assert lib.pulbm_batch_create(0, 9, 4, None, C.byref(out)) == B.EINVAL
    assert lib.pulbm_batch_create(0, 2, 0, None, C.byref(out)) == B.EINVAL
    assert not out.value


def test_stream_copy_argument_checks(lib):
    """The bandwidth probe refuses bad arguments on the host, before any HIP
    call (the addresses below are never dereferenced)."""
    ms = C.c_double()
    a, b = 1 << 20, 1 << 24
    assert lib.pulbm_stream_copy(None, b, 4096, 0, 1, None, C.byref(ms)) == B.EINVAL
    assert lib.pulbm_stream_copy(a, b, 4096, 0, 1, None, None) == B.EINVAL
    assert lib.pulbm_stream_copy(a, b, 4095, 0, 1, None, C.byref(ms)) == B.EINVAL
    assert lib.pulbm_stream_copy(a + 8, b, 4096, 0, 1, None, C.byref(ms)) == B.EINVAL
    assert lib.pulbm_stream_copy(a, b, 0, 0, 1, None, C.byref(ms)) == B.EINVAL
    assert lib.pulbm_stream_copy(a, b, 4096, 4, 1, None, C.byref(ms)) == B.EINVAL
    assert lib.pulbm_stream_copy(a, b, 4096, 0, 0, None, C.byref(ms)) == B.EINVAL
    assert lib.pulbm_stream_copy(a, a + 2048, 4096, 0, 1, None, C.byref(ms)) == B.EINVAL
    assert "overlap" in lib.pulbm_last_error().decode()


def test_last_error_is_thread_local(lib):
    cfg, _, _ = W.config_static_droplet_2d()
    p = B.make_params(cfg)
    p.nx = 0
    assert _req(lib, p)[0] == B.EINVAL
    mine = lib.pulbm_last_error().decode()
    assert mine
    seen = []
    t = threading.Thread(target=lambda: seen.append(lib.pulbm_last_error().decode()))
    t.start()
    t.join()
    assert seen == [""]
    assert lib.pulbm_last_error().decode() == mine


@pytest.mark.parametrize("change,msg", [
    (dict(wall=(2, 0, 0)), "last axis"),                          # open end on x in 3D
    (dict(block=((4, 4, 4), (5, 8, 8))), "2 nodes thick"),        # 1-node block
    (dict(block=((0, 4, 4), (6, 8, 8))), "periodic"),             # across a periodic face
    (dict(wall=(0, 0, 2), block=((4, 4, 10), (8, 8, 16))), "open end"),
    (dict(block=((4, 4, 4), (8, 8, 20))), "exceeds"),
    (dict(p_top=float("inf")), "p_top"),
])
def test_invalid_boundaries_rejected(lib, change, msg):
    cfg = W.base_case(3, 16, 12, 16, **change)
    rc, _ = _req(lib, B.make_params(cfg))
    assert rc == B.EINVAL
    err = lib.pulbm_last_error().decode()
    assert err and msg in err


def test_block_and_open_end_accepted(lib):
    cfg = W.base_case(3, 16, 12, 16, wall=(1, 1, 2), block=((4, 3, 0), (8, 7, 5)), p_top=0.1)
    rc, size = _req(lib, B.make_params(cfg))
    assert rc == 0 and size > 0
    # 2D: the open end is on y
    cfg2 = W.base_case(2, 16, 12, wall=(1, 2, 0), block=((4, 0, 0), (8, 5, 1)))
    rc, _ = _req(lib, B.make_params(cfg2))
    assert rc == 0
