"""Benchmark of the coupled phase-field + P-u LBE step on one MI355X.

Workload (default): the 3D 128^3 periodic droplet (R = 24, rho ratio 1000,
W = 4, sigma = 0.005, nu = 0.05) translated with u = (0.05, 0.02, 0),
D3Q27 hydro + D3Q19 phase field, FP32 storage and compute.  A step is one
full coupled time step (moments, pressure, collide + stream) of the whole
grid; the state is resident in HBM before timing starts.

Prints one JSON line: MLUPS of the whole step, the roofline of the dominant
kernel (collide + stream) from HIP-event times, the same workload with FP16
storage, and the CPU reference timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per node of each kernel, 3D D3Q27 + D3Q19 (values per node
# times their width, each read or written once): moments reads 46 populations
# and writes phi, u*(3), S, M2(6); pressure reads u*(3), P, phi, S and writes
# P; velocity reads P, u*(3), phi and writes u(3); collide reads phi, u(3),
# M2(6), h(19) and writes 46 populations.
POP_VALUES_3D = 46
KERNELS = ("moments", "pressure", "velocity", "collide")


def kernel_bytes(store_bytes, aux_bytes=4):
    return {
        "moments": POP_VALUES_3D * store_bytes + 11 * aux_bytes,
        "pressure": 7 * aux_bytes,
        "velocity": 8 * aux_bytes,
        "collide": 19 * store_bytes + 10 * aux_bytes + POP_VALUES_3D * store_bytes,
    }


def state_bytes(store_bytes, aux_bytes=4):
    """Read and write of the state (46 populations and the pressure) once."""
    return 2 * (POP_VALUES_3D * store_bytes + aux_bytes)


def run_gpu(cfg, fields, steps, warmup):
    import torch

    from paper_2512_01027_amd import binding as B

    c = B.Case(cfg)
    c.init_fields(*fields)
    c.step(warmup)
    c.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.step(steps)
    c.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = c.step_timed(max(3, min(steps, 20)))
    nt = max(3, min(steps, 20))
    d = c.diagnostics(allow_diverged=True)
    c.close()
    return dt, ms / nt, d


def cpu_baseline(cfg, fields):
    import oracle

    ncells = cfg["nx"] * cfg["ny"] * cfg["nz"]
    o = oracle.OracleCase(cfg)
    o.init_fields(*fields)
    o.step(1)  # warm
    t0 = time.perf_counter()
    n = 0
    while n < 2 or (time.perf_counter() - t0 < 8.0 and n < 10):
        o.step(1)
        n += 1
    dt = time.perf_counter() - t0
    return {"value": round(ncells * n / dt / 1e6, 4), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": f"{cfg['nx']}x{cfg['ny']}x{cfg['nz']} grid, {n} steps (FP64)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=128, help="grid edge of the 3D droplet workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch

        src = torch.ones(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        nbytes = src.numel() * 4
        print(json.dumps({"copy_probe_bytes": nbytes, "dispatches": 6,
                          "copy_GBs_read_plus_write": round(2 * nbytes / dt / 1e9, 1)}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    from paper_2512_01027_amd import workloads as W

    cfg, fields, _ = W.config_galilean_droplet_3d(args.n)
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    dt, ms, diag = run_gpu(cfg, fields, args.steps, args.warmup)
    mlups = N * args.steps / dt / 1e6
    kb = kernel_bytes(4)
    ach = kb["collide"] * N / (ms[3] * 1e-3) / 1e9
    out = {
        "metric": "coupled-lattice MLUPS (D3Q27 hydro + D3Q19 phase field)",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D {args.n}^3 periodic translated droplet R={24 * args.n // 128}, "
                               "rho ratio 1000, FP32 store", "nodes": N, "store": "fp32"},
        "roofline": {"bound": "hbm", "kernel": "k_collide", "achieved": round(ach, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "kernel_ms": {k: round(float(v), 4) for k, v in zip(KERNELS, ms)},
        "kernel_GBs": {k: round(kb[k] * N / (float(v) * 1e-3) / 1e9, 1) for k, v in zip(KERNELS, ms)},
        "effective_state_GBs": round(mlups * 1e6 * state_bytes(4) / 1e9, 1),
        "nonfinite": diag["nonfinite"],
    }
    if not args.no_fp16:
        cfg16 = dict(cfg, store="fp16")
        dt16, ms16, _ = run_gpu(cfg16, fields, args.steps, args.warmup)
        out["fp16_store"] = {"value": round(N * args.steps / dt16 / 1e6, 2), "unit": "MLUPS",
                             "ratio_vs_fp32": round(dt / dt16, 3),
                             "kernel_ms": {k: round(float(v), 4) for k, v in zip(KERNELS, ms16)}}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, fields)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
