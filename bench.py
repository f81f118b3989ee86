"""Benchmark of the coupled phase-field + P-u LBE step on one MI355X.

Workload (the headline line): the 3D 128^3 periodic droplet (R = 24, density
ratio 1000, W = 4, sigma = 0.005, nu = 0.05) translated with
u = (0.05, 0.02, 0), D3Q27 hydro + D3Q19 phase field, FP32 storage and
compute.  A step is one full coupled time step of the whole grid (moments,
pressure, velocity, collide + stream); the state is resident in HBM before
timing starts.  Synthetic, seeded inputs.

Printed as one JSON line:
  value          MLUPS of the whole step (wall clock over --steps steps)
  roofline       the dominant kernel (collide + stream): algorithmic bytes per
                 launch / its average HIP-event time, against 8 TB/s; traffic
                 = HBM bytes per launch from the committed rocprofv3 counter
                 summary when it was taken on the current kernel sources
  hbm            state bytes per node-update x MLUPS, against the peak and
                 against a device copy measured here
  fp16_store     the same workload with FP16 storage
  d3q19_hydro    the same workload on D3Q19 for the hydrodynamic populations
                 too (the lattice of the paper's 3D runs), FP32 and FP16
  workloads      throughput at the real sizes of the 3D rising bubble (256^3,
                 walls in z; FP32, FP16 and BF16 storage), the dam break
                 (512 x 256 x 256, walls on all faces; FP16 and FP32), the
                 dam break against a block with an open top (585 x 182 x 182)
                 and the head-on droplet collision (256 x 192 x 192, D3Q19)
  serving        a seeded Poisson stream of droplet / bubble requests served
                 by continuous batching, p50 / p99 latency and aggregate MLUPS,
                 beside the same stream run one case at a time
  cpu_baseline   the FP64 CPU reference on a bounded sample of the workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "coupled-lattice MLUPS, % HBM peak; p50/p99 case latency; FP16 vs FP32 store"
COUNTERS = os.path.join(ROOT, "profiles", "galilean_droplet_128cube_hbm_counters.txt")
# Algorithmic bytes per node of each kernel, 3D D3Q27 + D3Q19 (values per node
# times their width, each read or written once): moments reads 46 populations
# and writes phi, u*(3), P*, M2(6); pressure reads P*, u*(3), phi and writes
# P; velocity reads P, u*(3), phi and writes u(3); collide reads phi, u(3),
# M2(6), h(19) and writes 46 populations.  2-byte storage also reads the
# previous-step phi in moments and collide (the h codec's reference) and the
# previous-step u in moments (the g codec's reference).  With D3Q19 hydro the
# populations per node are 38.
POP_VALUES_3D = 46
KERNELS = ("moments", "pressure", "velocity", "collide")


def kernel_bytes(store_bytes, aux_bytes=4, pops=POP_VALUES_3D, dim=3):
    # 2-byte storage: the populations are stored less shifts made of the
    # previous step's phi (h) and u (g), read back beside them
    ref = aux_bytes if store_bytes == 2 else 0
    uref = dim * aux_bytes if store_bytes == 2 else 0
    return {
        "moments": pops * store_bytes + ref + uref + 11 * aux_bytes,
        "pressure": 6 * aux_bytes,
        "velocity": 8 * aux_bytes,
        "collide": 19 * store_bytes + ref + 10 * aux_bytes + pops * store_bytes,
    }


def state_bytes(store_bytes, aux_bytes=4, pops=POP_VALUES_3D):
    """Read and write of the state (the populations and the pressure) once."""
    return 2 * (pops * store_bytes + aux_bytes)


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
    nt = max(3, min(steps, 20))
    ms = c.step_timed(nt)
    d = c.diagnostics(allow_diverged=True)
    c.close()
    return dt, ms / nt, d


def copy_bandwidth(mib=1024, reps=5):
    """Read + write GB/s of a plain device copy (torch)."""
    import torch

    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    gbs = 2 * src.numel() * 4 / dt / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbs, 1)


def traffic_of(kernel_name, n):
    """HBM bytes per launch of a kernel from the committed counter summary,
    if it was taken on the current kernel sources for this grid."""
    from paper_2512_01027_amd import profsum

    rec = profsum.load_traffic(COUNTERS)
    if rec is None or rec["source_sha256"] != profsum.source_hash() or rec["nodes"] != n ** 3:
        return None
    k = rec["kernels"].get(kernel_name)
    return None if k is None else int(round(k["read_bytes"] + k["write_bytes"]))


def serving_leg(n_cases=64, step_scale=0.1):
    """Saturated burst (every request at t = 0: the capacity of each mode),
    then a Poisson stream at 0.8 x the batched capacity."""
    import torch

    from paper_2512_01027_amd import serving as SV

    reqs = SV.make_stream(n_cases, "fp16", step_scale)
    mean_work = sum(r.work for r in reqs) / len(reqs)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    SV.set_arrivals(reqs, None)
    burst_b = SV.run_batched(reqs, budget)
    SV.set_arrivals(reqs, None)
    burst_s = SV.run_sequential(reqs)
    rate = 0.8 * burst_b["MLUPS"] * 1e6 / mean_work
    SV.set_arrivals(reqs, rate)
    pois_b = SV.run_batched(reqs, budget)
    SV.set_arrivals(reqs, rate)
    pois_s = SV.run_sequential(reqs)
    SV.set_arrivals(reqs, rate)
    pois_sjf = SV.run_batched(reqs, budget, policy="sjf")
    # the same request mix restricted to small cases (at most 64^3 / 256^2
    # nodes), each far from filling the GPU on its own
    small = SV.make_stream(n_cases, "fp16", step_scale, case_seed=4, max_nodes=64 ** 3)
    SV.set_arrivals(small, None)
    small_b = SV.run_batched(small, budget)
    SV.set_arrivals(small, None)
    small_s = SV.run_sequential(small)
    return {"saturated": SV.compare(burst_b, burst_s), "poisson": SV.compare(pois_b, pois_s),
            "poisson_least_work_first": SV.compare(pois_sjf, pois_s),
            "small_cases_saturated": SV.compare(small_b, small_s),
            "sample": (f"{n_cases} requests (seed 3): 75% 3D n in [32,192], 25% 2D n in [128,1024] "
                       f"(log-uniform), droplet / rising bubble, density ratio 10/100/1000, "
                       f"steps U{{1000..10000}} x {step_scale}; FP16 storage; batch budget "
                       f"{budget / 2**30:.0f} GiB; saturated: all at t=0; poisson: arrivals (seed 2) at "
                       f"{rate:.2f}/s = 0.8 x batched capacity / mean work; small_cases: {n_cases} requests "
                       f"(seed 4) of at most 64^3 nodes, all at t=0")}


def table1_leg(t_end=1.0, samples=4):
    """The 2D rising bubble of Sec. III.D, Table I cases 1 and 2 (200 x 400,
    FP32 storage) run to t_end time units of sqrt(2R/g), with the bubble's
    centroid height, rise velocity / U_g (U_g = sqrt(2Rg)) and circularity at
    equal intervals.  The benchmark's reference values are not available here:
    these are reported, not compared."""
    import torch

    from paper_2512_01027_amd import analysis as A
    from paper_2512_01027_amd import binding as B
    from paper_2512_01027_amd import workloads as W

    out = {}
    for case in (1, 2):
        cfg, f, unit = W.config_table1_bubble(case, "fp32")
        ug = (2 * 50.0 * 1.36e-8) ** 0.5
        c = B.Case(cfg)
        c.init_fields(*f)
        c.sync()
        n_total = int(round(t_end * unit))
        marks = [int(round(n_total * (k + 1) / samples)) for k in range(samples)]
        series, done, busy = [], 0, 0.0
        for m in marks:
            t0 = time.perf_counter()
            c.step(m - done)
            c.sync()
            torch.cuda.synchronize()
            busy += time.perf_counter() - t0
            done = m
            phi, _, u = c.read_fields()
            series.append({"t": round(m / unit, 4), "centroid_y": round(A.centroid(phi[0])[1], 3),
                           "rise_velocity_over_Ug": round(A.rise_velocity(phi[0], u[:, 0])[1] / ug, 4),
                           "circularity": round(A.circularity(phi[0]), 4)})
        d = c.diagnostics(allow_diverged=True)
        c.close()
        out[f"case{case}"] = {"steps": n_total, "MLUPS": round(cfg["nx"] * cfg["ny"] * n_total / busy / 1e6, 1),
                              "nonfinite": d["nonfinite"], "series": series}
    return out


def workloads_leg(steps=100, warmup=10, only=None, only_store=None):
    """MLUPS, effective HBM GB/s (state bytes per node update x MLUPS) and the
    collide kernel's GB/s (algorithmic bytes / HIP-event time) of the large
    workloads at their real sizes (``only``: one of them, in one storage)."""
    import gc

    from paper_2512_01027_amd import workloads as W

    runs = [("rising_bubble_256cube", lambda st: W.config_rising_bubble_3d(256, store=st), ("fp32", "fp16", "bf16")),
            ("dam_break_512x256x256", lambda st: W.config_dam_break_3d(store=st), ("fp16", "fp32")),
            ("dam_break_block_585x182x182", lambda st: W.config_dam_break_block(store=st), ("fp16", "fp32")),
            ("head_on_collision_256x192x192", lambda st: W.config_head_on_collision(store=st), ("fp32", "fp16"))]
    out = {}
    for name, make, stores in runs:
        if only is not None:
            if name != only:
                continue
            stores = (only_store,)
        leg = {}
        cfg, fields, _ = make(stores[0])
        n = cfg["nx"] * cfg["ny"] * cfg["nz"]
        for st in stores:
            sb = {"fp32": 4, "fp16": 2, "bf16": 2}[st]
            dt, ms, dg = run_gpu(dict(cfg, store=st), fields, steps, warmup)
            m = n * steps / dt / 1e6
            pops = cfg["q_hydro"] + cfg["q_phase"]
            eff = m * 1e6 * state_bytes(sb, pops=pops) / 1e9
            leg[st] = {"MLUPS": round(m, 1), "effective_GBs": round(eff, 1),
                       "effective_frac_of_peak": round(eff / HBM_PEAK_GBS, 4),
                       "collide_GBs": round(kernel_bytes(sb, pops=pops)["collide"] * n / (ms[3] * 1e-3) / 1e9, 1),
                       "kernel_ms": {k: round(float(v), 4) for k, v in zip(KERNELS, ms)},
                       "nonfinite": dg["nonfinite"]}
        leg["nodes"] = n
        leg["steps"] = steps
        out[name] = leg
        del fields
        gc.collect()
    return out


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
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-table1", action="store_true")
    ap.add_argument("--no-d3q19", action="store_true")
    ap.add_argument("--no-workloads", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--workload-only", default=None, metavar="NAME",
                    help="only run one real-size workload of the workloads leg (for profiling)")
    ap.add_argument("--store", default="fp32", help="storage of --workload-only")
    args = ap.parse_args()
    if args.workload_only:
        print(json.dumps({"workloads": workloads_leg(args.steps, args.warmup, args.workload_only, args.store)}))
        return
    if args.copy_probe:
        print(json.dumps({"copy_probe_bytes": args.copy_probe << 20, "dispatches": 6,
                          "copy_GBs_read_plus_write": copy_bandwidth(args.copy_probe)}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    from paper_2512_01027_amd import workloads as W

    cfg, fields, _ = W.config_galilean_droplet_3d(args.n)
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    dt, ms, diag = run_gpu(cfg, fields, args.steps, args.warmup)
    mlups = N * args.steps / dt / 1e6
    kb = kernel_bytes(4)
    ach = kb["collide"] * N / (ms[3] * 1e-3) / 1e9
    copy_gbs = copy_bandwidth()
    eff = mlups * 1e6 * state_bytes(4) / 1e9
    out = {
        "metric": METRIC,
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
        "config": {"workload": f"3D {args.n}^3 periodic droplet R={24 * args.n // 128} translated with "
                               "u=(0.05,0.02,0), rho ratio 1000, D3Q27 hydro + D3Q19 phase field, "
                               "FP32 store and compute", "nodes": N, "store": "fp32"},
        "roofline": {"bound": "hbm", "kernel": "k_collide<3, float, false>", "achieved": round(ach, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": traffic_of("pulbm::k_collide<3, float, false>", args.n),
                     "algorithmic_bytes_per_launch": kb["collide"] * N},
        "hbm": {"state_bytes_per_node_update": state_bytes(4), "effective_GBs": round(eff, 1),
                "frac_of_peak": round(eff / HBM_PEAK_GBS, 4), "device_copy_GBs": copy_gbs,
                "frac_of_copy": round(eff / copy_gbs, 4)},
        "kernel_ms": {k: round(float(v), 4) for k, v in zip(KERNELS, ms)},
        "kernel_GBs": {k: round(kb[k] * N / (float(v) * 1e-3) / 1e9, 1) for k, v in zip(KERNELS, ms)},
        "nonfinite": diag["nonfinite"],
    }
    if not args.no_fp16:
        cfg16 = dict(cfg, store="fp16")
        dt16, ms16, _ = run_gpu(cfg16, fields, args.steps, args.warmup)
        kb16 = kernel_bytes(2)
        m16 = N * args.steps / dt16 / 1e6
        out["fp16_store"] = {"value": round(m16, 2), "unit": "MLUPS", "ratio_vs_fp32": round(dt / dt16, 3),
                             "kernel_ms": {k: round(float(v), 4) for k, v in zip(KERNELS, ms16)},
                             "collide_GBs": round(kb16["collide"] * N / (ms16[3] * 1e-3) / 1e9, 1),
                             "effective_GBs": round(m16 * 1e6 * state_bytes(2) / 1e9, 1)}
        if not args.no_serving:
            out["serving"] = serving_leg()
    if not args.no_d3q19:
        leg = {}
        for store, sb in (("fp32", 4), ("fp16", 2)):
            d19, ms19, dg19 = run_gpu(dict(cfg, store=store, q_hydro=19), fields, args.steps, args.warmup)
            kb19 = kernel_bytes(sb, pops=38)
            m19 = N * args.steps / d19 / 1e6
            # a periodic D3Q19 case in 4-byte storage rebuilds u inside the
            # collide kernel (which then also reads the new P) and launches
            # no velocity kernel
            fused = sb >= 4
            kms = {k: round(float(v), 4) for k, v in zip(KERNELS, ms19)}
            if fused:
                kms["velocity"] = None
            cb = kb19["collide"] + (4 if fused else 0)
            leg[store] = {"value": round(m19, 2), "unit": "MLUPS", "velocity_in_collide": fused,
                          "kernel_ms": kms,
                          "collide_GBs": round(cb * N / (ms19[3] * 1e-3) / 1e9, 1),
                          "effective_GBs": round(m19 * 1e6 * state_bytes(sb, pops=38) / 1e9, 1),
                          "nonfinite": dg19["nonfinite"]}
        out["d3q19_hydro"] = leg
    if not args.no_workloads:
        out["workloads"] = workloads_leg()
    if not args.no_table1:
        out["table1_rising_bubble"] = table1_leg()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, fields)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
