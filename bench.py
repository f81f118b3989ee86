"""Benchmark of the coupled phase-field + P-u LBE step on one MI355X.

Workload of the headline line: the 3D dam break on 512 x 256 x 256 nodes
(33.5M), no-slip walls on all six faces, gravity 2e-6 along -z, a water
column 128 x 256 x 128 in the corner (density ratio 1000, W = 4,
sigma = 0.005, nu 0.01 water / 0.15 air), D3Q27 hydro + D3Q19 phase field,
FP16 shifted storage with FP32 compute.  A step is one full coupled time step
of the whole grid (moments, pressure, velocity, collide + stream); the state
is resident in HBM before timing starts.  Synthetic, seeded inputs.

Printed as one JSON line:
  value          MLUPS of the whole step (wall clock over --steps steps)
  roofline       the step (its four kernels together): the state bytes per
                 node update of the storage mode (216 B in FP16: 46 two-byte
                 populations and the FP32 P and u, each read and written
                 once) x nodes / the summed average HIP-event time of the four
                 kernels, against 8 TB/s; traffic = HBM bytes per step from
                 the committed rocprofv3 counter summary when it was taken on
                 the current kernel sources.  The collide kernel's own bytes
                 over its own time are reported beside it ("collide").
  hbm            state bytes per node update x MLUPS (wall clock), against
                 the peak, a torch device copy and the library's streaming
                 copy probe measured here
  fp32_store     the same workload with FP32 storage (400 B per node update)
  galilean_droplet_128cube  the 128^3 translated droplet, FP32 and FP16,
                 D3Q27 and D3Q19 hydro
  static_droplet_2d  the 64^2 FP64 droplet, 2000 steps: time per step
  workloads      the 256^3 rising bubble (FP32 / FP16 / BF16), the dam break
                 against a block (585 x 182 x 182) and the head-on collision
                 (256 x 192 x 192, D3Q19)
  serving        a seeded Poisson stream of droplet / bubble requests served
                 by continuous batching, p50 / p99 latency and aggregate MLUPS,
                 beside the same stream run one case at a time
  table1_rising_bubble  the 2D Table I bubbles to one time unit
  cpu_baseline   the FP64 CPU reference on bounded samples: the dam break at
                 a quarter of the linear size on every host thread and on one,
                 and the 64^2 droplet's 2000 steps in full
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
KERNELS = ("moments", "pressure", "velocity", "collide")
STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}
# Committed counter summaries, by workload: bench.py uses their traffic only
# while the kernel sources hash to the value they were taken on.
COUNTERS = {
    "dam_break": os.path.join(ROOT, "profiles", "dam_break_512x256x256_hbm_counters.txt"),
}
# Kernel names as rocprofv3 reports them, per lattice set and storage type.
_CT = {"fp64": "double", "fp32": "float", "fp16": "_Float16", "bf16": "unsigned short"}


def kernel_names(ls, store):
    """rocprofv3 names of a step's kernels; the collide kernel is one per step
    parity (even, odd), and a step runs one of them."""
    s, a = _CT[store], ("double" if store == "fp64" else "float")
    return {"moments": f"pulbm::k_moments<{ls}, {s}>", "pressure": f"pulbm::k_pressure<{ls}, {a}>",
            "velocity": f"pulbm::k_velocity<{ls}, {a}>",
            "collide": (f"pulbm::k_collide<{ls}, {s}, false, 0>", f"pulbm::k_collide<{ls}, {s}, false, 1>")}


def kernel_bytes(store_bytes, aux_bytes=4, pops=46, dim=3, q_phase=19):
    """Algorithmic bytes per node of each kernel (values per node times their
    width, each read or written once): moments reads the populations and
    writes phi, u*(dim), P*, M2 (6 in 3D); pressure reads P*, u*, phi and
    writes P; velocity reads P, u*, phi and writes u; collide reads phi, u,
    M2 and h and writes every population.  2-byte storage keeps M2 in two
    bytes per value (two to a 32-bit word, 4 bytes for the 3 values in 2D),
    and also reads the previous-step phi in moments and collide (the h
    codec's reference) and the previous-step u in moments (the g codec's
    reference)."""
    ref = aux_bytes if store_bytes == 2 else 0
    uref = dim * aux_bytes if store_bytes == 2 else 0
    nm = 6 if dim == 3 else 3
    m2 = 4 * ((nm + 1) // 2) if store_bytes == 2 else nm * aux_bytes
    return {
        "moments": pops * store_bytes + ref + uref + (2 + dim) * aux_bytes + m2,
        "pressure": (3 + dim) * aux_bytes,
        "velocity": (2 + 2 * dim) * aux_bytes,
        "collide": q_phase * store_bytes + ref + (1 + dim) * aux_bytes + m2 + pops * store_bytes,
    }


def state_bytes(store_bytes, aux_bytes=4, pops=46, dim=3):
    """Algorithmic bytes of one node update: the state read and written once.
    The state is the populations and the macroscopic P and u carried from one
    step to the next (the pressure is carried next to the populations, and the
    velocity is the reference of the 2-byte codecs): 400 B in 3D FP32 storage,
    216 B in FP16 or BF16 storage (P and u FP32)."""
    return 2 * (pops * store_bytes + (1 + dim) * aux_bytes)


def run_gpu(cfg, fields, steps, warmup, warm_fn=None):
    """MLUPS-relevant timings of one case: wall clock over `steps` steps after
    `warmup` untimed ones, then per-kernel HIP-event times over a further
    min(steps, 20) steps (at least 3)."""
    import torch

    from paper_2512_01027_amd import binding as B

    c = B.Case(cfg)
    c.init_fields(*fields)
    c.sync()
    if warm_fn is not None:
        warm_fn()
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
    """Read + write GB/s of a plain device copy: torch's, and the library's
    streaming copy probe in its four access modes (best reported)."""
    import torch

    from paper_2512_01027_amd import binding as B

    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    nbytes = src.numel() * 4
    out = {"torch_copy_GBs": round(2 * nbytes / dt / 1e9, 1)}
    stream = torch.cuda.current_stream().cuda_stream
    modes = {}
    for mode, name in ((0, "plain"), (1, "nt_loads"), (2, "nt_stores"), (3, "nt_both")):
        ms = B.stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, mode, reps, stream)
        modes[name] = round(2 * nbytes / (ms * 1e-3) / 1e9, 1)
    out["stream_copy_GBs"] = modes
    out["best_copy_GBs"] = max([out["torch_copy_GBs"]] + list(modes.values()))
    del src, dst
    torch.cuda.empty_cache()
    return out


def step_traffic(workload, ls, store, nodes):
    """HBM bytes per step (sum over the step's kernels, per launch) from the
    committed counter summary, if it was taken on the current kernel sources
    for this grid; None otherwise."""
    from paper_2512_01027_amd import profsum

    rec = profsum.load_traffic(COUNTERS[workload])
    if rec is None or rec["source_sha256"] != profsum.source_hash() or rec["nodes"] != nodes:
        return None, None
    names = kernel_names(ls, store)
    per = {}
    for k, name in names.items():
        # a per-parity pair counts as the mean of its two launches
        group = name if isinstance(name, tuple) else (name,)
        rs = [rec["kernels"].get(nm) for nm in group]
        if any(r is None for r in rs):
            if k == "velocity":
                continue
            return None, None
        per[k] = int(round(sum(r["read_bytes"] + r["write_bytes"] for r in rs) / len(rs)))
    return sum(per.values()), per


def leg(cfg, fields, steps, warmup, warm_fn=None):
    """Throughput, the step's roofline figures and the kernel times of one
    storage mode of a 3D workload."""
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    sb = STORE_BYTES[cfg["store"]]
    pops = cfg["q_hydro"] + cfg["q_phase"]
    dt, ms, dg = run_gpu(cfg, fields, steps, warmup, warm_fn)
    mlups = n * steps / dt / 1e6
    kb = kernel_bytes(sb, pops=pops, q_phase=cfg["q_phase"])
    kms = {k: round(float(v), 4) for k, v in zip(KERNELS, ms)}
    # the collide kernel rebuilt u: the step launches no velocity kernel, and
    # the event pair around the empty slot reads about 5 us (a real launch on
    # these grids takes more than 15 us)
    fused = kms["velocity"] < 0.010
    if fused:
        kms["velocity"] = None
    step_ms = float(sum(v for v in ms))
    sbytes = state_bytes(sb, pops=pops)
    return {
        "MLUPS": round(mlups, 2),
        "ms_per_step": round(dt / steps * 1e3, 4),
        "kernel_ms": kms,
        "step_kernel_ms": round(step_ms, 4),
        "state_bytes_per_node_update": sbytes,
        "step_GBs": round(sbytes * n / (step_ms * 1e-3) / 1e9, 1),
        "step_frac_of_peak": round(sbytes * n / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "effective_GBs": round(mlups * 1e6 * sbytes / 1e9, 1),
        "collide_GBs": round((kb["collide"] + (4 if fused else 0)) * n / (ms[3] * 1e-3) / 1e9, 1),
        "collide_bytes_per_node": kb["collide"] + (4 if fused else 0),
        "velocity_in_collide": fused,
        "nonfinite": dg["nonfinite"],
    }


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
    pol = dict(policy="big_fifo", fill_nodes=4 << 20, fill_with_big=1 << 20, max_wait=6.0 * step_scale)
    burst_b = SV.run_batched(reqs, budget, **pol)
    SV.set_arrivals(reqs, None)
    burst_s = SV.run_sequential(reqs)
    rate = 0.8 * burst_b["MLUPS"] * 1e6 / mean_work
    SV.set_arrivals(reqs, rate)
    pois_b = SV.run_batched(reqs, budget, **pol)
    SV.set_arrivals(reqs, rate)
    pois_s = SV.run_sequential(reqs)
    small = SV.make_stream(n_cases, "fp16", step_scale, case_seed=4, max_nodes=64 ** 3)
    SV.set_arrivals(small, None)
    small_b = SV.run_batched(small, budget)
    SV.set_arrivals(small, None)
    small_s = SV.run_sequential(small)
    return {"saturated": SV.compare(burst_b, burst_s), "poisson": SV.compare(pois_b, pois_s),
            "small_cases_saturated": SV.compare(small_b, small_s),
            "sample": (f"{n_cases} requests (seed 3): 75% 3D n in [32,192], 25% 2D n in [128,1024] "
                       f"(log-uniform), droplet / rising bubble, density ratio 10/100/1000, "
                       f"steps U{{1000..10000}} x {step_scale}; FP16 storage; batch budget "
                       f"{budget / 2**30:.0f} GiB; saturated: all at t=0; poisson: arrivals (seed 2) at "
                       f"{rate:.2f}/s = 0.8 x batched capacity / mean work; batched admission big_fifo (cases "
                       f"of 1.5M nodes or more one at a time, smaller ones alongside up to 4M nodes, 1M beside a "
                       f"large one unless waiting longer than {6.0 * step_scale:.1f} s); "
                       f"small_cases: {n_cases} requests (seed 4) of at most 64^3 nodes, all at t=0, FIFO")}


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
    """Throughput and the step's roofline figures of the other large
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
        elif name.startswith("dam_break_512"):
            continue  # the headline workload
        res = {}
        cfg, fields, _ = make(stores[0])
        for st in stores:
            res[st] = leg(dict(cfg, store=st), fields, steps, warmup)
        res["nodes"] = cfg["nx"] * cfg["ny"] * cfg["nz"]
        res["steps"] = steps
        out[name] = res
        del fields
        gc.collect()
    return out


def galilean_leg(steps, warmup, n=128):
    from paper_2512_01027_amd import workloads as W

    cfg, fields, _ = W.config_galilean_droplet_3d(n)
    res = {}
    for qh in (27, 19):
        for st in ("fp32", "fp16"):
            res[f"d3q{qh}_{st}"] = leg(dict(cfg, store=st, q_hydro=qh), fields, steps, warmup)
    for qh in (27, 19):
        res[f"d3q{qh}_fp16_over_fp32"] = round(res[f"d3q{qh}_fp16"]["MLUPS"] / res[f"d3q{qh}_fp32"]["MLUPS"], 3)
    res["nodes"] = n ** 3
    return res


def static_droplet_leg(steps=2000):
    """The 64^2 FP64 droplet of 2000 steps (the parity configuration):
    time per step; 4096 nodes cannot fill the GPU, so this is latency."""
    import torch

    from paper_2512_01027_amd import binding as B
    from paper_2512_01027_amd import workloads as W

    cfg, f, _ = W.config_static_droplet_2d()
    c = B.Case(cfg)
    c.init_fields(*f)
    c.step(20)
    c.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.step(steps)
    c.sync()
    dt = time.perf_counter() - t0
    c.close()
    return {"steps": steps, "ms_per_step": round(dt / steps * 1e3, 4),
            "MLUPS": round(64 * 64 * steps / dt / 1e6, 2)}


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(cfg, fields, seconds, min_steps):
    import oracle

    o = oracle.OracleCase(cfg)
    o.init_fields(*fields)
    o.step(1)  # warm
    t0 = time.perf_counter()
    n = 0
    while n < min_steps or time.perf_counter() - t0 < seconds:
        o.step(1)
        n += 1
    dt = time.perf_counter() - t0
    return cfg["nx"] * cfg["ny"] * cfg["nz"] * n / dt / 1e6, n


def cpu_baseline():
    """The FP64 CPU reference as it stands, on bounded samples (about 25 s
    of host time): the dam break workload at a quarter of its linear size
    (128 x 64 x 64, same parameters) on every host thread and on one, and the
    64^2 static droplet's 2000 steps in full."""
    import oracle
    from paper_2512_01027_amd import workloads as W

    all_threads = oracle.num_threads()
    cfg, f, _ = W.config_dam_break_3d(nx=128, ny=64, nz=64, store="fp64")
    oracle.set_num_threads(all_threads)
    v_all, n_all = _oracle_rate(cfg, f, 8.0, 3)
    oracle.set_num_threads(1)
    v_one, n_one = _oracle_rate(cfg, f, 6.0, 2)
    c1, f1, _ = W.config_static_droplet_2d()
    oracle.set_num_threads(all_threads)
    o = oracle.OracleCase(c1)
    o.init_fields(*f1)
    t0 = time.perf_counter()
    o.step(2000)
    t_c1 = time.perf_counter() - t0
    return {"value": round(v_all, 4), "unit": "MLUPS", "cores": all_threads, "kind": "oracle",
            "sample": (f"dam break at a quarter of the linear size (128x64x64, walls on all faces, "
                       f"D3Q27/D3Q19, FP64), {n_all} steps on {all_threads} threads"),
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": {"value": round(v_one, 4), "unit": "MLUPS", "steps": n_one},
            "static_droplet_2d_full": {"steps": 2000, "seconds": round(t_c1, 3),
                                       "MLUPS": round(64 * 64 * 2000 / t_c1 / 1e6, 4),
                                       "threads": all_threads}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-table1", action="store_true")
    ap.add_argument("--no-galilean", action="store_true")
    ap.add_argument("--no-workloads", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="the headline workload alone (profiling)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the device copies of MIB MiB (counter calibration)")
    ap.add_argument("--workload-only", default=None, metavar="NAME",
                    help="only run one real-size workload of the workloads leg (for profiling)")
    ap.add_argument("--store", default="fp32", help="storage of --workload-only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (a single case is not "
                                   "sharded across GPUs); --gpus must be 1"}))
        sys.exit(2)
    if args.workload_only:
        print(json.dumps({"workloads": workloads_leg(args.steps, args.warmup, args.workload_only, args.store)}))
        return
    if args.copy_probe:
        print(json.dumps({"copy_probe_bytes": args.copy_probe << 20, "copies": copy_bandwidth(args.copy_probe)}))
        return
    if args.headline_only:
        args.no_cpu = args.no_serving = args.no_table1 = args.no_galilean = args.no_workloads = True

    from paper_2512_01027_amd import workloads as W

    cfg, fields, _ = W.config_dam_break_3d(store="fp16")
    N = cfg["nx"] * cfg["ny"] * cfg["nz"]
    copies = {}

    def warm():  # the device copies run here, between init and the warm-up steps
        copies.update(copy_bandwidth())

    h = leg(cfg, fields, args.steps, args.warmup, warm)
    mlups = h["MLUPS"]
    sb = h["state_bytes_per_node_update"]
    traffic, per_kernel = step_traffic("dam_break", 3, "fp16", N)
    out = {
        "metric": METRIC,
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16 store / f32 compute",
        "data": "synthetic",
        "config": {"workload": "3D dam break 512x256x256 (33.5M nodes), no-slip walls on all faces, g=2e-6 "
                               "in -z, water column 128x256x128 in the corner, rho ratio 1000, W=4, "
                               "sigma=0.005, nu 0.01/0.15, D3Q27 hydro + D3Q19 phase field, FP16 shifted "
                               "store, FP32 compute", "nodes": N, "store": "fp16"},
        "roofline": {"bound": "hbm", "kernel": "step (k_moments + k_pressure + k_velocity + k_collide)",
                     "achieved": h["step_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": h["step_frac_of_peak"], "traffic": traffic,
                     "algorithmic_bytes_per_launch": sb * N, "bytes_per_node_update": sb,
                     "step_kernel_ms": h["step_kernel_ms"], "traffic_per_kernel": per_kernel,
                     "collide": {"achieved": h["collide_GBs"], "frac": round(h["collide_GBs"] / HBM_PEAK_GBS, 4),
                                 "bytes_per_node": h["collide_bytes_per_node"], "ms": h["kernel_ms"]["collide"]}},
        "hbm": {"state_bytes_per_node_update": sb, "effective_GBs": h["effective_GBs"],
                "frac_of_peak": round(h["effective_GBs"] / HBM_PEAK_GBS, 4), **copies,
                "frac_of_best_copy": round(h["effective_GBs"] / copies["best_copy_GBs"], 4)},
        "kernel_ms": h["kernel_ms"],
        "nonfinite": h["nonfinite"],
    }
    if not args.no_fp32:
        h32 = leg(dict(cfg, store="fp32"), fields, args.steps, args.warmup)
        out["fp32_store"] = h32
        out["fp16_over_fp32"] = round(mlups / h32["MLUPS"], 3)
    del fields
    if not args.no_galilean:
        out["galilean_droplet_128cube"] = galilean_leg(args.steps, args.warmup)
        out["static_droplet_2d"] = static_droplet_leg()
    if not args.no_workloads:
        out["workloads"] = workloads_leg()
    if not args.no_serving:
        out["serving"] = serving_leg()
    if not args.no_table1:
        out["table1_rising_bubble"] = table1_leg()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
