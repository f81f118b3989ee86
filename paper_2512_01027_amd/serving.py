"""Request loop of the serving mode: continuous batching of many cases on one
GPU through the batch calls of libpulbm.so (pulbm_batch_*).

Requests arrive as a seeded Poisson stream.  The loop admits arrived requests
in arrival order while the batch has a free slot and room in its memory
budget (the library answers EAGAIN otherwise), advances every resident case
k steps per captured-graph replay, and takes finished cases out as soon as a
poll reports them, which frees their slot and memory for the next arrivals.
Latency of a request = completion time - arrival time.

The same stream run one case at a time (first come, first served, the
single-case API) is the comparison.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import binding as B
from . import workloads as W


@dataclass
class Request:
    rid: int
    cfg: dict
    fields: tuple
    steps: int
    kind: str
    arrival: float
    nodes: int = 0
    done: float = math.nan

    @property
    def work(self) -> int:
        return self.nodes * self.steps


def make_stream(n_cases: int, store: str = "fp16", step_scale: float = 0.1, case_seed: int = 3,
                max_nodes: int | None = None):
    """Seeded requests (shapes, parameters and step counts of the serving
    workload; step counts multiplied by step_scale)."""
    rng = np.random.Generator(np.random.PCG64(case_seed))
    out = []
    while len(out) < n_cases:
        case = W.serving_case(rng, store, max_nodes)
        if case is None:
            continue
        cfg, f, steps, kind = case
        nodes = cfg["nx"] * cfg["ny"] * cfg["nz"]
        out.append(Request(len(out), cfg, f, max(1, int(round(steps * step_scale))), kind, 0.0, nodes))
    return out


def set_arrivals(reqs, rate_per_s: float | None, seed: int = 2):
    """Poisson arrivals at rate_per_s; None: every request arrives at once."""
    if rate_per_s is None:
        t = np.zeros(len(reqs))
    else:
        rng = np.random.Generator(np.random.PCG64(seed))
        t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=len(reqs)))
    for r, a in zip(reqs, t):
        r.arrival = float(a)
        r.done = math.nan


def _summary(reqs, makespan):
    lat = np.array([r.done - r.arrival for r in reqs])
    work = sum(r.work for r in reqs)
    return {"cases": len(reqs), "node_updates": int(work), "makespan_s": round(makespan, 4),
            "MLUPS": round(work / makespan / 1e6, 2),
            "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
            "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
            "latency_mean_s": round(float(lat.mean()), 4)}


def run_batched(reqs, hbm_budget: int, store: str = "fp16", k: int = 50, max_slots: int = 64,
                fill_nodes: int = 12 << 20, admit_per_round: int = 4, policy: str = "fifo",
                big_nodes: int = 3 << 19, fill_with_big: int | None = None, max_wait: float | None = None,
                progress=None):
    """Continuous batching.  Returns the summary; sets each request's done.

    Waiting requests are admitted in arrival order ("fifo") or least work
    (nodes x steps) first ("sjf"), a few per round so that the GPU starts on
    the first ones while later ones are set up, and only while the resident
    cases hold fewer than fill_nodes nodes (enough to fill the GPU: more would
    only share it among more cases and lengthen every latency).

    "big_fifo": a request of at least big_nodes nodes (one that fills the GPU
    on its own) is admitted only when no other such case is resident, in
    arrival order, so large cases run one after another at nearly the full
    rate, as one at a time would run them; smaller requests are admitted in
    arrival order alongside, while the resident small cases hold fewer than
    fill_nodes nodes (fill_with_big while a large case is resident, so that
    the large case, which every resident case slows as all of them advance
    in lock-step, keeps most of the GPU), and may overtake a large request
    that waits.  A small request then never queues behind a large one, and a
    large one never shares the GPU with another large one.  max_wait: a
    small request that has waited longer than this (seconds) is admitted
    past the fill limit, so that small requests arriving in a burst beside a
    long large case do not wait for it.

    progress(finished, total, elapsed), when given, is called after every
    completion.
    """
    if policy not in ("fifo", "sjf", "big_fifo"):
        raise ValueError(f"unknown admission policy {policy!r}")
    if fill_with_big is None:
        fill_with_big = fill_nodes
    bt = B.Batch(hbm_budget, store=store, max_slots=max_slots)
    pending = sorted(reqs, key=lambda r: r.arrival)
    waiting: list[Request] = []
    resident: dict[int, Request] = {}
    t0 = time.perf_counter()
    i = 0
    finished = 0
    peak = 0
    while finished < len(reqs):
        now = time.perf_counter() - t0
        while i < len(pending) and pending[i].arrival <= now:
            waiting.append(pending[i])
            i += 1
        if policy == "sjf":
            waiting.sort(key=lambda r: (r.work, r.arrival))
        admitted = 0
        if policy == "big_fifo":
            big_resident = any(r.nodes >= big_nodes for r in resident.values())
            small_held = sum(r.nodes for r in resident.values() if r.nodes < big_nodes)
            i_w = 0
            while i_w < len(waiting) and admitted < admit_per_round:
                r = waiting[i_w]
                big = r.nodes >= big_nodes
                if big and big_resident:
                    i_w += 1  # waits; later small requests may pass it
                    continue
                cap = fill_with_big if big_resident else fill_nodes
                aged = max_wait is not None and now - r.arrival > max_wait
                if not big and small_held and small_held + r.nodes > cap and not aged:
                    i_w += 1
                    continue
                slot = bt.admit(r.cfg, *r.fields, r.steps)
                if slot is None:
                    break
                resident[slot] = r
                waiting.pop(i_w)
                admitted += 1
                if big:
                    big_resident = True
                else:
                    small_held += r.nodes
        while policy != "big_fifo" and waiting and admitted < admit_per_round:
            held = sum(r.nodes for r in resident.values())
            if resident and held + waiting[0].nodes > fill_nodes:
                break
            r = waiting[0]
            slot = bt.admit(r.cfg, *r.fields, r.steps)
            if slot is None:
                break
            resident[slot] = r
            waiting.pop(0)
            admitted += 1
        peak = max(peak, len(resident))
        if not resident:
            if i < len(pending):
                time.sleep(max(0.0, pending[i].arrival - (time.perf_counter() - t0)))
            continue
        bt.advance(k)
        for s in bt.poll():
            r = resident.pop(s)
            bt.take(s)
            r.done = time.perf_counter() - t0
            finished += 1
            if progress is not None:
                progress(finished, len(reqs), r.done)
    makespan = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    bt.close()
    out = _summary(reqs, makespan)
    out.update({"peak_resident": peak, "advance_steps": k, "fill_nodes": fill_nodes, "policy": policy})
    if policy == "big_fifo":
        out.update({"big_nodes": big_nodes, "fill_with_big": fill_with_big, "max_wait": max_wait})
    return out


def run_sequential(reqs, progress=None):
    """One case at a time, first come first served, single-case API."""
    t0 = time.perf_counter()
    for k, r in enumerate(sorted(reqs, key=lambda r: r.arrival)):
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        c = B.Case(r.cfg)
        c.init_fields(*r.fields)
        c.step(r.steps)
        c.read_fields()
        c.close()
        r.done = time.perf_counter() - t0
        if progress is not None:
            progress(k + 1, len(reqs), r.done)
    makespan = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return _summary(reqs, makespan)


def compare(batched: dict, sequential: dict) -> dict:
    return {"batched": batched, "sequential": sequential,
            "throughput_ratio": round(batched["MLUPS"] / sequential["MLUPS"], 3),
            "p99_ratio": round(batched["latency_p99_s"] / sequential["latency_p99_s"], 3)}


def _records(reqs):
    return [{"rid": r.rid, "nodes": r.nodes, "steps": r.steps, "kind": r.kind, "dim": r.cfg["dim"],
             "arrival_s": round(r.arrival, 4), "done_s": round(r.done, 4),
             "latency_s": round(r.done - r.arrival, 4)} for r in reqs]


def main(argv=None):
    """The serving stream at its stated size, one mode per run:

        python -m paper_2512_01027_amd.serving batched    --cases 500 --rate auto --out F
        python -m paper_2512_01027_amd.serving sequential --cases 500 --rate R    --out F

    The request stream (seed 3) has full step counts (1000..10000).  --rate
    auto calibrates the capacity on a saturated burst of the first --calib
    requests (batched, big_fifo) and sets the Poisson rate to 0.8 x that
    capacity / the stream's mean work; give the printed rate to the other
    mode's run.  --rate burst: every request arrives at time 0 (the
    saturated capacity of each mode).  Each completion is printed as it happens; --out receives one
    JSON line per request and a summary line."""
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("batched", "sequential"))
    ap.add_argument("--cases", type=int, default=500)
    ap.add_argument("--step-scale", type=float, default=1.0)
    ap.add_argument("--rate", default="auto")
    ap.add_argument("--calib", type=int, default=40)
    ap.add_argument("--policy", default="big_fifo")
    ap.add_argument("--fill-nodes", type=int, default=4 << 20)
    ap.add_argument("--fill-with-big", type=int, default=1 << 20)
    ap.add_argument("--max-wait", type=float, default=6.0)
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--budget-frac", type=float, default=0.8)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    reqs = make_stream(a.cases, "fp16", a.step_scale)
    print(f"stream of {len(reqs)} requests built in {time.perf_counter() - t0:.0f} s", flush=True)
    mean_work = sum(r.work for r in reqs) / len(reqs)
    import torch

    free, _ = torch.cuda.mem_get_info()
    budget = int(a.budget_frac * free)
    out = {"mode": a.mode, "cases": len(reqs), "step_scale": a.step_scale, "mean_work": mean_work,
           "budget_GiB": round(budget / 2 ** 30, 1)}
    if a.rate == "auto":
        calib = reqs[: a.calib]
        set_arrivals(calib, None)
        cap = run_batched(calib, budget, k=a.k, policy=a.policy, fill_nodes=a.fill_nodes)
        rate = 0.8 * cap["MLUPS"] * 1e6 / mean_work
        out["calibration"] = cap
        print(f"calibration: {cap['MLUPS']} MLUPS on {len(calib)} requests -> rate {rate:.6f}/s", flush=True)
    elif a.rate == "burst":
        rate = None
    else:
        rate = float(a.rate)
    out["rate_per_s"] = rate
    set_arrivals(reqs, rate)

    last = [time.perf_counter()]

    def progress(k, n, t):
        if k % 10 == 0 or k == n or time.perf_counter() - last[0] > 30:
            last[0] = time.perf_counter()
            print(f"{a.mode}: {k}/{n} done at {t:.1f} s", flush=True)

    if a.mode == "batched":
        res = run_batched(reqs, budget, k=a.k, policy=a.policy, fill_nodes=a.fill_nodes,
                          fill_with_big=a.fill_with_big, max_wait=a.max_wait, progress=progress)
    else:
        res = run_sequential(reqs, progress=progress)
    out["summary"] = res
    with open(a.out, "w") as f:
        for rec in _records(reqs):
            f.write(json.dumps(rec) + "\n")
        f.write(json.dumps(out) + "\n")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    import sys

    sys.exit(main())

