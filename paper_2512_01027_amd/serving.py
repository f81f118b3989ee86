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
                fill_nodes: int = 12 << 20, admit_per_round: int = 4, policy: str = "fifo"):
    """Continuous batching.  Returns the summary; sets each request's done.

    Waiting requests are admitted in arrival order ("fifo") or least work
    (nodes x steps) first ("sjf"), a few per round so that the GPU starts on
    the first ones while later ones are set up, and only while the resident
    cases hold fewer than fill_nodes nodes (enough to fill the GPU: more would
    only share it among more cases and lengthen every latency).
    """
    if policy not in ("fifo", "sjf"):
        raise ValueError(f"unknown admission policy {policy!r}")
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
        while waiting and admitted < admit_per_round:
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
    makespan = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    bt.close()
    out = _summary(reqs, makespan)
    out.update({"peak_resident": peak, "advance_steps": k, "fill_nodes": fill_nodes, "policy": policy})
    return out


def run_sequential(reqs):
    """One case at a time, first come first served, single-case API."""
    t0 = time.perf_counter()
    for r in sorted(reqs, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if now < r.arrival:
            time.sleep(r.arrival - now)
        c = B.Case(r.cfg)
        c.init_fields(*r.fields)
        c.step(r.steps)
        c.read_fields()
        c.close()
        r.done = time.perf_counter() - t0
    makespan = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return _summary(reqs, makespan)


def compare(batched: dict, sequential: dict) -> dict:
    return {"batched": batched, "sequential": sequential,
            "throughput_ratio": round(batched["MLUPS"] / sequential["MLUPS"], 3),
            "p99_ratio": round(batched["latency_p99_s"] / sequential["latency_p99_s"], 3)}
