"""Long runs of the large 3D workloads at their real sizes (GPU only).

    python -m paper_2512_01027_amd.longruns galilean [--out FILE]
    python -m paper_2512_01027_amd.longruns rising_bubble [--out FILE]
    python -m paper_2512_01027_amd.longruns dam_break [--out FILE]
    python -m paper_2512_01027_amd.longruns head_on [--out FILE]
    python -m paper_2512_01027_amd.longruns dam_block [--out FILE] [--store fp16|fp32] [--seconds T]

galilean
    The 128^3 droplet (R = 24) translated with u = (0.05, 0.02, 0) for 5000
    steps in FP64 and FP32 storage: shape drift ||phi(5000) - phi0 moved by
    (250, 100, 0)|| / ||phi0||, the centroid velocity error, and FP32
    against FP64 (relative L2 of phi, u and the mean-subtracted P).
rising_bubble
    The 256^3 rising bubble (walls in z, g = -1e-6 z, R = 32 at a quarter
    height) with FP32, FP16 and BF16 storage against the FP64 storage mode of
    the same library at steps 1000, 2000 and 4000: relative L2 of phi, u and
    the mean-subtracted P.  The FP64 mode is the reference at this size; it
    is itself held to the FP64 CPU reference on small and short cases and on
    sampled windows of this very workload.  FP16 is gated at 1e-3 on u and P.
dam_break
    The 512 x 256 x 256 dam break (walls on all faces, g = -2e-6 z) with FP16
    storage against FP32 storage at steps 5000, 10000 and 20000: the induced
    airflow error ||u_16 - u_32|| / ||u_32|| over the nodes where the FP32
    run has phi < 0.5.  A splash is chaotic, so this is reported, not gated.
head_on
    The head-on droplet collision at Re = 1715, We = 58.4 (two droplets of
    D = 64 nodes closing at U = 0.06 in a 256 x 192 x 192 periodic box,
    D3Q19) in FP32 and FP16 storage to 8 time units D / U: droplet count,
    disc radius / R, length along the axis / D, the largest air speed / U,
    and the FP16 airflow against FP32 over phi < 0.5.  Reported, not gated.
dam_block
    The dam break against a block in the container of Sec. III (585 x 182 x
    182 nodes, open top at P = 0, walls elsewhere): the front's position,
    the water reaching the block's side, the largest speed and phi's mass
    drift at fixed intervals.  The geometry run only: the experiment's
    sensor records are out of scope.

Every result is printed as one JSON line as soon as it is known (and
appended to --out when given), so a long run shows its progress.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import binding as B
from . import workloads as W


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class _Emit:
    def __init__(self, path):
        self.path = path

    def __call__(self, rec):
        line = json.dumps(rec)
        print(line, flush=True)
        if self.path:
            with open(self.path, "a") as fh:
                fh.write(line + "\n")


def _run(cfg, fields, marks, emit, tag, keep):
    """Run one case through the marks; return keep(fields) at each mark."""
    c = B.Case(cfg)
    c.init_fields(*fields)
    c.sync()
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    out, done, busy = [], 0, 0.0
    for m in marks:
        t0 = time.perf_counter()
        c.step(m - done)
        c.sync()
        busy += time.perf_counter() - t0
        done = m
        out.append(keep(c.read_fields()))
        d = c.diagnostics(allow_diverged=True)
        emit({"run": tag, "store": cfg["store"], "step": m, "MLUPS": round(n * done / busy / 1e6, 1),
              "nonfinite": d["nonfinite"], "umax": d["umax"]})
    c.close()
    return out


def _errors(got, ref):
    (pg, Pg, ug), (pr, Pr, ur) = got, ref
    return {"phi": _rel(pg, pr), "u": _rel(ug, ur), "P": _rel(Pg - Pg.mean(), Pr - Pr.mean())}


def galilean(emit, steps=5000, n=128):
    from . import analysis as A

    cfg, fields, _ = W.config_galilean_droplet_3d(n)
    u0 = (0.05, 0.02, 0.0)
    shift = tuple(int(round(v * steps)) for v in u0)
    out = {}
    for store in ("fp64", "fp32"):
        out[store] = _run(dict(cfg, store=store), fields, [steps], emit, "galilean", lambda f: f)[0]
        phi = out[store][0]
        # move the droplet back by the distance the flow carries it
        back = np.roll(phi, shift=(-shift[2], -shift[1], -shift[0]), axis=(0, 1, 2))
        c0 = A.centroid(1.0 - np.clip(fields[0], 0, 1))
        c1 = A.centroid(1.0 - np.clip(back, 0, 1))
        emit({"run": "galilean", "store": store, "step": steps,
              "shape_drift": float(f"{_rel(back, fields[0]):.3e}"),
              "centroid_velocity_error": [float(f"{(b - a) / steps:.3e}") for a, b in zip(c0, c1)]})
    emit({"run": "galilean", "compare": "fp32 vs fp64", "step": steps,
          **{k: float(f"{v:.3e}") for k, v in _errors(out["fp32"], out["fp64"]).items()}})
    return True


def rising_bubble(emit, marks=(1000, 2000, 4000), n=256):
    cfg, fields, _ = W.config_rising_bubble_3d(n, store="fp64")
    ref = _run(cfg, fields, marks, emit, "rising_bubble", lambda f: f)
    # the method's own response to a perturbation far below FP32 rounding
    # (phi0 x (1 + 1e-10 N(0,1)), PCG64 seed 17): the delta-theta switches
    # make the discrete map discontinuous, so no storage can stay closer to
    # the FP64 run than this
    rng = np.random.Generator(np.random.PCG64(17))
    phi_p = fields[0] * (1.0 + 1e-10 * rng.standard_normal(fields[0].shape))
    pert = _run(cfg, (phi_p, fields[1], fields[2]), marks, emit, "rising_bubble_perturbed", lambda f: f)
    for m, a, b in zip(marks, pert, ref):
        emit({"run": "rising_bubble", "compare": "fp64 perturbed 1e-10 vs fp64", "step": m,
              **{k: float(f"{v:.3e}") for k, v in _errors(a, b).items()}})
    del pert, phi_p
    ok = True
    for store in ("fp32", "fp16", "bf16"):
        got = _run(dict(cfg, store=store), fields, marks, emit, "rising_bubble", lambda f: f)
        for m, a, b in zip(marks, got, ref):
            e = _errors(a, b)
            gate = None
            if store == "fp16":
                gate = e["u"] <= 1e-3 and e["P"] <= 1e-3
                ok = ok and gate
            emit({"run": "rising_bubble", "compare": f"{store} vs fp64", "step": m,
                  **{k: float(f"{v:.3e}") for k, v in e.items()}, "fp16_gate_1e-3": gate})
    return ok


def dam_break(emit, marks=(5000, 10000, 20000), nu_light=0.15):
    cfg, fields, _ = W.config_dam_break_3d(store="fp32", nu_light=nu_light)
    emit({"run": "dam_break", "nu_water": cfg["nu_heavy"], "nu_air": cfg["nu_light"]})
    ref = _run(cfg, fields, marks, emit, "dam_break", lambda f: (f[0] < 0.5, f[2]))
    got = _run(dict(cfg, store="fp16"), fields, marks, emit, "dam_break", lambda f: f[2])
    for m, (air, u32), u16 in zip(marks, ref, got):
        emit({"run": "dam_break", "compare": "fp16 vs fp32", "step": m, "air_nodes": int(air.sum()),
              "airflow_rel_l2": float(f"{_rel(u16[:, air], u32[:, air]):.3e}"),
              "u_rel_l2_all": float(f"{_rel(u16, u32):.3e}")})
    return True


def head_on(emit, t_end=8.0, every=0.5):
    from . import analysis as A

    off = (0.37, 0.29, 0.61)  # off the grid's mirror planes
    cfg, fields, unit = W.config_head_on_collision(store="fp32", offset=off)
    D, U = 64.0, 0.06
    axis = (cfg["ny"] / 2.0 + off[1], cfg["nz"] / 2.0 + off[2])
    marks = [int(round(unit * every * (k + 1))) for k in range(int(round(t_end / every)))]

    def keep(f):
        phi, _, u = f
        r, L = A.collision_extent(phi, axis_yz=axis)
        return {"droplets": A.droplet_count(phi), "disc_radius_over_R": round(r / (D / 2), 3),
                "length_over_D": round(L / D, 3), "air_speed_over_U": round(A.max_air_speed(phi, u) / U, 4),
                "air": phi < 0.5, "u": u}

    out = {}
    for store in ("fp32", "fp16"):
        out[store] = _run(dict(cfg, store=store), fields, marks, emit, "head_on", keep)
        for m, rec in zip(marks, out[store]):
            emit({"run": "head_on", "store": store, "t_over_D_U": round(m / unit, 3),
                  **{k: v for k, v in rec.items() if k not in ("air", "u")}})
        if store == "fp32":
            continue
        for m, a, b in zip(marks, out["fp32"], out["fp16"]):
            air = a["air"]
            emit({"run": "head_on", "compare": "fp16 vs fp32", "t_over_D_U": round(m / unit, 3),
                  "airflow_rel_l2": float(f"{_rel(b['u'][:, air], a['u'][:, air]):.3e}")})
    return True


def dam_block(emit, store="fp16", seconds=2.0, every=0.1):
    """The geometry run: the water column released against the block, with
    the front's position (the smallest x where a column of the floor layer
    holds water), the water on the block's face side, the largest speed and
    phi's mass every `every` seconds of the workload's time scale."""
    cfg, fields, info = W.config_dam_break_block(store=store)
    per_s = info["steps_per_second"]
    marks = [int(round(per_s * every * (k + 1))) for k in range(int(round(seconds / every)))]
    face = info["block_face_x"]
    mass0 = float(fields[0].sum())

    def keep(f):
        phi, _, u = f
        wet = np.nonzero((phi[0] > 0.5).any(axis=0))[0]
        return {"front_x": int(wet.min()) if wet.size else None,
                "water_before_face": round(float(np.clip(phi[:, :, :face], 0, 1).sum()), 1),
                "umax": round(float(np.sqrt((u * u).sum(axis=0)).max()), 5),
                "phi_mass_rel_drift": float(f"{(float(phi.sum()) - mass0) / mass0:.3e}")}

    recs = _run(cfg, fields, marks, emit, "dam_block", keep)
    for m, rec in zip(marks, recs):
        emit({"run": "dam_block", "store": store, "step": m, "t_over_unit": round(m / per_s, 3), **rec})
    return True


def main(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=("galilean", "rising_bubble", "dam_break", "head_on", "dam_block"))
    ap.add_argument("--out", default=None)
    ap.add_argument("--store", default="fp16")
    ap.add_argument("--seconds", type=float, default=2.0)
    ap.add_argument("--nu-light", type=float, default=0.15, help="dam_break: air viscosity")
    args = ap.parse_args(argv)
    emit = _Emit(args.out)
    if args.which == "dam_block":
        ok = dam_block(emit, args.store, args.seconds)
    elif args.which == "dam_break":
        ok = dam_break(emit, nu_light=args.nu_light)
    else:
        ok = {"galilean": galilean, "rising_bubble": rising_bubble, "dam_break": dam_break,
              "head_on": head_on}[args.which](emit)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
