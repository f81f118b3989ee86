"""Summaries of rocprofv3 CSV output for the kernels of libpulbm.so.

    python -m paper_2512_01027_amd.profsum stats  <dir with *_kernel_stats.csv>
    python -m paper_2512_01027_amd.profsum hbm    <fetch dir> <write dir> <copy fetch dir> <copy write dir> <nodes>
    python -m paper_2512_01027_amd.profsum issue  <dir of an SQ counter run> <trace dir>

``hbm`` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch) into HBM bytes per
launch.  Each counter is scaled by what it reads for a plain device copy of
known size (the ``--copy-probe`` run of bench.py: bytes moved / counter
value), and the result is printed per kernel and per lattice node, followed
by one ``traffic_json`` line that bench.py reads.  The line carries the
SHA-256 of the kernel sources, so a summary taken before a kernel change is
not used for the changed kernel.

``issue`` turns SQ instruction counters (SQ_WAVES, SQ_INSTS_VALU,
SQ_INSTS_LDS, SQ_INSTS_SALU) into instructions per wavefront and sets the
VALU issue time they imply beside the kernel's average duration from a
kernel trace.  Issue model: without packed FP32 a wave64 VALU instruction
occupies its SIMD for 4 cycles; 1024 SIMDs (256 CUs x 4) at 2.4 GHz.
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/kernels.hpp", "csrc/lattice.hpp", "csrc/codec.hpp", "csrc/pulbm.hip")

# rocprofv3 leaves kernels templated on _Float16 in their mangled form:
# _ZN5pulbm<len><name>ILi<lattice set>E<type>[Lb<0|1>E[Li<parity>E]]E...
_MANGLED = re.compile(r"_ZN5pulbm\d+(k_[a-z]+)ILi(\d)E(DF16_|[dft])(?:Lb([01])E(?:Li(\d)E)?)?E")
_TYPES = {"DF16_": "_Float16", "d": "double", "f": "float", "t": "unsigned short"}


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name: str) -> str:
    m = _MANGLED.match(name)
    if m:
        flag = "" if m.group(4) is None else (", true" if m.group(4) == "1" else ", false")
        par = "" if m.group(5) is None else f", {m.group(5)}"
        name = f"pulbm::{m.group(1)}<{m.group(2)}, {_TYPES[m.group(3)]}{flag}{par}>"
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*", "", name)
    return name.replace("void ", "")


def _one(pattern):
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise SystemExit(f"no file matches {pattern}")
    return hits[0]


def counters(d):
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))):
        acc[(short(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def stats(d):
    rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*kernel_stats.csv")))))
    out = ["kernel | calls | avg_us | min_us | max_us | pct"]
    for r in rows:
        out.append(f"{short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f}")
    return "\n".join(out)


def hbm(fetch_dir, write_dir, cfetch_dir, cwrite_dir, nodes):
    f, w = counters(fetch_dir), counters(write_dir)
    cf, cw = counters(cfetch_dir), counters(cwrite_dir)
    copy = "__amd_rocclr_copyBuffer"
    # the copy probe moves 1 GiB: bytes read = bytes written = 2^30
    kf = 2 ** 30 / (cf[(copy, "FETCH_SIZE")] * 1024)
    kw = 2 ** 30 / (cw[(copy, "WRITE_SIZE")] * 1024)
    out = [f"calibration: FETCH_SIZE x {kf:.4f}, WRITE_SIZE x {kw:.4f} (1 GiB device copy)",
           "kernel | FETCH KiB/dispatch | WRITE KiB/dispatch | HBM read MB | HBM write MB | read B/node | write B/node"]
    table = {}
    for (k, c) in sorted(f):
        if c != "FETCH_SIZE" or not k.startswith("pulbm::"):
            continue
        fk, wk = f[(k, "FETCH_SIZE")], w.get((k, "WRITE_SIZE"), 0.0)
        rb, wb = fk * 1024 * kf, wk * 1024 * kw
        table[k] = {"read_bytes": rb, "write_bytes": wb}
        out.append(f"{k} | {fk:.1f} | {wk:.1f} | {rb / 1e6:.1f} | {wb / 1e6:.1f} | "
                   f"{rb / nodes:.1f} | {wb / nodes:.1f}")
    out.append("traffic_json " + json.dumps({"source_sha256": source_hash(), "nodes": nodes,
                                            "calibration": {"FETCH_SIZE": kf, "WRITE_SIZE": kw},
                                            "kernels": table}))
    return "\n".join(out)


SIMDS, CLOCK_HZ, VALU_CYCLES = 1024, 2.4e9, 4


def issue(sq_dir, trace_dir):
    c = counters(sq_dir)
    dur = {}
    for r in csv.DictReader(open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv")))):
        dur[short(r["Name"])] = float(r["AverageNs"]) / 1e3
    out = ["kernel | waves/dispatch | VALU/wave | LDS/wave | SALU/wave | VALU issue us | avg us | issue share"]
    for (k, name) in sorted(c):
        if name != "SQ_WAVES" or not k.startswith("pulbm::") or c[(k, name)] <= 0:
            continue
        waves = c[(k, "SQ_WAVES")]
        valu = c.get((k, "SQ_INSTS_VALU"), 0.0) / waves
        lds = c.get((k, "SQ_INSTS_LDS"), 0.0) / waves
        salu = c.get((k, "SQ_INSTS_SALU"), 0.0) / waves
        t_issue = waves * valu * VALU_CYCLES / (SIMDS * CLOCK_HZ) * 1e6
        d = dur.get(k)
        share = f"{t_issue / d:.2f}" if d else "-"
        out.append(f"{k} | {waves:.0f} | {valu:.0f} | {lds:.0f} | {salu:.0f} | {t_issue:.1f} | "
                   f"{d if d is not None else float('nan'):.2f} | {share}")
    return "\n".join(out)


def load_traffic(path):
    """The traffic_json record of a committed summary, or None."""
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_json "):
            return json.loads(line[len("traffic_json "):])
    return None


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(stats(argv[1]))
    elif len(argv) == 6 and argv[0] == "hbm":
        print(hbm(argv[1], argv[2], argv[3], argv[4], int(argv[5])))
    elif len(argv) == 3 and argv[0] == "issue":
        print(issue(argv[1], argv[2]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
