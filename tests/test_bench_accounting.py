"""The algorithmic byte counts behind the benchmark's roofline (each value a
kernel reads or writes, counted once, in its storage width), against the
per-kernel counts derived by hand from what each kernel reads and writes."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_fp32_d3q27_bytes_per_node():
    kb = bench.kernel_bytes(4)
    # moments: 46 populations in, phi, u*(3), P*, M2(6) out
    assert kb["moments"] == 46 * 4 + 11 * 4 == 228
    # pressure: P* (the previous P is already in it), u*(3), phi in, P out
    assert kb["pressure"] == 6 * 4
    # velocity: new P, u*(3), phi in, u(3) out
    assert kb["velocity"] == 8 * 4
    # collide: h(19), phi, u(3), M2(6) in, 46 populations out
    assert kb["collide"] == 19 * 4 + 10 * 4 + 46 * 4 == 300
    assert sum(kb.values()) == 584
    # state: populations, P and u, read and written once
    assert bench.state_bytes(4) == 2 * (46 * 4 + 4 * 4) == 400
    assert bench.state_bytes(2) == 2 * (46 * 2 + 4 * 4) == 216
    assert bench.state_bytes(8, aux_bytes=8, pops=18, dim=2) == 2 * (18 * 8 + 3 * 8) == 336


def test_fp16_bytes_per_node():
    kb = bench.kernel_bytes(2)
    # the 2-byte codecs read the previous step's phi (4 B) in both kernels
    # and the previous step's u (12 B) in moments; M2's six values take two
    # bytes each (phi, u*, P* stay 4-byte: 20 B)
    assert kb["moments"] == 46 * 2 + 4 + 12 + 20 + 12 == 140
    assert kb["collide"] == 19 * 2 + 4 + 16 + 12 + 46 * 2 == 162
    # 2D: three M2 values in two 32-bit words
    kb2 = bench.kernel_bytes(2, pops=18, dim=2, q_phase=9)
    assert kb2["moments"] == 18 * 2 + 4 + 8 + 16 + 8


def test_d3q19_hydro_populations():
    kb = bench.kernel_bytes(4, pops=38)
    assert kb["moments"] == 38 * 4 + 44
    assert kb["collide"] == 19 * 4 + 40 + 38 * 4
