"""The benchmark's contract on the host: one GPU only, and stored counter
traffic used only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_stored_traffic_only_for_matching_sources():
    import bench
    stored = json.load(open(os.path.join(ROOT, "profiles", "traffic_stencil27_160_fp64.json")))
    assert bench.stored_traffic(stored["kernel_source_hash"]) == stored["hbm_bytes_per_launch"]
    assert bench.stored_traffic("0" * 16) is None
    assert len(bench.kernel_source_hash()) == 16


def test_paper_context_is_context_only():
    import bench
    ctx = bench.PAPER_CONTEXT
    assert set(ctx["model_ceiling_gfs"]) == {"snb", "xeon_phi", "k20"}
    assert "context" in ctx["note"]


def test_errors_against_the_oracle_on_host():
    """The benchmark's error report: zero for the oracle's own products, and
    the normwise / componentwise errors of a known perturbation."""
    import numpy as np
    import bench
    import oracle
    import synth
    A = synth.lap5(12)
    x = synth.uniform(A.ncols, 7)
    xr = oracle.round_f32(x).astype(np.float64)
    y = oracle.crs_spmv_hi(A, x)
    yq = oracle.crs_spmv_hi(A, xr)
    bad = yq.copy()
    bad[5] += 1e-3
    out = bench.errors_vs_oracle(y, [("stencil27_160", "exact", "f32", yq), ("stencil27_160", "bad", "f32", bad)],
                                 {"stencil27_160": (A, x)})
    assert out["headline_fp64"]["normwise"] == 0 and out["headline_fp64"]["componentwise"] == 0
    assert out["stencil27_160"]["exact"] == {"normwise": 0.0, "componentwise": 0.0}
    scale = oracle.crs_absmv(A, xr)
    want_c = float("%.3g" % (1e-3 / scale[5]))
    want_n = float("%.3g" % (1e-3 / np.linalg.norm(yq)))
    assert out["stencil27_160"]["bad"] == {"normwise": want_n, "componentwise": want_c}


def test_source_hash_ignores_comments_only(tmp_path):
    """The hash that gates the stored counter traffic changes with the code
    and not with its comments or layout."""
    import bench
    a = tmp_path / "k.hip"
    a.write_text("// kernel\n__global__ void k(int *p) { p[0] = 1; /* one */ }\n")
    h0 = bench.source_hash([str(a)])
    a.write_text("// the kernel, reworded\n__global__ void k(int *p) {\n  p[0] = 1;  /* the value one */\n}\n")
    assert bench.source_hash([str(a)]) == h0
    a.write_text("// kernel\n__global__ void k(int *p) { p[0] = 2; /* one */ }\n")
    assert bench.source_hash([str(a)]) != h0


def test_read_write_bound_arithmetic():
    """The read/write bound of the benchmark line: reads at the read probe's
    rate, then writes at the write probe's rate, against the measured time;
    with counters, the same for the counted bytes."""
    import bench
    probes = {"read_gbs": 8000.0, "write_gbs": 4000.0}
    r = bench.read_write_bound(8e9, 4e9, probes, 2.5e-3)  # 1 ms of reads, 1 ms of writes
    assert r["us"] == 2000.0 and r["frac"] == 0.8
    r = bench.read_write_bound(8e9, 4e9, probes, 2.5e-3, traffic=(16e9, 0.0))
    assert "counted_frac" not in r  # a zero write count is no measurement
    r = bench.read_write_bound(8e9, 4e9, probes, 2.5e-3, traffic=(16e9, 4e9))
    assert r["counted_us"] == 3000.0 and r["counted_frac"] == 1.2
