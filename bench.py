"""Benchmark of the SELL-C-sigma spMVM on one MI355X.

One step is one FP64 SELL-C-sigma spMVM y = A x on the 27-point stencil over
a 160^3 grid (n = 4,096,000, 109,215,352 nonzeros; values U[0.5,1.5), x
U[-1,1)), the regular, bandwidth-bound workload. The timed region holds K
back-to-back products with matrix, x and y resident in device memory,
bracketed by device synchronisations and timed with HIP events on the stream
the kernels run on. GF/s counts the useful 2 * nnz flops per product.

Printed as one JSON line, with
  roofline: the method's algorithmic bytes of one product (padded matrix at
            12 B per slot, x and y once, chunk metadata) over the measured
            time per product, against the 8 TB/s HBM peak; beside them the
            bytes the x-window format itself moves (10 B per slot and the
            window tables) and their fraction; traffic = HBM bytes per
            product from the hardware counters recorded under profiles/ when
            the kernel sources are unchanged since, else null;
  cpu_baseline: the CPU oracle (CRS, double, OpenMP over rows) on the same
            matrix on the host cores;
  errors_vs_oracle: normwise and componentwise errors of the headline FP64
            product and of every reduced-precision result against the
            oracle (computed after all timing, in the CPU leg);
  forms:    FP32 / BF16 value storage (x window and int32 indices), the
            block form (k right-hand sides) on the power-law n = 1,000,000
            matrix, the batched launch over 64 power-law matrices, and the
            power-law n = 2,000,000 matrix;
  probes:   read-only and copy bandwidth (the paper's roofline b).
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spMVM GF/s + HBM GB/s vs 8 TB/s roofline; FP64 plain vs block-k/FP32/BF16"
PEAK_HBM_GBS = 8000.0
HEADLINE = dict(workload="stencil27_160", C=32, sigma=1)
# The paper's own figures on its 2013 hardware (Sect. 5.2): context, not
# targets. Model ceilings P_bar = b * beta / 6 with beta = 1 and the best
# measured bandwidth of each device; the dense 8000^2 matrix; rail4284 on
# the K20 with one and 32 threads per row.
PAPER_CONTEXT = {
    "note": "2013 hardware (Sandy Bridge Xeon E5-2680, Xeon Phi 5110P, Tesla K20c); context only",
    "model_ceiling_gfs": {"snb": 7.2, "xeon_phi": 27.5, "k20": 25.2},
    "dense_8000_gfs": {"snb": 7.3, "xeon_phi": 23.0, "k20": 17.0, "k20_16_threads_per_row": 31.0},
    "rail4284_k20_gfs": {"1_thread_per_row": 0.5, "32_threads_per_row": 4.5},
}


def source_hash(paths) -> str:
    """Hash of C/C++/HIP sources without their comments and with whitespace
    collapsed, so that an edit of a comment leaves it unchanged."""
    h = hashlib.sha256()
    for p in sorted(paths):
        with open(p, encoding="utf-8") as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(os.path.basename(p).encode())
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    """Hash of the HIP sources: the stored counter traffic is valid only for
    the code it was measured on."""
    return source_hash(glob.glob(os.path.join(ROOT, "paper_1307_6209_amd", "csrc", "*")))


def stored_traffic(src_hash: str, split: bool = False):
    """The stored HBM bytes per launch of the headline kernel (with split,
    the (fetched, written) pair), when taken on the current kernel sources."""
    p = TRAFFIC_FILE
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != src_hash:
        return None
    if split:
        return d.get("fetch_bytes_per_launch"), d.get("write_bytes_per_launch")
    return d.get("hbm_bytes_per_launch")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stencil27_160_fp64.json")


def store_traffic(fetch_db: str, write_db: str) -> dict:
    """Host side: from the rocprofv3 databases of the two counter runs of
    --pmc-pass (FETCH_SIZE, then WRITE_SIZE), the headline kernel's HBM
    bytes per dispatch, each counter scaled by what it reads for the copy
    probe of known size run in the same pass (512 MiB read and written), and
    stored with the hash of the kernel sources they were taken on."""
    import sqlite3

    def per_kernel(db, counter):
        con = sqlite3.connect(db)
        cols = [r[1] for r in con.execute("pragma table_info(counters_collection)")]
        vals = {}
        for row in con.execute("select * from counters_collection"):
            d = dict(zip(cols, row))
            if d["counter_name"] == counter:
                vals.setdefault(d["kernel_name"], []).append(float(d["value"]))
        return vals

    fetch, write = per_kernel(fetch_db, "FETCH_SIZE"), per_kernel(write_db, "WRITE_SIZE")
    prod = [k for k in fetch if k.startswith("void sell::dev::k_spmv")]
    if not prod or not any("k_copy" in k for k in fetch):
        raise SystemExit("store-traffic: no product or copy-probe dispatches in %s (run bench.py --pmc-pass)" % fetch_db)
    head = max(prod, key=lambda k: len(fetch[k]))  # the 5 products of the pass
    copy = [k for k in fetch if "k_copy" in k][0]
    copy_bytes = 1 << 29  # half of the probe's 1 GiB is read, half written
    mean = lambda v: sum(v) / len(v)  # noqa: E731
    ff = copy_bytes / (mean(fetch[copy]) * 1024.0)
    wf = copy_bytes / (mean(write[copy]) * 1024.0)
    fb, wb = mean(fetch[head]) * 1024.0 * ff, mean(write[head]) * 1024.0 * wf
    out = {"kernel": head, "workload": "stencil27_160, SELL-32-1, FP64",
           "command_fetch": "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_fetch -o fetch -- python3 bench.py --pmc-pass",
           "command_write": "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_write -o write -- python3 bench.py --pmc-pass",
           "fetch_kib_per_dispatch": round(mean(fetch[head]), 1), "write_kib_per_dispatch": round(mean(write[head]), 1),
           "copy_calibration": {"bytes_read_and_written": copy_bytes, "fetch_kib": round(mean(fetch[copy]), 1),
                                "write_kib": round(mean(write[copy]), 1), "fetch_factor": round(ff, 4),
                                "write_factor": round(wf, 4)},
           "hbm_bytes_per_launch": int(round(fb + wb)), "fetch_bytes_per_launch": int(round(fb)),
           "write_bytes_per_launch": int(round(wb)), "kernel_source_hash": kernel_source_hash()}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


def to_dev(A):
    import torch
    return (torch.from_numpy(A.rpt).cuda(), torch.from_numpy(A.col).cuda(), torch.from_numpy(A.val).cuda())


def progress(*a):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print("bench:", *a, file=sys.stderr, flush=True)


def time_calls(fn, steps: int, warmup: int, repeats: int = 5):
    """Seconds per call of fn after `warmup` calls: `steps` back-to-back calls
    cut into `repeats` groups, each timed by its own events; the median group
    average (repeats = 1: the average over exactly `steps` calls)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    per = max(1, steps // repeats) if repeats > 1 else steps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(repeats)]
    for e0, e1 in evs:
        e0.record()
        for _ in range(per):
            fn()
        e1.record()
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) * 1e-3 / per for e0, e1 in evs)
    return ts[len(ts) // 2]


def cpu_baseline(A, x, budget_s: float = 10.0, C: int = 32, sigma: int = 1) -> dict:
    """The oracle's CRS product on the host cores (OpenMP over rows), the
    same product on one core, and the oracle's SELL-C-sigma build time."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    sched = oracle.schedule_for(A)

    def per_call(nthreads, budget):
        t0 = time.perf_counter()
        oracle.crs_spmv(A, x, nthreads=nthreads, sched=sched)
        t1 = time.perf_counter() - t0
        reps = int(max(3, min(20000, budget / max(t1, 1e-6))))
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.crs_spmv(A, x, nthreads=nthreads, sched=sched)
        return (time.perf_counter() - t0) / reps, reps

    t, reps = per_call(threads, budget_s)
    t_one, reps_one = per_call(1, budget_s / 2)
    t0 = time.perf_counter()
    oracle.sell_build(A, C, sigma)
    t_build = time.perf_counter() - t0
    return {"value": round(2.0 * A.nnz / t * 1e-9, 3), "unit": "GF/s", "cores": threads, "kind": "oracle",
            "sample": "full %s matrix (%d nonzeros), CRS product in double, %d repetitions, OpenMP %s" % (
                A.name, A.nnz, reps, "static" if sched == 0 else "guided,1"),
            "one_core_value": round(2.0 * A.nnz / t_one * 1e-9, 3), "one_core_repetitions": reps_one,
            "sell_build_ms": round(t_build * 1e3, 1), "sell_build_format": "SELL-%d-%d" % (C, sigma)}


def errors_vs_oracle(y_head, checks, checks_x) -> dict:
    """Errors of the benchmarked results against the oracle (long double
    CRS product, rounded once): the FP64 headline product against A x, and
    every reduced-precision result against A x^ (x^ = x rounded to binary32,
    the input those forms multiply), as the normwise error
    ||y - y_ref||_2 / ||y_ref||_2 and the componentwise
    max_i |y_i - y_ref_i| / (|A||x^|)_i."""
    import numpy as np
    import oracle

    def errs(y, yref, scale):
        d = np.abs(y - yref)
        return {"normwise": float("%.3g" % (np.linalg.norm(d) / max(np.linalg.norm(yref), 1e-300))),
                "componentwise": float("%.3g" % np.max(d / np.where(scale > 0, scale, 1.0)))}

    A, x = checks_x["stencil27_160"]
    out = {"headline_fp64": errs(y_head, oracle.crs_spmv_hi(A, x), oracle.crs_absmv(A, x))}
    out["headline_fp64"]["componentwise_bound"] = 1e-13
    refs = {}
    for wl, key, _vd, y in checks:
        if wl not in refs:
            A, x = checks_x[wl]
            xr = oracle.round_f32(x).astype(np.float64)
            refs[wl] = (oracle.crs_spmv_hi(A, xr), oracle.crs_absmv(A, xr))
        yref, scale = refs[wl]
        out.setdefault(wl, {})[key] = errs(y, yref, scale)
    return out


def cpu_baseline_leg(A, x, y_head, checks, checks_x) -> tuple:
    """The part of the benchmark that runs the CPU oracle: its timing on the
    host cores, and the errors of the benchmarked results against it (after
    every timed region)."""
    base = cpu_baseline(A, x, C=HEADLINE["C"], sigma=HEADLINE["sigma"])
    return base, errors_vs_oracle(y_head, checks, checks_x)


def graph_time(fn, launches: int, replays: int = 5) -> float:
    """Seconds per call of fn from a captured graph of `launches` calls,
    replayed back to back (launch overhead amortised)."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        fn()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            for _ in range(launches):
                fn()
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(replays):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / (replays * launches)


def cold_time(fn, flush, reps: int = 21) -> float:
    """Median seconds of single calls of fn, each timed by its own events
    right after a read-modify-write of `flush` (1 GiB: evicts every L2 and
    the 256 MB Infinity Cache)."""
    import torch
    fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        flush.add_(1.0)
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    return ts[len(ts) // 2] * 1e-3


def read_write_bound(read_bytes, write_bytes, probes, sec, traffic=None) -> dict:
    """Time to read read_bytes at the read probe's rate and then write
    write_bytes at the write probe's rate, and the measured time's fraction
    of it; with stored counters (fetched, written) also for those bytes."""
    t = read_bytes / (probes["read_gbs"] * 1e9) + write_bytes / (probes["write_gbs"] * 1e9)
    out = {"read_bytes": int(read_bytes), "write_bytes": int(write_bytes), "us": round(t * 1e6, 2),
           "frac": round(t / sec, 4),
           "basis": "bytes the format moves: reads at read_gbs, the result's writes at write_gbs, in turn"}
    if traffic and traffic[0] and traffic[1]:
        tc = traffic[0] / (probes["read_gbs"] * 1e9) + traffic[1] / (probes["write_gbs"] * 1e9)
        out["counted_us"] = round(tc * 1e6, 2)
        out["counted_frac"] = round(tc / sec, 4)
    return out


def block_ceiling(A, inf, k, t, probes) -> dict:
    """Ceilings of the block form Y = A X (k = 16, 32, 64) from the probes,
    against its measured time t. (1) One random row of X (8k bytes) per
    nonzero at the random-row probe's rate over an array of X's size, the
    matrix (12 B per slot, cl and cs, the permutation) at the read rate and
    Y at the write rate, in turn. (2) The rows of X and Y at the rate of the
    probe that mixes them (four random rows read per row written), the
    matrix at the read rate."""
    from paper_1307_6209_amd import sellcs
    rows_pow2 = 1 << (A.nrows - 1).bit_length()
    rows_gbs = sellcs.sell_probe_bandwidth({16: 3, 32: 4, 64: 5}[k], rows_pow2 * 8 * k, 5)
    mixed_gbs = sellcs.sell_probe_bandwidth({16: 7, 32: 8, 64: 9}[k], rows_pow2 * 8 * k, 5)
    mat = 12 * inf["padded"] + 12 * inf["nchunks"] + 4 * A.nrows
    tc = (8.0 * k * A.nnz / (rows_gbs * 1e9) + mat / (probes["read_gbs"] * 1e9)
          + 8.0 * k * A.nrows / (probes["write_gbs"] * 1e9))
    tm = 8.0 * k * (A.nnz + A.nrows) / (mixed_gbs * 1e9) + mat / (probes["read_gbs"] * 1e9)
    return {"rows_probe_gbs": round(rows_gbs, 1), "ceiling_us": round(tc * 1e6, 2),
            "us": round(t * 1e6, 2), "frac": round(tc / t, 4),
            "mixed_probe_gbs": round(mixed_gbs, 1),
            "mixed_ceiling_us": round(tm * 1e6, 2), "frac_mixed": round(tm / t, 4),
            "x_rows_per_s_g": round(A.nnz / t * 1e-9, 2),
            "probe_rows_per_s_g": round(rows_gbs / (8.0 * k), 2)}


def run_forms(args, probes, checks, checks_x) -> dict:
    import torch
    import numpy as np
    import synth
    from paper_1307_6209_amd import sellcs
    out = {}
    flush = torch.zeros(1 << 27, dtype=torch.float64, device="cuda")
    # the small, cache-resident 5-point Laplacian 128^2 (SELL-32-1): per-call
    # time from back-to-back launches and from a graph of 1000 launches
    A = synth.workload("lap5_128")
    r, c, v = to_dev(A)
    h = sellcs.sell_build(r, c, v, A.ncols, 32, 1)
    x = torch.from_numpy(synth.uniform(A.ncols, synth.SEED_X)).cuda()
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    t_eager = time_calls(lambda: sellcs.sell_spmv(h, x, y), 1000, 20)
    t_graph = graph_time(lambda: sellcs.sell_spmv(h, x, y), 1000)
    out["lap5_128"] = {"us_per_call_stream": round(t_eager * 1e6, 3), "us_per_call_graph": round(t_graph * 1e6, 3),
                       "gfs_graph": round(2.0 * A.nnz / t_graph * 1e-9, 2)}
    h.close()
    del r, c, v
    # block form on the power-law n = 1,000,000 matrix
    progress("block form")
    A = synth.workload("powerlaw_1m")
    r, c, v = to_dev(A)
    spmmv, ceiling = {}, {}
    for C, sg in ((32, 1024), (32, A.nrows)):
        h = sellcs.sell_build(r, c, v, A.ncols, C, sg, kmax=64)
        inf = h.info
        for k in (1, 4, 8, 16, 32, 64):
            X = torch.from_numpy(synth.block_vector(A.ncols, k)).cuda()
            Y = torch.empty(A.nrows, k, dtype=torch.float64, device="cuda")
            t = time_calls(lambda: sellcs.sell_spmmv(h, X, Y), max(10, args.steps // 10), 3)
            spmmv["C%d_sigma%d_k%d" % (C, sg, k)] = round(2.0 * A.nnz * k / t * 1e-9, 2)
            if sg == A.nrows and k in (16, 32, 64):
                ceiling["k%d" % k] = block_ceiling(A, inf, k, t, probes)
            if sg == A.nrows and k in (1, 8, 32):
                t = cold_time(lambda: sellcs.sell_spmmv(h, X, Y), flush)
                spmmv["C%d_sigma%d_k%d_cold" % (C, sg, k)] = round(2.0 * A.nnz * k / t * 1e-9, 2)
        h.close()
    out["spmmv_powerlaw_1m_gfs"] = spmmv
    out["spmmv_powerlaw_1m_sigma_n_ceiling"] = ceiling
    # the block form autotuned over C, sigma and the pass width (0: the
    # automatic choice, which includes the one-pass kernels)
    tuned = {}
    for k in (8, 32):
        tk = sellcs.sell_autotune(r, c, v, A.ncols, k=k, C=(16, 32, 64), sigma=(1024, A.nrows), unroll=(8,),
                                  ktile=(0, 8, 16, 32), reps=5)
        tuned["k%d" % k] = {key: tk[key] for key in ("C", "sigma", "ktile", "candidates")}
        tuned["k%d" % k]["gfs"] = round(tk["gflops"], 2)
    out["spmmv_powerlaw_1m_autotuned"] = tuned
    del r, c, v
    # 64 uneven power-law matrices in one graph launch (sigma 1024, and
    # sigma = n_b, the fastest on these matrices in the sigma sweep)
    progress("batched launch")
    mats = synth.batch_workload(64)
    devs = [to_dev(B) for B in mats]
    xs = [torch.from_numpy(synth.uniform(B.ncols, 5 + i)).cuda() for i, B in enumerate(mats)]
    ys = [torch.empty(B.nrows, dtype=torch.float64, device="cuda") for B in mats]
    nnz = sum(B.nnz for B in mats)
    for tag, sig in (("sigma1024", lambda B: 1024), ("sigma_n", lambda B: B.nrows)):
        hs = [sellcs.sell_build(rr, cc, vv, B.ncols, 32, sig(B)) for (rr, cc, vv), B in zip(devs, mats)]
        b = sellcs.sell_batch_create(hs)
        bv = sellcs.BatchVectors(b, xs, ys)  # marshalled once: the launches are not host-bound
        t = time_calls(lambda: sellcs.sell_batch_spmv(b, bv), max(10, args.steps // 10), 3)
        t_seq = time_calls(lambda: [sellcs.sell_spmv(hh, xx, yy) for hh, xx, yy in zip(hs, xs, ys)],
                           max(5, args.steps // 50), 2)
        t_cold = cold_time(lambda: sellcs.sell_batch_spmv(b, bv), flush)
        bp = sellcs.sell_batch_create_persistent(hs)
        bpv = sellcs.BatchVectors(bp, xs, ys)
        t_pers = time_calls(lambda: sellcs.sell_batch_spmv(bp, bpv), max(10, args.steps // 10), 3)
        out["batch64_%s" % tag] = {"gfs": round(2.0 * nnz / t * 1e-9, 2), "us": round(t * 1e6, 2),
                                   "separate_launches_us": round(t_seq * 1e6, 2),
                                   "cold_gfs": round(2.0 * nnz / t_cold * 1e-9, 2),
                                   "persistent_us": round(t_pers * 1e6, 2)}
        bp.close()
        b.close()
        for hh in hs:
            hh.close()
    # one C for the batch and a sigma per matrix, chosen by the batch autotuner
    tb = sellcs.sell_batch_autotune([(rr, cc, vv, B.ncols) for (rr, cc, vv), B in zip(devs, mats)],
                                    C=(16, 32, 64), sigma=(1, 64, 1024, 1 << 40), reps=20)
    hist = {}
    for sg in tb["sigmas"]:
        key = "all rows" if sg >= 1 << 40 else str(sg)
        hist[key] = hist.get(key, 0) + 1
    out["batch64_autotuned"] = {"C": tb["C"], "gfs": round(tb["gflops"], 2), "us": round(tb["us_per_call"], 2),
                                "sigma_counts": hist, "candidates": tb["candidates"]}
    # the autotuned batch in both launch forms, vectors marshalled once
    hs = [sellcs.sell_build(rr, cc, vv, B.ncols, tb["C"], sg) for ((rr, cc, vv), B), sg in
          zip(zip(devs, mats), tb["sigmas"])]
    for key, form in (("us_timed", sellcs.sell_batch_create), ("persistent_us", sellcs.sell_batch_create_persistent)):
        bb = form(hs)
        bbv = sellcs.BatchVectors(bb, xs, ys)
        t = time_calls(lambda: sellcs.sell_batch_spmv(bb, bbv), max(10, args.steps // 10), 3)
        out["batch64_autotuned"][key] = round(t * 1e6, 2)
        bb.close()
    for hh in hs:
        hh.close()
    del devs
    # power-law n = 2,000,000: plain and globally sorted
    progress("power-law 2M")
    A = synth.workload("powerlaw_2m")
    r, c, v = to_dev(A)
    x = torch.from_numpy(synth.uniform(A.ncols)).cuda()
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    pl = {}
    for C, s in ((32, 1), (32, 2**14), (32, A.nrows), (16, A.nrows)):
        h = sellcs.sell_build(r, c, v, A.ncols, C, s)
        t = time_calls(lambda: sellcs.sell_spmv(h, x, y), max(20, args.steps // 5), 5)
        t_cold = cold_time(lambda: sellcs.sell_spmv(h, x, y), flush)
        pl["C%d_sigma%d" % (C, s)] = {"gfs": round(2.0 * A.nnz / t * 1e-9, 2), "beta": round(h.info["beta"], 4),
                                      "cold_gfs": round(2.0 * A.nnz / t_cold * 1e-9, 2),
                                      # one x gather per nonzero, against the random-gather probe
                                      "frac_of_gather_probe": round(8.0 * A.nnz / t * 1e-9 / probes["gather_16mib_gbs"],
                                                                    4)}
        h.close()
    # the C x sigma grid of the irregular workload: beta and GF/s for C in
    # {16, 32, 64, 128} and sigma in {1, C, 2^10, 2^14, n} (sigma = C gives the
    # layout of sigma = 1)
    grid = {}
    for C in (16, 32, 64, 128):
        for s in (1, C, 2**10, 2**14, A.nrows):
            h = sellcs.sell_build(r, c, v, A.ncols, C, s)
            t = time_calls(lambda: sellcs.sell_spmv(h, x, y), max(10, args.steps // 20), 3)
            grid["C%d_sigma%d" % (C, s)] = {"beta": round(h.info["beta"], 4), "gfs": round(2.0 * A.nnz / t * 1e-9, 2)}
            h.close()
    pl["c_sigma_grid"] = grid
    # lanes stopped at their rows' ends (row lengths kept, the GPU form of the
    # kernel of Sect. 3.4): the loads of padding are skipped, the idle lanes
    # of a chunk's short rows remain
    for s in (1, 2**10, 2**14, A.nrows):
        h = sellcs.sell_build(r, c, v, A.ncols, 32, s, row_lengths=True)
        t = time_calls(lambda: sellcs.sell_spmv(h, x, y), max(20, args.steps // 5), 5)
        pl["C32_sigma%d_row_lengths" % s] = {"gfs": round(2.0 * A.nnz / t * 1e-9, 2), "beta": round(h.info["beta"], 4)}
        h.close()
    # reduced-precision storage at the globally sorted layout (int32 column
    # indices: the uniform half of the columns leaves no x window); the
    # results go to the oracle leg for their errors
    xf = x.float()
    for vd, ad in (("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")):
        h = sellcs.sell_build(r, c, v, A.ncols, 32, A.nrows, val_dtype=vd, acc_dtype=ad)
        yf = torch.empty(A.nrows, dtype=torch.float64 if ad == "f64" else torch.float32, device="cuda")
        t = time_calls(lambda: sellcs.sell_spmv(h, xf, yf), max(20, args.steps // 5), 5)
        key = "C32_sigma%d_%s_val_%s_acc" % (A.nrows, vd, ad)
        pl[key] = {"gfs": round(2.0 * A.nnz / t * 1e-9, 2), "index": "int32" if h.info["xwindow"] == 0 else "uint16"}
        checks.append(("powerlaw_2m", key, vd, yf.double().cpu().numpy()))
        h.close()
    checks_x["powerlaw_2m"] = (A, x.cpu().numpy())
    hs_ = sellcs.sell_build(r, c, v, A.ncols, 32, A.nrows, permute_columns=True)
    xp = torch.empty_like(x)
    sellcs.sell_permute(hs_, x, xp)
    t = time_calls(lambda: sellcs.sell_spmv(hs_, xp, y), max(20, args.steps // 5), 5)
    pl["C32_sigma%d_symmetric" % A.nrows] = {"gfs": round(2.0 * A.nnz / t * 1e-9, 2), "beta": round(hs_.info["beta"], 4)}
    hs_.close()
    for L in (1, 4):
        t = time_calls(lambda: sellcs.sell_crs_spmv(r, c, v, x, y, A.ncols, lanes_per_row=L), max(20, args.steps // 5), 5)
        pl["crs_L%d" % L] = {"gfs": round(2.0 * A.nnz / t * 1e-9, 2)}
    out["powerlaw_2m"] = pl
    del r, c, v
    # few rows, long rows: dense 8000^2 and a rail4284-shaped matrix (Sect. 5.2)
    progress("dense and rail-shaped")
    for name, Cs in (("dense_8000", (32, 128)), ("rail_like", (32, 128))):
        B = synth.workload(name)
        rr, cc, vv = to_dev(B)
        xb = torch.from_numpy(synth.uniform(B.ncols)).cuda()
        yb = torch.empty(B.nrows, dtype=torch.float64, device="cuda")
        res = {}
        for C in Cs:
            for sg in (1, B.nrows):
                hb = sellcs.sell_build(rr, cc, vv, B.ncols, C, sg)
                t = time_calls(lambda: sellcs.sell_spmv(hb, xb, yb), max(20, args.steps // 10), 5)
                res["C%d_sigma%d" % (C, sg)] = {"gfs": round(2.0 * B.nnz / t * 1e-9, 2), "beta": round(hb.info["beta"], 4)}
                hb.close()
        t = time_calls(lambda: sellcs.sell_crs_spmv(rr, cc, vv, xb, yb, B.ncols, lanes_per_row=64),
                       max(20, args.steps // 10), 5)
        res["crs_L64"] = {"gfs": round(2.0 * B.nnz / t * 1e-9, 2)}
        out[name] = res
        del rr, cc, vv
    return out


def model_report(model, b_read, gfs, achieved, inf, A, sizes, traffic) -> dict:
    """The code-balance model (Sect. 4) with the measured read bandwidth as b:
    balance at the ideal alpha = 1/N_nzc, the resulting bound, and alpha
    solved from the counter traffic when it is available."""
    nnzr = A.nnz / A.nrows
    bal = model.general_balance(1.0 / nnzr, inf["beta"], nnzr, inf["C"], 1, sizes)
    p_model = b_read / bal
    rep = {"b_read_gbs": b_read, "frac_of_b_read": round(achieved / b_read, 4),
           "balance_ideal_alpha_bytes_per_flop": round(bal, 4), "P_model_gfs": round(p_model, 1),
           "frac_of_model": round(gfs / p_model, 4), "P_bar_paper_gfs": round(model.best_attainable(b_read, inf["beta"]), 1)}
    if traffic:
        alpha = model.general_alpha_from_volume(traffic, A.nnz, inf["beta"], nnzr, inf["C"], 1, sizes)
        bal_m = model.general_balance(alpha, inf["beta"], nnzr, inf["C"], 1, sizes)
        rep["alpha_measured"] = round(alpha, 5)
        rep["alpha_ideal"] = round(1.0 / nnzr, 5)
        # the model's bound with the measured right-hand-side traffic
        rep["P_model_alpha_measured_gfs"] = round(b_read / bal_m, 1)
        rep["frac_of_model_alpha_measured"] = round(gfs / (b_read / bal_m), 4)
    return rep


SWEEP_SIGMAS = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768, 65536, 131072,
                262144, 524288, 1048576, 2_000_000]


def sigma_sweep(args):
    """SELL-32-sigma on the power-law n = 2,000,000 matrix for sigma = 1 ..
    n: beta, time and GF/s per sigma (the analog of the paper's sigma study of
    kkt_power, Sect. 5.3). Under a counter run (--pmc-pass) each sigma runs
    exactly 3 products so the dispatches can be attributed. --row-lengths:
    the same with the lanes stopped at their rows' ends."""
    import torch
    import synth
    from paper_1307_6209_amd import sellcs
    A = synth.workload("powerlaw_2m")
    r, c, v = to_dev(A)
    x = torch.from_numpy(synth.uniform(A.ncols, synth.SEED_X + 1)).cuda()
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    rows = []
    for sg in SWEEP_SIGMAS:
        h = sellcs.sell_build(r, c, v, A.ncols, 32, sg, row_lengths=args.row_lengths)
        if args.pmc_pass:
            for _ in range(3):
                sellcs.sell_spmv(h, x, y)
            torch.cuda.synchronize()
            t = float("nan")
        else:
            t = time_calls(lambda: sellcs.sell_spmv(h, x, y), 100, 10)
        inf = h.info
        rows.append({"sigma": sg, "beta": inf["beta"], "padded": inf["padded"], "nchunks": inf["nchunks"],
                     "nsplit": inf["nsplit"], "us": round(t * 1e6, 2), "gfs": round(2.0 * A.nnz / t * 1e-9, 2)})
        h.close()
    if args.pmc_pass:
        sellcs.sell_probe_bandwidth(1, 1 << 30, 1)
        torch.cuda.synchronize()
    print(json.dumps({"sigma_sweep": "powerlaw_2m", "C": 32, "n": A.nrows, "nnz": A.nnz,
                      "row_lengths": bool(args.row_lengths), "rows": rows}))


def block_pass(args):
    """The block form on the power-law n = 1,000,000 matrix, SELL-32-n, k =
    16, 32, 64 (the one-pass kernel with 8 or 16 lanes per row): time per
    product, or under a counter run (--pmc-pass) exactly 3 products per k and
    one copy probe for the counter calibration."""
    import torch
    import synth
    from paper_1307_6209_amd import sellcs
    A = synth.workload("powerlaw_1m")
    r, c, v = to_dev(A)
    h = sellcs.sell_build(r, c, v, A.ncols, 32, A.nrows, kmax=64)
    inf = h.info
    rows = []
    for k in (16, 32, 64):
        X = torch.from_numpy(synth.block_vector(A.ncols, k)).cuda()
        Y = torch.empty(A.nrows, k, dtype=torch.float64, device="cuda")
        if args.pmc_pass:
            for _ in range(3):
                sellcs.sell_spmmv(h, X, Y)
            torch.cuda.synchronize()
            t = float("nan")
        else:
            t = time_calls(lambda: sellcs.sell_spmmv(h, X, Y), 50, 5)
        rows.append({"k": k, "us": round(t * 1e6, 2), "gfs": round(2.0 * A.nnz * k / t * 1e-9, 2)})
        del X, Y
    probes = None
    if args.pmc_pass:
        sellcs.sell_probe_bandwidth(1, 1 << 30, 1)
        torch.cuda.synchronize()
    else:
        probes = {"read_gbs": round(sellcs.sell_probe_bandwidth(0, 4 << 30, 10), 1),
                  "write_gbs": round(sellcs.sell_probe_bandwidth(6, 4 << 30, 10), 1)}
        for row in rows:
            row["ceiling"] = block_ceiling(A, inf, row["k"], row["us"] * 1e-6, probes)
    print(json.dumps({"block_pass": "powerlaw_1m", "C": 32, "sigma": A.nrows, "n": A.nrows, "nnz": A.nnz,
                      "padded": inf["padded"], "beta": inf["beta"], "nsplit": inf["nsplit"], "probes": probes,
                      "rows": rows}))


def batch_pass(args):
    """The batched launch over the 64 power-law matrices (n log-uniform in
    [10^3, 2*10^5]), SELL-32-n_b: time per launch of both forms, or under a
    counter run (--pmc-pass) exactly 3 launches of each form and one copy
    probe for the counter calibration."""
    import torch
    import synth
    from paper_1307_6209_amd import sellcs
    mats = synth.batch_workload(64)
    devs = [to_dev(B) for B in mats]
    xs = [torch.from_numpy(synth.uniform(B.ncols, 5 + i)).cuda() for i, B in enumerate(mats)]
    ys = [torch.empty(B.nrows, dtype=torch.float64, device="cuda") for B in mats]
    hs = [sellcs.sell_build(rr, cc, vv, B.ncols, 32, B.nrows) for (rr, cc, vv), B in zip(devs, mats)]
    nnz = sum(B.nnz for B in mats)
    rows = []
    for form in ("sell_batch_create", "sell_batch_create_persistent"):
        b = getattr(sellcs, form)(hs)
        bv = sellcs.BatchVectors(b, xs, ys)
        if args.pmc_pass:
            for _ in range(3):
                sellcs.sell_batch_spmv(b, bv)
            torch.cuda.synchronize()
            t = float("nan")
        else:
            t = time_calls(lambda: sellcs.sell_batch_spmv(b, bv), 200, 20)
        rows.append({"form": form, "us": round(t * 1e6, 2), "gfs": round(2.0 * nnz / t * 1e-9, 2)})
        b.close()
    if args.pmc_pass:
        sellcs.sell_probe_bandwidth(1, 1 << 30, 1)
        torch.cuda.synchronize()
    print(json.dumps({"batch_pass": "powerlaw x 64", "C": 32, "sigma": "n_b", "rows_total": sum(B.nrows for B in mats),
                      "nnz": nnz, "padded": sum(h.info["padded"] for h in hs),
                      "x_bytes": 8 * sum(B.ncols for B in mats), "rows": rows}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-forms", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed headline products (for a kernel trace of exactly that kernel)")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="short run for hardware counters: a few products and one copy probe")
    ap.add_argument("--sigma-sweep", action="store_true", help="SELL-32-sigma sweep on the power-law matrix")
    ap.add_argument("--row-lengths", action="store_true",
                    help="with --sigma-sweep: lanes stopped at their rows' ends (build option row_lengths)")
    ap.add_argument("--block-pass", action="store_true",
                    help="block form k = 16, 32, 64 on the power-law 1M matrix (with --pmc-pass: for counters)")
    ap.add_argument("--batch-pass", action="store_true",
                    help="batched launch over 64 power-law matrices (with --pmc-pass: for counters)")
    ap.add_argument("--store-traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="host only: write the headline's counter traffic from two --pmc-pass counter runs")
    ap.add_argument("--probe-sweep", action="store_true",
                    help="random-gather and random-row probes over array sizes 1 MiB .. 4 GiB, and the read probe")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the SELL-C-sigma product here is a single-device kernel "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.store_traffic:
        print(json.dumps(store_traffic(*args.store_traffic)))
        return

    import torch
    import synth
    from paper_1307_6209_amd import model, sellcs

    torch.cuda.set_device(0)
    if args.sigma_sweep:
        sigma_sweep(args)
        return
    if args.block_pass:
        block_pass(args)
        return
    if args.batch_pass:
        batch_pass(args)
        return
    if args.probe_sweep:
        res = {"read_4gib_gbs": round(sellcs.sell_probe_bandwidth(0, 4 << 30, 10), 1)}
        for mib in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 4096):
            g = sellcs.sell_probe_bandwidth(2, mib << 20, 5)
            res["gather_%dmib_ggather_per_s" % mib] = round(g / 8.0, 1)
        # random whole rows of 128 / 256 / 512 bytes (the block form's X rows
        # at k = 16 / 32 / 64), in G rows/s
        for kind, rb in ((3, 128), (4, 256), (5, 512)):
            for mib in (4, 16, 64, 128, 256, 512, 1024, 4096):
                g = sellcs.sell_probe_bandwidth(kind, mib << 20, 5)
                res["rows%d_%dmib_grows_per_s" % (rb, mib)] = round(g / rb, 2)
        # four random rows read per row written in order (the block form's
        # mix), in G rows/s read and written
        for kind, rb in ((7, 128), (8, 256), (9, 512)):
            for mib in (64, 128, 256, 512, 1024):
                g = sellcs.sell_probe_bandwidth(kind, mib << 20, 5)
                res["rows%d_mixed_%dmib_grows_per_s" % (rb, mib)] = round(g / rb, 2)
        # write-only and copy streams over 4 GiB
        res["write_4gib_gbs"] = round(sellcs.sell_probe_bandwidth(6, 4 << 30, 10), 1)
        res["copy_4gib_gbs"] = round(sellcs.sell_probe_bandwidth(1, 4 << 30, 10), 1)
        print(json.dumps({"probe_sweep": res}))
        return
    A = synth.workload(HEADLINE["workload"])
    x_np = synth.uniform(A.ncols, synth.SEED_X + 2)
    r, c, v = to_dev(A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = sellcs.sell_build(r, c, v, A.ncols, HEADLINE["C"], HEADLINE["sigma"])
    build_s = time.perf_counter() - t0
    inf = h.info
    x = torch.from_numpy(x_np).cuda()
    y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")

    if args.pmc_pass:
        for _ in range(5):
            sellcs.sell_spmv(h, x, y)
        torch.cuda.synchronize()
        sellcs.sell_probe_bandwidth(1, 1 << 30, 1)  # copy of 512 MiB -> 512 MiB: the counter calibration
        torch.cuda.synchronize()
        print(json.dumps({"pmc_pass": True, "padded": inf["padded"]}))
        return

    probes = {"read_gbs": round(sellcs.sell_probe_bandwidth(0, 4 << 30, 10), 1),
              "copy_gbs": round(sellcs.sell_probe_bandwidth(1, 4 << 30, 10), 1),
              # random 8-byte gathers (8 B counted per gather) over arrays the
              # size of the power-law x (16 MiB) and far beyond the MALL
              "gather_16mib_gbs": round(sellcs.sell_probe_bandwidth(2, 16 << 20, 5), 1),
              "gather_2gib_gbs": round(sellcs.sell_probe_bandwidth(2, 2 << 30, 5), 1),
              "write_gbs": round(sellcs.sell_probe_bandwidth(6, 4 << 30, 10), 1)}
    # reads and writes taking turns on the memory: a copy of B bytes would
    # take B / read + B / write; the copy probe checks that model
    probes["copy_predicted_by_read_and_write_gbs"] = round(
        2.0 / (1.0 / probes["read_gbs"] + 1.0 / probes["write_gbs"]), 1)

    sec = time_calls(lambda: sellcs.sell_spmv(h, x, y), args.steps, args.warmup, repeats=1)
    gfs = 2.0 * A.nnz / sec * 1e-9
    torch.cuda.synchronize()
    y_head = y.cpu().numpy()
    # algorithmic bytes of the method (12 B per padded slot: FP64 value and
    # int32 column index; x and y once; the permutation when sigma > 1; cl and
    # cs per chunk) and the bytes the x-window format itself moves (2-byte
    # window positions plus the window tables)
    sizes_alg = model.sizes_for("f64", "f64", HEADLINE["sigma"] > 1)
    alg = model.algorithmic_bytes(A.nrows, A.ncols, inf["padded"], inf["nchunks"], 1, sizes_alg)
    sizes = model.sizes_for("f64", "f64", HEADLINE["sigma"] > 1, xwindow=inf["xwindow"] == 1,
                            segments_per_chunk=inf["xsegments"] / max(1, inf["nchunks"]),
                            group_chunks=max(1, inf["xwindow_group_chunks"]))
    moved = model.algorithmic_bytes(A.nrows, A.ncols, inf["padded"], inf["nchunks"], 1, sizes)
    achieved = alg / sec * 1e-9
    achieved_moved = moved / sec * 1e-9
    src_hash = kernel_source_hash()
    traffic = stored_traffic(src_hash)
    nnzr = A.nnz / A.nrows
    line = {
        "metric": METRIC,
        "value": round(gfs, 2),
        "unit": "GF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "stencil27_160 (27-point stencil, 160^3 grid)", "n": A.nrows, "nnz": A.nnz,
                   "format": "SELL-%d-%d" % (HEADLINE["C"], HEADLINE["sigma"]), "beta": round(inf["beta"], 6),
                   "padded_slots": inf["padded"],
                   "index": "uint16 window positions (x window staged in LDS)" if inf["xwindow"] else "int32",
                   "x_window_segments": inf["xsegments"], "x_window_max_elements": inf["xwindow_max"],
                   "x_window_group_chunks": inf["xwindow_group_chunks"],
                   "values": "f64", "x": "f64", "y": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg,
                     "algorithmic_bytes_basis": "12 B per padded slot (FP64 value + int32 index), x and y once, "
                                                "12 B per chunk (cl, cs)",
                     "moved_bytes_per_launch": moved,
                     "moved_bytes_basis": "the x-window format: 10 B per slot (FP64 value + 16-bit window "
                                          "position), x and y once, chunk metadata and window tables",
                     "achieved_moved_bytes": round(achieved_moved, 1),
                     "frac_moved_bytes": round(achieved_moved / PEAK_HBM_GBS, 4),
                     "traffic_source": ("stored FETCH_SIZE + WRITE_SIZE counter measurement "
                                        "(profiles/traffic_stencil27_160_fp64.json), copy-calibrated, taken on "
                                        "kernel sources with hash %s" % src_hash) if traffic else
                                       "null: no counter measurement for the current kernel sources (hash %s)"
                                       % src_hash},
        "model": model_report(model, probes["read_gbs"], gfs, achieved_moved, inf, A, sizes, traffic),
        "read_write_bound": read_write_bound(moved - 8 * A.nrows, 8 * A.nrows, probes, sec,
                                             stored_traffic(src_hash, split=True) if traffic else None),
        "build_ms": round(build_s * 1e3, 2),
        "probes": probes,
        "kernel_source_hash": src_hash,
        "paper_context": PAPER_CONTEXT,
    }
    if args.headline_only:
        h.close()
        print(json.dumps(line))
        return
    checks, checks_x = [], {"stencil27_160": (A, x_np)}
    progress("headline %.2f GF/s; precision forms" % gfs)
    # precision forms on the same matrix (values FP32 / BF16, x rounded to
    # FP32, accumulation FP32 / FP64), at the headline C and at C = 64, with
    # the x window (16-bit window positions) and with the int32 column
    # indices; the results go to the oracle leg for their errors
    forms = {"x_window_uint16_positions": {}, "int32_col_indices": {}}
    xf = x.float()
    for path, xw in (("x_window_uint16_positions", 0), ("int32_col_indices", -1)):
        for vd, ad in (("f32", "f32"), ("f32", "f64"), ("bf16", "f32"), ("bf16", "f64")):
            for C in sorted({HEADLINE["C"], 64}):
                hf = sellcs.sell_build(r, c, v, A.ncols, C, HEADLINE["sigma"], val_dtype=vd, acc_dtype=ad, xwindow=xw)
                if hf.info["xwindow"] != (1 if xw == 0 else 0):
                    raise RuntimeError("%s: unexpected x path for %s/%s C=%d" % (path, vd, ad, C))
                yf = torch.empty(A.nrows, dtype=torch.float64 if ad == "f64" else torch.float32, device="cuda")
                t = time_calls(lambda: sellcs.sell_spmv(hf, xf, yf), max(50, args.steps // 4), 10)
                key = "%s_val_%s_acc_C%d" % (vd, ad, C)
                forms[path][key] = round(2.0 * A.nnz / t * 1e-9, 2)
                checks.append(("stencil27_160", "%s.%s" % (path, key), vd, yf.double().cpu().numpy()))
                hf.close()
    line["forms_stencil27_160_gfs"] = forms
    # the paper's comparison on one device: CRS (one lane per row, and L lanes
    # per row with a cross-lane reduction) against SELL-C-sigma
    crs = {}
    for L in (1, 4, 8, 16, 32):
        t = time_calls(lambda: sellcs.sell_crs_spmv(r, c, v, x, y, A.ncols, lanes_per_row=L), max(50, args.steps // 4),
                       10)
        crs["crs_L%d" % L] = round(2.0 * A.nnz / t * 1e-9, 2)
    crs["sell_%d_%d" % (HEADLINE["C"], HEADLINE["sigma"])] = round(gfs, 2)
    # the same layout multiplied with the global column indices (x gathered
    # through L2) instead of the x window in LDS
    hg = sellcs.sell_build(r, c, v, A.ncols, HEADLINE["C"], HEADLINE["sigma"], xwindow=-1)
    t = time_calls(lambda: sellcs.sell_spmv(hg, x, y), max(50, args.steps // 4), 10)
    crs["sell_%d_%d_global_index" % (HEADLINE["C"], HEADLINE["sigma"])] = round(2.0 * A.nnz / t * 1e-9, 2)
    hg.close()
    line["crs_vs_sell_stencil27_160_gfs"] = crs
    # SELL-32-1 against SELL-32-sigma autotuned over sigma = 2^0 .. 2^17 and n, unroll and x path
    sig_space = tuple(1 << i for i in range(18)) + (A.nrows,)
    tuned = sellcs.sell_autotune(r, c, v, A.ncols, k=1, C=(32,), sigma=sig_space, unroll=(4, 8, 16), xwindow=(-1, 0),
                                 xwindow_chunks=(4, 8), reps=20)
    line["autotuned_stencil27_160"] = {key: (round(val, 3) if isinstance(val, float) else val)
                                       for key, val in tuned.items()}
    h.close()
    del r, c, v
    if not args.no_forms:
        line["forms"] = run_forms(args, probes, checks, checks_x)
    if not args.no_cpu:
        progress("CPU oracle leg")
        line["cpu_baseline"], line["errors_vs_oracle"] = cpu_baseline_leg(A, x_np, y_head, checks, checks_x)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
