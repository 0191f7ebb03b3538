"""Benchmark of the DID hot path on one MI355X.

A step is one full DID iteration (Alg. 3: column pass with the C sweep, V and W messages,
their fixed-order reduction, and the incremental B update) on the resident workload
M = 5000, N = 1,000,000, K = 50 in float32 with 64 column blocks; X is generated on the
device (X = B0 C0 + |0.01 N(0,1)|, U[0,1] factors) and stays in HBM.

Prints one JSON line:
  value          iterations/s of the whole job (inputs resident in HBM at the start),
  roofline       the dominant kernel (column or row pass) against the roofline that bounds
                 it: HBM (algorithmic bytes against 8 TB/s) or the float32-accurate MFMA
                 peak of its split-fp16 products, whichever time floor is larger; with
                 iter_frac (the whole iteration's algorithmic bytes against 8 TB/s) and
                 limiter (what the committed SQ counters show stalls the pass),
  precision_form X stored as bf16 with the residual refreshed every iteration or carried
                 and refreshed every 10: iterations/s, speedup over the plain form, and the
                 objective error against the FP64 oracle (original X and bf16(X)) on the
                 first column block over 50 iterations,
  batched_form   48 served-distribution jobs advanced as one batch against one after
                 another: instance-iterations/s and speedup, and the batch again with the
                 tiles did_autotune picks per shape class against the default tiles,
  served_form    a shortened served run (300 jobs of the Poisson schedule, their X
                 generated on the device before the clock starts): solves/s, p50/p99
                 latency, queue depth, share of jobs stopped by the 1e-4 rule, and the
                 same jobs under a 1e-2 rule (early retirements free slots),
  cpu_baseline   the FP64 oracle timed on a bounded sample of the same workload.

``--workload paper`` runs the experiments' synthetic shape instead (M = 5, K = 3,
N = 10^5 ... 10^8, X = B0 C0 with U[0,1] factors): iterations and seconds to the stopping
rule ||E^t||^2 <= 1e-6 ||E^0||^2 for DID and for the DBCD ablation, beside the paper's
Table 2 (16 CPU nodes), and iterations/s at N = 10^8 as the line's value.

``--workload batch`` advances a set of jobs drawn from the served workload's shape
distribution (M ~ U{100..4000}, N ~ LogU[1e3, 2e5], K ~ U{5..64}) for --steps
iterations, once one instance after another (the plain form) and once as one batch
(grouped persistent kernels replayed from a hipGraph), and reports the batched rate, its
speedup and the bitwise agreement of the results, then tunes the tiles of each shape
class among the jobs and reports the tuned batch against the default tiles.  ``--workload serve`` runs the serving
form: Poisson arrivals at 200 jobs/s, admission by a 200 GB budget, continuous batching,
each job to 50 iterations or a relative objective change below 1e-4; it reports solves/s
and p50/p99 latency from the scheduled arrival to retirement.  ``--workload nsweep`` times
the large workload's recipe at N = 1.25e5 ... 1e6 (the method's cost per iteration is
linear in N) and reports the time per iteration and per 10^5 columns at each size.
``--workload planted`` (500 x 2000, K = 10) and ``--workload image`` (784 x 70000, K = 16)
time the small shapes, whose iterations are replayed from a captured graph, beside the
launch floor: the replay time of a graph of as many empty dependent kernels.

The engine keeps float32 X in 32x32 tile order (one copy per pass, made at init, or at a
served job's admission) for the MFMA-path workloads, the batch and both served workloads;
--x-given reads it as given (column-major) instead.  The tiled copies triple each served
job's X memory, and serving is faster with them (1000 jobs: 87–93 against 68 solves/s).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--x-given]
                       [--workload large|large_bf16|image|planted|nsweep|paper|batch|serve]
                       [--serve-jobs J] [--serve-slots S] [--serve-bf16] [--serve-tiled]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DID iters/s + HBM GB/s (M=5000,N=1e6,K=50); served solves/s, p50/p99 latency"
PEAK_F16_MFMA_TFLOPS = 2500.0  # MI355X dense fp16 (and bf16) matrix peak
# The passes form every float32 product from three fp16 MFMA products of scaled two-way
# splits of the operands, so their float32-accurate peak is the fp16 peak over three.
SPLIT_PRODUCTS = 3
PEAK_SPLIT_TFLOPS = PEAK_F16_MFMA_TFLOPS / SPLIT_PRODUCTS
PEAK_HBM_GBS = 8000.0
# the arithmetic the path computes in: products float32-accurate from three fp16 MFMAs of
# scaled two-way splits with float32 accumulation; sweep, B update and objective in float64
DTYPE = "f32 (split-fp16x3 MFMA, fp32 accumulate; fp64 sweep, B update, objective)"

WORKLOADS = {
    "large": dict(M=5000, N=1_000_000, K=50, n_blocks=64,
                  desc="plain FP32 DID, M=5000 N=1000000 K=50, 64 column blocks, X=B0*C0+|0.01*N(0,1)|, "
                       "B0,C0~U[0,1], X resident in HBM"),
    "large_bf16": dict(M=5000, N=1_000_000, K=50, n_blocks=64, x_bf16=True,
                       desc="precision form: X stored as bf16 (RNE), B/C/residual float32-accurate, float64 "
                            "objective; M=5000 N=1000000 K=50, 64 column blocks, X=B0*C0+|0.01*N(0,1)|"),
    "image": dict(M=784, N=70_000, K=16, n_blocks=4,
                  desc="plain FP32 DID, M=784 N=70000 K=16, 4 column blocks, image-like X in [0,1]"),
    "planted": dict(M=500, N=2000, K=10, n_blocks=1,
                    desc="plain FP32 DID, M=500 N=2000 K=10, noiseless X=B0*C0"),
    "batch": dict(M=0, N=0, K=0, n_blocks=0, jobs=48,
                  desc="batched form: 48 jobs with M~U{100..4000}, N~LogU[1e3,2e5], K~U{5..64}, "
                       "X=max(0,B0*C0+0.02*N(0,1)), advanced together vs one after another"),
    "serve": dict(M=0, N=0, K=0, n_blocks=0, jobs=1000,
                  desc="serving form: Poisson arrivals at 200 jobs/s, M~U{100..4000}, N~LogU[1e3,2e5], "
                       "K~U{5..64}, X=max(0,B0*C0+0.02*N(0,1)) float32, 200 GB budget, <=50 iterations or "
                       "relative objective change <1e-4"),
    "nsweep": dict(M=5000, N=1_000_000, K=50, n_blocks=64, sizes=(125_000, 250_000, 500_000, 1_000_000),
                   desc="linear-in-N sweep of the large workload's recipe: M=5000 K=50, 64 column blocks, "
                        "N=125000..1000000, X=B0*C0+|0.01*N(0,1)|, X resident in HBM in tile order"),
    "paper": dict(M=5, N=100_000_000, K=3, n_blocks=16,
                  desc="experiments' synthetic shape: M=5 K=3, N=1e5..1e8, X=B0*C0 with B0,C0~U[0,1], "
                       "stopping rule ||E||^2 <= 1e-6 ||E0||^2, DID and DBCD (thin-matrix path)"),
}

# Table 2 of the paper (16 CPU nodes, one core each; C + GSL + OpenMPI): iterations to the
# stopping rule and seconds for DID and DBCD on the synthetic sets M = 5, K = 3.
PAPER_TABLE2 = {
    100_000: dict(iterations=549, did_s=1.17, dbcd_s=1.42),
    1_000_000: dict(iterations=396, did_s=8.61, dbcd_s=14.04),
    10_000_000: dict(iterations=654, did_s=106.60, dbcd_s=126.01),
    100_000_000: dict(iterations=302, did_s=610.09, dbcd_s=785.57),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_counts(M, N, K, xbytes=4):
    """Algorithmic work of one iteration and of the dominant kernel.

    Iteration bytes: X read once (xbytes MN: 4 for float32, 2 for the bf16 storage form), C
    read and written (8KN), B read (4MK).  A pass (column or row) per launch: flops 4MNK
    (E = X - BC and H = B^T E, or E' and W = E' C'^T, 2MNK each); bytes xbytes MN + 8KN.
    """
    return dict(
        iter_bytes=xbytes * M * N + 8.0 * K * N + 4.0 * M * K,
        pass_flops=4.0 * M * N * K,
        pass_bytes=xbytes * M * N + 8.0 * K * N,
    )


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("did_kernels.hip", "did_kernels.h", "did_thin.hip"):
        with open(os.path.join(ROOT, "paper_1802_08938_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None.

    Used only if the summary was taken on the current kernel source (hash match)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def sq_limiter(kernel):
    """What limits a pass, from the committed SQ counter summary (when it was taken on the
    current kernel sources): MFMA busy fraction, non-MFMA VALU instructions per MFMA and
    the share of wave cycles spent waiting.  None when the summary is stale or absent."""
    path = os.path.join(ROOT, "profiles", "sq_counters_large.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if f"kernel source sha256[:16]: {kernel_source_hash()}" not in text:
        return None
    col = 1 if kernel == "column_pass" else 2
    vals = {}
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 3:
            vals[cells[0]] = cells[col]
    try:
        mfma = float(vals["MFMA busy per SIMD, fraction of busy cycles (`SQ_VALU_MFMA_BUSY_CYCLES` / 1024 / busy cycles)"])
        valu = float(vals["non-MFMA VALU instructions per MFMA"])
        wait = float(vals["`SQ_WAIT_ANY` / `SQ_WAVE_CYCLES`"])
        clk = float(vals["implied clock, GHz (busy cycles / duration)"])
    except (KeyError, ValueError):
        return None
    # one wave64 VALU instruction occupies the SIMD 4 cycles, an MFMA 32x32x16 32 cycles;
    # the two overlap only in part (a wave's VALU work runs beside an MFMA in flight)
    valu_busy = mfma * valu * 4.0 / 32.0
    issue = mfma + valu_busy
    if issue >= 0.9:
        kind = "issue (MFMA and VALU pipes saturated)"
    elif wait >= 0.25:
        kind = "latency and issue (waves wait on memory/LDS while MFMA+VALU fill part of the cycles)"
    else:
        kind = "mixed"
    return {"label": kind, "mfma_busy": mfma, "valu_per_mfma": valu, "valu_busy_est": round(valu_busy, 3),
            "mfma_plus_valu_est": round(issue, 3),
            "wait_frac": wait, "clock_ghz": clk, "source": "profiles/sq_counters_large.md"}


def timed_iterations(torch, did, h, stream, warmup, steps, profile_iters=3):
    """ms per iteration over `steps` timed iterations (HIP events on the engine's stream,
    no per-stage events), then per-stage milliseconds from `profile_iters` profiled ones."""
    did.did_iterate(h, warmup)
    did.did_sync(h)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    did.did_iterate(h, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    stages, n_it = {}, 0
    if profile_iters:
        did.did_profile(h, True)
        did.did_iterate(h, profile_iters)
        stages, n_it = did.did_profile_read(h)
        did.did_profile(h, False)
    return ms, stages, max(n_it, 1)


def make_input(torch, name, cfg):
    from workloads import image_like, large_halfnormal_device, planted_lowrank

    M, N, K = cfg["M"], cfg["N"], cfg["K"]
    if name in ("large", "large_bf16"):
        return large_halfnormal_device(torch, M=M, N=N, K=K, seed=3, n_blocks=cfg["n_blocks"])
    import numpy as np

    X = image_like(M, N, K, seed=2)[0] if name == "image" else planted_lowrank(M, N, K, seed=1)[0]
    return torch.from_numpy(np.ascontiguousarray(X.astype(np.float32).T)).to("cuda")


def cpu_baseline(name, cfg):
    """Time the FP64 oracle on a bounded sample of the workload (about 10-30 s of CPU)."""
    import numpy as np
    import threadpoolctl

    import oracle
    from workloads import image_like, large_halfnormal, planted_lowrank, uniform_init

    M, N, K = cfg["M"], cfg["N"], cfg["K"]
    if name in ("large", "large_bf16"):
        X, _ = large_halfnormal(M, N, K, seed=3, n_blocks=cfg["n_blocks"], take_blocks=1)
        frac = X.shape[1] / N
        sample = (f"one oracle DID iteration on column block 0 ({M}x{X.shape[1]}, 1/{cfg['n_blocks']} "
                  f"of the workload), scaled x{cfg['n_blocks']}: per-iteration cost is linear in N")
    elif name == "image":
        X = image_like(M, N, K, seed=2)[0]
        frac = 1.0
        sample = "one oracle DID iteration on the full workload"
    else:
        X = planted_lowrank(M, N, K, seed=1)[0]
        frac = 1.0
        sample = "oracle DID iterations on the full workload"
    X = X.astype(np.float32).astype(np.float64)
    B0, C0 = uniform_init(M, X.shape[1], K, seed=12345)
    info = threadpoolctl.threadpool_info()
    threads = max([d.get("num_threads", 1) for d in info] or [1])
    reps = 1 if name != "planted" else 20
    t0 = time.perf_counter()
    oracle.did_run(X, B0, C0, reps, P=1, history=False)
    dt = (time.perf_counter() - t0) / reps
    it_s = frac / dt  # iterations/s of the full workload
    # the same sample on one core (the paper's nodes ran one core each)
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        oracle.did_run(X, B0, C0, reps, P=1, history=False)
        dt1 = (time.perf_counter() - t0) / reps
    return {"value": it_s, "unit": "iter/s", "cores": threads, "kind": "oracle",
            "sample": sample + f"; {dt:.2f} s per sampled iteration; numpy float64, BLAS threads={threads}, "
                               f"host cpu_count={os.cpu_count()}",
            "single_core": {"value": frac / dt1, "unit": "iter/s", "cores": 1,
                            "seconds_per_sampled_iteration": round(dt1, 3)}}


def device_env(torch):
    """The device and software the numbers were taken on."""
    p = torch.cuda.get_device_properties(0)
    env = {"device": p.name, "gcn_arch": getattr(p, "gcnArchName", None),
           "compute_units": p.multi_processor_count, "hbm_bytes": p.total_memory,
           "hip": torch.version.hip, "torch": torch.__version__}
    try:
        from ctypes import byref, c_int, cdll

        hip = cdll.LoadLibrary("libamdhip64.so")
        clk = c_int(0)
        # hipDeviceAttributeClockRate (kHz): the peak engine clock
        attr = 5
        if hip.hipDeviceGetAttribute(byref(clk), attr, 0) == 0:
            env["max_engine_clock_mhz"] = clk.value // 1000
    except OSError:
        pass
    return env


def launch_floor(torch, n_kernels, replays=200):
    """Time per replay of a captured graph of n_kernels dependent one-element kernels
    (torch's in-place add): what launching one iteration's kernels costs when they do no
    work, the floor for shapes whose kernels are short."""
    x = torch.zeros(1, device="cuda")
    for _ in range(3):
        x.add_(1.0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(n_kernels):
            x.add_(1.0)
    for _ in range(10):
        g.replay()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(replays):
        g.replay()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / replays


# kernels one iteration of the MFMA path launches: column pass, f reduction, clearing of
# the C maxima, sweep, W-order packing, V partials, V reduction, row pass, W reduction,
# clearing of the B maxima, B update, H-order packing, G reduction
KERNELS_PER_ITERATION = 13


def emit(torch, line):
    line["env"] = device_env(torch)
    print(json.dumps(line), flush=True)


def _solve_to_eps(torch, did, X, M, N, K, alg, stream, eps, cap, n_blocks):
    """Iterations to the stopping rule from the seed-12345 initial factors, then the time of
    exactly that many iterations from the same start (HIP events on the engine's stream)."""
    def start():
        o = did.did_default_opts()
        o.n_blocks = n_blocks
        o.borrow_x = 1
        o.algorithm = alg
        o.stream = stream.cuda_stream
        return did.did_init_ex(X, M, N, K, 12345, o)

    h = start()
    try:
        did.did_iterate(h, cap)
        f = did.did_history(h) + [did.did_objective(h)]
    finally:
        did.did_free(h)
    t_eps = next((t for t, v in enumerate(f) if v <= eps * f[0]), None)
    if t_eps is None:
        return None, None, f[-1] / f[0]
    h = start()
    try:
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        did.did_iterate(h, t_eps)
        ev1.record(stream)
        torch.cuda.synchronize()
        seconds = ev0.elapsed_time(ev1) / 1e3
    finally:
        did.did_free(h)
    return t_eps, seconds, f[t_eps] / f[0]


def run_paper_shape(args, torch, did):
    from workloads import paper_synthetic_device

    cfg = WORKLOADS["paper"]
    M, K = cfg["M"], cfg["K"]
    stream = torch.cuda.Stream()
    table = []
    X = None
    sizes = [n for n in sorted(PAPER_TABLE2) if n <= args.paper_max_n]
    for N in sizes:
        del X
        torch.cuda.empty_cache()
        log(f"paper shape N={N}: generating")
        X = paper_synthetic_device(torch, N, M=M, K=K, seed=4)
        torch.cuda.synchronize()
        row = {"N": N}
        if args.no_table:
            continue
        for name, alg in (("did", did.DID_ALG_DID), ("dbcd", did.DID_ALG_DBCD)):
            log(f"paper shape N={N}: {name} to eps")
            t, sec, ratio = _solve_to_eps(torch, did, X, M, N, K, alg, stream, 1e-6, 5000, cfg["n_blocks"])
            row[f"{name}_iterations"] = t
            row[f"{name}_seconds"] = None if sec is None else round(sec, 5)
            row[f"{name}_final_ratio"] = ratio
        ref = PAPER_TABLE2[N]
        row["paper_iterations"] = ref["iterations"]
        row["paper_did_seconds"] = ref["did_s"]
        row["paper_dbcd_seconds"] = ref["dbcd_s"]
        table.append(row)
    # steady-state rate at the largest N, DID, with the per-stage split
    N = sizes[-1]
    opts = did.did_default_opts()
    opts.n_blocks = cfg["n_blocks"]
    opts.borrow_x = 1
    opts.stream = stream.cuda_stream
    h = did.did_init_ex(X, M, N, K, 12345, opts)
    try:
        did.did_iterate(h, args.warmup)
        did.did_profile(h, True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        log(f"timing {args.steps} DID steps at N={N}")
        ev0.record(stream)
        did.did_iterate(h, args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        stages, n_it = did.did_profile_read(h)
        did.did_profile(h, False)
    finally:
        did.did_free(h)
    kern_ms = stages["column_pass"] / max(n_it, 1)
    # thin pass: X read once (4MN), C read and written (8KN)
    kbytes = 4.0 * M * N + 8.0 * K * N
    achieved = kbytes / (kern_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 4),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 data; fp64 sweep, messages and objective (thin path, no MFMA)",
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "M": M, "N": N, "K": K, "n_blocks": cfg["n_blocks"]},
        "stage_ms_per_iter": {k: round(v / max(n_it, 1), 4) for k, v in stages.items()},
        "roofline": {"bound": "hbm", "kernel": "thin_pass", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic("thin_pass", "paper"),
                     "kernel_ms": round(kern_ms, 4), "bytes_per_launch": kbytes},
        "table2": table,
        "table2_note": "GPU seconds = time of exactly t_eps iterations from the same start; paper's seconds are "
                       "its Table 2 on 16 CPU nodes (one core each), other random data of the same recipe",
    }
    emit(torch, line)


def run_nsweep(args, torch, did):
    from workloads import large_halfnormal_device

    cfg = WORKLOADS["nsweep"]
    M, K = cfg["M"], cfg["K"]
    stream = torch.cuda.Stream()
    rows = []
    X = None
    for N in cfg["sizes"]:
        del X
        torch.cuda.empty_cache()
        log(f"nsweep N={N}: generating")
        X = large_halfnormal_device(torch, M=M, N=N, K=K, seed=3, n_blocks=cfg["n_blocks"])
        torch.cuda.synchronize()
        opts = did.did_default_opts()
        opts.n_blocks = cfg["n_blocks"]
        opts.borrow_x = 1
        opts.x_tiled = 0 if args.x_given else 1
        opts.stream = stream.cuda_stream
        h = did.did_init_ex(X, M, N, K, 12345, opts)
        try:
            did.did_iterate(h, args.warmup)
            did.did_profile(h, True)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            log(f"nsweep N={N}: timing {args.steps} steps")
            ev0.record(stream)
            did.did_iterate(h, args.steps)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / args.steps
            stages, n_it = did.did_profile_read(h)
            did.did_profile(h, False)
        finally:
            did.did_free(h)
        n_it = max(n_it, 1)
        rows.append({"N": N, "ms_per_iter": round(ms, 4), "ms_per_1e5_columns": round(ms * 1e5 / N, 4),
                     "column_pass_ms": round(stages["column_pass"] / n_it, 4),
                     "row_pass_ms": round(stages["row_pass"] / n_it, 4),
                     "other_ms": round(sum(v for k, v in stages.items() if k not in ("column_pass", "row_pass")) / n_it, 4)})
    del X
    per = [r["ms_per_1e5_columns"] for r in rows]
    last = rows[-1]
    line = {
        "metric": METRIC,
        "value": round(1000.0 / last["ms_per_iter"], 4),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": last["ms_per_iter"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "M": M, "N": last["N"], "K": K, "n_blocks": cfg["n_blocks"]},
        "sweep": rows,
        "per_column_cost_spread": round(max(per) / min(per), 4),
    }
    emit(torch, line)


def _job_inputs(torch, jobs, x_dtype):
    from workloads import serving_x_device

    g = torch.Generator(device="cuda")
    out = []
    for j in jobs:
        g.manual_seed(j["seed"])
        out.append(serving_x_device(torch, j["M"], j["N"], j["K"], j["seed"], generator=g))
    return out


def batch_measure(torch, did, n_jobs, T, W, x_given, tune=True):
    """Plain form (instances one after another) against the batched form on the same jobs
    from the served workload's shape distribution; returns a dict of rates."""
    import numpy as np

    from workloads import serving_jobs

    jobs = serving_jobs(n_jobs, seed=5)
    log(f"batch: generating {len(jobs)} inputs")
    Xs = _job_inputs(torch, jobs, did.DID_F32)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()

    def make_all():
        hs = []
        for j, X in zip(jobs, Xs):
            o = did.did_default_opts()
            o.borrow_x = 1
            o.x_tiled = 0 if x_given else 1
            o.stream = stream.cuda_stream
            hs.append(did.did_init_ex(X, j["M"], j["N"], j["K"], 1000 + j["seed"], o))
        return hs

    flops_it = sum(8.0 * j["M"] * j["N"] * j["K"] for j in jobs)
    # plain form: each instance alone, one after another, on one stream
    hs = make_all()
    for h in hs:
        did.did_iterate(h, W)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    log(f"batch: plain form, {T} iterations per job")
    ev0.record(stream)
    for h in hs:
        did.did_iterate(h, T)
    ev1.record(stream)
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1)
    plain_C = []
    for h, j in zip(hs, jobs):
        C = np.empty((j["N"], j["K"]), np.float32)
        did.did_factors(h, None, C)
        plain_C.append(C)
        did.did_free(h)
    # batched form: the same jobs from the same start
    hs = make_all()
    b = did.did_batch_create(stream.cuda_stream)
    try:
        for h in hs:
            did.did_batch_add(b, h)
        did.did_batch_iterate(b, W)
        did.did_batch_sync(b)
        log(f"batch: batched form, {T} iterations")
        ev0.record(stream)
        did.did_batch_iterate(b, T)
        ev1.record(stream)
        torch.cuda.synchronize()
        batch_ms = ev0.elapsed_time(ev1)
        f_default = np.array(did.did_batch_objectives(b))
        same = True
        for h, j, Cp in zip(hs, jobs, plain_C):
            did.did_batch_remove(b, h)
            C = np.empty((j["N"], j["K"]), np.float32)
            did.did_factors(h, None, C)
            same = same and np.array_equal(C, Cp)
    finally:
        did.did_batch_free(b)
        for h in hs:
            did.did_free(h)
    tuned = tuned_batch(torch, did, jobs, Xs, stream, T, W, x_given, batch_ms, f_default) if tune else None
    del Xs
    torch.cuda.empty_cache()
    n_it = len(jobs) * T
    return {"jobs": len(jobs), "iterations_per_job": T, "ms_per_batched_iteration": round(batch_ms / T, 4),
            "instance_iter_s": round(n_it / (batch_ms / 1e3), 2),
            "plain_form_instance_iter_s": round(n_it / (plain_ms / 1e3), 2),
            "speedup_vs_plain_form": round(plain_ms / batch_ms, 3),
            "batched_tflops_fp32_equiv": round(flops_it * T / (batch_ms / 1e3) / 1e12, 2),
            "plain_tflops_fp32_equiv": round(flops_it * T / (plain_ms / 1e3) / 1e12, 2),
            "results_bitwise_equal_to_plain": bool(same),
            "objective_error_vs_plain_form": 0.0 if same else None,
            "tuned_tiles": tuned,
            "x_layout": "as given (column-major)" if x_given else "tile order (x_tiled=1)"}


def _log2_class(v):
    c = 0
    while v > 1:
        v = (v + 1) >> 1
        c += 1
    return c


def tuned_batch(torch, did, jobs, Xs, stream, T, W, x_given, default_ms, f_default):
    """The same batch after did_autotune picked the tiles (column-pass block waves, row-pass
    ranges) of each shape class among the jobs (tuned on the class's first job); against
    the default tiles.  The tuning table is cleared afterwards."""
    import time

    import numpy as np

    classes = {}
    for j in jobs:
        classes.setdefault((j["K"] <= 32, _log2_class(j["M"]), _log2_class(j["N"])), j)
    did.did_autotune_clear()
    picks = {}
    try:
        t0 = time.perf_counter()
        for key, j in classes.items():
            rb, cw, _ = did.did_autotune(j["M"], j["N"], j["K"], did.DID_F32, 0 if x_given else 1)
            picks[f"{rb}/{cw}"] = picks.get(f"{rb}/{cw}", 0) + 1
        tune_s = time.perf_counter() - t0
        log(f"batch: tuned {len(classes)} shape classes in {tune_s:.1f} s")
        hs = []
        for j, X in zip(jobs, Xs):
            o = did.did_default_opts()
            o.borrow_x = 1
            o.x_tiled = 0 if x_given else 1
            o.stream = stream.cuda_stream
            hs.append(did.did_init_ex(X, j["M"], j["N"], j["K"], 1000 + j["seed"], o))
        b = did.did_batch_create(stream.cuda_stream)
        try:
            for h in hs:
                did.did_batch_add(b, h)
            did.did_batch_iterate(b, W)
            did.did_batch_sync(b)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            did.did_batch_iterate(b, T)
            ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            f = np.array(did.did_batch_objectives(b))
        finally:
            did.did_batch_free(b)
            for h in hs:
                did.did_free(h)
    finally:
        did.did_autotune_clear()
    return {"shape_classes": len(classes), "tuning_s": round(tune_s, 2),
            "choices_row_blocks_col_waves": picks,
            "ms_per_batched_iteration": round(ms / T, 4),
            "speedup_vs_default_tiles": round(default_ms / ms, 3),
            # the tiles change only summation order: the objectives after the same iterations
            "objective_max_rel_diff_vs_default_tiles": float(np.max(np.abs(f - f_default) / f_default))}


def run_batch(args, torch, did):
    cfg = WORKLOADS["batch"]
    r = batch_measure(torch, did, cfg["jobs"], args.steps, args.warmup, args.x_given, tune=not args.no_tune)
    line = {
        "metric": METRIC,
        "value": r["instance_iter_s"],
        "unit": "instance-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_batched_iteration"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "jobs": r["jobs"], "x_layout": r["x_layout"]},
    }
    line.update({k: v for k, v in r.items() if k not in ("jobs", "x_layout")})
    emit(torch, line)


PREGEN_CAP = 120 << 30  # X of all jobs generated before the clock starts when it fits


def serve_measure(torch, did, n_jobs, slots, bf16, tiled, max_iter=50, rel_tol=1e-4, reserve_gib=-1):
    """Poisson arrivals (200 jobs/s) into the server; latency from the scheduled arrival to
    retirement.  Returns a dict of throughput, latency and queue figures.  When the jobs'
    X fit in PREGEN_CAP they are all generated on the device before the clock starts (the
    inputs are resident in HBM, and the timed region holds only the server's work);
    otherwise each is generated at its arrival, inside the timed region."""
    import numpy as np

    from workloads import serving_jobs, serving_x_device

    jobs = serving_jobs(n_jobs, seed=5, rate=200.0)
    pregen = sum(4 * j["M"] * j["N"] for j in jobs) <= PREGEN_CAP
    so = did.did_server_default_opts()
    so.hbm_budget = 200 << 30
    so.max_active = slots
    so.max_iter = max_iter
    so.rel_tol = rel_tol
    so.x_tiled = 1 if tiled else 0  # float32 jobs keep X in tile order
    # with the inputs resident before the clock, the server reserves 64 GiB at creation for
    # its jobs' buffers (about 45 GB in use at the peak of the 300-job run), so that no
    # admission inside the timed region allocates device memory
    so.arena_reserve_gib = (64 if pregen else 0) if reserve_gib < 0 else reserve_gib
    stream = torch.cuda.Stream()
    so.stream = stream.cuda_stream
    srv = did.did_server_create(so)
    gen = torch.Generator(device="cuda")
    side = torch.cuda.Stream()
    # client-side cap on generated, not yet admitted data: the device holds it beside the
    # server's budget and the released jobs' memory the server keeps for reuse (up to 48 GB)
    total = torch.cuda.get_device_properties(torch.cuda.current_device()).total_memory
    queued_x_cap = int(min(100 << 30, max(4 << 30, total - so.hbm_budget - (56 << 30))))
    if pregen:  # the inputs are resident already: nothing to hold back
        queued_x_cap = 1 << 62
    pending = list(range(n_jobs))
    live = {}  # job id -> (index, X tensor, submit time)
    lat, iters, qwait = [], [], []
    max_queue, steps, occ = 0, 0, []
    queued_bytes = 0
    pre = {}
    if pregen:
        with torch.cuda.stream(side):
            for i, j in enumerate(jobs):
                gen.manual_seed(j["seed"])
                pre[i] = serving_x_device(torch, j["M"], j["N"], j["K"], j["seed"], generator=gen)
        side.synchronize()
    log(f"serve: {n_jobs} jobs, {so.max_active} slots, inputs "
        f"{'generated before the clock' if pregen else 'generated at arrival'}")
    t0 = time.perf_counter()
    done = 0
    try:
        while done < n_jobs:
            now = time.perf_counter() - t0
            while pending and jobs[pending[0]]["t"] <= now and queued_bytes < queued_x_cap:
                i = pending.pop(0)
                j = jobs[i]
                if pregen:
                    X = pre.pop(i)
                else:
                    gen.manual_seed(j["seed"])
                    with torch.cuda.stream(side):
                        X = serving_x_device(torch, j["M"], j["N"], j["K"], j["seed"], generator=gen)
                    side.synchronize()
                jid = did.did_server_submit(srv, X, j["M"], j["N"], j["K"], 1000 + j["seed"],
                                            did.DID_BF16 if bf16 else did.DID_F32)
                live[jid] = (i, X, time.perf_counter() - t0)
                queued_bytes += 4 * j["M"] * j["N"]
            running, queued, fin = did.did_server_step(srv)
            steps += 1
            occ.append(running)
            max_queue = max(max_queue, queued)
            if fin or running == 0:
                for jid in list(live):
                    st, it, f, l, q = did.did_server_poll(srv, jid)
                    if st == did.DID_JOB_QUEUED:
                        continue
                    i, X, ts = live[jid]
                    if st in (did.DID_JOB_DONE, did.DID_JOB_FAILED):
                        if st == did.DID_JOB_FAILED:
                            try:  # the reason the job failed
                                did.did_server_result(srv, jid)
                                why = ""
                            except did.DidError as e:
                                why = str(e)
                            raise RuntimeError(f"job {i} failed: {why}")
                        lat.append(ts - jobs[i]["t"] + l)
                        iters.append(it)
                        qwait.append(q)
                        did.did_server_release(srv, jid)
                        del live[jid]
                        done += 1
            # charge generated data until the job is admitted
            queued_bytes = sum(4 * jobs[i]["M"] * jobs[i]["N"] for jid, (i, _, _) in live.items()
                               if did.did_server_poll(srv, jid)[0] == did.DID_JOB_QUEUED)
            if running == 0 and queued == 0 and pending:
                time.sleep(max(0.0, min(0.002, jobs[pending[0]]["t"] - (time.perf_counter() - t0))))
        wall = time.perf_counter() - t0
        used, peak = did.did_server_memory(srv)
        arena_allocs, arena_reuses, arena_frees, _ = did.did_server_arena_stats(srv)
    finally:
        did.did_server_free(srv)
    torch.cuda.empty_cache()
    lat = np.array(lat)
    iters = np.array(iters)
    flops = sum(8.0 * jobs[i]["M"] * jobs[i]["N"] * jobs[i]["K"] for i in range(n_jobs))
    return {"jobs": n_jobs, "slots": slots, "x_storage": "bf16" if bf16 else "f32",
            "x_layout": "tile order" if (bf16 or tiled) else "as given (column-major)",
            "inputs": "generated on the device before the clock" if pregen else "generated at arrival (timed)",
            "arenas": {"reserve_gib": so.arena_reserve_gib, "allocated": arena_allocs,
                       "reused_or_carved": arena_reuses, "freed": arena_frees},
            "solves_per_s": round(n_jobs / wall, 2), "wall_s": round(wall, 3), "steps": steps,
            "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
            "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
            "latency_mean_s": round(float(lat.mean()), 4),
            "queue_wait_p50_s": round(float(np.percentile(qwait, 50)), 4),
            "iterations_mean": round(float(np.mean(iters)), 2),
            "share_stopped_by_rel_tol": round(float(np.mean(iters < max_iter)), 4),
            "rel_tol": rel_tol, "max_iter": max_iter,
            "arrival_span_s": round(jobs[-1]["t"], 3),
            "max_queue_depth": max_queue,
            "mean_running": round(float(np.mean(occ)), 2),
            "peak_budget_bytes": peak,
            "offered_tflops_fp32_equiv_at_mean_iters": round(flops / len(jobs) * float(np.mean(iters)) * 200.0 / 1e12,
                                                             1)}


def run_serve(args, torch, did):
    cfg = WORKLOADS["serve"]
    n_jobs = args.serve_jobs or cfg["jobs"]
    r = serve_measure(torch, did, n_jobs, args.serve_slots, args.serve_bf16, not args.x_given,
                      reserve_gib=args.serve_reserve)
    line = {
        "metric": METRIC,
        "value": r["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": 0,
        "ms_per_step": round(r["wall_s"] * 1e3 / max(r["steps"], 1), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {"workload": cfg["desc"] + ("; X stored as bf16" if args.serve_bf16 else ""), "jobs": n_jobs,
                   "slots": r["slots"], "x_storage": r["x_storage"], "x_layout": r["x_layout"]},
    }
    line.update({k: v for k, v in r.items() if k not in ("jobs", "slots", "x_storage", "x_layout", "steps")})
    emit(torch, line)


def precision_form(torch, did, X, M, N, K, n_blocks, plain_ms, steps):
    """The precision form on the large workload: X stored as bf16, the residual refreshed
    every iteration (refresh_every 1) or carried with a refresh every 10 iterations
    (refresh_every 10); iterations/s and speedup over the plain float32 form.  Per run, the
    objective error against the FP64 oracle is taken on the workload's first column block
    (5000 x 15625) over 50 iterations from the oracle's initial factors: against the
    oracle on the original X and on bf16(X), from the trajectories that
    tests/golden/make_trajectories.py stored (oracle/ only)."""
    import json

    import numpy as np

    from workloads import large_halfnormal, to_f32_colmajor, uniform_init

    out = {"x_storage": "bf16 (round to nearest even), two tiled copies", "residual": "float32",
           "objective": "float64"}
    stream = torch.cuda.Stream()
    for r in (1, 10):
        o = did.did_default_opts()
        o.n_blocks = n_blocks
        o.x_dtype = did.DID_BF16
        o.refresh_every = r
        o.stream = stream.cuda_stream
        log(f"precision form: bf16 X, refresh_every={r}")
        h = did.did_init_ex(X, M, N, K, 12345, o)
        try:
            ms, stages, n_it = timed_iterations(torch, did, h, stream, 10 if r > 1 else 2, steps, profile_iters=0)
        finally:
            did.did_free(h)
        torch.cuda.empty_cache()
        out[f"refresh_every_{r}"] = {"iter_s": round(1000.0 / ms, 3), "ms_per_iter": round(ms, 4),
                                     "speedup_vs_plain_f32": round(plain_ms / ms, 3)}
    # objective error against the oracle on a slice, from the stored oracle trajectories
    gdir = os.path.join(ROOT, "tests", "golden")
    try:
        g_bf = json.load(open(os.path.join(gdir, "traj_large_slice_b1_bf16.json")))
        g_32 = json.load(open(os.path.join(gdir, "traj_large_slice_b1.json")))
    except OSError:
        out["objective_error_vs_fp64_oracle"] = None
        return out
    Xs = to_f32_colmajor(large_halfnormal(M, N, K, seed=3, n_blocks=64, take_blocks=1)[0])
    Ms, Ns = Xs.shape
    B0, C0 = uniform_init(Ms, Ns, K, 12345)
    Xd = torch.from_numpy(np.ascontiguousarray(Xs.T)).to("cuda")
    Bd = torch.from_numpy(np.ascontiguousarray(B0.astype(np.float32).T)).to("cuda")
    Cd = torch.from_numpy(np.ascontiguousarray(C0.astype(np.float32).T)).to("cuda")
    torch.cuda.synchronize()
    T = g_bf["T"]
    fo_bf, fo_32 = np.array(g_bf["f"]), np.array(g_32["f"])
    errs = {}
    for name, dtype, r in (("plain_f32", did.DID_F32, 1), ("bf16_refresh_every_1", did.DID_BF16, 1),
                           ("bf16_refresh_every_10", did.DID_BF16, 10)):
        o = did.did_default_opts()
        o.x_dtype = dtype
        o.refresh_every = r
        h = did.did_init_from_factors(Xd, Ms, Ns, K, Bd, Cd, o)
        try:
            did.did_iterate(h, T)
            fg = np.append(did.did_history(h), did.did_objective(h))
        finally:
            did.did_free(h)
        errs[name] = {"vs_oracle_on_x_max_over_t": float(np.max(np.abs(fg - fo_32) / fo_32)),
                      "vs_oracle_on_x_at_T": float(abs(fg[-1] - fo_32[-1]) / fo_32[-1]),
                      "vs_oracle_on_bf16x_max_over_t": float(np.max(np.abs(fg - fo_bf) / fo_bf)),
                      "vs_oracle_on_bf16x_at_T": float(abs(fg[-1] - fo_bf[-1]) / fo_bf[-1])}
    out["objective_error_vs_fp64_oracle"] = {
        "slice": f"first column block {Ms}x{Ns}, K={K}, {T} iterations from uniform_init(12345) factors",
        **errs}
    del Xd, Bd, Cd
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="large workload: skip the precision, batched and served forms (profiling runs)")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch workload and batched form: skip the tuned-tiles leg (profiling runs)")
    ap.add_argument("--paper-max-n", type=float, default=1e8, help="paper workload: largest N")
    ap.add_argument("--no-table", action="store_true", help="paper workload: skip the runs to the stopping rule")
    ap.add_argument("--serve-jobs", type=int, default=0, help="serve workload: number of jobs (default 1000)")
    ap.add_argument("--serve-slots", type=int, default=64, help="serve workload: batch slots")
    ap.add_argument("--serve-bf16", action="store_true", help="serve workload: store each job's X as bf16")
    ap.add_argument("--serve-reserve", type=int, default=-1,
                    help="GiB the server reserves at creation for its jobs' buffers (default: 64 when the "
                         "inputs are generated before the clock, else 0)")
    ap.add_argument("--x-given", action="store_true",
                    help="float32 X read as given (column-major) instead of kept in tile order")
    ap.add_argument("--serve-tiled", action="store_true",
                    help="serve workload: float32 jobs keep X in tile order (the default; the flag is "
                         "accepted so that recorded commands still run)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the DID engine here is single-GPU "
              "(multi-GPU sharding is a design note only); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1802_08938_amd as did

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "paper":
        run_paper_shape(args, torch, did)
        return
    if args.workload == "nsweep":
        run_nsweep(args, torch, did)
        return
    if args.workload == "batch":
        run_batch(args, torch, did)
        return
    if args.workload == "serve":
        run_serve(args, torch, did)
        return
    cfg = WORKLOADS[args.workload]
    M, N, K = cfg["M"], cfg["N"], cfg["K"]
    log(f"generating {args.workload} input {M}x{N} on the device")
    X = make_input(torch, args.workload, cfg)
    torch.cuda.synchronize()
    # a dedicated (default-priority) stream: the engine's kernels and the timing events
    # must share it; torch's current stream is the null stream, whose handle is 0
    stream = torch.cuda.Stream()
    opts = did.did_default_opts()
    opts.n_blocks = cfg["n_blocks"]
    opts.borrow_x = 0 if cfg.get("x_bf16") else 1
    opts.x_dtype = did.DID_BF16 if cfg.get("x_bf16") else did.DID_F32
    # the engine keeps X in 32x32 tile order, one copy per pass (made once at init; the
    # bf16 form always does)
    opts.x_tiled = 0 if args.x_given else 1
    opts.stream = stream.cuda_stream
    t0 = time.perf_counter()
    h = did.did_init_ex(X, M, N, K, 12345, opts)
    init_s = time.perf_counter() - t0
    log(f"init {init_s:.2f} s; warmup {args.warmup}; timing {args.steps} steps")
    assert opts.stream, "engine stream must be explicit"
    try:
        ms, stages, n_it = timed_iterations(torch, did, h, stream, args.warmup, args.steps, profile_iters=3)
        f_last = did.did_objective(h)
        hist = did.did_history(h)
        n_total = did.did_iterations(h)
    finally:
        did.did_free(h)
    f32_ref = None
    if cfg.get("x_bf16"):
        # the plain float32 form from the same initial factors and iteration count, for the
        # objective gap of the bf16 storage form
        o2 = did.did_default_opts()
        o2.n_blocks = cfg["n_blocks"]
        o2.borrow_x = 1
        o2.stream = stream.cuda_stream
        h2 = did.did_init_ex(X, M, N, K, 12345, o2)
        try:
            did.did_iterate(h2, n_total)
            f32_ref = did.did_objective(h2)
        finally:
            did.did_free(h2)
    it_s = 1000.0 / ms
    cnt = algorithmic_counts(M, N, K, 2 if cfg.get("x_bf16") else 4)
    dom = max(("column_pass", "row_pass"), key=lambda k: stages[k])
    dom_ms = stages[dom] / n_it
    secs = dom_ms * 1e-3
    traffic = measured_traffic(dom, args.workload)
    KP = 32 if K <= 32 else 64
    issued = SPLIT_PRODUCTS * 4.0 * M * N * KP  # fp16 MFMA flops the pass issues (K padded to KP)
    tflops = cnt["pass_flops"] / secs / 1e12  # float32-accurate flops
    gbs = cnt["pass_bytes"] / secs / 1e9      # algorithmic HBM bytes
    # the roofline that bounds the pass: the larger of its two time floors
    hbm_bound = cnt["pass_bytes"] / (PEAK_HBM_GBS * 1e9) >= cnt["pass_flops"] / (PEAK_SPLIT_TFLOPS * 1e12)
    if hbm_bound:
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic}
    else:
        roof = {"bound": "mfma", "kernel": dom, "achieved": round(tflops, 3), "peak": round(PEAK_SPLIT_TFLOPS, 2),
                "unit": "TFLOP/s", "frac": round(tflops / PEAK_SPLIT_TFLOPS, 4), "traffic": traffic}
    # the whole iteration against the same roof: its algorithmic bytes (X once, C read and
    # written, B read) over the measured time per iteration
    iter_gbs = cnt["iter_bytes"] / (ms * 1e-3) / 1e9
    roof.update({
        "iter_frac": round(iter_gbs / PEAK_HBM_GBS, 4), "iter_bytes": cnt["iter_bytes"],
        "iter_note": "iteration algorithmic bytes / ms_per_step / 8 TB/s; the two passes read X twice per "
                     "iteration (the sweep needs whole columns, the W messages whole rows)",
        "limiter": sq_limiter(dom),
        "bound_note": "bound = the roof whose time floor is larger for the pass's algorithmic work; limiter = "
                      "what the committed SQ counters show stalls the pass (null when they were taken on other "
                      "kernel sources)",
        "kernel_ms": round(dom_ms, 4), "bytes_per_launch": cnt["pass_bytes"], "flops_per_launch": cnt["pass_flops"],
        "f32_accurate_tflops": round(tflops, 3), "f32_accurate_peak_tflops": round(PEAK_SPLIT_TFLOPS, 2),
        "f32_accurate_frac": round(tflops / PEAK_SPLIT_TFLOPS, 4),
        "peak_note": "float32-accurate flops (4MNK per pass) against the fp16 MFMA peak / 3 (three fp16 "
                     "products per float32 product); algorithmic bytes (X once, C read and written) "
                     "against 8 TB/s",
        "mfma_f16_issued_tflops": round(issued / secs / 1e12, 1),
        "mfma_f16_issued_frac": round(issued / secs / 1e12 / PEAK_F16_MFMA_TFLOPS, 4),
        "hbm_algorithmic_gbs": round(gbs, 1), "hbm_algorithmic_frac": round(gbs / PEAK_HBM_GBS, 4)})
    if traffic is not None:
        roof["hbm_measured_gbs"] = round(traffic / secs / 1e9, 1)
    line = {
        "metric": METRIC,
        "value": round(it_s, 4),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE,
        "data": "synthetic",
        "config": {"workload": cfg["desc"], "M": M, "N": N, "K": K, "n_blocks": cfg["n_blocks"],
                   "x_layout": "as given (column-major)" if args.x_given and not cfg.get("x_bf16") else
                               "two copies in 32x32 tile order (one per pass), made once at init (x_tiled=1)"},
        "hbm_gbs_algorithmic": round(iter_gbs, 2),
        "stage_ms_per_iter": {k: round(v / n_it, 4) for k, v in stages.items()},
        "objective_last": f_last,
        "objective_ratio": (f_last / hist[0]) if hist else None,
        "init_s": round(init_s, 3),
        "roofline": roof,
    }
    if args.workload in ("planted", "image"):
        floor_ms = launch_floor(torch, KERNELS_PER_ITERATION)
        line["launch_floor"] = {
            "kernels_per_iteration": KERNELS_PER_ITERATION, "graph_replay_ms": round(floor_ms, 4),
            "iter_s_at_floor": round(1000.0 / floor_ms, 1), "ms_per_step_over_floor": round(ms / floor_ms, 2),
            "note": "a captured graph of as many dependent one-element kernels as one iteration launches, "
                    "replayed: the iteration's cost if its kernels did no work"}
    if f32_ref is not None:
        line["config"]["x_storage"] = "bf16"
        line["objective_f32_form_same_iterations"] = f32_ref
        line["objective_rel_diff_vs_f32_form"] = (f_last - f32_ref) / f32_ref
    if args.workload == "large" and not args.no_forms:
        # the other forms of the metric on the same GPU: precision (bf16 X, refresh every
        # iteration or every 10), batched, served
        line["precision_form"] = precision_form(torch, did, X, M, N, K, cfg["n_blocks"], ms, 20)
        del X
        torch.cuda.empty_cache()
        line["batched_form"] = batch_measure(torch, did, WORKLOADS["batch"]["jobs"], 10, 2, args.x_given)
        # float32 jobs keep X in tile order like the other forms (each job's two tiled copies
        # are made at its admission, inside the timed region), unless --x-given
        tiled = not args.x_given
        line["served_form"] = serve_measure(torch, did, args.serve_jobs or 300, args.serve_slots, False, tiled,
                                            reserve_gib=args.serve_reserve)
        line["served_form"]["note"] = ("a shortened run of the served workload: the first jobs of the same "
                                       "Poisson schedule (200 jobs/s), 200 GB budget, all inputs resident in "
                                       "HBM before the clock starts; " +
                                       ("X kept in tile order, copied at admission" if tiled else "X read as given") +
                                       ("; the jobs' buffers carved from a reserve made when the server starts"
                                        if line["served_form"]["arenas"]["reserve_gib"] > 0 else ""))
        # the same jobs with a stopping rule loose enough to fire: retirements free slots
        # mid-mix and the queue is admitted as they do
        es = serve_measure(torch, did, args.serve_jobs or 300, args.serve_slots, False, tiled, rel_tol=1e-2,
                           reserve_gib=args.serve_reserve)
        line["served_form"]["early_stop"] = {k: es[k] for k in (
            "rel_tol", "solves_per_s", "latency_p50_s", "latency_p99_s", "iterations_mean",
            "share_stopped_by_rel_tol", "max_queue_depth")}
    else:
        del X
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(args.workload, cfg)
    emit(torch, line)


if __name__ == "__main__":
    main()
