"""Benchmark of the sparse TT decomposition hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision fp64|fp32|bf16]
                    [--dynamic-delta] [--key-bits B] [--matrix-input] [--roofline FAMILY]
                    [--method cps|fasttt] [--p P]

One step is one pass of the whole hot path over the workload's nonzeros, all in
libttsparse kernels (the plan is built on a second stream beside the decomposition,
as it needs only the coordinates; --no-overlap builds it afterwards):
  tt_sparse_decompose   ingest, sort, parallel-vector rounding of every level,
                        left-to-right QR sweep, right-to-left truncated-SVD sweep
  tt_eval_plan_create   sort of the nonzero coordinates and their prefix trie
  tt_eval_plan_forward  the TT at every nonzero coordinate (left products kept)
  tt_eval_plan_backward gradient of sum_n val[n] * TT(i_n) w.r.t. every core
The FP64 run also times the FP32 form of the same step ("mixed"), the sparse stage
against HBM ("roofline.sparse_hbm"; inside the step, and with the decomposition run
by itself after the timed steps, "t_ms_alone" / "stage_ms_alone") and the bond-2 Gram slice on the 5-way 200^5
tensor with 10^7 nonzeros in FP64/FP32/BF16 ("c4_slice": its Gram kernel against the
FP64 matrix-core peak, errors against oracle values stored in tests/golden).
With --matrix-input (the Laplacian workload) the step starts from the sparse matrix
and first runs tt_matrix_to_tensor, the front-end of the MPO form.  With
--dynamic-delta the truncation thresholds follow Algorithm 8; with --key-bits B the
parallel test groups canonical values rounded to B fraction bits.  With --method
fasttt the decomposition is the paper's fiber-trie variant (tt_fasttt_decompose,
p from --p or Algorithm 9).
Inputs are resident in HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "nonzeros decomposed/sec at fixed eps (FP64 vs mixed) + HBM/MFMA roofline %"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0  # dense
# Kernel families with live timers, and what bounds each.  The roofline object is
# reported for the family that takes the most time per step (chosen live below).
FAMILY_BOUND = {
    "jacobi": "alu", "eval_forward": "alu", "eval_up": "alu", "eval_grad": "alu", "cholesky": "alu",
    "trsm": "alu", "gemm": "mfma", "gemm_lp": "mfma",
    "sort_scatter": "hbm", "level_group": "hbm", "level_canon": "hbm", "mpo_coords": "hbm",
}
# Families whose every launch is one workgroup (one CU of 256): their roofline line
# also states the fraction of one CU's share of the peak.
SINGLE_WORKGROUP = {"jacobi", "cholesky"}
NUM_CU = 256
# The paper's own end-to-end FastTT rates for workloads run here, derived as nonzeros
# / reported time (Table 2: FDM matrices, eps = 1e-14, on a 32-core x86 server).
# Another machine's numbers: context.
PUBLISHED = {
    (f"fdm3d_n{n}_{c}", "fasttt"): (nnz / t, f"Table 2, FastTT, FDM n={n} {c}, {t} s, 32-core CPU")
    for n, c, nnz, t in ((20, "pattern", 53600, 0.788), (30, "pattern", 183600, 2.88), (20, "random", 53600, 1.67),
                         (30, "random", 183600, 12.4), (40, "random", 438400, 57.5))
}
# Per-launch HBM traffic of profiled kernels, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes scaled by a plain copy of known size (profiles/traffic_*.txt).  A figure is
# used only for the workload it was taken on, and only while the source file that
# holds the kernel is unchanged.
PROFILES = os.path.join(ROOT, "profiles")


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="kron8d_n32_t64")
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    p.add_argument("--matrix-input", action="store_true",
                   help="start from the workload's sparse matrix (laplace2d_qtt_L10): the step then also runs the "
                        "matrix -> tensor front-end of the MPO form")
    p.add_argument("--method", default="cps", choices=["cps", "fasttt"],
                   help="cps: column-parallel sweep (tt_sparse_decompose); fasttt: the fiber-trie variant")
    p.add_argument("--p", type=int, default=0, help="fasttt: the middle core p (0: Algorithm 9)")
    p.add_argument("--key-bits", type=int, default=0,
                   help="tolerant parallel test: canonical values rounded to this many fraction bits (0: exact)")
    p.add_argument("--dynamic-delta", action="store_true",
                   help="per-bond truncation thresholds from the remaining error budget (Algorithm 8)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-mixed", action="store_true", help="skip the FP32 leg of the FP64 run")
    p.add_argument("--no-slice", action="store_true",
                   help="skip the bond-2 Gram slice leg (5-way 200^5 tensor, 10^7 nonzeros)")
    p.add_argument("--slice-only", type=int, default=0, metavar="REPS",
                   help="only run the bond-2 Gram slice leg with REPS timed calls per precision (profiling)")
    p.add_argument("--slice-precisions", default="fp64,fp32,bf16", help="precisions of the slice leg")
    p.add_argument("--no-hbm", action="store_true",
                   help="skip roofline.sparse_hbm (its device-copy calibration and the decomposition "
                        "run alone): for profiling runs whose kernel tables must hold only the steps")
    p.add_argument("--no-overlap", action="store_true",
                   help="build the evaluation plan after the decomposition instead of beside it")
    p.add_argument("--cpu-sample", type=int, default=20000, help="entries of the oracle's eval/backward sample")
    p.add_argument("--roofline", default="auto",
                   help="kernel family for the roofline object ('auto': the one with the most time per step)")
    p.add_argument("--stage", default=None, choices=["sparse", "decompose", "eval"],
                   help="time one stage alone (for its profiler counters): 'sparse' runs only the sparse "
                        "stage, 'decompose' the decomposition, 'eval' the plan, forward and backward on the "
                        "decomposed tensor")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="only run a plain device-to-device copy of MIB MiB five times (profiler calibration)")
    return p.parse_args()


def cpu_baseline(idx, val, dims, eps, sample, gpu_cores=None, precision="fp64", max_rank=0, dynamic=False,
                 key_bits=0, method="cps", p=0):
    """The oracle (single-threaded FP64 C++), timed on this host on a bounded sample.

    Also returns ||B_gpu - B_oracle||_F / ||A||_F for the GPU result `gpu_cores`
    (computed after the timing, with the oracle's stable TT-difference norm).
    """
    import oracle

    oracle.build(force=False)
    t_runs = []
    for _ in range(3):  # median of three runs of the whole decomposition
        t0 = time.perf_counter()
        if method == "fasttt":
            from oracle import ftt

            res = ftt.decompose(idx, val, dims, eps, p=p, max_rank=max_rank)
            res.cores = [np.ascontiguousarray(c) for c in res.cores]
        else:
            res = oracle.decompose(idx, val, dims, eps, max_rank=max_rank, dynamic_delta=dynamic,
                                   key_bits=key_bits)
        t_runs.append(time.perf_counter() - t0)
    t_dec = float(np.median(t_runs))
    rng = np.random.Generator(np.random.PCG64(11))
    pick = rng.choice(len(val), min(sample, len(val)), replace=False)
    t0 = time.perf_counter()
    y = oracle.eval_entries(res.cores, idx[pick])
    oracle.eval_grad(res.cores, idx[pick], val[pick])
    t_eval = time.perf_counter() - t0
    del y
    t_step = t_dec + t_eval * (len(val) / len(pick))
    base = {
        "value": len(val) / t_step,
        "unit": "nnz/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"full FP64 decomposition of the workload (median of 3: {t_dec:.2f} s; runs "
                   f"{', '.join(f'{t:.2f}' for t in t_runs)} s) + eval/backward on {len(pick)} of "
                   f"{len(val)} nonzeros ({t_eval:.2f} s, scaled linearly to all nonzeros)"),
        "host": host_info(),
    }
    err = None
    if gpu_cores is not None:
        err = error_vs_oracle(res, gpu_cores, precision)
    return base, err, res


def error_vs_oracle(res, gpu_cores, precision):
    import oracle

    c64 = [np.ascontiguousarray(c, dtype=np.float64) for c in gpu_cores]
    return {"precision": precision, "rel_fro": oracle.tt_diff_norm(c64, res.cores) / res.norm,
            "ranks_gpu": [int(c.shape[0]) for c in c64] + [1], "ranks_oracle": list(res.ranks)}


def host_info():
    """CPU model and core counts of this host (the oracle uses one core)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable, "oracle_threads": 1}


def sparse_alg_bytes(nnz, d, level_sizes):
    """Algorithmic bytes of the sparse stage (ingest, sort, every level): read the COO
    once, each level once, write each next level and each N_k once:
    nnz (4d + 8) + 16 nnz + sum_{k>=2} 20 nnz_k + sum_k (20 nnz_{k+1} + 12 nnz(N_k)),
    nnz_k the entries of level k (nnz_{k+1} = the columns of level k)."""
    b = nnz * (4 * d + 8) + 16 * nnz
    prev = None
    for ncols, _beta, nnz_n in level_sizes:
        if prev is not None:
            b += 20 * prev
        b += 20 * ncols + 12 * nnz_n
        prev = ncols
    return float(b)


def copy_gbps(mib=1024, reps=5):
    """Bytes moved per second by a plain device-to-device copy (read + write)."""
    import torch

    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 8 / (ms / 1000.0) / 1e9


def _traffic(family, workload, method):
    """(bytes per launch, source) from profiles/traffic_<family>.txt if it was taken on this
    workload and method and its kernel source is unchanged since, else None."""
    import hashlib

    path = os.path.join(PROFILES, f"traffic_{family}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    src = fields.get("source")
    key = "traffic_bytes_per_launch" if "traffic_bytes_per_launch" in fields else "traffic_bytes_per_step"
    if not src or key not in fields:
        return None
    if fields.get("workload") != workload or fields.get("method", "cps") != method:
        return None  # measured on another workload: other launch shapes
    with open(os.path.join(ROOT, src), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != fields.get("source_sha256"):
            return None  # the kernel changed since the counters were taken
    return float(fields[key]), os.path.relpath(path, ROOT)


def calibrate_copy(mib):
    import torch

    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                      "copies": 6, "ms_per_copy": ms, "copy_GBps": 2 * n * 8 / (ms / 1000.0) / 1e9}), flush=True)


def stage_only(args):
    """One stage of the step alone, --warmup untimed and --steps timed repetitions, so that
    profiler counters of its kernels are not mixed with the rest of the step.  Prints its
    time per step and its algorithmic bytes per step (sparse: the formula of
    sparse_alg_bytes; eval: the sum over the evaluation kernels' live timers)."""
    import torch

    import paper_1908_02721_amd as tts
    from paper_1908_02721_amd import _lib, synth

    idx, val, dims, eps = synth.workload(args.workload)
    gi = torch.from_numpy(np.ascontiguousarray(idx)).cuda()
    gv = torch.from_numpy(np.ascontiguousarray(val)).cuda()
    out = {"stage": args.stage, "workload": args.workload, "steps": args.steps, "warmup": args.warmup}
    if args.stage in ("sparse", "decompose"):
        sparse_only = args.stage == "sparse"

        def run():
            return tts.decompose(gi, gv, dims, eps, sparse_only=sparse_only, precision=args.precision)
    else:
        tt = tts.decompose(gi, gv, dims, eps, precision=args.precision)
        cores = tt.cores
        gy = gv if cores[0].dtype == torch.float64 else gv.float()

        def run():
            plan = tts.EvalPlan(gi, dims)
            plan.forward(cores, save=True)
            plan.backward(cores, gy, use_saved=True)
            return plan
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = run()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / args.steps
    out["ms_per_step"] = ms
    if args.stage in ("sparse", "decompose"):
        out["algo_bytes_per_step"] = sparse_alg_bytes(len(val), len(dims), r.level_sizes())
        out["stage_ms"] = r.times_ms
        if args.stage == "decompose":
            out["ranks"] = r.ranks
            out["note"] = "algo_bytes_per_step: the sparse stage's only"
    else:
        fam = {}
        for f in ("eval_forward", "eval_up", "eval_grad"):
            _lib.kernel_timer_start(f)
            run()
            torch.cuda.synchronize()
            k_ms, k_n, k_bytes, k_flops = _lib.kernel_timer_read()
            _lib.kernel_timer_start(None)
            fam[f] = {"launches": k_n, "kernel_ms": k_ms, "algo_bytes": k_bytes, "algo_flops": k_flops}
        out["families"] = fam
        out["algo_bytes_per_step"] = sum(v["algo_bytes"] for v in fam.values())
    out["algo_GBps"] = out["algo_bytes_per_step"] / (ms / 1000.0) / 1e9
    print(json.dumps(out), flush=True)


def c4_slice_leg(reps=3, precisions=("fp64", "fp32", "bf16")):
    """The bond-2 Gram slice (tt_sparse_gram_slice) on the 5-way 200^5 tensor with 10^7
    N(0,1) nonzeros, in the three precisions: whole-call nonzeros/s, stage times, the
    Gram kernel's FP64 MFMA rate from the live timer, and the error against the
    oracle's values stored at seeded positions (tests/golden)."""
    import torch

    import paper_1908_02721_amd as tts
    from paper_1908_02721_amd import _lib, synth

    golden = os.path.join(ROOT, "tests", "golden", "slice_random5d_n200_nnz10m.json")
    with open(golden) as f:
        gold = json.load(f)
    idx, val, dims, _ = synth.workload(gold["workload"])
    gi = torch.from_numpy(idx).cuda()
    gv = torch.from_numpy(val).cuda()
    out = {"workload": gold["workload"], "dims": list(dims), "nnz": len(val), "reps": reps}
    for prec in precisions:
        gs = tts.gram_slice(gi, gv, dims, precision=prec)  # warm-up
        del gs
        torch.cuda.synchronize()
        _lib.kernel_timer_start("slice_gram")
        tot, stages = [], []
        for r in range(reps):
            gs = tts.gram_slice(gi, gv, dims, precision=prec)
            tot.append(gs.times_ms["total"])
            stages.append(gs.slice_ms)
            if r < reps - 1:
                del gs
        k_ms, k_n, k_bytes, k_flops = _lib.kernel_timer_read()
        _lib.kernel_timer_start(None)
        tf = k_flops / (k_ms / 1000.0) / 1e12
        m, n2 = gold["m"], dims[1]
        # error against the oracle's samples (the same scales as tests/test_gpu_slice.py)
        x = gold["x2"]
        sp = gs.slot_ptr().cpu().numpy()
        bc = gs.blk_col().cpu().numpy()
        b = np.array([sp[i] + np.searchsorted(bc[sp[i]:sp[i + 1]], j) for i, j in zip(x["i"], x["j"])])
        xv = gs.x2_view()[torch.from_numpy(b).cuda(), torch.from_numpy(np.asarray(x["a"])).cuda()]
        ex = np.abs(xv.double().cpu().numpy() - np.asarray(x["v"])) / np.asarray(x["scale"])
        g = gold["gram"]
        off = gs.gram_offset(np.asarray(g["q"]), np.asarray(g["q2"]))
        gvv = gs.gram_view()[torch.from_numpy(off).cuda()].cpu().numpy()
        eg = np.abs(gvv - np.asarray(g["v"])) / np.asarray(g["scale"])
        med = {k: float(np.median([st[k] for st in stages])) for k in stages[0]}
        out[prec] = {
            "ms_median": float(np.median(tot)),
            "nnz_per_s": len(val) / (float(np.median(tot)) / 1000.0),
            "slice_ms": med,
            "gram_kernel": {"bound": "mfma", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": tf / FP64_PEAK_TFLOPS, "calls": k_n, "launches_per_call": 2,
                            "kernel_ms_per_call": k_ms / k_n, "algo_flops_per_call": k_flops / k_n,
                            "algo_bytes_per_call": k_bytes / k_n},
            "x2_dtype": "f64" if gs.x2_dtype == torch.float64 else "f32",
            "gram_traffic_per_call": (_traffic("slice_gram", gold["workload"], "cps") or (None,))[0]
            if prec == "fp64" else None,
            "error_vs_oracle": {"x2_max": float(np.max(ex)), "x2_median": float(np.median(ex)),
                                "gram_max": float(np.max(eg)), "gram_median": float(np.median(eg)),
                                "wnorm2_rel": abs(gs.wnorm2 - gold["norm2"]) / gold["norm2"],
                                "samples": len(ex), "scales": "x2: sum |c R_1[a, g]|; gram: sqrt(G_qq G_q2q2)"},
        }
        del gs
        torch.cuda.synchronize()
    return out


def main():
    args = _parse()
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is design-only.",
              file=sys.stderr)
        sys.exit(2)
    if args.stage:
        stage_only(args)
        return
    if args.slice_only:
        print(json.dumps({"c4_slice": c4_slice_leg(args.slice_only, tuple(args.slice_precisions.split(",")))}),
              flush=True)
        return
    import torch

    import paper_1908_02721_amd as tts
    from paper_1908_02721_amd import synth

    idx, val, dims, eps = synth.workload(args.workload)
    nnz = len(val)
    gi = torch.from_numpy(np.ascontiguousarray(idx)).cuda()
    gv = torch.from_numpy(np.ascontiguousarray(val)).cuda()
    matrix = None
    if args.matrix_input:
        if synth.WORKLOADS[args.workload]["kind"] != "laplace":
            sys.exit("--matrix-input needs a workload with a matrix form (laplace2d_qtt_L10)")
        r, c, v, m_dims, n_dims = synth.laplacian_matrix(synth.WORKLOADS[args.workload]["L"])
        matrix = (torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda(), m_dims, n_dims)
        gv = torch.from_numpy(np.ascontiguousarray(v)).cuda()

    # The evaluation plan depends only on the coordinates: it is built on a second
    # stream by a worker thread while the decomposition runs (the library calls
    # release the GIL), and its kernels fill the decomposition's read-back gaps.
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()

    def step(precision):
        ci = tts.matrix_to_tensor(*matrix) if matrix is not None else gi
        box = {}

        def build_plan():
            side.wait_stream(main)  # the coordinates are ready
            box["plan"] = tts.EvalPlan(ci, dims, stream=side)

        th = None
        if args.no_overlap:
            build_plan()
        else:
            th = threading.Thread(target=build_plan)
            th.start()
        try:
            if args.method == "fasttt":
                tt = tts.fasttt_decompose(ci, gv, dims, eps, p=args.p, precision=precision)
            else:
                tt = tts.decompose(ci, gv, dims, eps, precision=precision, dynamic_delta=args.dynamic_delta,
                                   key_bits=args.key_bits)
        finally:
            if th is not None:
                th.join()
        cores = tt.cores
        gy = gv if cores[0].dtype == torch.float64 else gv.float()
        # one plan per step: the sort and trie of the coordinates serve the forward and
        # the backward, and the backward reuses the forward's left products
        plan = box["plan"]
        side.wait_stream(main)  # the cores are ready
        with torch.cuda.stream(side):
            y = plan.forward(cores, save=True, stream=side)
            grads = plan.backward(cores, gy, use_saved=True, stream=side)
        main.wait_stream(side)
        return tt, y, grads

    def timed(precision, steps):
        times, dec_ms, stage = [], [], []
        t_all0 = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            tt, y, grads = step(precision)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            dec_ms.append(tt.times_ms["total"])
            stage.append(tt.times_ms)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t_all0
        return tt, t_all, times, dec_ms, stage

    for _ in range(args.warmup):
        step(args.precision)
    torch.cuda.synchronize()
    from paper_1908_02721_amd import _lib

    family = args.roofline
    if family == "auto":
        # time every family over two steps and take the one with the most time
        best = (-1.0, None)
        for fam in FAMILY_BOUND:
            _lib.kernel_timer_start(fam)
            for _ in range(2):
                step(args.precision)
            torch.cuda.synchronize()
            ms, n, _, _ = _lib.kernel_timer_read()
            _lib.kernel_timer_start(None)
            if n and ms > best[0]:
                best = (ms, fam)
        family = best[1]
    _lib.kernel_timer_start(family)
    tt, t_all, times, dec_ms, stage = timed(args.precision, args.steps)
    k_ms, k_n, k_bytes, k_flops = _lib.kernel_timer_read()
    _lib.kernel_timer_start(None)
    ms_per_step = 1000.0 * t_all / args.steps
    value = nnz / (t_all / args.steps)
    stage_med = {k: float(np.median([st[k] for st in stage])) for k in stage[0]}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (value / PUBLISHED[(args.workload, args.method)][0]
                        if (args.workload, args.method) in PUBLISHED else None),
        "dtype": "f64" if args.precision == "fp64" else args.precision,
        "data": "synthetic",
        "config": {"workload": args.workload, "dims": list(dims), "nnz": nnz, "eps": eps,
                   "precision": args.precision, "dynamic_delta": bool(args.dynamic_delta),
                   "matrix_input": bool(args.matrix_input), "key_bits": args.key_bits, "method": args.method,
                   "ranks": tt.ranks},
        "decompose_ms_median": float(np.median(dec_ms)),
        "decompose_nnz_per_s": nnz / (float(np.median(dec_ms)) / 1000.0),
        "stage_ms": stage_med,
        "step_ms_min": 1000.0 * min(times),
        "step_ms_median": 1000.0 * float(np.median(times)),
    }
    if (args.workload, args.method) in PUBLISHED:
        out["baseline"] = {"value": PUBLISHED[(args.workload, args.method)][0], "unit": "nnz/s",
                           "source": PUBLISHED[(args.workload, args.method)][1]}
    bound = FAMILY_BOUND.get(family, "alu")
    if k_n and k_ms > 0:
        if bound == "hbm":
            achieved = k_bytes / (k_ms / 1000.0) / 1e9
            peak, unit = HBM_PEAK_GBS, "GB/s"
        else:
            achieved = k_flops / (k_ms / 1000.0) / 1e12
            unit = "TFLOP/s"
            if family == "gemm_lp":
                peak = BF16_PEAK_TFLOPS if args.precision == "bf16" else FP32_PEAK_TFLOPS
            elif args.precision != "fp64" and family in ("eval_forward", "eval_up", "eval_grad"):
                peak = FP32_PEAK_TFLOPS
            else:
                peak = FP64_PEAK_TFLOPS
        tr = _traffic(family, args.workload, args.method) if args.precision == "fp64" else None
        out["roofline"] = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                           "traffic": tr[0] if tr else None, "traffic_source": tr[1] if tr else None,
                           "kernel": family, "launches_per_step": k_n / args.steps,
                           "kernel_ms_per_step": k_ms / args.steps,
                           "algo_bytes_per_launch": k_bytes / k_n, "algo_flops_per_launch": k_flops / k_n}
        if family == "jacobi":
            out["roofline"]["flops_note"] = "per launch: one sweep's flops times the sweeps the launch reported"
        if family in SINGLE_WORKGROUP:
            out["roofline"]["single_workgroup"] = True
            out["roofline"]["frac_of_one_cu"] = achieved / (peak / NUM_CU)
    if args.method == "cps" and not args.no_hbm:
        # the sparse stage (ingest, sort, every level) against HBM: algorithmic bytes over
        # its time, against the spec and against a device copy measured here
        b_alg = sparse_alg_bytes(nnz, len(dims), tt.level_sizes())
        t_sparse = stage_med["ingest"] + stage_med["sort"] + stage_med["sparse_levels"]
        gbps = b_alg / (t_sparse / 1000.0) / 1e9
        cp = copy_gbps()
        # the same decomposition alone, without the plan's sort and trie beside it on
        # the GPU: what the stage itself takes
        alone = []
        for _ in range(args.steps):
            tta = tts.decompose(gi, gv, dims, eps, precision=args.precision, dynamic_delta=args.dynamic_delta,
                                key_bits=args.key_bits)
            alone.append(tta.times_ms)
            del tta
        alone_med = {k: float(np.median([st[k] for st in alone])) for k in alone[0]}
        t_alone = alone_med["ingest"] + alone_med["sort"] + alone_med["sparse_levels"]
        gbps_alone = b_alg / (t_alone / 1000.0) / 1e9
        out["decompose_alone_ms_median"] = alone_med["total"]
        out["stage_ms_alone"] = alone_med
        out.setdefault("roofline", {})["sparse_hbm"] = {
            "bound": "hbm", "algo_bytes": b_alg, "t_ms": t_sparse, "achieved": gbps, "unit": "GB/s",
            "peak": HBM_PEAK_GBS, "frac": gbps / HBM_PEAK_GBS, "copy_GBps": cp, "frac_of_copy": gbps / cp,
            "t_ms_alone": t_alone, "achieved_alone": gbps_alone, "frac_alone": gbps_alone / HBM_PEAK_GBS,
            "frac_of_copy_alone": gbps_alone / cp,
            "note": "t_ms: inside the step, with the evaluation plan built beside it on a second stream; "
                    "t_ms_alone: the decomposition run by itself",
            "level_sizes": tt.level_sizes()}
    mixed_tt = None
    if args.precision == "fp64" and not args.no_mixed:
        # the precision form on the same workload: FP32 contractions, FP64 Grams/R/SVD
        step("fp32")
        torch.cuda.synchronize()
        mixed_tt, m_all, m_times, m_dec, m_stage = timed("fp32", args.steps)
        out["mixed"] = {"precision": "fp32", "value": nnz / (m_all / args.steps), "unit": "nnz/s",
                        "ms_per_step": 1000.0 * m_all / args.steps,
                        "decompose_ms_median": float(np.median(m_dec)),
                        "decompose_nnz_per_s": nnz / (float(np.median(m_dec)) / 1000.0),
                        "stage_ms": {k: float(np.median([st[k] for st in m_stage])) for k in m_stage[0]},
                        "ranks": mixed_tt.ranks,
                        "bf16": "not run: this workload's eps is below bfloat16's resolution (see c4_slice)"}
        if eps < 1e-6:
            out["mixed"]["eps_note"] = (f"eps = {eps:g} is below what FP32 contractions resolve: the FP32 result's "
                                        "error is FP32 rounding (~1e-7 relative), see error_vs_oracle")
    if not args.no_slice and args.method == "cps":
        out["c4_slice"] = c4_slice_leg(3, tuple(args.slice_precisions.split(",")))
    if not args.no_cpu_baseline:
        cores_host = [c.cpu().numpy() for c in tt.cores]
        out["cpu_baseline"], out["error_vs_oracle"], res = cpu_baseline(
            idx, val, dims, eps, args.cpu_sample, cores_host, args.precision, dynamic=args.dynamic_delta,
            key_bits=args.key_bits, method=args.method, p=args.p)
        if mixed_tt is not None:
            out["mixed"]["error_vs_oracle"] = error_vs_oracle(res, [c.cpu().numpy() for c in mixed_tt.cores], "fp32")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
