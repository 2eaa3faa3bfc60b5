"""Benchmark of the lattice FMM hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large_uniform|small_uniform]

A step is one whole solve of the hot path on one batch of synthetic input already resident
in HBM: tree construction (Morton keys, radix sort, levels, lists) plus the evaluation
passes (P2M, M2M, M2L, L2L, L2P and near field), from device xy and f to device u.  W
untimed steps, then K timed steps bracketed by device synchronisation.  Prints one JSON line.

The default workload is 1,000,000 distinct sources uniform in a 4096 x 4096 box with N(0,1)
loads made exactly zero-sum, targets = sources, FP64.  The accuracy of the timed result is
measured against the FP64 oracle on 1,000 sampled targets, which is also the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Msources/s at rel.err ≤1e-10 (FP64) vs ≤1e-7 (mixed); p50/p99 solve latency"

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6       # FP64 vector and FP64 matrix (MFMA) alike
PEAK_HBM_GBS = 8000.0
RANK = 48                     # skeleton size the kernels are compiled for

WORKLOADS = {
    "large_uniform": ("1,000,000 distinct sources uniform in a 4096x4096 box of Z^2, N(0,1) loads "
                      "mean-subtracted to an exact zero sum, targets = sources"),
    "small_uniform": ("1,000 distinct sources uniform in a 256x256 box of Z^2, N(0,1) loads "
                      "mean-subtracted to an exact zero sum, targets = sources"),
}


def make_input(name):
    import workloads as wl
    if name == "large_uniform":
        return wl.config_large_uniform()
    return wl.config_small_uniform()


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_uniform", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-targets", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1105_3505_amd as lf

    xy, f = make_input(args.workload)
    n = len(xy)
    dev = torch.device("cuda:0")
    xy_d = torch.from_numpy(xy).to(dev)
    f_d = torch.from_numpy(f).to(dev)
    u_d = torch.empty(n, dtype=torch.float64, device=dev)
    ctx = lf.Context(0)
    stream = torch.cuda.current_stream()

    def step(timed_phases=None):
        plan = ctx.plan(xy_d, stream=stream)
        if timed_phases is not None:
            plan.set_timing(True)
        plan.execute(f_d, u_d, stream=stream)
        return plan

    for _ in range(max(args.warmup, 1)):
        step().close()
    torch.cuda.synchronize()

    lat, phases, info = [], [], None
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        plan = step(timed_phases=True)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
        phases.append(plan.phase_times())
        if info is None:
            info = plan.info()
        plan.close()
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_all
    ms_per_step = total_s * 1e3 / args.steps
    value = n / (ms_per_step * 1e-3) / 1e6

    # execute-only throughput on a resident plan
    plan = ctx.plan(xy_d, stream=stream)
    for _ in range(3):
        plan.execute(f_d, u_d, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(args.steps, 10)
    for _ in range(reps):
        plan.execute(f_d, u_d, stream=stream)
    torch.cuda.synchronize()
    exec_ms = (time.perf_counter() - t0) * 1e3 / reps
    u = u_d.cpu().numpy()
    plan.close()

    avg = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    dom = max(avg, key=avg.get)
    if dom == "m2l":
        flops = 2.0 * RANK * RANK * info["m2l_pairs"]
        achieved = flops / (avg[dom] * 1e-3) / 1e12
        roof = {"kernel": "m2l (FP64 MFMA)", "bound": "mfma", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": None, "work_per_launch": flops,
                "work_definition": "2 P^2 flops per interaction-list pair, P = 48"}
    elif dom == "leaf":
        flops = 2.0 * info["near_pairs"] + 2.0 * RANK * n
        achieved = flops / (avg[dom] * 1e-3) / 1e12
        roof = {"kernel": "leaf (near field + L2P)", "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": None, "work_per_launch": flops,
                "work_definition": "one FP64 FMA per near pair plus 2P flops of L2P per target",
                "pairs_per_s": info["near_pairs"] / (avg[dom] * 1e-3)}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": None, "traffic": None}

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "Msources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n_sources": n, "precision": "fp64",
                   "leaf_level": info["leaf_level"], "leaf_side": info["leaf_side"],
                   "max_leaf": 64, "rank": RANK, "eps": 1e-12},
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "execute_only_ms": exec_ms,
        "execute_only_msources_per_s": n / (exec_ms * 1e-3) / 1e6,
        "phase_ms": avg,
        "plan": info,
        "roofline": roof,
    }

    if not args.no_cpu_baseline:
        import workloads as wl
        from oracle import direct as od
        idx = wl.sample_targets(20, n, args.cpu_targets)
        t0 = time.perf_counter()
        ref = od.direct_sum(xy[idx], xy, f)
        cpu_s = time.perf_counter() - t0
        err = float(np.linalg.norm(u[idx] - ref) / np.linalg.norm(ref))
        result["rel_err_vs_oracle"] = err
        result["rel_err_sample"] = len(idx)
        result["cpu_baseline"] = {
            "value": len(idx) / cpu_s / 1e6, "unit": "Msources/s", "cores": od.threads(), "kind": "oracle",
            "sample": "%d sampled targets x %d sources (direct sum), %.2f s wall; the rate is targets "
                      "completed per second" % (len(idx), n, cpu_s)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
