"""Benchmark of the lattice FMM hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]
                [--workload large_uniform|small_uniform|clusters|batched|serving]
                [--precision fp64|mixed|mixed-bf16]

A step is one whole solve of the hot path on one batch of synthetic input already resident
in HBM: tree construction (Morton keys, radix sort, levels, lists) plus the evaluation
passes (P2M, M2M, M2L, L2L, L2P and near field), from device xy and f to device u.  W
untimed steps, then K timed steps bracketed by device synchronisation, with --inflight
independent solves in flight (default 3, one stream and one output buffer each: the host-bound
plan build of one solve overlaps the evaluation of the previous one).  The serial rate (one
solve after another on one stream) and the single-solve latency are reported beside it.
Prints one JSON line.

Workloads (all seeded, synthetic):
  large_uniform (default)  1,000,000 distinct sources uniform in a 4096 x 4096 box, FP64
  small_uniform            1,000 sources uniform in a 256 x 256 box
  clusters                 2,000,000 sources in 64 Gaussian clusters in a 2^20 x 2^20 region
                           (adaptive tree by default, --tree uniform for the uniform-depth one)
  batched                  512 independent instances (log-uniform sizes 1e3..1e5) per step
  serving                  Poisson stream of requests (sizes log-uniform 1e2..1e6) through
                           the continuous-batching server; reports p50/p99 latency
The accuracy of the timed result is measured against the FP64 oracle on sampled targets; the
oracle's time on that sample is the CPU baseline.
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
sys.path.insert(0, ROOT)

METRIC = "Msources/s at rel.err ≤1e-10 (FP64) vs ≤1e-7 (mixed); p50/p99 solve latency"

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6       # FP64 vector and FP64 matrix (MFMA) alike
PEAK_FP32_TFLOPS = 157.3      # FP32 matrix (MFMA)
PEAK_BF16_TFLOPS = 2500.0     # bf16 matrix (MFMA), dense
PEAK_HBM_GBS = 8000.0
RANK = 48                     # skeleton size the kernels are compiled for

WORKLOADS = {
    "large_uniform": ("1,000,000 distinct sources uniform in a 4096x4096 box of Z^2, N(0,1) loads "
                      "mean-subtracted to an exact zero sum, targets = sources"),
    "small_uniform": ("1,000 distinct sources uniform in a 256x256 box of Z^2, N(0,1) loads "
                      "mean-subtracted to an exact zero sum, targets = sources"),
    "clusters": ("2,000,000 distinct sources in 64 Gaussian clusters (sigma 2,000) in a 2^20 x 2^20 "
                 "region of Z^2, U(-1,1) loads mean-subtracted, targets = sources"),
    "batched": ("512 independent instances, sizes log-uniform in [1e3, 1e5], each uniform in a box of "
                "side ceil(4 sqrt N), N(0,1) loads mean-subtracted per instance, one forest plan per step"),
    "serving": ("Poisson arrivals of solve requests, sizes log-uniform in [1e2, 1e6], uniform or "
                "8-cluster layout per request, through the continuous-batching server"),
    "inclusions": ("lattice with 50,000 modified bars (removed, weakened, strengthened, added diagonals) in a "
                   "2000x2000 box, far field v = m1 + 0.5 m2: GMRES on mu + B S mu = -B S B v over the bars' "
                   "nodes, S by a resident plan"),
    "dirichlet": ("Dirichlet problem on the 16384x16384 box: 65,532 boundary nodes, the dipole operator D "
                  "applied by the FMM, GMRES on D q = g"),
}
TOLERANCE = {"fp64": 1e-10, "mixed": 1e-7, "mixed-bf16": 1e-7}
# M2L kernel, its matrix-core peak, and the matrix-core flops it executes per algorithmic flop
M2L_KERNEL = {"fp64": ("k_m2l", PEAK_FP64_TFLOPS, 1.0), "mixed": ("k_m2l_mixed", PEAK_FP32_TFLOPS, 3.0),
              "mixed-bf16": ("k_m2l_bf16", PEAK_BF16_TFLOPS, 6.0)}


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary of this workload, or None when there is none or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    sys.path.insert(0, os.path.join(ROOT, "paper_1105_3505_amd"))
    from profile_summary import kernel_sources_hash
    with open(path) as fh:
        t = json.load(fh)
    if t.get("sources_sha256") != kernel_sources_hash():
        return None
    entry = t["per_dispatch"].get(kernel)
    return None if entry is None else entry["bytes"]


def roofline(dom: str, dom_ms: float, info: dict, n: int, precision: str, workload: str,
             alone_ms: float = None) -> dict:
    """Roofline entry for the dominant phase `dom`, whose average duration over the timed
    solves (HIP events on the execute stream) is dom_ms; alone_ms, when given, is its duration
    in the solves run one at a time before the timed region (no other solve's kernels beside it),
    reported as the same entry's "alone" figures."""
    out = _roofline(dom, dom_ms, info, n, precision, workload)
    if alone_ms and out.get("achieved") is not None:
        ratio = dom_ms / alone_ms
        out["alone"] = {"ms": alone_ms, "achieved": out["achieved"] * ratio, "frac": out["frac"] * ratio}
    return out


def _roofline(dom: str, dom_ms: float, info: dict, n: int, precision: str, workload: str) -> dict:
    sec = dom_ms * 1e-3
    if dom == "m2l":
        flops = 2.0 * RANK * RANK * info["m2l_pairs"]
        achieved = flops / sec / 1e12
        kernel, peak, executed = M2L_KERNEL[precision]
        out = {"kernel": kernel, "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
               "frac": achieved / peak, "traffic": measured_traffic(workload, kernel), "work_per_launch": flops,
               "work_definition": "2 P^2 flops per interaction-list pair, P = 48"}
        if executed != 1.0:
            # split products: the matrix cores execute `executed` flops per algorithmic flop
            out["executed_frac"] = executed * achieved / peak
            out["fp64_equivalent_frac"] = achieved / PEAK_FP64_TFLOPS
        return out
    if dom == "leaf" and info.get("adaptive"):
        pairs = info["near_pairs"] + info["m2p_terms"]
        flops = 2.0 * pairs + 2.0 * RANK * n
        achieved = flops / sec / 1e12
        kernel = "k_near_adaptive<48>"
        return {"kernel": kernel, "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": measured_traffic(workload, kernel), "work_per_launch": flops,
                "work_definition": "one FP64 FMA per U-list pair and per W-list skeleton term, plus 2P "
                                   "flops of L2P per target",
                "pairs_per_s": pairs / sec}
    if dom == "leaf":
        flops = 2.0 * info["near_pairs"] + 2.0 * RANK * n
        achieved = flops / sec / 1e12
        side = info["leaf_side"]
        kernel = "k_near<48, %d>" % (0 if side <= 16 else (1 if side <= 32 else 2))
        if side >= 64:
            kernel = "k_near_staged<48>"
        return {"kernel": kernel, "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": measured_traffic(workload, kernel), "work_per_launch": flops,
                "work_definition": "one FP64 FMA per near pair plus 2P flops of L2P per target",
                "pairs_per_s": info["near_pairs"] / sec}
    return {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": None, "traffic": None}


# arithmetic of each path: FP64 throughout, or FP64 with the M2L products on split operands
DTYPE = {"fp64": "f64", "mixed": "f64 (M2L: f32 hi/lo products)", "mixed-bf16": "f64 (M2L: 3-part bf16 products)"}


def base_result(args, value, ms_per_step, config, dtype=None):
    if dtype is None:
        dtype = DTYPE.get(getattr(args, "precision", "fp64"), "f64")
    return {
        "metric": METRIC, "value": value, "unit": "Msources/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
    }


PHASES_ALL = ("gather", "p2m", "m2m", "m2l", "l2l", "leaf")


def measure(step, steps, torch, inflight):
    """Phase split, timed region and latencies of `step(timing, slot)` (one whole solve: plan
    build, execute, plan release; `slot` names the stream and output buffers it uses).

    First a few solves with HIP events between all phases (outside the timed region) pick the
    dominant phase.  The timed region then runs `steps` independent solves between two device
    synchronisations with `inflight` of them in flight: solve i goes to stream i % inflight, so
    the host-bound build of one solve overlaps the evaluation passes of the one before it.  Each
    records only the two events around the dominant phase (its duration on its own stream, for
    the roofline); those are read, and the plan released, once `inflight` newer solves have been
    enqueued.  Next the same solves one after another on one stream (the serial rate), last
    solve latencies with each solve synchronised on its own and no events."""
    from collections import deque
    phases = []
    for _ in range(min(steps, 5)):
        plan = step(PHASES_ALL, 0)
        torch.cuda.synchronize()
        phases.append(plan.phase_times())
        plan.close()
    avg = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    dom = max(avg, key=avg.get)
    dom_ms = []
    pending = deque()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        pending.append(step([dom], i % inflight))
        if len(pending) >= inflight:
            plan = pending.popleft()
            dom_ms.append(plan.phase_times()[dom])
            plan.close()
    while pending:
        plan = pending.popleft()
        dom_ms.append(plan.phase_times()[dom])
        plan.close()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(None, 0).close()
    torch.cuda.synchronize()
    serial_ms = (time.perf_counter() - t0) * 1e3 / steps
    lat = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan = step(None, 0)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
        plan.close()
    return {"ms_per_step": ms_per_step, "serial_ms": serial_ms, "lat": lat, "avg": avg, "dom": dom,
            "dom_ms": float(np.mean(dom_ms))}


def streams_for(inflight, torch):
    """Stream of each in-flight slot: the current stream, then new default-priority streams."""
    return [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(inflight - 1)]


def timing_fields(m, n, inflight):
    return {"inflight": inflight, "serial_ms_per_step": m["serial_ms"],
            "serial_msources_per_s": n / (m["serial_ms"] * 1e-3) / 1e6,
            "p50_ms": float(np.percentile(m["lat"], 50)), "p99_ms": float(np.percentile(m["lat"], 99)),
            "phase_ms": m["avg"]}


def cpu_baseline(xy, f, u, n_targets, seed=20):
    """Oracle direct sum on sampled targets: accuracy of u and the CPU rate."""
    import workloads as wl
    from oracle import direct as od
    idx = wl.sample_targets(seed, len(xy), n_targets)
    t0 = time.perf_counter()
    ref = od.direct_sum(xy[idx], xy, f)
    cpu_s = time.perf_counter() - t0
    err = float(np.linalg.norm(u[idx] - ref) / np.linalg.norm(ref))
    base = {"value": len(idx) / cpu_s / 1e6, "unit": "Msources/s", "cores": od.threads(), "kind": "oracle",
            "sample": "%d sampled targets x %d sources (direct sum), %.2f s wall; the rate is targets "
                      "completed per second" % (len(idx), len(xy), cpu_s)}
    return err, len(idx), base


def make_input(name):
    import workloads as wl
    return {"large_uniform": wl.config_large_uniform, "small_uniform": wl.config_small_uniform,
            "clusters": wl.config_clusters}[name]()


def run_single(args, torch, lf):
    xy, f = make_input(args.workload)
    n = len(xy)
    dev = torch.device("cuda:0")
    xy_d = torch.from_numpy(xy).to(dev)
    f_d = torch.from_numpy(f).to(dev)
    ctx = lf.Context(0, precision=args.precision, max_leaf=args.max_leaf, stencil=args.stencil,
                     adaptive=args.tree == "adaptive")
    streams = streams_for(args.inflight, torch)
    outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in streams]
    sorted_io = args.io == "sorted"
    if sorted_io:
        # loads already in the plan's Morton order (the sort of these points is the same for
        # every plan of them): potentials come back in that order too
        p0 = ctx.plan(xy_d)
        perm_d = torch.from_numpy(p0.export("perm").astype(np.int64)).to(dev)
        p0.close()
        f_in = f_d[perm_d].contiguous()
    else:
        f_in = f_d

    def step(timing, slot):
        st = streams[slot]
        plan = ctx.plan(xy_d, stream=st)
        if timing:
            plan.set_timing_phases(timing)
        if sorted_io:
            plan.execute_sorted(f_in, outs[slot], stream=st)
        else:
            plan.execute(f_in, outs[slot], stream=st)
        return plan

    for _ in range(max(args.warmup, 1)):
        for slot in range(len(streams)):
            step(None, slot).close()
    m = measure(step, args.steps, torch, args.inflight)
    ms_per_step = m["ms_per_step"]
    value = n / (ms_per_step * 1e-3) / 1e6
    torch.cuda.synchronize()
    same = all(torch.equal(o, outs[0]) for o in outs[1:])   # every slot computed the same solve

    # execute-only throughput on a resident plan (outside the timed steps: plan statistics)
    stream = streams[0]
    u_d = outs[0]
    plan = ctx.plan(xy_d, stream=stream)
    info = plan.info()
    run = (lambda: plan.execute_sorted(f_in, u_d, stream=stream)) if sorted_io else \
        (lambda: plan.execute(f_in, u_d, stream=stream))
    for _ in range(3):
        run()
    torch.cuda.synchronize()
    reps = max(args.steps, 10)
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    exec_ms = (time.perf_counter() - t0) * 1e3 / reps
    if sorted_io:   # back to the caller's order for the checks below
        u_caller = torch.empty_like(u_d)
        u_caller[perm_d] = u_d
        for o in outs:
            o.copy_(u_caller)
    u = u_d.cpu().numpy()
    plan.close()
    equation = None
    if args.stencil == 9:
        equation = nine_point_equation_residual(ctx, xy, f, torch)
    ctx.close()

    config = {"workload": WORKLOADS[args.workload], "n_sources": n, "precision": args.precision,
              "tree": args.tree, "leaf_level": info["leaf_level"], "leaf_side": info["leaf_side"],
              "max_leaf": args.max_leaf, "rank": RANK, "eps": 1e-12,
              "operator": "9-point isotropic" if args.stencil == 9 else "5-point",
              "io": "plan (Morton) order" if sorted_io else "caller order"}
    result = base_result(args, value, ms_per_step, config)
    result.update(timing_fields(m, n, args.inflight))
    result.update({"inflight_outputs_equal": same,
                   "execute_only_ms": exec_ms, "execute_only_msources_per_s": n / (exec_ms * 1e-3) / 1e6,
                   "plan": info,
                   "roofline": roofline(m["dom"], m["dom_ms"], info, n, args.precision, args.workload,
                                         m["avg"][m["dom"]])})
    if equation is not None:
        result["equation_residual"] = equation
        result["equation_residual_definition"] = ("max |A9 u - f| / max |u| over the 9-point stencils of 2,000 "
                                                  "sampled cells (u there from a plan with those targets)")
    if not args.no_cpu_baseline and args.stencil == 5:
        err, k, base = cpu_baseline(xy, f, u, args.cpu_targets)
        result["rel_err_vs_oracle"] = err
        result["rel_err_sample"] = k
        result["tolerance"] = TOLERANCE[args.precision]
        result["cpu_baseline"] = base
    elif not args.no_cpu_baseline:
        # the oracle's 9-point phi spans |m|_inf <= 128: its direct sum over the points of a
        # 128 x 128 corner of the input, timed, and compared with a plan of those points
        from oracle import direct as od
        sub = np.all(xy < 128, axis=1)
        xs, fs = xy[sub], f[sub]
        c2 = lf.Context(0, precision=args.precision, max_leaf=args.max_leaf, stencil=9)
        us = c2.plan(torch.from_numpy(xs).cuda()).execute(torch.from_numpy(fs).cuda()).cpu().numpy()
        c2.close()
        t0 = time.perf_counter()
        ref = od.direct_sum(xs, xs, fs, stencil=9)
        cpu_s = time.perf_counter() - t0
        result["rel_err_vs_oracle"] = float(np.linalg.norm(us - ref) / np.linalg.norm(ref))
        result["rel_err_sample"] = int(len(xs))
        result["tolerance"] = TOLERANCE[args.precision]
        result["cpu_baseline"] = {"value": len(xs) / cpu_s / 1e6, "unit": "Msources/s", "cores": od.threads(),
                                  "kind": "oracle",
                                  "sample": "9-point direct sum over the %d points of the 128x128 corner of the "
                                            "input (all targets), %.3f s" % (len(xs), cpu_s)}
    return result


def nine_point_equation_residual(ctx, xy, f, torch):
    """A9 u = f (the 9-point operator's equation) at the stencils of 2,000 sampled cells."""
    rng = np.random.default_rng(91)
    centres = xy[rng.choice(len(xy), size=2000, replace=False)].astype(np.int64)
    off = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [1, 1], [-1, 1], [1, -1], [-1, -1]])
    pts = (centres[None, :, :] + off[:, None, :]).reshape(-1, 2).astype(np.int32)
    plan = ctx.plan(torch.from_numpy(xy).cuda(), targets=torch.from_numpy(pts).cuda())
    u = plan.execute(torch.from_numpy(f).cuda()).cpu().numpy().reshape(9, -1)
    plan.close()
    a9u = (20 * u[0] - 4 * u[1:5].sum(axis=0) - u[5:].sum(axis=0)) / 6
    # loads at the centres (distinct cells: each centre is one source)
    idx = {tuple(p): i for i, p in enumerate(xy.tolist())}
    fc = np.array([f[idx[tuple(c)]] for c in centres.tolist()])
    return float(np.max(np.abs(a9u - fc)) / np.max(np.abs(u)))


def run_batched(args, torch, lf):
    import workloads as wl
    inst = wl.config_batched()
    n = sum(len(a) for a, _ in inst)
    xs = [torch.from_numpy(a).cuda() for a, _ in inst]
    fs = [torch.from_numpy(b).cuda() for _, b in inst]
    ctx = lf.Context(0, precision=args.precision, max_leaf=0 if args.autotune else args.max_leaf)
    tuned = None
    if args.autotune:
        # one N_leaf for the whole forest, timed on the forest (lfmm_autotune_batch), recorded
        # for every instance's size class; the timed plans then take it in automatic mode
        best, times = ctx.autotune_batch(xs, candidates=(16, 32, 64, 128), objective="execute", reps=2)
        tuned = {"max_leaf": best, "execute_ms": {str(c): round(t, 4) for c, t in times.items()}}
    streams = streams_for(args.inflight, torch)
    outs = [[torch.empty_like(b) for b in fs] for _ in streams]

    def step(timing, slot):
        st = streams[slot]
        plan = ctx.plan_batch(xs, stream=st)
        if timing:
            plan.set_timing_phases(timing)
        plan.execute_instances(fs, outs[slot], stream=st)
        return plan

    for _ in range(max(args.warmup, 1)):
        for slot in range(len(streams)):
            step(None, slot).close()
    m = measure(step, args.steps, torch, args.inflight)
    ms_per_step = m["ms_per_step"]
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for o in outs[1:] for a, b in zip(o, outs[0]))
    stream = streams[0]
    us = outs[0]
    plan = ctx.plan_batch(xs, stream=stream)
    info = plan.info()
    plan.execute_instances(fs, us, stream=stream)
    torch.cuda.synchronize()
    reps = max(args.steps, 5)
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.execute_instances(fs, us, stream=stream)
    torch.cuda.synchronize()
    exec_ms = (time.perf_counter() - t0) * 1e3 / reps
    plan.close()
    ctx.close()
    config = {"workload": WORKLOADS["batched"], "n_instances": len(inst), "n_sources": n,
              "precision": args.precision, "max_leaf": "autotuned (%d)" % tuned["max_leaf"] if tuned else args.max_leaf,
              "rank": RANK, "eps": 1e-12}
    result = base_result(args, n / (ms_per_step * 1e-3) / 1e6, ms_per_step, config)
    result.update(timing_fields(m, n, args.inflight))
    if tuned:
        result["autotuned_max_leaf"] = tuned
    result.update({"inflight_outputs_equal": same,
                   "execute_only_ms": exec_ms, "execute_only_msources_per_s": n / (exec_ms * 1e-3) / 1e6,
                   "plan": info,
                   "roofline": roofline(m["dom"], m["dom_ms"], info, n, args.precision, "batched",
                                         m["avg"][m["dom"]])})
    if not args.no_cpu_baseline:
        # accuracy on 100 sampled targets of every 8th instance; CPU rate over that sample
        from oracle import direct as od
        num = den = 0.0
        t0 = time.perf_counter()
        k = 0
        for i in range(0, len(inst), 8):
            xy, f = inst[i]
            idx = wl.sample_targets(1000 + i, len(xy), 100)
            ref = od.direct_sum(xy[idx], xy, f)
            u = us[i].cpu().numpy()[idx]
            num += float(np.sum((u - ref) ** 2))
            den += float(np.sum(ref ** 2))
            k += len(idx)
        cpu_s = time.perf_counter() - t0
        result["rel_err_vs_oracle"] = (num / den) ** 0.5
        result["rel_err_sample"] = k
        result["tolerance"] = TOLERANCE[args.precision]
        result["cpu_baseline"] = {"value": k / cpu_s / 1e6, "unit": "Msources/s", "cores": od.threads(),
                                  "kind": "oracle",
                                  "sample": "100 sampled targets of every 8th instance (%d targets), %.2f s "
                                            "wall; the rate is targets completed per second" % (k, cpu_s)}
    return result


def _laplacian_residual(u5):
    """Relative 5-point residual A u at stencil centres from the potentials at the centres and
    their four neighbours (rows: centre, +x, -x, +y, -y)."""
    c, e, w, n, s = u5
    return np.abs(4 * c - e - w - n - s)


def _stencils(pts):
    off = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1]], dtype=np.int32)
    return (pts[None, :, :] + off[:, None, :]).reshape(-1, 2)


def run_inclusions(args, torch, lf):
    """Section 10.1 at scale: one step is one GMRES solve of eq. 10.4 on a resident plan.  The
    value counts nodes of Omega_inc solved per second.  Accuracy at full size: the recovered u
    satisfies (A + B) u = 0 at sampled stencils away from the bars (A u = 0 there) and at the
    bars' nodes (A u + B u = 0), a property of the exact solution at any size."""
    import workloads as wl
    rng = np.random.default_rng(8)
    bars, delta = wl.inclusion_bars(rng, 50000, 2000)
    c1, c2 = 1.0, 0.5
    ctx = lf.Context(0)
    inc = lf.Inclusions(ctx, bars, delta)
    nn = len(inc.nodes)
    mu = torch.empty(nn, dtype=torch.float64, device="cuda")
    for _ in range(max(args.warmup, 1)):
        inc.solve(c1, c2, mu, tol=1e-12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = inc.solve(c1, c2, mu, tol=1e-12)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # one S apply on the resident plan (the operator GMRES applies once per iteration)
    plan = ctx.plan(torch.from_numpy(inc.nodes).cuda())
    s_out = torch.empty_like(mu)
    plan.execute(mu, s_out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        plan.execute(mu, s_out)
    torch.cuda.synchronize()
    apply_ms = (time.perf_counter() - t0) * 1e3 / 20
    plan.close()
    # (A + B) u = 0: stencils at sampled nodes and at sampled free lattice points of the box
    smp = rng.choice(nn, size=2000, replace=False)
    free = rng.integers(0, 2000, size=(2000, 2)).astype(np.int32)
    centres = np.vstack([inc.nodes[smp], free]).astype(np.int32)
    pts = _stencils(centres)
    u = inc.potential(c1, c2, mu, torch.from_numpy(pts).cuda()).cpu().numpy().reshape(5, -1)
    au = 4 * u[0] - u[1] - u[2] - u[3] - u[4]
    # B u at the sampled nodes: from the bars at each node, with u at their other ends
    others = {}
    for (a1, a2, b1, b2), d in zip(bars.tolist(), delta.tolist()):
        others.setdefault((a1, a2), []).append(((b1, b2), d))
        others.setdefault((b1, b2), []).append(((a1, a2), d))
    cen = [tuple(c) for c in centres.tolist()]
    ends = sorted({p for c in cen for p, _ in others.get(c, [])})
    ue = dict(zip(ends, inc.potential(c1, c2, mu, torch.from_numpy(np.array(ends, np.int32)).cuda()).cpu().numpy()))
    bu = np.zeros(len(centres))
    for k, c in enumerate(cen):
        for p, d in others.get(c, []):
            bu[k] += d * (u[0][k] - ue[p])
    scale = np.max(np.abs(u[0] - (c1 * centres[:, 0] + c2 * centres[:, 1])))
    resid = float(np.max(np.abs(au + bu)) / scale)
    inc.close()
    ctx.close()
    config = {"workload": WORKLOADS["inclusions"], "n_bars": len(bars), "n_nodes": nn, "gmres_tol": 1e-12}
    result = base_result(args, nn / (ms * 1e-3) / 1e6, ms, config)
    result.update({"iterations": st["iterations"], "rel_residual": st["rel_residual"],
                   "ms_per_iteration": ms / max(st["iterations"], 1), "s_apply_ms": apply_ms,
                   "s_apply_msources_per_s": nn / (apply_ms * 1e-3) / 1e6,
                   "equation_residual": resid,
                   "equation_residual_definition": "max |(A+B)u| at 4,000 sampled stencils / max |u - v| there"})
    if not args.no_cpu_baseline:
        from oracle import direct as od
        idx = wl.sample_targets(80, nn, 2000)
        mu_h = mu.cpu().numpy()
        t0 = time.perf_counter()
        ref = od.direct_sum(inc.nodes[idx], inc.nodes, mu_h)
        cpu_s = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": len(idx) / cpu_s / 1e6, "unit": "Msources/s", "cores": od.threads(),
                                  "kind": "oracle",
                                  "sample": "one S apply (direct sum) at %d sampled nodes x %d nodes, %.2f s; the "
                                            "rate is targets completed per second" % (len(idx), nn, cpu_s)}
        del ref
    return result


def run_dirichlet(args, torch, lf):
    """Section 10.2 at scale: one step is one GMRES solve of eq. 10.7; the value counts boundary
    nodes solved per second.  Accuracy at full size: D applied by the FMM against the oracle's
    direct sum on sampled boundary nodes, the true residual of the solve, and A u = 0 at sampled
    interior stencils (the property that makes u = D q the solution)."""
    import workloads as wl
    from oracle import extensions as ox
    N = 16384
    gamma, codes, _ = wl.box_boundary(N, N)
    n = len(gamma)
    rng = np.random.default_rng(9)
    g = np.sin(1e-3 * gamma[:, 0]) * np.cos(7e-4 * gamma[:, 1]) + 0.05 * rng.standard_normal(n)
    ctx = lf.Context(0)
    dirp = lf.Dirichlet(ctx, gamma, codes)
    g_d = torch.from_numpy(g).cuda()
    q = torch.empty_like(g_d)
    for _ in range(max(args.warmup, 1)):
        dirp.solve(g_d, q, tol=1e-12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = dirp.solve(g_d, q, tol=1e-12)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    out = torch.empty_like(g_d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        dirp.apply(q, out)
    torch.cuda.synchronize()
    apply_ms = (time.perf_counter() - t0) * 1e3 / 20
    qh = q.cpu().numpy()
    # interior stencils
    centres = rng.integers(2, N - 1, size=(3000, 2)).astype(np.int32)
    u = dirp.potential(q, torch.from_numpy(_stencils(centres)).cuda()).cpu().numpy().reshape(5, -1)
    lap = float(np.max(np.abs(4 * u[0] - u[1] - u[2] - u[3] - u[4])) / np.max(np.abs(u[0])))
    config = {"workload": WORKLOADS["dirichlet"], "n_boundary": n, "box": N, "gmres_tol": 1e-12}
    result = base_result(args, n / (ms * 1e-3) / 1e6, ms, config)
    result.update({"iterations": st["iterations"], "rel_residual": st["rel_residual"],
                   "ms_per_iteration": ms / max(st["iterations"], 1), "d_apply_ms": apply_ms,
                   "d_apply_msources_per_s": 2 * n / (apply_ms * 1e-3) / 1e6,
                   "interior_laplacian_residual": lap})
    if not args.no_cpu_baseline:
        from oracle import direct as od
        idx = wl.sample_targets(90, n, 2000)
        t0 = time.perf_counter()
        ref = ox.d_apply(gamma, codes, qh, gamma[idx])
        cpu_s = time.perf_counter() - t0
        d_full = out.cpu().numpy()[idx]
        result["rel_err_vs_oracle"] = float(np.linalg.norm(d_full - ref) / np.linalg.norm(ref))
        result["rel_err_sample"] = len(idx)
        result["tolerance"] = TOLERANCE["fp64"]
        result["cpu_baseline"] = {"value": len(idx) / cpu_s / 1e6, "unit": "Msources/s", "cores": od.threads(),
                                  "kind": "oracle",
                                  "sample": "D q by direct sum at %d sampled boundary nodes x %d dipole ends, %.2f s; "
                                            "the rate is targets completed per second" % (len(idx), 2 * n, cpu_s)}
    dirp.close()
    ctx.close()
    return result


def run_serving(args, torch, lf):
    """Serving protocol: a stream of args.requests requests (the first args.warm_requests of each
    run are warm-up and left out of the latency statistics).  First a closed-loop run (every
    request submitted at once) measures the sustainable rate mu (requests per second); then
    Poisson arrivals at lambda = rho mu for each rho of --loads (value: the rho = 0.8 run), or at
    the fixed --rate."""
    import workloads as wl
    m = args.requests
    w = min(args.warm_requests, m - 1)
    reqs = []
    for i in range(m):
        reqs.append(wl.config_serving_request(5, i))
        if (i + 1) % 200 == 0:
            print("serving: %d of %d requests generated" % (i + 1, m), file=sys.stderr, flush=True)
    n_total = sum(len(r[0]) for r in reqs)
    n_counted = sum(len(r[0]) for r in reqs[w:])
    dev = [(torch.from_numpy(xy).cuda(), torch.from_numpy(f).cuda()) for xy, f, _ in reqs]
    us = [torch.empty_like(f) for _, f in dev]
    ctx = lf.Context(0, precision=args.precision, max_leaf=args.max_leaf)
    srv = lf.Server(ctx, max_batch=args.max_batch, max_inflight=3)

    def run_stream(gaps):
        """Submits request i at time sum(gaps[:i + 1]) (all at once when gaps is None)."""
        tickets = [None] * m
        t_start = time.perf_counter()

        def client():
            t = t_start
            for i in range(m):
                if gaps is not None:
                    t += gaps[i]
                    d = t - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                tickets[i] = srv.submit(dev[i][0], dev[i][1], us[i])

        th = threading.Thread(target=client)
        th.start()
        th.join()
        stats = [srv.wait(t)[1] for t in tickets]
        makespan = time.perf_counter() - t_start
        lat = np.array([(s["t_done"] - s["t_submit"]) * 1e3 for s in stats[w:]])
        t_first = min(s["t_submit"] for s in stats[w:])
        t_last = max(s["t_done"] for s in stats[w:])
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "msources_per_s": n_counted / (t_last - t_first) / 1e6,
                "iterations": len({s["batch_id"] for s in stats}), "makespan_s": makespan}

    run_stream(None)                     # warm-up: operators of every leaf side, memory pool
    closed = run_stream(None)
    mu = m / closed["makespan_s"]
    print("serving: closed loop %.1f requests/s" % mu, file=sys.stderr, flush=True)
    runs = {}
    rng = np.random.default_rng(6)
    if args.rate > 0:
        plan_rates = {"fixed": args.rate}
    else:
        plan_rates = {"%.2f" % float(r): float(r) * mu for r in args.loads.split(",")}
    for key, lam in plan_rates.items():
        gaps = rng.exponential(1.0 / lam, size=m)
        r = run_stream(gaps)
        print("serving: load %s done (p99 %.2f ms)" % (key, r["p99_ms"]), file=sys.stderr, flush=True)
        r["rate_per_s"] = lam
        r["offered_msources_per_s"] = n_total / float(np.sum(gaps)) / 1e6
        runs[key] = r
    srv.close()
    ctx.close()
    main_key = "fixed" if args.rate > 0 else ("0.80" if "0.80" in runs else next(iter(runs)))
    main = runs[main_key]
    config = {"workload": WORKLOADS["serving"], "requests": m, "warm_requests": w,
              "n_sources_total": n_total, "precision": args.precision, "max_batch": args.max_batch,
              "max_inflight": 3, "protocol": ("Poisson arrivals at %s" % ("a fixed rate" if args.rate > 0 else
                                                                         "lambda = rho mu, mu closed-loop")),
              "rho": None if args.rate > 0 else float(main_key)}
    result = base_result(args, main["msources_per_s"], main["makespan_s"] * 1e3 / m, config)
    result.update({"p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"],
                   "closed_loop": {"requests_per_s": mu, "msources_per_s": closed["msources_per_s"],
                                   "p50_ms": closed["p50_ms"], "p99_ms": closed["p99_ms"]},
                   "loads": runs})
    if not args.no_cpu_baseline:
        from oracle import direct as od
        num = den = 0.0
        k = 0
        t0 = time.perf_counter()
        for i in range(0, m, max(1, m // 20)):
            xy, f, _ = reqs[i]
            idx = wl.sample_targets(3000 + i, len(xy), 100)
            ref = od.direct_sum(xy[idx], xy, f)
            u = us[i].cpu().numpy()[idx]
            num += float(np.sum((u - ref) ** 2))
            den += float(np.sum(ref ** 2))
            k += len(idx)
        cpu_s = time.perf_counter() - t0
        result["rel_err_vs_oracle"] = (num / den) ** 0.5
        result["rel_err_sample"] = k
        result["tolerance"] = TOLERANCE[args.precision]
        result["cpu_baseline"] = {"value": k / cpu_s / 1e6, "unit": "Msources/s", "cores": od.threads(),
                                  "kind": "oracle",
                                  "sample": "100 sampled targets of 20 requests (%d targets), %.2f s wall; "
                                            "the rate is targets completed per second" % (k, cpu_s)}
    return result


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_uniform", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=sorted(TOLERANCE))
    ap.add_argument("--max-leaf", type=int, default=None,
                    help="N_leaf (default 64; 32 on the adaptive tree)")
    ap.add_argument("--tree", choices=("uniform", "adaptive"), default=None,
                    help="tree of Section 6: uniform depth, or adaptive (refined while a box holds more than "
                         "N_leaf points); default adaptive for clusters, uniform otherwise")
    ap.add_argument("--stencil", type=int, default=5, choices=(5, 9),
                    help="lattice operator: the 5-point Laplacian of the paper or the isotropic 9-point one")
    ap.add_argument("--autotune", action="store_true",
                    help="batched: N_leaf chosen by lfmm_autotune_batch on the whole forest before the timed steps")
    ap.add_argument("--io", choices=("caller", "sorted"), default="caller",
                    help="single-plan workloads: loads and potentials in the caller's order (lfmm_execute) or "
                         "in the plan's Morton order (lfmm_execute_sorted)")
    ap.add_argument("--inflight", type=int, default=3,
                    help="independent solves in flight in the timed region, one stream each")
    ap.add_argument("--cpu-targets", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests in the stream")
    ap.add_argument("--warm-requests", type=int, default=200,
                    help="serving: first requests of each run left out of the latency statistics")
    ap.add_argument("--loads", default="0.5,0.8,0.95",
                    help="serving: arrival rates as fractions of the closed-loop rate (0.8 gives value)")
    ap.add_argument("--rate", type=float, default=0.0, help="serving: fixed arrivals per second instead")
    ap.add_argument("--max-batch", type=int, default=64, help="serving: requests per iteration")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first fill and copy a buffer of this many MiB (a known-traffic reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.tree is None:
        args.tree = "adaptive" if args.workload == "clusters" else "uniform"
    if args.max_leaf is None:
        args.max_leaf = 32 if args.tree == "adaptive" else 64
    if args.inflight < 1:
        ap.error("--inflight must be at least 1")
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1105_3505_amd as lf

    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batched":
        result = run_batched(args, torch, lf)
    elif args.workload == "inclusions":
        result = run_inclusions(args, torch, lf)
    elif args.workload == "dirichlet":
        result = run_dirichlet(args, torch, lf)
    elif args.workload == "serving":
        result = run_serving(args, torch, lf)
    else:
        result = run_single(args, torch, lf)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
