#!/usr/bin/env python3
"""Benchmark of batched Picard-Chebyshev propagation on one MI355X.

One step = one full propagation of the workload (ephemeris table, warm starts, all
Picard iterations of all segments, convergence tests, chaining, end states) with the
initial conditions already resident in HBM.  Default workload: the N-body Venus
ensemble, 4096 ICs, Sun + 8 planets, 450 days in 8 segments of 128 CGL nodes, FP64,
tol 1e-12.

Prints one JSON line: IC-segment propagations/s (the workload's ICs x segments per
second), checked against the FP64 CPU oracle on a sample (<= 1e-10 relative), with the
roofline of the propagation kernel and the oracle's own rate on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
METRIC = "IC-segment propagations/s at <=1e-10 rel err; batched/mixed vs plain GPU speedup"


def algorithmic_flops(w, iters):
    """Algorithmic FP64 work of the Picard iterations actually run: per IC, segment and
    iteration, the folded fit/integrate/evaluate product (6 columns x 2 N^2) plus the
    dynamics at N nodes (20 flops per body interaction, Sun + P perturbers, and 3 for
    the precomputed indirect term)."""
    P = w.pert.shape[0]
    total = 0.0
    for g in w.groups:
        it = iters[g.ic_offset:g.ic_offset + g.n_ic, :g.segments]
        it = np.where(it > 0, it, 0).astype(np.float64)
        N = g.nodes
        per_iter = 12.0 * N * N + (20.0 * (P + 1) + 3.0) * N
        total += per_iter * it.sum()
    return total


def rel_err(a, b):
    er = np.linalg.norm(a[:, :3] - b[:, :3], axis=1) / np.linalg.norm(b[:, :3], axis=1)
    ev = np.linalg.norm(a[:, 3:] - b[:, 3:], axis=1) / np.linalg.norm(b[:, 3:], axis=1)
    return np.maximum(er, ev)


def oracle_states(w, idx):
    import oracle
    model = oracle.Model(w.mu_sun, w.pert, w.epoch)
    out = np.zeros((idx.size, 6))
    iters = np.zeros((idx.size, max(g.segments for g in w.groups)), dtype=np.int32)
    for g in w.groups:
        sel = np.nonzero((idx >= g.ic_offset) & (idx < g.ic_offset + g.n_ic))[0]
        if sel.size:
            s, it = oracle.propagate(w.ics[idx[sel]], g.t0, g.tf, g.nodes, g.segments, g.tol, model,
                                     init=w.init)
            out[sel] = s
            iters[sel, :g.segments] = it
    return out, iters, oracle.propagate.last_threads


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="nbody-venus-4096")
    ap.add_argument("--tile-pairs", type=int, default=0)
    ap.add_argument("--graph", action="store_true", help="replay the call as a captured HIP graph")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32-fp64"],
                    help="sweep arithmetic (default: the workload's)")
    ap.add_argument("--switch-tol", type=float, default=0.0, help="FP32 -> FP64 switch (0: library default)")
    ap.add_argument("--autotune", action="store_true", help="pick the job shape with the autotuner first")
    ap.add_argument("--check-ics", type=int, default=64, help="ICs checked against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="wall-time budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="steps of the per-iteration (plain) path timed for the speedup; 0 skips")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the initial conditions are independent and a "
              f"multi-GPU run would only shard them; --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2301_03989_amd import build, pcprop, workloads
    build.ensure_built()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.calibrate_copy:
        # a plain copy of known size: the reference that scales FETCH_SIZE / WRITE_SIZE
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}), flush=True)
        return

    w = workloads.WORKLOADS[args.workload]()
    n_ic = w.n_ic
    ic_segments = sum(g.n_ic * g.segments for g in w.groups)
    ctx = pcprop.Context(0)
    ctx.set_timing(True)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch)
    init = "kepler" if w.init == 0 else "cold"
    precision = args.precision or ("fp32-fp64" if w.precision == 1 else "fp64")
    states = torch.empty((n_ic, 6), dtype=torch.float64, device="cuda")

    if args.autotune:
        chosen = ctx.autotune(ics, groups, model)
        print(f"bench: autotuner chose tile_pairs={chosen}", flush=True)

    def step():
        return ctx.propagate_batched(ics, groups, model, init=init, tile_pairs=args.tile_pairs, out=states,
                                     graph=args.graph, precision=precision, switch_tol=args.switch_tol)

    print(f"bench: {w.name}: {n_ic} ICs, {ic_segments} IC-segments, warmup {args.warmup}", flush=True)
    for _ in range(args.warmup):
        r = step()
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    kernel_ms = []
    t_start.record()
    for _ in range(args.steps):
        r = step()
        kernel_ms.append(ctx.last_kernel_ms())
    t_end.record()
    torch.cuda.synchronize()
    ms_per_step = t_start.elapsed_time(t_end) / args.steps
    print(f"bench: {args.steps} steps, {ms_per_step:.3f} ms/step, kernel {np.mean(kernel_ms):.3f} ms", flush=True)
    status = r["status"]
    iters = r["iters"].cpu().numpy()
    gpu_states = r["states"].cpu().numpy()

    fp64_ref = None
    if precision != "fp64":
        # the same propagation with FP64 sweeps only, for the mixed-precision speedup
        f64_states = torch.empty_like(states)
        ctx.propagate_batched(ics, groups, model, init=init, out=f64_states)
        torch.cuda.synchronize()
        q0 = torch.cuda.Event(enable_timing=True)
        q1 = torch.cuda.Event(enable_timing=True)
        nq = max(1, min(args.steps, 5))
        q0.record()
        for _ in range(nq):
            rq = ctx.propagate_batched(ics, groups, model, init=init, out=f64_states)
        q1.record()
        torch.cuda.synchronize()
        f64_ms = q0.elapsed_time(q1) / nq
        it64 = rq["iters"].cpu().numpy()
        fp64_ref = {"precision": "fp64", "ms_per_step": round(f64_ms, 4), "steps": nq,
                    "speedup_mixed_vs_fp64": round(f64_ms / ms_per_step, 3),
                    "mean_iterations_per_segment_fp64": round(float(it64[it64 > 0].mean()), 3),
                    "max_rel_diff_vs_fp64": float(rel_err(gpu_states, rq["states"].cpu().numpy()).max())}
        print(f"bench: all-FP64 {f64_ms:.3f} ms/step, mixed-precision speedup {f64_ms / ms_per_step:.2f}x",
              flush=True)

    plain = None
    if args.plain_steps > 0 and precision == "fp64":
        # the same propagation with per-iteration kernels and a host loop (plain GPU path)
        plain_states = torch.empty_like(states)
        ctx.propagate_batched(ics, groups, model, init=init, path="plain", out=plain_states)
        torch.cuda.synchronize()
        p0 = torch.cuda.Event(enable_timing=True)
        p1 = torch.cuda.Event(enable_timing=True)
        p0.record()
        for _ in range(args.plain_steps):
            rp = ctx.propagate_batched(ics, groups, model, init=init, path="plain", out=plain_states)
        p1.record()
        torch.cuda.synchronize()
        plain_ms = p0.elapsed_time(p1) / args.plain_steps
        plain = {"path": "plain", "ms_per_step": round(plain_ms, 4), "steps": args.plain_steps,
                 "speedup_batched_vs_plain": round(plain_ms / ms_per_step, 3),
                 "max_rel_diff_vs_batched": float(rel_err(rp["states"].cpu().numpy(), gpu_states).max())}
        print(f"bench: plain path {plain_ms:.3f} ms/step, batched speedup {plain_ms / ms_per_step:.2f}x",
              flush=True)

    # accuracy gate against the FP64 oracle on an evenly spaced sample
    idx = np.unique(np.linspace(0, n_ic - 1, min(args.check_ics, n_ic)).astype(np.int64))
    ref, ref_iters, _ = oracle_states(w, idx)
    errs = rel_err(gpu_states[idx], ref)
    max_err = float(errs.max())
    iter_diff = int(np.abs(iters[idx] - ref_iters).max())
    valid = (max_err <= 1e-10) and status == 0
    print(f"bench: max rel err vs oracle on {idx.size} ICs: {max_err:.3e} (iteration diff {iter_diff})",
          flush=True)

    flops = algorithmic_flops(w, iters)
    kms = float(np.mean(kernel_ms))
    achieved = flops / (kms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
                "kernel": "pc_fused_kernel", "kernel_ms": round(kms, 4),
                "flops_per_launch": flops}

    cpu = None
    if not args.no_cpu_baseline:
        # oracle rate on a bounded sample of the same workload, all host threads
        rng = np.random.default_rng(0)
        probe = np.sort(rng.choice(n_ic, size=min(16, n_ic), replace=False))
        t0 = time.perf_counter()
        oracle_states(w, probe)
        per_ic = (time.perf_counter() - t0) / probe.size
        k = int(min(n_ic, max(probe.size, args.cpu_seconds / max(per_ic, 1e-9))))
        sample = np.sort(rng.choice(n_ic, size=k, replace=False))
        t0 = time.perf_counter()
        _, _, threads = oracle_states(w, sample)
        dt = time.perf_counter() - t0
        sample_segments = sum(
            int(((sample >= g.ic_offset) & (sample < g.ic_offset + g.n_ic)).sum()) * g.segments
            for g in w.groups)
        cpu = {"value": round(sample_segments / dt, 3), "unit": "IC-segment propagations/s",
               "cores": int(threads), "kind": "oracle",
               "sample": f"{k} of {n_ic} ICs (all segments), {dt:.1f} s wall on {threads} threads"}
        print(f"bench: oracle {cpu['value']} IC-segments/s on {threads} threads", flush=True)

    line = {
        "metric": METRIC,
        "value": round(ic_segments / (ms_per_step * 1e-3), 3) if valid else None,
        "unit": "IC-segment propagations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_ic": n_ic, "segments": [g.segments for g in w.groups][:4],
                   "nodes": sorted({g.nodes for g in w.groups}), "tol": w.groups[0].tol,
                   "perturbers": int(w.pert.shape[0]), "path": "fused", "graph": bool(args.graph), "precision": precision,
                   "tile_pairs": args.tile_pairs or "tuned"},
        "accuracy": {"max_rel_err_vs_oracle": max_err, "p99_rel_err_vs_oracle": float(np.percentile(errs, 99)),
                     "median_rel_err_vs_oracle": float(np.median(errs)), "checked_ics": int(idx.size),
                     "max_iteration_diff": iter_diff, "status": int(status),
                     "mean_iterations_per_segment": round(float(iters[iters > 0].mean()), 3)},
        "segment_iterations_per_s": round(float(np.where(iters > 0, iters, 0).sum()) /
                                          (ms_per_step * 1e-3), 1),
        "vs_plain": plain,
        "vs_fp64": fp64_ref,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
