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
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    """sha256 over the HIP sources and the ABI header, in a fixed order: the identity of
    the kernels a counter summary was taken on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2301_03989_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "include", "pcprop.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of ``kernel`` on ``workload`` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size), or None when there is
    none or the kernels have changed since it was taken."""
    path = os.path.join(PROFILES, f"{kernel}.{workload}.traffic.md")
    if not os.path.exists(path):
        return None, "no counter summary"
    vals = {}
    with open(path) as fh:
        for line in fh:
            m = line.strip().lstrip("-* ").split(":", 1)
            if len(m) == 2:
                vals[m[0].strip().strip("`")] = m[1].strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash():
        return None, "kernels changed since the counters were taken"
    try:
        return float(vals["traffic_bytes_per_launch"]), path
    except (KeyError, ValueError):
        return None, "malformed counter summary"


def algorithmic_flops(w, iters):
    """Algorithmic FP64 work of the Picard iterations actually run: per IC, segment and
    iteration, the folded fit/integrate/evaluate product (6 columns x 2 N^2) plus the
    dynamics at N nodes (20 flops per body interaction, Sun + P perturbers, and 3 for
    the precomputed indirect term; with the Einstein-Infeld-Hoffmann model 96 per body:
    offset, distance powers, potential, the projections and products of its terms and
    their accumulation, and 15 per point for v^2, the term in the potential and the
    indirect term)."""
    P = w.pert.shape[0]
    eih = getattr(w, "inv_c2", 0.0) > 0.0
    total = 0.0
    for g in w.groups:
        it = iters[g.ic_offset:g.ic_offset + g.n_ic, :g.segments]
        it = np.where(it > 0, it, 0).astype(np.float64)
        N = g.nodes
        force = (96.0 * (P + 1) + 15.0) if eih else (20.0 * (P + 1) + 3.0)
        per_iter = 12.0 * N * N + force * N
        total += per_iter * it.sum()
    return total


def rel_err(a, b):
    er = np.linalg.norm(a[:, :3] - b[:, :3], axis=1) / np.linalg.norm(b[:, :3], axis=1)
    ev = np.linalg.norm(a[:, 3:] - b[:, 3:], axis=1) / np.linalg.norm(b[:, 3:], axis=1)
    return np.maximum(er, ev)


def oracle_states(w, idx):
    import oracle
    model = oracle.Model(w.mu_sun, w.pert, w.epoch, inv_c2=w.inv_c2)
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


def adjoint_flops(w, iters, adj_iters, resolve=True):
    """Algorithmic FP64 work of one adjoint call: the forward re-solve of every segment
    (as algorithmic_flops; not when the forward's node states are read instead) plus, per
    adjoint sweep, the transposed product (6 columns x 2 N^2) and the Hessian-vector
    products H w_v at N nodes (30 flops per body: offset, distance powers, the projection
    d (d.w) and the accumulation) and the 12 flops that form mu_new."""
    P = w.pert.shape[0]
    total = algorithmic_flops(w, iters) if resolve else 0.0
    for g in w.groups:
        it = adj_iters[g.ic_offset:g.ic_offset + g.n_ic, :g.segments]
        it = np.where(it > 0, it, 0).astype(np.float64)
        N = g.nodes
        total += (12.0 * N * N + (30.0 * (P + 1) + 12.0) * N) * it.sum()
    return total


def run_adjoint(args):
    """Forward propagation with segment checkpoints, then the adjoint of the final state
    (seed: a fixed random dL/dy_final per IC); one step = both calls."""
    import torch

    import oracle
    from paper_2301_03989_amd import pcprop, workloads
    w = workloads.WORKLOADS[args.workload or "nbody-venus-16384-256d"]()
    n_ic = w.n_ic
    ic_segments = sum(g.n_ic * g.segments for g in w.groups)
    ctx = pcprop.Context(0)
    ctx.set_timing(True)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    gbar_np = np.random.default_rng(7).standard_normal((n_ic, 6))
    gbar = torch.tensor(gbar_np, dtype=torch.float64, device="cuda")

    def step():
        f = ctx.propagate_batched(ics, groups, model, want_bounds=True, want_nodes=args.adjoint_nodes,
                                  tile_pairs=2048)
        fwd_ms = ctx.last_kernel_ms()
        grad, adj_it, st = ctx.adjoint(f["bounds"], gbar, groups, model,
                                       fwd_nodes=f["nodes"] if args.adjoint_nodes else None)
        return f, grad, adj_it, st, fwd_ms, ctx.last_kernel_ms()

    print(f"bench: adjoint of {w.name}: {n_ic} ICs, {ic_segments} IC-segments", flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fwd_ms, adj_ms = [], []
    e0.record()
    for _ in range(args.steps):
        f, grad, adj_it, st, fm, am = step()
        fwd_ms.append(fm)
        adj_ms.append(am)
    e1.record()
    torch.cuda.synchronize()
    ms_per_step = e0.elapsed_time(e1) / args.steps
    iters = f["iters"].cpu().numpy()
    ait = adj_it.cpu().numpy()
    g_np = grad.cpu().numpy()
    print(f"bench: {ms_per_step:.3f} ms/step (forward kernel {np.mean(fwd_ms):.3f} ms, adjoint kernel "
          f"{np.mean(adj_ms):.3f} ms)", flush=True)

    g0 = w.groups[0]
    idx = np.unique(np.linspace(0, n_ic - 1, max(1, min(args.check_ics, 4))).astype(np.int64))
    om = oracle.Model(w.mu_sun, w.pert, w.epoch, inv_c2=w.inv_c2)
    ref = oracle.adjoint(w.ics[idx], g0.t0, g0.tf, g0.nodes, g0.segments, g0.tol, om, gbar_np[idx])
    gerr = np.linalg.norm(g_np[idx] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    valid = bool(gerr.max() <= 1e-8 and st == 0 and f["status"] == 0)
    print(f"bench: max rel gradient err vs oracle on {idx.size} ICs: {gerr.max():.3e}", flush=True)

    flops = adjoint_flops(w, iters, ait, resolve=not args.adjoint_nodes)
    kms = float(np.mean(adj_ms))
    achieved = flops / (kms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None,
                "traffic_source": "not collected for the adjoint kernel",
                "kernel": "pc_adjoint_kernel", "kernel_ms": round(kms, 4), "flops_per_launch": flops}
    cpu = None
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(0)
        t0 = time.perf_counter()
        probe = np.sort(rng.choice(n_ic, size=1, replace=False))
        oracle.adjoint(w.ics[probe], g0.t0, g0.tf, g0.nodes, g0.segments, g0.tol, om, gbar_np[probe])
        per_ic = time.perf_counter() - t0
        k = int(min(n_ic, max(1, args.cpu_seconds / max(per_ic, 1e-9))))
        sample = np.sort(rng.choice(n_ic, size=k, replace=False))
        t0 = time.perf_counter()
        oracle.adjoint(w.ics[sample], g0.t0, g0.tf, g0.nodes, g0.segments, g0.tol, om, gbar_np[sample])
        dt = time.perf_counter() - t0
        threads = oracle.propagate.last_threads
        cpu = {"value": round(k * g0.segments / dt, 3), "unit": "IC-segment gradients/s", "cores": int(threads),
               "kind": "oracle",
               "sample": f"{k} of {n_ic} ICs, forward + dense implicit-derivative solve per segment, "
                         f"{dt:.1f} s wall (propagation on {threads} threads, solves on numpy's BLAS)"}
    line = {
        "metric": METRIC + " (forward + adjoint)",
        "value": round(ic_segments / (ms_per_step * 1e-3), 3) if valid else None,
        "unit": "IC-segment gradients/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n_ic": n_ic, "segments": g0.segments, "nodes": g0.nodes, "tol": g0.tol,
                   "perturbers": int(w.pert.shape[0]), "seed": "random dL/dy_final",
                   "checkpoints": "node states" if args.adjoint_nodes else "segment bounds"},
        "accuracy": {"max_rel_grad_err_vs_oracle": float(gerr.max()), "checked_ics": int(idx.size),
                     "status_forward": int(f["status"]), "status_adjoint": int(st),
                     "mean_adjoint_sweeps_per_segment": round(float(ait[ait > 0].mean()), 3),
                     "mean_iterations_per_segment": round(float(iters[iters > 0].mean()), 3)},
        "forward_kernel_ms": round(float(np.mean(fwd_ms)), 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None, help="default nbody-venus-4096")
    ap.add_argument("--tile-pairs", type=int, default=0)
    ap.add_argument("--job-list", type=int, default=0,
                    help="ICs per job in column blocks (0 automatic, 1 off, 2/4/8)")
    ap.add_argument("--graph", action="store_true", help="replay the call as a captured HIP graph")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32-fp64"],
                    help="sweep arithmetic (default: the workload's)")
    ap.add_argument("--switch-tol", type=float, default=0.0, help="FP32 -> FP64 switch (0: library default)")
    ap.add_argument("--autotune", action="store_true", help="pick the job shape with the autotuner first")
    ap.add_argument("--check-ics", type=int, default=64, help="ICs checked against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="wall-time budget of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-streams", type=int, default=1,
                    help="streams of the plain path's outer level (one host thread each)")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="steps of the per-iteration (plain) path timed for the speedup; 0 skips")
    ap.add_argument("--adjoint-nodes", action="store_true",
                    help="with --adjoint: keep the forward's node states and read them in the adjoint "
                         "instead of re-solving each segment from its checkpoint")
    ap.add_argument("--adjoint", action="store_true",
                    help="time forward (with checkpoints) + adjoint of the final state; default "
                         "workload then nbody-venus-16384-256d")
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

    if args.adjoint:
        run_adjoint(args)
        return

    w = workloads.WORKLOADS[args.workload or "nbody-venus-4096"]()
    n_ic = w.n_ic
    ic_segments = sum(g.n_ic * g.segments for g in w.groups)
    ctx = pcprop.Context(0)
    ctx.set_timing(True)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    init = "kepler" if w.init == 0 else "cold"
    precision = args.precision or ("fp32-fp64" if w.precision == 1 else "fp64")
    states = torch.empty((n_ic, 6), dtype=torch.float64, device="cuda")

    if args.autotune:
        chosen = ctx.autotune(ics, groups, model)
        print(f"bench: autotuner chose tile_pairs={chosen}", flush=True)

    def step():
        return ctx.propagate_batched(ics, groups, model, init=init, tile_pairs=args.tile_pairs, out=states,
                                     graph=args.graph, precision=precision, switch_tol=args.switch_tol,
                                     job_list=args.job_list)

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
        pkw = dict(init=init, path="plain", out=plain_states, streams=args.plain_streams)
        ctx.propagate_batched(ics, groups, model, **pkw)
        torch.cuda.synchronize()
        p0 = torch.cuda.Event(enable_timing=True)
        p1 = torch.cuda.Event(enable_timing=True)
        p0.record()
        for _ in range(args.plain_steps):
            rp = ctx.propagate_batched(ics, groups, model, **pkw)
        p1.record()
        torch.cuda.synchronize()
        plain_ms = p0.elapsed_time(p1) / args.plain_steps
        plain = {"path": "plain", "streams": args.plain_streams, "ms_per_step": round(plain_ms, 4),
                 "steps": args.plain_steps,
                 "speedup_batched_vs_plain": round(plain_ms / ms_per_step, 3),
                 "max_rel_diff_vs_batched": float(rel_err(rp["states"].cpu().numpy(), gpu_states).max())}
        print(f"bench: plain path ({args.plain_streams} stream(s)) {plain_ms:.3f} ms/step, "
              f"batched speedup {plain_ms / ms_per_step:.2f}x", flush=True)

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
    traffic, traffic_src = measured_traffic("pc_fused_kernel", w.name) if precision == "fp64" else \
        (None, "counters taken on the FP64 path only")
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "traffic_source": os.path.relpath(traffic_src, ROOT) if traffic is not None else traffic_src,
                "kernel": "pc_fused_kernel", "kernel_ms": round(kms, 4),
                "flops_per_launch": flops}
    if precision != "fp64":
        # the FP32 -> FP64 schedule does most of its work on FP32 matrix cores and skips the
        # force in its increment sweeps: its FP64 flop count over the FP64 peak is a
        # speed figure, not a pipe utilisation
        roofline["basis"] = "FP64-equivalent flops of the FP64 schedule; not a utilisation"

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
        sample_segments = sum(
            int(((sample >= g.ic_offset) & (sample < g.ic_offset + g.n_ic)).sum()) * g.segments
            for g in w.groups)
        # repeat the sample until the budget is spent (a whole small workload runs in seconds)
        reps, dt = 0, 0.0
        while reps == 0 or dt < args.cpu_seconds:
            t0 = time.perf_counter()
            _, _, threads = oracle_states(w, sample)
            dt += time.perf_counter() - t0
            reps += 1
        cpu = {"value": round(reps * sample_segments / dt, 3), "unit": "IC-segment propagations/s",
               "cores": int(threads), "kind": "oracle",
               "sample": f"{k} of {n_ic} ICs (all segments), {reps} pass(es), {dt:.1f} s wall on {threads} threads"}
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
        "config": {"workload": w.name, "n_ic": n_ic, "segments": sorted({g.segments for g in w.groups}),
                   "nodes": sorted({g.nodes for g in w.groups}), "tol": w.groups[0].tol,
                   "perturbers": int(w.pert.shape[0]), "path": "fused", "graph": bool(args.graph), "precision": precision,
                   "tile_pairs": args.tile_pairs or "tuned", "job_list": args.job_list or "auto"},
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
