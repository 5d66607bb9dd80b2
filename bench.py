#!/usr/bin/env python3
"""Benchmark of batched Picard-Chebyshev propagation on one MI355X.

One step = one full propagation of the workload (ephemeris table, warm starts, all
Picard iterations of all segments, convergence tests, chaining, end states and
segment-boundary states) with the initial conditions already resident in HBM.  Default
workload: the uneven two-level batch, 65536 ICs in 15 groups (64, 128 and 256 CGL nodes
x 8 to 40 segments of pi/4 TU, eccentricities up to 0.6), Sun + 8 planets, FP64,
tol 1e-12, in one persistent launch replayed from a captured HIP graph, job shape and
job lengths from the autotuner.

Prints one JSON line: IC-segment propagations/s (the workload's ICs x segments per
second), valid when a stratified sample checked against the FP64 CPU oracle at every
segment boundary is within 1e-10 relative (or within the trajectory's own conditioning,
measured on the oracle, for the rare ICs through a planet's Hill sphere), with the same
batch on the per-iteration (plain) path on 1 and 10 streams, the mixed-precision
sub-record on the 262144-IC N-body ensemble, the roofline of the propagation kernel
against the datasheet and on-chip ceilings, and the oracle's own rate on the host cores
(all cores and one).
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


def adjoint_flops(w, iters, adj_iters, resolve=True):
    """Algorithmic FP64 work of one adjoint call: the forward re-solve of every segment
    (as algorithmic_flops; not when the forward's node states are read instead) plus, per
    adjoint sweep, the transposed product (6 columns x 2 N^2) and the Hessian-vector
    products H w_v at N nodes (30 flops per body: offset, distance powers, the projection
    d (d.w) and the accumulation) and the 12 flops that form mu_new.  With the
    Einstein-Infeld-Hoffmann model the products are (da/dr)^T w_v and (da/dv)^T w_v: 190
    flops per body (offset and distance powers, the potential and Newtonian sums, the
    scalar products and factors of the relativistic bracket, its derivative in r, and the
    two accumulations) and 34 per point (v^2, u.N and the combination of the sums)."""
    P = w.pert.shape[0]
    eih = getattr(w, "inv_c2", 0.0) > 0.0
    total = algorithmic_flops(w, iters) if resolve else 0.0
    for g in w.groups:
        it = adj_iters[g.ic_offset:g.ic_offset + g.n_ic, :g.segments]
        it = np.where(it > 0, it, 0).astype(np.float64)
        N = g.nodes
        vjp = (190.0 * (P + 1) + 34.0) if eih else 30.0 * (P + 1)
        total += (12.0 * N * N + (vjp + 12.0) * N) * it.sum()
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
    idx = np.unique(np.linspace(0, n_ic - 1, max(1, min(args.check_ics or 8, n_ic))).astype(np.int64))
    om = oracle.Model(w.mu_sun, w.pert, w.epoch, inv_c2=w.inv_c2)
    ref = oracle.adjoint(w.ics[idx], g0.t0, g0.tf, g0.nodes, g0.segments, g0.tol, om, gbar_np[idx])
    gerr = np.linalg.norm(g_np[idx] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    valid = bool(gerr.max() <= 1e-8 and st == 0 and f["status"] == 0)
    print(f"bench: max rel gradient err vs oracle on {idx.size} ICs: {gerr.max():.3e}", flush=True)

    flops = adjoint_flops(w, iters, ait, resolve=not args.adjoint_nodes)
    kms = float(np.mean(adj_ms))
    achieved = flops / (kms * 1e-3) / 1e12
    traffic, traffic_src = measured_traffic("pc_adjoint_kernel", w.name + ("-nodes" if args.adjoint_nodes else ""))
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "traffic_source": traffic_src,
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


def cpu_model():
    """The host CPU's model name and the cores this process may run on."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    return name, affinity


def stratified_sample(w, per_group, seed):
    """A seeded sample of ``per_group`` ICs from every group of ``w`` (sorted indices)."""
    rng = np.random.default_rng(seed)
    return np.concatenate([g.ic_offset + np.sort(rng.choice(g.n_ic, size=min(per_group, g.n_ic), replace=False))
                           for g in w.groups])


def boundary_errors(gpu_bounds, ref_bounds):
    """Per-IC max of rel_err over the segment boundaries the reference uses (final state
    included); ref rows that are all zero (past a group's segments) are skipped."""
    n, k, _ = ref_bounds.shape
    used = np.any(ref_bounds != 0.0, axis=2)
    ref = np.where(used.reshape(-1, 1), ref_bounds.reshape(-1, 6), 1.0)
    e = rel_err(gpu_bounds.reshape(-1, 6), ref).reshape(n, k)
    return np.where(used, e, 0.0).max(axis=1)


def oracle_run(w, idx, threads=0, order=1):
    """Oracle states, iterations and segment-boundary states of the ICs ``idx`` of ``w``,
    and the wall time and thread count it took (``order`` 2: the second-order form)."""
    import oracle
    model = oracle.Model(w.mu_sun, w.pert, w.epoch, inv_c2=w.inv_c2)
    S_max = max(g.segments for g in w.groups)
    states = np.zeros((idx.size, 6))
    iters = np.zeros((idx.size, S_max), dtype=np.int32)
    bounds = np.zeros((idx.size, S_max + 1, 6))
    t0 = time.perf_counter()
    used = 1
    for g in w.groups:
        sel = np.nonzero((idx >= g.ic_offset) & (idx < g.ic_offset + g.n_ic))[0]
        if sel.size:
            s, it, b = oracle.propagate(w.ics[idx[sel]], g.t0, g.tf, g.nodes, g.segments, g.tol, model,
                                        init=w.init, want_bounds=True, threads=threads, order=order)
            states[sel], iters[sel, :g.segments], bounds[sel, :g.segments + 1] = s, it, b
            used = max(used, oracle.propagate.last_threads)
    return states, iters, bounds, time.perf_counter() - t0, used


def ic_segments(w, idx):
    return int(sum(((idx >= g.ic_offset) & (idx < g.ic_offset + g.n_ic)).sum() * g.segments for g in w.groups))


def sensitivity(w, idx, reps=4, rel=1e-14):
    """The oracle's own spread at the segment boundaries under (1 +- rel) scalings of the
    ICs ``idx`` (random signs, ``reps`` draws): the conditioning of those trajectories."""
    rng = np.random.default_rng(0)
    _, _, base, _, _ = oracle_run(w, idx)
    worst = np.zeros(idx.size)
    from paper_2301_03989_amd.workloads import Workload
    for _ in range(reps):
        ics = w.ics.copy()
        ics[idx] = w.ics[idx] * (1.0 + rel * rng.choice([-1.0, 1.0], size=(idx.size, 6)))
        wp = Workload(w.name, ics, w.groups, w.pert, w.init, w.precision, w.mu_sun, w.epoch, w.inv_c2)
        _, _, b, _, _ = oracle_run(wp, idx)
        worst = np.maximum(worst, boundary_errors(b, base))
    return worst


def accuracy_gate(w, bounds, iters, idx, ref_bounds, ref_iters):
    """Per-IC error at every segment boundary against the oracle.  An IC passes at
    <= 1e-10; an IC above it passes only if the oracle itself moves by at least 1/30 of its
    error under 1e-14 changes of the IC (a trajectory through a planet's Hill sphere,
    conditioning-limited), and such ICs must be rare (<= 1 % of the sample)."""
    err = boundary_errors(bounds[idx], ref_bounds)
    bad = np.nonzero(err > 1e-10)[0]
    kappa = sensitivity(w, idx[bad]) if bad.size else np.zeros(0)
    ok = bool(np.all(err[bad] <= 30.0 * kappa) and bad.size <= max(1, idx.size // 100))
    good = err <= 1e-10
    dit = np.abs(iters[idx][good] - ref_iters[good])
    return ok, err, bad, kappa, int(dit.max()) if dit.size else 0


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None, help="default uneven-batch-65536")
    ap.add_argument("--tile-pairs", type=int, default=0)
    ap.add_argument("--job-list", type=int, default=0,
                    help="ICs per job in column blocks (0 automatic, 1 off, 2/4/8)")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a captured graph")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32-fp64"],
                    help="sweep arithmetic (default: the workload's)")
    ap.add_argument("--switch-tol", type=float, default=0.0, help="FP32 -> FP64 switch (0: library default)")
    ap.add_argument("--no-autotune", action="store_true", help="use the untuned job shape and job lengths")
    ap.add_argument("--check-per-group", type=int, default=128,
                    help="ICs per group checked against the oracle (stratified sample)")
    ap.add_argument("--check-ics", type=int, default=0,
                    help="check an evenly spaced sample of this many ICs instead")
    ap.add_argument("--cpu-1t-per-group", type=int, default=6,
                    help="ICs per group of the oracle's one-thread timing sample (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="--adjoint: about this much wall time of the oracle's adjoint for the CPU baseline")
    ap.add_argument("--plain-streams", default="1,10",
                    help="stream counts of the plain path's outer level to time ('' skips the plain path)")
    ap.add_argument("--plain-steps", type=int, default=2,
                    help="steps of the per-iteration (plain) path timed for the speedup")
    ap.add_argument("--mixed-workload", default="nbody-venus-262144-fp32-fp64",
                    help="workload of the mixed-precision sub-record ('' skips it)")
    ap.add_argument("--mixed-steps", type=int, default=3)
    ap.add_argument("--mixed-check-ics", type=int, default=1024)
    ap.add_argument("--no-ceilings", action="store_true", help="skip the on-chip ceiling loops")
    ap.add_argument("--second-order-workload", default="uneven-batch-65536",
                    help="workload of the second-order sub-record ('' skips it)")
    ap.add_argument("--second-order-steps", type=int, default=5)
    ap.add_argument("--flyby-hill", type=float, default=5.0,
                    help="threshold (Hill radii) of the flyby-isolation sub-record on the group-max plain "
                         "path (0 skips it)")
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

    w = workloads.WORKLOADS[args.workload or "uneven-batch-65536"]()
    n_ic = w.n_ic
    S_max = max(g.segments for g in w.groups)
    n_icseg = sum(g.n_ic * g.segments for g in w.groups)
    ctx = pcprop.Context(0)

    ceilings = None
    if not args.no_ceilings:
        mf, fm, cp = ctx.measure_ceilings(1024)
        ceilings = {"fp64_mfma_tflops": round(mf, 2), "fp64_fma_tflops": round(fm, 2), "copy_gbs": round(cp, 1),
                    "how": "pc_measure_ceilings: independent v_mfma_f64_16x16x4 chains (2 waves per SIMD), "
                           "independent FP64 FMA chains (8 waves per SIMD), a 512 MiB device copy; best of 5 "
                           "after about 50 ms of untimed runs"}
        print(f"bench: on-chip ceilings: FP64 MFMA {mf:.1f} TFLOP/s, FP64 FMA {fm:.1f} TFLOP/s, copy {cp:.0f} GB/s",
              flush=True)

    ctx.set_timing(True)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    init = "kepler" if w.init == 0 else "cold"
    precision = args.precision or ("fp32-fp64" if w.precision == 1 else "fp64")
    states = torch.empty((n_ic, 6), dtype=torch.float64, device="cuda")
    iters_t = torch.zeros((n_ic, S_max), dtype=torch.int32, device="cuda")
    bounds_t = torch.empty((n_ic, S_max + 1, 6), dtype=torch.float64, device="cuda")
    graph = not args.no_graph

    tuned = None
    if not args.no_autotune and precision == "fp64" and args.tile_pairs == 0 and args.job_list == 0 \
            and w.inv_c2 == 0.0:
        t0 = time.perf_counter()
        chosen = ctx.autotune(ics, groups, model)
        nps = sorted({max(16, 1 << (g.nodes - 1).bit_length()) for g in w.groups})
        tuned = {"tile_pairs": chosen, "job_list": {str(np_): ctx.job_list(np_) or "rule" for np_ in nps},
                 "seconds": round(time.perf_counter() - t0, 2)}
        print(f"bench: autotuner: {tuned}", flush=True)

    def step():
        return ctx.propagate_batched(ics, groups, model, init=init, tile_pairs=args.tile_pairs, out=states,
                                     iters_out=iters_t, bounds_out=bounds_t, graph=graph, precision=precision,
                                     switch_tol=args.switch_tol, job_list=args.job_list)

    print(f"bench: {w.name}: {n_ic} ICs, {n_icseg} IC-segments, warmup {args.warmup}", flush=True)
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
    print(f"bench: {args.steps} steps, {ms_per_step:.3f} ms/step, kernel {np.mean(kernel_ms):.3f} ms"
          f"{' (graph: whole graph)' if graph else ''}", flush=True)
    status = r["status"]
    iters = iters_t.cpu().numpy()
    gpu_states = states.cpu().numpy()
    gpu_bounds = bounds_t.cpu().numpy()

    plain = []
    streams_list = [int(x) for x in args.plain_streams.split(",") if x.strip()] if precision == "fp64" else []
    for ns in streams_list:
        # the same propagation with per-iteration kernels and a host loop (plain GPU path),
        # its groups on ns streams driven from this thread
        plain_states = torch.empty_like(states)
        pkw = dict(init=init, path="plain", out=plain_states, streams=min(ns, len(groups)))
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
        plain.append({"path": "plain", "streams": pkw["streams"], "ms_per_step": round(plain_ms, 4),
                      "steps": args.plain_steps, "status": int(rp["status"]),
                      "speedup_batched_vs_plain": round(plain_ms / ms_per_step, 3),
                      "max_rel_diff_vs_batched": float(rel_err(rp["states"].cpu().numpy(), gpu_states).max())})
        print(f"bench: plain path ({pkw['streams']} stream(s)) {plain_ms:.3f} ms/step, "
              f"batched speedup {plain_ms / ms_per_step:.2f}x", flush=True)

    # accuracy gate against the FP64 oracle: a stratified sample (every group), at every
    # segment boundary; the oracle's wall time on it is also the all-core CPU baseline
    if args.check_ics:
        idx = np.unique(np.linspace(0, n_ic - 1, min(args.check_ics, n_ic)).astype(np.int64))
    else:
        idx = stratified_sample(w, args.check_per_group, seed=2024)
    ref_states, ref_iters, ref_bounds, ref_wall, ref_threads = oracle_run(w, idx)
    ok, errs, bad, kappa, iter_diff = accuracy_gate(w, gpu_bounds, iters, idx, ref_bounds, ref_iters)
    max_err = float(errs.max())
    valid = ok and status == 0
    print(f"bench: oracle check on {idx.size} ICs: max rel err {max_err:.3e} at the segment boundaries, "
          f"{bad.size} conditioning-limited (their oracle sensitivity {np.round(kappa, 14).tolist()}), "
          f"iteration diff {iter_diff}; gate {'passed' if valid else 'FAILED'}", flush=True)
    per_group = {}
    for g in w.groups:
        sel = (idx >= g.ic_offset) & (idx < g.ic_offset + g.n_ic)
        if sel.any():
            per_group[f"N{g.nodes}-S{g.segments}"] = float(errs[sel].max())

    flops = algorithmic_flops(w, iters)
    kms = float(np.mean(kernel_ms))
    achieved = flops / (kms * 1e-3) / 1e12
    traffic, traffic_src = measured_traffic("pc_fused_kernel", w.name) if precision == "fp64" else \
        (None, "counters taken on the FP64 path only")
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "traffic_source": os.path.relpath(traffic_src, ROOT) if traffic is not None else traffic_src,
                "kernel": "pc_fused_kernel", "kernel_ms": round(kms, 4),
                "kernel_ms_basis": "HIP events around the replayed graph (table copy, ephemeris kernel, "
                                   "propagation kernel, status copy)" if graph else
                                  "HIP events around the propagation kernel",
                "flops_per_launch": flops,
                "flops_basis": "sum over ICs, segments and iterations run of 12 N^2 + (20 (P+1) + 3) N"}
    if ceilings:
        roofline["on_chip"] = dict(ceilings)
        roofline["frac_of_on_chip_mfma"] = round(achieved / ceilings["fp64_mfma_tflops"], 4)
    if precision != "fp64":
        # the FP32 -> FP64 schedule does most of its work on FP32 matrix cores and skips the
        # force in its increment sweeps: its FP64 flop count over the FP64 peak is a
        # speed figure, not a pipe utilisation
        roofline["basis"] = "FP64-equivalent flops of the FP64 schedule; not a utilisation"

    mixed = None
    if args.mixed_workload and precision == "fp64":
        mixed = run_mixed(args, workloads.WORKLOADS[args.mixed_workload](), pcprop)

    second = None
    if args.second_order_workload and precision == "fp64":
        second = run_second_order(args, workloads.WORKLOADS[args.second_order_workload](), pcprop)

    flyby = None
    if args.flyby_hill > 0 and precision == "fp64" and w.inv_c2 == 0.0:
        flyby = run_flyby(args, ctx, w, pcprop)

    cpu = None
    if not args.no_cpu_baseline:
        name, affinity = cpu_model()
        seg = ic_segments(w, idx)
        cpu = {"value": round(seg / ref_wall, 3), "unit": "IC-segment propagations/s", "cores": int(ref_threads),
               "kind": "oracle",
               "sample": f"the accuracy sample: {idx.size} of {n_ic} ICs ({args.check_per_group} per group, "
                         f"all segments, {seg} IC-segments), {ref_wall:.1f} s wall on {ref_threads} threads; "
                         f"ICs are independent, so the rate extrapolates linearly",
               "cpu": name, "affinity_cores": affinity}
        if args.cpu_1t_per_group > 0:
            idx1 = stratified_sample(w, args.cpu_1t_per_group, seed=7)
            _, _, _, wall1, th1 = oracle_run(w, idx1, threads=1)
            seg1 = ic_segments(w, idx1)
            cpu["one_core"] = {"value": round(seg1 / wall1, 3), "cores": int(th1),
                               "sample": f"{idx1.size} ICs ({args.cpu_1t_per_group} per group), {seg1} "
                                         f"IC-segments, {wall1:.1f} s wall"}
        print(f"bench: oracle {cpu['value']} IC-segments/s on {ref_threads} threads"
              + (f", {cpu['one_core']['value']} on 1" if "one_core" in cpu else "") + f" ({name})", flush=True)

    line = {
        "metric": METRIC,
        "value": round(n_icseg / (ms_per_step * 1e-3), 3) if valid else None,
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
        "config": {"workload": w.name, "n_ic": n_ic, "groups": len(w.groups),
                   "segments": sorted({g.segments for g in w.groups}),
                   "nodes": sorted({g.nodes for g in w.groups}), "tol": sorted({g.tol for g in w.groups}),
                   "perturbers": int(w.pert.shape[0]), "path": "fused", "graph": graph, "precision": precision,
                   "tile_pairs": args.tile_pairs or (tuned["tile_pairs"] if tuned else "rule"),
                   "job_list": args.job_list or (tuned["job_list"] if tuned else "rule"),
                   "autotuned": tuned is not None},
        "accuracy": {"max_rel_err_vs_oracle": max_err, "p99_rel_err_vs_oracle": float(np.percentile(errs, 99)),
                     "median_rel_err_vs_oracle": float(np.median(errs)), "checked_ics": int(idx.size),
                     "checked_at": "every segment boundary and the final state",
                     "above_1e-10": int(bad.size), "above_1e-10_oracle_sensitivity": [float(k) for k in kappa],
                     "max_rel_err_per_group": per_group, "max_iteration_diff": iter_diff, "status": int(status),
                     "mean_iterations_per_segment": round(float(iters[iters > 0].mean()), 3)},
        "segment_iterations_per_s": round(float(np.where(iters > 0, iters, 0).sum()) / (ms_per_step * 1e-3), 1),
        "vs_plain": plain or None,
        "mixed_precision": mixed,
        "second_order": second,
        "flyby_isolation": flyby,
        "autotune": tuned,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def run_second_order(args, w, pcprop):
    """The second-order sub-record: the workload with first-order sweeps (the iteration of
    Sec. 2.2) and with second-order sweeps (velocity and position both from the acceleration
    fit), the same fused FP64 kernel; time, sweeps per segment, and each form's error against
    the oracle run in the same form on a seeded sample (stratified over the groups), at every
    segment boundary.  A context of its own, tuned for this workload with first-order
    sweeps; both forms run with the job lengths it picked."""
    import torch
    n_ic = w.n_ic
    S = max(g.segments for g in w.groups)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    ctx = pcprop.Context(0)
    ctx.autotune(ics, groups, model)
    idx = stratified_sample(w, max(1, 64 // len(w.groups)), seed=11)
    res = {}
    for order in (1, 2):
        st = torch.empty((n_ic, 6), dtype=torch.float64, device="cuda")
        it = torch.zeros((n_ic, S), dtype=torch.int32, device="cuda")
        bd = torch.empty((n_ic, S + 1, 6), dtype=torch.float64, device="cuda")
        kw = dict(order=order, out=st, iters_out=it, bounds_out=bd)
        ctx.propagate_batched(ics, groups, model, **kw)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.second_order_steps):
            r = ctx.propagate_batched(ics, groups, model, **kw)
        e1.record()
        torch.cuda.synchronize()
        _, ref_it, ref_b, _, _ = oracle_run(w, idx, order=order)
        iters = it.cpu().numpy()
        err = boundary_errors(bd.cpu().numpy()[idx], ref_b)
        res[order] = {"ms_per_step": round(e0.elapsed_time(e1) / args.second_order_steps, 4),
                      "status": int(r["status"]),
                      "mean_sweeps_per_segment": round(float(iters[iters > 0].mean()), 3),
                      "max_rel_err_vs_oracle_same_form": float(err.max()),
                      "max_sweep_diff_vs_oracle": int(np.abs(iters[idx] - ref_it).max())}
        res[order]["states"] = st.cpu().numpy()
    dif = rel_err(res[2].pop("states"), res[1].pop("states"))
    diff = float(dif.max())
    n_icseg = sum(g.n_ic * g.segments for g in w.groups)
    out = {"workload": w.name, "n_ic": n_ic, "steps": args.second_order_steps,
           "first_order": res[1], "second_order": res[2],
           "ic_segments_per_s_second_order": round(n_icseg / (res[2]["ms_per_step"] * 1e-3), 1),
           "speedup_second_vs_first": round(res[1]["ms_per_step"] / res[2]["ms_per_step"], 3),
           "max_rel_diff_between_forms": diff,
           "median_rel_diff_between_forms": float(np.median(dif)),
           "p99_rel_diff_between_forms": float(np.percentile(dif, 99)),
           "checked_ics": int(idx.size),
           "valid": bool(res[2]["max_rel_err_vs_oracle_same_form"] <= 1e-10 and res[2]["status"] == 0)}
    print(f"bench: {w.name}: second-order {res[2]['ms_per_step']:.3f} ms/step "
          f"({res[2]['mean_sweeps_per_segment']} sweeps/segment), first-order {res[1]['ms_per_step']:.3f} ms/step "
          f"({res[1]['mean_sweeps_per_segment']}), speedup {out['speedup_second_vs_first']}x, max err vs its "
          f"oracle {res[2]['max_rel_err_vs_oracle_same_form']:.2e}, forms differ by {diff:.1e} at most "
          f"(median {np.median(dif):.1e}, p99 {np.percentile(dif, 99):.1e})", flush=True)
    return out


def run_flyby(args, ctx, w, pcprop):
    """The flyby-isolation sub-record: the workload on the plain path under the group-max
    stopping rule (the paper's per-system convergence) with the outer level on 10 streams,
    each group as one outer group and with its flyby ICs (two-body prediction within
    --flyby-hill Hill radii of a planet) in a group of their own; time and mean sweeps per
    segment of the quiet ICs, and, under the per-IC rule on the fused path, the mean sweeps
    of the flyby and of the quiet ICs."""
    import torch
    S = max(g.segments for g in w.groups)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    ratio = ctx.flyby_ratio(ics, groups, model).cpu().numpy()
    quiet = ratio >= args.flyby_hill
    res = {}
    for hill in (0.0, args.flyby_hill):
        it = torch.zeros((w.n_ic, S), dtype=torch.int32, device="cuda")
        kw = dict(path="plain", conv="group", flyby_hill=hill, iters_out=it, streams=10)
        ctx.propagate_batched(ics, groups, model, **kw)   # untimed: first launches of its kernels
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.propagate_batched(ics, groups, model, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        iters = it.cpu().numpy()
        res[hill] = {"ms": round(ms, 2), "status": int(r["status"]),
                     "mean_sweeps_per_segment_quiet": round(float(iters[quiet][iters[quiet] > 0].mean()), 3),
                     "mean_sweeps_per_segment_all": round(float(iters[iters > 0].mean()), 3)}
    # the same ICs under the per-IC rule (fused path): do the flyby ICs need more sweeps?
    it = torch.zeros((w.n_ic, S), dtype=torch.int32, device="cuda")
    ctx.propagate_batched(ics, groups, model, iters_out=it)
    iters = it.cpu().numpy()
    per_ic = {"mean_sweeps_per_segment_quiet": round(float(iters[quiet][iters[quiet] > 0].mean()), 3),
              "mean_sweeps_per_segment_flyby": round(float(iters[~quiet][iters[~quiet] > 0].mean()), 3)
              if (~quiet).any() else None}
    out = {"workload": w.name, "path": "plain", "conv": "group", "streams": 10, "hill_radii": args.flyby_hill,
           "isolated_ics": int((~quiet).sum()), "n_ic": w.n_ic, "per_ic_rule_fused": per_ic,
           "without_isolation": res[0.0], "with_isolation": res[args.flyby_hill],
           "speedup": round(res[0.0]["ms"] / res[args.flyby_hill]["ms"], 3)}
    print(f"bench: flyby isolation ({(~quiet).sum()} of {w.n_ic} ICs within {args.flyby_hill} Hill radii), group-max "
          f"plain path: {res[0.0]['ms']:.1f} -> {res[args.flyby_hill]['ms']:.1f} ms, quiet ICs' sweeps "
          f"{res[0.0]['mean_sweeps_per_segment_quiet']} -> {res[args.flyby_hill]['mean_sweeps_per_segment_quiet']}; "
          f"per-IC rule: flyby ICs {per_ic['mean_sweeps_per_segment_flyby']} sweeps/segment, quiet "
          f"{per_ic['mean_sweeps_per_segment_quiet']}", flush=True)
    return out


def run_mixed(args, w, pcprop):
    """The mixed-precision sub-record: the workload under the FP32 -> FP64 schedule and all
    in FP64, the same kernel and call, with per-IC errors of both against the FP64 oracle on
    a seeded sample (at every segment boundary).  A context of its own, its FP64 run tuned
    for this workload."""
    import torch
    n_ic = w.n_ic
    S = max(g.segments for g in w.groups)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    ctx = pcprop.Context(0)
    ctx.autotune(ics, groups, model)
    res = {}
    for prec in ("fp32-fp64", "fp64"):
        st = torch.empty((n_ic, 6), dtype=torch.float64, device="cuda")
        it = torch.zeros((n_ic, S), dtype=torch.int32, device="cuda")
        bd = torch.empty((n_ic, S + 1, 6), dtype=torch.float64, device="cuda")
        kw = dict(precision=prec, out=st, iters_out=it, bounds_out=bd)
        ctx.propagate_batched(ics, groups, model, **kw)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.mixed_steps):
            r = ctx.propagate_batched(ics, groups, model, **kw)
        e1.record()
        torch.cuda.synchronize()
        res[prec] = (e0.elapsed_time(e1) / args.mixed_steps, r["status"], it.cpu().numpy(), bd.cpu().numpy())
    idx = np.sort(np.random.default_rng(7).choice(n_ic, size=min(args.mixed_check_ics, n_ic), replace=False))
    _, ref_it, ref_b, _, _ = oracle_run(w, idx)
    e_mix = boundary_errors(res["fp32-fp64"][3][idx], ref_b)
    e_64 = boundary_errors(res["fp64"][3][idx], ref_b)
    ms_mix, ms_64 = res["fp32-fp64"][0], res["fp64"][0]
    it_mix, it_64 = res["fp32-fp64"][2], res["fp64"][2]
    out = {"workload": w.name, "n_ic": n_ic, "steps": args.mixed_steps,
           "ms_per_step_mixed": round(ms_mix, 4), "ms_per_step_fp64": round(ms_64, 4),
           "speedup_mixed_vs_fp64": round(ms_64 / ms_mix, 3),
           "ic_segments_per_s_mixed": round(sum(g.n_ic * g.segments for g in w.groups) / (ms_mix * 1e-3), 1),
           "status": [int(res["fp32-fp64"][1]), int(res["fp64"][1])],
           "checked_ics": int(idx.size),
           "mixed_rel_err_vs_oracle": {"max": float(e_mix.max()), "p99": float(np.percentile(e_mix, 99)),
                                       "median": float(np.median(e_mix))},
           "fp64_rel_err_vs_oracle": {"max": float(e_64.max()), "p99": float(np.percentile(e_64, 99)),
                                      "median": float(np.median(e_64))},
           "mean_sweeps_per_segment": {"mixed": round(float(it_mix[it_mix > 0].mean()), 3),
                                       "fp64": round(float(it_64[it_64 > 0].mean()), 3),
                                       "oracle_sample": round(float(ref_it[ref_it > 0].mean()), 3)},
           "valid": bool(e_mix.max() <= 1e-10 and e_64.max() <= 1e-10 and res["fp32-fp64"][1] == 0)}
    print(f"bench: {w.name}: mixed {ms_mix:.3f} ms/step, FP64 {ms_64:.3f} ms/step, "
          f"speedup {ms_64 / ms_mix:.2f}x, max err vs oracle {e_mix.max():.2e} (FP64 {e_64.max():.2e}) "
          f"on {idx.size} ICs", flush=True)
    return out


if __name__ == "__main__":
    main()
