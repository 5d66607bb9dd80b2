"""Shared helpers of the parity tests: run a workload on the oracle and on the HIP
path and measure per-IC relative position/velocity errors."""
import numpy as np

import oracle


def rel_err(a, b):
    """Per-IC max(|dr|/|r|, |dv|/|v|) of states a against reference b ([n, 6])."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 6)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 6)
    er = np.linalg.norm(a[:, :3] - b[:, :3], axis=1) / np.linalg.norm(b[:, :3], axis=1)
    ev = np.linalg.norm(a[:, 3:] - b[:, 3:], axis=1) / np.linalg.norm(b[:, 3:], axis=1)
    return np.maximum(er, ev)


def oracle_run(w, idx=None, want_nodes=False, want_bounds=False, **kw):
    """Oracle results for the ICs ``idx`` of workload ``w`` (all by default):
    states [k, 6], iters [k, S_max] (and nodes / bounds when asked)."""
    idx = np.arange(w.n_ic) if idx is None else np.asarray(idx)
    S_max = max(g.segments for g in w.groups)
    N_max = max(g.nodes for g in w.groups)
    states = np.zeros((idx.size, 6))
    iters = np.zeros((idx.size, S_max), dtype=np.int32)
    nodes = np.zeros((idx.size, S_max, N_max, 6)) if want_nodes else None
    bounds = np.zeros((idx.size, S_max + 1, 6)) if want_bounds else None
    model = oracle.Model(w.mu_sun, w.pert, w.epoch, inv_c2=w.inv_c2)
    for g in w.groups:
        sel = np.nonzero((idx >= g.ic_offset) & (idx < g.ic_offset + g.n_ic))[0]
        if sel.size == 0:
            continue
        out = oracle.propagate(w.ics[idx[sel]], g.t0, g.tf, g.nodes, g.segments, g.tol, model,
                               init=w.init, want_nodes=want_nodes, want_bounds=want_bounds, **kw)
        states[sel] = out[0]
        iters[sel, :g.segments] = out[1]
        k = 2
        if want_bounds:
            bounds[sel, :g.segments + 1] = out[k]
            k += 1
        if want_nodes:
            nodes[sel, :g.segments, :g.nodes] = out[k]
    res = {"states": states, "iters": iters}
    if want_nodes:
        res["nodes"] = nodes
    if want_bounds:
        res["bounds"] = bounds
    return res


def oracle_sensitivity(w, idx, rel=1e-14, reps=4, seed=0):
    """Conditioning of the ICs ``idx`` of workload ``w`` measured on the oracle: the largest
    per-IC relative change of the segment-boundary states (final state included) when each
    IC component is scaled by (1 +- rel), random signs, over ``reps`` draws.  Two FP64
    implementations whose rounding differs at the 1e-16..1e-14 level can differ by about
    this much on these ICs however exactly each follows the method."""
    rng = np.random.default_rng(seed)
    idx = np.asarray(idx)
    base = oracle_run(w, idx, want_bounds=True)["bounds"]
    worst = np.zeros(idx.size)
    for _ in range(reps):
        wp = Workload_like(w, w.ics.copy())
        wp.ics[idx] = w.ics[idx] * (1.0 + rel * rng.choice([-1.0, 1.0], size=(idx.size, 6)))
        b = oracle_run(wp, idx, want_bounds=True)["bounds"]
        worst = np.maximum(worst, boundary_err(b, base))
    return worst


def boundary_err(a, b):
    """Per-IC max over segment boundaries (final state included) of rel_err; a, b
    [n, S+1, 6], rows of all-zero reference (unused boundaries) skipped."""
    a = np.asarray(a)
    b = np.asarray(b)
    n, k, _ = b.shape
    used = np.any(b != 0.0, axis=2)
    e = rel_err(a.reshape(-1, 6), np.where(used.reshape(-1, 1), b.reshape(-1, 6), 1.0)).reshape(n, k)
    return np.where(used, e, 0.0).max(axis=1)


def Workload_like(w, ics):
    """A copy of workload ``w`` with other initial conditions."""
    from paper_2301_03989_amd.workloads import Workload
    return Workload(w.name, ics, w.groups, w.pert, w.init, w.precision, w.mu_sun, w.epoch, w.inv_c2,
                    dict(w.meta))
