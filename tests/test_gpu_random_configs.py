"""Randomised configurations against the oracle: node counts 3..256 (every padding and job
shape), 1-3 segments, forward and backward spans, relative and absolute tolerances, warm
and cold starts, both paths, both precisions, point-mass and relativistic dynamics, and
the 1024-pair shape where it applies; and multi-group batches of eccentric orbits with
job lengths, graph replays, plain-path streams and the group-max rule.  Seeded, so every
case is reproducible by its id."""
import numpy as np
import pytest
import torch

from paper_2301_03989_amd import workloads as W
from tests._parity import oracle_run, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_03989_amd import build, pcprop
    build.ensure_built()
    return pcprop.Context(0)


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    N = int(rng.integers(3, 257))
    S = int(rng.integers(1, 4))
    n = int(rng.integers(5, 40))
    days = float(rng.uniform(20.0, 120.0)) * S
    w = W.nbody_venus(n, seed=200 + seed, days=days, segments=S, nodes=N,
                      tol=float(rng.choice([1e-10, 1e-12, 1e-13])))
    if rng.random() < 0.3:                       # backward span
        g = w.groups[0]
        g.t0, g.tf = g.tf, g.t0
    if rng.random() < 0.3:
        w.inv_c2 = 1.0 / W.C_AU_TU**2
    w.init = 1 if rng.random() < 0.2 else 0
    kw = dict(init="cold" if w.init else "kepler", tol_mode="abs" if rng.random() < 0.25 else "rel")
    r = rng.random()
    if r < 0.25:
        kw["path"] = "plain"
    elif r < 0.5:
        kw["precision"] = "fp32-fp64"
    np_ = max(16, 1 << int(np.ceil(np.log2(N))))
    if np_ * 8 <= 1024 and rng.random() < 0.3:
        kw["tile_pairs"] = 1024
    return w, kw


@pytest.mark.parametrize("seed", range(64))
def test_random_configuration(pc, seed):
    from paper_2301_03989_amd import pcprop
    w, kw = _case(seed)
    g = w.groups[0]
    print(f"case {seed}: N {g.nodes} S {g.segments} n {w.n_ic} tol {g.tol} inv_c2 {w.inv_c2} span "
          f"{g.t0:.3f}->{g.tf:.3f} {kw}", flush=True)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    r = pc.propagate_batched(ics, groups, model, **kw)
    torch.cuda.synchronize()
    o = oracle_run(w, tol_mode=1 if kw.get("tol_mode") == "abs" else 0)
    assert r["status"] in (pcprop.PC_OK, pcprop.PC_ENOTCONV), r["status"]
    err = rel_err(r["states"].cpu().numpy(), o["states"])
    assert err.max() < 1e-10, err.max()
    d = r["iters"].cpu().numpy() - o["iters"]
    assert d.min() >= -1 and d.max() <= (12 if kw.get("precision") else 1), (d.min(), d.max())


def _batch(seed):
    """A seeded multi-group batch of eccentric orbits (2-6 groups of the uneven recipe:
    node counts 64/128/256 or random, 1-3 segments) and random call options."""
    rng = np.random.default_rng(5000 + seed)
    w = W.uneven_batch(int(rng.integers(60, 400)), seed=300 + seed)
    keep = sorted(rng.choice(len(w.groups), size=int(rng.integers(2, 7)), replace=False))
    groups, parts, off = [], [], 0
    for gi in keep:
        g = w.groups[gi]
        n = int(min(g.n_ic, rng.integers(4, 40)))
        parts.append(w.ics[g.ic_offset:g.ic_offset + n])
        S = int(rng.integers(1, 4))
        N = g.nodes if rng.random() < 0.6 else int(rng.integers(3, 257))
        groups.append(W.Group(off, n, 0.0, S * np.pi / 4.0, N, S, float(rng.choice([1e-11, 1e-12]))))
        off += n
    b = W.Workload("random-batch", np.concatenate(parts), groups, w.pert)
    kw = {}
    r = rng.random()
    if r < 0.2:
        kw = dict(path="plain", streams=int(rng.integers(1, 5)))
        if rng.random() < 0.4:
            kw["conv"] = "group"
    elif r < 0.4:
        kw = dict(precision="fp32-fp64")
    else:
        kw = dict(job_list=int(rng.choice([0, 1, 2, 4, 8])), graph=bool(rng.random() < 0.3))
    return b, kw


@pytest.mark.parametrize("seed", range(32))
def test_random_batch(pc, seed):
    from paper_2301_03989_amd import pcprop
    import oracle
    b, kw = _batch(seed)
    print(f"batch {seed}: " + ", ".join(f"N {g.nodes} S {g.segments} n {g.n_ic}" for g in b.groups) + f" {kw}",
          flush=True)
    ics = torch.tensor(b.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in b.groups]
    r = pc.propagate_batched(ics, groups, pcprop.Model(b.mu_sun, b.pert, b.epoch), **kw)
    torch.cuda.synchronize()
    assert r["status"] in (pcprop.PC_OK, pcprop.PC_ENOTCONV), r["status"]
    states, iters = r["states"].cpu().numpy(), r["iters"].cpu().numpy()
    if kw.get("conv") == "group":
        m = oracle.Model(b.mu_sun, b.pert, b.epoch)
        for g in b.groups:
            sl = slice(g.ic_offset, g.ic_offset + g.n_ic)
            so, io = oracle.propagate(b.ics[sl], g.t0, g.tf, g.nodes, g.segments, g.tol, m, conv=1)
            assert rel_err(states[sl], so).max() < 1e-10
            assert np.abs(iters[sl, :g.segments] - io).max() <= 1
        return
    o = oracle_run(b)
    assert rel_err(states, o["states"]).max() < 1e-10
    d = iters - o["iters"]
    # the precision schedule's counts follow the slowest IC of each job (eccentric orbits
    # spread them widely); the FP64 counts are the oracle's
    assert d.min() >= -1 and d.max() <= (20 if kw.get("precision") else 1), (d.min(), d.max())


def _option_case(seed):
    """A seeded case of one of the later options: second-order sweeps (with or without the
    integral error feedback), adaptive refinement under a sweep budget (first- or
    second-order sweeps), flyby isolation (per-IC or group-max rule), or a hot start from
    the oracle's node states of nearby ICs."""
    rng = np.random.default_rng(9000 + seed)
    mode = ["order2", "feedback", "refine", "flyby", "guess", "order2_refine"][seed % 6]
    kw, okw = {}, {}
    if mode in ("order2", "feedback"):
        N = int(rng.integers(3, 257))
        S = int(rng.integers(1, 4))
        w = W.nbody_venus(int(rng.integers(5, 40)), seed=400 + seed, days=float(rng.uniform(20, 90)) * S,
                          segments=S, nodes=N, tol=float(rng.choice([1e-11, 1e-12])))
        if rng.random() < 0.3:
            g = w.groups[0]
            g.t0, g.tf = g.tf, g.t0
        kw = dict(order=2, feedback=int(mode == "feedback"))
        okw = dict(order=2, feedback=int(mode == "feedback"))
    elif mode == "refine":
        w = W.long_segments(int(rng.integers(8, 40)), seed=500 + seed, nodes=int(rng.integers(48, 129)),
                            segments=int(rng.integers(1, 4)))
        budget, depth = int(rng.integers(16, 29)), int(rng.integers(1, 4))
        kw = dict(refine=depth, max_iter=budget)
        okw = dict(refine=depth, max_iter=budget)
    elif mode == "order2_refine":
        # second-order sweeps take about half the first-order count: a smaller budget
        w = W.long_segments(int(rng.integers(8, 40)), seed=550 + seed, nodes=int(rng.integers(48, 257)),
                            segments=int(rng.integers(1, 4)))
        budget, depth = int(rng.integers(8, 15)), int(rng.integers(1, 4))
        kw = dict(refine=depth, max_iter=budget, order=2)
        okw = dict(refine=depth, max_iter=budget, order=2)
    elif mode == "flyby":
        u = W.uneven_batch(int(rng.integers(200, 600)), seed=600 + seed)
        keep = sorted(rng.choice(len(u.groups), size=int(rng.integers(2, 5)), replace=False))
        groups, parts, off = [], [], 0
        for gi in keep:
            g = u.groups[gi]
            n = int(min(g.n_ic, rng.integers(8, 60)))
            parts.append(u.ics[g.ic_offset:g.ic_offset + n])
            S = int(rng.integers(1, 4))
            groups.append(W.Group(off, n, 0.0, S * np.pi / 4.0, g.nodes, S, 1e-12))
            off += n
        w = W.Workload("flyby-batch", np.concatenate(parts), groups, u.pert)
        kw = dict(flyby_hill=float(rng.uniform(4.0, 8.0)))
        if rng.random() < 0.5:
            kw.update(path="plain", conv="group")
    else:
        w = W.nbody_venus(int(rng.integers(5, 40)), seed=700 + seed, days=float(rng.uniform(40, 120)), segments=2,
                          nodes=int(rng.integers(16, 129)))
        w.init = 2            # the oracle's hot start (the GPU call names it below)
        kw = dict(init="guess")
    return mode, w, kw, okw


@pytest.mark.parametrize("seed", range(40))
def test_random_options(pc, seed):
    from paper_2301_03989_amd import pcprop
    import oracle
    mode, w, kw, okw = _option_case(seed)
    print(f"option case {seed} ({mode}): " + ", ".join(f"N {g.nodes} S {g.segments} n {g.n_ic}" for g in w.groups)
          + f" {kw}", flush=True)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch)
    m = oracle.Model(w.mu_sun, w.pert, w.epoch)
    if mode == "guess":
        # node states of nearby ICs, from the oracle, as the guess of both sides
        g = w.groups[0]
        near = w.ics * (1.0 + 1e-7 * np.random.default_rng(seed).standard_normal(w.ics.shape))
        _, _, guess = oracle.propagate(near, g.t0, g.tf, g.nodes, g.segments, g.tol, m, want_nodes=True)
        kw["guess"] = torch.tensor(guess, dtype=torch.float64, device="cuda")
        okw["guess"] = guess
    r = pc.propagate_batched(ics, groups, model, want_bounds=True, **kw)
    torch.cuda.synchronize()
    assert r["status"] in (pcprop.PC_OK, pcprop.PC_ENOTCONV), r["status"]
    states, iters = r["states"].cpu().numpy(), r["iters"].cpu().numpy()
    if mode == "flyby":
        ratio = np.concatenate([oracle.flyby_ratio(w.ics[g.ic_offset:g.ic_offset + g.n_ic], g.t0, g.tf, g.segments, m)
                                for g in w.groups])
        hill = kw["flyby_hill"]
        assert np.min(np.abs(ratio / hill - 1.0)) > 1e-9
        conv = 1 if kw.get("conv") == "group" else 0
        for g in w.groups:
            idx = np.arange(g.ic_offset, g.ic_offset + g.n_ic)
            fly = ratio[idx] < hill
            for part in ((idx[~fly], idx[fly]) if conv else (idx,)):
                if part.size == 0:
                    continue
                so, io = oracle.propagate(w.ics[part], g.t0, g.tf, g.nodes, g.segments, g.tol, m, conv=conv)
                assert rel_err(states[part], so).max() < 1e-10
                assert np.abs(iters[part, :g.segments] - io).max() <= 1
        return
    o = oracle_run(w, **okw)
    assert rel_err(states, o["states"]).max() < 1e-10
    d = np.abs(iters - o["iters"])
    if mode in ("refine", "order2_refine"):   # a budget hit one sweep apart splits a segment differently
        assert (np.all(d <= 2, axis=1)).mean() >= 0.9
    else:
        assert d.max() <= 1, d.max()
