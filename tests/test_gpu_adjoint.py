"""Adjoint (reverse-mode gradient through the converged propagation) on the GPU against
the oracle's implicit derivative of the discrete fixed point (a dense linear solve per
segment, itself pinned by finite differences and a variational STM in the CPU suite).

Bar: per-IC relative gradient error (2-norm over the six components) <= 1e-8; the forward
re-solve converges to 1e-13 and the adjoint sweeps to 1e-13, so the two derivatives are
taken at iterates that differ by ~1e-13.
"""
import numpy as np
import pytest

import oracle
from paper_2301_03989_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GTOL = 1e-8


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_03989_amd import build, pcprop
    build.ensure_built()
    return pcprop.Context(0)


def _setup(w):
    from paper_2301_03989_amd import pcprop
    g = w.groups[0]
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    return ics, groups, pcprop.Model(1.0, w.pert, 0.0), oracle.Model(1.0, w.pert, 0.0), g


def _gerr(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def test_adjoint_final_state_matches_oracle(pc):
    w = W.nbody_venus(24, seed=105, days=76.8, segments=3, nodes=64, tol=1e-13)
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True)
    assert fwd["status"] == 0
    gbar = np.random.default_rng(1).standard_normal((w.n_ic, 6))
    grad, adj_it, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model)
    assert st == 0 and (adj_it.cpu().numpy() > 1).all()
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar)
    assert _gerr(grad.cpu().numpy(), ref).max() < GTOL


def test_adjoint_node_seeds_match_oracle(pc):
    w = W.nbody_venus(10, seed=106, days=51.2, segments=2, nodes=48, tol=1e-13)
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True)
    rng = np.random.default_rng(4)
    gn = np.zeros((w.n_ic, 2, 48, 6))
    gn[:, 0, 7] = rng.standard_normal((w.n_ic, 6))
    gn[:, 1, 30] = rng.standard_normal((w.n_ic, 6))
    gbar = np.zeros((w.n_ic, 6))
    grad, _, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model,
                             gbar_nodes=torch.tensor(gn, device="cuda"))
    assert st == 0
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar, gn)
    assert _gerr(grad.cpu().numpy(), ref).max() < GTOL


def test_autograd_function(pc):
    from paper_2301_03989_amd import autograd
    w = W.nbody_venus(16, seed=107, days=51.2, segments=2, nodes=64, tol=1e-13)
    ics, groups, model, om, g = _setup(w)
    x = ics.clone().requires_grad_(True)
    c = torch.tensor(np.random.default_rng(5).standard_normal((w.n_ic, 6)), device="cuda")
    states = autograd.propagate(x, groups, model, pc=pc)
    loss = (states * c).sum()
    (gx,) = torch.autograd.grad(loss, x)
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, c.cpu().numpy())
    assert _gerr(gx.cpu().numpy(), ref).max() < GTOL
    # node states kept for the backward pass instead of re-solving from checkpoints
    x2 = ics.clone().requires_grad_(True)
    loss2 = (autograd.propagate(x2, groups, model, pc=pc, store_nodes=True) * c).sum()
    (gx2,) = torch.autograd.grad(loss2, x2)
    assert _gerr(gx2.cpu().numpy(), gx.cpu().numpy()).max() < 1e-12


def test_adjoint_sixteen_perturbers_global_records(pc):
    """16 perturbers at 128 nodes: the records no longer fit beside the adjoint's scratch in
    LDS, so the Hessian products read them from global memory."""
    from paper_2301_03989_amd import pcprop
    base = W.planet_elements()
    extra = base.copy()
    extra[:, 0] *= 0.37
    extra[:, 6] += 2.1
    pert = np.concatenate([base, extra])
    w = W.nbody_venus(12, seed=112, days=40.0, segments=2, nodes=128, tol=1e-13)
    g = w.groups[0]
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    model, om = pcprop.Model(1.0, pert, 0.0), oracle.Model(1.0, pert, 0.0)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True, want_nodes=True)
    assert fwd["status"] == 0
    gbar = np.random.default_rng(12).standard_normal((w.n_ic, 6))
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar)
    for nodes in (None, fwd["nodes"]):
        grad, _, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model, fwd_nodes=nodes)
        assert st == 0
        assert _gerr(grad.cpu().numpy(), ref).max() < GTOL


@pytest.mark.parametrize("nodes", [24, 64, 100])
def test_adjoint_from_stored_node_states(pc, nodes):
    """The forward call's node states in place of the re-solves: the same gradients (the
    forward and a re-solve compute the same iterates, up to rounding where their job shapes
    differ), also against the oracle, with end-state and node seeds."""
    w = W.nbody_venus(37, seed=111, days=50.0, segments=3, nodes=nodes, tol=1e-13)
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True, want_nodes=True)
    assert fwd["status"] == 0
    rng = np.random.default_rng(nodes)
    gbar = rng.standard_normal((w.n_ic, 6))
    gn = np.zeros((w.n_ic, 3, nodes, 6))
    gn[:, 1, nodes // 2] = rng.standard_normal((w.n_ic, 6))
    gnt = torch.tensor(gn, device="cuda")
    args = (fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model)
    a, _, sa = pc.adjoint(*args, gbar_nodes=gnt)
    b, _, sb = pc.adjoint(*args, gbar_nodes=gnt, fwd_nodes=fwd["nodes"])
    assert sa == sb == 0
    assert _gerr(b.cpu().numpy(), a.cpu().numpy()).max() < 1e-12
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar, gn)
    assert _gerr(b.cpu().numpy(), ref).max() < GTOL


def _venus_min_seeds(nodes, w, om, g, tau):
    """Seeds of L = min over the CGL nodes of |r - r_Venus| (the discrete minimum, with the
    minimising node held fixed): dL/dr at that node = (r - r_V)/|r - r_V|."""
    n, S, N, _ = nodes.shape
    h = (g.tf - g.t0) / S
    gn = np.zeros_like(nodes)
    dmin = np.zeros(n)
    for m in range(n):
        best = (np.inf, 0, 0)
        for s in range(S):
            for j in range(N):
                t = g.t0 + h * s + 0.5 * h * (tau[j] + 1.0)
                d = nodes[m, s, j, :3] - oracle.ephem(w.pert[1], 0.0, t)
                dn = np.linalg.norm(d)
                if dn < best[0]:
                    best = (dn, s, j, d)
        dmin[m] = best[0]
        gn[m, best[1], best[2], :3] = best[3] / best[0]
    return gn, dmin


def test_min_venus_distance_gradient(pc):
    w = W.nbody_venus(6, seed=108, days=153.6, segments=3, nodes=64, tol=1e-13)
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True, want_nodes=True)
    tau = oracle.nodes(g.nodes)
    gn, dmin = _venus_min_seeds(fwd["nodes"].cpu().numpy(), w, om, g, tau)
    gbar = np.zeros((w.n_ic, 6))
    grad, _, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model,
                             gbar_nodes=torch.tensor(gn, device="cuda"))
    assert st == 0
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar, gn)
    assert _gerr(grad.cpu().numpy(), ref).max() < GTOL
    # and against central differences (h = 1e-7) of the oracle's objective, minimising node held fixed and
    # iterations frozen at 40 so the perturbed maps are converged to rounding, not to tol
    hstep = 1e-7
    sel = np.argwhere(gn[..., 0] != 0)
    for m in range(2):
        _, s_, j_ = sel[sel[:, 0] == m][0]
        t = g.t0 + (g.tf - g.t0) / g.segments * s_ + 0.5 * (g.tf - g.t0) / g.segments * (tau[j_] + 1.0)
        rv = oracle.ephem(w.pert[1], 0.0, t)
        fd = np.zeros(6)
        for k in range(6):
            e = np.zeros(6)
            e[k] = hstep
            _, _, npl = oracle.propagate(w.ics[m:m + 1] + e, g.t0, g.tf, g.nodes, g.segments, g.tol, om,
                                         fixed_iters=40, want_nodes=True)
            _, _, nmi = oracle.propagate(w.ics[m:m + 1] - e, g.t0, g.tf, g.nodes, g.segments, g.tol, om,
                                         fixed_iters=40, want_nodes=True)
            fd[k] = (np.linalg.norm(npl[0, s_, j_, :3] - rv) - np.linalg.norm(nmi[0, s_, j_, :3] - rv)) / (2 * hstep)
        assert np.linalg.norm(grad.cpu().numpy()[m] - fd) / np.linalg.norm(fd) < 1e-6


def test_adjoint_full_size_sampled(pc):
    """The 16384-IC, 256-day, 5-segment, 128-node ensemble: every IC's gradient is computed on
    the GPU; a seeded sample of 64 of them (with the first and last IC) is checked against
    the oracle."""
    w = W.adjoint_ensemble()
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True)
    assert fwd["status"] == 0
    gbar = np.zeros((w.n_ic, 6))
    gbar[:, 0] = 1.0                         # d x_final / d y0
    grad, adj_it, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model)
    assert st == 0
    gr = grad.cpu().numpy()
    assert np.isfinite(gr).all()
    idx = np.unique(np.concatenate([[0, w.n_ic - 1], np.random.default_rng(12).choice(w.n_ic, 62, replace=False)]))
    ref = oracle.adjoint(w.ics[idx], g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar[idx])
    assert _gerr(gr[idx], ref).max() < GTOL


def test_adjoint_argument_errors(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(4, nodes=64, days=30.0, segments=1)
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True)
    # the adjoint linearises the first-order map: order 2 is refused
    with pytest.raises(pcprop.PcError):
        pc.adjoint(fwd["bounds"], torch.zeros((4, 6), dtype=torch.float64, device="cuda"), groups, model, order=2)
    # the adjoint linearises the map converged per IC: the group-max rule is refused
    w = W.nbody_venus(4, days=30.0, segments=1)
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True)
    with pytest.raises(pcprop.PcError) as e:
        pc.adjoint(fwd["bounds"], torch.zeros((4, 6), dtype=torch.float64, device="cuda"), groups, model,
                   conv="group")
    assert e.value.code == pcprop.PC_EINVAL


@pytest.mark.parametrize("nodes", [12, 24, 100, 200, 256])
def test_adjoint_every_job_shape(pc, nodes):
    """16 to 128 ICs per job (NP = 16, 32, 128) and the 8-IC node-row jobs (NP = 256), with a
    ragged IC count."""
    w = W.nbody_venus(41, seed=109, days=40.0, segments=2, nodes=nodes, tol=1e-13)
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True)
    gbar = np.random.default_rng(nodes).standard_normal((w.n_ic, 6))
    grad, _, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model)
    assert st == fwd["status"] and st in (0, 2)   # 2: a forward sweep hit max_iter on both sides
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar)
    assert _gerr(grad.cpu().numpy(), ref).max() < GTOL


def test_adjoint_mixed_groups_and_backward(pc):
    """Two groups with different node counts and spans in one call, one of them propagated
    backwards in time."""
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(20, seed=110, days=60.0, segments=2, nodes=64, tol=1e-13)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    tf = w.groups[0].tf
    groups = [pcprop.Group(0, 9, 0.0, tf, 64, 2, 1e-13), pcprop.Group(9, 11, 0.0, -0.6 * tf, 100, 3, 1e-13)]
    model = pcprop.Model(1.0, w.pert, 0.0)
    om = oracle.Model(1.0, w.pert, 0.0)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True)
    assert fwd["status"] == 0
    gbar = np.random.default_rng(3).standard_normal((w.n_ic, 6))
    grad, _, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model)
    assert st == 0
    gr = grad.cpu().numpy()
    for G in groups:
        sl = slice(G.ic_offset, G.ic_offset + G.n_ic)
        ref = oracle.adjoint(w.ics[sl], G.t0, G.tf, G.nodes, G.segments, G.tol, om, gbar[sl])
        assert _gerr(gr[sl], ref).max() < GTOL


@pytest.mark.parametrize("seed", range(12))
def test_adjoint_random_configuration(pc, seed):
    """Seeded random adjoint cases against the oracle: node counts 3..256, 1-3 segments,
    forward or backward spans, final-state and node seeds, checkpoints or stored nodes."""
    rng = np.random.default_rng(700 + seed)
    N = int(rng.integers(3, 257))
    S = int(rng.integers(1, 4))
    n = int(rng.integers(2, 7))
    w = W.nbody_venus(n, seed=800 + seed, days=float(rng.uniform(15.0, 40.0)) * S, segments=S, nodes=N,
                      tol=1e-13)
    if rng.random() < 0.3:
        g0 = w.groups[0]
        g0.t0, g0.tf = g0.tf, g0.t0
    ics, groups, model, om, g = _setup(w)
    stored = bool(rng.random() < 0.4)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True, want_nodes=stored)
    assert fwd["status"] == 0
    gbar = rng.standard_normal((n, 6))
    gn = None
    if rng.random() < 0.5:
        gn = np.zeros((n, S, N, 6))
        gn[:, rng.integers(0, S), rng.integers(0, N)] = rng.standard_normal((n, 6))
    print(f"adjoint case {seed}: N {N} S {S} n {n} span {g.t0:.3f}->{g.tf:.3f} stored {stored} "
          f"node seeds {gn is not None}", flush=True)
    grad, _, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model,
                             gbar_nodes=None if gn is None else torch.tensor(gn, device="cuda"),
                             fwd_nodes=fwd["nodes"] if stored else None)
    assert st == 0
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar, gn)
    assert _gerr(grad.cpu().numpy(), ref).max() < GTOL


def test_adjoint_node_row_jobs_stored_nodes_and_node_seeds(pc):
    """256-node jobs (node-row layout, lane pairs exchanging components) from the forward's
    stored node states, with seeds on interior nodes of both strips of a wave and on the
    last node, three segments, against the oracle; the re-solve gives the same gradient."""
    w = W.nbody_venus(13, seed=111, days=90.0, segments=3, nodes=256, tol=1e-13)
    ics, groups, model, om, g = _setup(w)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True, want_nodes=True)
    assert fwd["status"] == 0
    rng = np.random.default_rng(17)
    gbar = rng.standard_normal((w.n_ic, 6))
    gn = np.zeros((w.n_ic, 3, 256, 6))
    for j in (5, 21, 130, 255):
        gn[:, rng.integers(0, 3), j] = rng.standard_normal((w.n_ic, 6))
    gnt = torch.tensor(gn, device="cuda")
    a, it_a, st_a = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model,
                               gbar_nodes=gnt, fwd_nodes=fwd["nodes"])
    b, it_b, st_b = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model, gbar_nodes=gnt)
    assert st_a == 0 and st_b == 0
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar, gn)
    assert _gerr(a.cpu().numpy(), ref).max() < GTOL
    assert _gerr(b.cpu().numpy(), ref).max() < GTOL
    assert _gerr(a.cpu().numpy(), b.cpu().numpy()).max() < 1e-12


# -- the relativistic dynamics ------------------------------------------------------------
# The Einstein-Infeld-Hoffmann acceleration depends on the velocity: J^T w gains the
# velocity rows' (da/dv)^T w_v and the position rows take (da/dr)^T w_v of the full
# acceleration.  The oracle forms both by the complex step on its own restatement of the
# sums (pinned to finite differences of propagations in the CPU suite).  With the
# exaggerated 1/c^2 the point-mass derivative misses the gradient by far more than the
# bar, so a dropped or wrong relativistic term fails; the physical 1/c^2 checks the
# workload's own scale.

def _eih_setup(n, nodes, inv_c2, seed, days=40.0, segments=2):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(n, seed=seed, days=days, segments=segments, nodes=nodes, tol=1e-13)
    g = w.groups[0]
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    return (w, ics, groups, pcprop.Model(1.0, w.pert, 0.0, inv_c2), oracle.Model(1.0, w.pert, 0.0, inv_c2=inv_c2),
            g)


@pytest.mark.parametrize("inv_c2", [1e-4, 1.0 / W.C_AU_TU ** 2])
@pytest.mark.parametrize("nodes", [24, 100, 256])
def test_relativistic_adjoint_matches_oracle(pc, nodes, inv_c2):
    """Transposed jobs (24, 100 nodes) and 8-IC node-row jobs (256 nodes, lane pairs
    exchanging positions, velocities and the products), with a ragged IC count."""
    w, ics, groups, model, om, g = _eih_setup(9, nodes, inv_c2, seed=130 + nodes)
    print(f"relativistic adjoint: N {nodes} inv_c2 {inv_c2:.3e}", flush=True)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True)
    assert fwd["status"] == 0
    gbar = np.random.default_rng(nodes).standard_normal((w.n_ic, 6))
    grad, adj_it, st = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model)
    assert st == 0 and (adj_it.cpu().numpy()[:, :g.segments] > 1).all()
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar)
    gr = grad.cpu().numpy()
    assert _gerr(gr, ref).max() < GTOL
    if inv_c2 > 1e-6:
        pm = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, oracle.Model(1.0, w.pert, 0.0), gbar)
        assert _gerr(gr, pm).min() > 100 * GTOL


@pytest.mark.parametrize("nodes", [64, 256])
def test_relativistic_adjoint_stored_nodes_and_node_seeds(pc, nodes):
    """From the forward's stored node states and from re-solves, with seeds on interior
    nodes and the last one, three segments, against the oracle."""
    w, ics, groups, model, om, g = _eih_setup(10, nodes, 1e-4, seed=140 + nodes, days=60.0, segments=3)
    fwd = pc.propagate_batched(ics, groups, model, want_bounds=True, want_nodes=True)
    assert fwd["status"] == 0
    rng = np.random.default_rng(nodes + 1)
    gbar = rng.standard_normal((w.n_ic, 6))
    gn = np.zeros((w.n_ic, 3, nodes, 6))
    for j in (3, nodes // 2 + 1, nodes - 1):
        gn[:, rng.integers(0, 3), j] = rng.standard_normal((w.n_ic, 6))
    gnt = torch.tensor(gn, device="cuda")
    a, _, st_a = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model, gbar_nodes=gnt,
                            fwd_nodes=fwd["nodes"])
    b, _, st_b = pc.adjoint(fwd["bounds"], torch.tensor(gbar, device="cuda"), groups, model, gbar_nodes=gnt)
    assert st_a == 0 and st_b == 0
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, gbar, gn)
    assert _gerr(a.cpu().numpy(), ref).max() < GTOL
    assert _gerr(b.cpu().numpy(), ref).max() < GTOL
    assert _gerr(a.cpu().numpy(), b.cpu().numpy()).max() < 1e-12


def test_relativistic_autograd_function(pc):
    """The torch.autograd wrapper with the relativistic model: the backward pass is the
    relativistic adjoint, from checkpoints and from stored node states."""
    from paper_2301_03989_amd import autograd
    w, ics, groups, model, om, g = _eih_setup(12, 48, 1e-4, seed=150)
    c = torch.tensor(np.random.default_rng(6).standard_normal((w.n_ic, 6)), device="cuda")
    ref = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, om, c.cpu().numpy())
    for store in (False, True):
        x = ics.clone().requires_grad_(True)
        loss = (autograd.propagate(x, groups, model, pc=pc, store_nodes=store) * c).sum()
        (gx,) = torch.autograd.grad(loss, x)
        assert _gerr(gx.cpu().numpy(), ref).max() < GTOL, store
