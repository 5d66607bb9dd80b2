"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: per-IC relative position and velocity error <= 1e-10 at the final state and at
every segment boundary; iteration counts within +-1 (where the stopping decision sits
within rounding of the tolerance).  Kernel-level hooks (operator product, force,
Kepler warm start) are compared at the rounding level.
"""
import numpy as np
import pytest

import oracle
from paper_2301_03989_amd import workloads as W
from tests._parity import oracle_run, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_03989_amd import build, pcprop
    build.ensure_built()
    return pcprop.Context(0)


def _run(pc, w, idx=None, **kw):
    """HIP results for the ICs ``idx`` of workload w (all groups, one call)."""
    from paper_2301_03989_amd import pcprop
    sub = w if idx is None else w.subset(idx)
    ics = torch.tensor(sub.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in sub.groups]
    model = pcprop.Model(sub.mu_sun, sub.pert, sub.epoch, sub.inv_c2)
    kw.setdefault("init", "kepler" if sub.init == 0 else "cold")
    r = pc.propagate_batched(ics, groups, model, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}, sub


# ---------------------------------------------------------------------------
# kernel-level hooks
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N", [3, 4, 7, 16, 33, 64, 100, 128, 200, 256])
def test_operator_matches_oracle(pc, N):
    K = pc.get_operator(N)
    np.testing.assert_allclose(K, oracle.operator(N), rtol=0, atol=2e-15 * max(1, N / 32))
    assert np.all(K[0] == 0.0)


@pytest.mark.parametrize("N,ncols", [(3, 5), (16, 16), (64, 37), (128, 100), (200, 33), (256, 48)])
def test_mfma_product_matches_oracle_update(pc, N, ncols):
    rng = np.random.default_rng(N * 1000 + ncols)
    F = rng.standard_normal((N, ncols))
    y0 = rng.standard_normal(ncols)
    scale = 0.37
    Y = pc.apply_operator(torch.tensor(F, device="cuda"), torch.tensor(y0, device="cuda"), scale, N)
    ref = oracle.picard_step(scale * F, y0)
    np.testing.assert_allclose(Y.cpu().numpy(), ref, rtol=0, atol=5e-15 * max(1.0, N / 16))


def test_force_matches_oracle(pc):
    from paper_2301_03989_amd import pcprop
    rng = np.random.default_rng(5)
    n = 4099
    pert = W.planet_elements()
    r = rng.uniform(-1.2, 1.2, (3, n))
    r[:, :64] *= 0.3
    t = rng.uniform(-5.0, 30.0, n)
    a = pc.eval_force(torch.tensor(r, device="cuda"), torch.tensor(t, device="cuda"),
                      pcprop.Model(1.0, pert, 0.0)).cpu().numpy()
    m = oracle.Model(1.0, pert, 0.0)
    ref = np.stack([oracle.accel_t(r[:, i], t[i], m) for i in range(n)], axis=1)
    err = np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert np.median(err) < 1e-15 and err.max() < 1e-13, (np.median(err), err.max())


def test_kepler_matches_oracle(pc):
    w = W.uneven_batch(512, seed=9)
    rng = np.random.default_rng(1)
    dt = rng.uniform(-6.0, 6.0, w.n_ic)
    dt[:8] = 0.0
    y, ok = pc.eval_kepler(torch.tensor(w.ics.T.copy(), device="cuda"), torch.tensor(dt, device="cuda"))
    y, ok = y.cpu().numpy().T, ok.cpu().numpy()
    assert ok.all()
    ref = np.stack([oracle.kepler(w.ics[i], dt[i])[1] for i in range(w.n_ic)])
    assert rel_err(y, ref).max() < 1e-12
    np.testing.assert_array_equal(y[:8], w.ics[:8])
    _, ok2 = pc.eval_kepler(torch.tensor([[1.0], [0.0], [0.0], [0.0], [1.5], [0.0]], dtype=torch.float64, device="cuda"),
                            torch.tensor([1.0], dtype=torch.float64, device="cuda"))
    assert ok2.item() == 0


# ---------------------------------------------------------------------------
# whole path
# ---------------------------------------------------------------------------
def test_sun_only_kepler_ensemble(pc):
    w = W.sun_only_kepler()
    r, _ = _run(pc, w, want_nodes=True, want_bounds=True)
    o = oracle_run(w, want_nodes=True, want_bounds=True)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < TOL
    assert rel_err(r["nodes"].reshape(-1, 6), o["nodes"].reshape(-1, 6)).max() < TOL
    assert np.abs(r["iters"] - o["iters"]).max() <= 1
    # one period returns to the start (closed form)
    assert rel_err(r["states"], w.ics).max() < 1e-11


@pytest.mark.parametrize("n_ic", [1, 17, 250])
def test_nbody_subset_parity(pc, n_ic):
    w = W.nbody_venus(n_ic)
    r, _ = _run(pc, w, want_bounds=True)
    o = oracle_run(w, want_bounds=True)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < TOL
    assert np.abs(r["iters"] - o["iters"]).max() <= 1


def _many_bodies(n_pert):
    """The eight planets and, past eight, copies of them shifted in phase with other masses."""
    base = W.planet_elements()
    extra = base.copy()
    extra[:, 0] *= 0.37
    extra[:, 6] += 2.1
    return np.concatenate([base, extra])[:n_pert]


@pytest.mark.parametrize("n_pert,nodes,precision", [(5, 64, "fp64"), (16, 64, "fp64"), (16, 256, "fp64"),
                                                    (16, 256, "fp32-fp64"), (16, 128, "fp32-fp64")])
def test_perturber_counts_and_record_paths(pc, n_pert, nodes, precision):
    """Perturber counts that leave the four-body chunks ragged (5) and the maximum (16); at
    256 nodes with 16 bodies a segment's records exceed the LDS share and the kernels read
    them from global memory.  Both job shapes and the precision schedule."""
    w0 = W.nbody_venus(29, days=80.0, segments=2, nodes=nodes, tol=1e-12)
    w = W.Workload("many", w0.ics, w0.groups, _many_bodies(n_pert))
    r, _ = _run(pc, w, want_bounds=True, precision=precision)
    o = oracle_run(w, want_bounds=True)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < TOL
    if precision == "fp64":
        assert np.abs(r["iters"] - o["iters"]).max() <= 1
        p, _ = _run(pc, w, path="plain")
        assert rel_err(p["states"], o["states"]).max() < TOL
    if n_pert == 16:   # one body past the limit is refused
        from paper_2301_03989_amd import pcprop
        with pytest.raises(pcprop.PcError) as e:
            _run(pc, W.Workload("too-many", w0.ics, w0.groups, np.concatenate([w.pert, w.pert[:1]])))
        assert e.value.code == pcprop.PC_EINVAL


def test_fixed_iterations_agree_to_rounding(pc):
    w = W.nbody_venus(40)
    r, _ = _run(pc, w, fixed_iters=6, want_nodes=True)
    o = oracle_run(w, fixed_iters=6, want_nodes=True)
    assert (r["iters"] == 6).all() and (o["iters"] == 6).all()
    assert rel_err(r["nodes"].reshape(-1, 6), o["nodes"].reshape(-1, 6)).max() < 1e-12


@pytest.mark.parametrize("nodes", [3, 5, 16, 40, 64, 200, 256])
def test_node_counts_and_padding(pc, nodes):
    w = W.nbody_venus(21, days=60.0, segments=2, nodes=nodes, tol=1e-12)
    kw = {}
    if nodes < 40:   # few nodes cannot reach 1e-12 over 30 days: compare fixed sweeps instead
        kw = dict(fixed_iters=8)
    r, _ = _run(pc, w, **kw)
    o = oracle_run(w, **kw)
    assert rel_err(r["states"], o["states"]).max() < (1e-12 if kw else TOL)
    assert np.abs(r["iters"] - o["iters"]).max() <= 1


@pytest.mark.parametrize("nodes", [17, 33, 65, 129])
def test_node_counts_just_past_a_power_of_two(pc, nodes):
    """One node past a power of two pads to twice the count; the products stop after the
    last 16-node block holding a node (K_N is zero past N), the shortest k range against
    the padded one.  First-order FP64 sweeps, the precision schedule and second-order
    sweeps against the oracle."""
    w = W.nbody_venus(21, seed=300 + nodes, days=40.0, segments=2, nodes=nodes, tol=1e-12)
    kw = dict(fixed_iters=8) if nodes < 40 else {}
    print(f"past a power of two: N {nodes} {kw}", flush=True)
    r, _ = _run(pc, w, **kw)
    o = oracle_run(w, **kw)
    assert rel_err(r["states"], o["states"]).max() < (1e-12 if kw else TOL)
    assert np.abs(r["iters"] - o["iters"]).max() <= 1
    if not kw:
        m, _ = _run(pc, w, precision="fp32-fp64")
        assert rel_err(m["states"], o["states"]).max() < 1e-11
        r2, _ = _run(pc, w, order=2)
        o2 = oracle_run(w, order=2)
        assert rel_err(r2["states"], o2["states"]).max() < TOL
        assert np.abs(r2["iters"] - o2["iters"]).max() <= 1


def test_degenerate_and_ragged_batches(pc):
    """Smallest and most ragged shapes in one call: a single IC at the minimum of three
    nodes and one segment, a single IC at 256 nodes (seven idle columns of its 8-IC job),
    one IC more than a 16-IC block at 16 nodes, and a two-IC group going backward."""
    base = W.nbody_venus(21)
    day = 1.0 / W.TU_DAYS
    groups = [W.Group(0, 1, 0.0, 2.0 * day, 3, 1, 1e-12),
              W.Group(1, 1, 0.0, 40.0 * day, 256, 1, 1e-12),
              W.Group(2, 17, 0.0, 30.0 * day, 16, 3, 1e-12),
              W.Group(19, 2, 10.0 * day, -20.0 * day, 64, 2, 1e-12)]
    w = W.Workload("degenerate", base.ics, groups, base.pert)
    r, _ = _run(pc, w)
    o = oracle_run(w)
    assert (r["iters"][:, 0] > 0).all() and r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL
    assert np.abs(r["iters"] - o["iters"]).max() <= 1


def test_empty_and_malformed_batches_are_refused(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(8)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch)
    g = w.groups[0]
    bad = [
        [],                                                                        # no groups
        [pcprop.Group(0, 0, g.t0, g.tf, g.nodes, g.segments, g.tol)],              # empty group
        [pcprop.Group(0, 8, g.t0, g.tf, 257, g.segments, g.tol)],                  # too many nodes
        [pcprop.Group(0, 8, g.t0, g.tf, 2, g.segments, g.tol)],                    # too few nodes
        [pcprop.Group(4, 8, g.t0, g.tf, g.nodes, g.segments, g.tol)],              # past the ICs
        [pcprop.Group(0, 8, g.t0, g.t0, g.nodes, g.segments, g.tol)],              # empty span
        [pcprop.Group(0, 8, g.t0, g.tf, g.nodes, g.segments, 0.0)],                # no tolerance
    ]
    for groups in bad:
        with pytest.raises((pcprop.PcError, ValueError)):
            pc.propagate_batched(ics, groups, model)
    with pytest.raises((pcprop.PcError, ValueError)):
        pc.propagate_batched(ics[:0], [pcprop.Group(0, 1, g.t0, g.tf, g.nodes, g.segments, g.tol)], model)


def test_tile_shapes_agree(pc):
    w = W.nbody_venus(40, nodes=128)
    a, _ = _run(pc, w, tile_pairs=2048)
    b, _ = _run(pc, w, tile_pairs=1024)
    assert rel_err(a["states"], b["states"]).max() < 1e-13


def test_backward_and_cold_start(pc):
    w = W.nbody_venus(24)
    g = w.groups[0]
    fwd, _ = _run(pc, w)
    wb = W.Workload("back", fwd["states"], [W.Group(0, 24, g.tf, g.t0, g.nodes, g.segments, 1e-13)], w.pert)
    back, _ = _run(pc, wb)
    o = oracle_run(wb)
    assert rel_err(back["states"], o["states"]).max() < TOL
    assert rel_err(back["states"], w.ics).max() < 1e-9
    wc = W.nbody_venus(24, days=56.25, segments=1)
    wc.init = 1
    c, _ = _run(pc, wc)
    oc = oracle_run(wc)
    assert rel_err(c["states"], oc["states"]).max() < TOL
    assert np.abs(c["iters"] - oc["iters"]).max() <= 1


def test_mixed_groups_one_call(pc):
    w = W.uneven_batch(600, seed=21)
    # shorten the spans for the oracle: keep the group shapes, 1-3 segments each
    for g in w.groups:
        g.segments = 1 + g.segments // 16
        g.tf = g.segments * np.pi / 4.0
    idx = np.concatenate([np.arange(g.ic_offset, g.ic_offset + min(g.n_ic, 9)) for g in w.groups])
    r, sub = _run(pc, w, idx)
    o = oracle_run(sub)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL
    assert np.abs(r["iters"] - o["iters"]).max() <= 1


def test_batch_composition_invariance(pc):
    w = W.nbody_venus(64)
    a, _ = _run(pc, w)
    perm = np.random.default_rng(0).permutation(64)
    wp = W.Workload("perm", w.ics[perm], w.groups, w.pert)
    b, _ = _run(pc, wp)
    # same IC, different batch-mates: results agree to rounding; convergence is per IC
    assert rel_err(b["states"], a["states"][perm]).max() < 1e-13
    one, _ = _run(pc, w, idx=[5])
    assert rel_err(one["states"], a["states"][5:6]).max() < 1e-13


def test_status_codes(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(20)
    r, _ = _run(pc, w, max_iter=1)
    assert r["status"] == pcprop.PC_ENOTCONV and (r["iters"] == -1).all()
    bad = w.ics.copy()
    bad[3, 1] = np.nan
    wb = W.Workload("bad", bad, w.groups, w.pert)
    r, _ = _run(pc, wb)
    assert r["status"] == pcprop.PC_ENONFINITE
    assert (r["iters"][3] == -2).all() and np.isnan(r["states"][3]).all()
    ok = np.delete(np.arange(20), 3)
    assert (r["iters"][ok] > 0).all()
    with pytest.raises(pcprop.PcError):
        pc.propagate(torch.tensor(w.ics, device="cuda"), 0.0, 0.0, 128, 8, 1e-12)
    with pytest.raises(pcprop.PcError):
        pc.propagate(torch.tensor(w.ics, device="cuda"), 0.0, 1.0, 2, 8, 1e-12)
    with pytest.raises(pcprop.PcError):
        pc.propagate(torch.tensor(w.ics, device="cuda"), 0.0, 1.0, 64, 0, 1e-12)


def test_full_size_nbody_sampled(pc):
    """The full 4096-IC N-body Venus ensemble in the launch configuration the benchmark
    times; every 64th IC is checked against the oracle."""
    w = W.nbody_venus()
    r, _ = _run(pc, w)
    assert r["status"] == 0
    idx = np.arange(0, w.n_ic, 64)
    o = oracle_run(w, idx)
    assert rel_err(r["states"][idx], o["states"]).max() < TOL
    assert np.abs(r["iters"][idx] - o["iters"]).max() <= 1


# ---------------------------------------------------------------------------
# plain path: per-iteration kernels and host loop
# ---------------------------------------------------------------------------
def test_plain_path_matches_oracle(pc):
    w = W.nbody_venus(250)
    r, _ = _run(pc, w, path="plain", want_bounds=True)
    o = oracle_run(w, want_bounds=True)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < TOL
    assert np.abs(r["iters"] - o["iters"]).max() <= 1


def test_plain_and_fused_agree(pc):
    w = W.nbody_venus(40)
    a, _ = _run(pc, w, fixed_iters=7, want_nodes=True)
    b, _ = _run(pc, w, fixed_iters=7, want_nodes=True, path="plain")
    # same discrete map and operation order per product; the two kernels differ only in
    # where the compiler contracts multiply-adds, a rounding-level difference that the
    # 8 chained segments amplify to a few 1e-14
    assert rel_err(a["nodes"].reshape(-1, 6), b["nodes"].reshape(-1, 6)).max() < 1e-13
    c, _ = _run(pc, w)
    d, _ = _run(pc, w, path="plain")
    assert rel_err(c["states"], d["states"]).max() < 1e-13
    assert np.abs(c["iters"] - d["iters"]).max() <= 1


def test_plain_path_groups_and_status(pc):
    from paper_2301_03989_amd import pcprop
    w = W.uneven_batch(600, seed=21)
    for g in w.groups:
        g.segments = 1 + g.segments // 16
        g.tf = g.segments * np.pi / 4.0
    idx = np.concatenate([np.arange(g.ic_offset, g.ic_offset + min(g.n_ic, 5)) for g in w.groups])
    r, sub = _run(pc, w, idx, path="plain")
    o = oracle_run(sub)
    assert rel_err(r["states"], o["states"]).max() < TOL
    wn = W.nbody_venus(20)
    bad = wn.ics.copy()
    bad[3, 1] = np.nan
    r, _ = _run(pc, W.Workload("bad", bad, wn.groups, wn.pert), path="plain")
    assert r["status"] == pcprop.PC_ENONFINITE and (r["iters"][3] == -2).all()
    r, _ = _run(pc, wn, path="plain", max_iter=1)
    assert r["status"] == pcprop.PC_ENOTCONV and (r["iters"] == -1).all()


# ---------------------------------------------------------------------------
# graph capture and autotuner
# ---------------------------------------------------------------------------
def test_graph_replays_match_eager(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(300)
    g = w.groups[0]
    ics = torch.tensor(w.ics, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    model = pcprop.Model(1.0, w.pert, 0.0)
    ref = pc.propagate_batched(ics, groups, model)
    ref_s, ref_i = ref["states"].clone(), ref["iters"].clone()
    out = torch.empty_like(ref_s)
    for rep in range(4):
        r = pc.propagate_batched(ics, groups, model, graph=True, out=out)
        assert r["status"] == 0
        assert torch.equal(r["states"], ref_s), rep
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        assert torch.isfinite(x.sum())
        torch.cuda.synchronize()
    # same pointers, new contents: the replay reads the current inputs
    ics2 = torch.tensor(W.nbody_venus(300, seed=77).ics, device="cuda")
    ics.copy_(ics2)
    r = pc.propagate_batched(ics, groups, model, graph=True, out=out)
    ref2 = pc.propagate_batched(ics, groups, model)
    assert torch.equal(r["states"], ref2["states"])
    o = oracle_run(W.Workload("seed77", ics2.cpu().numpy(), w.groups, w.pert), np.arange(0, 300, 50))
    assert rel_err(r["states"].cpu().numpy()[::50], o["states"]).max() < TOL


def test_graph_recaptured_when_the_staging_buffer_grows(pc):
    """A captured graph copies its tables from the context's pinned staging buffer; a call
    that needs a larger buffer reallocates it, and the next graph call with the same
    signature must be captured again rather than replay copies from the freed buffer."""
    from paper_2301_03989_amd import pcprop
    ctx = pcprop.Context(0)
    w = W.nbody_venus(64, days=112.5, segments=2)
    g = w.groups[0]
    ics = torch.tensor(w.ics, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    model = pcprop.Model(1.0, w.pert, 0.0)
    ref = ctx.propagate_batched(ics, groups, model)["states"].clone()
    # every output pointer is part of the replay signature: keep all of them across calls
    out = torch.empty_like(ref)
    iters = torch.zeros((w.n_ic, g.segments), dtype=torch.int32, device="cuda")
    c0 = ctx.graph_captures()
    for _ in range(2):
        r = ctx.propagate_batched(ics, groups, model, graph=True, out=out, iters_out=iters)
        assert r["status"] == 0 and torch.equal(r["states"], ref)
    assert ctx.graph_captures() == c0 + 1
    # 40000 one-IC groups of 3 nodes: descriptor tables beyond the 4 MiB staging buffer
    n_big = 40000
    big = torch.tensor(np.tile(w.ics[:1], (n_big, 1)), device="cuda")
    bgroups = [pcprop.Group(i, 1, 0.0, 0.05, 3, 1, 1e-12) for i in range(n_big)]
    rb = ctx.propagate_batched(big, bgroups, pcprop.Model(1.0, None, 0.0))
    assert rb["status"] == 0
    r = ctx.propagate_batched(ics, groups, model, graph=True, out=out, iters_out=iters)
    assert ctx.graph_captures() == c0 + 2
    assert r["status"] == 0 and torch.equal(r["states"], ref)


def test_autotune_records_a_shape(pc):
    from paper_2301_03989_amd import pcprop
    ctx = pcprop.Context(0)
    w = W.nbody_venus(512)
    g = w.groups[0]
    ics = torch.tensor(w.ics, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    model = pcprop.Model(1.0, w.pert, 0.0)
    ref = ctx.propagate_batched(ics, groups, model)
    chosen = ctx.autotune(ics, groups, model)
    assert chosen in (1024, 2048)
    assert ctx.tile_pairs(128) == chosen
    assert ctx.job_list(128) in (0, 1, 2, 4, 8)
    a = ctx.propagate_batched(ics, groups, model)
    b = ctx.propagate_batched(ics, groups, model, tile_pairs=2048)
    assert rel_err(a["states"].cpu().numpy(), b["states"].cpu().numpy()).max() < 1e-13
    assert rel_err(a["states"].cpu().numpy(), ref["states"].cpu().numpy()).max() < 1e-13
    ctx.set_tile_pairs(128, 0)
    assert ctx.tile_pairs(128) == 0
    with pytest.raises(pcprop.PcError):
        ctx.set_tile_pairs(256, 1024)
    with pytest.raises(pcprop.PcError):
        ctx.set_job_list(128, 3)


def test_autotune_per_node_count_job_lengths(pc):
    """On a batch of three node counts the tuner records a job length per padded node
    count; results do not depend on the job length (columns are refilled with further ICs
    of the same segment, each IC's iteration is unchanged)."""
    from paper_2301_03989_amd import pcprop
    ctx = pcprop.Context(0)
    w = W.uneven_batch(3000, seed=41)
    for gr in w.groups:
        gr.segments = 1 + gr.segments // 16
        gr.tf = gr.segments * np.pi / 4.0
    ics = torch.tensor(w.ics, device="cuda")
    groups = [pcprop.Group(gr.ic_offset, gr.n_ic, gr.t0, gr.tf, gr.nodes, gr.segments, gr.tol) for gr in w.groups]
    model = pcprop.Model(1.0, w.pert, 0.0)
    ref = ctx.propagate_batched(ics, groups, model)
    ctx.autotune(ics, groups, model)
    assert ctx.tile_pairs(256) == 2048
    for np_ in (64, 128, 256):
        assert ctx.job_list(np_) in (0, 1, 2, 4, 8)
    ctx.set_job_list(64, 8)
    ctx.set_job_list(128, 1)
    ctx.set_job_list(256, 4)
    for r in (ctx.propagate_batched(ics, groups, model), ):
        assert r["status"] == 0
        assert np.array_equal(r["iters"].cpu().numpy(), ref["iters"].cpu().numpy())
        assert rel_err(r["states"].cpu().numpy(), ref["states"].cpu().numpy()).max() < 1e-13


# ---------------------------------------------------------------------------
# precision schedule: FP32 sweeps, then FP64 sweeps to the FP64 fixed point
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_ic", [7, 250])
def test_fp32_then_fp64_matches_fp64_oracle(pc, n_ic):
    w = W.nbody_venus(n_ic, seed=104)
    r, _ = _run(pc, w, precision="fp32-fp64", want_bounds=True)
    o = oracle_run(w, want_bounds=True)
    assert r["status"] == 0
    err = rel_err(r["states"], o["states"])
    assert err.max() < TOL, err.max()
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < TOL
    assert (r["iters"] >= 2).all()
    # increment jobs (16-IC columns at 128 nodes): increment sweeps converge at the Picard
    # rate until no IC of the job changes by more than tol, then every IC stops on an FP64
    # sweep that changed it by less than tol: near the FP64 iteration's accuracy, mostly one
    # sweep after the FP64 iteration stops (more where the job's slowest IC holds it)
    assert err.max() < 1e-11, err.max()
    d = r["iters"] - o["iters"]
    assert d.min() >= -1 and d.max() <= 3, (d.min(), d.max())
    assert d.mean() <= 1.5, d.mean()


@pytest.mark.parametrize("nodes", [48, 100, 200])
def test_fp32_then_fp64_padded_nodes_and_nonfinite_ic(pc, nodes):
    """Increment sweeps on job shapes padded past N (48 of 64, 100 of 128 and 200 of 256
    nodes: rows past N of the force array, written by the FP32 sweeps, meet zero operator
    columns once FP64 sweeps resume), with a non-finite IC in the job."""
    w = W.nbody_venus(40, seed=105, nodes=nodes, segments=2, days=112.5)
    w.ics = w.ics.copy()
    w.ics[3, 1] = np.nan
    r, _ = _run(pc, w, precision="fp32-fp64")
    o = oracle_run(w)
    assert (r["iters"][3] == -2).all() and np.isnan(r["states"][3]).all()
    ok = np.arange(w.n_ic) != 3
    assert (r["iters"][ok] > 0).all()
    err = rel_err(r["states"][ok], o["states"][ok])
    assert err.max() < 1e-11, err.max()


def test_fp32_then_fp64_node_row_jobs(pc):
    """Increment sweeps on 8-IC jobs (256 nodes, node-row layout: lane pairs exchange the
    position and its change for the gravity gradient) against the FP64 oracle, with the
    same bars as the 128-node jobs."""
    w = W.nbody_venus(60, seed=106, nodes=256, segments=4, days=225.0)
    r, _ = _run(pc, w, precision="fp32-fp64", want_bounds=True)
    o = oracle_run(w, want_bounds=True)
    assert r["status"] == 0
    err = rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6))
    assert err.max() < 1e-11, err.max()
    d = r["iters"] - o["iters"]
    assert d.min() >= -1 and d.max() <= 3, (d.min(), d.max())
    assert d.mean() <= 1.5, d.mean()


def test_fp32_then_fp64_mixed_groups(pc):
    w = W.uneven_batch(600, seed=22)
    for g in w.groups:
        g.segments = 1 + g.segments // 16
        g.tf = g.segments * np.pi / 4.0
    idx = np.concatenate([np.arange(g.ic_offset, g.ic_offset + min(g.n_ic, 6)) for g in w.groups])
    r, sub = _run(pc, w, idx, precision="fp32-fp64")
    o = oracle_run(sub)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL


@pytest.mark.parametrize("conv", ["ic", "group"])
def test_plain_path_on_several_streams(pc, conv):
    """The outer level on several streams (Sec. 5.4): 15 groups spread over 2, 4 and 16
    streams, all driven from the calling thread, give the one-stream results bit for bit,
    with the per-IC and the group-max rule."""
    from paper_2301_03989_amd import pcprop
    w = W.uneven_batch(450, seed=23)
    for g in w.groups:
        g.segments = 1 + g.segments // 16
        g.tf = g.segments * np.pi / 4.0
    a, _ = _run(pc, w, path="plain", conv=conv)
    assert a["status"] == 0
    for ns in (2, 4, 16):
        b, _ = _run(pc, w, path="plain", conv=conv, streams=ns)
        assert np.array_equal(a["states"], b["states"]), ns
        assert np.array_equal(a["iters"], b["iters"]), ns
    with pytest.raises(pcprop.PcError):
        _run(pc, w, streams=2)                  # fused path: one launch, no streams
    with pytest.raises(pcprop.PcError):
        _run(pc, w, path="plain", streams=17)


def test_fp32_then_fp64_rejected_on_plain_path(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(4)
    with pytest.raises(pcprop.PcError):
        _run(pc, w, precision="fp32-fp64", path="plain")


# ---------------------------------------------------------------------------
# every register layout of the job shapes, node by node
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nodes,tile", [(12, 2048), (24, 2048), (48, 2048), (100, 2048), (200, 2048),
                                        (48, 1024), (100, 1024)])
def test_node_states_every_job_shape(pc, nodes, tile):
    """Node outputs at fixed sweeps for NP = 16 .. 256 (16 to 128 ICs per job, transposed
    blocks; 8 ICs per job, node-row blocks) with a ragged IC count, against the oracle."""
    w = W.nbody_venus(37, seed=31, days=40.0, segments=2, nodes=nodes)
    r, _ = _run(pc, w, fixed_iters=6, want_nodes=True, want_bounds=True, tile_pairs=tile)
    o = oracle_run(w, fixed_iters=6, want_nodes=True, want_bounds=True)
    assert rel_err(r["nodes"].reshape(-1, 6), o["nodes"].reshape(-1, 6)).max() < 1e-12
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < 1e-12
    assert (r["iters"] == 6).all()


# ---------------------------------------------------------------------------
# jobs with more ICs than columns (refilled columns) against one-block jobs
# ---------------------------------------------------------------------------
def _eccentric(n, seed, nodes, segments, tol=1e-12):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.7, 1.0, n)
    e = rng.uniform(0.0, 0.6, n)
    inc = rng.uniform(0.0, 10.0, n) * W.DEG
    raan, argp, M = (rng.uniform(0.0, 360.0, n) * W.DEG for _ in range(3))
    ics = W.elements_to_states(a, e, inc, raan, argp, M)
    return W.Workload("ecc", ics, [W.Group(0, n, 0.0, segments * np.pi / 4, nodes, segments, tol)],
                      W.planet_elements())


@pytest.mark.parametrize("tile, list_, precision", [(1024, 1, "fp64"), (2048, 1, "fp64"), (2048, 4, "fp64"),
                                                   (2048, 1, "fp32-fp64")])
def test_absolute_tolerance_mode(pc, tile, list_, precision):
    """The absolute stopping rule (tol on |dr| and |dv| at every node) on 8-IC, 16-IC and
    refilled-column jobs and under the precision schedule, against the oracle's absolute
    mode.  On these eccentric orbits (|r| from 0.3 to 1.6) the absolute rule stops other
    ICs at other sweeps than the relative rule."""
    w = _eccentric(70, 5, 64, 4, tol=1e-11)
    r, _ = _run(pc, w, tol_mode="abs", tile_pairs=tile, job_list=list_, precision=precision, want_bounds=True)
    o = oracle_run(w, tol_mode=1, want_bounds=True)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < TOL
    if precision == "fp64":
        # (under the precision schedule an IC also takes its job's FP32 sweeps: counts differ)
        assert np.abs(r["iters"] - o["iters"]).max() <= 1
    assert (oracle_run(w)["iters"] != o["iters"]).any()


def _two_groups(tol=1e-11):
    """70 eccentric ICs in two groups (48 nodes x 3 segments, 64 nodes x 2 segments)."""
    w = _eccentric(70, 13, 48, 3, tol)
    h = np.pi / 4
    groups = [W.Group(0, 40, 0.0, 3 * h, 48, 3, tol), W.Group(40, 30, 0.0, 2 * h, 64, 2, tol)]
    return W.Workload("ecc2", w.ics, groups, w.pert)


@pytest.mark.parametrize("tol_mode", ["rel", "abs"])
def test_group_max_convergence_matches_oracle(pc, tol_mode):
    """Group-max stopping rule on the plain path: one sweep count per group and segment,
    the oracle's group count within one sweep, states within the parity bar; the per-IC
    rule stops some ICs earlier on the same inputs."""
    w = _two_groups()
    r, _ = _run(pc, w, path="plain", conv="group", tol_mode=tol_mode, want_bounds=True)
    o = oracle_run(w, conv=1, tol_mode=0 if tol_mode == "rel" else 1, want_bounds=True)
    assert r["status"] == 0
    for g in w.groups:
        sl = slice(g.ic_offset, g.ic_offset + g.n_ic)
        it = r["iters"][sl, :g.segments]
        assert (it == it[0]).all()
        assert np.abs(it[0] - o["iters"][sl, :g.segments][0]).max() <= 1
        b, ob = r["bounds"][sl, :g.segments + 1], o["bounds"][sl, :g.segments + 1]
        assert rel_err(b.reshape(-1, 6), ob.reshape(-1, 6)).max() < TOL
    assert rel_err(r["states"], o["states"]).max() < TOL
    # first segment (same start for both rules): every IC's own first sweep below tol comes
    # no later than the group's
    per_ic, _ = _run(pc, w, path="plain", tol_mode=tol_mode)
    assert (per_ic["iters"][:, 0] <= r["iters"][:, 0]).all() and (per_ic["iters"][:, 0] < r["iters"][:, 0]).any()


def test_group_max_status_and_rejections(pc):
    from paper_2301_03989_amd import pcprop
    w = _two_groups()
    bad = w.ics.copy()
    bad[5, 2] = np.inf
    r, _ = _run(pc, W.Workload("bad", bad, w.groups, w.pert), path="plain", conv="group")
    o = oracle_run(W.Workload("bad", bad, w.groups, w.pert), conv=1)
    assert r["status"] == pcprop.PC_ENONFINITE and (r["iters"][5, :3] == -2).all()
    keep = np.arange(w.n_ic) != 5
    assert np.abs(r["iters"][keep] - o["iters"][keep]).max() <= 1
    assert rel_err(r["states"][keep], o["states"][keep]).max() < TOL
    r, _ = _run(pc, w, path="plain", conv="group", max_iter=3)
    assert r["status"] == pcprop.PC_ENOTCONV
    for g in w.groups:
        assert (r["iters"][g.ic_offset:g.ic_offset + g.n_ic, :g.segments] == -1).all()
    o = oracle_run(w, fixed_iters=3)
    assert rel_err(r["states"], o["states"]).max() < 1e-12
    with pytest.raises(pcprop.PcError) as e:
        _run(pc, w, conv="group")
    assert e.value.code == pcprop.PC_EINVAL


@pytest.mark.parametrize("nodes,list_", [(24, 8), (64, 2), (100, 4), (128, 8), (200, 4)])
def test_refilled_columns_match_one_block_jobs(pc, nodes, list_):
    """Every IC's iterates do not depend on which column or job runs it: refilled-column
    jobs give the one-block results (states, node states, checkpoints, sweep records), with
    a ragged IC count and non-finite ICs among them.  Bit for bit on the transposed shapes
    (up to 128 nodes); at 256 nodes the two job bodies are compiled with different
    multiply-add contractions, so there the bar is rounding (1e-13)."""
    w = _eccentric(301, 41, nodes, 3)
    w.ics[[5, 77, 200]] = np.nan
    a, _ = _run(pc, w, want_nodes=True, want_bounds=True, job_list=1)
    b, _ = _run(pc, w, want_nodes=True, want_bounds=True, job_list=list_)
    assert a["status"] == b["status"]
    np.testing.assert_array_equal(a["iters"], b["iters"])
    for k in ("states", "nodes", "bounds"):
        np.testing.assert_array_equal(np.isnan(a[k]), np.isnan(b[k]))
        if nodes <= 128:
            np.testing.assert_array_equal(np.nan_to_num(a[k]), np.nan_to_num(b[k]))
        else:
            fin = np.isfinite(a[k]).reshape(-1, 6).all(axis=1)
            x, y = a[k].reshape(-1, 6)[fin], b[k].reshape(-1, 6)[fin]
            keep = np.linalg.norm(x[:, :3], axis=1) > 0   # unused node slots are zero
            assert rel_err(y[keep], x[keep]).max() < 1e-13
    assert (a["iters"][[5, 77, 200]] == -2).all()


def test_refilled_columns_against_oracle_and_fixed_sweeps(pc):
    w = _eccentric(150, 42, 64, 4)
    r, _ = _run(pc, w, want_bounds=True, job_list=4)
    o = oracle_run(w, want_bounds=True)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < TOL
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < TOL
    assert np.abs(r["iters"] - o["iters"]).max() <= 1
    f, _ = _run(pc, w, fixed_iters=5, job_list=8)
    assert (f["iters"] == 5).all()
    of = oracle_run(w, fixed_iters=5)
    assert rel_err(f["states"], of["states"]).max() < 1e-12


def test_refilled_columns_mixed_groups_and_status(pc):
    """An uneven batch (three node counts, uneven sizes) with automatic job lists, and a
    max_iter too small to converge (status and records as on one-block jobs)."""
    w = W.uneven_batch(2000, seed=23)
    for g in w.groups:
        g.segments = 1 + g.segments // 20
        g.tf = g.segments * np.pi / 4.0
    a, _ = _run(pc, w, job_list=1)
    b, _ = _run(pc, w, job_list=0)
    assert rel_err(b["states"], a["states"]).max() < 1e-13
    np.testing.assert_array_equal(a["iters"], b["iters"])
    c, _ = _run(pc, w, job_list=1, max_iter=3)
    d, _ = _run(pc, w, job_list=4, max_iter=3)
    assert c["status"] == d["status"] == 2
    np.testing.assert_array_equal(c["iters"], d["iters"])
    assert rel_err(d["states"], c["states"]).max() < 1e-13
