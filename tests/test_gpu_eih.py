"""The Einstein-Infeld-Hoffmann dynamics on the HIP path against the oracle's (the
relativistic restricted problem of Sec. 5.4.1): every job shape (transposed and 8-column),
physical and exaggerated 1/c^2, backward propagation, node states, the precision schedule,
graph replays, and the calls it refuses."""
import numpy as np
import pytest
import torch

import oracle
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


def _run(pc, w, **kw):
    from paper_2301_03989_amd import pcprop
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    r = pc.propagate_batched(ics, groups, model, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


def _venus(n, nodes, inv_c2, days=112.5, segments=2, seed=106):
    w = W.nbody_venus(n, seed=seed, days=days, segments=segments, nodes=nodes)
    w.inv_c2 = inv_c2
    return w


@pytest.mark.parametrize("nodes,tile", [(16, 2048), (48, 2048), (64, 2048), (100, 2048), (128, 2048),
                                        (200, 2048), (256, 2048), (64, 1024), (40, 1024), (128, 1024)])
@pytest.mark.parametrize("inv_c2", [1e-4, 1.0 / W.C_AU_TU**2])
def test_eih_matches_oracle(pc, nodes, tile, inv_c2):
    w = _venus(40, nodes, inv_c2)
    r = _run(pc, w, tile_pairs=tile)
    o = oracle_run(w)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < 1e-11
    assert np.abs(r["iters"] - o["iters"]).max() <= 1


def test_eih_differs_from_point_masses_as_the_oracle_does(pc):
    """With an exaggerated 1/c^2 the relativistic result is far from the point-mass one,
    by the same amount on both sides."""
    w = _venus(24, 64, 1e-4)
    w0 = _venus(24, 64, 0.0)
    d_gpu = rel_err(_run(pc, w)["states"], _run(pc, w0)["states"])
    d_orc = rel_err(oracle_run(w)["states"], oracle_run(w0)["states"])
    assert d_gpu.min() > 1e-6
    assert np.abs(d_gpu - d_orc).max() < 1e-10


def test_eih_node_states_backward_and_sun_only(pc):
    w = _venus(20, 64, 1e-4)
    r = _run(pc, w, want_nodes=True, want_bounds=True)
    o = oracle_run(w, want_nodes=True, want_bounds=True)
    n = r["nodes"][:, :, :64].reshape(-1, 6)
    assert rel_err(n, o["nodes"].reshape(-1, 6)).max() < 1e-11
    assert rel_err(r["bounds"].reshape(-1, 6), o["bounds"].reshape(-1, 6)).max() < 1e-11
    # backward: from the end states back to the start
    wb = _venus(20, 64, 1e-4)
    g = wb.groups[0]
    wb.ics = r["states"].copy()
    g.t0, g.tf = g.tf, g.t0
    rb = _run(pc, wb)
    assert rel_err(rb["states"], w.ics).max() < 1e-9
    assert rel_err(rb["states"], oracle_run(wb)["states"]).max() < 1e-11
    # Sun only: no perturber records
    ws = _venus(20, 48, 1e-3)
    ws.pert = np.zeros((0, 7))
    assert rel_err(_run(pc, ws)["states"], oracle_run(ws)["states"]).max() < 1e-11


@pytest.mark.parametrize("nodes,inv_c2,extra", [(64, 1.0 / W.C_AU_TU**2, 3), (128, 1.0 / W.C_AU_TU**2, 3),
                                                (100, 1e-6, 3), (64, 1e-4, 15), (256, 1.0 / W.C_AU_TU**2, 12)])
def test_eih_precision_schedule(pc, nodes, inv_c2, extra):
    """FP32 -> FP64 schedule with the relativistic model: the FP64 sweeps evaluate it, the
    increment sweeps linearise with the point-mass gradient; every IC still stops on an
    FP64 sweep, near the FP64 iteration's accuracy.  The gradient misses the O(1/c^2)
    terms, so an exaggerated 1/c^2 (1e-4) leaves the increments' limit farther off and
    more FP64 sweeps follow (a CPU prototype of the schedule needed the same)."""
    w = _venus(40, nodes, inv_c2)
    r = _run(pc, w, precision="fp32-fp64")
    o = oracle_run(w)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < 1e-11
    d = r["iters"] - o["iters"]
    assert d.min() >= -1 and d.max() <= extra, (d.min(), d.max())


@pytest.mark.parametrize("nodes", [64, 128, 256])
def test_eih_plain_path(pc, nodes):
    """The per-iteration (plain) path with the relativistic force kernel: against the
    oracle, and against the fused path."""
    w = _venus(40, nodes, 1.0 / W.C_AU_TU**2)
    r = _run(pc, w, path="plain")
    f = _run(pc, w)
    o = oracle_run(w)
    assert r["status"] == 0
    assert rel_err(r["states"], o["states"]).max() < 1e-11
    assert rel_err(r["states"], f["states"]).max() < 1e-13
    assert np.abs(r["iters"] - o["iters"]).max() <= 1


def test_eih_refused_where_not_supported(pc):
    from paper_2301_03989_amd import pcprop
    w = _venus(8, 64, 1e-8)
    for kw in (dict(path="plain", conv="group"),):
        with pytest.raises(pcprop.PcError):
            _run(pc, w, **kw)
    with pytest.raises(pcprop.PcError):
        _run(pc, _venus(8, 64, -1e-8))
    with pytest.raises(pcprop.PcError):
        pc.eval_force(torch.zeros((3, 4), dtype=torch.float64, device="cuda") + 0.7,
                      torch.zeros(4, dtype=torch.float64, device="cuda"),
                      pcprop.Model(1.0, w.pert, 0.0, 1e-8))
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    g = w.groups[0]
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    with pytest.raises(pcprop.PcError):   # order 2 is refused with the relativistic model
        pc.propagate_batched(ics, groups, pcprop.Model(1.0, w.pert, 0.0, 1e-8), order=2)


def test_eih_graph_replay_and_model_switch(pc):
    """Captured and replayed calls equal eager ones; changing only 1/c^2 between calls of
    the same shapes and pointers re-captures (the model is part of the graph's key)."""
    from paper_2301_03989_amd import pcprop
    w = _venus(24, 64, 1e-4)
    g = w.groups[0]
    ics = torch.tensor(w.ics, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    m1 = pcprop.Model(1.0, w.pert, 0.0, 1e-4)
    m0 = pcprop.Model(1.0, w.pert, 0.0, 0.0)
    ref1 = pc.propagate_batched(ics, groups, m1)["states"].clone()
    ref0 = pc.propagate_batched(ics, groups, m0)["states"].clone()
    assert not torch.equal(ref1, ref0)
    out = torch.empty_like(ref1)
    for rep in range(3):
        r = pc.propagate_batched(ics, groups, m1, graph=True, out=out)
        assert r["status"] == 0 and torch.equal(r["states"], ref1), rep
        r = pc.propagate_batched(ics, groups, m0, graph=True, out=out)
        assert r["status"] == 0 and torch.equal(r["states"], ref0), rep
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        assert torch.isfinite(x.sum())
        torch.cuda.synchronize()
