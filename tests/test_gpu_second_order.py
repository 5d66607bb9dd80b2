"""Second-order sweeps on the HIP path against the oracle's second-order form.

The second-order form (velocity and position both integrated from the acceleration
fit, the position twice) is the development of the method that Sec. 1 cites as
applicable to the augmented system and Sec. 7 expects a further speed-up from.  Bar:
1e-10 relative at every segment boundary against the oracle run with order 2; the
sweep counts within one; fixed sweeps agree to rounding.
"""
import numpy as np
import pytest

import oracle
from paper_2301_03989_amd import workloads as W
from tests._parity import boundary_err, rel_err

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


def _gpu(pc, w, **kw):
    from paper_2301_03989_amd import pcprop
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    kw.setdefault("init", "kepler" if w.init == 0 else "cold")
    r = pc.propagate_batched(ics, groups, model, want_bounds=True, order=2, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


def _oracle(w, **kw):
    S = max(g.segments for g in w.groups)
    st = np.zeros((w.n_ic, 6))
    it = np.zeros((w.n_ic, S), dtype=np.int32)
    bd = np.zeros((w.n_ic, S + 1, 6))
    m = oracle.Model(w.mu_sun, w.pert, w.epoch)
    for g in w.groups:
        sl = slice(g.ic_offset, g.ic_offset + g.n_ic)
        a, b, c = oracle.propagate(w.ics[sl], g.t0, g.tf, g.nodes, g.segments, g.tol, m, init=w.init,
                                   want_bounds=True, order=2, **kw)
        st[sl], it[sl, :g.segments], bd[sl, :g.segments + 1] = a, b, c
    return st, it, bd


@pytest.mark.parametrize("nodes,tile", [(16, 2048), (33, 2048), (64, 2048), (100, 2048), (128, 2048),
                                        (16, 1024), (48, 1024), (64, 1024), (200, 2048), (256, 2048)])
def test_second_order_matches_oracle(pc, nodes, tile):
    w = W.nbody_venus(37, seed=nodes + tile, days=112.5, segments=2, nodes=nodes)
    r = _gpu(pc, w, tile_pairs=tile)
    st, it, bd = _oracle(w)
    assert r["status"] == 0
    assert boundary_err(r["bounds"], bd).max() <= TOL
    assert np.abs(r["iters"] - it).max() <= 1


def test_fixed_sweeps_agree_to_rounding(pc):
    w = W.nbody_venus(40, seed=3, days=112.5, segments=2)
    r = _gpu(pc, w, fixed_iters=12)
    st, it, bd = _oracle(w, fixed_iters=12)
    assert np.all(r["iters"] == 12)
    assert rel_err(r["states"], st).max() < 1e-13


def test_backward_cold_start_and_groups(pc):
    w = W.nbody_venus(24, seed=5, days=112.5, segments=2, nodes=64)
    g = w.groups[0]
    g.t0, g.tf = g.tf, g.t0                      # backward
    w.init = 1                                   # cold start
    r = _gpu(pc, w)
    st, it, bd = _oracle(w)
    assert r["status"] == 0 and boundary_err(r["bounds"], bd).max() <= TOL
    assert np.abs(r["iters"] - it).max() <= 1
    # groups of 64, 128 and 256 nodes of the eccentric batch in one call
    wu = W.uneven_batch(600, seed=11)
    for g in wu.groups:
        g.segments = 1 + g.segments // 16
        g.tf = g.segments * np.pi / 4.0
    r = _gpu(pc, wu)
    st, it, bd = _oracle(wu)
    assert r["status"] == 0 and boundary_err(r["bounds"], bd).max() <= TOL
    assert np.abs(r["iters"] - it).max() <= 1


def test_fewer_sweeps_than_first_order(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(512, seed=8)
    g = w.groups[0]
    ics = torch.tensor(w.ics, device="cuda")
    groups = [pcprop.Group(0, w.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol)]
    model = pcprop.Model(1.0, w.pert, 0.0)
    one = pc.propagate_batched(ics, groups, model)
    two = pc.propagate_batched(ics, groups, model, order=2)
    i1, i2 = one["iters"].cpu().numpy(), two["iters"].cpu().numpy()
    assert one["status"] == 0 and two["status"] == 0
    assert i2.mean() < 0.7 * i1.mean()
    # the two forms are different discretisations of the same dynamics
    assert rel_err(two["states"].cpu().numpy(), one["states"].cpu().numpy()).max() < 1e-10


@pytest.mark.parametrize("nodes,tile", [(16, 2048), (64, 2048), (100, 2048), (128, 2048), (48, 1024),
                                        (200, 2048), (256, 2048)])
def test_feedback_matches_oracle(pc, nodes, tile):
    """Second-order sweeps with the integral error feedback against the oracle's feedback
    form: states at every boundary to the bar, sweep counts within one."""
    w = W.nbody_venus(37, seed=nodes + 7 * tile, days=112.5, segments=2, nodes=nodes)
    r = _gpu(pc, w, tile_pairs=tile, feedback=1)
    st, it, bd = _oracle(w, feedback=1)
    assert r["status"] == 0
    assert boundary_err(r["bounds"], bd).max() <= TOL
    assert np.abs(r["iters"] - it).max() <= 1


def test_feedback_fixed_sweeps_and_global_records(pc):
    # fixed sweeps: the same arithmetic to rounding; 16 perturbers at 64 nodes in the
    # 1024-pair shape read their records from global memory (3264 doubles, past the 3072 the
    # shape keeps in LDS)
    w = W.nbody_venus(40, seed=5, days=112.5, segments=2)
    r = _gpu(pc, w, fixed_iters=6, feedback=1)
    st, it, bd = _oracle(w, fixed_iters=6, feedback=1)
    assert rel_err(r["states"], st).max() < 1e-12
    w = W.nbody_venus(40, seed=6, days=112.5, segments=2, nodes=64)
    pert16 = np.concatenate([w.pert, w.pert * np.array([0.5, 1.02, 1, 1, 1, 1, 1]) + np.array([0, 0, 0, 0, 0, 0, 1.0])])
    w16 = W.Workload("p16", w.ics, w.groups, pert16, w.init)
    r = _gpu(pc, w16, feedback=1, tile_pairs=1024)
    st, it, bd = _oracle(w16, feedback=1)
    assert r["status"] == 0 and boundary_err(r["bounds"], bd).max() <= TOL


def test_node_row_feedback_fixed_sweeps_global_records_and_backward(pc):
    """The feedback on 8-IC jobs (256 nodes, node-row layout: lane pairs exchange the
    position and its change for da, the mixed column blocks take their zero halves by
    select): fixed sweeps to rounding, 16 perturbers (records in global memory) and a
    backward span against the oracle; ragged IC counts."""
    w = W.nbody_venus(21, seed=12, days=112.5, segments=2, nodes=256)
    r = _gpu(pc, w, fixed_iters=6, feedback=1)
    st, it, bd = _oracle(w, fixed_iters=6, feedback=1)
    assert rel_err(r["states"], st).max() < 1e-12
    w = W.nbody_venus(13, seed=13, days=112.5, segments=2, nodes=220)
    pert16 = np.concatenate([w.pert, w.pert * np.array([0.5, 1.02, 1, 1, 1, 1, 1]) + np.array([0, 0, 0, 0, 0, 0, 1.0])])
    w16 = W.Workload("p16", w.ics, w.groups, pert16, w.init)
    r = _gpu(pc, w16, feedback=1)
    st, it, bd = _oracle(w16, feedback=1)
    assert r["status"] == 0 and boundary_err(r["bounds"], bd).max() <= TOL
    assert np.abs(r["iters"] - it).max() <= 1
    wb = W.nbody_venus(11, seed=14, days=80.0, segments=2, nodes=256)
    wb.groups[0].t0, wb.groups[0].tf = wb.groups[0].tf, wb.groups[0].t0
    r = _gpu(pc, wb, feedback=1)
    st, it, bd = _oracle(wb, feedback=1)
    assert r["status"] == 0 and boundary_err(r["bounds"], bd).max() <= TOL


@pytest.mark.parametrize("nodes", [128, 256])
def test_feedback_takes_fewer_sweeps_at_high_node_counts(pc, nodes):
    w = W.nbody_venus(64, seed=9, nodes=nodes)
    two = _gpu(pc, w)
    fb = _gpu(pc, w, feedback=1)
    assert two["status"] == 0 and fb["status"] == 0
    assert fb["iters"].mean() < two["iters"].mean()
    assert rel_err(fb["states"], two["states"]).max() < 1e-10


def test_feedback_takes_fewer_sweeps_than_second_order(pc):
    w = W.nbody_venus(512, seed=8)
    two = _gpu(pc, w)
    fb = _gpu(pc, w, feedback=1)
    i2, ifb = two["iters"], fb["iters"]
    assert two["status"] == 0 and fb["status"] == 0
    assert ifb.mean() < 0.8 * i2.mean()
    # the same fixed point (to the stopping tolerance's truncation)
    assert rel_err(fb["states"], two["states"]).max() < 1e-10


def test_second_order_refusals(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(16, days=56.25, segments=1)
    g = w.groups[0]
    ics = torch.tensor(w.ics, device="cuda")
    model = pcprop.Model(1.0, w.pert, 0.0)
    bad = [dict(groups=None, kw=dict(precision="fp32-fp64")),
           dict(groups=None, kw=dict(path="plain")),
           dict(groups=None, kw=dict(tile_pairs=1024, **{}), nodes=128)]
    for case in bad:
        nodes = case.get("nodes", g.nodes)
        groups = case["groups"] or [pcprop.Group(0, 16, g.t0, g.tf, nodes, 1, g.tol)]
        with pytest.raises(pcprop.PcError) as e:
            pc.propagate_batched(ics, groups, model, order=2, **case["kw"])
        assert e.value.code == pcprop.PC_EINVAL
    with pytest.raises(pcprop.PcError):
        pc.propagate_batched(ics, [pcprop.Group(0, 16, g.t0, g.tf, g.nodes, 1, g.tol)],
                             pcprop.Model(1.0, w.pert, 0.0, 1e-8), order=2)
    with pytest.raises(pcprop.PcError) as e:   # feedback belongs to the second-order form
        pc.propagate_batched(ics, [pcprop.Group(0, 16, g.t0, g.tf, g.nodes, 1, g.tol)], model, feedback=1)
    assert e.value.code == pcprop.PC_EINVAL


def test_node_row_second_order_fixed_sweeps_backward_and_nodes(pc):
    """256-node jobs (8 ICs, node-row layout, two MFMAs into the mixed column block) with a
    ragged IC count: fixed sweeps to rounding, backward and cold start, and the node states
    against the oracle's."""
    w = W.nbody_venus(19, seed=12, days=112.5, segments=2, nodes=256)
    r = _gpu(pc, w, fixed_iters=9)
    st, it, bd = _oracle(w, fixed_iters=9)
    assert np.all(r["iters"] == 9)
    assert rel_err(r["states"], st).max() < 1e-13
    g = w.groups[0]
    g.t0, g.tf = g.tf, g.t0
    w.init = 1
    r = _gpu(pc, w, want_nodes=True)
    st, it, bd = _oracle(w)
    assert r["status"] == 0 and boundary_err(r["bounds"], bd).max() <= TOL
    assert np.abs(r["iters"] - it).max() <= 1
    m = oracle.Model(w.mu_sun, w.pert, w.epoch)
    o = oracle.propagate(w.ics[:5], g.t0, g.tf, g.nodes, g.segments, g.tol, m, init=1, want_nodes=True, order=2)
    nodes = r["nodes"][:5, :, :256]
    err = np.abs(nodes - o[2]).max() / np.abs(o[2]).max()
    assert err < 1e-10, err


@pytest.mark.parametrize("nodes", [64, 100, 128, 200, 256])
def test_second_order_refilled_columns(pc, nodes):
    """Jobs longer than one column block (a stopped IC's column takes the next IC of the
    segment) under second-order sweeps: against the oracle, and the same sweep counts and
    states as one-block jobs."""
    w = W.nbody_venus(150, seed=20 + nodes, days=112.5, segments=2, nodes=nodes)
    a = _gpu(pc, w, job_list=4)
    b = _gpu(pc, w, job_list=1)
    st, it, bd = _oracle(w)
    assert a["status"] == 0 and b["status"] == 0
    assert boundary_err(a["bounds"], bd).max() <= TOL
    assert np.abs(a["iters"] - it).max() <= 1
    assert np.array_equal(a["iters"], b["iters"])
    assert rel_err(a["states"], b["states"]).max() < 1e-13
