"""Hot start on the HIP path (init = guess: every segment starts from caller-supplied
node states, Sec. 2.1) against the oracle started from the same node states."""
import numpy as np
import pytest

import oracle
from paper_2301_03989_amd import workloads as W
from tests._parity import boundary_err

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


def _args(w):
    from paper_2301_03989_amd import pcprop
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]
    return ics, groups, pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)


def _oracle(w, guess, **kw):
    """Oracle per group, init 2 with the guess rows of that group ([n, S_max, N_max, 6])."""
    S = max(g.segments for g in w.groups)
    st = np.zeros((w.n_ic, 6))
    it = np.zeros((w.n_ic, S), dtype=np.int32)
    bd = np.zeros((w.n_ic, S + 1, 6))
    m = oracle.Model(w.mu_sun, w.pert, w.epoch, inv_c2=w.inv_c2)
    for g in w.groups:
        sl = slice(g.ic_offset, g.ic_offset + g.n_ic)
        gq = guess[sl, :g.segments, :g.nodes]
        a, b, c = oracle.propagate(w.ics[sl], g.t0, g.tf, g.nodes, g.segments, g.tol, m, init=2, guess=gq,
                                   want_bounds=True, **kw)
        st[sl], it[sl, :g.segments], bd[sl, :g.segments + 1] = a, b, c
    return st, it, bd


def _nearby_guess(pc, w, eps=1e-10, **kw):
    """GPU node states of the ICs scaled by (1 + eps): a hot start for the same ICs."""
    ics, groups, model = _args(w)
    r = pc.propagate_batched(ics * (1 + eps), groups, model, want_nodes=True, **kw)
    assert r["status"] == 0
    return r["nodes"]


@pytest.mark.parametrize("path,order,nodes", [("fused", 1, 128), ("fused", 1, 256), ("fused", 1, 24),
                                              ("fused", 2, 64), ("plain", 1, 128), ("plain", 1, 256)])
def test_hot_start_matches_oracle(pc, path, order, nodes):
    w = W.nbody_venus(40, seed=nodes + order, days=112.5, segments=3, nodes=nodes)
    guess = _nearby_guess(pc, w)
    ics, groups, model = _args(w)
    r = pc.propagate_batched(ics, groups, model, want_bounds=True, init="guess", guess=guess, path=path,
                             order=order)
    assert r["status"] == 0
    st, it, bd = _oracle(w, guess.cpu().numpy(), order=order)
    assert boundary_err(r["bounds"].cpu().numpy(), bd).max() <= TOL
    assert np.abs(r["iters"].cpu().numpy() - it).max() <= 1
    # and fewer sweeps than the warm start
    r0 = pc.propagate_batched(ics, groups, model, path=path, order=order)
    assert r["iters"].float().mean() < r0["iters"].float().mean()


def test_point_mass_guess_for_relativistic_model_and_mixed_groups(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(48, seed=12, days=112.5, segments=2)
    ics, groups, model = _args(w)
    pm = pc.propagate_batched(ics, groups, model, want_nodes=True)["nodes"]
    w.inv_c2 = 1.0 / W.C_AU_TU ** 2
    ics, groups, me = _args(w)
    for precision in ("fp64", "fp32-fp64"):
        r = pc.propagate_batched(ics, groups, me, want_bounds=True, init="guess", guess=pm, precision=precision)
        assert r["status"] == 0
        st, it, bd = _oracle(w, pm.cpu().numpy())
        assert boundary_err(r["bounds"].cpu().numpy(), bd).max() <= TOL, precision
    # groups of different node and segment counts: the guess uses the call's strides
    wu = W.uneven_batch(300, seed=13)
    for g in wu.groups:
        g.segments = 1 + g.segments // 16
        g.tf = g.segments * np.pi / 4.0
    guess = _nearby_guess(pc, wu)
    guess[5, 0, 3] = float("nan")              # a non-finite row: that node starts from y0
    ics, groups, model = _args(wu)
    r = pc.propagate_batched(ics, groups, model, want_bounds=True, init="guess", guess=guess)
    assert r["status"] == 0
    st, it, bd = _oracle(wu, guess.cpu().numpy())
    assert boundary_err(r["bounds"].cpu().numpy(), bd).max() <= TOL
    # a guess buffer goes with init "guess" only
    with pytest.raises(pcprop.PcError):
        pc.propagate_batched(ics, groups, model, guess=guess)
    with pytest.raises(pcprop.PcError):
        pc.propagate_batched(ics, groups, model, init="guess")
