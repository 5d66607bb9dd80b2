"""The allocation-free entry point (pc_propagate_batched_noalloc) against
pc_propagate_batched, through the C ABI.  Both run the same fused-path kernels on the same
plan, so their outputs must agree bit for bit; two calls in a row, the second smaller,
check that the static scratch keeps nothing of the previous call that matters."""
import numpy as np
import pytest

from paper_2301_03989_amd import workloads as W
from tests._parity import oracle_run, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_03989_amd import build, pcprop
    build.ensure_built()
    return pcprop.Context(0)


def _groups(w):
    from paper_2301_03989_amd import pcprop
    return [pcprop.Group(g.ic_offset, g.n_ic, g.t0, g.tf, g.nodes, g.segments, g.tol) for g in w.groups]


def _both(pc, w, **opts):
    """The workload through pc_propagate_batched, then through the allocation-free call into
    preallocated outputs; returns both result dicts (host arrays)."""
    from paper_2301_03989_amd import pcprop
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    groups = _groups(w)
    model = pcprop.Model(w.mu_sun, w.pert, w.epoch, w.inv_c2)
    S = max(g.segments for g in w.groups)
    ref = pc.propagate_batched(ics, groups, model, want_bounds=True, **opts)
    out = torch.full((w.n_ic, 6), np.nan, dtype=torch.float64, device="cuda")
    iters = torch.zeros((w.n_ic, S), dtype=torch.int32, device="cuda")
    bounds = torch.full((w.n_ic, S + 1, 6), np.nan, dtype=torch.float64, device="cuda")
    r = pc.propagate_batched_noalloc(ics, groups, model, out=out, iters_out=iters, bounds_out=bounds, **opts)
    torch.cuda.synchronize()
    host = lambda d: {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in d.items()}
    return host(ref), host(r)


def _same(a, b):
    assert a["status"] == b["status"] == 0
    for k in ("states", "iters", "bounds"):
        assert np.array_equal(a[k], b[k]), k


def test_two_calls_in_a_row_match_the_workspace_call(pc):
    # a multi-group batch (64, 128 and 256 nodes, several segments), then a smaller call
    big = W.uneven_batch(3000, seed=31)
    big = W.Workload(big.name, big.ics, [W.Group(g.ic_offset, g.n_ic, g.t0, g.t0 + 3 * np.pi / 4, g.nodes, 3, g.tol)
                                         for g in big.groups], big.pert, big.init)
    a, b = _both(pc, big)
    _same(a, b)
    small = W.nbody_venus(200, seed=9, days=112.5, segments=2)
    a2, b2 = _both(pc, small)
    _same(a2, b2)
    o = oracle_run(small, np.arange(0, 200, 20))
    assert rel_err(b2["states"][::20], o["states"]).max() <= 1e-10


def test_precision_schedule_and_relativistic_model(pc):
    mixed = W.nbody_venus(512, seed=12, days=112.5, segments=2)
    a, b = _both(pc, mixed, precision="fp32-fp64")
    _same(a, b)
    eih = W.nbody_venus(256, seed=13, days=112.5, segments=2)
    eih.inv_c2 = 1.0 / W.C_AU_TU ** 2
    a, b = _both(pc, eih)
    _same(a, b)


def test_refusals(pc):
    from paper_2301_03989_amd import pcprop
    w = W.nbody_venus(64, seed=14, days=56.25, segments=1)
    ics = torch.tensor(w.ics, dtype=torch.float64, device="cuda")
    model = pcprop.Model(1.0, w.pert, 0.0)
    out = torch.empty((64, 6), dtype=torch.float64, device="cuda")
    iters = torch.zeros((64, 1), dtype=torch.int32, device="cuda")
    fresh = pcprop.Context(0)
    g37 = [pcprop.Group(0, 64, 0.0, 0.5, 37, 1, 1e-12)]
    with pytest.raises(pcprop.PcError) as e:   # operators of 37 nodes not built in this context
        fresh.propagate_batched_noalloc(ics, g37, model, out=out, iters_out=iters)
    assert e.value.code == pcprop.PC_EINVAL
    fresh.propagate_batched(ics, g37, model)
    r = fresh.propagate_batched_noalloc(ics, g37, model, out=out, iters_out=iters)
    assert r["status"] == 0
    for kw in ({"path": "plain"}, {"graph": True}):
        with pytest.raises(pcprop.PcError) as e:
            fresh.propagate_batched_noalloc(ics, g37, model, out=out, iters_out=iters, **kw)
        assert e.value.code == pcprop.PC_EINVAL
    # 500 segments of 256 nodes: 128000 records of 288 bytes, beyond the 32 MiB scratch
    fresh.propagate_batched(ics[:1], [pcprop.Group(0, 1, 0.0, 0.5, 256, 1, 1e-12)], model)
    g_big = [pcprop.Group(0, 1, 0.0, 500 * 0.05, 256, 500, 1e-12)]
    it_big = torch.zeros((1, 500), dtype=torch.int32, device="cuda")
    with pytest.raises(pcprop.PcError) as e:
        fresh.propagate_batched_noalloc(ics[:1], g_big, model, out=out[:1], iters_out=it_big)
    assert e.value.code == pcprop.PC_ENOMEM
    assert "scratch" in str(e.value)
