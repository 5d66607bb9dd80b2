"""Parity at the full shapes of the batched and mixed-precision workloads.

The uneven 65536-IC batch (15 groups: 64, 128 and 256 nodes x 8 to 40 segments of
pi/4 TU, eccentricities up to 0.6) runs whole in one fused launch; a seeded stratified
sample of 128 ICs per group is compared with the oracle at every segment boundary.
The 262144-IC N-body ensemble runs whole in FP64 and under the FP32 -> FP64 schedule;
a seeded sample of 1024 ICs is compared with the FP64 oracle.

Bar: per-IC relative position/velocity error <= 1e-10 at every segment boundary
(final state included).  A few ICs of the eccentric batch pass planets inside their
Hill spheres; there a change of 1e-14 in the initial state moves the result by more
than 1e-11 on the oracle itself, and the bar for those ICs is 30 times the largest change the
oracle shows under four such perturbations (the trajectory's own conditioning, which no
FP64 implementation with another rounding order can beat).  Every other IC is held to
1e-10, and the conditioning-limited ICs must be rare (at most 1 % of the sample).
"""
import numpy as np
import pytest

from paper_2301_03989_amd import workloads as W
from tests._parity import boundary_err, oracle_run, oracle_sensitivity, rel_err

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
    r = pc.propagate_batched(ics, groups, model, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


def stratified(w, per_group, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([g.ic_offset + np.sort(rng.choice(g.n_ic, size=min(per_group, g.n_ic), replace=False))
                           for g in w.groups])


def check_against_oracle(w, r, idx, label):
    o = oracle_run(w, idx, want_bounds=True)
    err = boundary_err(r["bounds"][idx], o["bounds"])
    bad = np.nonzero(err > TOL)[0]
    kappa = np.zeros(idx.size)
    if bad.size:
        kappa[bad] = oracle_sensitivity(w, idx[bad])
        assert np.all(err[bad] <= 30.0 * kappa[bad]), (label, idx[bad], err[bad], kappa[bad])
        assert bad.size <= max(1, idx.size // 100), (label, bad.size)
    # the stopping decision may flip within rounding of tol: counts agree within one sweep
    # except where the trajectory is conditioning-limited
    good = err <= TOL
    dit = np.abs(r["iters"][idx][good] - o["iters"][good])
    assert dit.max() <= 1, (label, dit.max())
    print(f"{label}: {idx.size} ICs, max err {err.max():.3e} (at or below 1e-10: {good.sum()}, "
          f"conditioning-limited: {bad.size}, their 1e-14 sensitivity {kappa[bad].round(13).tolist()})", flush=True)
    return err


def test_uneven_batch_full_shape(pc):
    w = W.uneven_batch()
    r = _gpu(pc, w, want_bounds=True)
    assert r["status"] == 0
    assert np.all(r["iters"][:, 0] > 0)
    for g in w.groups:   # every segment of every IC converged
        assert np.all(r["iters"][g.ic_offset:g.ic_offset + g.n_ic, :g.segments] > 0)
    idx = stratified(w, 128, seed=2024)
    err = check_against_oracle(w, r, idx, "uneven-batch-65536")
    for g in w.groups:
        sel = (idx >= g.ic_offset) & (idx < g.ic_offset + g.n_ic)
        print(f"  N={g.nodes:3d} S={g.segments:2d}: max err {err[sel].max():.2e}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32-fp64"])
def test_mixed_precision_workload_full_shape(pc, precision):
    w = W.mixed_precision()
    r = _gpu(pc, w, want_bounds=True, precision=precision)
    assert r["status"] == 0
    idx = np.sort(np.random.default_rng(7).choice(w.n_ic, size=1024, replace=False))
    o = oracle_run(w, idx, want_bounds=True)
    err = boundary_err(r["bounds"][idx], o["bounds"])
    assert err.max() <= TOL, err.max()
    dit = r["iters"][idx] - o["iters"]
    if precision == "fp64":
        assert np.abs(dit).max() <= 1
    else:   # the schedule's count is usually one above the FP64 one (parity unpinned)
        assert dit.min() >= -1 and dit.max() <= 3 and dit.mean() <= 1.5
    print(f"nbody-venus-262144 {precision}: max err {err.max():.3e} on {idx.size} ICs", flush=True)
