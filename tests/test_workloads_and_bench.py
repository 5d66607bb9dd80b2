"""The synthetic input recipes and the benchmark's host-side helpers, on the CPU: the
stated shapes and element ranges of the workloads, and the bookkeeping bench.py reports
(flop counts, samples, boundary errors, the one-GPU contract)."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2301_03989_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _elements(states):
    """a, e and inclination of heliocentric states (mu = 1)."""
    r, v = states[:, :3], states[:, 3:]
    rn = np.linalg.norm(r, axis=1)
    v2 = np.einsum("ij,ij->i", v, v)
    a = 1.0 / (2.0 / rn - v2)
    h = np.cross(r, v)
    evec = np.cross(v, h) - r / rn[:, None]
    e = np.linalg.norm(evec, axis=1)
    inc = np.arccos(h[:, 2] / np.linalg.norm(h, axis=1))
    return a, e, inc


def test_elements_round_trip():
    rng = np.random.default_rng(1)
    a = rng.uniform(0.5, 2.0, 50)
    e = rng.uniform(0.0, 0.7, 50)
    inc = rng.uniform(0.0, 0.5, 50)
    s = W.elements_to_states(a, e, inc, *(rng.uniform(0, 2 * np.pi, 50) for _ in range(3)))
    a2, e2, i2 = _elements(s)
    np.testing.assert_allclose(a2, a, rtol=1e-12)
    np.testing.assert_allclose(e2, e, atol=1e-12)
    np.testing.assert_allclose(i2, inc, atol=1e-12)


def test_uneven_batch_recipe():
    w = W.uneven_batch()
    assert w.n_ic == 65536 and len(w.groups) == 15
    shapes = sorted((g.nodes, g.segments) for g in w.groups)
    assert shapes == sorted((N, S) for N in (64, 128, 256) for S in (8, 16, 24, 32, 40))
    off = 0
    for g in w.groups:
        assert g.ic_offset == off and g.n_ic > 0 and g.tol == 1e-12 and g.t0 == 0.0
        assert np.isclose(g.tf, g.segments * np.pi / 4.0)
        off += g.n_ic
    assert off == w.n_ic
    a, e, inc = _elements(w.ics)
    assert a.min() >= 0.7 - 1e-12 and a.max() <= 1.0 + 1e-12
    assert e.max() <= 0.6 + 1e-12
    assert inc.max() <= np.radians(10.0) + 1e-12
    assert w.pert.shape == (8, 7)


def test_paper_configuration_recipe():
    w = W.WORKLOADS["paper-configuration-13509"]()
    (g,) = w.groups
    assert w.n_ic == 13509 and g.nodes == 200 and g.segments == 1 and g.tol == 1e-12
    assert w.init == 1
    a0 = W.REF_ORBIT["a"]
    assert np.isclose(g.tf, 0.87 * 2 * np.pi * a0 ** 1.5)
    # 1/c^2 in AU and Gaussian time units: c = 173.14 AU/day
    assert np.isclose(1.0 / np.sqrt(w.inv_c2) / W.TU_DAYS, 173.1446, rtol=1e-5)
    ref = W._perturbed_ensemble(1, 0, dr=0.0, dv=0.0)[0]
    assert np.abs(w.ics - ref).max() <= 1e-4 + 1e-15


def test_subset_keeps_the_group_structure():
    w = W.uneven_batch(600, seed=3)
    idx = np.concatenate([np.arange(g.ic_offset, g.ic_offset + min(3, g.n_ic)) for g in w.groups])
    sub = w.subset(idx)
    assert sub.n_ic == idx.size and len(sub.groups) == len(w.groups)
    for gs, g in zip(sub.groups, w.groups):
        assert (gs.nodes, gs.segments, gs.tf, gs.tol) == (g.nodes, g.segments, g.tf, g.tol)
        np.testing.assert_array_equal(sub.ics[gs.ic_offset:gs.ic_offset + gs.n_ic],
                                      w.ics[g.ic_offset:g.ic_offset + gs.n_ic])


def test_algorithmic_flops_per_iteration():
    w = W.nbody_venus(3, nodes=128, segments=2)
    iters = np.array([[10, 12], [0, 5], [-1, 7]], dtype=np.int32)   # non-positive records count 0
    n_it = 10 + 12 + 5 + 7
    assert bench.algorithmic_flops(w, iters) == n_it * (12 * 128 ** 2 + (20 * 9 + 3) * 128)
    w.inv_c2 = 1e-8
    assert bench.algorithmic_flops(w, iters) == n_it * (12 * 128 ** 2 + (96 * 9 + 15) * 128)


def test_adjoint_flops_per_sweep():
    w = W.nbody_venus(2, nodes=64, segments=2)
    iters = np.array([[10, 12], [9, 0]], dtype=np.int32)
    adj = np.array([[4, 5], [6, -1]], dtype=np.int32)
    fwd = bench.algorithmic_flops(w, iters)
    per = 12 * 64 ** 2 + (30 * 9 + 12) * 64
    assert bench.adjoint_flops(w, iters, adj, resolve=False) == 15 * per
    assert bench.adjoint_flops(w, iters, adj) == fwd + 15 * per
    w.inv_c2 = 1e-8
    assert bench.adjoint_flops(w, iters, adj, resolve=False) == 15 * (12 * 64 ** 2 + (190 * 9 + 34 + 12) * 64)
    assert W.WORKLOADS["nbody-venus-16384-256d-eih"]().inv_c2 == 1.0 / W.C_AU_TU ** 2


def test_stratified_sample_and_boundary_errors():
    w = W.uneven_batch(600, seed=4)
    idx = bench.stratified_sample(w, 5, seed=2)
    assert idx.size == sum(min(5, g.n_ic) for g in w.groups)
    for g in w.groups:
        inside = idx[(idx >= g.ic_offset) & (idx < g.ic_offset + g.n_ic)]
        assert inside.size == min(5, g.n_ic) and np.all(np.diff(inside) > 0)
    ref = np.zeros((2, 3, 6))
    ref[:, :2] = 1.0
    gpu = ref.copy()
    gpu[0, 1, 0] = 1.0 + 1e-9
    gpu[1, 2] = 123.0              # past the reference's segments: not compared
    err = bench.boundary_errors(gpu, ref)
    assert err[1] == 0.0 and np.isclose(err[0], 1e-9 / np.sqrt(3.0), rtol=1e-6)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "not supported" in (r.stdout + r.stderr)
