"""Pins of the oracle's group-max stopping rule (one decision for all the ICs of a group,
on the largest error over them; Sec. 3.2, and the whole-system maximum of the paper's
CUDA program, Sec. 5.4.2).

The group mode shares the sweep arithmetic with the per-IC mode, so these checks pin
what differs: where the group stops.  The stopping decision is recomputed here in numpy
from fixed-sweep runs (the error of step (vi) between the node states of k - 1 and k
sweeps), independently of the C code's own error and maximum.
"""
import numpy as np
import pytest

import oracle
from paper_2301_03989_amd import workloads as W


def _eccentric(n, seed, nodes, segments, tol):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.7, 1.0, n)
    e = rng.uniform(0.0, 0.6, n)
    inc = rng.uniform(0.0, 10.0, n) * W.DEG
    raan, argp, M = (rng.uniform(0.0, 360.0, n) * W.DEG for _ in range(3))
    ics = W.elements_to_states(a, e, inc, raan, argp, M)
    return ics, 0.0, segments * np.pi / 4, nodes, segments, tol


def _model():
    return oracle.Model(1.0, W.planet_elements(), 0.0)


def _run(ics, t0, tf, N, S, tol, **kw):
    return oracle.propagate(ics, t0, tf, N, S, tol, _model(), **kw)


def _step_error(a, b, rel=True):
    """Error (vi) per IC between node states a and b [n, N, 6] (2-norms per node, max over
    nodes of max(position, velocity)), written out in numpy."""
    dr = np.linalg.norm(a[..., :3] - b[..., :3], axis=-1)
    dv = np.linalg.norm(a[..., 3:] - b[..., 3:], axis=-1)
    if rel:
        dr = dr / np.linalg.norm(a[..., :3], axis=-1)
        dv = dv / np.linalg.norm(a[..., 3:], axis=-1)
    return np.maximum(dr, dv).max(axis=-1)


def test_group_of_one_is_the_per_ic_rule():
    ics, t0, tf, N, S, tol = _eccentric(3, 7, 48, 3, 1e-12)
    for m in range(3):
        a = _run(ics[m:m + 1], t0, tf, N, S, tol, want_bounds=True, want_nodes=True)
        b = _run(ics[m:m + 1], t0, tf, N, S, tol, want_bounds=True, want_nodes=True, conv=1)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("rel", [True, False])
def test_group_stops_at_the_first_sweep_where_every_error_is_below_tol(rel):
    """One segment: the group's count k is the first sweep at which the largest error over
    the ICs (recomputed from fixed-sweep node states) is below tol; the group's states are
    the k-sweep states of every IC; the per-IC rule stops some ICs earlier."""
    ics, t0, tf, N, S, tol = _eccentric(24, 11, 48, 1, 1e-11)
    mode = 0 if rel else 1
    g = _run(ics, t0, tf, N, S, tol, tol_mode=mode, want_nodes=True, conv=1)
    k = int(g[1][0, 0])
    assert (g[1][:, 0] == k).all() and k > 1
    nodes = {j: _run(ics, t0, tf, N, S, tol, fixed_iters=j, want_nodes=True)[2][:, 0] for j in (k - 1, k)}
    prev = _run(ics, t0, tf, N, S, tol, fixed_iters=k - 2, want_nodes=True)[2][:, 0] if k > 2 else None
    e_k = _step_error(nodes[k], nodes[k - 1], rel)
    assert e_k.max() < tol
    if prev is not None:
        assert _step_error(nodes[k - 1], prev, rel).max() >= tol
    assert np.array_equal(g[2][:, 0], nodes[k])
    per_ic = _run(ics, t0, tf, N, S, tol, tol_mode=mode)[1][:, 0]
    assert per_ic.max() <= k and per_ic.min() < k


def test_group_first_segment_equals_fixed_sweeps_and_later_segments_chain():
    """Several segments: boundary 1 is the k1-sweep state of every IC, and the group's
    count in every segment is one number shared by all its ICs."""
    ics, t0, tf, N, S, tol = _eccentric(16, 3, 40, 3, 1e-11)
    g = _run(ics, t0, tf, N, S, tol, want_bounds=True, conv=1)
    for s in range(S):
        assert len(set(g[1][:, s].tolist())) == 1
    k1 = int(g[1][0, 0])
    f = _run(ics, t0, tf, N, S, tol, fixed_iters=k1, want_bounds=True)
    assert np.array_equal(g[2][:, 1], f[2][:, 1])
    # the second segment restarts from the group's boundary 1: a one-segment group run
    # from those states over the second segment's interval gives the same count and states
    h = (tf - t0) / S
    g2 = _run(g[2][:, 1], t0 + h, t0 + 2 * h, N, 1, tol, want_bounds=True, conv=1)
    assert (g2[1][:, 0] == g[1][:, 1]).all()
    assert np.array_equal(g2[2][:, 1], g[2][:, 2])


def test_non_finite_ic_leaves_the_group():
    ics, t0, tf, N, S, tol = _eccentric(12, 5, 40, 2, 1e-11)
    bad = ics.copy()
    bad[4, 0] = np.nan
    g = _run(bad, t0, tf, N, S, tol, conv=1)
    ref = _run(np.delete(ics, 4, axis=0), t0, tf, N, S, tol, conv=1)
    assert (g[1][4] == -2).all() and np.isnan(g[0][4]).all()
    assert np.array_equal(np.delete(g[0], 4, axis=0), ref[0])
    assert np.array_equal(np.delete(g[1], 4, axis=0), ref[1])


def test_group_not_converged_within_max_iter():
    ics, t0, tf, N, S, tol = _eccentric(8, 9, 40, 2, 1e-12)
    g = _run(ics, t0, tf, N, S, tol, max_iter=4, conv=1)
    f = _run(ics, t0, tf, N, S, tol, fixed_iters=4)
    assert (g[1] == -1).all()
    assert np.array_equal(g[0], f[0])
