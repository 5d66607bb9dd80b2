"""Pins of the oracle's hot start (init 2: every segment starts from caller-supplied node
states, Sec. 2.1's guesses from a simpler model or another propagation).

The Picard-Chebyshev map has one fixed point per segment whatever the initial iterate,
so a hot start must reach the result of the warm start (to the stopping tolerance's
level), and it must do so in fewer sweeps the closer the guess: the converged node
states themselves are reproduced at the first sweep.
"""
import numpy as np
import pytest

import oracle
from paper_2301_03989_amd import workloads as W
from tests._parity import rel_err


def _venus(n=6):
    w = W.nbody_venus(n)
    return w, w.groups[0], oracle.Model(1.0, w.pert)


def test_converged_nodes_are_reproduced_in_one_sweep():
    w, g, m = _venus()
    st, it, nodes = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, want_nodes=True)
    st2, it2, nodes2 = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, init=2,
                                        guess=nodes, want_nodes=True)
    assert np.all(it2 == 1)
    assert rel_err(st2, st).max() < 1e-12
    assert np.abs(nodes2 - nodes).max() < 1e-11


def test_guess_from_nearby_ics_reaches_the_warm_start_result_in_fewer_sweeps():
    """Node states of ICs changed by 1e-10 (relative) are a closer guess than the two-body
    one (which misses the planets' perturbations, ~1e-6 relative): fewer sweeps, the same
    fixed point to the stopping tolerance's level over the eight segments."""
    w, g, m = _venus()
    _, _, near = oracle.propagate(w.ics * (1 + 1e-10), g.t0, g.tf, g.nodes, g.segments, g.tol, m,
                                  want_nodes=True)
    st, it = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m)
    st2, it2 = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, init=2, guess=near)
    assert rel_err(st2, st).max() < 5e-11
    assert it2.mean() < 0.85 * it.mean()


def test_point_mass_guess_for_the_relativistic_model():
    """Sec. 2.1: a guess from a simpler model's propagation; the relativistic model (EIH)
    started from the point-mass node states reaches its own warm-start result."""
    w, g, m = _venus()
    me = oracle.Model(1.0, w.pert, inv_c2=1.0 / W.C_AU_TU ** 2)
    _, _, pm = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, want_nodes=True)
    st, it = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, me)
    st2, it2 = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, me, init=2, guess=pm)
    assert rel_err(st2, st).max() < 5e-11
    assert it2.mean() < it.mean()


def test_non_finite_guess_rows_fall_back_to_the_initial_state():
    """A row of NaN in the guess starts that node from the segment's initial state (the
    cold start's value there); the result is the same fixed point."""
    w, g, m = _venus(3)
    _, _, near = oracle.propagate(w.ics * (1 + 1e-8), g.t0, g.tf, g.nodes, g.segments, g.tol, m, want_nodes=True)
    bad = near.copy()
    bad[:, :, 5:9] = np.nan
    st, _ = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m)
    st2, it2 = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, init=2, guess=bad)
    assert (it2 > 0).all()
    assert rel_err(st2, st).max() < 5e-11


def test_second_order_hot_start_and_argument_checks():
    w, g, m = _venus(3)
    st, it, nodes = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, order=2, want_nodes=True)
    st2, it2 = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, order=2, init=2, guess=nodes)
    assert np.all(it2 == 1) and rel_err(st2, st).max() < 1e-12
    with pytest.raises(ValueError):
        oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, init=2)
    with pytest.raises(ValueError):
        oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, guess=nodes)
