"""Pins of the oracle's second-order form (velocity and position both integrated from
the acceleration samples) and of its integral error feedback.

Sec. 1 cites a second-order version of the method, with an integral error feedback, as
developments that carry over to the augmented system, and Sec. 7 expects a further
speed-up from them; the paper gives no formulas.  The oracle's form (orc_propagate,
order 2) fits the accelerations with the degree N-2 series of step (ii), integrates it
once for the velocity and twice for the position.  These tests hold it to what the
mathematics fixes, not to itself: numpy's Chebyshev integration twice over (polynomial
exactness), the aliased mode, the Kepler closed form, scipy's DOP853 and the
reversibility of the dynamics; the feedback must leave the converged result alone.
"""
import numpy as np
import numpy.polynomial.chebyshev as C
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_2301_03989_amd import workloads as W


@pytest.mark.parametrize("N", [3, 4, 7, 16, 64, 128, 200, 256])
def test_double_integral_of_polynomials_of_degree_N_minus_2_is_exact(N):
    rng = np.random.default_rng(100 + N)
    tau = np.cos(np.pi * (N - 1 - np.arange(N)) / (N - 1))
    for deg in sorted({0, 1, max(0, N // 2), N - 2}):
        coef = rng.standard_normal((deg + 1, 3)) / np.arange(1, deg + 2)[:, None]
        a = np.stack([C.chebval(tau, coef[:, c]) for c in range(3)], axis=1)
        x0, v0 = rng.standard_normal(3), rng.standard_normal(3)
        w2 = 0.37
        x, v = oracle.second_order_step(a, x0, v0, w2)
        for c in range(3):
            I1 = C.chebint(coef[:, c], lbnd=-1)            # vanishes at -1
            I2 = C.chebint(I1, lbnd=-1)
            ev = v0[c] + w2 * C.chebval(tau, I1)
            ex = x0[c] + w2 * v0[c] * (tau + 1) + w2 * w2 * C.chebval(tau, I2)
            sc = 1.0 + np.abs(ex).max() + np.abs(ev).max()
            np.testing.assert_allclose(v[:, c], ev, rtol=0, atol=3e-14 * sc * max(1, N / 64))
            np.testing.assert_allclose(x[:, c], ex, rtol=0, atol=3e-14 * sc * max(1, N / 64))


@pytest.mark.parametrize("N", [3, 4, 9, 64, 256])
def test_aliased_mode_is_annihilated(N):
    a = np.repeat(((-1.0) ** np.arange(N))[:, None], 3, axis=1)
    x0, v0 = np.array([1.0, -2.0, 0.5]), np.array([0.3, 0.1, -0.7])
    x, v = oracle.second_order_step(a, x0, v0, 0.8)
    tau = oracle.nodes(N)
    np.testing.assert_allclose(v, np.tile(v0, (N, 1)), rtol=0, atol=1e-14)
    np.testing.assert_allclose(x, x0 + 0.8 * v0 * (tau[:, None] + 1), rtol=0, atol=1e-14)


def test_velocity_update_is_the_first_order_update_of_the_velocity():
    """The velocity of the second-order update equals the first-order update of the
    velocity components from the same (w2-scaled) accelerations (steps ii-v)."""
    N = 33
    rng = np.random.default_rng(3)
    a = rng.standard_normal((N, 3))
    v0 = rng.standard_normal(3)
    _, v = oracle.second_order_step(a, np.zeros(3), v0, 0.6)
    ref = oracle.picard_step(0.6 * a, v0)
    np.testing.assert_allclose(v, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("feedback", [0, 1])
def test_sun_only_nodes_match_kepler_closed_form(feedback):
    w = W.sun_only_kepler(8)
    t0 = np.array([g.t0 for g in w.groups])
    tf = np.array([g.tf for g in w.groups])
    st, it, nodes = oracle.propagate(w.ics, t0, tf, 64, 4, 1e-13, init=1, want_nodes=True,
                                     order=2, feedback=feedback)
    assert (it > 0).all()
    tau = oracle.nodes(64)
    for m in range(w.n_ic):
        h = (tf[m] - t0[m]) / 4
        for s in range(4):
            for j in range(0, 64, 7):
                ok, ref = oracle.kepler(w.ics[m], h * s + 0.5 * h * (tau[j] + 1))
                y = nodes[m, s, j]
                assert np.linalg.norm(y[:3] - ref[:3]) / np.linalg.norm(ref[:3]) < 1e-11
                assert np.linalg.norm(y[3:] - ref[3:]) / np.linalg.norm(ref[3:]) < 1e-11
    np.testing.assert_allclose(st, w.ics, rtol=0, atol=1e-11)


def test_nbody_matches_dop853_and_the_first_order_result():
    w = W.nbody_venus(4)
    g = w.groups[0]
    model = oracle.Model(1.0, w.pert)
    s1, _ = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, model)
    for fb in (0, 1):
        s2, it = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, model, order=2, feedback=fb)
        assert (it > 0).all()
        for m in range(w.n_ic):
            sol = solve_ivp(lambda t, y: np.concatenate([y[3:], oracle.accel_t(y[:3], t, model)]),
                            (g.t0, g.tf), w.ics[m], method="DOP853", rtol=1e-13, atol=1e-16)
            ref = sol.y[:, -1]
            for s in (s2[m], s1[m]):
                assert np.linalg.norm(s[:3] - ref[:3]) / np.linalg.norm(ref[:3]) < 1e-10
                assert np.linalg.norm(s[3:] - ref[3:]) / np.linalg.norm(ref[3:]) < 1e-10


def test_backward_returns_to_start():
    w = W.nbody_venus(3)
    g = w.groups[0]
    model = oracle.Model(1.0, w.pert)
    fwd, _ = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, 1e-13, model, order=2)
    back, it = oracle.propagate(fwd, g.tf, g.t0, g.nodes, g.segments, 1e-13, model, order=2)
    assert (it > 0).all()
    np.testing.assert_allclose(back, w.ics, rtol=0, atol=5e-11)


def test_feedback_keeps_the_fixed_point_and_takes_fewer_sweeps():
    """At convergence the position change that the feedback integrates vanishes: with and
    without it the second-order iteration reaches the same discrete fixed point (fixed
    sweeps well past convergence agree to rounding), and with it the stopping rule is met
    in fewer sweeps.  Both take fewer sweeps than the first-order iteration."""
    w = W.nbody_venus(6)
    g = w.groups[0]
    model = oracle.Model(1.0, w.pert)
    a, _ = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, model, order=2, fixed_iters=30)
    b, _ = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, model, order=2, feedback=1,
                            fixed_iters=30)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)
    _, i1 = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, model)
    _, i2 = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, model, order=2)
    _, i3 = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, model, order=2, feedback=1)
    assert i2.mean() < 0.7 * i1.mean()
    assert i3.mean() < 0.8 * i2.mean()


def test_argument_checks():
    w = W.nbody_venus(2)
    g = w.groups[0]
    with pytest.raises(ValueError):
        oracle.propagate(w.ics, g.t0, g.tf, g.nodes, 1, g.tol, order=3)
    with pytest.raises(ValueError):
        oracle.propagate(w.ics, g.t0, g.tf, g.nodes, 1, g.tol, order=1, feedback=1)
