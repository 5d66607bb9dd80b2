"""Pins of the oracle's Einstein-Infeld-Hoffmann dynamics (the relativistic restricted
N-body model of Sec. 5.4.1), each against something the formula of orc_accel_eih does not
share: the point-mass model (the limit 1/c^2 -> 0), the textbook first post-Newtonian
acceleration of a test body about one resting mass (the Sun-only special case), the
general-relativistic perihelion advance 6 pi mu / (c^2 a (1 - e^2)) per orbit, the time
derivative of the perturber positions (their velocities), and a small-step Runge-Kutta
integration of the same equations (the Picard-Chebyshev iteration with a velocity-
dependent force), and the Lorentz boost of a resting mass (a mass in uniform motion, which
checks the terms in the perturbers' velocities), and the Euler-Lagrange equations of the
first post-Newtonian Lagrangian solved numerically (which pins every term, the perturbers'
accelerations and potentials included, up to O(1/c^4)).  The adjoint's derivatives of the
same sums (the complex step on a numpy restatement) are pinned to the C function, to its
central differences and, through the adjoint, to finite differences of propagations."""
import numpy as np
import pytest

import oracle
from paper_2301_03989_amd import workloads as W


def _states(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.6, 1.4, n)
    e = rng.uniform(0.0, 0.5, n)
    inc = rng.uniform(0.0, 20.0, n) * W.DEG
    raan, argp, M = (rng.uniform(0.0, 360.0, n) * W.DEG for _ in range(3))
    return W.elements_to_states(a, e, inc, raan, argp, M)


def test_zero_inv_c2_is_the_point_mass_model():
    pert = W.planet_elements()
    m = oracle.Model(1.0, pert, 0.0)
    for i, y in enumerate(_states(20, 1)):
        t = 0.37 * i
        a0 = oracle.accel_t(y[:3], t, m)
        a1 = oracle.accel_eih_t(y, t, m)
        assert np.abs(a1 - a0).max() <= 1e-15 * np.abs(a0).max()


@pytest.mark.parametrize("inv_c2", [1e-3, 1e-6])
def test_sun_only_is_the_first_post_newtonian_test_body(inv_c2):
    """One resting mass: a = -mu r/r^3 + mu/(c^2 r^3) [(4 mu/r - v^2) r + 4 (r.v) v]
    (harmonic coordinates, beta = gamma = 1)."""
    mu = 1.3
    m = oracle.Model(mu, None, 0.0, inv_c2=inv_c2)
    for y in _states(20, 2):
        r, v = y[:3], y[3:]
        rn = np.linalg.norm(r)
        ref = -mu * r / rn**3 + inv_c2 * mu / rn**3 * ((4.0 * mu / rn - v @ v) * r + 4.0 * (r @ v) * v)
        got = oracle.accel_eih_t(y, 0.0, m)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
        # and the correction itself, to nine digits (the subtraction of the Newtonian
        # term leaves a few ulps of the whole acceleration)
        corr = ref + mu * r / rn**3
        assert np.abs((got + mu * r / rn**3) - corr).max() <= 1e-9 * np.abs(corr).max()


def test_perihelion_advance():
    """Sun only, a = 1, e = 0.3, 1/c^2 = 1e-4: over ten orbits the Laplace-Runge-Lenz
    vector turns by 10 x 6 pi mu / (c^2 a (1 - e^2)) (first order in 1/c^2)."""
    inv_c2, a, e = 1e-4, 1.0, 0.3
    y0 = W.elements_to_states(np.array([a]), np.array([e]), np.zeros(1), np.zeros(1),
                              np.zeros(1), np.zeros(1))[0]   # at perihelion
    m = oracle.Model(1.0, None, 0.0, inv_c2=inv_c2)
    orbits, per = 10, 16
    P = 2 * np.pi * a**1.5
    st, it = oracle.propagate(y0[None], 0.0, orbits * P, 64, orbits * per, 1e-13, m)
    assert (it > 0).all()

    def lrl(y):
        r, v = y[:3], y[3:]
        return np.cross(v, np.cross(r, v)) - r / np.linalg.norm(r)

    A0, A1 = lrl(y0), lrl(st[0])
    dw = np.arctan2(np.cross(A0, A1)[2], A0 @ A1)
    expect = orbits * 6 * np.pi * inv_c2 / (a * (1 - e * e))
    assert abs(dw / expect - 1.0) < 0.02, (dw, expect)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_uniformly_moving_mass_is_the_boosted_resting_one(seed):
    """A mass in uniform motion (velocity V, no acceleration) and a body moving with it at
    offset d: in their common rest frame the body feels the resting-mass acceleration
    -mu d'/|d'|^3 (1 - 4 mu/(c^2 |d'|)) (pinned above), with d' the offset lengthened by
    gamma along V; the Lorentz transformation of an acceleration for a body at rest in the
    moving frame divides its component along V by gamma^3 and the rest by gamma^2.  The
    relativistic sums must agree to first order in 1/c^2 (this checks their terms in the
    mass's velocity)."""
    rng = np.random.default_rng(seed)
    inv_c2, mu = 1e-6, 0.8
    V = rng.uniform(-1.5, 1.5, 3)
    rb = rng.uniform(-1.0, 1.0, 3)
    d = rng.uniform(-1.0, 1.0, 3)
    d *= rng.uniform(0.3, 1.2) / np.linalg.norm(d)
    y = np.concatenate([rb + d, V])
    got = oracle.accel_eih_bodies(y, rb[None], V[None], np.zeros((1, 3)), [mu], [0.0], inv_c2)
    gamma = 1.0 / np.sqrt(1.0 - inv_c2 * (V @ V))
    u = V / np.linalg.norm(V)
    dp = d + (gamma - 1.0) * (d @ u) * u                    # offset in the rest frame
    rp = np.linalg.norm(dp)
    ap = -mu * dp / rp**3 * (1.0 - 4.0 * mu * inv_c2 / rp)
    ref = (ap @ u) * u / gamma**3 + (ap - (ap @ u) * u) / gamma**2
    newton = -mu * d / np.linalg.norm(d)**3
    # the first-order correction itself (about 1e-6 of the acceleration) to 1e-5 of it
    assert np.abs((got - newton) - (ref - newton)).max() <= 1e-5 * np.abs(ref - newton).max()


def test_perturber_velocity_is_the_derivative_of_its_position():
    for el in W.planet_elements():
        for t in (0.0, 3.3, 17.0):
            h = 1e-5
            rp, _ = oracle.ephem_state(el, 0.0, t + h)
            rm, _ = oracle.ephem_state(el, 0.0, t - h)
            r, v = oracle.ephem_state(el, 0.0, t)
            assert np.allclose(r, oracle.ephem(el, 0.0, t), rtol=0, atol=1e-15)
            fd = (rp - rm) / (2 * h)
            assert np.abs(fd - v).max() <= 1e-8 * np.linalg.norm(v)


def test_picard_chebyshev_with_eih_matches_small_step_rk4():
    """N-body EIH with an exaggerated 1/c^2 = 1e-4 (the relativistic terms near 1e-4 of
    the acceleration): the oracle's iteration against 40000 RK4 steps over 100 days."""
    w = W.nbody_venus(3, days=100.0, segments=4, nodes=64)
    m = oracle.Model(1.0, w.pert, 0.0, inv_c2=1e-4)
    g = w.groups[0]
    st, it = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, 1e-13, m)
    assert (it > 0).all()
    for i in range(3):
        ref = oracle.rk4(w.ics[i], g.t0, g.tf, 40000, m)
        err = max(np.linalg.norm(st[i, :3] - ref[:3]) / np.linalg.norm(ref[:3]),
                  np.linalg.norm(st[i, 3:] - ref[3:]) / np.linalg.norm(ref[3:]))
        assert err < 1e-11, err
    # the relativistic terms matter at this 1/c^2: the point-mass result is far away
    st0, _ = oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, 1e-13, oracle.Model(1.0, w.pert, 0.0))
    assert np.linalg.norm(st0[0, :3] - st[0, :3]) / np.linalg.norm(st[0, :3]) > 1e-6


def test_eih_refused_by_group_mode():
    w = W.nbody_venus(2, days=20.0, segments=1, nodes=16)
    m = oracle.Model(1.0, w.pert, 0.0, inv_c2=1e-8)
    g = w.groups[0]
    with pytest.raises(ValueError):
        oracle.propagate(w.ics, g.t0, g.tf, g.nodes, g.segments, 1e-12, m, conv=1)


# -- the relativistic adjoint ------------------------------------------------------------
# The adjoint needs da/dr and da/dv of the relativistic force.  The oracle takes them by
# the complex step on a numpy restatement of the sums; the restatement is pinned to the C
# function, the derivatives to central differences of the C function, and the adjoint
# built on them to finite differences of whole propagations.

@pytest.mark.parametrize("inv_c2", [1e-3, 1.0 / W.C_AU_TU ** 2])
def test_numpy_restatement_matches_the_c_sums(inv_c2):
    pert = W.planet_elements()
    m = oracle.Model(1.0, pert, 0.0, inv_c2=inv_c2)
    for i, y in enumerate(_states(12, 4)):
        t = 0.53 * i
        bodies = oracle._eih_major_bodies(t, m)
        a_np = oracle._eih_accel_np(y, *bodies, inv_c2)
        ind = sum(p[0] * oracle.ephem(p, 0.0, t) / np.linalg.norm(oracle.ephem(p, 0.0, t)) ** 3 for p in pert)
        a_c = oracle.accel_eih_t(y, t, m)
        assert np.abs(a_np - ind - a_c).max() <= 1e-14 * np.abs(a_c).max()


def test_relativistic_jacobian_matches_central_differences():
    pert = W.planet_elements()
    m = oracle.Model(1.0, pert, 0.0, inv_c2=1e-3)   # exaggerated: the velocity block is O(1/c^2)
    for i, y in enumerate(_states(6, 5)):
        t = 0.71 * i
        J = oracle.accel_eih_jac_t(y, t, m)
        h = 1e-6
        fd = np.stack([(oracle.accel_eih_t(y + h * e, t, m) - oracle.accel_eih_t(y - h * e, t, m)) / (2 * h)
                       for e in np.eye(6)], axis=1)
        np.testing.assert_allclose(J, fd, rtol=0, atol=2e-8 * np.abs(J).max())
        assert np.abs(J[:, 3:]).max() > 1e-4 * np.abs(J[:, :3]).max()      # da/dv is there
        assert np.abs(J[:, :3] - J[:, :3].T).max() > 1e-9 * np.abs(J).max()  # and da/dr is not symmetric


@pytest.mark.parametrize("inv_c2", [1e-3, 1e-4])
def test_relativistic_adjoint_matches_finite_differences(inv_c2):
    # finite differences of the map iterated to a fixed number of sweeps, against the
    # implicit derivative at the converged point; the point-mass adjoint misses them
    w = W.nbody_venus(2, days=112.5, segments=2, nodes=48, tol=1e-13)
    g = w.groups[0]
    m = oracle.Model(1.0, w.pert, 0.0, inv_c2=inv_c2)
    gbar = np.random.default_rng(11).standard_normal((2, 6))
    gr = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, m, gbar)
    h = 1e-6
    fd = np.zeros((2, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        sp, _ = oracle.propagate(w.ics + e, g.t0, g.tf, g.nodes, g.segments, g.tol, m, fixed_iters=40)
        sm, _ = oracle.propagate(w.ics - e, g.t0, g.tf, g.nodes, g.segments, g.tol, m, fixed_iters=40)
        fd[:, k] = ((sp - sm) * gbar).sum(axis=1) / (2 * h)
    np.testing.assert_allclose(gr, fd, rtol=0, atol=1e-8 * np.abs(fd).max())
    pm = oracle.adjoint(w.ics, g.t0, g.tf, g.nodes, g.segments, g.tol, oracle.Model(1.0, w.pert, 0.0), gbar)
    assert np.abs(pm - fd).max() > 100 * 1e-8 * np.abs(fd).max()


# -- the first post-Newtonian Lagrangian ---------------------------------------------------
# The relativistic N-body equations are the Euler-Lagrange equations of the 1PN Lagrangian
# in harmonic coordinates (the Einstein-Infeld-Hoffmann Lagrangian), with the test body's own
# acceleration replaced by its Newtonian value inside the O(1/c^2) terms.  For a massless
# body, the terms linear in its mass are, per unit mass (eps = 1/c^2, rho_b = |r - r_b|,
# n_b = (r - r_b)/rho_b, U_b the potential at body b of the other major bodies):
#   L = v^2/2 + eps v^4/8
#       + sum_b mu_b/rho_b [1 + eps (3 v^2 + 3 v_b^2 - 7 v.v_b - (n_b.v)(n_b.v_b))/2]
#       - eps/2 (sum_b mu_b/rho_b)^2 - eps sum_b mu_b U_b/rho_b.
# Solving d/dt dL/dv = dL/dr exactly, for major bodies on prescribed paths, therefore gives
# the relativistic acceleration up to O(eps^2).  The check below differentiates L
# numerically and never uses the acceleration formula, so it pins every term of it: the
# major bodies' velocities, their accelerations (through d/dt of dL/dv) and their
# potentials.  A wrong term leaves an O(eps) difference, which halves when eps halves
# instead of falling by four.

def _paths(seed):
    """Three major bodies in uniform acceleration (positions, velocities, accelerations at
    t = 0), their parameters, and a massless body's state."""
    rng = np.random.default_rng(seed)
    r0 = rng.normal(size=(3, 3)) * 1.2
    v0 = rng.normal(size=(3, 3)) * 0.4
    a0 = rng.normal(size=(3, 3)) * 0.5
    mu = rng.uniform(0.05, 0.3, 3)
    y = np.concatenate([rng.normal(size=3) * 0.3, rng.normal(size=3) * 0.5])
    U = np.array([sum(mu[c] / np.linalg.norm(r0[b] - r0[c]) for c in range(3) if c != b) for b in range(3)])
    return r0, v0, a0, mu, U + 0.7, y                # + a distant mass's constant potential


def _lagrangian(r, v, t, body, eps):
    r0, v0, a0, mu, U = body
    L = 0.5 * v @ v + eps * (v @ v) ** 2 / 8
    phi = 0.0
    for b in range(len(mu)):
        rb, vb = r0[b] + v0[b] * t + 0.5 * a0[b] * t * t, v0[b] + a0[b] * t
        d = r - rb
        rho = np.linalg.norm(d)
        n = d / rho
        L += mu[b] / rho * (1 + eps * (3 * v @ v + 3 * vb @ vb - 7 * v @ vb - (n @ v) * (n @ vb)) / 2)
        L -= eps * mu[b] * U[b] / rho
        phi += mu[b] / rho
    return L - eps * phi * phi / 2


def _grad(f, x, h=1e-6):
    e = np.eye(len(x))
    return np.stack([(f(x + h * e[k]) - f(x - h * e[k])) / (2 * h) for k in range(len(x))], axis=-1)


def _momentum(r, v, t, body, eps):
    """dL/dv, differentiated by hand (checked against central differences of L below)."""
    r0, v0, a0, mu, U = body
    p = v + eps * (v @ v) * v / 2
    for b in range(len(mu)):
        rb, vb = r0[b] + v0[b] * t + 0.5 * a0[b] * t * t, v0[b] + a0[b] * t
        d = r - rb
        rho = np.linalg.norm(d)
        n = d / rho
        p = p + eps * mu[b] / rho * (6 * v - 7 * vb - n * (n @ vb)) / 2
    return p


def _euler_lagrange_accel(y, body, eps, h=1e-6):
    """Acceleration from d/dt dL/dv = dL/dr, the derivatives of L and of dL/dv by central
    differences: (d2L/dv dv) a = dL/dr - (d2L/dv dr) v - d2L/dv dt."""
    r, v = y[:3], y[3:]
    p = lambda rr, vv, t: _momentum(rr, vv, t, body, eps)
    assert np.allclose(p(r, v, 0.0), _grad(lambda w: _lagrangian(r, w, 0.0, body, eps), v), rtol=0, atol=1e-9)
    dLdr = _grad(lambda w: _lagrangian(w, v, 0.0, body, eps), r, h)
    Jr = _grad(lambda w: p(w, v, 0.0), r, h)
    Jv = _grad(lambda w: p(r, w, 0.0), v, h)
    dpt = (p(r, v, h) - p(r, v, -h)) / (2 * h)
    return np.linalg.solve(Jv, dLdr - Jr @ v - dpt)


@pytest.mark.parametrize("seed", range(4))
def test_euler_lagrange_equations_of_the_1pn_lagrangian(seed):
    r0, v0, a0, mu, U, y = _paths(seed)
    body = (r0, v0, a0, mu, U)
    newton = oracle.accel_eih_bodies(y, r0, v0, a0, mu, U, 0.0)
    assert np.linalg.norm(_euler_lagrange_accel(y, body, 0.0) - newton) < 1e-7
    d = {}
    for eps in (4e-4, 2e-4):
        a = oracle.accel_eih_bodies(y, r0, v0, a0, mu, U, eps)
        assert np.linalg.norm(a - newton) > 50 * eps * eps       # the 1PN part is O(eps)
        d[eps] = np.linalg.norm(_euler_lagrange_accel(y, body, eps) - a)
    assert d[4e-4] < 20 * 4e-4 ** 2, d
    assert 3.7 < d[4e-4] / d[2e-4] < 4.3, d                      # O(eps^2), not O(eps)
