"""Pins of the oracle's flyby screen (orc_flyby_ratio): the smallest distance of an IC's
two-body prediction to any perturber, in Hill radii a_p (mu_p/3)^(1/3), over the CGL
sample points of every segment (the outer-level isolation of flyby sub-groups, Sec. 3.2;
flyby detection, Sec. 7).  Pinned by closed forms of coplanar circular motion, computed
here without any Kepler solver: two circular orbits at their own angular rates, and an IC
that shares a perturber's circular orbit a fixed angle behind it (constant chord)."""
import numpy as np

import oracle

MU = 3.040e-6   # an Earth-like mass ratio


def _samples(t0, tf, S, K):
    h = (tf - t0) / S
    out = []
    for s in range(S):
        Ts, Te = t0 + h * s, t0 + h * (s + 1)
        w1, w2 = 0.5 * (Te + Ts), 0.5 * (Te - Ts)
        out.append(w2 * -np.cos(np.pi * np.arange(K) / (K - 1)) + w1)
    return np.concatenate(out)


def _circular_ic(r, phase):
    v = r ** -0.5
    return np.array([r * np.cos(phase), r * np.sin(phase), 0.0, -v * np.sin(phase), v * np.cos(phase), 0.0])


def test_two_circular_orbits_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(6):
        r1, a, ph1, ph2 = rng.uniform(0.6, 1.4), rng.uniform(0.7, 1.3), rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi)
        t0, tf, S = rng.uniform(-1, 1), rng.uniform(3, 12), int(rng.integers(1, 6))
        pert = np.array([[MU, a, 0.0, 0.0, 0.0, 0.0, ph2]])
        got = oracle.flyby_ratio(_circular_ic(r1, ph1)[None], t0, tf, S, oracle.Model(1.0, pert, 0.0), samples=16)[0]
        t = _samples(t0, tf, S, 16)
        x = r1 * np.stack([np.cos(ph1 + r1 ** -1.5 * (t - t0)), np.sin(ph1 + r1 ** -1.5 * (t - t0))])
        xp = a * np.stack([np.cos(ph2 + a ** -1.5 * t), np.sin(ph2 + a ** -1.5 * t)])
        want = np.linalg.norm(x - xp, axis=0).min() / (a * (MU / 3) ** (1 / 3))
        assert abs(got - want) <= 1e-10 * want, (got, want)


def test_shared_circular_orbit_keeps_a_constant_chord():
    a, delta = 1.0, 0.02
    pert = np.array([[MU, a, 0.0, 0.0, 0.0, 0.0, 0.3]])
    ic = _circular_ic(a, 0.3 - delta)
    got = oracle.flyby_ratio(ic[None], 0.0, 20.0, 7, oracle.Model(1.0, pert, 0.0))[0]
    want = 2 * a * np.sin(delta / 2) / (a * (MU / 3) ** (1 / 3))
    assert abs(got - want) <= 1e-10 * want


def test_hill_radius_scaling_unbound_orbits_and_massless_bodies():
    pert = np.array([[3.0, 2.0, 0.0, 0.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0]])
    ic = _circular_ic(1.0, 0.0)
    # mu_p = 3: the Hill radius is a_p itself; the massless body is skipped
    r = oracle.flyby_ratio(ic[None], 0.0, 0.0 + 1e-9, 1, oracle.Model(1.0, pert, 0.0), samples=2)[0]
    assert abs(r - 1.0 / 2.0) < 1e-8
    only_massless = oracle.flyby_ratio(ic[None], 0.0, 1.0, 1, oracle.Model(1.0, pert[1:], 0.0))[0]
    assert np.isinf(only_massless)
    hyper = ic.copy()
    hyper[3:] *= 1.6   # above escape speed
    assert oracle.flyby_ratio(hyper[None], 0.0, 1.0, 2, oracle.Model(1.0, pert, 0.0))[0] == 0.0
