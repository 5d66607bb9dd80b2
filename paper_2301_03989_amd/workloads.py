"""Seeded synthetic workloads (heliocentric ensembles) for propagation runs.

This module only draws inputs: initial conditions, perturber elements and the
run settings of each workload.  It holds none of the propagation method's
arithmetic; the conversion from orbital elements to Cartesian states used to
build the initial conditions is input generation, done here in numpy.

Units: mu_Sun = 1, AU, and the time unit TU = 1/k days with k the Gaussian
gravitational constant, so an a = 1 AU orbit has period 2 pi TU.

The paper's own workload (13509 initial conditions from a Solar Orbiter-like
Venus resonance optimisation, 200 nodes over about 0.87 orbital periods, one
segment per initial condition, relativistic N-body dynamics with real
ephemerides; Sec. 6.1-6.2) is not available.  The ensembles below stand in for
it: Venus-resonant heliocentric orbits near a = 0.75 AU, perturbed by the Sun
plus eight planets as point masses on seeded Keplerian orbits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

K_GAUSS = 0.01720209895
TU_DAYS = 1.0 / K_GAUSS          # 58.1324409... days per time unit
DEG = math.pi / 180.0

# (name, mu_p = planet/Sun mass ratio, semi-major axis in AU)
PLANETS = (
    ("Mercury", 1.66e-7, 0.38710),
    ("Venus", 2.448e-6, 0.72333),
    ("EarthMoon", 3.040e-6, 1.00000),
    ("Mars", 3.227e-7, 1.52366),
    ("Jupiter", 9.548e-4, 5.20336),
    ("Saturn", 2.859e-4, 9.53707),
    ("Uranus", 4.366e-5, 19.19126),
    ("Neptune", 5.151e-5, 30.06896),
)
PLANET_SEED = 230103989


def planet_elements(seed: int = PLANET_SEED) -> np.ndarray:
    """Perturber table [8, 7]: (mu_p, a, e, inc, raan, argp, M0), angles in rad,
    M0 at epoch 0.  a = textbook value x U[0.99, 1.01], e ~ U[0, 0.05],
    inc ~ U[0, 3 deg], raan, argp, M0 ~ U[0, 360 deg)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((len(PLANETS), 7))
    for p, (_, mu, a) in enumerate(PLANETS):
        out[p, 0] = mu
        out[p, 1] = a * rng.uniform(0.99, 1.01)
        out[p, 2] = rng.uniform(0.0, 0.05)
        out[p, 3] = rng.uniform(0.0, 3.0) * DEG
        out[p, 4] = rng.uniform(0.0, 360.0) * DEG
        out[p, 5] = rng.uniform(0.0, 360.0) * DEG
        out[p, 6] = rng.uniform(0.0, 360.0) * DEG
    return out


def elements_to_states(a, e, inc, raan, argp, M) -> np.ndarray:
    """Cartesian states [n, 6] (mu = 1) of orbits given by classical elements."""
    a, e, inc, raan, argp, M = (np.asarray(v, dtype=np.float64).reshape(-1)
                                for v in (a, e, inc, raan, argp, M))
    E = np.where(e < 0.8, M, np.pi)
    for _ in range(60):
        E = E - (E - e * np.sin(E) - M) / (1.0 - e * np.cos(E))
    cE, sE = np.cos(E), np.sin(E)
    b = a * np.sqrt(1.0 - e * e)
    rr = a * (1.0 - e * cE)
    n = np.sqrt(1.0 / a ** 3)
    xp, yp = a * (cE - e), b * sE
    vxp, vyp = -a * a * n * sE / rr, a * b * n * cE / rr
    cO, sO, cw, sw, ci, si = (np.cos(raan), np.sin(raan), np.cos(argp), np.sin(argp),
                              np.cos(inc), np.sin(inc))
    P = np.stack([cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si], axis=1)
    Q = np.stack([-cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si], axis=1)
    r = xp[:, None] * P + yp[:, None] * Q
    v = vxp[:, None] * P + vyp[:, None] * Q
    return np.concatenate([r, v], axis=1)


@dataclass
class Group:
    """One outer-level group (two-level augmentation): ICs [ic_offset, ic_offset+n_ic)
    sharing nodes, segments, interval and tolerance."""
    ic_offset: int
    n_ic: int
    t0: float
    tf: float
    nodes: int
    segments: int
    tol: float


@dataclass
class Workload:
    name: str
    ics: np.ndarray                      # [n, 6]
    groups: list                         # list[Group]
    pert: np.ndarray                     # [P, 7] perturber elements (P = 0: Sun only)
    init: int = 0                        # 0 Kepler warm start, 1 cold start
    precision: int = 0                   # 0 FP64, 1 FP32 sweeps then FP64
    mu_sun: float = 1.0
    epoch: float = 0.0
    inv_c2: float = 0.0                  # > 0: Einstein-Infeld-Hoffmann dynamics, 1/c^2
    meta: dict = field(default_factory=dict)

    @property
    def n_ic(self):
        return int(self.ics.shape[0])

    def subset(self, idx):
        """A workload made of the ICs at ``idx`` (indices into ``ics``), with the
        group structure restricted to them.  Used for bounded oracle samples."""
        idx = np.asarray(idx)
        parts, groups, off = [], [], 0
        for g in self.groups:
            sel = idx[(idx >= g.ic_offset) & (idx < g.ic_offset + g.n_ic)]
            if sel.size == 0:
                continue
            parts.append(self.ics[sel])
            groups.append(Group(off, int(sel.size), g.t0, g.tf, g.nodes, g.segments, g.tol))
            off += int(sel.size)
        return Workload(self.name + "-subset", np.concatenate(parts), groups, self.pert,
                        self.init, self.precision, self.mu_sun, self.epoch, self.inv_c2, dict(self.meta))


# ---------------------------------------------------------------------------
# Reference orbit of the N-body ensembles: a Venus-crossing orbit at a = 0.75 AU.
# M0 is chosen so that the nominal trajectory keeps at least 0.05 AU from
# Venus over the 450-day span (checked by the test suite with the oracle).
REF_ORBIT = dict(a=0.75, e=0.2, inc=3.0 * DEG, raan=0.0, argp=0.0, M0=235.0 * DEG)


def _perturbed_ensemble(n, seed, dr=1e-4, dv=1e-4):
    rng = np.random.default_rng(seed)
    ref = elements_to_states(REF_ORBIT["a"], REF_ORBIT["e"], REF_ORBIT["inc"],
                             REF_ORBIT["raan"], REF_ORBIT["argp"], REF_ORBIT["M0"])[0]
    delta = np.concatenate([rng.uniform(-dr, dr, size=(n, 3)),
                            rng.uniform(-dv, dv, size=(n, 3))], axis=1)
    return ref[None, :] + delta


def sun_only_kepler(n_ic: int = 64, seed: int = 101) -> Workload:
    """Sun-only two-body ensemble: a ~ U[0.7, 1.0], e ~ U[0, 0.3], inc ~ U[0, 10 deg],
    raan/argp/M ~ U[0, 360 deg); one orbital period of each IC in 4 segments of
    64 nodes, tol 1e-13, cold start.  Each IC is its own group (its own period)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.7, 1.0, n_ic)
    e = rng.uniform(0.0, 0.3, n_ic)
    inc = rng.uniform(0.0, 10.0, n_ic) * DEG
    raan, argp, M = (rng.uniform(0.0, 360.0, n_ic) * DEG for _ in range(3))
    ics = elements_to_states(a, e, inc, raan, argp, M)
    period = 2.0 * np.pi * a ** 1.5
    groups = [Group(i, 1, 0.0, float(period[i]), 64, 4, 1e-13) for i in range(n_ic)]
    return Workload("sun-only-kepler-64", ics, groups, np.zeros((0, 7)), init=1,
                    meta=dict(a=a, e=e, inc=inc, period=period))


def nbody_venus(n_ic: int = 4096, seed: int = 102, days: float = 450.0, segments: int = 8,
                nodes: int = 128, tol: float = 1e-12, precision: int = 0,
                name: str = "nbody-venus-4096") -> Workload:
    """Sun + 8 planets; n_ic ICs = reference orbit + dr_k ~ U[-1e-4, 1e-4] AU,
    dv_k ~ U[-1e-4, 1e-4] AU/TU; span `days` in `segments` equal segments of
    `nodes` nodes; Kepler warm start."""
    ics = _perturbed_ensemble(n_ic, seed)
    tf = days / TU_DAYS
    return Workload(name, ics, [Group(0, n_ic, 0.0, tf, nodes, segments, tol)],
                    planet_elements(), init=0, precision=precision,
                    meta=dict(days=days))


def uneven_batch(n_ic: int = 65536, seed: int = 103) -> Workload:
    """Uneven two-level batch: a ~ U[0.7, 1.0], e ~ U[0, 0.6], inc ~ U[0, 10 deg];
    15 groups = nodes {64, 128, 256} x segments {8, 16, 24, 32, 40} with sizes
    from a seeded multinomial; each segment lasts pi/4 TU (1/8 of an a = 1 orbit)."""
    rng = np.random.default_rng(seed)
    shapes = [(N, S) for N in (64, 128, 256) for S in (8, 16, 24, 32, 40)]
    w = rng.uniform(0.5, 1.5, len(shapes))
    sizes = rng.multinomial(n_ic - len(shapes), w / w.sum()) + 1
    a = rng.uniform(0.7, 1.0, n_ic)
    e = rng.uniform(0.0, 0.6, n_ic)
    inc = rng.uniform(0.0, 10.0, n_ic) * DEG
    raan, argp, M = (rng.uniform(0.0, 360.0, n_ic) * DEG for _ in range(3))
    ics = elements_to_states(a, e, inc, raan, argp, M)
    groups, off = [], 0
    for (N, S), sz in zip(shapes, sizes):
        groups.append(Group(off, int(sz), 0.0, S * np.pi / 4.0, N, S, 1e-12))
        off += int(sz)
    return Workload("uneven-batch-65536", ics, groups, planet_elements(), init=0)


def eccentric(nodes: int, n_ic: int = 16384, seed: int = 108, segments: int = 16) -> Workload:
    """One node count of the uneven batch's recipe: a ~ U[0.7, 1.0], e ~ U[0, 0.6],
    inc ~ U[0, 10 deg], ``segments`` segments of pi/4 TU at ``nodes`` nodes, tol 1e-12,
    Sun + 8 planets.  Used to profile the job body of each node count on its own."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.7, 1.0, n_ic)
    e = rng.uniform(0.0, 0.6, n_ic)
    inc = rng.uniform(0.0, 10.0, n_ic) * DEG
    raan, argp, M = (rng.uniform(0.0, 360.0, n_ic) * DEG for _ in range(3))
    ics = elements_to_states(a, e, inc, raan, argp, M)
    return Workload(f"eccentric-{n_ic}-n{nodes}", ics,
                    [Group(0, n_ic, 0.0, segments * np.pi / 4.0, nodes, segments, 1e-12)], planet_elements(), init=0)


def long_segments(n_ic: int = 4096, seed: int = 107, nodes: int = 128, segments: int = 2,
                  seg_len: float = np.pi, e_max: float = 0.4) -> Workload:
    """Long segments: a ~ U[0.7, 1.0], e ~ U[0, e_max], inc ~ U[0, 10 deg], Sun + 8
    planets, ``segments`` segments of ``seg_len`` TU (default half an orbit of a = 1) at
    ``nodes`` nodes, tol 1e-12, Kepler warm start.  At the defaults the ICs need 20 to 32
    sweeps per segment (median 26), and the change between sweeps settles near 1e-14, far
    below tol, so a sweep budget of 24 (max_iter) leaves most segments unconverged for a
    reason other than rounding: the input of adaptive segment refinement.  (Much longer
    segments at 256 nodes settle at 1e-12..1e-11, where a 1e-12 stopping rule no longer
    separates converged from unconverged.)"""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.7, 1.0, n_ic)
    e = rng.uniform(0.0, e_max, n_ic)
    inc = rng.uniform(0.0, 10.0, n_ic) * DEG
    raan, argp, M = (rng.uniform(0.0, 360.0, n_ic) * DEG for _ in range(3))
    ics = elements_to_states(a, e, inc, raan, argp, M)
    return Workload(f"long-segments-{n_ic}", ics, [Group(0, n_ic, 0.0, segments * seg_len, nodes, segments, 1e-12)],
                    planet_elements(), init=0)


def mixed_precision(n_ic: int = 262144, seed: int = 104) -> Workload:
    """The N-body Venus ensemble at 262144 ICs, FP32 sweeps then FP64 refinement."""
    return nbody_venus(n_ic, seed, precision=1, name="nbody-venus-262144-fp32-fp64")


def adjoint_ensemble(n_ic: int = 16384, seed: int = 105, nodes: int = 128, eih: bool = False) -> Workload:
    """The N-body Venus ensemble at 16384 ICs over 256 days in 5 segments, tol 1e-13
    (128 nodes; the 256-node variant runs the adjoint's node-row jobs; eih: with the
    relativistic dynamics at the physical 1/c^2)."""
    w = nbody_venus(n_ic, seed, days=256.0, segments=5, tol=1e-13, nodes=nodes,
                    name="nbody-venus-16384-256d" + ("" if nodes == 128 else f"-n{nodes}") + ("-eih" if eih else ""))
    if eih:
        w.inv_c2 = 1.0 / (C_AU_TU * C_AU_TU)
    return w


# speed of light in AU per time unit (299792.458 km/s, 1 AU = 149597870.7 km)
C_AU_TU = 299792.458 * TU_DAYS * 86400.0 / 149597870.7


def relativistic(n_ic: int = 4096, seed: int = 102) -> Workload:
    """The N-body Venus ensemble with the Einstein-Infeld-Hoffmann dynamics (the
    paper's relativistic restricted problem, Sec. 5.4.1): 1/c^2 in AU/TU units."""
    w = nbody_venus(n_ic, seed, name="nbody-venus-4096-eih")
    w.inv_c2 = 1.0 / (C_AU_TU * C_AU_TU)
    return w


def paper_configuration(n_ic: int = 13509, seed: int = 113) -> Workload:
    """A stand-in for the paper's own timing run (Sec. 6): 13509 ICs, the relativistic
    dynamics, one segment of 200 nodes over 0.87 of the orbital period, relative tolerance
    1e-12, cold start (about 40 sweeps, as the paper reports 41-42).  The paper's ICs come
    from a Venus-resonance optimisation that is not available; these are the Venus
    ensemble's reference orbit (a = 0.75, e = 0.2) perturbed by up to 1e-4 in each
    component."""
    ics = _perturbed_ensemble(n_ic, seed)
    tf = 0.87 * 2.0 * np.pi * REF_ORBIT["a"] ** 1.5
    w = Workload("paper-configuration-13509", ics, [Group(0, n_ic, 0.0, tf, 200, 1, 1e-12)],
                 planet_elements(), init=1)
    w.inv_c2 = 1.0 / (C_AU_TU * C_AU_TU)
    return w


WORKLOADS = {
    "sun-only-kepler-64": sun_only_kepler,
    "nbody-venus-4096": nbody_venus,
    "uneven-batch-65536": uneven_batch,
    "nbody-venus-262144-fp32-fp64": mixed_precision,
    "nbody-venus-16384-256d": adjoint_ensemble,
    "nbody-venus-16384-256d-n256": lambda: adjoint_ensemble(nodes=256),
    "nbody-venus-16384-256d-eih": lambda: adjoint_ensemble(eih=True),
    "nbody-venus-4096-eih": relativistic,
    "eccentric-16384-n64": lambda: eccentric(64),
    "eccentric-16384-n128": lambda: eccentric(128),
    "eccentric-16384-n256": lambda: eccentric(256),
    "long-segments-4096": long_segments,
    "paper-configuration-13509": paper_configuration,
}
