"""FP64 CPU oracle for batched Picard-Chebyshev propagation (ctypes wrapper).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import this package.  It shares no
code with the HIP path.  The arithmetic lives in ``pc_oracle.c``; this module
only builds it with gcc (on first use, or when the source is newer than the
library) and marshals numpy arrays.

Paper: Masat, Colombo, Boutonnet, arXiv 2301.03989.  Each function cites the
passage it follows in ``pc_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pc_oracle.c")
_LIB = os.path.join(_HERE, "libpc_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile pc_oracle.c into libpc_oracle.so with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_propagate.restype = ctypes.c_int
        lib.orc_propagate.argtypes = [
            ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
            ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp, _ip, _dp, _dp, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int]
        lib.orc_second_order_step.restype = None
        lib.orc_second_order_step.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, _dp, _dp]
        lib.orc_propagate_group.restype = ctypes.c_int
        lib.orc_propagate_group.argtypes = [
            ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
            ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
            ctypes.c_int, _dp, ctypes.c_double, _dp, _ip, _dp, _dp, ctypes.c_int]
        lib.orc_picard_step.restype = None
        lib.orc_picard_step.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        lib.orc_nodes.restype = None
        lib.orc_nodes.argtypes = [ctypes.c_int, _dp]
        lib.orc_accel.restype = None
        lib.orc_accel.argtypes = [_dp, ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]
        lib.orc_accel_t.restype = None
        lib.orc_accel_t.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp,
                                    ctypes.c_double, _dp]
        lib.orc_ephem.restype = None
        lib.orc_ephem.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp]
        lib.orc_kepler.restype = ctypes.c_int
        lib.orc_kepler.argtypes = [_dp, ctypes.c_double, _dp]
        lib.orc_accel_jac_t.restype = None
        lib.orc_accel_jac_t.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp,
                                        ctypes.c_double, _dp]
        lib.orc_rk4.restype = None
        lib.orc_rk4.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_long,
                                ctypes.c_double, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp]
        lib.orc_accel_eih_t.restype = None
        lib.orc_accel_eih_t.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp,
                                        ctypes.c_double, ctypes.c_double, _dp]
        lib.orc_accel_eih_bodies.restype = None
        lib.orc_accel_eih_bodies.argtypes = [_dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, ctypes.c_double, _dp]
        lib.orc_flyby_ratio.restype = None
        lib.orc_flyby_ratio.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, _dp]
        lib.orc_ephem_state.restype = None
        lib.orc_ephem_state.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp, _dp]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp if a.dtype == np.float64 else _ip)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Model:
    """Point-mass force model: Sun (mu_sun) plus perturbers on Keplerian orbits.

    ``pert`` is an array [n_pert, 7] of (mu_p, a, e, inc, raan, argp, M0) with
    angles in radians and M0 the mean anomaly at ``epoch``.  ``inv_c2`` > 0 (1/c^2
    in the model's units) selects the Einstein-Infeld-Hoffmann dynamics (orc_accel_eih).
    """

    def __init__(self, mu_sun=1.0, pert=None, epoch=0.0, inv_c2=0.0):
        self.mu_sun = float(mu_sun)
        self.pert = _f64(np.zeros((0, 7)) if pert is None else pert).reshape(-1, 7)
        self.epoch = float(epoch)
        self.inv_c2 = float(inv_c2)

    @property
    def n_pert(self):
        return int(self.pert.shape[0])

    def _pert_ptr(self):
        # ctypes needs a valid pointer even when there are no perturbers
        if self.n_pert == 0:
            self._dummy = np.zeros(7)
            return _ptr(self._dummy)
        return _ptr(self.pert)


def propagate(ics, t0, tf, nodes, segments, tol, model=None, *, tol_mode=0, max_iter=64,
              fixed_iters=0, init=0, want_bounds=False, want_nodes=False, threads=0, conv=0,
              order=1, feedback=0, guess=None, refine=0):
    """Propagate ICs [n,6] over [t0, tf] (scalars or per-IC arrays).

    Returns (states[n,6], iters[n,segments]) and, when asked, the segment-boundary
    states [n,S+1,6] and the node states [n,S,N,6].  ``init``: 0 Kepler, 1 cold.
    ``conv``: 0 = stopping rule per IC; 1 = one stopping decision for all the ICs, on
    the largest error over them (orc_propagate_group; scalar t0 and tf, no fixed sweeps).
    ``order``: 1 = the first-order iteration, 2 = the second-order form (velocity and
    position both from the accelerations); ``feedback``: 1 = the second-order form with
    integral error feedback (orc_propagate).  ``init`` 2 starts every segment from
    ``guess`` [n, S, N, 6] (node states of an earlier propagation).  ``refine`` > 0: a
    segment that does not converge is solved again as 2, 4, ... 2^refine equal sub-segments
    (orc_propagate; not with node outputs or a guess).
    """
    lib = _load()
    model = model or Model()
    ics = _f64(ics).reshape(-1, 6)
    n = ics.shape[0]
    t0a = _f64(np.broadcast_to(np.asarray(t0, dtype=np.float64), (n,)))
    tfa = _f64(np.broadcast_to(np.asarray(tf, dtype=np.float64), (n,)))
    S, N = int(segments), int(nodes)
    states = np.zeros((n, 6))
    iters = np.zeros((n, S), dtype=np.int32)
    bounds = np.zeros((n, S + 1, 6)) if want_bounds else None
    nodes_out = np.zeros((n, S, N, 6)) if want_nodes else None
    if order not in (1, 2) or (feedback and order != 2):
        raise ValueError("order must be 1 or 2, and feedback needs order 2")
    if (init == 2) != (guess is not None):
        raise ValueError("init 2 takes a guess [n, S, N, 6], and only it does")
    garr = _f64(guess, (n, S, N, 6)) if guess is not None else None
    if refine and (want_nodes or guess is not None or conv == 1):
        raise ValueError("refinement takes no node outputs, no guess and the per-IC rule")
    if conv == 1:
        if order != 1 or init == 2:
            raise ValueError("group-max convergence is written for the first-order iteration")
        if np.ndim(t0) or np.ndim(tf) or fixed_iters or model.inv_c2:
            raise ValueError("group-max convergence takes one t0 and tf, no fixed sweeps and "
                             "the point-mass model")
        used = lib.orc_propagate_group(n, _ptr(ics), float(t0), float(tf), N, S, float(tol),
                                       int(tol_mode), int(max_iter), int(init), model.mu_sun,
                                       model.n_pert, model._pert_ptr(), model.epoch, _ptr(states),
                                       iters.ctypes.data_as(_ip), _ptr(bounds), _ptr(nodes_out),
                                       int(threads))
    else:
        used = lib.orc_propagate(n, _ptr(ics), _ptr(t0a), _ptr(tfa), N, S, float(tol), int(tol_mode),
                                 int(max_iter), int(fixed_iters), int(init), model.mu_sun,
                                 model.n_pert, model._pert_ptr(), model.epoch, model.inv_c2, _ptr(states),
                                 iters.ctypes.data_as(_ip), _ptr(bounds), _ptr(nodes_out), int(threads),
                                 int(order), int(feedback), _ptr(garr), int(refine))
    out = [states, iters]
    if want_bounds:
        out.append(bounds)
    if want_nodes:
        out.append(nodes_out)
    propagate.last_threads = used
    return tuple(out)


propagate.last_threads = 1


def flyby_ratio(ics, t0, tf, segments, model, samples=16):
    """Smallest distance of each IC's two-body prediction to any perturber, in Hill radii,
    over ``samples`` CGL points per segment of [t0, tf] (orc_flyby_ratio); 0 for an IC whose
    orbit is not elliptic."""
    lib = _load()
    ics = _f64(ics).reshape(-1, 6)
    out = np.zeros(ics.shape[0])
    lib.orc_flyby_ratio(ics.shape[0], _ptr(ics), float(t0), float(tf), int(segments), int(samples),
                        model.n_pert, model._pert_ptr(), model.epoch, _ptr(out))
    return out


def picard_step(g, y0):
    """Steps (ii)-(v) of one iteration for one trajectory: g [N, ncomp] (w2-scaled
    force matrix) and y0 [ncomp] -> y [N, ncomp]."""
    lib = _load()
    g = _f64(g)
    if g.ndim == 1:
        g = g[:, None]
    N, nc = g.shape
    y0 = _f64(y0).reshape(nc)
    y = np.zeros((N, nc))
    lib.orc_picard_step(N, nc, _ptr(g), _ptr(y0), _ptr(y))
    return y


def second_order_step(a, x0, v0, w2):
    """One second-order update for a single trajectory: accelerations a [N, 3] at the nodes,
    initial position x0 [3] and velocity v0 [3], half-length w2 -> (x [N, 3], v [N, 3])."""
    lib = _load()
    a = _f64(a).reshape(-1, 3)
    N = a.shape[0]
    x0, v0 = _f64(x0).reshape(3), _f64(v0).reshape(3)
    x, v = np.zeros((N, 3)), np.zeros((N, 3))
    lib.orc_second_order_step(N, _ptr(a), _ptr(x0), _ptr(v0), float(w2), _ptr(x), _ptr(v))
    return x, v


def operator2(N):
    """The linear maps a -> (x - x0 - w2 v0 (tau + 1)) / w2^2 and a -> (v - v0) / w2 of the
    second-order update, as N x N matrices (K2, K1) built from unit vectors."""
    K2, K1 = np.zeros((N, N)), np.zeros((N, N))
    for l in range(N):
        a = np.zeros((N, 3))
        a[l, 0] = 1.0
        x, v = second_order_step(a, np.zeros(3), np.zeros(3), 1.0)
        K2[:, l], K1[:, l] = x[:, 0], v[:, 0]
    return K2, K1


def operator(N):
    """The linear map g -> y - y0 of steps (ii)-(v), as an N x N matrix built by
    applying the oracle's update to unit vectors."""
    return picard_step(np.eye(N), np.zeros(N))


def nodes(N):
    lib = _load()
    tau = np.zeros(N)
    lib.orc_nodes(int(N), _ptr(tau))
    return tau


def accel(r, rp, mup, mu_sun=1.0):
    """Acceleration at r [3] from perturbers at rp [P,3] with parameters mup [P]."""
    lib = _load()
    r = _f64(r).reshape(3)
    rp = _f64(rp).reshape(-1, 3)
    mup = _f64(mup).reshape(-1)
    a = np.zeros(3)
    dummy = np.zeros(3)
    lib.orc_accel(_ptr(r), rp.shape[0], _ptr(rp) if rp.size else _ptr(dummy),
                  _ptr(mup) if mup.size else _ptr(dummy), float(mu_sun), _ptr(a))
    return a


def accel_t(r, t, model):
    lib = _load()
    r = _f64(r).reshape(3)
    a = np.zeros(3)
    lib.orc_accel_t(_ptr(r), float(t), model.mu_sun, model.n_pert, model._pert_ptr(),
                    model.epoch, _ptr(a))
    return a


def ephem(el, epoch, t):
    lib = _load()
    el = _f64(el).reshape(7)
    r = np.zeros(3)
    lib.orc_ephem(_ptr(el), float(epoch), float(t), _ptr(r))
    return r


def kepler(y0, dt):
    """Two-body (mu = 1) propagation of y0 by dt; returns (ok, y)."""
    lib = _load()
    y0 = _f64(y0).reshape(6)
    y = np.zeros(6)
    rc = lib.orc_kepler(_ptr(y0), float(dt), _ptr(y))
    return rc == 0, y


def rk4(y0, t0, tf, nsteps, model):
    lib = _load()
    y0 = _f64(y0).reshape(6)
    y = np.zeros(6)
    lib.orc_rk4(_ptr(y0), float(t0), float(tf), int(nsteps), model.mu_sun, model.n_pert,
                model._pert_ptr(), model.epoch, model.inv_c2, _ptr(y))
    return y


def accel_eih_t(y, t, model):
    """Einstein-Infeld-Hoffmann acceleration at the state y (r, v) and time t."""
    lib = _load()
    y = _f64(y).reshape(6)
    a = np.zeros(3)
    lib.orc_accel_eih_t(_ptr(y), float(t), model.mu_sun, model.n_pert, model._pert_ptr(),
                        model.epoch, model.inv_c2, _ptr(a))
    return a


def accel_eih_bodies(y, rb, vb, ab, mub, Ub, inv_c2):
    """The Einstein-Infeld-Hoffmann sums for a massless body at y (r, v) and major bodies
    with positions rb, velocities vb, accelerations ab [nb, 3], parameters mub and
    potentials Ub [nb] (no indirect term)."""
    lib = _load()
    y = _f64(y).reshape(6)
    rb, vb, ab = (_f64(x).reshape(-1, 3) for x in (rb, vb, ab))
    mub, Ub = _f64(mub).reshape(-1), _f64(Ub).reshape(-1)
    a = np.zeros(3)
    lib.orc_accel_eih_bodies(_ptr(y), rb.shape[0], _ptr(rb), _ptr(vb), _ptr(ab), _ptr(mub), _ptr(Ub),
                             float(inv_c2), _ptr(a))
    return a


def ephem_state(el, epoch, t):
    """Position and velocity of a perturber with elements el at time t."""
    lib = _load()
    el = _f64(el).reshape(7)
    r, v = np.zeros(3), np.zeros(3)
    lib.orc_ephem_state(_ptr(el), float(epoch), float(t), _ptr(r), _ptr(v))
    return r, v


def accel_jac_t(r, t, model):
    """da/dr (3x3) of the force model at (r, t)."""
    lib = _load()
    r = _f64(r).reshape(3)
    J = np.zeros(9)
    lib.orc_accel_jac_t(_ptr(r), float(t), model.mu_sun, model.n_pert, model._pert_ptr(),
                        model.epoch, _ptr(J))
    return J.reshape(3, 3)


def _eih_major_bodies(t, model):
    """Major-body states of the relativistic model at time t, as orc_accel_eih builds them:
    the Sun at rest at the origin, the perturbers on their Keplerian orbits (mu = 1) with
    the accelerations of those orbits, and each body's potential of the other major bodies."""
    nb = model.n_pert + 1
    rb, vb, ab = np.zeros((nb, 3)), np.zeros((nb, 3)), np.zeros((nb, 3))
    mub = np.empty(nb)
    mub[0] = model.mu_sun
    for p in range(model.n_pert):
        r, v = ephem_state(model.pert[p], model.epoch, t)
        rb[p + 1], vb[p + 1] = r, v
        ab[p + 1] = -r / np.linalg.norm(r) ** 3
        mub[p + 1] = model.pert[p, 0]
    Ub = np.array([sum(mub[k] / np.linalg.norm(rb[b] - rb[k]) for k in range(nb) if k != b)
                   for b in range(nb)])
    return rb, vb, ab, mub, Ub


def _eih_accel_np(y, rb, vb, ab, mub, Ub, inv_c2):
    """The relativistic sums of Sec. 5.4.1 (PPN beta = gamma = 1, massless body), restated
    in numpy so that they also take a complex state (no indirect term):
      a = sum_b -mu_b d_b / rho_b^3 [1 - (4 Phi + U_b - v^2 - 2 v_b^2 + 4 v.v_b
                                          + 3/2 (d_b.v_b / rho_b)^2 + 1/2 d_b.a_b) / c^2]
        + sum_b mu_b / (c^2 rho_b^3) [d_b.(4 v - 3 v_b)] (v - v_b) + 7/2 sum_b mu_b a_b / (c^2 rho_b)
    with d_b = r - r_b, rho_b = |d_b| (the plain sum of squares, analytic for a complex
    step) and Phi = sum_b mu_b / rho_b."""
    r, v = y[:3], y[3:]
    d = r[None, :] - rb
    rho = np.sqrt((d * d).sum(axis=1))
    phi = (mub / rho).sum()
    v2 = (v * v).sum()
    a = np.zeros(3, dtype=np.result_type(y, 1.0))
    for b in range(rb.shape[0]):
        db, wb, gb = d[b], vb[b], ab[b]
        i3 = 1.0 / rho[b] ** 3
        brk = 1.0 - inv_c2 * (4.0 * phi + Ub[b] - v2 - 2.0 * (wb * wb).sum() + 4.0 * (v * wb).sum()
                              + 1.5 * ((db * wb).sum() / rho[b]) ** 2 + 0.5 * (db * gb).sum())
        a = a - mub[b] * i3 * db * brk
        a = a + inv_c2 * mub[b] * i3 * (db * (4.0 * v - 3.0 * wb)).sum() * (v - wb)
        a = a + 3.5 * inv_c2 * mub[b] * gb / rho[b]
    return a


def accel_eih_jac_t(y, t, model, h=1e-30):
    """da/d(r, v) (3 x 6) of the relativistic acceleration at state y and time t, by the
    complex step: column k is Im a(y + i h e_k) / h, exact to rounding (the indirect term
    does not depend on the state)."""
    bodies = _eih_major_bodies(t, model)
    y = _f64(y).reshape(6)
    J = np.zeros((3, 6))
    for k in range(6):
        yc = y.astype(np.complex128)
        yc[k] += 1j * h
        J[:, k] = _eih_accel_np(yc, *bodies, model.inv_c2).imag / h
    return J


def adjoint(ics, t0, tf, nodes, segments, tol, model=None, gbar_final=None, gbar_nodes=None, *,
            init=0, tol_mode=0, max_iter=64):
    """Gradient dL/dy0 [n, 6] of a loss L(y_final, node states) through the converged
    Picard-Chebyshev map, by implicit differentiation of its discrete fixed point.

    Per segment the converged node states satisfy Y = 1 y0^T + K G(Y), G_j = w2 f(Y_j, t_j)
    (Sec. 2.2 with the fit/integrate/evaluate steps as the linear map K, obtained here by
    applying the oracle's update to unit vectors).  With J_j = w2 df/dy at node j, the
    adjoint mu solves (I - K J)^T mu = gbar (a dense 6N x 6N solve, numpy), and
    dL/dy0 = sum_j mu_j.  With the relativistic model J_j also has the velocity block
    w2 da/dv (accel_eih_jac_t).  Segments are chained backwards: the end node of segment
    s-1 is the initial state of segment s, so its seed is the gradient of segment s.

    gbar_final [n, 6] = dL/dy_final; gbar_nodes [n, S, N, 6] = dL/dY (optional).
    """
    model = model or Model()
    ics = _f64(ics).reshape(-1, 6)
    n = ics.shape[0]
    S, N = int(segments), int(nodes)
    t0a = np.broadcast_to(np.asarray(t0, dtype=np.float64), (n,))
    tfa = np.broadcast_to(np.asarray(tf, dtype=np.float64), (n,))
    _, _, Ys = propagate(ics, t0a, tfa, N, S, tol, model, init=init, tol_mode=tol_mode, max_iter=max_iter,
                         want_nodes=True)
    K = operator(N)
    tau = nodes_(N)
    gbar_final = np.zeros((n, 6)) if gbar_final is None else _f64(gbar_final).reshape(n, 6)
    grads = np.zeros((n, 6))
    eye6 = np.eye(6)
    for m in range(n):
        lam = gbar_final[m].copy()
        h = (tfa[m] - t0a[m]) / S
        for s in range(S - 1, -1, -1):
            Ts, Te = t0a[m] + h * s, t0a[m] + h * (s + 1)
            w1, w2 = 0.5 * (Te + Ts), 0.5 * (Te - Ts)
            Jb = np.zeros((N, 6, 6))
            for j in range(N):
                Jb[j, :3, 3:] = w2 * np.eye(3)
                if model.inv_c2:   # the relativistic force depends on the velocity too
                    Jb[j, 3:, :] = w2 * accel_eih_jac_t(Ys[m, s, j], w2 * tau[j] + w1, model)
                else:
                    Jb[j, 3:, :3] = w2 * accel_jac_t(Ys[m, s, j, :3], w2 * tau[j] + w1, model)
            # M[(j,a),(l,b)] = delta - K[j,l] J_l[a,b]
            M = np.eye(6 * N) - np.einsum("jl,lab->jalb", K, Jb).reshape(6 * N, 6 * N)
            gb = np.zeros((N, 6))
            gb[N - 1] += lam
            if gbar_nodes is not None:
                gb += gbar_nodes[m, s]
            mu = np.linalg.solve(M.T, gb.reshape(-1)).reshape(N, 6)
            lam = mu.sum(axis=0)
        grads[m] = lam
    return grads


nodes_ = nodes
