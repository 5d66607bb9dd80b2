/*
 * pc_oracle.c -- plain FP64 CPU oracle for batched Picard-Chebyshev propagation.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load this library.  It shares no
 * code, header, table or constant generator with the HIP path: it is a slow,
 * step-by-step restatement of the method used to check the GPU results.
 *
 * Paper: Masat, Colombo, Boutonnet, "GPU-based high-precision orbital
 * propagation of large sets of initial conditions through Picard-Chebyshev
 * augmentation" (arXiv 2301.03989).
 *
 * What is computed, per initial condition (IC), independently of all others
 * (the paper's "independent runs" workflow, Sec. 5.1, with a per-IC stopping
 * rule, i.e. the per-block error of Sec. 3.2 with blocks of one member):
 *
 *   segments    T_s = t0 + s (tf - t0) / S, s = 0..S, integrated in sequence
 *               (piecewise integration, Sec. 2.2; tf < t0 integrates backward)
 *   nodes       tau_j = -cos(j pi / (N-1)), t_j = w2 tau_j + w1,
 *               w1 = (T_{s+1} + T_s)/2, w2 = (T_{s+1} - T_s)/2   (Sec. 2.2, eqs. chnodes1/2)
 *   guess       cold: y_j = y0; warm: two-body Kepler (mu = 1) from y0   (Sec. 2.1)
 *   iteration   (i)   g_j = w2 f(y_j, t_j)                 (force matrix F, Sec. 2.2)
 *               (ii)  c_k = 2/(N-1) sum''_j g_j T_k(tau_j), k = 0..N-2   (Chebyshev fit)
 *               (iii) b_k = (c_{k-1} - c_{k+1}) / (2k), k = 1..N-1, c_{N-1} = c_N = 0
 *               (iv)  b_0 = 2 y0 - 2 sum_k (-1)^k b_k     (the "B_1 = S A F + 2 y_0" row)
 *               (v)   y_j = b_0/2 + sum_k b_k T_k(tau_j)   (Y = C B)
 *               (vi)  e = max_j max(|dr_j|/|r_j|, |dv_j|/|v_j|); stop when e < tol
 *   chaining    y0 of segment s+1 = last node of segment s
 *
 * The paper defines A, C and S only by citation (Sec. 2.2); steps (ii)-(v)
 * are the Chebyshev fit/integrate/evaluate they stand for, with the constant
 * term in the half-coefficient convention that the "2 y_0" term implies.
 *
 * Force model (point masses, heliocentric frame with the indirect term):
 *   a(r,t) = -mu_S r/|r|^3 - sum_p mu_p [ (r - r_p)/|r - r_p|^3 + r_p/|r_p|^3 ]
 * with perturber p on a fixed Keplerian orbit about the Sun (mu = 1).  The
 * paper's own model is relativistic EIH with real ephemerides (Sec. 5.4.1);
 * this point-mass model is the workload's substitute for it.  As the paper
 * does (Sec. 5.4.1), perturber positions are evaluated once per node before
 * the iterations of a segment.
 *
 * Relativistic option (inv_c2 = 1/c^2 > 0): the paper's restricted N-body
 * problem in the Einstein-Infeld-Hoffmann form it cites (Sec. 5.4.1: the
 * acceleration depends on the position and velocity of the propagated body
 * and on the positions, velocities, accelerations and potentials of the
 * major bodies), restated in orc_accel_eih for a massless body with the PPN
 * parameters beta = gamma = 1.  The major bodies are the Sun, fixed at the
 * origin, and the perturbers on their Keplerian orbits, whose velocities and
 * accelerations are the time derivatives of those orbits; the Newtonian
 * indirect term is kept, so that inv_c2 = 0 gives the point-mass model.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Two-body Kepler orbits (mu = 1)                                           */
/* ------------------------------------------------------------------------ */

/* Solve Kepler's equation E - e sin E = M for the eccentric anomaly (Newton). */
static double orc_solve_kepler_E(double M, double e)
{
    double Mr = fmod(M, 2.0 * ORC_PI);
    if (Mr > ORC_PI) Mr -= 2.0 * ORC_PI;
    if (Mr < -ORC_PI) Mr += 2.0 * ORC_PI;
    double E = (e < 0.8) ? Mr : (Mr >= 0 ? ORC_PI : -ORC_PI);
    for (int it = 0; it < 100; ++it) {
        double f = E - e * sin(E) - Mr;
        double fp = 1.0 - e * cos(E);
        double dE = f / fp;
        E -= dE;
        if (fabs(dE) <= 1e-16 * (1.0 + fabs(E))) break;
    }
    return E + (M - Mr);
}

/* Heliocentric position of a body with elements
 * el = {mu_p, a, e, inc, raan, argp, M0} (angles in radians) at time t,
 * where M0 is the mean anomaly at time `epoch`. */
void orc_ephem(const double* el, double epoch, double t, double r[3])
{
    double a = el[1], e = el[2], inc = el[3], raan = el[4], argp = el[5], M0 = el[6];
    double n = sqrt(1.0 / (a * a * a));
    double E = orc_solve_kepler_E(M0 + n * (t - epoch), e);
    double xp = a * (cos(E) - e);
    double yp = a * sqrt(1.0 - e * e) * sin(E);
    double cO = cos(raan), sO = sin(raan), cw = cos(argp), sw = sin(argp);
    double ci = cos(inc), si = sin(inc);
    /* perifocal unit vectors P (towards pericentre) and Q */
    double P[3] = { cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si };
    double Q[3] = { -cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si };
    for (int k = 0; k < 3; ++k) r[k] = xp * P[k] + yp * Q[k];
}

/* Position and velocity of the body of orc_ephem: the velocity is the time derivative
 * of the same Keplerian orbit, dE/dt = n / (1 - e cos E). */
void orc_ephem_state(const double* el, double epoch, double t, double r[3], double v[3])
{
    double a = el[1], e = el[2], inc = el[3], raan = el[4], argp = el[5], M0 = el[6];
    double n = sqrt(1.0 / (a * a * a));
    double E = orc_solve_kepler_E(M0 + n * (t - epoch), e);
    double b = a * sqrt(1.0 - e * e);
    double Ed = n / (1.0 - e * cos(E));
    double xp = a * (cos(E) - e), yp = b * sin(E);
    double xd = -a * sin(E) * Ed, yd = b * cos(E) * Ed;
    double cO = cos(raan), sO = sin(raan), cw = cos(argp), sw = sin(argp);
    double ci = cos(inc), si = sin(inc);
    double P[3] = { cO * cw - sO * sw * ci, sO * cw + cO * sw * ci, sw * si };
    double Q[3] = { -cO * sw - sO * cw * ci, -sO * sw + cO * cw * ci, cw * si };
    for (int k = 0; k < 3; ++k) {
        r[k] = xp * P[k] + yp * Q[k];
        v[k] = xd * P[k] + yd * Q[k];
    }
}

/* Two-body propagation (mu = 1) of y0 by dt, through the Lagrange f and g
 * coefficients written in the eccentric-anomaly difference dE.  Elliptic
 * orbits only.  Returns 0 on success, -1 if the orbit is not elliptic or
 * the state is degenerate (the caller then falls back to a cold start). */
int orc_kepler(const double y0[6], double dt, double y[6])
{
    const double* r0 = y0;
    const double* v0 = y0 + 3;
    double r0n = sqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
    double v02 = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    if (!(r0n > 0.0) || !isfinite(r0n) || !isfinite(v02)) return -1;
    double alpha = 2.0 / r0n - v02;       /* = 1/a */
    if (!(alpha > 0.0)) return -1;
    double a = 1.0 / alpha;
    double sqa = sqrt(a);
    double n = sqrt(alpha * alpha * alpha);
    double sig = r0[0] * v0[0] + r0[1] * v0[1] + r0[2] * v0[2]; /* r.v / sqrt(mu) */
    double c1 = 1.0 - r0n / a;            /* e cos E0 */
    double s1 = sig / sqa;                /* e sin E0 */
    double Mdt = n * dt;
    double x = Mdt;
    for (int it = 0; it < 100; ++it) {
        double sx = sin(x), cx = cos(x);
        double F = x - c1 * sx + s1 * (1.0 - cx) - Mdt;
        double Fp = 1.0 - c1 * cx + s1 * sx;
        double dx = F / Fp;
        x -= dx;
        if (fabs(dx) <= 1e-16 * (1.0 + fabs(x))) break;
    }
    double sx = sin(x), cx = cos(x);
    double rn = a + (r0n - a) * cx + sig * sqa * sx;
    double f = 1.0 - (a / r0n) * (1.0 - cx);
    double g = dt - (x - sx) / n;
    double fd = -sqa * sx / (rn * r0n);
    double gd = 1.0 - (a / rn) * (1.0 - cx);
    for (int k = 0; k < 3; ++k) {
        y[k] = f * r0[k] + g * v0[k];
        y[3 + k] = fd * r0[k] + gd * v0[k];
    }
    for (int k = 0; k < 6; ++k)
        if (!isfinite(y[k])) return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Force model                                                               */
/* ------------------------------------------------------------------------ */

/* Acceleration at r given perturber positions rp[p][3] and parameters mup[p]. */
void orc_accel(const double r[3], int n_pert, const double* rp, const double* mup,
               double mu_sun, double acc[3])
{
    double rn2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rn = sqrt(rn2);
    double s = mu_sun / (rn2 * rn);
    for (int k = 0; k < 3; ++k) acc[k] = -s * r[k];
    for (int p = 0; p < n_pert; ++p) {
        const double* q = rp + 3 * p;
        double d[3] = { r[0] - q[0], r[1] - q[1], r[2] - q[2] };
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double dn = sqrt(d2);
        double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        double qn = sqrt(q2);
        double sd = mup[p] / (d2 * dn);     /* direct term */
        double sq = mup[p] / (q2 * qn);     /* indirect term: Sun's acceleration towards p */
        for (int k = 0; k < 3; ++k) acc[k] -= sd * d[k] + sq * q[k];
    }
}

/* Einstein-Infeld-Hoffmann acceleration of a massless body at (r, v) = y, PPN beta =
 * gamma = 1, written for the major bodies b: the Sun (index -1: at the origin, at rest,
 * unaccelerated, parameter mu_sun) and the perturbers at rp[p] with velocities vp[p] and
 * parameters mup[p], each on a Keplerian orbit about the Sun (gravitational parameter 1),
 * so accelerated by -rp/|rp|^3.  With d = r - r_b, rho = |d|, the potential at the body
 * Phi = sum_b mu_b / rho_b and U_b = sum_{k != b} mu_k / |r_b - r_k| at body b:
 *   a = sum_b -mu_b d / rho^3 [1 - (4 Phi + U_b - v^2 - 2 v_b^2 + 4 v.v_b
 *                                   + 3/2 (d.v_b / rho)^2 + 1/2 d.a_b) / c^2]
 *     + sum_b mu_b / (c^2 rho^3) [d.(4 v - 3 v_b)] (v - v_b)
 *     + 7/2 sum_b mu_b a_b / (c^2 rho)
 * plus the Newtonian indirect term -sum_p mu_p rp/|rp|^3 of the heliocentric frame
 * (orc_accel_eih).  orc_accel_eih_bodies evaluates the sums for any nb major bodies with
 * positions rb, velocities vb, accelerations ab, parameters mub and potentials Ub. */
void orc_accel_eih_bodies(const double y[6], int nb, const double* rb, const double* vb, const double* ab,
                          const double* mub, const double* Ub, double inv_c2, double acc[3])
{
    const double* r = y;
    const double* v = y + 3;
    double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double phi = 0.0;
    for (int b = 0; b < nb; ++b) {
        double dx = r[0] - rb[3 * b], dy = r[1] - rb[3 * b + 1], dz = r[2] - rb[3 * b + 2];
        phi += mub[b] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    for (int k = 0; k < 3; ++k) acc[k] = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double* xb = rb + 3 * b;
        const double* wb = vb + 3 * b;
        const double* gb = ab + 3 * b;
        double d[3] = { r[0] - xb[0], r[1] - xb[1], r[2] - xb[2] };
        double rho = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double i3 = 1.0 / (rho * rho * rho);
        double vbv = v[0] * wb[0] + v[1] * wb[1] + v[2] * wb[2];
        double vb2 = wb[0] * wb[0] + wb[1] * wb[1] + wb[2] * wb[2];
        double dvb = (d[0] * wb[0] + d[1] * wb[1] + d[2] * wb[2]) / rho;
        double dab = d[0] * gb[0] + d[1] * gb[1] + d[2] * gb[2];
        double brk = 1.0 - inv_c2 * (4.0 * phi + Ub[b] - v2 - 2.0 * vb2 + 4.0 * vbv + 1.5 * dvb * dvb + 0.5 * dab);
        double dw = d[0] * (4.0 * v[0] - 3.0 * wb[0]) + d[1] * (4.0 * v[1] - 3.0 * wb[1]) +
                    d[2] * (4.0 * v[2] - 3.0 * wb[2]);
        for (int k = 0; k < 3; ++k) {
            acc[k] += -mub[b] * i3 * d[k] * brk;
            acc[k] += inv_c2 * mub[b] * i3 * dw * (v[k] - wb[k]);
            acc[k] += 3.5 * inv_c2 * mub[b] * gb[k] / rho;
        }
    }
}

void orc_accel_eih(const double y[6], int n_pert, const double* rp, const double* vp, const double* mup,
                   double mu_sun, double inv_c2, double acc[3])
{
    /* major-body states: the Sun at rest at the origin, the perturbers on their orbits */
    double rb[3 * 65], vb[3 * 65], ab[3 * 65], mub[65], Ub[65];
    int nb = n_pert + 1;
    for (int k = 0; k < 3; ++k) rb[k] = vb[k] = ab[k] = 0.0;
    mub[0] = mu_sun;
    for (int p = 0; p < n_pert; ++p) {
        const double* q = rp + 3 * p;
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        for (int k = 0; k < 3; ++k) {
            rb[3 * (p + 1) + k] = q[k];
            vb[3 * (p + 1) + k] = vp[3 * p + k];
            ab[3 * (p + 1) + k] = -q[k] / (qn * qn * qn);
        }
        mub[p + 1] = mup[p];
    }
    for (int b = 0; b < nb; ++b) {
        Ub[b] = 0.0;
        for (int k = 0; k < nb; ++k) {
            if (k == b) continue;
            double dx = rb[3 * b] - rb[3 * k], dy = rb[3 * b + 1] - rb[3 * k + 1], dz = rb[3 * b + 2] - rb[3 * k + 2];
            Ub[b] += mub[k] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
    orc_accel_eih_bodies(y, nb, rb, vb, ab, mub, Ub, inv_c2, acc);
    for (int p = 0; p < n_pert; ++p) {   /* indirect term */
        const double* q = rp + 3 * p;
        double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        double sq = mup[p] / (q2 * sqrt(q2));
        for (int k = 0; k < 3; ++k) acc[k] -= sq * q[k];
    }
}

/* orc_accel_eih at time t with the perturber states from their elements. */
void orc_accel_eih_t(const double y[6], double t, double mu_sun, int n_pert, const double* pert,
                     double epoch, double inv_c2, double acc[3])
{
    double rp[3 * 64], vp[3 * 64], mup[64];
    int np = n_pert > 64 ? 64 : n_pert;
    for (int p = 0; p < np; ++p) {
        orc_ephem_state(pert + 7 * p, epoch, t, rp + 3 * p, vp + 3 * p);
        mup[p] = pert[7 * p];
    }
    orc_accel_eih(y, np, rp, vp, mup, mu_sun, inv_c2, acc);
}

/* Jacobian da/dr (3x3, row-major) of the force model at r with perturbers at rp:
 * for every attracting body with parameter mu at offset d = r - r_b,
 *   d/dr [-mu d/|d|^3] = -mu (I/|d|^3 - 3 d d^T/|d|^5);
 * the indirect term does not depend on r. */
void orc_accel_jac(const double r[3], int n_pert, const double* rp, const double* mup, double mu_sun,
                   double J[9])
{
    for (int k = 0; k < 9; ++k) J[k] = 0.0;
    for (int b = -1; b < n_pert; ++b) {
        double d[3], mu;
        if (b < 0) { d[0] = r[0]; d[1] = r[1]; d[2] = r[2]; mu = mu_sun; }
        else {
            for (int k = 0; k < 3; ++k) d[k] = r[k] - rp[3 * b + k];
            mu = mup[b];
        }
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double dn = sqrt(d2);
        double i3 = 1.0 / (d2 * dn), i5 = i3 / d2;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                J[3 * a + c] -= mu * ((a == c ? i3 : 0.0) - 3.0 * d[a] * d[c] * i5);
    }
}

/* da/dr at (r, t) with perturber positions from their elements. */
void orc_accel_jac_t(const double r[3], double t, double mu_sun, int n_pert, const double* pert,
                     double epoch, double J[9])
{
    double rp[3 * 64], mup[64];
    int np = n_pert > 64 ? 64 : n_pert;
    for (int p = 0; p < np; ++p) {
        orc_ephem(pert + 7 * p, epoch, t, rp + 3 * p);
        mup[p] = pert[7 * p];
    }
    orc_accel_jac(r, np, rp, mup, mu_sun, J);
}

/* Acceleration at (r, t) with perturber positions from their elements. */
void orc_accel_t(const double r[3], double t, double mu_sun, int n_pert, const double* pert,
                 double epoch, double acc[3])
{
    double rp[3 * 64], mup[64];
    int np = n_pert > 64 ? 64 : n_pert;
    for (int p = 0; p < np; ++p) {
        orc_ephem(pert + 7 * p, epoch, t, rp + 3 * p);
        mup[p] = pert[7 * p];
    }
    orc_accel(r, np, rp, mup, mu_sun, acc);
}

/* ------------------------------------------------------------------------ */
/* Chebyshev machinery at the N Chebyshev-Gauss-Lobatto nodes                */
/* ------------------------------------------------------------------------ */

/* tau_j = -cos(j pi / (N-1)), eq. chnodes2. */
static double orc_tau(int j, int N)
{
    return -cos(ORC_PI * (double)j / (double)(N - 1));
}

/* T_k(tau_j).  Since tau_j = cos(pi (N-1-j)/(N-1)), T_k(tau_j) =
 * cos(k pi (N-1-j)/(N-1)); the integer angle k (N-1-j) is reduced modulo
 * 2(N-1) and folded into [0, N-1] so the cosine argument lies in [0, pi]. */
static double orc_T(int k, int j, int N)
{
    long m = ((long)k * (long)(N - 1 - j)) % (2L * (N - 1));
    if (m > N - 1) m = 2L * (N - 1) - m;
    return cos(ORC_PI * (double)m / (double)(N - 1));
}

/* Steps (ii)-(v) of one Picard-Chebyshev iteration for one trajectory with
 * `ncomp` state components: given the force matrix g[N][ncomp] (already
 * scaled by w2) and the initial state y0[ncomp], produce y[N][ncomp].
 * `Tkj` is the table T_k(tau_j), [N][N] row-major by k. */
static void orc_picard_update(int N, int ncomp, const double* Tkj, const double* g,
                              const double* y0, double* y, double* cbuf, double* bbuf)
{
    for (int comp = 0; comp < ncomp; ++comp) {
        /* (ii) fit: c_k, k = 0..N-2; c_{N-1} = c_N = 0 (degree N-2 fit) */
        for (int k = 0; k <= N; ++k) cbuf[k] = 0.0;
        for (int k = 0; k <= N - 2; ++k) {
            double s = 0.0;
            for (int j = 0; j < N; ++j) {
                double w = (j == 0 || j == N - 1) ? 0.5 : 1.0;
                s += w * g[j * ncomp + comp] * Tkj[k * N + j];
            }
            cbuf[k] = 2.0 / (double)(N - 1) * s;
        }
        /* (iii) integrate: b_k = (c_{k-1} - c_{k+1}) / (2k), k = 1..N-1 */
        for (int k = 1; k <= N - 1; ++k) bbuf[k] = (cbuf[k - 1] - cbuf[k + 1]) / (2.0 * k);
        /* (iv) constant term from the initial condition: y(tau = -1) = y0 */
        double alt = 0.0;
        for (int k = 1; k <= N - 1; ++k) alt += ((k & 1) ? -1.0 : 1.0) * bbuf[k];
        bbuf[0] = 2.0 * y0[comp] - 2.0 * alt;
        /* (v) evaluate the series at the nodes */
        for (int j = 0; j < N; ++j) {
            double s = 0.5 * bbuf[0];
            for (int k = 1; k <= N - 1; ++k) s += bbuf[k] * Tkj[k * N + j];
            y[j * ncomp + comp] = s;
        }
    }
}

/* Test hook: one Picard update for a single trajectory (steps ii-v).
 * g[N][ncomp] is the w2-scaled force matrix, y0[ncomp] the initial state. */
void orc_picard_step(int N, int ncomp, const double* g, const double* y0, double* y)
{
    double* Tkj = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* cbuf = (double*)malloc(sizeof(double) * (size_t)(N + 2));
    double* bbuf = (double*)malloc(sizeof(double) * (size_t)(N + 2));
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j) Tkj[k * N + j] = orc_T(k, j, N);
    orc_picard_update(N, ncomp, Tkj, g, y0, y, cbuf, bbuf);
    free(Tkj); free(cbuf); free(bbuf);
}

/* Test hook: the CGL nodes. */
void orc_nodes(int N, double* tau)
{
    for (int j = 0; j < N; ++j) tau[j] = orc_tau(j, N);
}

/*
 * Second-order form (the version of the method for x'' = a(x, v, t) that Sec. 1 cites
 * as a further development applicable to the augmented system): velocity and position
 * are both obtained from the acceleration samples, the position by integrating the new
 * velocity series rather than the previous velocity iterate.  For one trajectory, with
 * a[N][3] the unscaled accelerations at the nodes, x0, v0 the initial state and w2 the
 * half-length of the segment (dt = w2 dtau):
 *   (ii)  c_k = 2/(N-1) sum''_j a_j T_k(tau_j), k = 0..N-2      (the fit of step ii)
 *   (iii) velocity series b_k = (c_{k-1} - c_{k+1}) / (2k), k = 1..N-1, and
 *         b_0 = -2 sum_k (-1)^k b_k, so that the series vanishes at tau = -1;
 *         v_j = v0 + w2 (b_0/2 + sum_{k=1}^{N-1} b_k T_k(tau_j))
 *   (iv)  position series d_k = (b_{k-1} - b_{k+1}) / (2k), k = 1..N (b_N = b_{N+1} = 0,
 *         b_0 taken with its half weight, as in the integral of b_0/2 T_0), and
 *         d_0 = -2 sum_k (-1)^k d_k;
 *         x_j = x0 + w2 v0 (tau_j + 1) + w2^2 (d_0/2 + sum_{k=1}^{N} d_k T_k(tau_j))
 * so x is the exact double integral of the degree N-2 fit (degree N), v its single one.
 * Tkj: T_k(tau_j) for k = 0..N, [N+1][N] row-major by k.
 */
static void orc_second_order_update(int N, const double* Tkj, const double* a, const double* x0,
                                    const double* v0, double w2, const double* tau, double* x, double* v,
                                    double* cbuf, double* bbuf, double* dbuf)
{
    for (int comp = 0; comp < 3; ++comp) {
        for (int k = 0; k <= N + 1; ++k) cbuf[k] = bbuf[k] = dbuf[k] = 0.0;
        for (int k = 0; k <= N - 2; ++k) {
            double s = 0.0;
            for (int j = 0; j < N; ++j) {
                double w = (j == 0 || j == N - 1) ? 0.5 : 1.0;
                s += w * a[3 * j + comp] * Tkj[k * N + j];
            }
            cbuf[k] = 2.0 / (double)(N - 1) * s;
        }
        for (int k = 1; k <= N - 1; ++k) bbuf[k] = (cbuf[k - 1] - cbuf[k + 1]) / (2.0 * k);
        double alt = 0.0;
        for (int k = 1; k <= N - 1; ++k) alt += ((k & 1) ? -1.0 : 1.0) * bbuf[k];
        bbuf[0] = -2.0 * alt;
        for (int k = 1; k <= N; ++k) dbuf[k] = (bbuf[k - 1] - bbuf[k + 1]) / (2.0 * k);
        alt = 0.0;
        for (int k = 1; k <= N; ++k) alt += ((k & 1) ? -1.0 : 1.0) * dbuf[k];
        dbuf[0] = -2.0 * alt;
        for (int j = 0; j < N; ++j) {
            double sv = 0.5 * bbuf[0], sx = 0.5 * dbuf[0];
            for (int k = 1; k <= N - 1; ++k) sv += bbuf[k] * Tkj[k * N + j];
            for (int k = 1; k <= N; ++k) sx += dbuf[k] * Tkj[k * N + j];
            v[3 * j + comp] = v0[comp] + w2 * sv;
            x[3 * j + comp] = x0[comp] + w2 * v0[comp] * (tau[j] + 1.0) + w2 * w2 * sx;
        }
    }
}

/* Test hook: one second-order update (steps ii-iv above) for a single trajectory. */
void orc_second_order_step(int N, const double* a, const double* x0, const double* v0, double w2,
                           double* x, double* v)
{
    double* Tkj = (double*)malloc(sizeof(double) * (size_t)(N + 1) * N);
    double* tau = (double*)malloc(sizeof(double) * (size_t)N);
    double* cbuf = (double*)malloc(sizeof(double) * (size_t)(N + 2));
    double* bbuf = (double*)malloc(sizeof(double) * (size_t)(N + 2));
    double* dbuf = (double*)malloc(sizeof(double) * (size_t)(N + 2));
    for (int k = 0; k <= N; ++k)
        for (int j = 0; j < N; ++j) Tkj[k * N + j] = orc_T(k, j, N);
    for (int j = 0; j < N; ++j) tau[j] = orc_tau(j, N);
    orc_second_order_update(N, Tkj, a, x0, v0, w2, tau, x, v, cbuf, bbuf, dbuf);
    free(Tkj); free(tau); free(cbuf); free(bbuf); free(dbuf);
}

/* ------------------------------------------------------------------------ */
/* Whole propagation                                                         */
/* ------------------------------------------------------------------------ */

/* Status codes per IC and segment, as stored in iters_out:
 *   k >= 1 : converged after k iterations
 *   -1     : not converged within max_iter (the last iterate is kept)
 *   -2     : non-finite state (the IC stops; later segments also -2)      */

/* Error of step (vi) between two iterates of one trajectory. */
static double orc_iter_error(int N, const double* ynew, const double* yold, int tol_mode)
{
    double e = 0.0;
    for (int j = 0; j < N; ++j) {
        const double* a = ynew + 6 * j;
        const double* b = yold + 6 * j;
        double dr = 0, rr = 0, dv = 0, vv = 0;
        for (int k = 0; k < 3; ++k) {
            dr += (a[k] - b[k]) * (a[k] - b[k]);
            rr += a[k] * a[k];
            dv += (a[3 + k] - b[3 + k]) * (a[3 + k] - b[3 + k]);
            vv += a[3 + k] * a[3 + k];
        }
        double ep, ev;
        if (tol_mode == 0) { ep = sqrt(dr) / sqrt(rr); ev = sqrt(dv) / sqrt(vv); }
        else { ep = sqrt(dr); ev = sqrt(dv); }
        if (!(ep <= INFINITY) || !(ev <= INFINITY)) return NAN;
        double m = ep > ev ? ep : ev;
        if (m > e) e = m;
    }
    return e;
}

/*
 * Propagate n_ic trajectories.
 *   ics[n][6]          initial states at t0[n]
 *   t0[n], tf[n]       per-IC interval (tf < t0: backward)
 *   N, S               nodes per segment, number of segments
 *   tol, tol_mode      stopping tolerance; 0 = relative, 1 = absolute
 *   max_iter           iteration cap per segment
 *   fixed_iters        if > 0, every segment runs exactly this many
 *                      iterations and reports that count (no stopping rule)
 *   init               0 = Kepler warm start, 1 = cold start, 2 = the node states in
 *                      guess[n][S][N][6] (a hot start from an earlier propagation, Sec. 2.1;
 *                      a non-finite row starts from the segment's initial state)
 *   mu_sun, n_pert, pert[n_pert][7], epoch : force model
 *   states_out[n][6]   final states
 *   iters_out[n][S]    per-segment iteration counts / status
 *   bounds_out         [n][S+1][6] segment-boundary states, or NULL
 *   nodes_out          [n][S][N][6] converged node states, or NULL
 *   nthreads           OpenMP threads (<= 0: library default)
 *   order              1: the iteration of Sec. 2.2 on the first-order system (steps
 *                      i-vi above); 2: the second-order form (orc_second_order_update),
 *                      the same stopping rule (vi) on the position and velocity iterates
 *   feedback           order 2 only, 1 = integral error feedback, read here as: the
 *                      sweep's accelerations were taken at the previous position iterate,
 *                      so the change dx_j that the sweep makes to the position is fed back
 *                      through the linear part of the dynamics, da_j = (da/dr)_j dx_j (the
 *                      point-mass gravity gradient at the previous iterate), and the
 *                      integrals of da (orc_second_order_update with zero initial state)
 *                      are added to the new velocity and position.  At the fixed point dx
 *                      vanishes, so the converged result is that of order 2 without it.
 * Returns the number of threads used.
 */
/* What every segment solve of one orc_propagate call shares: the settings, the node
 * grid and T_k(tau_j), and the force model. */
typedef struct {
    int N, tol_mode, max_iter, fixed_iters, init, order, feedback, np;
    double tol, mu_sun, epoch, inv_c2;
    const double* pert;
    const double* Tkj;
    const double* tau;
    const double* mup;
} OrcRun;

/* Per-thread buffers of the segment solve. */
typedef struct {
    double *Y, *Yn, *G, *rp, *vp, *cbuf, *bbuf, *dbuf, *A2, *X2, *V2, *dX2, *dV2;
} OrcWork;

/*
 * One segment [Ts, Te] of one trajectory from the initial state y0 (Sec. 2.2): perturber
 * states at the nodes, the initial guess (Sec. 2.1; seg_guess [N][6] for a hot start, else
 * NULL), then Picard iterations (steps i-vi) until the error (vi) is below tol.  The
 * newest iterate is left in W->Y.  Returns the status of the segment: k >= 1 converged
 * after k iterations, -1 not converged within max_iter, -2 non-finite.
 */
static int orc_segment(const OrcRun* R, OrcWork* W, const double y0[6], double Ts, double Te,
                       const double* seg_guess)
{
    const int N = R->N, np = R->np;
    const double* tau = R->tau;
    const double w1 = 0.5 * (Te + Ts), w2 = 0.5 * (Te - Ts);
    /* perturber positions (and velocities, for EIH) at the nodes, before iterating
       (Sec. 5.4.1) */
    for (int j = 0; j < N; ++j) {
        double tj = w2 * tau[j] + w1;
        for (int p = 0; p < np; ++p) {
            if (R->inv_c2 != 0.0)
                orc_ephem_state(R->pert + 7 * p, R->epoch, tj, W->rp + 3 * (j * np + p), W->vp + 3 * (j * np + p));
            else
                orc_ephem(R->pert + 7 * p, R->epoch, tj, W->rp + 3 * (j * np + p));
        }
    }
    /* initial guess */
    int cold = (R->init == 1);
    if (seg_guess) {
        for (int j = 0; j < N; ++j) {
            const double* gq = seg_guess + 6 * j;
            int fin = 1;
            for (int k = 0; k < 6; ++k) fin = fin && isfinite(gq[k]);
            memcpy(W->Y + 6 * j, fin ? gq : y0, sizeof(double) * 6);
        }
    } else if (!cold) {
        for (int j = 0; j < N; ++j) {
            double dt = w2 * (tau[j] + 1.0);
            if (orc_kepler(y0, dt, W->Y + 6 * j) != 0) { cold = 1; break; }
        }
    }
    if (cold)
        for (int j = 0; j < N; ++j) memcpy(W->Y + 6 * j, y0, sizeof(double) * 6);
    /* Picard iterations */
    int status = -1;
    int n_it = R->fixed_iters > 0 ? R->fixed_iters : R->max_iter;
    for (int it = 1; it <= n_it; ++it) {
        double *Y = W->Y, *Yn = W->Yn;
        /* (i) force matrix */
        for (int j = 0; j < N; ++j) {
            double acc[3];
            if (R->inv_c2 != 0.0)
                orc_accel_eih(Y + 6 * j, np, W->rp + 3 * j * np, W->vp + 3 * j * np, R->mup, R->mu_sun, R->inv_c2, acc);
            else
                orc_accel(Y + 6 * j, np, W->rp + 3 * j * np, R->mup, R->mu_sun, acc);
            for (int k = 0; k < 3; ++k) {
                W->G[6 * j + k] = w2 * Y[6 * j + 3 + k];
                W->G[6 * j + 3 + k] = w2 * acc[k];
                W->A2[3 * j + k] = acc[k];
            }
        }
        if (R->order == 2) {
            /* second-order form: velocity and position from the accelerations */
            orc_second_order_update(N, R->Tkj, W->A2, y0, y0 + 3, w2, tau, W->X2, W->V2, W->cbuf, W->bbuf, W->dbuf);
            if (R->feedback) {
                const double zero[3] = {0.0, 0.0, 0.0};
                for (int j = 0; j < N; ++j) {
                    double J[9], dx[3];
                    orc_accel_jac(Y + 6 * j, np, W->rp + 3 * j * np, R->mup, R->mu_sun, J);
                    for (int k = 0; k < 3; ++k) dx[k] = W->X2[3 * j + k] - Y[6 * j + k];
                    for (int k = 0; k < 3; ++k)
                        W->A2[3 * j + k] = J[3 * k] * dx[0] + J[3 * k + 1] * dx[1] + J[3 * k + 2] * dx[2];
                }
                orc_second_order_update(N, R->Tkj, W->A2, zero, zero, w2, tau, W->dX2, W->dV2, W->cbuf, W->bbuf,
                                        W->dbuf);
                for (int i = 0; i < 3 * N; ++i) {
                    W->X2[i] += W->dX2[i];
                    W->V2[i] += W->dV2[i];
                }
            }
            for (int j = 0; j < N; ++j)
                for (int k = 0; k < 3; ++k) {
                    Yn[6 * j + k] = W->X2[3 * j + k];
                    Yn[6 * j + 3 + k] = W->V2[3 * j + k];
                }
        } else {
            /* (ii)-(v) */
            orc_picard_update(N, 6, R->Tkj, W->G, y0, Yn, W->cbuf, W->bbuf);
        }
        /* (vi) */
        double e = orc_iter_error(N, Yn, Y, R->tol_mode);
        W->Y = Yn;   /* the newest iterate */
        W->Yn = Y;
        if (isnan(e)) { status = -2; break; }
        if (R->fixed_iters > 0) { if (it == n_it) status = it; continue; }
        if (e < R->tol) { status = it; break; }
    }
    return status;
}

/*
 * Propagate n_ic trajectories.
 *   ics[n][6]          initial states at t0[n]
 *   t0[n], tf[n]       per-IC interval (tf < t0: backward)
 *   N, S               nodes per segment, number of segments
 *   tol, tol_mode      stopping tolerance; 0 = relative, 1 = absolute
 *   max_iter           iteration cap per segment
 *   fixed_iters        if > 0, every segment runs exactly this many
 *                      iterations and reports that count (no stopping rule)
 *   init               0 = Kepler warm start, 1 = cold start, 2 = the node states in
 *                      guess[n][S][N][6] (a hot start from an earlier propagation, Sec. 2.1;
 *                      a non-finite row starts from the segment's initial state)
 *   mu_sun, n_pert, pert[n_pert][7], epoch : force model
 *   states_out[n][6]   final states
 *   iters_out[n][S]    per-segment iteration counts / status
 *   bounds_out         [n][S+1][6] segment-boundary states, or NULL
 *   nodes_out          [n][S][N][6] converged node states, or NULL
 *   nthreads           OpenMP threads (<= 0: library default)
 *   order              1: the iteration of Sec. 2.2 on the first-order system (steps
 *                      i-vi above); 2: the second-order form (orc_second_order_update),
 *                      the same stopping rule (vi) on the position and velocity iterates
 *   feedback           order 2 only, 1 = integral error feedback, read here as: the
 *                      sweep's accelerations were taken at the previous position iterate,
 *                      so the change dx_j that the sweep makes to the position is fed back
 *                      through the linear part of the dynamics, da_j = (da/dr)_j dx_j (the
 *                      point-mass gravity gradient at the previous iterate), and the
 *                      integrals of da (orc_second_order_update with zero initial state)
 *                      are added to the new velocity and position.  At the fixed point dx
 *                      vanishes, so the converged result is that of order 2 without it.
 *   refine             adaptive segment refinement (0 = off): a segment whose iterations do
 *                      not converge within max_iter is solved again from its initial state
 *                      as 2, then 4, ... up to 2^refine equal sub-segments of the same N,
 *                      each a complete segment solve (own warm start, own iterations),
 *                      chained in order, until every sub-segment converges.  This is the
 *                      piecewise remedy of Sec. 2.2 (shorter pieces where the span is too
 *                      long for the iteration to converge), applied per segment as the
 *                      adaptive variant cited in Sec. 1 sets segment lengths.  The segment
 *                      then records the sum of its sub-segments' iteration counts; if the
 *                      finest split still has a sub-segment at -1, it records -1 and keeps
 *                      that split's end state.  Not with nodes_out or a guess (a split
 *                      segment has no states at the original nodes).
 * Returns the number of threads used.
 */
int orc_propagate(int n_ic, const double* ics, const double* t0, const double* tf,
                  int N, int S, double tol, int tol_mode, int max_iter, int fixed_iters,
                  int init, double mu_sun, int n_pert, const double* pert, double epoch,
                  double inv_c2, double* states_out, int* iters_out, double* bounds_out,
                  double* nodes_out, int nthreads, int order, int feedback, const double* guess,
                  int refine)
{
    int used = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    if (refine > 0 && (nodes_out || guess)) return -1;
    double* Tkj = (double*)malloc(sizeof(double) * (size_t)(N + 1) * N);   /* k = 0..N */
    double* tau = (double*)malloc(sizeof(double) * (size_t)N);
    for (int k = 0; k <= N; ++k)
        for (int j = 0; j < N; ++j) Tkj[k * N + j] = orc_T(k, j, N);
    for (int j = 0; j < N; ++j) tau[j] = orc_tau(j, N);
    double mup[64];
    int np = n_pert > 64 ? 64 : n_pert;
    for (int p = 0; p < np; ++p) mup[p] = pert[7 * p];
    OrcRun R;
    R.N = N; R.tol_mode = tol_mode; R.max_iter = max_iter; R.fixed_iters = fixed_iters;
    R.init = init == 2 ? 0 : init; R.order = order; R.feedback = feedback; R.np = np;
    R.tol = tol; R.mu_sun = mu_sun; R.epoch = epoch; R.inv_c2 = inv_c2;
    R.pert = pert; R.Tkj = Tkj; R.tau = tau; R.mup = mup;

#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        used = omp_get_num_threads();
#endif
        OrcWork W;
        W.Y = (double*)malloc(sizeof(double) * (size_t)N * 6);
        W.Yn = (double*)malloc(sizeof(double) * (size_t)N * 6);
        W.G = (double*)malloc(sizeof(double) * (size_t)N * 6);
        W.rp = (double*)malloc(sizeof(double) * (size_t)N * 3 * (np > 0 ? np : 1));
        W.vp = (double*)malloc(sizeof(double) * (size_t)N * 3 * (np > 0 ? np : 1));
        W.cbuf = (double*)malloc(sizeof(double) * (size_t)(N + 2));
        W.bbuf = (double*)malloc(sizeof(double) * (size_t)(N + 2));
        W.dbuf = (double*)malloc(sizeof(double) * (size_t)(N + 2));
        W.A2 = (double*)malloc(sizeof(double) * (size_t)N * 3);    /* order 2: a at the nodes */
        W.X2 = (double*)malloc(sizeof(double) * (size_t)N * 3);
        W.V2 = (double*)malloc(sizeof(double) * (size_t)N * 3);
        W.dX2 = (double*)malloc(sizeof(double) * (size_t)N * 3);
        W.dV2 = (double*)malloc(sizeof(double) * (size_t)N * 3);
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m < n_ic; ++m) {
            double y0[6];
            memcpy(y0, ics + 6 * m, sizeof(y0));
            int dead = 0;
            for (int k = 0; k < 6; ++k) if (!isfinite(y0[k])) dead = 1;
            if (bounds_out) memcpy(bounds_out + ((size_t)m * (S + 1)) * 6, y0, sizeof(y0));
            for (int s = 0; s < S; ++s) {
                int* it_out = iters_out + (size_t)m * S + s;
                if (dead) {
                    *it_out = -2;
                    for (int k = 0; k < 6; ++k) y0[k] = NAN;
                    if (bounds_out) memcpy(bounds_out + ((size_t)m * (S + 1) + s + 1) * 6, y0, sizeof(y0));
                    if (nodes_out)
                        for (int j = 0; j < N; ++j)
                            memcpy(nodes_out + (((size_t)m * S + s) * N + j) * 6, y0, sizeof(y0));
                    continue;
                }
                double h = (tf[m] - t0[m]) / (double)S;
                double Ts = t0[m] + h * s;
                double Te = t0[m] + h * (s + 1);
                const double* sg = init == 2 ? guess + ((size_t)m * S + s) * N * 6 : NULL;
                int status = orc_segment(&R, &W, y0, Ts, Te, sg);
                double yend[6];
                memcpy(yend, W.Y + 6 * (N - 1), sizeof(yend));
                /* adaptive refinement: 2, 4, ... equal sub-segments from the same y0 */
                for (int d = 1; status == -1 && d <= refine; ++d) {
                    const int parts = 1 << d;
                    const double hq = (Te - Ts) / (double)parts;
                    double yq[6];
                    memcpy(yq, y0, sizeof(yq));
                    int total = 0, st = 0;
                    for (int q = 0; q < parts; ++q) {
                        int sq = orc_segment(&R, &W, yq, Ts + hq * q, Ts + hq * (q + 1), NULL);
                        memcpy(yq, W.Y + 6 * (N - 1), sizeof(yq));
                        if (sq == -2) { st = -2; break; }
                        if (sq == -1) st = -1;
                        else total += sq;
                    }
                    status = st < 0 ? st : total;
                    memcpy(yend, yq, sizeof(yend));
                }
                *it_out = status;
                if (status == -2) dead = 1;
                if (nodes_out)
                    memcpy(nodes_out + (((size_t)m * S + s) * N) * 6, W.Y, sizeof(double) * 6 * N);
                memcpy(y0, yend, sizeof(y0));
                if (dead) for (int k = 0; k < 6; ++k) y0[k] = NAN;
                if (bounds_out) memcpy(bounds_out + ((size_t)m * (S + 1) + s + 1) * 6, y0, sizeof(y0));
            }
            memcpy(states_out + 6 * m, y0, sizeof(y0));
        }
        free(W.Y); free(W.Yn); free(W.G); free(W.rp); free(W.vp); free(W.cbuf); free(W.bbuf);
        free(W.dbuf); free(W.A2); free(W.X2); free(W.V2); free(W.dX2); free(W.dV2);
    }
    free(Tkj); free(tau);
    return used;
}

/*
 * Group-max convergence.  Sec. 3.2 lets the stopping rule act on the whole augmented
 * system or on blocks of it, and the paper's CUDA program (Sec. 5.4.2) stops once the
 * largest error over the whole system is below tol.  Here the n_ic ICs of one group
 * (common t0, tf) take their sweeps in lockstep: in each segment every IC still finite
 * takes sweep after sweep until the largest error (vi) over those ICs is below tol, and
 * every one of them returns that sweep's iterate, so all of them report the same count.
 * An IC whose state turns non-finite leaves the group (status -2, as in orc_propagate)
 * and no longer enters the maximum.  When max_iter sweeps do not bring the maximum below
 * tol, every IC still in the group reports -1 and keeps its last iterate.
 * Arguments as orc_propagate, with one t0 and tf for the group and no fixed-sweep mode.
 * Returns the number of threads used.
 */
int orc_propagate_group(int n_ic, const double* ics, double t0, double tf, int N, int S, double tol,
                        int tol_mode, int max_iter, int init, double mu_sun, int n_pert,
                        const double* pert, double epoch, double* states_out, int* iters_out,
                        double* bounds_out, double* nodes_out, int nthreads)
{
    int used = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#pragma omp single
    used = omp_get_num_threads();
#endif
    const size_t NS = (size_t)N * 6;
    double* Tkj = (double*)malloc(sizeof(double) * (size_t)N * N);
    double* tau = (double*)malloc(sizeof(double) * (size_t)N);
    double* Y = (double*)malloc(sizeof(double) * NS * n_ic);      /* current iterate per IC */
    double* Yn = (double*)malloc(sizeof(double) * NS * n_ic);     /* next iterate per IC */
    double* G = (double*)malloc(sizeof(double) * NS * n_ic);      /* force matrix per IC */
    double* cb = (double*)malloc(sizeof(double) * (size_t)(N + 2) * 2 * n_ic);
    double* y0 = (double*)malloc(sizeof(double) * 6 * (size_t)n_ic);
    double* err = (double*)malloc(sizeof(double) * (size_t)n_ic);
    int* dead = (int*)malloc(sizeof(int) * (size_t)n_ic);
    int np = n_pert > 64 ? 64 : n_pert;
    double* rp = (double*)malloc(sizeof(double) * (size_t)N * 3 * (np > 0 ? np : 1));
    double mup[64];
    for (int p = 0; p < np; ++p) mup[p] = pert[7 * p];
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j) Tkj[k * N + j] = orc_T(k, j, N);
    for (int j = 0; j < N; ++j) tau[j] = orc_tau(j, N);

    for (int m = 0; m < n_ic; ++m) {
        memcpy(y0 + 6 * m, ics + 6 * m, sizeof(double) * 6);
        dead[m] = 0;
        for (int k = 0; k < 6; ++k) if (!isfinite(y0[6 * m + k])) dead[m] = 1;
        if (bounds_out) memcpy(bounds_out + ((size_t)m * (S + 1)) * 6, y0 + 6 * m, sizeof(double) * 6);
    }
    const double h = (tf - t0) / (double)S;
    for (int s = 0; s < S; ++s) {
        const double Ts = t0 + h * s, Te = t0 + h * (s + 1);
        const double w1 = 0.5 * (Te + Ts), w2 = 0.5 * (Te - Ts);
        /* perturber positions at the nodes, before iterating (Sec. 5.4.1) */
        for (int j = 0; j < N; ++j) {
            double tj = w2 * tau[j] + w1;
            for (int p = 0; p < np; ++p) orc_ephem(pert + 7 * p, epoch, tj, rp + 3 * (j * np + p));
        }
        /* initial guess of every IC still in the group, as in orc_propagate */
#pragma omp parallel for schedule(dynamic, 1)
        for (int m = 0; m < n_ic; ++m) {
            if (dead[m]) continue;
            double* Ym = Y + NS * m;
            int cold = (init == 1);
            if (!cold) {
                for (int j = 0; j < N; ++j)
                    if (orc_kepler(y0 + 6 * m, w2 * (tau[j] + 1.0), Ym + 6 * j) != 0) { cold = 1; break; }
            }
            if (cold)
                for (int j = 0; j < N; ++j) memcpy(Ym + 6 * j, y0 + 6 * m, sizeof(double) * 6);
        }
        int status = -1;
        for (int it = 1; it <= max_iter; ++it) {
            /* one sweep (i)-(vi) of every IC still in the group */
#pragma omp parallel for schedule(dynamic, 1)
            for (int m = 0; m < n_ic; ++m) {
                if (dead[m]) continue;
                double* Ym = Y + NS * m;
                double* Ynm = Yn + NS * m;
                double* Gm = G + NS * m;
                for (int j = 0; j < N; ++j) {
                    double acc[3];
                    orc_accel(Ym + 6 * j, np, rp + 3 * j * np, mup, mu_sun, acc);
                    for (int k = 0; k < 3; ++k) {
                        Gm[6 * j + k] = w2 * Ym[6 * j + 3 + k];
                        Gm[6 * j + 3 + k] = w2 * acc[k];
                    }
                }
                orc_picard_update(N, 6, Tkj, Gm, y0 + 6 * m, Ynm, cb + (size_t)(N + 2) * 2 * m,
                                  cb + (size_t)(N + 2) * (2 * m + 1));
                err[m] = orc_iter_error(N, Ynm, Ym, tol_mode);
                memcpy(Ym, Ynm, sizeof(double) * NS);   /* Y is now the newest iterate */
            }
            /* the group's error: the largest over the ICs still in it */
            double emax = 0.0;
            for (int m = 0; m < n_ic; ++m) {
                if (dead[m]) continue;
                if (isnan(err[m])) {
                    dead[m] = 2;   /* left the group in this segment */
                    continue;
                }
                if (err[m] > emax) emax = err[m];
            }
            if (emax < tol) { status = it; break; }
        }
        for (int m = 0; m < n_ic; ++m) {
            int* it_out = iters_out + (size_t)m * S + s;
            double* Ym = Y + NS * m;
            if (dead[m] == 1) {   /* non-finite before this segment */
                *it_out = -2;
                for (int k = 0; k < 6; ++k) y0[6 * m + k] = NAN;
                if (nodes_out)
                    for (int j = 0; j < N; ++j)
                        memcpy(nodes_out + (((size_t)m * S + s) * N + j) * 6, y0 + 6 * m, sizeof(double) * 6);
            } else {
                *it_out = dead[m] == 2 ? -2 : status;
                if (nodes_out) memcpy(nodes_out + (((size_t)m * S + s) * N) * 6, Ym, sizeof(double) * NS);
                memcpy(y0 + 6 * m, Ym + 6 * (N - 1), sizeof(double) * 6);
                if (dead[m] == 2) {
                    dead[m] = 1;
                    for (int k = 0; k < 6; ++k) y0[6 * m + k] = NAN;
                }
            }
            if (bounds_out) memcpy(bounds_out + ((size_t)m * (S + 1) + s + 1) * 6, y0 + 6 * m, sizeof(double) * 6);
        }
    }
    memcpy(states_out, y0, sizeof(double) * 6 * (size_t)n_ic);
    free(Tkj); free(tau); free(Y); free(Yn); free(G); free(cb); free(y0); free(err); free(dead); free(rp);
    return used;
}

/*
 * Flyby detection for the outer level.  Sec. 3.2 proposes isolating a sub-group of
 * trajectories that experience a planetary flyby into its own outer group, since their
 * dynamics differ from the rest; Sec. 7 lists flyby detection as future work.  Reading
 * (a screen before the propagation, on what is known then): the two-body (mu = 1)
 * prediction of each IC from its initial state at t0, the same motion the warm start of
 * Sec. 2.1 uses, is sampled at the `samples` CGL points of each of the S equal segments of
 * [t0, tf] (t = w2 tau_k + w1 per segment, eq. chnodes) and compared with every perturber's
 * ephemeris position at those times; ratio_out[m] is the smallest distance found, in
 * units of that perturber's Hill radius a_p (mu_p / 3)^(1/3).  A massless perturber
 * (mu_p = 0) has no sphere of influence and is skipped (INFINITY when nothing remains);
 * an IC whose orbit is not elliptic gets 0.  An IC is isolated when its ratio is below
 * the caller's threshold.
 */
void orc_flyby_ratio(int n_ic, const double* ics, double t0, double tf, int S, int samples, int n_pert,
                     const double* pert, double epoch, double* ratio_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int m = 0; m < n_ic; ++m) {
        const double* y0 = ics + 6 * m;
        const double h = (tf - t0) / (double)S;
        double best = INFINITY;
        for (int s = 0; s < S && best > 0.0; ++s) {
            const double Ts = t0 + h * s, Te = t0 + h * (s + 1);
            const double w1 = 0.5 * (Te + Ts), w2 = 0.5 * (Te - Ts);
            for (int k = 0; k < samples; ++k) {
                const double t = w2 * orc_tau(k, samples) + w1;
                double y[6];
                if (orc_kepler(y0, t - t0, y) != 0) { best = 0.0; break; }
                for (int p = 0; p < n_pert; ++p) {
                    const double* el = pert + 7 * p;
                    if (!(el[0] > 0.0)) continue;
                    double rp[3];
                    orc_ephem(el, epoch, t, rp);
                    const double dx = y[0] - rp[0], dy = y[1] - rp[1], dz = y[2] - rp[2];
                    const double d = sqrt(dx * dx + dy * dy + dz * dz);
                    const double rh = el[1] * cbrt(el[0] / 3.0);
                    const double q = d / rh;
                    if (q < best) best = q;
                }
            }
        }
        ratio_out[m] = best;
    }
}

/* ------------------------------------------------------------------------ */
/* Independent integrator for pinning: classical fixed-step RK4              */
/* ------------------------------------------------------------------------ */

static void orc_rhs(const double* y, double t, double mu_sun, int n_pert, const double* pert,
                    double epoch, double inv_c2, double* dy)
{
    double acc[3];
    if (inv_c2 != 0.0) orc_accel_eih_t(y, t, mu_sun, n_pert, pert, epoch, inv_c2, acc);
    else orc_accel_t(y, t, mu_sun, n_pert, pert, epoch, acc);
    for (int k = 0; k < 3; ++k) { dy[k] = y[3 + k]; dy[3 + k] = acc[k]; }
}

/* Integrate y' = (v, a(r,v,t)) from t0 to tf with `nsteps` RK4 steps. */
void orc_rk4(const double y0[6], double t0, double tf, long nsteps, double mu_sun, int n_pert,
             const double* pert, double epoch, double inv_c2, double y[6])
{
    double h = (tf - t0) / (double)nsteps;
    double k1[6], k2[6], k3[6], k4[6], tmp[6];
    memcpy(y, y0, sizeof(double) * 6);
    for (long i = 0; i < nsteps; ++i) {
        double t = t0 + h * (double)i;
        orc_rhs(y, t, mu_sun, n_pert, pert, epoch, inv_c2, k1);
        for (int k = 0; k < 6; ++k) tmp[k] = y[k] + 0.5 * h * k1[k];
        orc_rhs(tmp, t + 0.5 * h, mu_sun, n_pert, pert, epoch, inv_c2, k2);
        for (int k = 0; k < 6; ++k) tmp[k] = y[k] + 0.5 * h * k2[k];
        orc_rhs(tmp, t + 0.5 * h, mu_sun, n_pert, pert, epoch, inv_c2, k3);
        for (int k = 0; k < 6; ++k) tmp[k] = y[k] + h * k3[k];
        orc_rhs(tmp, t + h, mu_sun, n_pert, pert, epoch, inv_c2, k4);
        for (int k = 0; k < 6; ++k) y[k] += h / 6.0 * (k1[k] + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
    }
}
