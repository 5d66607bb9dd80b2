// pc_device.h -- device-side building blocks shared by the fused and the plain kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include "pc_internal.h"

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define PC_PI 3.14159265358979323846

// Moves inside a row of 16 lanes through DPP (no LDS round trip, unlike a lane shuffle).
// CTRL: 0xB1 quad_perm [1,0,3,2] (lane ^ 1), 0x4E quad_perm [2,3,0,1] (lane ^ 2),
// 0x128 row_ror:8 (lane ^ 8), 0x141 row_half_mirror (7 - lane in each 8),
// 0x140 row_mirror (15 - lane).  Callers keep the source lanes active.
template <int CTRL>
static __device__ __forceinline__ int pc_dpp(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
static __device__ __forceinline__ float pc_dpp(float v)
{
    return __builtin_bit_cast(float, pc_dpp<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
static __device__ __forceinline__ double pc_dpp(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)pc_dpp<CTRL>((int)(unsigned)b);
    const unsigned hi = (unsigned)pc_dpp<CTRL>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum (OR) over the 16 lanes of a row, the butterfly over lane ^ 1, ^ 2, ^ 4, ^ 8: after
// the two quad steps every quad holds one value, so the mirrored lanes (7 - lane within
// each 8, then 15 - lane) hold what lane ^ 4 and lane ^ 8 hold, and every lane ends with
// the butterfly's result bit for bit.
static __device__ __forceinline__ double pc_row_sum16(double v)
{
    v += pc_dpp<0xB1>(v);
    v += pc_dpp<0x4E>(v);
    v += pc_dpp<0x141>(v);
    v += pc_dpp<0x140>(v);
    return v;
}
static __device__ __forceinline__ int pc_row_or16(int v)
{
    v |= pc_dpp<0xB1>(v);
    v |= pc_dpp<0x4E>(v);
    v |= pc_dpp<0x141>(v);
    v |= pc_dpp<0x140>(v);
    return v;
}

static __device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c)
{
    // D = A(16x4) B(4x16) + C.  Operand lanes: A[l%16][l/16], B[l/16][l%16];
    // result lanes on gfx950: D[l/16 + 4r][l%16] in element r.
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

static __device__ __forceinline__ f32x4 mfma16f(float a, float b, f32x4 c)
{
    // f32 16x16x4: same operand lanes as the f64 form; result D[4(l/16) + r][l%16] in element r
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// max that propagates NaN from either argument
static __device__ __forceinline__ double nmax(double a, double b)
{
    return (a > b || a != a) ? a : b;
}

// ---------------------------------------------------------------------------
// Two-body orbits (gravitational parameter 1)
// ---------------------------------------------------------------------------

// Eccentric anomaly from the mean anomaly (Kepler's equation, Newton's method).
// Returns E modulo 2 pi.
static __device__ double pc_ecc_anomaly(double M, double e)
{
    const double Mr = M - 2.0 * PC_PI * rint(M / (2.0 * PC_PI));
    double E = (e < 0.8) ? Mr : (Mr >= 0.0 ? PC_PI : -PC_PI);
    for (int it = 0; it < 60; ++it) {
        double sE, cE;
        sincos(E, &sE, &cE);
        const double dE = (E - e * sE - Mr) / (1.0 - e * cE);
        E -= dE;
        if (fabs(dE) <= 1e-10 * (1.0 + fabs(E))) break;   // quadratic: the next error is ~dE^2
    }
    return E;
}

static __device__ void pc_body_position(const PcBodyDev& B, double dt_epoch, double r[3])
{
    const double E = pc_ecc_anomaly(B.M0 + B.n * dt_epoch, B.e);
    double sE, cE;
    sincos(E, &sE, &cE);
    const double xp = B.a * (cE - B.e);
    const double yp = B.b * sE;
    for (int k = 0; k < 3; ++k) r[k] = xp * B.P[k] + yp * B.Q[k];
}

// Position and velocity of a body on its Keplerian orbit (gravitational parameter 1):
// the velocity is the time derivative of the position, dE/dt = n / (1 - e cos E).
static __device__ void pc_body_state(const PcBodyDev& B, double dt_epoch, double r[3], double v[3])
{
    const double E = pc_ecc_anomaly(B.M0 + B.n * dt_epoch, B.e);
    double sE, cE;
    sincos(E, &sE, &cE);
    const double Ed = B.n / (1.0 - B.e * cE);
    const double xp = B.a * (cE - B.e), yp = B.b * sE;
    const double xd = -B.a * sE * Ed, yd = B.b * cE * Ed;
    for (int k = 0; k < 3; ++k) {
        r[k] = xp * B.P[k] + yp * B.Q[k];
        v[k] = xd * B.P[k] + yd * B.Q[k];
    }
}

// Warm start (Sec. 2.1): propagate y0 by dt on its osculating ellipse, through the
// Lagrange coefficients f, g, fdot, gdot written in the eccentric-anomaly change x:
//   F(x) = x - (1 - r0/a) sin x + (r0.v0/sqrt(a)) (1 - cos x) - n dt = 0.
// Solved by Halley's iteration x -= 2 F F' / (2 F'^2 - F F''), cubically convergent; F''
// comes from the same sine and cosine as F and F', so a step costs what a Newton step
// does and three steps replace five from the mean-anomaly start.  The error after a step
// is about K e^3, e the error before it (close to the step) and K = O(1) for e < 0.8, so
// a step below 1e-5 leaves an error near 1e-15 and the loop stops there; the
// sine and cosine at the final x follow from those of the last step by its second-order
// Taylor expansion (the dropped cubic term is under 2e-16).  The warm start is only the
// initial guess: the iteration converges to the same fixed point from any nearby one.
// The state goes in and out by value (registers, no stack traffic); a non-elliptic or
// degenerate state returns NaN components.
struct PcState6 {
    double c[6];
};

static __device__ __attribute__((noinline)) PcState6 pc_kepler_state(PcState6 s0, double dt)
{
    const double* y0 = s0.c;
    PcState6 out;
    const double r0n = sqrt(y0[0] * y0[0] + y0[1] * y0[1] + y0[2] * y0[2]);
    const double v02 = y0[3] * y0[3] + y0[4] * y0[4] + y0[5] * y0[5];
    const double alpha = 2.0 / r0n - v02;          // 1/a
    if (!(r0n > 0.0) || !isfinite(r0n) || !isfinite(v02) || !(alpha > 0.0)) {
#pragma unroll
        for (int k = 0; k < 6; ++k) out.c[k] = (double)NAN;
        return out;
    }
    const double a = 1.0 / alpha;
    const double sqa = sqrt(a);
    const double n = alpha * sqrt(alpha);          // mean motion
    const double sig = y0[0] * y0[3] + y0[1] * y0[4] + y0[2] * y0[5];
    const double ec = 1.0 - r0n * alpha;           // e cos E0
    const double es = sig / sqa;                   // e sin E0
    const double ndt = n * dt;
    double x = ndt;
    double sx, cx;
    bool done = false;
    for (int it = 0; it < 60; ++it) {
        sincos(x, &sx, &cx);
        const double F = x - ec * sx + es * (1.0 - cx) - ndt;
        const double F1 = 1.0 - ec * cx + es * sx;
        const double F2 = ec * sx + es * cx;
        const double dx = 2.0 * F * F1 / (2.0 * F1 * F1 - F * F2);
        x -= dx;
        if (fabs(dx) <= 1e-5) {
            // sin and cos of x = x_prev - dx
            const double h2 = 0.5 * dx * dx;
            const double s1 = sx - dx * cx - h2 * sx;
            const double c1 = cx + dx * sx - h2 * cx;
            sx = s1;
            cx = c1;
            done = true;
            break;
        }
    }
    if (!done) sincos(x, &sx, &cx);
    const double rn = a + (r0n - a) * cx + sig * sqa * sx;
    const double f = 1.0 - (a / r0n) * (1.0 - cx);
    const double g = dt - (x - sx) / n;
    const double fd = -sqa * sx / (rn * r0n);
    const double gd = 1.0 - (a / rn) * (1.0 - cx);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        out.c[k] = f * y0[k] + g * y0[3 + k];
        out.c[3 + k] = fd * y0[k] + gd * y0[3 + k];
    }
    return out;
}

// Array form of the warm start; false when the result is not finite (y then unspecified).
static __device__ __forceinline__ bool pc_kepler(const double (&y0)[6], double dt, double (&y)[6])
{
    PcState6 s0;
#pragma unroll
    for (int k = 0; k < 6; ++k) s0.c[k] = y0[k];
    const PcState6 r = pc_kepler_state(s0, dt);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        y[k] = r.c[k];
        ok = ok && isfinite(r.c[k]);
    }
    return ok;
}

// mu / x^(3/2) in full FP64 for finite x > 0, the attraction factor of a point mass at
// squared distance x: from the hardware estimate y of 1/sqrt(x) and e = 1 - x y^2 (x y^2
// with y^2 rounded), x^(-3/2) = (y^2)^(3/2) (1 - e)^(-3/2) = y^3 (1 + 3e/2 + 15e^2/8 + O(e^3)).
// The series coefficients come premultiplied into the mass (mu1 = 3 mu / 2,
// mu2 = 15 mu / 8), so a point-body pair costs six operations after the estimate.  With
// |e| near 2^-22 the dropped terms are below 2^-63 relative.
static __device__ __forceinline__ double pc_mu_r3(double x, double mu, double mu1, double mu2)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double t = y * y;
    const double e = fma(-x, t, 1.0);
    return (y * t) * fma(e, fma(mu2, e, mu1), mu);
}

// ---------------------------------------------------------------------------
// Force model: point masses in the heliocentric frame with the indirect term,
//   a = -mu_S r/|r|^3 - sum_p mu_p (r - r_p)/|r - r_p|^3 - sum_p mu_p r_p/|r_p|^3.
// rec[p] = (r_p, mu_p) for p < P; rec[P] = (precomputed indirect sum, 0).
// ---------------------------------------------------------------------------
static __device__ __forceinline__ void pc_accel(double x, double y, double z, const double4* rec,
                                                int P, double mu_sun, double& ax, double& ay,
                                                double& az)
{
    const double s = pc_mu_r3(x * x + y * y + z * z, mu_sun, 1.5 * mu_sun, 1.875 * mu_sun);
    ax = -s * x;
    ay = -s * y;
    az = -s * z;
    for (int p = 0; p < P; ++p) {
        const double4 q = rec[p];
        const double dx = x - q.x, dy = y - q.y, dz = z - q.z;
        const double sd = pc_mu_r3(dx * dx + dy * dy + dz * dz, q.w, 1.5 * q.w, 1.875 * q.w);
        ax -= sd * dx;
        ay -= sd * dy;
        az -= sd * dz;
    }
    const double4 ind = rec[P];
    ax -= ind.x;
    ay -= ind.y;
    az -= ind.z;
}


// ---------------------------------------------------------------------------
// Shared pieces of the propagation kernels
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(1))) double* gconst_dp;
typedef const __attribute__((address_space(1))) float* gconst_fp;
typedef const __attribute__((address_space(1))) char* gconst_cp;
typedef double pc_d2v __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) pc_d2v* gconst_d2p;

// Base address of per-segment records that is one value per wave (scalar registers): a
// load then adds only the lane's 32-bit byte offset, a global load with a scalar base and
// no per-lane 64-bit address arithmetic.  Callers pass records of one segment of one job,
// the same for every lane of the wave.
static __device__ __forceinline__ gconst_cp pc_wave_base(const void* e)
{
    const uint64_t v = reinterpret_cast<uint64_t>(e);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (gconst_cp)((((uint64_t)hi) << 32) | lo);
}
static __device__ __forceinline__ double4 pc_load_d4(gconst_cp q)
{
    const gconst_d2p p = (gconst_d2p)q;
    const pc_d2v a = p[0], b = p[1];
    return make_double4(a.x, a.y, b.x, b.y);
}
typedef __attribute__((address_space(1))) double* gdp;
typedef __attribute__((address_space(1))) int32_t* gi32p;

// Global-memory views of the buffers the kernel parameters point to.  Pointers read from
// the parameter block are generic, so the compiler emits flat loads and stores for them;
// a flat access counts against the LDS counter too, so the next wait for an LDS read also
// waits for it to reach memory, and it may alias LDS, so loads around LDS stores are
// issued one at a time.  Through these views the accesses are global instructions.
static __device__ __forceinline__ gdp pc_gd(double* q) { return (gdp)q; }
static __device__ __forceinline__ gconst_dp pc_gcd(const double* q) { return (gconst_dp)q; }
static __device__ __forceinline__ gi32p pc_gi(int32_t* q) { return (gi32p)q; }

// Shared-memory arena of one workgroup (sized for the largest job shape).
template <int PAIRS>
struct PcSmem {
    static constexpr int REC = PAIRS >= 2048 ? 7040 : 3072;   // doubles of ephemeris kept in LDS
    double F[6 * PAIRS];          // [node][F comp 6][IC]: velocity (0..2), acceleration (3..5)
    double Rec[REC];              // [node][body 0..P][3]: perturber positions, then the indirect term
    double Y0[6 * (PAIRS / 16)];  // [comp][IC] initial state of the current segment
    double Mu[3 * PC_MAX_PERT_DEV];   // perturber mu, then 3 mu / 2, then 15 mu / 8 (pc_mu_r3)
    int Flag[(PAIRS / 256) * 16]; // per wave, per IC: bit 0 not converged, bit 1 non-finite, bit 2 large change
    int Keep[PAIRS / 256];        // per wave: an iterating IC still changes by more than the FP32 switch
    int Go[PAIRS / 256];          // per wave (or IC group): some IC still iterates after this sweep
    int Active[PAIRS / 16];
    int Dead[PAIRS / 16];
};

// After the stopping rule (taken by threads tid < T on their IC's status word), the waves
// that hold status words note whether some IC still iterates; the barrier that ends the
// sweep makes the notes visible to every wave (one barrier instead of a barrier-reduction).
// The notes are rewritten only after the next sweep's first barrier, when every wave has
// read them.
template <int PAIRS, int NP, class Lane>
static __device__ __forceinline__ void pc_note_active(PcSmem<PAIRS>& sm, const Lane& L)
{
    constexpr int T = PAIRS / NP;
    if (L.wave * 64 < T) {
        const int tid = L.wave * 64 + L.lane;
        const unsigned long long b = __ballot(tid < T && sm.Active[tid]);
        if (L.lane == 0) sm.Go[L.wave] = b != 0ull;
    }
}
template <int PAIRS, int NP>
static __device__ __forceinline__ bool pc_any_active(const PcSmem<PAIRS>& sm)
{
    constexpr int T = PAIRS / NP;
    int a = 0;
#pragma unroll
    for (int w = 0; w < (T + 63) / 64; ++w) a |= sm.Go[w];
    return a != 0;
}

// The same for R points at one node j (the transposed job layout): the bodies go in
// chunks of four whose records are read together, so the wave waits on LDS once per chunk;
// past the last body the indirect-term record (always present) stands in with zero mass.
template <int R>
static __device__ __forceinline__ void pc_force_lds_node(const double (&x)[R], const double (&y)[R],
                                                         const double (&z)[R], int j, int P, double mu_sun,
                                                         const double* srec, const double* smu,
                                                         double (&ax)[R], double (&ay)[R], double (&az)[R])
{
    const double* rec = srec + j * 3 * (P + 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double s = pc_mu_r3(x[r] * x[r] + y[r] * y[r] + z[r] * z[r], mu_sun, 1.5 * mu_sun, 1.875 * mu_sun);
        ax[r] = -s * x[r];
        ay[r] = -s * y[r];
        az[r] = -s * z[r];
    }
    for (int b0 = 0; b0 < P; b0 += 4) {
        double qx[4], qy[4], qz[4], mu[4], mu1[4], mu2[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int b = b0 + k < P ? b0 + k : P;
            const int bm = b0 + k < P ? b0 + k : 0;
            mu[k] = b0 + k < P ? smu[bm] : 0.0;
            mu1[k] = b0 + k < P ? smu[PC_MAX_PERT_DEV + bm] : 0.0;
            mu2[k] = b0 + k < P ? smu[2 * PC_MAX_PERT_DEV + bm] : 0.0;
            qx[k] = rec[3 * b];
            qy[k] = rec[3 * b + 1];
            qz[k] = rec[3 * b + 2];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double dx = x[r] - qx[k], dy = y[r] - qy[k], dz = z[r] - qz[k];
                const double sd = pc_mu_r3(dx * dx + dy * dy + dz * dz, mu[k], mu1[k], mu2[k]);
                ax[r] -= sd * dx;
                ay[r] -= sd * dy;
                az[r] -= sd * dz;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        ax[r] -= rec[3 * P];
        ay[r] -= rec[3 * P + 1];
        az[r] -= rec[3 * P + 2];
    }
}

// Accelerations at R points whose perturber records sit in LDS (compact [node][body][3]).
template <int R>
static __device__ __forceinline__ void pc_force_lds(const double (&x)[R], const double (&y)[R],
                                                    const double (&z)[R], const int (&jr)[R], int P,
                                                    double mu_sun, const double* srec, const double* smu,
                                                    double (&ax)[R], double (&ay)[R], double (&az)[R])
{
    const int stride = 3 * (P + 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double s = pc_mu_r3(x[r] * x[r] + y[r] * y[r] + z[r] * z[r], mu_sun, 1.5 * mu_sun, 1.875 * mu_sun);
        ax[r] = -s * x[r];
        ay[r] = -s * y[r];
        az[r] = -s * z[r];
    }
    for (int b = 0; b < P; ++b) {
        const double mu = smu[b], mu1 = smu[PC_MAX_PERT_DEV + b], mu2 = smu[2 * PC_MAX_PERT_DEV + b];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double* q = srec + jr[r] * stride + 3 * b;
            const double dx = x[r] - q[0], dy = y[r] - q[1], dz = z[r] - q[2];
            const double sd = pc_mu_r3(dx * dx + dy * dy + dz * dz, mu, mu1, mu2);
            ax[r] -= sd * dx;
            ay[r] -= sd * dy;
            az[r] -= sd * dz;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double* q = srec + jr[r] * stride + 3 * P;
        ax[r] -= q[0];
        ay[r] -= q[1];
        az[r] -= q[2];
    }
}

// FP32 variant for the early sweeps of the precision schedule: the differences to the
// perturbers are formed in FP64, everything after them in FP32.
template <int R>
static __device__ __forceinline__ void pc_force_lds32(const double (&x)[R], const double (&y)[R],
                                                      const double (&z)[R], const int (&jr)[R], int P,
                                                      double mu_sun, const double* srec, const double* smu,
                                                      double (&ax)[R], double (&ay)[R], double (&az)[R])
{
    const int stride = 3 * (P + 1);
    float fx[R], fy[R], fz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float xf = (float)x[r], yf = (float)y[r], zf = (float)z[r];
        const float ir = rsqrtf(xf * xf + yf * yf + zf * zf);
        const float s = (float)mu_sun * (ir * ir * ir);
        fx[r] = -s * xf;
        fy[r] = -s * yf;
        fz[r] = -s * zf;
    }
    for (int b = 0; b < P; ++b) {
        const float mu = (float)smu[b];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double* q = srec + jr[r] * stride + 3 * b;
            const float dx = (float)(x[r] - q[0]), dy = (float)(y[r] - q[1]), dz = (float)(z[r] - q[2]);
            const float id = rsqrtf(dx * dx + dy * dy + dz * dz);
            const float sd = mu * (id * id * id);
            fx[r] -= sd * dx;
            fy[r] -= sd * dy;
            fz[r] -= sd * dz;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double* q = srec + jr[r] * stride + 3 * P;
        ax[r] = (double)(fx[r] - (float)q[0]);
        ay[r] = (double)(fy[r] - (float)q[1]);
        az[r] = (double)(fz[r] - (float)q[2]);
    }
}

// Same with the records read from global memory ((x, y, z, mu) per body, then the indirect term).
template <int R>
static __device__ __forceinline__ void pc_force_glb(const double (&x)[R], const double (&y)[R],
                                                    const double (&z)[R], const int (&jr)[R], int P,
                                                    double mu_sun, const double4* grec,
                                                    double (&ax)[R], double (&ay)[R], double (&az)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double s = pc_mu_r3(x[r] * x[r] + y[r] * y[r] + z[r] * z[r], mu_sun, 1.5 * mu_sun, 1.875 * mu_sun);
        ax[r] = -s * x[r];
        ay[r] = -s * y[r];
        az[r] = -s * z[r];
    }
    // each body's records are loaded where they are used: the other wave on the SIMD
    // covers the wait, while holding the next body's records too raises the register
    // pressure of the 256-node bodies into spills (6 % slower with one buffer, 19 % with two)
    const gconst_cp base = pc_wave_base(grec);
    uint32_t vo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) vo[r] = (uint32_t)jr[r] * (uint32_t)(P + 1) * 32u;
    for (int b = 0; b < P; ++b) {
        double4 q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) q[r] = pc_load_d4((base + (size_t)b * 32) + vo[r]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double dx = x[r] - q[r].x, dy = y[r] - q[r].y, dz = z[r] - q[r].z;
            const double sd = pc_mu_r3(dx * dx + dy * dy + dz * dz, q[r].w, 1.5 * q[r].w, 1.875 * q[r].w);
            ax[r] -= sd * dx;
            ay[r] -= sd * dy;
            az[r] -= sd * dz;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double4 q = pc_load_d4((base + (size_t)P * 32) + vo[r]);
        ax[r] -= q.x;
        ay[r] -= q.y;
        az[r] -= q.z;
    }
}

// One attracting body's term of H w at offset d (squared length x): with A = mu/|d|^3 from
// the premultiplied series of pc_mu_r3 and 1/|d|^2 = y^2 (1 + e + e^2) from the same
// estimate y (error of order e^3), h -= A w - 3 A/|d|^2 (d.w) d.
static __device__ __forceinline__ void pc_hess_term(double dx, double dy, double dz, double wx, double wy,
                                                    double wz, double mu, double mu1, double mu2, double& hx,
                                                    double& hy, double& hz)
{
    const double x = dx * dx + dy * dy + dz * dz;
    const double y = __builtin_amdgcn_rsq(x);
    const double t = y * y;
    const double e = fma(-x, t, 1.0);
    const double A = (y * t) * fma(e, fma(mu2, e, mu1), mu);
    const double i2 = fma(t, fma(e, e, e), t);
    const double c = (A * i2) * (3.0 * (dx * wx + dy * wy + dz * wz));
    hx = fma(c, dx, fma(-A, wx, hx));
    hy = fma(c, dy, fma(-A, wy, hy));
    hz = fma(c, dz, fma(-A, wz, hz));
}

// H w for the symmetric force Jacobian H = da/dr at R points: every attracting body with
// parameter mu at offset d contributes -mu (w/|d|^3 - 3 d (d.w)/|d|^5); the indirect term
// does not depend on r.  Records as in pc_force_lds (LDS) or pc_force_glb (global).
template <int R, bool LDSREC>
static __device__ __forceinline__ void pc_hess_apply(const double (&x)[R], const double (&y)[R],
                                                     const double (&z)[R], const double (&wx)[R],
                                                     const double (&wy)[R], const double (&wz)[R],
                                                     const int (&jr)[R], int P, double mu_sun,
                                                     const double* srec, const double* smu, const double4* grec,
                                                     double (&hx)[R], double (&hy)[R], double (&hz)[R])
{
    const double ms1 = 1.5 * mu_sun, ms2 = 1.875 * mu_sun;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        hx[r] = hy[r] = hz[r] = 0.0;
        pc_hess_term(x[r], y[r], z[r], wx[r], wy[r], wz[r], mu_sun, ms1, ms2, hx[r], hy[r], hz[r]);
    }
    const int stride = 3 * (P + 1);
    for (int b = 0; b < P; ++b) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double qx, qy, qz, mu, mu1, mu2;
            if constexpr (LDSREC) {
                const double* q = srec + jr[r] * stride + 3 * b;
                qx = q[0]; qy = q[1]; qz = q[2];
                mu = smu[b];
                mu1 = smu[PC_MAX_PERT_DEV + b];
                mu2 = smu[2 * PC_MAX_PERT_DEV + b];
            } else {
                const double4 q = grec[(size_t)jr[r] * (P + 1) + b];
                qx = q.x; qy = q.y; qz = q.z;
                mu = q.w;
                mu1 = 1.5 * q.w;
                mu2 = 1.875 * q.w;
            }
            pc_hess_term(x[r] - qx, y[r] - qy, z[r] - qz, wx[r], wy[r], wz[r], mu, mu1, mu2, hx[r], hy[r], hz[r]);
        }
    }
}

// Shape of a job: PAIRS = NP x T (node, IC) pairs, NT threads in W waves; every wave owns
// six 16x16 blocks of the iterate.  WIDE (T >= 16): one 16-node strip x the six component
// blocks of one 16-IC group, computed transposed (IC rows, node columns), so that lane l
// holds node l%16 of the strip for ICs l/16 + 4r, r = 0..3 (one node per lane: the force
// reads each perturber record once for its four points).  Otherwise (T == 8): two strips
// x three blocks of two components x 8 ICs, node rows; lane l holds nodes l/16 + 4r and
// components hi, 2+hi, 4+hi of IC l%8 (hi = bit 3 of l).
template <int PAIRS, int NP>
struct PcShape {
    static constexpr int NT = PAIRS / 4;
    static constexpr int W = NT / 64;
    static constexpr int T = PAIRS / NP;
    static constexpr int ROW = 6 * T;      // doubles per node row of F
    static constexpr int NQ = NP / 4;      // k-steps of the 16x16x4 product
    static constexpr bool WIDE = T >= 16;
    static constexpr int G16 = WIDE ? T / 16 : 1;
    static constexpr int H = WIDE ? 1 : 2; // strips per wave
    static_assert(T >= 8 && T <= PAIRS / 16, "unsupported job shape");
};

struct PcLane {
    int lane, wave, strip0, grp, hi;
    int wide;
    int ic_base, ic_step;   // the lane's element r belongs to IC ic_base + ic_step r of the job
    int nq;                 // k steps the products run: the 16-node blocks that hold a node < N
};

// nq: K_N's fragments are zero in every column at or past N, so the products stop after
// the last 16-node block holding a node (4 k steps each; at least two blocks when the
// padded count has them, which the k loop's prologue needs)
template <int PAIRS, int NP>
static __device__ __forceinline__ PcLane pc_lane_geometry(int tid, int N)
{
    using Sh = PcShape<PAIRS, NP>;
    PcLane L;
    L.nq = Sh::NQ > 4 ? min(Sh::NQ, max(8, ((N + 15) >> 4) << 2)) : Sh::NQ;
    L.lane = tid & 63;
    L.wave = tid >> 6;
    L.strip0 = Sh::WIDE ? L.wave / Sh::G16 : 2 * L.wave;
    L.grp = Sh::WIDE ? L.wave - L.strip0 * Sh::G16 : 0;
    L.hi = Sh::WIDE ? 0 : (L.lane >> 3) & 1;
    L.wide = Sh::WIDE;
    L.ic_base = Sh::WIDE ? L.grp * 16 + (L.lane >> 4) : (L.lane & 7);
    L.ic_step = Sh::WIDE ? 4 : 0;
    return L;
}

// node of the lane's element r in strip h (MFMA f64 result layout: D[l/16 + 4r][l%16];
// WIDE blocks are transposed, so their node is the column l%16)
static __device__ __forceinline__ int pc_node(const PcLane& L, int h, int r)
{
    return L.wide ? L.strip0 * 16 + (L.lane & 15) : (L.strip0 + h) * 16 + (L.lane >> 4) + 4 * r;
}

// IC (index within the job) of the lane's element r
static __device__ __forceinline__ int pc_ic(const PcLane& L, int r)
{
    return L.ic_base + L.ic_step * r;
}

// IC whose stopping-rule flag lane l < 16 returns from pc_product: grp * 16 + l (WIDE),
// l % 8 (T == 8)
template <int PAIRS, int NP>
static __device__ __forceinline__ int pc_flag_ic(const PcLane& L)
{
    return PcShape<PAIRS, NP>::WIDE ? L.grp * 16 + (L.lane & 15) : (L.lane & 7);
}

// Column of IC m in node row j of the LDS force array F[node][comp][IC].  WIDE jobs XOR
// the IC's place in its 16-IC group with j % 16: a row is 6T doubles, a multiple of the
// bank count, so without it the 16 lanes of a row group (one node each, same IC) would
// all hit one bank.  Readers of a 16-column group still see a permutation of it.
template <int PAIRS, int NP>
static __device__ __forceinline__ int pc_fcol(int j, int m)
{
    return PcShape<PAIRS, NP>::WIDE ? (m ^ (j & 15)) : m;
}

// Software-pipelined k loop of a 16x16x4 product over nq steps (a multiple of 4, at most
// NQ, at least 8 when NQ is; NQ fixes the layout of the operands).  The A operand of step q
// (a K_N fragment, read from L2) is loaded DK steps ahead into a ring of DK registers, the
// B operands (LDS) one step ahead into two buffers, and the loop body is unrolled DK
// times, so both rings rotate by register renaming.  A register move out of a ring would
// make the wave wait for the load it copies right after issuing it.
// loadB(q, q % 4, buffer) gets the phase as a compile-time constant after unrolling;
// loadA0(u) supplies the first DK A operands (registers kept across calls, or loads).
// SG_DS / SG_MFMA / SG_VMEM > 0 pin the order of one step in the steady-state loop for
// the scheduler: the B reads of the next step, this step's MFMAs, then the A read DK
// steps ahead (left to itself, the scheduler sinks the reads below the MFMAs that free
// their registers, and the wave then waits on each read right after issuing it).
template <int NQ, int NB, class AT, class BT, int SG_DS = 0, int SG_MFMA = 0, int SG_VMEM = 0, class LA0,
          class LA, class LB, class MM>
static __device__ __forceinline__ void pc_kloop(int nq, LA0 loadA0, LA loadA, LB loadB, MM mma)
{
    constexpr int DK = 4;
    static_assert(NQ % DK == 0, "k steps must be a multiple of the A ring depth");
    AT ka[DK];
    BT bb[2][NB];
#pragma unroll
    for (int u = 0; u < DK; ++u) ka[u] = loadA0(u);
    loadB(0, 0, bb[0]);
    auto steps = [&](int q0) {
#pragma unroll
        for (int u = 0; u < DK; ++u) {
            loadB(q0 + u + 1, (u + 1) & 3, bb[(u + 1) & 1]);
            mma(ka[u], bb[u & 1]);
            ka[u] = loadA(q0 + u + DK);
            if constexpr (SG_MFMA > 0) {
                __builtin_amdgcn_sched_group_barrier(0x100, SG_DS, 0);     // DS reads
                __builtin_amdgcn_sched_group_barrier(0x008, SG_MFMA, 0);   // MFMA
                __builtin_amdgcn_sched_group_barrier(0x020, SG_VMEM, 0);   // VMEM reads
            }
        }
    };
    // the first DK steps outside the loop: their products start from the caller's
    // accumulators directly (a zero start becomes the MFMA's inline constant instead of
    // register moves on every sweep)
    if constexpr (NQ > DK) steps(0);
    auto rest = [&](int n) __attribute__((always_inline)) {
#pragma unroll 1
        for (int q0 = DK; q0 < n - DK; q0 += DK) steps(q0);
#pragma unroll
        for (int u = 0; u < DK; ++u) {   // the last DK steps load nothing past the end
            if (u + 1 < DK) loadB(n - DK + u + 1, (u + 1) & 3, bb[(u + 1) & 1]);
            mma(ka[u], bb[u & 1]);
        }
    };
    // a job whose nodes fill every k step keeps the compile-time bound (constant B
    // offsets in the last steps); a shorter one runs to its own bound, one value per wave
    // (a scalar, which keeps the loop and the B addresses off the vector registers)
    if constexpr (NQ > 2 * DK) {
        if (nq < NQ) {
            rest(__builtin_amdgcn_readfirstlane(nq));
            return;
        }
    }
    rest(NQ);
}

struct PcPairD {
    double a0, a1;
};

// The first four FP64 A operands of the lane's strip (and, for 8-IC jobs, of its second
// strip), loaded once per job: every product then starts without waiting on L2.
template <int PAIRS, int NP>
static __device__ __forceinline__ void pc_kpre_load(gconst_dp kp0, double (&kpre)[8])
{
    constexpr int NQ = NP / 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        kpre[u] = kp0[u * 64];
        kpre[4 + u] = PcShape<PAIRS, NP>::WIDE ? 0.0 : kp0[(NQ + u) * 64];
    }
}
struct PcPairF {
    float a0, a1;
};

// Stopping-rule thresholds in fma form, fixed per segment: a squared change d2 passes
// against the squared norm y2 when d2 < a y2 + b, with (a, b) = (tol^2, 0) for the relative
// rule and (0, tol^2) for the absolute one (the same comparisons as d2 < tol^2 y2 and
// d2 < tol^2 for finite norms, with no branch on the mode).  (sa, sb): the same for the
// precision switch.
struct PcTol {
    double ta, tb, sa, sb;
};
static __device__ __forceinline__ PcTol pc_tol(int tol_mode, double t2, double sw2)
{
    return tol_mode == 0 ? PcTol{t2, 0.0, sw2, 0.0} : PcTol{0.0, t2, 0.0, sw2};
}

// Epilogue of a transposed (WIDE) product: acc <- base + w2 acc, where base is y0 (a Picard
// sweep, INCR false) or the previous iterate itself (an increment sweep, INCR true); the
// stopping-rule flags of Sec. 2.2 against the previous iterate yc, OR-ed over the strip's
// nodes, returned by lane i < 16 for local IC i.  SW: evaluate the switch test (bit 2).
template <int PAIRS, int NP, bool INCR, bool SW = true>
static __device__ __forceinline__ int pc_wide_epilogue(const double* sY0, const double (&yc)[6][4],
                                                       f64x4 (&acc)[6], double w2, const PcTol& tl, int N,
                                                       const PcLane& L)
{
    constexpr int T = PcShape<PAIRS, NP>::T;
    const bool node_ok = pc_node(L, 0, 0) < N;
    int fr = 0;   // element r's flags in bits 4r..4r+2
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = pc_ic(L, r);
        double pd = 0.0, py = 0.0, vd = 0.0, vy = 0.0;
#pragma unroll
        for (int b = 0; b < 6; ++b) {
            const double yn = (INCR ? yc[b][r] : sY0[b * T + m]) + w2 * acc[b][r];
            acc[b][r] = yn;
            const double d = yn - yc[b][r];
            if (b < 3) { pd += d * d; py += yn * yn; }
            else { vd += d * d; vy += yn * yn; }
        }
        const bool ok = pd < fma(tl.ta, py, tl.tb) && vd < fma(tl.ta, vy, tl.tb);
        const bool lo = !SW || (pd < fma(tl.sa, py, tl.sb) && vd < fma(tl.sa, vy, tl.sb));
        // the previous iterate is finite, so a non-finite change shows in the new norms
        const bool nf = !isfinite(py + vy);
        fr |= ((ok ? 0 : 1) | (nf ? 2 : 0) | (lo ? 0 : 4)) << (4 * r);
    }
    if (!node_ok) fr = 0;
    // OR over the strip's 16 nodes (the lanes of one row group)
    fr = pc_row_or16(fr);
    // lane i < 16 returns the flag of local IC i = (i & 3) + 4 (i >> 2), held by the lanes
    // of row group i & 3 in element i >> 2
    return (__shfl(fr, 16 * (L.lane & 3)) >> (4 * ((L.lane >> 2) & 3))) & 7;
}

// Epilogue of an 8-IC job's product (node-row layout: element (3h + cb, r) is comp 2cb + hi
// of node pc_node(L, h, r) of IC l % 8): y_new = y0 + w2 acc (INCR: yc + w2 acc), the
// position and velocity
// change norms summed over the lane pair (l, l ^ 8) that shares the IC's components, and
// the stopping-rule flags OR-ed over the lane's nodes and its partner's.  The caller ORs
// the four row groups.
template <int PAIRS, int NP, bool SW, bool INCR = false>
static __device__ __forceinline__ int pc_row_epilogue(const double* sY0, const double (&yc)[6][4],
                                                      f64x4 (&acc)[6], double w2, const PcTol& tl, int N,
                                                      const PcLane& L)
{
    constexpr int T = PcShape<PAIRS, NP>::T;
    const int hi = L.hi;
    const int my_m = pc_ic(L, 0);
    int flag = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, h, r);
            double dd[3], yy[3];
#pragma unroll
            for (int cb = 0; cb < 3; ++cb) {
                const double base = INCR ? yc[3 * h + cb][r] : sY0[(2 * cb + hi) * T + my_m];
                const double yn = base + w2 * acc[3 * h + cb][r];
                acc[3 * h + cb][r] = yn;
                const double d = yn - yc[3 * h + cb][r];
                dd[cb] = d * d;
                yy[cb] = yn * yn;
            }
            double pd = dd[0] + (hi ? 0.0 : dd[1]);
            double py = yy[0] + (hi ? 0.0 : yy[1]);
            double vd = (hi ? dd[1] : 0.0) + dd[2];
            double vy = (hi ? yy[1] : 0.0) + yy[2];
            pd += pc_dpp<0x128>(pd);   // lane ^ 8
            py += pc_dpp<0x128>(py);
            vd += pc_dpp<0x128>(vd);
            vy += pc_dpp<0x128>(vy);
            if (j < N) {
                const bool ok = pd < fma(tl.ta, py, tl.tb) && vd < fma(tl.ta, vy, tl.tb);
                const bool lo = !SW || (pd < fma(tl.sa, py, tl.sb) && vd < fma(tl.sa, vy, tl.sb));
                const bool nf = !isfinite(py + vy);
                flag |= (ok ? 0 : 1) | (nf ? 2 : 0) | (lo ? 0 : 4);
            }
        }
    }
    flag |= pc_dpp<0x128>(flag);
    return flag;
}

// Increment sweep of the precision schedule: Y_new = Y + w2 K_N dF with
// dF, the change of F (pc_publish_chord), held in LDS as FP32 (sD, [node][comp 6][IC]
// with the column swizzle of pc_fcol) and multiplied on the FP32 matrix cores; the sum
// into Y stays FP64.  The FP32 rounding is relative to the increment, so it shrinks as the
// sweeps converge instead of leaving a floor at the FP32 precision of Y.  Returns the
// flags as pc_product.
template <int PAIRS, int NP>
static __device__ __forceinline__ int pc_product_incr(const float* sD, gconst_fp kp0f, const double (&yc)[6][4],
                                                      f64x4 (&acc)[6], double w2, const PcTol& tl, int N,
                                                      const PcLane& L)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ;
    const int lane = L.lane;
    f32x4 accf[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) accf[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (!Sh::WIDE) {
        // 8-IC jobs: the node-row FP32 product of pc_product (K_N rows permuted in kp0f so
        // that the f32 result layout matches the f64 one) on dF, added to the iterate
        gconst_fp kp1f = kp0f + (size_t)NQ * 64;
        const float* bp = sD + (lane >> 4) * ROW + (lane & 15);
        pc_kloop<NQ, 3, PcPairF, float>(L.nq, 
            [&](int q) { return PcPairF{kp0f[q * 64], kp1f[q * 64]}; },
            [&](int q) { return PcPairF{kp0f[q * 64], kp1f[q * 64]}; },
            [&](int q, int, float (&bq)[3]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) bq[c] = bp[q * 4 * ROW + 16 * c];
            },
            [&](const PcPairF& ka, const float (&bq)[3]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) accf[c] = mfma16f(ka.a0, bq[c], accf[c]);
#pragma unroll
                for (int c = 0; c < 3; ++c) accf[3 + c] = mfma16f(ka.a1, bq[c], accf[3 + c]);
            });
#pragma unroll
        for (int b = 0; b < 6; ++b) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[b][r] = (double)accf[b][r];
        }
        int flag = pc_row_epilogue<PAIRS, NP, true, true>(nullptr, yc, acc, w2, tl, N, L);
        flag |= __shfl_xor(flag, 16);
        flag |= __shfl_xor(flag, 32);
        return flag;
    }
    // IC rows read in the order perm(i) = i/4 + 4 (i%4), so the f32 result layout puts IC
    // l/16 + 4r in element r as the f64 one does
    const int i = lane & 15, pi = (i >> 2) + 4 * (i & 3);
    const float* bp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        bp[u] = sD + (lane >> 4) * ROW + L.grp * 16 + (pi ^ ((4 * u + (lane >> 4)) & 15));
    pc_kloop<NQ, 6, float, float, 3, 6, 1>(L.nq, 
        [&](int q) { return kp0f[q * 64]; }, [&](int q) { return kp0f[q * 64]; },
        [&](int q, int u, float (&bq)[6]) {
#pragma unroll
            for (int b = 0; b < 6; ++b) bq[b] = bp[u][q * 4 * ROW + b * T];
        },
        [&](float ka, const float (&bq)[6]) {
#pragma unroll
            for (int b = 0; b < 6; ++b) accf[b] = mfma16f(bq[b], ka, accf[b]);
        });
#pragma unroll
    for (int b = 0; b < 6; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[b][r] = (double)accf[b][r];
    }
    return pc_wide_epilogue<PAIRS, NP, true>(nullptr, yc, acc, w2, tl, N, L);
}

// y_new = y0 + w2 K_N F on the matrix cores (Sec. 2.2 with A, C and S folded into K_N) for
// the lane's six blocks, FP64 or (FP32) FP32 products accumulated into FP64; acc receives
// y_new.  Also evaluates the stopping rule of Sec. 2.2 against the previous iterate yc in
// squared form (|dr|^2 < tol^2 |r|^2 and the same for v, or without the norms in absolute
// mode) and returns in lanes 0..15 the flags of IC pc_flag_ic, OR-ed over its nodes:
// bit 0 = some node not converged, bit 1 = non-finite, bit 2 = some node changed by more
// than sqrt(sw2) (relative).  WIDE blocks are computed as (K_N F)^T = F^T K_N^T: the F
// slice is the A operand and the K_N fragment the B operand.  SW: evaluate bit 2.
template <int PAIRS, int NP, bool FP32 = false, bool SW = true>
static __device__ __forceinline__ int pc_product(const double* sF, const double* sY0, gconst_dp kp0,
                                                  const double (&kpre)[8], gconst_fp kp0f,
                                                  const double (&yc)[6][4], f64x4 (&acc)[6],
                                                  double w2, const PcTol& tl, int N,
                                                  const PcLane& L)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ;
    const int lane = L.lane;
#pragma unroll
    for (int b = 0; b < 6; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    int flag = 0;
    if constexpr (FP32) {
        // FP32 sweep: FP32 fragments of K_N (rows permuted so the f32 result layout matches
        // the f64 one), FP32 copies of the B operands, FP64 accumulation into y0 below
        f32x4 accf[6];
#pragma unroll
        for (int b = 0; b < 6; ++b) accf[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (Sh::WIDE) {
            // the f32 result holds A row 4(l/16) + r in element r: reading IC row i from
            // column perm(i) = i/4 + 4 (i%4) puts IC l/16 + 4r there, as in the f64 layout
            const int i = lane & 15, pi = (i >> 2) + 4 * (i & 3);
            const double* bp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                bp[u] = sF + (lane >> 4) * ROW + L.grp * 16 + (pi ^ ((4 * u + (lane >> 4)) & 15));
            pc_kloop<NQ, 6, float, float>(L.nq, 
                [&](int q) { return kp0f[q * 64]; }, [&](int q) { return kp0f[q * 64]; },
                [&](int q, int u, float (&bq)[6]) {
#pragma unroll
                    for (int b = 0; b < 6; ++b) bq[b] = (float)bp[u][q * 4 * ROW + b * T];
                },
                [&](float ka, const float (&bq)[6]) {
#pragma unroll
                    for (int b = 0; b < 6; ++b) accf[b] = mfma16f(bq[b], ka, accf[b]);
                });
        } else {
            gconst_fp kp1f = kp0f + (size_t)NQ * 64;
            const double* bp = sF + (lane >> 4) * ROW + (lane & 15);
            pc_kloop<NQ, 3, PcPairF, float>(L.nq, 
                [&](int q) { return PcPairF{kp0f[q * 64], kp1f[q * 64]}; },
                [&](int q) { return PcPairF{kp0f[q * 64], kp1f[q * 64]}; },
                [&](int q, int, float (&bq)[3]) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) bq[c] = (float)bp[q * 4 * ROW + 16 * c];
                },
                [&](const PcPairF& ka, const float (&bq)[3]) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) accf[c] = mfma16f(ka.a0, bq[c], accf[c]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) accf[3 + c] = mfma16f(ka.a1, bq[c], accf[3 + c]);
                });
        }
#pragma unroll
        for (int b = 0; b < 6; ++b) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[b][r] = (double)accf[b][r];
        }
    }
    if constexpr (Sh::WIDE) {
        // K_N strip streamed from L2 four k-steps ahead; B operands one k-step ahead
        if constexpr (!FP32) {
            // row 4q + l/16 of F: its column for IC l%16 depends on q % 4 through the swizzle
            const double* bp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                bp[u] = sF + (lane >> 4) * ROW + L.grp * 16 + ((lane & 15) ^ ((4 * u + (lane >> 4)) & 15));
            pc_kloop<NQ, 6, double, double, 3, 6, 1>(L.nq, 
                [&](int u) { return kpre[u]; }, [&](int q) { return kp0[q * 64]; },
                [&](int q, int u, double (&bq)[6]) {
#pragma unroll
                    for (int b = 0; b < 6; ++b) bq[b] = bp[u][q * 4 * ROW + b * T];
                },
                [&](double ka, const double (&bq)[6]) {
#pragma unroll
                    for (int b = 0; b < 6; ++b) acc[b] = mfma16(bq[b], ka, acc[b]);
                });
        }
        return pc_wide_epilogue<PAIRS, NP, false, SW>(sY0, yc, acc, w2, tl, N, L);
    } else {
        if constexpr (!FP32) {
            gconst_dp kp1 = kp0 + (size_t)NQ * 64;
            const double* bp = sF + (lane >> 4) * ROW + (lane & 15);
            pc_kloop<NQ, 3, PcPairD, double>(L.nq, 
                [&](int u) { return PcPairD{kpre[u], kpre[4 + u]}; },
                [&](int q) { return PcPairD{kp0[q * 64], kp1[q * 64]}; },
                [&](int q, int, double (&bq)[3]) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) bq[c] = bp[q * 4 * ROW + 16 * c];
                },
                [&](const PcPairD& ka, const double (&bq)[3]) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[c] = mfma16(ka.a0, bq[c], acc[c]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[3 + c] = mfma16(ka.a1, bq[c], acc[3 + c]);
                });
        }
        flag = pc_row_epilogue<PAIRS, NP, SW>(sY0, yc, acc, w2, tl, N, L);
    }
    flag |= __shfl_xor(flag, 16);
    flag |= __shfl_xor(flag, 32);
    return flag;
}

struct PcQuadD {
    double k0, k1, q0, q1;   // K_N and K2_N fragments of the wave's two strips
};

// Second-order sweep: the velocity and the position both come from the acceleration
// columns of F (comps 3..5), v_new = v0 + w2 K_N a and
// x_new = x0 + w2 v0 (tau_j + 1) + w2^2 K2_N a, with K2_N the double-integration operator
// (the degree N-2 fit integrated twice, zero value and slope at tau = -1).
// WIDE shapes: per k step a lane loads the two operators' fragments (kp1: K_N, kp2: K2_N)
// and three F values, and issues six MFMAs, as the first-order product does.
// 8-IC jobs (node-row layout, a column block holding comps 2cb and 2cb + 1 of the 8 ICs):
// block 0 (x, y) is K2_N times (a_x, a_y) and block 2 (v_y, v_z) K_N times (a_y, a_z), but
// block 1 (z, v_x) needs K2_N for its low half and K_N for its high half, so it takes two
// MFMAs whose B operands are zero in the other half (read from F's velocity columns, which
// second-order sweeps keep at zero): four MFMAs per strip and k step against three.
// tp = tau_j + 1 of the lane's nodes (WIDE: tp[0]; 8-IC jobs: tp[4h + r]).  Flags as
// pc_product.
template <int PAIRS, int NP>
static __device__ __forceinline__ int pc_product2(const double* sF, const double* sY0, gconst_dp kp1,
                                                   gconst_dp kp2, const double (&kpre)[8],
                                                   const double (&yc)[6][4], f64x4 (&acc)[6], double w2,
                                                   const double (&tp)[8], const PcTol& tl, int N, const PcLane& L)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ;
    const int lane = L.lane;
#pragma unroll
    for (int b = 0; b < 6; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    if constexpr (!Sh::WIDE) {
        const int hi = L.hi, m = lane & 7;
        // per-lane F columns of the four B operands (comp * T + IC; comp 0 is zero)
        const double* row = sF + (lane >> 4) * ROW;
        const double* b0 = row + (hi ? 4 : 3) * T + m;   // a_x | a_y
        const double* b1 = row + (hi ? 0 : 5) * T + m;   // a_z | 0
        const double* b2 = row + (hi ? 3 : 0) * T + m;   // 0   | a_x
        const double* b3 = row + (hi ? 5 : 4) * T + m;   // a_y | a_z
        gconst_dp kp1b = kp1 + (size_t)NQ * 64, kp2b = kp2 + (size_t)NQ * 64;
        pc_kloop<NQ, 4, PcQuadD, double>(L.nq, 
            [&](int q) { return PcQuadD{kp1[q * 64], kp1b[q * 64], kp2[q * 64], kp2b[q * 64]}; },
            [&](int q) { return PcQuadD{kp1[q * 64], kp1b[q * 64], kp2[q * 64], kp2b[q * 64]}; },
            [&](int q, int, double (&bq)[4]) {
                const int o = q * 4 * ROW;
                bq[0] = b0[o];
                bq[1] = b1[o];
                bq[2] = b2[o];
                bq[3] = b3[o];
            },
            [&](const PcQuadD& ka, const double (&bq)[4]) {
                // the two MFMAs into block 1 of a strip are five MFMAs apart
                acc[0] = mfma16(ka.q0, bq[0], acc[0]);
                acc[1] = mfma16(ka.q0, bq[1], acc[1]);
                acc[2] = mfma16(ka.k0, bq[3], acc[2]);
                acc[3] = mfma16(ka.q1, bq[0], acc[3]);
                acc[4] = mfma16(ka.q1, bq[1], acc[4]);
                acc[5] = mfma16(ka.k1, bq[3], acc[5]);
                acc[1] = mfma16(ka.k0, bq[2], acc[1]);
                acc[4] = mfma16(ka.k1, bq[2], acc[4]);
            });
        // position elements (block 0, and block 1 in the low lane): w2 acc + v0 (tau + 1),
        // so the common epilogue's y0 + w2 acc gives x0 + w2 v0 (tau + 1) + w2^2 K2_N a
        const double v0a = sY0[(3 + hi) * T + m], v0z = sY0[5 * T + m];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double t = tp[4 * h + r];
                acc[3 * h][r] = fma(w2, acc[3 * h][r], t * v0a);
                acc[3 * h + 1][r] = hi ? acc[3 * h + 1][r] : fma(w2, acc[3 * h + 1][r], t * v0z);
            }
        }
        int flag = pc_row_epilogue<PAIRS, NP, false>(sY0, yc, acc, w2, tl, N, L);
        flag |= __shfl_xor(flag, 16);
        flag |= __shfl_xor(flag, 32);
        return flag;
    } else {
        const double tp1 = tp[0];
        const double* bp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            bp[u] = sF + (lane >> 4) * ROW + L.grp * 16 + ((lane & 15) ^ ((4 * u + (lane >> 4)) & 15));
        pc_kloop<NQ, 3, PcPairD, double, 3, 6, 2>(L.nq, 
            [&](int u) { return PcPairD{kpre[u], kpre[4 + u]}; },
            [&](int q) { return PcPairD{kp1[q * 64], kp2[q * 64]}; },
            [&](int q, int u, double (&bq)[3]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) bq[c] = bp[u][q * 4 * ROW + (3 + c) * T];
            },
            [&](const PcPairD& ka, const double (&bq)[3]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] = mfma16(bq[c], ka.a1, acc[c]);
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[3 + c] = mfma16(bq[c], ka.a0, acc[3 + c]);
            });
        // position: x0 + w2 v0 (tau + 1) + w2^2 acc; the common epilogue adds w2 * acc to
        // its base, so the position blocks become w2 acc + v0 (tau + 1) first
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = pc_ic(L, r);
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c][r] = fma(w2, acc[c][r], tp1 * sY0[(3 + c) * T + m]);
        }
        return pc_wide_epilogue<PAIRS, NP, false, false>(sY0, yc, acc, w2, tl, N, L);
    }
}

// Linear change of the point-mass acceleration over a position change, at R points of
// node j: g = (da/dr)(r) dr = sum over the Sun (at the origin) and the perturbers of
// mu (3 d (d . dr) / |d|^5 - dr / |d|^3), d the point's offset from the mass (the indirect
// term does not depend on the position).  mu/|d|^3 as pc_mu_r3, and 1/|d|^2 from the same
// estimate t of 1/|d|^2 as t (1 + e + e^2), e = 1 - |d|^2 t.  Records in LDS (compact
// [node][body][3], masses in smu) or, when they do not fit there, double4 (x, y, z, mu)
// in global memory.
template <int R, bool ONE_NODE = true>
static __device__ __forceinline__ void pc_grad_dot_node(const double (&x)[R], const double (&y)[R],
                                                        const double (&z)[R], const double (&dx)[R],
                                                        const double (&dy)[R], const double (&dz)[R],
                                                        const int (&jr)[R], int P, double mu_sun, bool rec_lds,
                                                        const double* srec, const double* smu, const double4* grec,
                                                        double (&gx)[R], double (&gy)[R], double (&gz)[R])
{
    auto add = [&](int r, double ox, double oy, double oz, double mu) {
        const double qx = x[r] - ox, qy = y[r] - oy, qz = z[r] - oz;
        const double q2 = qx * qx + qy * qy + qz * qz;
        const double yv = __builtin_amdgcn_rsq(q2);
        const double t = yv * yv;
        const double e = fma(-q2, t, 1.0);
        const double inv2 = fma(t, fma(e, e, e), t);
        const double sd = mu * (yv * t) * fma(e, fma(1.875, e, 1.5), 1.0);
        const double k = 3.0 * sd * inv2 * (qx * dx[r] + qy * dy[r] + qz * dz[r]);
        gx[r] += fma(k, qx, -sd * dx[r]);
        gy[r] += fma(k, qy, -sd * dy[r]);
        gz[r] += fma(k, qz, -sd * dz[r]);
    };
#pragma unroll
    for (int r = 0; r < R; ++r) {
        gx[r] = gy[r] = gz[r] = 0.0;
        add(r, 0.0, 0.0, 0.0, mu_sun);
    }
    // body b's record at node j (ONE_NODE: every point at node jr[0], one read for all)
    auto rec = [&](int j, int b, double& ox, double& oy, double& oz, double& mu) {
        if (rec_lds) {
            const double* q = srec + j * 3 * (P + 1) + 3 * b;
            ox = q[0];
            oy = q[1];
            oz = q[2];
            mu = smu[b];
        } else {
            const double4 q = grec[(size_t)j * (P + 1) + b];
            ox = q.x;
            oy = q.y;
            oz = q.z;
            mu = q.w;
        }
    };
    for (int b = 0; b < P; ++b) {
        if constexpr (ONE_NODE) {
            double ox, oy, oz, mu;
            rec(jr[0], b, ox, oy, oz, mu);
#pragma unroll
            for (int r = 0; r < R; ++r) add(r, ox, oy, oz, mu);
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double ox, oy, oz, mu;
                rec(jr[r], b, ox, oy, oz, mu);
                add(r, ox, oy, oz, mu);
            }
        }
    }
}

// Second-order sweep with integral error feedback.  The sweep's accelerations
// were taken at the previous position iterate; the position it predicts,
// x = x0 + w2 v0 (tau_j + 1) + w2^2 K2_N a, changes that iterate by dx, and the linear change
// of the acceleration over dx, da = (da/dr) dx at the previous iterate, is integrated like
// the accelerations and added: v_new = v0 + w2 K_N (a + da), x_new = x0 + w2 v0 (tau_j + 1) +
// w2^2 K2_N (a + da).  da is published in the velocity columns of F, which second-order
// products do not read, and its product accumulates onto the first one (one barrier in
// between).  At the fixed point dx vanishes, so the converged iterate is the second-order
// one.  Flags as pc_product.
// 8-IC jobs (node-row layout, as pc_product2): the velocity columns hold da, so both
// products take the zero halves of their mixed operands by select instead of from those
// columns; each lane forms da at the four points of strip hi, taking the position and
// change components it lacks from its partner (l ^ 8).
template <int PAIRS, int NP>
static __device__ __forceinline__ int pc_product2_fb(double* sF, const double* sY0, gconst_dp kp1, gconst_dp kp2,
                                                      const double (&kpre)[8], const double (&yc)[6][4],
                                                      f64x4 (&acc)[6], double w2, const double (&tp)[8],
                                                      const PcTol& tl, int N, const PcLane& L, int P, double mu_sun,
                                                      bool rec_lds, const double* sRec, const double* sMu,
                                                      const double4* grec)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ;
    const int lane = L.lane;
#pragma unroll
    for (int b = 0; b < 6; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    if constexpr (!Sh::WIDE) {
        const int hi = L.hi, m = lane & 7;
        const double* row = sF + (lane >> 4) * ROW;
        gconst_dp kp1b = kp1 + (size_t)NQ * 64, kp2b = kp2 + (size_t)NQ * 64;
        // K2_N and K_N products of the columns c0 = base, c1, c2 (accelerations: base 3;
        // da: base 0) into the position and velocity blocks, as pc_product2
        auto product = [&](int base) {
            const double* b0 = row + (base + hi) * T + m;       // c0 | c1
            const double* b1 = row + (base + 2) * T + m;        // c2 | 0
            const double* b2 = row + base * T + m;              // 0  | c0
            const double* b3 = row + (base + 1 + hi) * T + m;   // c1 | c2
            pc_kloop<NQ, 4, PcQuadD, double>(L.nq,
                [&](int q) { return PcQuadD{kp1[q * 64], kp1b[q * 64], kp2[q * 64], kp2b[q * 64]}; },
                [&](int q) { return PcQuadD{kp1[q * 64], kp1b[q * 64], kp2[q * 64], kp2b[q * 64]}; },
                [&](int q, int, double (&bq)[4]) {
                    const int o = q * 4 * ROW;
                    const double v1 = b1[o], v2 = b2[o];
                    bq[0] = b0[o];
                    bq[1] = hi ? 0.0 : v1;
                    bq[2] = hi ? v2 : 0.0;
                    bq[3] = b3[o];
                },
                [&](const PcQuadD& ka, const double (&bq)[4]) {
                    acc[0] = mfma16(ka.q0, bq[0], acc[0]);
                    acc[1] = mfma16(ka.q0, bq[1], acc[1]);
                    acc[2] = mfma16(ka.k0, bq[3], acc[2]);
                    acc[3] = mfma16(ka.q1, bq[0], acc[3]);
                    acc[4] = mfma16(ka.q1, bq[1], acc[4]);
                    acc[5] = mfma16(ka.k1, bq[3], acc[5]);
                    acc[1] = mfma16(ka.k0, bq[2], acc[1]);
                    acc[4] = mfma16(ka.k1, bq[2], acc[4]);
                });
        };
        product(3);
        // predicted position and its change from the previous iterate: block 3h holds
        // comp hi of strip h, block 3h + 1 comp 2 in the low lane
        const double x0a = sY0[hi * T + m], x0z = sY0[2 * T + m];
        const double v0a = sY0[(3 + hi) * T + m], v0z = sY0[5 * T + m];
        double xs[4], ys[4], zs[4], ddx[4], ddy[4], ddz[4], gx[4], gy[4], gz[4];
        int jr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double d0[2], d1[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double t = tp[4 * h + r];
                d0[h] = (x0a + w2 * fma(w2, acc[3 * h][r], t * v0a)) - yc[3 * h][r];
                d1[h] = (x0z + w2 * fma(w2, acc[3 * h + 1][r], t * v0z)) - yc[3 * h + 1][r];
            }
            // the lane's points are those of strip hi
            const double s1 = pc_dpp<0x128>(hi ? yc[0][r] : yc[3][r]);   // lo: y(0); hi: x(1)
            const double s2 = pc_dpp<0x128>(yc[4][r]);                   // hi: z(1)
            const double g1 = pc_dpp<0x128>(hi ? d0[0] : d0[1]);         // lo: dy(0); hi: dx(1)
            const double g2 = pc_dpp<0x128>(d1[1]);                      // hi: dz(1)
            xs[r] = hi ? s1 : yc[0][r];
            ys[r] = hi ? yc[3][r] : s1;
            zs[r] = hi ? s2 : yc[1][r];
            ddx[r] = hi ? g1 : d0[0];
            ddy[r] = hi ? d0[1] : g1;
            ddz[r] = hi ? g2 : d1[0];
            const int j = pc_node(L, hi, r);
            jr[r] = j < N ? j : N - 1;
        }
        pc_grad_dot_node<4, false>(xs, ys, zs, ddx, ddy, ddz, jr, P, mu_sun, rec_lds, sRec, sMu, grec, gx, gy,
                                   gz);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, hi, r);
            if (j < N) {
                double* f = sF + j * ROW + m;
                f[0 * T] = gx[r];
                f[1 * T] = gy[r];
                f[2 * T] = gz[r];
            }
        }
        __syncthreads();   // every node's da published
        product(0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double t = tp[4 * h + r];
                acc[3 * h][r] = fma(w2, acc[3 * h][r], t * v0a);
                acc[3 * h + 1][r] = hi ? acc[3 * h + 1][r] : fma(w2, acc[3 * h + 1][r], t * v0z);
            }
        }
        int flag = pc_row_epilogue<PAIRS, NP, false>(sY0, yc, acc, w2, tl, N, L);
        flag |= __shfl_xor(flag, 16);
        flag |= __shfl_xor(flag, 32);
        return flag;
    }
    const double tp1 = tp[0];
    const double* bp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        bp[u] = sF + (lane >> 4) * ROW + L.grp * 16 + ((lane & 15) ^ ((4 * u + (lane >> 4)) & 15));
    auto product = [&](int c0) {
        pc_kloop<NQ, 3, PcPairD, double, 3, 6, 2>(L.nq, 
            [&](int u) { return PcPairD{kpre[u], kpre[4 + u]}; },
            [&](int q) { return PcPairD{kp1[q * 64], kp2[q * 64]}; },
            [&](int q, int u, double (&bq)[3]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) bq[c] = bp[u][q * 4 * ROW + (c0 + c) * T];
            },
            [&](const PcPairD& ka, const double (&bq)[3]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] = mfma16(bq[c], ka.a1, acc[c]);
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[3 + c] = mfma16(bq[c], ka.a0, acc[3 + c]);
            });
    };
    product(3);
    // the predicted position, its change from the previous iterate, and da there
    const int j = pc_node(L, 0, 0);
    double ddx[4], ddy[4], ddz[4], gx[4], gy[4], gz[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = pc_ic(L, r);
        double d[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            d[c] = (sY0[c * T + m] + w2 * fma(w2, acc[c][r], tp1 * sY0[(3 + c) * T + m])) - yc[c][r];
        ddx[r] = d[0];
        ddy[r] = d[1];
        ddz[r] = d[2];
    }
    const int jj = j < N ? j : N - 1;
    const int jr[4] = {jj, jj, jj, jj};
    pc_grad_dot_node<4>(yc[0], yc[1], yc[2], ddx, ddy, ddz, jr, P, mu_sun, rec_lds, sRec, sMu, grec, gx, gy, gz);
    if (j < N) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double* f = sF + j * ROW + pc_fcol<PAIRS, NP>(j, pc_ic(L, r));
            f[0 * T] = gx[r];
            f[1 * T] = gy[r];
            f[2 * T] = gz[r];
        }
    }
    __syncthreads();   // every node's da published
    product(0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = pc_ic(L, r);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c][r] = fma(w2, acc[c][r], tp1 * sY0[(3 + c) * T + m]);
    }
    return pc_wide_epilogue<PAIRS, NP, false, false>(sY0, yc, acc, w2, tl, N, L);
}

// acc = K_N^T mu for the lane's six blocks (WIDE shapes, transposed like pc_product): the
// adjoint product, mu published in sF as [node][comp 6][IC] and kpT the lane's strip of
// K_N^T fragments.
template <int PAIRS, int NP>
static __device__ __forceinline__ void pc_product_adj(const double* sF, gconst_dp kpT, f64x4 (&acc)[6],
                                                      const PcLane& L)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ;
    const int lane = L.lane;
#pragma unroll
    for (int b = 0; b < 6; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    if constexpr (Sh::WIDE) {
        const double* bp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            bp[u] = sF + (lane >> 4) * ROW + L.grp * 16 + ((lane & 15) ^ ((4 * u + (lane >> 4)) & 15));
        pc_kloop<NQ, 6, double, double, 3, 6, 1>(L.nq, 
            [&](int q) { return kpT[q * 64]; }, [&](int q) { return kpT[q * 64]; },
            [&](int q, int u, double (&bq)[6]) {
#pragma unroll
                for (int b = 0; b < 6; ++b) bq[b] = bp[u][q * 4 * ROW + b * T];
            },
            [&](double ka, const double (&bq)[6]) {
#pragma unroll
                for (int b = 0; b < 6; ++b) acc[b] = mfma16(bq[b], ka, acc[b]);
            });
    } else {
        // 8-IC jobs: the forward product's node-row form with the K_N^T strips of the
        // wave's two row blocks; acc[3h + c] is column block c of strip h
        gconst_dp kpT1 = kpT + (size_t)NQ * 64;
        const double* bp = sF + (lane >> 4) * ROW + (lane & 15);
        pc_kloop<NQ, 3, PcPairD, double>(L.nq, 
            [&](int q) { return PcPairD{kpT[q * 64], kpT1[q * 64]}; },
            [&](int q) { return PcPairD{kpT[q * 64], kpT1[q * 64]}; },
            [&](int q, int, double (&bq)[3]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) bq[c] = bp[q * 4 * ROW + 16 * c];
            },
            [&](const PcPairD& ka, const double (&bq)[3]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] = mfma16(ka.a0, bq[c], acc[c]);
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[3 + c] = mfma16(ka.a1, bq[c], acc[3 + c]);
            });
    }
}

// OR of the per-wave flags of IC m (written as Flag[wave][lane] by lanes < 16).
template <int PAIRS, int NP>
static __device__ __forceinline__ int pc_gather_flags(const int* sFlag, int m)
{
    using Sh = PcShape<PAIRS, NP>;
    int f = 0;
    if constexpr (Sh::WIDE) {
        for (int w = m >> 4; w < Sh::W; w += Sh::G16) f |= sFlag[w * 16 + (m & 15)];
    } else {
        for (int w = 0; w < Sh::W; ++w) f |= sFlag[w * 16 + m];
    }
    return f;
}

// Dynamics of the lane's (node, IC) pairs from its registers, published with the
// velocities as the force matrix F = (v, a) of Sec. 2.2 into sF[node][comp'][IC].
// sRec/sMu: the segment's records in LDS (when rec_lds), grec: the same in global memory.
// VEL = false (second-order sweeps, which read the accelerations only): the velocity
// columns are not written (they stay zero from the segment's start, and the 8-IC
// second-order product reads them as zero B operands).
template <int PAIRS, int NP, bool FP32 = false, bool VEL = true>
static __device__ __forceinline__ void pc_publish(double* sF, const double (&yc)[6][4], const PcLane& L,
                                                  int N, int P, double mu_sun, bool rec_lds,
                                                  const double* sRec, const double* sMu, const double4* grec)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, ROW = Sh::ROW;
    const int hi = L.hi;
    if constexpr (Sh::WIDE) {
        // one node, four ICs: the same record index for every point
        double ax[4], ay[4], az[4];
        const int j = pc_node(L, 0, 0);
        const int jj = j < N ? j : N - 1;
        const int jr[4] = {jj, jj, jj, jj};
        if (rec_lds && FP32) pc_force_lds32<4>(yc[0], yc[1], yc[2], jr, P, mu_sun, sRec, sMu, ax, ay, az);
        else if (rec_lds) pc_force_lds_node<4>(yc[0], yc[1], yc[2], jj, P, mu_sun, sRec, sMu, ax, ay, az);
        else pc_force_glb<4>(yc[0], yc[1], yc[2], jr, P, mu_sun, grec, ax, ay, az);
        if (j < N) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double* f = sF + j * ROW + pc_fcol<PAIRS, NP>(j, pc_ic(L, r));
                if constexpr (VEL) {
                    f[0 * T] = yc[3][r];
                    f[1 * T] = yc[4][r];
                    f[2 * T] = yc[5][r];
                }
                f[3 * T] = ax[r];
                f[4 * T] = ay[r];
                f[5 * T] = az[r];
            }
        }
    } else {
        const int my_m = pc_ic(L, 0);
        // Lane pairs (l, l ^ 8) share the points of one IC: the low lane holds x and z, the
        // high lane y.  Each lane of the pair takes the force of one strip (hd = hi), so
        // both do half the work: the low lane gets y of strip 0 from its partner, the high
        // lane gets x and z of strip 1.
        double xs[4], ys[4], zs[4], ax[4], ay[4], az[4];
        int jr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double s1 = pc_dpp<0x128>(hi ? yc[0][r] : yc[3][r]);   // lane ^ 8
            const double s2 = pc_dpp<0x128>(yc[4][r]);
            xs[r] = hi ? s1 : yc[0][r];
            ys[r] = hi ? yc[3][r] : s1;
            zs[r] = hi ? s2 : yc[1][r];
            const int j = pc_node(L, hi, r);
            jr[r] = j < N ? j : N - 1;
        }
        if (rec_lds && FP32) pc_force_lds32<4>(xs, ys, zs, jr, P, mu_sun, sRec, sMu, ax, ay, az);
        else if (rec_lds) pc_force_lds<4>(xs, ys, zs, jr, P, mu_sun, sRec, sMu, ax, ay, az);
        else pc_force_glb<4>(xs, ys, zs, jr, P, mu_sun, grec, ax, ay, az);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, hi, r);
            if (j < N) {
                double* f = sF + j * ROW + my_m;
                f[3 * T] = ax[r];
                f[4 * T] = ay[r];
                f[5 * T] = az[r];
            }
        }
        if constexpr (VEL) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = pc_node(L, h, r);
                    if (j < N) {
                        double* f = sF + j * ROW + my_m;
                        if (hi) {
                            f[0 * T] = yc[3 * h + 1][r];   // vx (comp 3)
                            f[2 * T] = yc[3 * h + 2][r];   // vz (comp 5)
                        } else {
                            f[1 * T] = yc[3 * h + 2][r];   // vy (comp 4)
                        }
                    }
                }
            }
        }
    }
}

// Gravity gradient da/dr of the force model at R points of node j, in FP32, as the six
// entries (xx, yy, zz, xy, xz, yz) of the symmetric 3x3 matrix: every point mass (the Sun
// at the origin, the perturbers at their record positions) adds mu (3 d d^T / |d|^5 -
// I / |d|^3), d the offset of the point from the mass; the indirect term does not depend
// on the position.  Used as the linear map of the increment sweeps, whose limit moves by
// the error of G times the distance of the anchor from the solution: d is formed in FP64
// and then rounded (near a close approach, rounding the positions first would leave an
// error of 1e-5 in G and of about 1e-12 in the result), the rest is FP32.
template <int R, bool ONE_NODE = true>
static __device__ __forceinline__ void pc_grad_lds_node32(const double (&x)[R], const double (&y)[R],
                                                          const double (&z)[R], const int (&jr)[R], int P,
                                                          double mu_sun, const double* srec, const double* smu,
                                                          float (&G)[6][R])
{
    // ONE_NODE: the R points share node jr[0] (WIDE); else point r is at node jr[r]
    auto rec = [&](int r) { return srec + (ONE_NODE ? jr[0] : jr[r]) * 3 * (P + 1); };
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int e = 0; e < 6; ++e) G[e][r] = 0.0f;
    }
    auto add = [&](int r, float dx, float dy, float dz, float mu) {
        const float q = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
        const float q2 = q * q;
        const float m3 = mu * q * q2;          // mu / |d|^3
        const float m5 = 3.0f * m3 * q2;       // 3 mu / |d|^5
        const float tx = m5 * dx, ty = m5 * dy, tz = m5 * dz;
        G[0][r] += fmaf(tx, dx, -m3);
        G[1][r] += fmaf(ty, dy, -m3);
        G[2][r] += fmaf(tz, dz, -m3);
        G[3][r] = fmaf(tx, dy, G[3][r]);
        G[4][r] = fmaf(tx, dz, G[4][r]);
        G[5][r] = fmaf(ty, dz, G[5][r]);
    };
    const float ms = (float)mu_sun;
#pragma unroll
    for (int r = 0; r < R; ++r) add(r, (float)x[r], (float)y[r], (float)z[r], ms);
    for (int b = 0; b < P; ++b) {
        const float mu = (float)smu[b];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double* q = rec(r) + 3 * b;
            add(r, (float)(x[r] - q[0]), (float)(y[r] - q[1]), (float)(z[r] - q[2]), mu);
        }
    }
}

// 1/sqrt(x) in full FP64 for finite x > 0: the hardware estimate y, e = 1 - x y^2, and
// (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + O(e^3) (|e| near 2^-22, dropped terms below 2^-63).
static __device__ __forceinline__ double pc_rsqrt_full(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x, y * y, 1.0);
    return y * fma(e, fma(0.375, e, 0.5), 1.0);
}

// Records of the relativistic model per node: for every major body b = 0..P (0 = the
// central body) three double4, (r_b, U_b - 2 v_b^2), (v_b, mu_b), (a_b, 0), with U_b the
// potential of the other major bodies at b (the two terms of the bracket below that depend
// on body b alone, summed once per node), then the indirect term (ax, ay, az, 0).  A
// segment's records are stored slot-major, [slot][node], so that the lanes of a wave,
// which hold consecutive nodes, read consecutive double4.
constexpr int pc_eih_rec(int P) { return 3 * (P + 1) + 1; }


// A segment's records read from a base address and a slot stride that are one value per
// wave (scalar registers): each load adds only the 32-bit byte offset of the lane's node,
// a global load with a scalar base and no per-lane address arithmetic.  Every caller's
// records are those of one segment of one group, the same for all lanes of the wave.
struct PcEihRecs {
    gconst_cp base;   // slot 0, node 0
    uint32_t slot;    // bytes per slot (ns double4)
};
static __device__ __forceinline__ PcEihRecs pc_eih_recs(const double4* e, int ns)
{
    PcEihRecs E;
    E.base = pc_wave_base(e);
    E.slot = (uint32_t)__builtin_amdgcn_readfirstlane(ns) * 32u;
    return E;
}
static __device__ __forceinline__ double4 pc_eih_load(const PcEihRecs& E, int k, uint32_t vo)
{
    return pc_load_d4(E.base + (size_t)k * E.slot + vo);
}

// Einstein-Infeld-Hoffmann acceleration of R massless points (x, y, z, vx, vy, vz) at one
// node (PPN beta = gamma = 1, Sec. 5.4.1): with d = r - r_b, rho = |d| and the potential
// Phi = sum_b mu_b / rho_b at the point,
//   a = sum_b -mu_b d / rho^3 [1 - (4 Phi + U_b - v^2 - 2 v_b^2 + 4 v.v_b
//                                   + 3/2 (d.v_b / rho)^2 + 1/2 d.a_b) / c^2]
//     + sum_b mu_b / (c^2 rho^3) [d.(4 v - 3 v_b)] (v - v_b) + 7/2 sum_b mu_b a_b / (c^2 rho)
// minus the Newtonian indirect term.  The term in Phi is 4 Phi / c^2 sum_b mu_b d / rho^3,
// so one pass over the bodies accumulates Phi, that sum and the rest, and the term is
// added at the end (the same sum in another order).  e: the segment's records, slot k of
// node j at e[k ns + j]; point r sits at node jr[r] (ONE_NODE: all at jr[0], one load
// per record for the R points).
template <int R, bool ONE_NODE>
static __device__ __forceinline__ void pc_force_eih(const double (&x)[R], const double (&y)[R],
                                                    const double (&z)[R], const double (&vx)[R],
                                                    const double (&vy)[R], const double (&vz)[R],
                                                    const double4* __restrict__ e, const int (&jr)[R], int ns,
                                                    int P, double inv_c2, double (&ax)[R], double (&ay)[R],
                                                    double (&az)[R])
{
    const PcEihRecs E = pc_eih_recs(e, ns);
    uint32_t vo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) vo[r] = (uint32_t)jr[ONE_NODE ? 0 : r] * 32u;
    auto rec = [&](int k, int r) -> double4 { return pc_eih_load(E, k, vo[r]); };
    const double c35 = 3.5 * inv_c2;
    double phi[R], v2[R], nx[R], ny[R], nz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        phi[r] = 0.0;
        v2[r] = vx[r] * vx[r] + vy[r] * vy[r] + vz[r] * vz[r];
        ax[r] = ay[r] = az[r] = 0.0;
        nx[r] = ny[r] = nz[r] = 0.0;
    }
    // the next body's records are loaded while this one's terms are formed
    double4 qn = rec(0, 0), wn = rec(1, 0), gn = rec(2, 0);
    for (int b = 0; b <= P; ++b) {
        double4 q = qn, w = wn, g = gn;
        if (b < P) {
            qn = rec(3 * b + 3, 0);
            wn = rec(3 * b + 4, 0);
            gn = rec(3 * b + 5, 0);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!ONE_NODE && r > 0) {
                q = rec(3 * b, r);
                w = rec(3 * b + 1, r);
                g = rec(3 * b + 2, r);
            }
            const double mu = w.w;
            const double dx = x[r] - q.x, dy = y[r] - q.y, dz = z[r] - q.z;
            const double i1 = pc_rsqrt_full(dx * dx + dy * dy + dz * dz);
            const double m1 = mu * i1;
            const double m3 = m1 * i1 * i1;          // mu / rho^3
            phi[r] += m1;
            nx[r] = fma(m3, dx, nx[r]);
            ny[r] = fma(m3, dy, ny[r]);
            nz[r] = fma(m3, dz, nz[r]);
            const double vbv = vx[r] * w.x + vy[r] * w.y + vz[r] * w.z;
            const double dwb = dx * w.x + dy * w.y + dz * w.z;   // d.v_b
            const double dvb = dwb * i1;
            const double dab = dx * g.x + dy * g.y + dz * g.z;
            const double s = q.w - v2[r] + 4.0 * vbv + 1.5 * dvb * dvb + 0.5 * dab;   // q.w = U_b - 2 v_b^2
            const double k1 = -m3 * fma(-inv_c2, s, 1.0);
            const double dv = dx * vx[r] + dy * vy[r] + dz * vz[r];
            const double k2 = inv_c2 * m3 * fma(4.0, dv, -3.0 * dwb);   // d.(4 v - 3 v_b)
            const double k3 = c35 * m1;
            ax[r] += k1 * dx + k2 * (vx[r] - w.x) + k3 * g.x;
            ay[r] += k1 * dy + k2 * (vy[r] - w.y) + k3 * g.y;
            az[r] += k1 * dz + k2 * (vz[r] - w.z) + k3 * g.z;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double4 ind = rec(3 * (P + 1), r);
        const double f = 4.0 * inv_c2 * phi[r];
        ax[r] = fma(f, nx[r], ax[r]) - ind.x;
        ay[r] = fma(f, ny[r], ay[r]) - ind.y;
        az[r] = fma(f, nz[r], az[r]) - ind.z;
    }
}

// Vector-Jacobian product of the relativistic acceleration of pc_force_eih at R points:
// with s = u . a, gr = ds/dr = (da/dr)^T u and gv = ds/dv = (da/dv)^T u (the adjoint's
// J^T w with u = w_v).  Per body, with d, rho, m3 = mu/rho^3, m5 = 3 mu/rho^5,
// S = U_b - v^2 - 2 v_b^2 + 4 v.v_b + 3/2 (d.v_b/rho)^2 + 1/2 d.a_b, q = 4 v - 3 v_b and
// e = 1/c^2:
//   gv += e m3 [-(u.d)(2 v - 4 v_b) + (d.q) u + 4 (u.(v - v_b)) d]
//   gr += (1 - e S) (m5 (u.d) d - m3 u) + e m3 (u.d) dS/dr
//         + e (u.(v - v_b)) (m3 q - m5 (d.q) d) - 7/2 e (u.a_b) m3 d,
//   dS/dr = 3 (d.v_b/rho) (v_b - (d.v_b/rho) d/rho)/rho + a_b/2,
// and the terms through Phi = sum_b mu_b/rho_b, whose gradient is -N with
// N = sum_b m3 d: gr += -4 e Phi H - 4 e (u.N) N, H = sum_b (m5 (u.d) d - m3 u).  At
// e = 0 this is the point-mass Hessian product (symmetric in r).  The indirect term does
// not depend on the state.  Records and node indices as pc_force_eih.
template <int R, bool ONE_NODE>
static __device__ __forceinline__ void pc_eih_vjp(const double (&x)[R], const double (&y)[R],
                                                  const double (&z)[R], const double (&vx)[R],
                                                  const double (&vy)[R], const double (&vz)[R],
                                                  const double (&ux)[R], const double (&uy)[R],
                                                  const double (&uz)[R], const double4* __restrict__ e,
                                                  const int (&jr)[R], int ns, int P, double inv_c2,
                                                  double (&grx)[R], double (&gry)[R], double (&grz)[R],
                                                  double (&gvx)[R], double (&gvy)[R], double (&gvz)[R])
{
    const PcEihRecs E = pc_eih_recs(e, ns);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t vo = (uint32_t)jr[ONE_NODE ? 0 : r] * 32u;
        auto rec = [&](int k, int) -> double4 { return pc_eih_load(E, k, vo); };
        double phi = 0.0, v2 = vx[r] * vx[r] + vy[r] * vy[r] + vz[r] * vz[r];
        double nx = 0.0, ny = 0.0, nz = 0.0, hx = 0.0, hy = 0.0, hz = 0.0;
        double ax = 0.0, ay = 0.0, az = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
        for (int b = 0; b <= P; ++b) {
            const double4 q = rec(3 * b, r), w = rec(3 * b + 1, r), g = rec(3 * b + 2, r);
            const double mu = w.w;
            const double dx = x[r] - q.x, dy = y[r] - q.y, dz = z[r] - q.z;
            const double i1 = pc_rsqrt_full(dx * dx + dy * dy + dz * dz);
            const double m1 = mu * i1, m3 = m1 * i1 * i1, m5 = 3.0 * m3 * i1 * i1;
            phi += m1;
            nx = fma(m3, dx, nx);
            ny = fma(m3, dy, ny);
            nz = fma(m3, dz, nz);
            const double ud = ux[r] * dx + uy[r] * dy + uz[r] * dz;
            // Newtonian part of the bracket, kept apart for the term in Phi
            const double tx = m5 * ud * dx - m3 * ux[r], ty = m5 * ud * dy - m3 * uy[r], tz = m5 * ud * dz - m3 * uz[r];
            hx += tx;
            hy += ty;
            hz += tz;
            const double vbv = vx[r] * w.x + vy[r] * w.y + vz[r] * w.z;
            const double dwb = dx * w.x + dy * w.y + dz * w.z;
            const double dvb = dwb * i1;
            const double dab = dx * g.x + dy * g.y + dz * g.z;
            const double S = q.w - v2 + 4.0 * vbv + 1.5 * dvb * dvb + 0.5 * dab;   // q.w = U_b - 2 v_b^2
            const double dq = fma(4.0, dx * vx[r] + dy * vy[r] + dz * vz[r], -3.0 * dwb);
            const double uvw = ux[r] * (vx[r] - w.x) + uy[r] * (vy[r] - w.y) + uz[r] * (vz[r] - w.z);
            const double ug = ux[r] * g.x + uy[r] * g.y + uz[r] * g.z;
            // dS/dr
            const double c1 = 3.0 * dvb * i1, c2 = c1 * dvb * i1;
            const double sx = c1 * w.x - c2 * dx + 0.5 * g.x;
            const double sy = c1 * w.y - c2 * dy + 0.5 * g.y;
            const double sz = c1 * w.z - c2 * dz + 0.5 * g.z;
            const double k0 = -S;                       // times e, on the Newtonian bracket
            const double k1 = m3 * ud;                  // times e, on dS/dr
            const double k2 = uvw;                      // times e, on m3 q - m5 (d.q) d
            const double k3 = -3.5 * ug * m3;           // times e, on d
            ax += k0 * tx + k1 * sx + k2 * (m3 * (4.0 * vx[r] - 3.0 * w.x) - m5 * dq * dx) + k3 * dx;
            ay += k0 * ty + k1 * sy + k2 * (m3 * (4.0 * vy[r] - 3.0 * w.y) - m5 * dq * dy) + k3 * dy;
            az += k0 * tz + k1 * sz + k2 * (m3 * (4.0 * vz[r] - 3.0 * w.z) - m5 * dq * dz) + k3 * dz;
            // velocity gradient
            bx += m3 * (-ud * (2.0 * vx[r] - 4.0 * w.x) + dq * ux[r] + 4.0 * uvw * dx);
            by += m3 * (-ud * (2.0 * vy[r] - 4.0 * w.y) + dq * uy[r] + 4.0 * uvw * dy);
            bz += m3 * (-ud * (2.0 * vz[r] - 4.0 * w.z) + dq * uz[r] + 4.0 * uvw * dz);
        }
        const double un = ux[r] * nx + uy[r] * ny + uz[r] * nz;
        const double fp = -4.0 * inv_c2 * phi, fn = -4.0 * inv_c2 * un;
        grx[r] = hx + inv_c2 * ax + fp * hx + fn * nx;
        gry[r] = hy + inv_c2 * ay + fp * hy + fn * ny;
        grz[r] = hz + inv_c2 * az + fp * hz + fn * nz;
        gvx[r] = inv_c2 * bx;
        gvy[r] = inv_c2 * by;
        gvz[r] = inv_c2 * bz;
    }
}

// Publish F = (v, a) with the relativistic acceleration.  erec: the segment's records,
// pc_eih_rec(P) slots of N double4.  WIDE shapes: a lane's four points share node j.
// 8-column shapes: as in pc_publish, lane pairs (l, l ^ 8) hold the points of one IC (the
// low lane x, z, vy, the high lane y, vx, vz) and each lane evaluates one strip (hd = hi),
// taking the three components it lacks from its partner.
template <int PAIRS, int NP>
static __device__ __forceinline__ void pc_publish_eih(double* sF, const double (&yc)[6][4], const PcLane& L,
                                                      int N, int P, const double4* erec, double inv_c2)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, ROW = Sh::ROW;
    if constexpr (Sh::WIDE) {
        const int j = pc_node(L, 0, 0);
        if (j >= N) return;
        const int jr[4] = {j, j, j, j};
        double ax[4], ay[4], az[4];
        pc_force_eih<4, true>(yc[0], yc[1], yc[2], yc[3], yc[4], yc[5], erec, jr, N, P, inv_c2, ax, ay, az);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double* f = sF + j * ROW + pc_fcol<PAIRS, NP>(j, pc_ic(L, r));
            f[0 * T] = yc[3][r];
            f[1 * T] = yc[4][r];
            f[2 * T] = yc[5][r];
            f[3 * T] = ax[r];
            f[4 * T] = ay[r];
            f[5 * T] = az[r];
        }
    } else {
        const int hi = L.hi;
        const int my_m = pc_ic(L, 0);
        double xs[4], ys[4], zs[4], us[4], vs[4], ws[4], ax[4], ay[4], az[4];
        int jr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double e1 = pc_dpp<0x128>(hi ? yc[0][r] : yc[3][r]);   // lane ^ 8
            const double e2 = pc_dpp<0x128>(hi ? yc[1][r] : yc[4][r]);
            const double e3 = pc_dpp<0x128>(hi ? yc[2][r] : yc[5][r]);
            xs[r] = hi ? e1 : yc[0][r];
            ys[r] = hi ? yc[3][r] : e1;
            zs[r] = hi ? e2 : yc[1][r];
            us[r] = hi ? yc[4][r] : e2;
            vs[r] = hi ? e3 : yc[2][r];
            ws[r] = hi ? yc[5][r] : e3;
            const int j = pc_node(L, hi, r);
            jr[r] = j < N ? j : N - 1;
        }
        pc_force_eih<4, false>(xs, ys, zs, us, vs, ws, erec, jr, N, P, inv_c2, ax, ay, az);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, hi, r);
            if (j < N) {
                double* f = sF + j * ROW + my_m;
                f[3 * T] = ax[r];
                f[4 * T] = ay[r];
                f[5 * T] = az[r];
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = pc_node(L, h, r);
                if (j < N) {
                    double* f = sF + j * ROW + my_m;
                    if (hi) {
                        f[0 * T] = yc[3 * h + 1][r];   // vx (comp 3)
                        f[2 * T] = yc[3 * h + 2][r];   // vz (comp 5)
                    } else {
                        f[1 * T] = yc[3 * h + 2][r];   // vy (comp 4)
                    }
                }
            }
        }
    }
}

// Publish for an increment sweep.  The increment of F = (v, a) from the last
// change dy of the iterate, to first order: dF = (dv, G dr), with G the gravity gradient
// at the anchor, the iterate after the last FP64 sweep (ANCHOR: evaluated here at yc and
// kept in sG, [node][6][IC] FP32, read back only by the same lane; else read from sG).
// dF goes to sD rounded to FP32.  act[r]: the lane's IC r iterates (others publish zero,
// so that no stale or non-finite value reaches the product).
template <int PAIRS, int NP>
static __device__ __forceinline__ void pc_publish_chord(float* sD, float* sG, const double (&yc)[6][4],
                                                        const float (&dy)[6][4], const int (&act)[4],
                                                        bool anchor, const PcLane& L, int N, int P,
                                                        double mu_sun, const double* sRec, const double* sMu)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, ROW = Sh::ROW;
    if constexpr (!Sh::WIDE) {
        // 8-IC jobs (node-row layout, lane pairs sharing an IC's components): each lane
        // stores dv for its own velocity components at its eight nodes, and forms G dr at
        // the four points of strip hi (G from the anchor's position, kept in sG by the same
        // lane), taking the components it lacks from its partner as pc_publish does
        const int hi = L.hi, m = pc_ic(L, 0);
        const bool on = act[0];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = pc_node(L, h, r);
                float* d = sD + j * ROW + m;
                const bool ok = j < N;   // rows past N stay zero (they meet zero operator columns)
#pragma unroll
                for (int cb = 0; cb < 3; ++cb) {
                    const int c = 2 * cb + hi;
                    if (c >= 3) d[(c - 3) * T] = ok ? dy[3 * h + cb][r] : 0.0f;
                }
            }
        }
        double xs[4], ys[4], zs[4];
        float rx[4], ry[4], rz[4];
        int jr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double e1 = pc_dpp<0x128>(hi ? yc[0][r] : yc[3][r]);   // lo: y(0); hi: x(1)
            const double e2 = pc_dpp<0x128>(yc[4][r]);                   // hi: z(1)
            const float f1 = pc_dpp<0x128>(hi ? dy[0][r] : dy[3][r]);    // lo: dy(0); hi: dx(1)
            const float f2 = pc_dpp<0x128>(dy[4][r]);                    // hi: dz(1)
            xs[r] = hi ? e1 : yc[0][r];
            ys[r] = hi ? yc[3][r] : e1;
            zs[r] = hi ? e2 : yc[1][r];
            rx[r] = hi ? f1 : dy[0][r];
            ry[r] = hi ? dy[3][r] : f1;
            rz[r] = hi ? f2 : dy[1][r];
            const int j = pc_node(L, hi, r);
            jr[r] = j < N ? j : N - 1;
        }
        float G[6][4];
        if (anchor) {
            pc_grad_lds_node32<4, false>(xs, ys, zs, jr, P, mu_sun, sRec, sMu, G);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float* g = sG + pc_node(L, hi, r) * 6 * T + m;
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    G[e][r] = on ? G[e][r] : 0.0f;
                    g[e * T] = G[e][r];
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float* g = sG + pc_node(L, hi, r) * 6 * T + m;
#pragma unroll
                for (int e = 0; e < 6; ++e) G[e][r] = g[e * T];
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, hi, r);
            const bool ok = j < N;
            float* d = sD + j * ROW + m;
            d[3 * T] = ok ? fmaf(G[0][r], rx[r], fmaf(G[3][r], ry[r], G[4][r] * rz[r])) : 0.0f;
            d[4 * T] = ok ? fmaf(G[3][r], rx[r], fmaf(G[1][r], ry[r], G[5][r] * rz[r])) : 0.0f;
            d[5 * T] = ok ? fmaf(G[4][r], rx[r], fmaf(G[5][r], ry[r], G[2][r] * rz[r])) : 0.0f;
        }
        return;
    }
    const int j = pc_node(L, 0, 0);
    if (j >= N) {   // rows past N meet zero operator columns: keep them zero (no stale NaN bits)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float* d = sD + j * ROW + pc_fcol<PAIRS, NP>(j, pc_ic(L, r));
#pragma unroll
            for (int c = 0; c < 6; ++c) d[c * T] = 0.0f;
        }
        return;
    }
    float G[6][4];
    if (anchor) {
        pc_grad_lds_node32<4>(yc[0], yc[1], yc[2], {j, j, j, j}, P, mu_sun, sRec, sMu, G);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float* g = sG + j * 6 * T + pc_fcol<PAIRS, NP>(j, pc_ic(L, r));
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                G[e][r] = act[r] ? G[e][r] : 0.0f;
                g[e * T] = G[e][r];
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float* g = sG + j * 6 * T + pc_fcol<PAIRS, NP>(j, pc_ic(L, r));
#pragma unroll
            for (int e = 0; e < 6; ++e) G[e][r] = g[e * T];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float* d = sD + j * ROW + pc_fcol<PAIRS, NP>(j, pc_ic(L, r));
        const float rx = dy[0][r], ry = dy[1][r], rz = dy[2][r];
        d[0 * T] = dy[3][r];
        d[1 * T] = dy[4][r];
        d[2 * T] = dy[5][r];
        d[3 * T] = fmaf(G[0][r], rx, fmaf(G[3][r], ry, G[4][r] * rz));
        d[4 * T] = fmaf(G[3][r], rx, fmaf(G[1][r], ry, G[5][r] * rz));
        d[5 * T] = fmaf(G[4][r], rx, fmaf(G[5][r], ry, G[2][r] * rz));
    }
}

// Load the lane's share of a [node][comp][IC] array with row stride `row` and comp stride
// `cs` (WIDE: yc[c][r]; T == 8: yc[3h + cb][r] = comp 2cb + hi); SWZ: an LDS array with
// the column swizzle of pc_fcol.
template <int PAIRS, int NP, bool SWZ = false, class Ptr>
static __device__ __forceinline__ void pc_load_share(Ptr base, size_t row, size_t cs, double (&yc)[6][4],
                                                     const PcLane& L, int N)
{
    using Sh = PcShape<PAIRS, NP>;
#pragma unroll
    for (int h = 0; h < Sh::H; ++h) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, h, r);
            const int jj = j < N ? j : N - 1;
            const int m = SWZ ? pc_fcol<PAIRS, NP>(jj, pc_ic(L, r)) : pc_ic(L, r);
            if constexpr (Sh::WIDE) {
#pragma unroll
                for (int c = 0; c < 6; ++c) yc[c][r] = base[jj * row + c * cs + m];
            } else {
#pragma unroll
                for (int cb = 0; cb < 3; ++cb) yc[3 * h + cb][r] = base[jj * row + (2 * cb + L.hi) * cs + m];
            }
        }
    }
}
