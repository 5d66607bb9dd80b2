// pc_kernels.hip -- gfx950 kernels of the batched Picard-Chebyshev propagator.
//
// Method: arXiv 2301.03989, Sec. 2.2 (matrix form of the Picard-Chebyshev iteration),
// Sec. 3 (augmentation of many trajectories on common nodes), Sec. 5.4 (GPU program:
// dynamics at every node, the fit/integrate/evaluate products, error and its reduction).
//
// The fused kernel gives each workgroup one job (T ICs x NP nodes of one group) and runs
// the whole propagation of those ICs on chip: for every segment it builds the initial
// guess, then repeats {force at all nodes (FP64 VALU), y_new = y0 + w2 K_N F (FP64 MFMA
// 16x16x4), per-IC error and stopping decision} until each IC has converged, chains the
// last node into the next segment and finally writes the end states.  The iterate and
// the force matrix never leave LDS, so HBM traffic is only the initial states, the
// ephemeris records and the results; K_N fragments are re-read from L2.
#include <hip/hip_runtime.h>
#include <math.h>
#include "pc_internal.h"

typedef double f64x4 __attribute__((ext_vector_type(4)));

#define PC_PI 3.14159265358979323846

static __device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c)
{
    // D = A(16x4) B(4x16) + C.  Operand lanes: A[l%16][l/16], B[l/16][l%16];
    // result lanes on gfx950: D[l/16 + 4r][l%16] in element r.
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
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
        if (fabs(dE) <= 1e-16 * (1.0 + fabs(E))) break;
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

// Warm start (Sec. 2.1): propagate y0 by dt on its osculating ellipse, through the
// Lagrange coefficients f, g, fdot, gdot written in the eccentric-anomaly change x:
//   x - (1 - r0/a) sin x + (r0.v0/sqrt(a)) (1 - cos x) = n dt.
// Returns false for non-elliptic or degenerate states.
static __device__ __attribute__((noinline)) bool pc_kepler(const double y0[6], double dt, double y[6])
{
    const double r0n = sqrt(y0[0] * y0[0] + y0[1] * y0[1] + y0[2] * y0[2]);
    const double v02 = y0[3] * y0[3] + y0[4] * y0[4] + y0[5] * y0[5];
    if (!(r0n > 0.0) || !isfinite(r0n) || !isfinite(v02)) return false;
    const double alpha = 2.0 / r0n - v02;          // 1/a
    if (!(alpha > 0.0)) return false;
    const double a = 1.0 / alpha;
    const double sqa = sqrt(a);
    const double n = alpha * sqrt(alpha);          // mean motion
    const double sig = y0[0] * y0[3] + y0[1] * y0[4] + y0[2] * y0[5];
    const double ec = 1.0 - r0n * alpha;           // e cos E0
    const double es = sig / sqa;                   // e sin E0
    const double ndt = n * dt;
    double x = ndt;
    for (int it = 0; it < 60; ++it) {
        double sx, cx;
        sincos(x, &sx, &cx);
        const double F = x - ec * sx + es * (1.0 - cx) - ndt;
        const double dx = F / (1.0 - ec * cx + es * sx);
        x -= dx;
        if (fabs(dx) <= 1e-16 * (1.0 + fabs(x))) break;
    }
    double sx, cx;
    sincos(x, &sx, &cx);
    const double rn = a + (r0n - a) * cx + sig * sqa * sx;
    const double f = 1.0 - (a / r0n) * (1.0 - cx);
    const double g = dt - (x - sx) / n;
    const double fd = -sqa * sx / (rn * r0n);
    const double gd = 1.0 - (a / rn) * (1.0 - cx);
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
        y[k] = f * y0[k] + g * y0[3 + k];
        y[3 + k] = fd * y0[k] + gd * y0[3 + k];
        ok = ok && isfinite(y[k]) && isfinite(y[3 + k]);
    }
    return ok;
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
    const double r2 = x * x + y * y + z * z;
    const double ir = rsqrt(r2);
    const double s = mu_sun * (ir * ir * ir);
    ax = -s * x;
    ay = -s * y;
    az = -s * z;
    for (int p = 0; p < P; ++p) {
        const double4 q = rec[p];
        const double dx = x - q.x, dy = y - q.y, dz = z - q.z;
        const double id = rsqrt(dx * dx + dy * dy + dz * dz);
        const double sd = q.w * (id * id * id);
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
// Ephemeris records: one thread per (group, segment, node)
// ---------------------------------------------------------------------------
__global__ void pc_ephem_kernel(const PcEphemParams p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_recs) return;
    int lo = 0, hi = p.n_groups - 1;             // last group with rec_offset <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.groups[mid].rec_offset <= i) lo = mid; else hi = mid - 1;
    }
    const PcGroupDev& G = p.groups[lo];
    const int64_t local = i - G.rec_offset;
    const int s = (int)(local / G.N);
    const int j = (int)(local - (int64_t)s * G.N);
    const double Ts = G.t0 + G.h * s, Te = G.t0 + G.h * (s + 1);
    const double t = 0.5 * (Te - Ts) * G.tau[j] + 0.5 * (Te + Ts);   // eq. chnodes1
    const int P = p.n_pert;
    double4* rec = reinterpret_cast<double4*>(p.recs) + i * (P + 1);
    double ix = 0.0, iy = 0.0, iz = 0.0;
    for (int b = 0; b < P; ++b) {
        double r[3];
        pc_body_position(p.bodies[b], t - p.epoch, r);
        const double mu = p.bodies[b].mu;
        rec[b] = make_double4(r[0], r[1], r[2], mu);
        const double q2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double iq = rsqrt(q2);
        const double sq = mu * (iq * iq * iq);
        ix += sq * r[0];
        iy += sq * r[1];
        iz += sq * r[2];
    }
    rec[P] = make_double4(ix, iy, iz, 0.0);
}

int pc_launch_ephem(const PcEphemParams& p, void* stream)
{
    if (p.n_recs <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t grid = (p.n_recs + bs - 1) / bs;
    hipLaunchKernelGGL(pc_ephem_kernel, dim3((unsigned)grid), dim3(bs), 0, (hipStream_t)stream, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused propagation kernel
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(1))) double* gconst_dp;

// Shared-memory arena of one workgroup (sized for the largest job shape).
template <int PAIRS>
struct PcSmem {
    static constexpr int REC = PAIRS >= 2048 ? 7040 : 3072;   // doubles of ephemeris kept in LDS
    double F[6 * PAIRS];          // [node][F comp 6][IC]: velocity (0..2), acceleration (3..5)
    double Rec[REC];              // [node][body 0..P][3]: perturber positions, then the indirect term
    double Y0[6 * (PAIRS / 16)];  // [comp][IC] initial state of the current segment
    double Mu[PC_MAX_PERT_DEV];   // perturber parameters
    int Flag[(PAIRS / 256) * 16]; // per wave, per IC: bit 0 not converged, bit 1 non-finite
    int Active[PAIRS / 16];
    int Dead[PAIRS / 16];
};

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
        const double ir = rsqrt(x[r] * x[r] + y[r] * y[r] + z[r] * z[r]);
        const double s = mu_sun * (ir * ir * ir);
        ax[r] = -s * x[r];
        ay[r] = -s * y[r];
        az[r] = -s * z[r];
    }
    for (int b = 0; b < P; ++b) {
        const double mu = smu[b];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double* q = srec + jr[r] * stride + 3 * b;
            const double dx = x[r] - q[0], dy = y[r] - q[1], dz = z[r] - q[2];
            const double id = rsqrt(dx * dx + dy * dy + dz * dz);
            const double sd = mu * (id * id * id);
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

// Same with the records read from global memory ((x, y, z, mu) per body, then the indirect term).
template <int R>
static __device__ __forceinline__ void pc_force_glb(const double (&x)[R], const double (&y)[R],
                                                    const double (&z)[R], const int (&jr)[R], int P,
                                                    double mu_sun, const double4* grec,
                                                    double (&ax)[R], double (&ay)[R], double (&az)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double ir = rsqrt(x[r] * x[r] + y[r] * y[r] + z[r] * z[r]);
        const double s = mu_sun * (ir * ir * ir);
        ax[r] = -s * x[r];
        ay[r] = -s * y[r];
        az[r] = -s * z[r];
    }
    for (int b = 0; b < P; ++b) {
        double4 q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) q[r] = grec[(size_t)jr[r] * (P + 1) + b];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double dx = x[r] - q[r].x, dy = y[r] - q[r].y, dz = z[r] - q[r].z;
            const double id = rsqrt(dx * dx + dy * dy + dz * dz);
            const double sd = q[r].w * (id * id * id);
            ax[r] -= sd * dx;
            ay[r] -= sd * dy;
            az[r] -= sd * dz;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double4 q = grec[(size_t)jr[r] * (P + 1) + P];
        ax[r] -= q.x;
        ay[r] -= q.y;
        az[r] -= q.z;
    }
}

// One job: T = PAIRS/NP ICs of one group, all segments.
//
// Ownership: every wave owns six 16x16 blocks of the iterate (node rows x component
// columns) for the whole job.  It keeps its blocks of the current iterate in registers
// (in the MFMA result layout), computes the dynamics for the (node, IC) pairs it owns
// straight from them, and publishes only the force matrix F = (v, a) to LDS, where the
// product y_new = y0 + w2 K_N F reads it as the B operand.  Compile-time NP makes every
// LDS offset an immediate and lets a wave hold its 16-row strip of K_N in registers.
template <int PAIRS, int NP>
__device__ __forceinline__ void pc_job(const PcParams& p, const PcJobDev& job, const PcGroupDev& g,
                                       PcSmem<PAIRS>& sm)
{
    constexpr int NT = PAIRS / 4;          // threads
    constexpr int W = NT / 64;             // waves
    constexpr int T = PAIRS / NP;          // ICs per job
    constexpr int ROW = 6 * T;             // doubles per node row of F
    constexpr int NQ = NP / 4;             // k-steps of the 16x16x4 product
    static_assert(T >= 8 && T <= PAIRS / 16, "unsupported job shape");
    constexpr bool WIDE = (T >= 16);       // WIDE: one strip x six component blocks per wave
    constexpr int G16 = WIDE ? T / 16 : 1; // 16-IC groups per job

    double* sF = sm.F;
    double* sY0 = sm.Y0;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int N = g.N, S = g.S;
    const int n = job.n;
    const int P = p.n_pert;
    const int64_t ic = job.ic0 + tid;      // this thread's IC when tid < n
    const bool rec_lds = N * 3 * (P + 1) <= PcSmem<PAIRS>::REC;
    const double t2 = g.tol * g.tol;

    // lane geometry
    const int strip0 = WIDE ? wave / G16 : 2 * wave;
    const int grp = WIDE ? wave - strip0 * G16 : 0;
    const int my_m = WIDE ? grp * 16 + (lane & 15) : (lane & 7);
    const int hi = WIDE ? 0 : (lane >> 3) & 1;          // T == 8: lane holds comps hi, 2+hi, 4+hi

    for (int i = tid; i < 6 * PAIRS; i += NT) sF[i] = 0.0;
    if (tid < T) {
        const double* y = p.ics + (job.ic0 + (tid < n ? tid : 0)) * 6;
        bool fin = true;
        for (int c = 0; c < 6; ++c) {
            const double v = y[c];
            sY0[c * T + tid] = v;
            fin = fin && isfinite(v);
        }
        sm.Dead[tid] = !fin;
    }
    if (tid < P) sm.Mu[tid] = 0.0;

    gconst_dp kp0 = (gconst_dp)g.kfrag + (size_t)strip0 * NQ * 64 + lane;
    __syncthreads();

    // the lane's share of the iterate: WIDE yc[comp][r] at node j0 + 4r;
    // T == 8: yc[3h + cb][r] = comp 2cb + hi at node (strip0 + h) * 16 + lane/16 + 4r
    double yc[6][4];
    int had_notconv = 0;
    for (int s = 0; s < S; ++s) {
        const double Ts = g.t0 + g.h * s, Te = g.t0 + g.h * (s + 1);
        const double w2 = 0.5 * (Te - Ts);

        if (tid < n) {
            if (p.bounds_out) {
                double* bo = p.bounds_out + ((size_t)ic * (p.iters_stride + 1) + s) * 6;
                for (int c = 0; c < 6; ++c) bo[c] = sY0[c * T + tid];
            }
            if (sm.Dead[tid] && p.iters_out) p.iters_out[(size_t)ic * p.iters_stride + s] = -2;
        }
        // this segment's ephemeris records into LDS (perturber positions precomputed per node, Sec. 5.4.1)
        const double4* grec = reinterpret_cast<const double4*>(p.recs) +
                              (size_t)(g.rec_offset + (int64_t)s * N) * (P + 1);
        if (rec_lds) {
            for (int i = tid; i < N * (P + 1); i += NT) {
                const double4 q = grec[i];
                sm.Rec[3 * i + 0] = q.x;
                sm.Rec[3 * i + 1] = q.y;
                sm.Rec[3 * i + 2] = q.z;
                if (i < P) sm.Mu[i] = q.w;
            }
        }
        // initial guess at every (node, IC) pair: warm (Kepler) or cold start, Sec. 2.1,
        // staged through the F area as [node][comp 6][IC]
        {
            const int pm = tid % T;
            double y0[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) y0[c] = sY0[c * T + pm];
            const bool warm = p.init == 0 && !sm.Dead[pm];
#pragma unroll 1
            for (int pr = tid; pr < PAIRS; pr += NT) {
                const int j = pr / T;
                double y[6];
                if (!(j < N && warm && pc_kepler(y0, w2 * (g.tau[j < N ? j : 0] + 1.0), y))) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) y[c] = y0[c];
                }
                double* dst = sF + j * ROW + pm;
#pragma unroll
                for (int c = 0; c < 6; ++c) dst[c * T] = y[c];
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < (WIDE ? 1 : 2); ++h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = (strip0 + h) * 16 + (lane >> 4) + 4 * r;
                const double* src = sF + j * ROW + my_m;
                if constexpr (WIDE) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) yc[c][r] = src[c * T];
                } else {
#pragma unroll
                    for (int cb = 0; cb < 3; ++cb) yc[3 * h + cb][r] = src[(2 * cb + hi) * T];
                }
            }
        }
        __syncthreads();   // staging read before F is rebuilt
        for (int i = tid; i < 6 * PAIRS; i += NT) sF[i] = 0.0;
        if (tid < T) sm.Active[tid] = (tid < n) && !sm.Dead[tid];
        __syncthreads();   // records and flags visible

        // publish F = (v, a(r)) of the lane's pairs (the force matrix of Sec. 2.2)
        auto publish = [&]() {
            if constexpr (WIDE) {
                double ax[4], ay[4], az[4];
                int jr[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = strip0 * 16 + (lane >> 4) + 4 * r;
                    jr[r] = j < N ? j : N - 1;
                }
                if (rec_lds) pc_force_lds<4>(yc[0], yc[1], yc[2], jr, P, p.mu_sun, sm.Rec, sm.Mu, ax, ay, az);
                else pc_force_glb<4>(yc[0], yc[1], yc[2], jr, P, p.mu_sun, grec, ax, ay, az);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = strip0 * 16 + (lane >> 4) + 4 * r;
                    if (j < N) {
                        double* f = sF + j * ROW + my_m;
                        f[0 * T] = yc[3][r];
                        f[1 * T] = yc[4][r];
                        f[2 * T] = yc[5][r];
                        f[3 * T] = ax[r];
                        f[4 * T] = ay[r];
                        f[5 * T] = az[r];
                    }
                }
            } else {
                // lanes with hi == 0 hold x (cb 0) and z (cb 1); y comes from the partner lane
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    double xs[4], ys[4], zs[4], ax[4], ay[4], az[4];
                    int jr[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = (strip0 + h) * 16 + (lane >> 4) + 4 * r;
                        jr[r] = j < N ? j : N - 1;
                        xs[r] = yc[3 * h][r];
                        ys[r] = __shfl_xor(yc[3 * h][r], 8);
                        zs[r] = yc[3 * h + 1][r];
                    }
                    if (!hi) {
                        if (rec_lds) pc_force_lds<4>(xs, ys, zs, jr, P, p.mu_sun, sm.Rec, sm.Mu, ax, ay, az);
                        else pc_force_glb<4>(xs, ys, zs, jr, P, p.mu_sun, grec, ax, ay, az);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = (strip0 + h) * 16 + (lane >> 4) + 4 * r;
                        if (j < N) {
                            double* f = sF + j * ROW + my_m;
                            if (hi) {
                                f[0 * T] = yc[3 * h + 1][r];   // vx (comp 3)
                                f[2 * T] = yc[3 * h + 2][r];   // vz (comp 5)
                            } else {
                                f[1 * T] = yc[3 * h + 2][r];   // vy (comp 4)
                                f[3 * T] = ax[r];
                                f[4 * T] = ay[r];
                                f[5 * T] = az[r];
                            }
                        }
                    }
                }
            }
        };
        if (sm.Active[my_m]) publish();
        __syncthreads();

        const int n_it = p.fixed_iters > 0 ? p.fixed_iters : p.max_iter;
        for (int it = 1; it <= n_it; ++it) {
            // (1) y_new = y0 + w2 K_N F on the FP64 matrix cores (Sec. 2.2, folded A, C, S)
            f64x4 acc[6];
#pragma unroll
            for (int b = 0; b < 6; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
            int flag = 0;   // bit 0: some node not converged, bit 1: non-finite
            if constexpr (WIDE) {
                // K_N strip streamed from L2 two k-steps ahead; B operands one k-step ahead
                const double* bp = sF + (lane >> 4) * ROW + grp * 16 + (lane & 15);
                double bc[6], bn[6];
                double ka = kp0[0], kb = (NQ > 1) ? kp0[64] : 0.0;
#pragma unroll
                for (int b = 0; b < 6; ++b) bc[b] = bp[b * T];
#pragma unroll 2
                for (int q = 0; q < NQ; ++q) {
                    const double kn = (q + 2 < NQ) ? kp0[(q + 2) * 64] : 0.0;
                    if (q + 1 < NQ) {
#pragma unroll
                        for (int b = 0; b < 6; ++b) bn[b] = bp[(q + 1) * 4 * ROW + b * T];
                    }
#pragma unroll
                    for (int b = 0; b < 6; ++b) acc[b] = mfma16(ka, bc[b], acc[b]);
#pragma unroll
                    for (int b = 0; b < 6; ++b) bc[b] = bn[b];
                    ka = kb;
                    kb = kn;
                }
                // (2) new iterate and its change (stopping rule of Sec. 2.2, squared form)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = strip0 * 16 + (lane >> 4) + 4 * r;
                    double pd = 0.0, py = 0.0, vd = 0.0, vy = 0.0;
#pragma unroll
                    for (int b = 0; b < 6; ++b) {
                        const double yn = sY0[b * T + my_m] + w2 * acc[b][r];
                        acc[b][r] = yn;
                        const double d = yn - yc[b][r];
                        if (b < 3) { pd += d * d; py += yn * yn; }
                        else { vd += d * d; vy += yn * yn; }
                    }
                    if (j < N) {
                        const bool ok = p.tol_mode == 0 ? (pd < t2 * py && vd < t2 * vy) : (pd < t2 && vd < t2);
                        const bool nf = !isfinite(pd + py + vd + vy);
                        flag |= (ok ? 0 : 1) | (nf ? 2 : 0);
                    }
                }
            } else {
                gconst_dp kp1 = kp0 + (size_t)NQ * 64;
                const double* bp = sF + (lane >> 4) * ROW + (lane & 15);
                double a0 = kp0[0], a1 = kp1[0];
                double a0n = 0.0, a1n = 0.0;
                double b0 = bp[0], b1 = bp[16], b2 = bp[32];
#pragma unroll 4
                for (int q = 0; q < NQ; ++q) {
                    double b0n = 0.0, b1n = 0.0, b2n = 0.0;
                    if (q + 1 < NQ) {
                        a0n = kp0[(q + 1) * 64];
                        a1n = kp1[(q + 1) * 64];
                        const double* bq = bp + (q + 1) * 4 * ROW;
                        b0n = bq[0];
                        b1n = bq[16];
                        b2n = bq[32];
                    }
                    acc[0] = mfma16(a0, b0, acc[0]);
                    acc[1] = mfma16(a0, b1, acc[1]);
                    acc[2] = mfma16(a0, b2, acc[2]);
                    acc[3] = mfma16(a1, b0, acc[3]);
                    acc[4] = mfma16(a1, b1, acc[4]);
                    acc[5] = mfma16(a1, b2, acc[5]);
                    a0 = a0n; a1 = a1n;
                    b0 = b0n; b1 = b1n; b2 = b2n;
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = (strip0 + h) * 16 + (lane >> 4) + 4 * r;
                        double dd[3], yy[3];
#pragma unroll
                        for (int cb = 0; cb < 3; ++cb) {
                            const double yn = sY0[(2 * cb + hi) * T + my_m] + w2 * acc[3 * h + cb][r];
                            acc[3 * h + cb][r] = yn;
                            const double d = yn - yc[3 * h + cb][r];
                            dd[cb] = d * d;
                            yy[cb] = yn * yn;
                        }
                        double pd = dd[0] + (hi ? 0.0 : dd[1]);
                        double py = yy[0] + (hi ? 0.0 : yy[1]);
                        double vd = (hi ? dd[1] : 0.0) + dd[2];
                        double vy = (hi ? yy[1] : 0.0) + yy[2];
                        pd += __shfl_xor(pd, 8);
                        py += __shfl_xor(py, 8);
                        vd += __shfl_xor(vd, 8);
                        vy += __shfl_xor(vy, 8);
                        if (j < N) {
                            const bool ok = p.tol_mode == 0 ? (pd < t2 * py && vd < t2 * vy) : (pd < t2 && vd < t2);
                            const bool nf = !isfinite(pd + py + vd + vy);
                            flag |= (ok ? 0 : 1) | (nf ? 2 : 0);
                        }
                    }
                }
                flag |= __shfl_xor(flag, 8);
            }
            // (3) per-IC flags: over the wave's rows (lanes of one IC), then across waves
            flag |= __shfl_xor(flag, 16);
            flag |= __shfl_xor(flag, 32);
            if (lane < 16) sm.Flag[wave * 16 + lane] = flag;
            const int act = sm.Active[my_m];
            __syncthreads();   // every wave is done reading F; flags complete

            // (4) stopping rule per IC (Sec. 2.2; per-block error of Sec. 3.2 with blocks of one IC)
            if (tid < T && sm.Active[tid]) {
                int f = 0;
                if constexpr (WIDE) {
                    for (int w = tid >> 4; w < W; w += G16) f |= sm.Flag[w * 16 + (tid & 15)];
                } else {
                    for (int w = 0; w < W; ++w) f |= sm.Flag[w * 16 + tid];
                }
                int rec = 0;
                if (f & 2) rec = -2;
                else if (p.fixed_iters > 0) rec = (it == p.fixed_iters) ? it : 0;
                else if (!(f & 1)) rec = it;
                else if (it == p.max_iter) rec = -1;
                if (rec != 0) {
                    sm.Active[tid] = 0;
                    if (rec == -2) sm.Dead[tid] = 1;
                    if (rec == -1) had_notconv = 1;
                    if (tid < n && p.iters_out) p.iters_out[(size_t)ic * p.iters_stride + s] = rec;
                }
            }
            // (5) ICs that were iterating take the new iterate and publish its F
            if (act) {
#pragma unroll
                for (int b = 0; b < 6; ++b) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) yc[b][r] = acc[b][r];
                }
                if (it < n_it) publish();
            }
            const int any = __syncthreads_or(tid < T ? sm.Active[tid] : 0);
            if (!any) break;
        }

        // converged node states of the segment (optional output)
        if (p.nodes_out && my_m < n) {
#pragma unroll
            for (int h = 0; h < (WIDE ? 1 : 2); ++h) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = (strip0 + h) * 16 + (lane >> 4) + 4 * r;
                    if (j < N) {
                        double* o = p.nodes_out +
                                    (((size_t)(job.ic0 + my_m) * p.iters_stride + s) * p.nodes_stride + j) * 6;
                        if constexpr (WIDE) {
#pragma unroll
                            for (int c = 0; c < 6; ++c) o[c] = yc[c][r];
                        } else {
#pragma unroll
                            for (int cb = 0; cb < 3; ++cb) o[2 * cb + hi] = yc[3 * h + cb][r];
                        }
                    }
                }
            }
        }
        // chaining: the last node starts the next segment (piecewise integration, Sec. 2.2)
        {
            const bool dead = sm.Dead[my_m];
#pragma unroll
            for (int h = 0; h < (WIDE ? 1 : 2); ++h) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = (strip0 + h) * 16 + (lane >> 4) + 4 * r;
                    if (j == N - 1) {
                        if constexpr (WIDE) {
#pragma unroll
                            for (int c = 0; c < 6; ++c) sY0[c * T + my_m] = dead ? (double)NAN : yc[c][r];
                        } else {
#pragma unroll
                            for (int cb = 0; cb < 3; ++cb)
                                sY0[(2 * cb + hi) * T + my_m] = dead ? (double)NAN : yc[3 * h + cb][r];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }

    if (tid < n) {
        double* so = p.states_out + (size_t)ic * 6;
        for (int c = 0; c < 6; ++c) so[c] = sY0[c * T + tid];
        if (p.bounds_out) {
            double* bo = p.bounds_out + ((size_t)ic * (p.iters_stride + 1) + S) * 6;
            for (int c = 0; c < 6; ++c) bo[c] = sY0[c * T + tid];
        }
        if (had_notconv) atomicAdd(&p.counters[0], 1);
        if (sm.Dead[tid]) atomicAdd(&p.counters[1], 1);
    }
    __syncthreads();
}

// One kernel per (job shape, padded node count): jobs [job_begin, job_end) of the plan all
// have NP padded nodes.  A workgroup loops over jobs with a grid stride, so a grid smaller
// than the job count makes the launch persistent.
template <int PAIRS, int NP>
__global__ __launch_bounds__(PAIRS / 4) void pc_fused_kernel(const PcParams p, int job_begin, int job_end)
{
    __shared__ PcSmem<PAIRS> sm;
    for (int jb = job_begin + blockIdx.x; jb < job_end; jb += gridDim.x) {
        const PcJobDev job = p.jobs[jb];
        const PcGroupDev g = p.groups[job.group];
        pc_job<PAIRS, NP>(p, job, g, sm);
    }
}

template <int PAIRS, int NP>
static void launch_np(const PcParams& p, int jb, int je, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((pc_fused_kernel<PAIRS, NP>), dim3(grid), dim3(PAIRS / 4), 0, st, p, jb, je);
}

int pc_launch_fused(const PcParams& p, int pairs, int NP, int job_begin, int job_end, int grid, void* stream)
{
    if (job_end <= job_begin) return hipSuccess;
    hipStream_t st = (hipStream_t)stream;
    if (grid <= 0 || grid > job_end - job_begin) grid = job_end - job_begin;
    if (pairs == 2048) {
        switch (NP) {
        case 16: launch_np<2048, 16>(p, job_begin, job_end, grid, st); break;
        case 32: launch_np<2048, 32>(p, job_begin, job_end, grid, st); break;
        case 64: launch_np<2048, 64>(p, job_begin, job_end, grid, st); break;
        case 128: launch_np<2048, 128>(p, job_begin, job_end, grid, st); break;
        case 256: launch_np<2048, 256>(p, job_begin, job_end, grid, st); break;
        default: return hipErrorInvalidValue;
        }
    } else if (pairs == 1024) {
        switch (NP) {
        case 16: launch_np<1024, 16>(p, job_begin, job_end, grid, st); break;
        case 32: launch_np<1024, 32>(p, job_begin, job_end, grid, st); break;
        case 64: launch_np<1024, 64>(p, job_begin, job_end, grid, st); break;
        case 128: launch_np<1024, 128>(p, job_begin, job_end, grid, st); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Test hooks
// ---------------------------------------------------------------------------

// Y[j][c] = y0[c] + scale * sum_l K[j][l] F[l][c]; one workgroup per 16 columns.
__global__ __launch_bounds__(256) void pc_apply_operator_kernel(int NP, const double* kfrag, int N,
                                                                int64_t n_cols, const double* F,
                                                                const double* y0, double scale, double* Y)
{
    __shared__ double sF[PC_MAX_NP_FOR_HOOK * 16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * 16;
    for (int i = tid; i < NP * 16; i += 256) {
        const int l = i >> 4, c = i & 15;
        sF[i] = (l < N && c0 + c < n_cols) ? F[(size_t)l * n_cols + c0 + c] : 0.0;
    }
    __syncthreads();
    const int NQ = NP >> 2;
    const int64_t col = c0 + (lane & 15);
    const double y0c = col < n_cols ? y0[col] : 0.0;
    for (int strip = wave; strip < NP / 16; strip += 4) {
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        const double* kp = kfrag + (size_t)strip * NQ * 64 + lane;
        for (int q = 0; q < NQ; ++q) acc = mfma16(kp[q * 64], sF[(4 * q + (lane >> 4)) * 16 + (lane & 15)], acc);
        for (int r = 0; r < 4; ++r) {
            const int j = strip * 16 + (lane >> 4) + 4 * r;
            if (j < N && col < n_cols) Y[(size_t)j * n_cols + col] = y0c + scale * acc[r];
        }
    }
}

int pc_launch_apply_operator(int NP, const double* kfrag, int N, int64_t n_cols, const double* F,
                             const double* y0, double scale, double* Y, void* stream)
{
    if (NP > PC_MAX_NP_FOR_HOOK) return hipErrorInvalidValue;
    const int64_t grid = (n_cols + 15) / 16;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(pc_apply_operator_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       NP, kfrag, N, n_cols, F, y0, scale, Y);
    return hipGetLastError();
}

__global__ void pc_eval_force_kernel(const double* r, const double* t, int64_t n, const PcBodyDev* bodies,
                                     int P, double epoch, double mu_sun, double* a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 rec[PC_MAX_PERT_DEV + 1];
    double ix = 0.0, iy = 0.0, iz = 0.0;
    for (int b = 0; b < P; ++b) {
        double q[3];
        pc_body_position(bodies[b], t[i] - epoch, q);
        rec[b] = make_double4(q[0], q[1], q[2], bodies[b].mu);
        const double iq = rsqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        const double sq = bodies[b].mu * (iq * iq * iq);
        ix += sq * q[0];
        iy += sq * q[1];
        iz += sq * q[2];
    }
    rec[P] = make_double4(ix, iy, iz, 0.0);
    double ax, ay, az;
    pc_accel(r[i], r[n + i], r[2 * n + i], rec, P, mu_sun, ax, ay, az);
    a[i] = ax;
    a[n + i] = ay;
    a[2 * n + i] = az;
}

int pc_launch_eval_force(const double* r, const double* t, int64_t n, const PcBodyDev* bodies,
                         int n_pert, double epoch, double mu_sun, double* a, void* stream)
{
    if (n <= 0) return hipSuccess;
    if (n_pert > PC_MAX_PERT_DEV) return hipErrorInvalidValue;
    const int bs = 256;
    hipLaunchKernelGGL(pc_eval_force_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0,
                       (hipStream_t)stream, r, t, n, bodies, n_pert, epoch, mu_sun, a);
    return hipGetLastError();
}

__global__ void pc_eval_kepler_kernel(const double* y0, const double* dt, int64_t n, double* y, int32_t* ok)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a[6], b[6];
    for (int c = 0; c < 6; ++c) a[c] = y0[c * n + i];
    const bool good = pc_kepler(a, dt[i], b);
    for (int c = 0; c < 6; ++c) y[c * n + i] = good ? b[c] : a[c];
    ok[i] = good ? 1 : 0;
}

int pc_launch_eval_kepler(const double* y0, const double* dt, int64_t n, double* y, int32_t* ok, void* stream)
{
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(pc_eval_kepler_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0,
                       (hipStream_t)stream, y0, dt, n, y, ok);
    return hipGetLastError();
}
