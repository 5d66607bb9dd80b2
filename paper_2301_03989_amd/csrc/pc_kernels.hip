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
#include "pc_device.h"

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
    const double Ts = G.t0 + G.h * (s + G.s0), Te = G.t0 + G.h * (s + G.s0 + 1);
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
    if (p.recs_eih) {
        // relativistic model: states, accelerations and potentials of the major bodies
        // (pc_eih_rec slots, slot-major within the segment); body 0, the central body,
        // rests at the origin
        const int N = G.N;
        double4* base = reinterpret_cast<double4*>(p.recs_eih) + (i - j) * pc_eih_rec(P) + j;
        auto er = [&](int slot) -> double4& { return base[(size_t)slot * N]; };
        double rb[PC_MAX_PERT_DEV][3], vb[PC_MAX_PERT_DEV][3];
        for (int b = 0; b < P; ++b) pc_body_state(p.bodies[b], t - p.epoch, rb[b], vb[b]);
        double u0 = 0.0;
        for (int b = 0; b < P; ++b) {
            const double q = sqrt(rb[b][0] * rb[b][0] + rb[b][1] * rb[b][1] + rb[b][2] * rb[b][2]);
            u0 += p.bodies[b].mu / q;
            double u = p.mu_sun / q;   // potential of the central body and the other perturbers
            for (int k = 0; k < P; ++k) {
                if (k == b) continue;
                const double dx = rb[b][0] - rb[k][0], dy = rb[b][1] - rb[k][1], dz = rb[b][2] - rb[k][2];
                u += p.bodies[k].mu / sqrt(dx * dx + dy * dy + dz * dz);
            }
            const double iq3 = 1.0 / (q * q * q);   // Keplerian orbit about the central body
            const double vb2 = vb[b][0] * vb[b][0] + vb[b][1] * vb[b][1] + vb[b][2] * vb[b][2];
            er(3 * (b + 1)) = make_double4(rb[b][0], rb[b][1], rb[b][2], u - 2.0 * vb2);
            er(3 * (b + 1) + 1) = make_double4(vb[b][0], vb[b][1], vb[b][2], p.bodies[b].mu);
            er(3 * (b + 1) + 2) = make_double4(-rb[b][0] * iq3, -rb[b][1] * iq3, -rb[b][2] * iq3, 0.0);
        }
        er(0) = make_double4(0.0, 0.0, 0.0, u0);
        er(1) = make_double4(0.0, 0.0, 0.0, p.mu_sun);
        er(2) = make_double4(0.0, 0.0, 0.0, 0.0);
        er(3 * (P + 1)) = make_double4(ix, iy, iz, 0.0);
    }
}

int pc_launch_ephem(const PcEphemParams& p, void* stream)
{
    if (p.n_recs <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t grid = (p.n_recs + bs - 1) / bs;
    hipLaunchKernelGGL(pc_ephem_kernel, dim3((unsigned)grid), dim3(bs), 0, (hipStream_t)stream, p);
    return hipGetLastError();
}

// Copies of contiguous runs of 32-bit words, one workgroup per descriptor.
__global__ __launch_bounds__(64) void pc_copy_runs_kernel(const PcCopyDev* __restrict__ list)
{
    const PcCopyDev c = list[blockIdx.x];
    const uint32_t* src = static_cast<const uint32_t*>(c.src);
    uint32_t* dst = static_cast<uint32_t*>(c.dst);
    for (int64_t i = threadIdx.x; i < c.words; i += blockDim.x) dst[i] = src[i];
}

// Flyby screen (the outer-level isolation of flyby sub-groups, Sec. 3.2): one thread per
// (IC, sample point); the thread propagates its IC by two-body motion (mu = 1, the warm
// start's) to its sample point of every segment, t = w2 tau_k + w1 (eq. chnodes1 with
// `samples` CGL points), and keeps the smallest distance to any perturber in units of
// its Hill radius a_p (mu_p/3)^(1/3); the IC's minimum over its threads is taken with an
// atomic minimum on the bit patterns (positive doubles order as unsigned integers).  An
// orbit that is not elliptic gives 0.  ratio must hold +inf for the screened ICs.
__global__ __launch_bounds__(256) void pc_flyby_kernel(PcFlybyParams p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_threads) return;
    int lo = 0, hi = p.n_groups - 1;             // last group with thread_offset <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.groups[mid].thread_offset <= i) lo = mid; else hi = mid - 1;
    }
    const PcGroupDev& G = p.groups[lo];
    const int64_t local = i - G.thread_offset;
    const int64_t m = G.ic_offset + local / p.samples;
    const int k = (int)(local % p.samples);
    const double tau = -cos(M_PI * (double)k / (double)(p.samples - 1));
    double y0[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) y0[c] = p.ics[m * 6 + c];
    double best = INFINITY;
    for (int s = 0; s < G.S && best > 0.0; ++s) {
        const double Ts = G.t0 + G.h * s, Te = G.t0 + G.h * (s + 1);
        const double t = 0.5 * (Te - Ts) * tau + 0.5 * (Te + Ts);
        double y[6];
        if (!pc_kepler(y0, t - G.t0, y)) {
            best = 0.0;
            break;
        }
        for (int b = 0; b < p.n_pert; ++b) {
            const PcBodyDev& B = p.bodies[b];
            if (!(B.mu > 0.0)) continue;
            double r[3];
            pc_body_position(B, t - p.epoch, r);
            const double dx = y[0] - r[0], dy = y[1] - r[1], dz = y[2] - r[2];
            const double q = sqrt(dx * dx + dy * dy + dz * dz) / (B.a * cbrt(B.mu / 3.0));
            best = fmin(best, q);
        }
    }
    atomicMin(reinterpret_cast<unsigned long long*>(p.ratio + m), (unsigned long long)__double_as_longlong(best));
}

int pc_launch_flyby(const PcFlybyParams& p, void* stream)
{
    if (p.n_threads <= 0) return hipSuccess;
    const int bs = 256;
    const int64_t grid = (p.n_threads + bs - 1) / bs;
    hipLaunchKernelGGL(pc_flyby_kernel, dim3((unsigned)grid), dim3(bs), 0, (hipStream_t)stream, p);
    return hipGetLastError();
}

int pc_launch_copy_runs(const PcCopyDev* list, int64_t n, void* stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(pc_copy_runs_kernel, dim3((unsigned)n), dim3(64), 0, (hipStream_t)stream, list);
    return hipGetLastError();
}

// One job: T = PAIRS/NP ICs of one group, all segments.
//
// Ownership: every wave owns six 16x16 blocks of the iterate (node rows x component
// columns) for the whole job.  It keeps its blocks of the current iterate in registers
// (in the MFMA result layout), computes the dynamics for the (node, IC) pairs it owns
// straight from them, and publishes only the force matrix F = (v, a) to LDS, where the
// product y_new = y0 + w2 K_N F reads it as the B operand.
// The workgroup's LDS arena, one per job shape (file scope, so that the non-inlined job
// bodies below address it as LDS).
__shared__ PcSmem<2048> g_smem2048;
__shared__ PcSmem<1024> g_smem1024;
template <int PAIRS>
static __device__ __forceinline__ PcSmem<PAIRS>& pc_smem();
template <>
__device__ __forceinline__ PcSmem<2048>& pc_smem<2048>() { return g_smem2048; }
template <>
__device__ __forceinline__ PcSmem<1024>& pc_smem<1024>() { return g_smem1024; }

// Segment s's ephemeris records (perturber data per node, Sec. 5.4.1) into LDS: positions
// as [node][body][3] with the indirect term as body P, and per body mu, 3 mu / 2 and
// 15 mu / 8 (the premultiplied series coefficients of pc_mu_r3).
template <int PAIRS>
static __device__ __forceinline__ void pc_stage_records(const double4* grec, int N, int P, PcSmem<PAIRS>& sm)
{
    for (int i = threadIdx.x; i < N * (P + 1); i += PAIRS / 4) {
        const double4 q = grec[i];
        sm.Rec[3 * i + 0] = q.x;
        sm.Rec[3 * i + 1] = q.y;
        sm.Rec[3 * i + 2] = q.z;
        if (i < P) {
            sm.Mu[i] = q.w;
            sm.Mu[PC_MAX_PERT_DEV + i] = 1.5 * q.w;
            sm.Mu[2 * PC_MAX_PERT_DEV + i] = 1.875 * q.w;
        }
    }
}

// Picard iterations of one segment for the job's ICs (initial states in sm.Y0): ephemeris
// records into LDS, initial guess, then sweeps until every IC of the job has stopped.
// On return yc holds the lane's share of the final iterate.  iters_out (may be null)
// receives the iteration records.
// MIXED: the job runs the FP32 -> FP64 precision schedule (compiled apart, so that FP64-only
// jobs carry none of its registers).
template <int PAIRS, int NP, bool MIXED = false, bool EIH = false, int SO = 0>
static __device__ __forceinline__ void pc_segment_solve(const PcParams& p, const PcGroupDev& g, int n, int64_t ic0,
                                                        int s, PcSmem<PAIRS>& sm, const PcLane& L, gconst_dp kp0,
                                                        double (&yc)[6][4], gi32p iters_out, int& had_notconv,
                                                        int rec_cap = PcSmem<PAIRS>::REC)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int NT = Sh::NT, T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ;
    double* sF = sm.F;
    double* sY0 = sm.Y0;
    const int tid = threadIdx.x;
    const int N = g.N;
    const int P = p.n_pert;
    const int64_t ic = ic0 + tid;
    const bool rec_lds = N * 3 * (P + 1) <= rec_cap;
    const int istride = p.iters_stride;
    const int fixed_iters = p.fixed_iters, max_iter = p.max_iter;
    const double mu_sun = p.mu_sun;
    const double t2 = g.tol * g.tol;
    const double Ts = g.t0 + g.h * (s + g.s0), Te = g.t0 + g.h * (s + g.s0 + 1);
    const double w2 = 0.5 * (Te - Ts);

    // this segment's ephemeris records into LDS (perturber data per node, Sec. 5.4.1)
    const double4* grec = reinterpret_cast<const double4*>(p.recs) +
                          (size_t)(g.rec_offset + (int64_t)s * N) * (P + 1);
    if (rec_lds) pc_stage_records<PAIRS>(grec, N, P, sm);
    // initial guess at every (node, IC) pair: warm (Kepler) or cold start, Sec. 2.1,
    // staged through the F area as [node][comp 6][IC]
    {
        const int pm = tid % T;
        double y0[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) y0[c] = sY0[c * T + pm];
        const bool warm = p.init == 0 && !sm.Dead[pm];
        const bool hot = p.init == 2 && !sm.Dead[pm] && pm < n;   // the caller's node states
#pragma unroll 1
        for (int pr = tid; pr < PAIRS; pr += NT) {
            const int j = pr / T;
            double y[6];
            bool have = false;
            if (hot && j < N) {
                const double* gp = p.guess + (((size_t)(ic0 + pm) * p.iters_stride + s) * p.nodes_stride + j) * 6;
                bool fin = true;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    y[c] = gp[c];
                    fin = fin && isfinite(y[c]);
                }
                have = fin;
            } else if (j < N && warm) {
                have = pc_kepler(y0, w2 * (pc_gcd(g.tau)[j] + 1.0), y);
            }
            if (!have) {
#pragma unroll
                for (int c = 0; c < 6; ++c) y[c] = y0[c];
            }
            double* dst = sF + j * ROW + pc_fcol<PAIRS, NP>(j, pm);
#pragma unroll
            for (int c = 0; c < 6; ++c) dst[c * T] = y[c];
        }
    }
    __syncthreads();
    pc_load_share<PAIRS, NP, true>(static_cast<const double*>(sF), ROW, T, yc, L, N);
    if (tid < T) sm.Active[tid] = (tid < n) && !sm.Dead[tid];
    __syncthreads();   // staging read before F is rebuilt
    for (int i = tid; i < 6 * PAIRS; i += NT) sF[i] = 0.0;
    __syncthreads();
    // precision schedule (uniform per job): an FP32 phase first when asked, then FP64
    // sweeps.  Sweep kinds: 0 FP64 Picard sweep, 1 FP32 Picard sweep (jobs whose records do
    // not fit in LDS), 2 FP32 increment sweep (after one FP64 sweep; records in LDS).
    // An increment sweep adds w2 K_N dF to the FP64 iterate, dF the change of F to first
    // order in the last change of the iterate, (dv, G dr), with G the gravity gradient at
    // the iterate of the last FP64 sweep (the anchor); dF and the product are FP32, and no
    // force is evaluated.  From an anchor these sweeps converge, at the Picard rate, to the
    // Newton step from it (error quadratic in the anchor's); the FP32 rounding they add is
    // relative to the increments.  Increment jobs run in stages: FP64 sweeps until no IC
    // changes by more than 1e-3 (-1; one sweep after a warm start); increments to the
    // switch threshold (0); one FP64 sweep (1) that re-anchors the iterate on y0 + w2 K_N F(Y),
    // dropping the rounding and the linearisation error of stage 0; increments again (2),
    // from the closer anchor, until no IC changes by more than tol; then FP64 sweeps (3),
    // the only ones the stopping rule is applied to, so that every IC stops on an FP64
    // sweep that changed it by less than tol (one sweep for most ICs; more where the
    // linearisation left more, as near close approaches, or where stage 2 hit its cap).
    const bool incr = rec_lds;
    // increment jobs open with FP64 sweeps until no IC changes by more than 1e-3 (stage
    // -1): the linearisation needs an anchor near the solution, which a warm start gives
    // after one sweep and a cold start after several
    bool fp32 = MIXED && !incr;
    int mode = fp32 ? 1 : 0;
    // default switch: the first increment stage hands over at a relative change of 1e-6
    // (on the 262144-IC N-body workload 1e-5, 1e-6 and 1e-7 took 96.5, 95.5 and 97.7 ms;
    // a later switch lengthens stage 0, an earlier one leaves a farther anchor for stage 2);
    // FP32 Picard sweeps stall near 1e-7
    const double sw2 = p.switch2 > 0.0 ? p.switch2 : (incr ? 1e-12 : 1e-8);
    PcTol tl = pc_tol(p.tol_mode, t2, (MIXED && incr) ? 1e-6 : sw2);
    int n32 = 0;
    int stage = (MIXED && incr) ? -1 : 0;
    float* sD = reinterpret_cast<float*>(sF);                // increment sweeps: dF, FP32
    float* sG = reinterpret_cast<float*>(sF + 3 * PAIRS);    // increment sweeps: G at the anchor
    int act[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) act[r] = sm.Active[pc_ic(L, r)];
    // relativistic model: the segment's records of the major bodies
    const double4* erec = nullptr;
    if constexpr (EIH)
        erec = reinterpret_cast<const double4*>(p.recs_eih) + (size_t)(g.rec_offset + (int64_t)s * N) * pc_eih_rec(P);
    if (act[0] | act[1] | act[2] | act[3]) {
        if constexpr (EIH) pc_publish_eih<PAIRS, NP>(sF, yc, L, N, P, erec, p.inv_c2);
        else if (MIXED && mode == 1) pc_publish<PAIRS, NP, MIXED>(sF, yc, L, N, P, mu_sun, rec_lds, sm.Rec, sm.Mu, grec);
        else pc_publish<PAIRS, NP, false, SO == 0>(sF, yc, L, N, P, mu_sun, rec_lds, sm.Rec, sm.Mu, grec);
    }
    __syncthreads();

    // FP32 fragments: natural order for the transposed WIDE product, row-permuted otherwise
    gconst_fp kp0f = (gconst_fp)(Sh::WIDE ? g.kfrag32 : g.kfrag32p) + (size_t)L.strip0 * NQ * 64 + L.lane;
    const int n_it = fixed_iters > 0 ? fixed_iters : max_iter;
    double kpre[8];
    pc_kpre_load<PAIRS, NP>(kp0, kpre);
    // second-order sweeps: the K2_N strip and its first fragments next to K_N's, and the
    // lane's node offset tau_j + 1 for the x0 + w2 v0 (tau_j + 1) term
    gconst_dp kp2 = nullptr;
    double tp[8] = {};
    if constexpr (SO) {
        kp2 = (gconst_dp)g.kfrag2 + (size_t)L.strip0 * NQ * 64 + L.lane;
        if constexpr (Sh::WIDE) {
#pragma unroll
            for (int u = 0; u < 4; ++u) kpre[4 + u] = kp2[u * 64];
            tp[0] = pc_gcd(g.tau)[pc_node(L, 0, 0)] + 1.0;
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int r = 0; r < 4; ++r) tp[4 * h + r] = pc_gcd(g.tau)[pc_node(L, h, r)] + 1.0;
            }
        }
    }
    for (int it = 1; it <= n_it; ++it) {
        // (1)-(2) product and stopping-rule flags
        f64x4 acc[6];
        int flag;
        if constexpr (MIXED && Sh::WIDE) {
            if (mode == 2)
                flag = pc_product_incr<PAIRS, NP>(sD, kp0f, yc, acc, w2, tl, N, L);
            else
                flag = pc_product<PAIRS, NP, false>(sF, sY0, kp0, kpre, kp0f, yc, acc, w2, tl, N, L);
        } else if constexpr (MIXED) {
            if (mode == 2)
                flag = pc_product_incr<PAIRS, NP>(sD, kp0f, yc, acc, w2, tl, N, L);
            else
                flag = mode == 1 ? pc_product<PAIRS, NP, true>(sF, sY0, kp0, kpre, kp0f, yc, acc, w2, tl, N, L)
                                 : pc_product<PAIRS, NP, false>(sF, sY0, kp0, kpre, kp0f, yc, acc, w2, tl, N, L);
        } else if constexpr (SO == 2) {
            flag = pc_product2_fb<PAIRS, NP>(sF, sY0, kp0, kp2, kpre, yc, acc, w2, tp, tl, N, L, P, mu_sun,
                                             rec_lds, sm.Rec, sm.Mu, grec);
        } else if constexpr (SO) {
            flag = pc_product2<PAIRS, NP>(sF, sY0, kp0, kp2, kpre, yc, acc, w2, tp, tl, N, L);
        } else {
            flag = pc_product<PAIRS, NP, false, false>(sF, sY0, kp0, kpre, kp0f, yc, acc, w2, tl, N, L);
        }
        if (L.lane < 16) sm.Flag[L.wave * 16 + L.lane] = flag;
#pragma unroll
        for (int r = 0; r < 4; ++r) act[r] = sm.Active[pc_ic(L, r)];
        if constexpr (MIXED) {
            const unsigned long long keep =
                __ballot(L.lane < 16 && sm.Active[pc_flag_ic<PAIRS, NP>(L)] && (flag & 4));
            if (L.lane == 0) sm.Keep[L.wave] = keep != 0ull;
        }
        __syncthreads();   // every wave is done reading F; flags complete

        // the job leaves FP32 once no iterating IC changes by more than the switch threshold
        const bool stops = !fp32;   // stopping rule applies
        bool next32 = false;
        if (fp32) {
            int k = 0;
            for (int w = 0; w < Sh::W; ++w) k |= sm.Keep[w];
            ++n32;
            next32 = k && n32 < p.max_fp32;
            if (MIXED && incr && !next32) stage = stage == 0 ? 1 : 3;
        } else if (MIXED && incr && stage == -1) {
            // FP64 sweeps until the anchor is close enough, then increments (stage 0)
            int k = 0;
            for (int w = 0; w < Sh::W; ++w) k |= sm.Keep[w];
            if (!k) {
                stage = 0;
                next32 = true;
                n32 = 0;
                tl = pc_tol(p.tol_mode, t2, sw2);
            }
        } else if (MIXED && incr && stage == 1) {
            // the re-anchoring sweep ran: increments again until no change exceeds tol
            stage = 2;
            next32 = true;
            n32 = 0;
            tl.sa = tl.ta;
            tl.sb = tl.tb;
        }
        // (3) stopping rule per IC (Sec. 2.2; per-block error of Sec. 3.2 with blocks of one IC);
        //     applied to FP64 sweeps only
        if (tid < T && sm.Active[tid]) {
            const int f = pc_gather_flags<PAIRS, NP>(sm.Flag, tid);
            int rec = 0;
            if (f & 2) rec = -2;
            else if (fixed_iters > 0) rec = (it == fixed_iters) ? it : 0;
            else if (stops && !(f & 1)) rec = it;
            else if (it == max_iter) rec = -1;
            if (rec != 0) {
                sm.Active[tid] = 0;
                if (rec == -2) sm.Dead[tid] = 1;
                if (rec == -1) had_notconv = 1;
                if (tid < n && iters_out) iters_out[(size_t)ic * istride + s] = rec;
            }
        }
        pc_note_active<PAIRS, NP>(sm, L);
        const int next_mode = next32 ? (incr ? 2 : 1) : 0;
        // (4) ICs that were iterating take the new iterate and publish its F (or, before an
        //     increment sweep, the change of F)
        if constexpr (MIXED) {
            if (next_mode == 2 && it < n_it) {
                float dy[6][4];
#pragma unroll
                for (int b = 0; b < 6; ++b) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        dy[b][r] = act[r] ? (float)(acc[b][r] - yc[b][r]) : 0.0f;
                        yc[b][r] = act[r] ? acc[b][r] : yc[b][r];
                    }
                }
                // after an FP64 sweep the new iterate is the anchor: G evaluated there
                pc_publish_chord<PAIRS, NP>(sD, sG, yc, dy, act, mode != 2, L, N, P, mu_sun, sm.Rec, sm.Mu);
                fp32 = next32;
                mode = next_mode;
                __syncthreads();   // F complete; the active notes visible
                if (!pc_any_active<PAIRS, NP>(sm)) break;
                continue;
            }
        }
        if constexpr (MIXED) {
            // back to FP64 after increment sweeps: the FP32 arrays left arbitrary bits in the
            // rows past N of the FP64 view, which meet zero operator columns; clear them
            if (mode == 2 && N < NP) {
                for (int i = N * ROW + tid; i < NP * ROW; i += NT) sF[i] = 0.0;
            }
        }
        if (act[0] | act[1] | act[2] | act[3]) {
#pragma unroll
            for (int b = 0; b < 6; ++b) {
#pragma unroll
                for (int r = 0; r < 4; ++r) yc[b][r] = act[r] ? acc[b][r] : yc[b][r];
            }
            if (it < n_it) {
                if constexpr (EIH) pc_publish_eih<PAIRS, NP>(sF, yc, L, N, P, erec, p.inv_c2);
                else if (MIXED && next_mode == 1)
                    pc_publish<PAIRS, NP, MIXED>(sF, yc, L, N, P, mu_sun, rec_lds, sm.Rec, sm.Mu, grec);
                else pc_publish<PAIRS, NP, false, SO == 0>(sF, yc, L, N, P, mu_sun, rec_lds, sm.Rec, sm.Mu, grec);
            }
        }
        fp32 = next32;
        mode = next_mode;
        __syncthreads();   // F complete; the active notes visible
        if (!pc_any_active<PAIRS, NP>(sm)) break;
    }
}

// Not inlined: one register allocation per node count, so the work-queue kernel that
// dispatches to all of them does not pay for the largest one everywhere.
template <int PAIRS, int NP, bool MIXED, bool EIH = false, int SO = 0>
__device__ __attribute__((noinline)) void pc_job(const PcParams& p, const PcJobDev& job, const PcGroupDev& g)
{
    PcSmem<PAIRS>& sm = pc_smem<PAIRS>();
    using Sh = PcShape<PAIRS, NP>;
    constexpr int T = Sh::T, NQ = Sh::NQ;

    double* sY0 = sm.Y0;
    const int tid = threadIdx.x;
    const PcLane L = pc_lane_geometry<PAIRS, NP>(tid, g.N);
    const int N = g.N, S = g.S;
    const int n = job.n;
    const int64_t ic = job.ic0 + tid;      // this thread's IC when tid < n
    // the buffers of the call, read once from the parameter block as global pointers
    const gdp g_bounds = pc_gd(p.bounds_out);
    const gdp g_nodes = pc_gd(p.nodes_out);
    const gi32p g_iters = pc_gi(p.iters_out);
    const int istride = p.iters_stride, nstride = p.nodes_stride;

    if (tid < T) {
        const gconst_dp y = pc_gcd(p.ics) + (job.ic0 + (tid < n ? tid : 0)) * 6;
        bool fin = true;
        for (int c = 0; c < 6; ++c) {
            const double v = y[c];
            sY0[c * T + tid] = v;
            fin = fin && isfinite(v);
        }
        sm.Dead[tid] = !fin;
    }
    gconst_dp kp0 = (gconst_dp)g.kfrag + (size_t)L.strip0 * NQ * 64 + L.lane;
    __syncthreads();

    double yc[6][4];       // the lane's share of the current iterate
    int had_notconv = 0;
    for (int s = 0; s < S; ++s) {
        if (tid < n) {
            if (g_bounds) {
                const gdp bo = g_bounds + ((size_t)ic * (istride + 1) + s) * 6;
                for (int c = 0; c < 6; ++c) bo[c] = sY0[c * T + tid];
            }
            if (sm.Dead[tid] && g_iters) g_iters[(size_t)ic * istride + s] = -2;
        }
        pc_segment_solve<PAIRS, NP, MIXED, EIH, SO>(p, g, n, job.ic0, s, sm, L, kp0, yc, g_iters, had_notconv);

        // converged node states of the segment (optional output), chaining (Sec. 2.2)
#pragma unroll
        for (int h = 0; h < Sh::H; ++h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = pc_node(L, h, r);
                const int m = pc_ic(L, r);
                const bool dead = sm.Dead[m];
                if (j >= N) continue;
                if (g_nodes && m < n) {
                    const gdp o = g_nodes + (((size_t)(job.ic0 + m) * istride + s) * nstride + j) * 6;
                    if constexpr (Sh::WIDE) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) o[c] = yc[c][r];
                    } else {
#pragma unroll
                        for (int cb = 0; cb < 3; ++cb) o[2 * cb + L.hi] = yc[3 * h + cb][r];
                    }
                }
                if (j == N - 1) {
                    if constexpr (Sh::WIDE) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) sY0[c * T + m] = dead ? (double)NAN : yc[c][r];
                    } else {
#pragma unroll
                        for (int cb = 0; cb < 3; ++cb)
                            sY0[(2 * cb + L.hi) * T + m] = dead ? (double)NAN : yc[3 * h + cb][r];
                    }
                }
            }
        }
        __syncthreads();
    }

    if (tid < n) {
        const gdp so = pc_gd(p.states_out) + (size_t)ic * 6;
        for (int c = 0; c < 6; ++c) so[c] = sY0[c * T + tid];
        if (g_bounds) {
            const gdp bo = g_bounds + ((size_t)ic * (istride + 1) + S) * 6;
            for (int c = 0; c < 6; ++c) bo[c] = sY0[c * T + tid];
        }
        if (had_notconv) atomicAdd(&p.counters[0], 1);
        if (sm.Dead[tid]) atomicAdd(&p.counters[1], 1);
    }
    __syncthreads();
}

// A job with more ICs than columns (n > T), FP64 sweeps.  Every column of the product is
// an independent fixed-point iteration (the product never mixes columns), so when an IC
// stops, its end state is stored and its column takes the next IC of the job for the same
// segment: the columns do not idle while a slower IC of the same block still iterates,
// only the tail of each segment does.  The job's ICs are dealt to its column groups (entry
// e to group e % GN); every wave of a group takes the same decisions from the same flags,
// so the two barriers per sweep stay the only ones.  Each IC's sequence of iterates is the
// one the one-block job body computes.  Between segments an IC's state lives in
// states_out (the end state of its last completed segment).
// SO = 1: second-order sweeps (pc_product2) instead of the first-order product.
template <int PAIRS, int NP, int SO = 0>
__device__ __attribute__((noinline)) void pc_job_list(const PcParams& p, const PcJobDev& job, const PcGroupDev& g)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int NT = Sh::NT, T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ;
    constexpr int COLS = Sh::WIDE ? 16 : 8;      // columns of one group
    constexpr int GN = Sh::WIDE ? Sh::G16 : 1;   // groups of the job
    constexpr int E = Sh::WIDE ? 4 : 1;          // columns a lane holds points of
    constexpr unsigned CMASK = (1u << COLS) - 1u;
    PcSmem<PAIRS>& sm = pc_smem<PAIRS>();
    double* sF = sm.F;
    double* sY0 = sm.Y0;
    const int tid = threadIdx.x;
    const PcLane L = pc_lane_geometry<PAIRS, NP>(tid, g.N);
    const int N = g.N, S = g.S, P = p.n_pert;
    const int n = job.n;
    const int grp = Sh::WIDE ? L.grp : 0;
    const int n_g = n > grp ? (n - grp + GN - 1) / GN : 0;   // entries of this wave's group
    const bool rec_lds = N * 3 * (P + 1) <= PcSmem<PAIRS>::REC;
    const PcTol tl = pc_tol(p.tol_mode, g.tol * g.tol, 0.0);
    gconst_dp kp0 = (gconst_dp)g.kfrag + (size_t)L.strip0 * NQ * 64 + L.lane;
    double kpre[8];
    pc_kpre_load<PAIRS, NP>(kp0, kpre);
    // second-order sweeps: the K2_N strip next to K_N's and the nodes' tau + 1
    gconst_dp kp2 = nullptr;
    double tp[8] = {};
    if constexpr (SO) {
        kp2 = (gconst_dp)g.kfrag2 + (size_t)L.strip0 * NQ * 64 + L.lane;
        if constexpr (Sh::WIDE) {
#pragma unroll
            for (int u = 0; u < 4; ++u) kpre[4 + u] = kp2[u * 64];
            tp[0] = pc_gcd(g.tau)[pc_node(L, 0, 0)] + 1.0;
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int r = 0; r < 4; ++r) tp[4 * h + r] = pc_gcd(g.tau)[pc_node(L, h, r)] + 1.0;
            }
        }
    }
    const bool flane = L.lane < COLS;             // lanes < COLS carry the per-column decisions
    const int fcol = L.lane & (COLS - 1);
    const bool owner = flane && L.strip0 == 0;    // one wave per group writes per-IC records
    auto ic_of = [&](int e) -> int64_t { return job.ic0 + grp + (int64_t)GN * e; };
    auto col_of = [&](int e) -> int { return Sh::WIDE ? pc_ic(L, e) - grp * 16 : (L.lane & 7); };
    int notconv = 0;
    // the buffers of the call, read once from the parameter block as global pointers
    const gconst_dp g_ics = pc_gcd(p.ics);
    const gdp g_states = pc_gd(p.states_out);
    const gdp g_bounds = pc_gd(p.bounds_out);
    const gdp g_nodes = pc_gd(p.nodes_out);
    const gi32p g_iters = pc_gi(p.iters_out);
    const int istride = p.iters_stride, nstride = p.nodes_stride;
    const int fixed_iters = p.fixed_iters, max_iter = p.max_iter;
    const double mu_sun = p.mu_sun;

    double yc[6][4];
    for (int s = 0; s < S; ++s) {
        const double Ts = g.t0 + g.h * (s + g.s0), Te = g.t0 + g.h * (s + g.s0 + 1);
        const double w2 = 0.5 * (Te - Ts);
        const gconst_dp src = s == 0 ? g_ics : g_states;
        const double4* grec = reinterpret_cast<const double4*>(p.recs) +
                              (size_t)(g.rec_offset + (int64_t)s * N) * (P + 1);
        // Warm (or cold) start, Sec. 2.1, of the group's columns in `rm`, column c taking entry
        // base + (its rank in rm).  The wave computes the points of its own node rows for
        // all those columns together (one Kepler solve per lane and pass), stages them in
        // the columns' F slots (free after the product), and the lanes that hold the points
        // read them back.
        auto warm_columns = [&](unsigned rm, int base) {
            constexpr int WN = 16 * Sh::H;               // node rows of this wave
            const int k = __popc(rm);
            for (int q = L.lane; q < WN * k; q += 64) {
                const int ci = q / WN, jn = q - ci * WN;
                unsigned m = rm;
                for (int t = 0; t < ci; ++t) m &= m - 1u;
                const int c = __ffs(m) - 1;
                const int j = L.strip0 * 16 + jn;
                if (j >= N) continue;
                const gconst_dp y0p = src + ic_of(base + ci) * 6;
                double y0[6];
                bool fin = true;
#pragma unroll
                for (int cc = 0; cc < 6; ++cc) {
                    y0[cc] = y0p[cc];
                    fin = fin && isfinite(y0[cc]);
                }
                double y[6];
                if (!(p.init == 0 && fin && pc_kepler(y0, w2 * (pc_gcd(g.tau)[j] + 1.0), y))) {
#pragma unroll
                    for (int cc = 0; cc < 6; ++cc) y[cc] = y0[cc];
                }
                double* f = sF + j * ROW + pc_fcol<PAIRS, NP>(j, grp * 16 + c);
#pragma unroll
                for (int cc = 0; cc < 6; ++cc) f[cc * T] = y[cc];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // staged points visible to the wave
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (!((rm >> col_of(e)) & 1u)) continue;
#pragma unroll
                for (int h = 0; h < Sh::H; ++h) {
#pragma unroll
                    for (int r = 0; r < (Sh::WIDE ? 1 : 4); ++r) {
                        const int j = pc_node(L, h, r);
                        if (j >= N) continue;
                        double* f = sF + j * ROW + pc_fcol<PAIRS, NP>(j, Sh::WIDE ? pc_ic(L, e) : (L.lane & 7));
                        // second-order sweeps keep F's velocity columns at zero: the lane
                        // that reads a staged velocity clears it
                        if constexpr (Sh::WIDE) {
#pragma unroll
                            for (int cc = 0; cc < 6; ++cc) {
                                yc[cc][e] = f[cc * T];
                                if (SO && cc < 3) f[cc * T] = 0.0;
                            }
                        } else {
#pragma unroll
                            for (int cb = 0; cb < 3; ++cb) {
                                yc[3 * h + cb][r] = f[(2 * cb + L.hi) * T];
                                if (SO && 2 * cb + L.hi < 3) f[(2 * cb + L.hi) * T] = 0.0;
                            }
                        }
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");   // read before the slots are rewritten
        };
        // the owner lane of a column writes its IC's y0 (product epilogue) and checkpoint
        auto own_column = [&](int en) {
            const int64_t icg = ic_of(en);
            const gconst_dp y0p = src + icg * 6;
            double v[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) v[c] = y0p[c];
#pragma unroll
            for (int c = 0; c < 6; ++c) sY0[c * T + grp * 16 + fcol] = v[c];
            if (g_bounds) {
                const gdp bo = g_bounds + ((size_t)icg * (istride + 1) + s) * 6;
#pragma unroll
                for (int c = 0; c < 6; ++c) bo[c] = v[c];
            }
        };

        if (rec_lds) pc_stage_records<PAIRS>(grec, N, P, sm);
        for (int i = tid; i < 6 * PAIRS; i += NT) sF[i] = 0.0;   // rows past N stay zero
        __syncthreads();   // records staged, F cleared
        // the group's first COLS entries into its columns
        int next = n_g < COLS ? n_g : COLS;                                   // uniform per group
        unsigned amask = next >= COLS ? CMASK : ((1u << next) - 1u);          // uniform per group
        int ent[E];
#pragma unroll
        for (int e = 0; e < E; ++e) ent[e] = col_of(e) < next ? col_of(e) : -1;
        warm_columns(amask, 0);
        int fent = fcol < next ? fcol : -1;   // flag lane: entry of its column
        int it0 = 0;                          // flag lane: sweep before its IC's first one
        if (owner && fent >= 0) own_column(fent);
        __syncthreads();   // y0 written
        if (amask) pc_publish<PAIRS, NP, false, SO == 0>(sF, yc, L, N, P, mu_sun, rec_lds, sm.Rec, sm.Mu, grec);
        __syncthreads();

        for (int it = 1;; ++it) {
            f64x4 acc[6];
            int flag;
            if constexpr (SO) flag = pc_product2<PAIRS, NP>(sF, sY0, kp0, kp2, kpre, yc, acc, w2, tp, tl, N, L);
            else flag = pc_product<PAIRS, NP, false, false>(sF, sY0, kp0, kpre, nullptr, yc, acc, w2, tl, N, L);
            if (L.lane < 16) sm.Flag[L.wave * 16 + L.lane] = flag;
            __syncthreads();   // every wave is done reading F; flags complete

            // stopping rule per IC (Sec. 2.2), taken identically by every wave of the group
            int rec = 0;
            if (flane && fent >= 0) {
                const int f = pc_gather_flags<PAIRS, NP>(sm.Flag, grp * 16 + fcol);
                const int k = it - it0;
                if (f & 2) rec = -2;
                else if (fixed_iters > 0) rec = (k == fixed_iters) ? k : 0;
                else if (!(f & 1)) rec = k;
                else if (k >= max_iter) rec = -1;
            }
            const unsigned smask = (unsigned)__ballot(rec != 0) & CMASK;
            const unsigned dmask = (unsigned)__ballot(rec == -2) & CMASK;
            if (owner && rec != 0) {
                if (g_iters) g_iters[(size_t)ic_of(fent) * istride + s] = rec;
                if (rec == -1) ++notconv;
            }
            // the columns that were iterating take the new iterate
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const bool act = (amask >> col_of(e)) & 1u;
#pragma unroll
                for (int b = 0; b < 6; ++b) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (Sh::WIDE ? r == e : true) yc[b][r] = act ? acc[b][r] : yc[b][r];
                    }
                }
            }
            if (smask) {
                // outputs of the ICs that stopped: node states, end state (node N-1, NaN when
                // non-finite) as the next segment's y0 and the checkpoint
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int c = col_of(e);
                    if (!((smask >> c) & 1u)) continue;
                    const int64_t icg = ic_of(ent[e]);
                    const bool dead = (dmask >> c) & 1u;
#pragma unroll
                    for (int h = 0; h < Sh::H; ++h) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            if (Sh::WIDE && r != e) continue;
                            const int j = Sh::WIDE ? pc_node(L, 0, 0) : pc_node(L, h, r);
                            if (j >= N) continue;
                            if (g_nodes) {
                                const gdp nd = g_nodes + (((size_t)icg * istride + s) * nstride + j) * 6;
                                if constexpr (Sh::WIDE) {
#pragma unroll
                                    for (int cc = 0; cc < 6; ++cc) nd[cc] = yc[cc][e];
                                } else {
#pragma unroll
                                    for (int cb = 0; cb < 3; ++cb) nd[2 * cb + L.hi] = yc[3 * h + cb][r];
                                }
                            }
                            if (j == N - 1) {
                                const gdp so = g_states + icg * 6;
                                const gdp bo = g_bounds ? g_bounds + ((size_t)icg * (istride + 1) + s + 1) * 6 : g_bounds;
                                if constexpr (Sh::WIDE) {
#pragma unroll
                                    for (int cc = 0; cc < 6; ++cc) {
                                        const double v = dead ? (double)NAN : yc[cc][e];
                                        so[cc] = v;
                                        if (bo) bo[cc] = v;
                                    }
                                } else {
#pragma unroll
                                    for (int cb = 0; cb < 3; ++cb) {
                                        const int cc = 2 * cb + L.hi;
                                        const double v = dead ? (double)NAN : yc[3 * h + cb][r];
                                        so[cc] = v;
                                        if (bo) bo[cc] = v;
                                    }
                                }
                            }
                        }
                    }
                }
                // refill: the stopped columns, in column order, take the group's next entries
                const int take = min(__popc(smask), n_g - next);
                unsigned rmask = 0u;
                {
                    unsigned m = smask;
                    for (int k = 0; k < take; ++k) {
                        rmask |= m & (0u - m);   // lowest stopped column
                        m &= m - 1u;
                    }
                }
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int c = col_of(e);
                    if ((rmask >> c) & 1u) ent[e] = next + __popc(rmask & ((1u << c) - 1u));
                    else if ((smask >> c) & 1u) ent[e] = -1;
                }
                if (rmask) warm_columns(rmask, next);
                if (flane) {
                    if ((rmask >> fcol) & 1u) {
                        fent = next + __popc(rmask & ((1u << fcol) - 1u));
                        it0 = it;
                        if (owner) own_column(fent);
                    } else if ((smask >> fcol) & 1u) {
                        fent = -1;
                    }
                }
                next += take;
                amask = (amask & ~smask) | rmask;
            }
            if (amask) pc_publish<PAIRS, NP, false, SO == 0>(sF, yc, L, N, P, mu_sun, rec_lds, sm.Rec, sm.Mu, grec);
            // every wave of an IC group holds the group's column mask: the first strip's waves
            // note it (rewritten only after the next sweep's first barrier)
            if (L.strip0 == 0 && L.lane == 0) sm.Go[L.grp] = amask != 0u;
            __syncthreads();   // F complete; the notes visible
            int go = 0;
#pragma unroll
            for (int q = 0; q < Sh::G16; ++q) go |= sm.Go[q];
            if (!go) break;
        }
    }
    if (notconv) atomicAdd(&p.counters[0], notconv);
    __syncthreads();   // every end state written
    for (int e = tid; e < n; e += NT) {
        const gconst_dp y = g_states + (job.ic0 + e) * 6;
        bool fin = true;
        for (int c = 0; c < 6; ++c) fin = fin && isfinite(y[c]);
        if (!fin) atomicAdd(&p.counters[1], 1);
    }
    __syncthreads();
}

// The job body for node count NP and the call's options: second-order sweeps (with the
// feedback on WIDE shapes), relativistic, refilled column lists, precision schedule or
// plain FP64 one-block jobs.
template <int PAIRS, int NP>
static __device__ __forceinline__ void pc_run_job(const PcParams& p, const PcJobDev& job, const PcGroupDev& g,
                                                  bool list, bool mixed, bool eih, bool order2)
{
    if (order2) {
        if (p.feedback) {
            pc_job<PAIRS, NP, false, false, 2>(p, job, g);
            return;
        }
        if (list) pc_job_list<PAIRS, NP, 1>(p, job, g);
        else pc_job<PAIRS, NP, false, false, 1>(p, job, g);
    } else if (eih && mixed) {
        pc_job<PAIRS, NP, true, true>(p, job, g);
    } else if (eih) {
        pc_job<PAIRS, NP, false, true>(p, job, g);
    } else if (list) {
        pc_job_list<PAIRS, NP>(p, job, g);
    } else if (mixed) {
        pc_job<PAIRS, NP, true>(p, job, g);
    } else {
        pc_job<PAIRS, NP, false>(p, job, g);
    }
}

// Persistent work-queue kernel: every workgroup takes the next job of the plan (jobs of
// all groups and node counts, longest first) until the queue is empty, so one launch
// runs an uneven two-level batch (Sec. 3.2) to completion.
// Two waves per SIMD: 512-thread workgroups fill a CU alone (their LDS arena is the
// CU's), 256-thread ones fit two workgroups, running two independent jobs, per CU.
template <int PAIRS>
__global__ __launch_bounds__(PAIRS / 4, 2) void pc_fused_kernel(const PcParams* __restrict__ pp)
{
    __shared__ int sJob;
    const PcParams& p = *pp;
    for (;;) {
        if (threadIdx.x == 0) sJob = atomicAdd(p.queue, 1);
        __syncthreads();
        const int jb = sJob;
        __syncthreads();
        if (jb >= p.n_jobs) break;
        // private copies: with them the job bodies need not preserve the caller's registers
        const PcJobDev job = p.jobs[jb];
        const PcGroupDev g = p.groups[job.group];
        const bool list = job.n > g.T;   // more ICs than columns: refilled columns (FP64 only)
        const bool mixed = p.precision == 1;
        const bool eih = p.inv_c2 != 0.0;   // relativistic model: one-block jobs
        const bool order2 = p.order == 2;   // second-order sweeps (with the integral error feedback when
                                            // asked, WIDE shapes): FP64, point masses
        switch (g.NP) {
        case 16: pc_run_job<PAIRS, 16>(p, job, g, list, mixed, eih, order2); break;
        case 32: pc_run_job<PAIRS, 32>(p, job, g, list, mixed, eih, order2); break;
        case 64: pc_run_job<PAIRS, 64>(p, job, g, list, mixed, eih, order2); break;
        case 128: pc_run_job<PAIRS, 128>(p, job, g, list, mixed, eih, order2); break;
        case 256:
            if constexpr (PAIRS >= 2048) pc_run_job<PAIRS, 256>(p, job, g, list, mixed, eih, order2);
            break;
        default: break;
        }
    }
}

int pc_fused_occupancy(int pairs, int* blocks_per_cu)
{
    if (pairs == 2048)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pc_fused_kernel<2048>, 512, 0);
    if (pairs == 1024)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pc_fused_kernel<1024>, 256, 0);
    return hipErrorInvalidValue;
}

int pc_launch_fused(const PcParams& p, const PcParams* p_dev, int pairs, int grid, void* stream)
{
    if (p.n_jobs <= 0) return hipSuccess;
    hipStream_t st = (hipStream_t)stream;
    if (grid <= 0 || grid > p.n_jobs) grid = p.n_jobs;
    if (pairs == 2048)
        hipLaunchKernelGGL(pc_fused_kernel<2048>, dim3(grid), dim3(512), 0, st, p_dev);
    else if (pairs == 1024)
        hipLaunchKernelGGL(pc_fused_kernel<1024>, dim3(grid), dim3(256), 0, st, p_dev);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint of the converged map (reverse sweep over segments)
// ---------------------------------------------------------------------------
// For a segment with converged node states Y = 1 y0^T + K G(Y), G_j = w2 f(Y_j, t_j), the
// derivative of a loss L(Y) with seed gbar = dL/dY is dL/dy0 = sum_j mu_j, where mu solves
// (I - K J)^T mu = gbar with J_j = w2 df/dy (implicit differentiation of the fixed point).
// mu is found by the adjoint fixed-point sweep mu <- gbar + J^T (K^T mu), which contracts
// like the forward Picard iteration; with f = (v, a(r)) and H = da/dr symmetric,
//   (J^T w)_r = w2 H w_v,   (J^T w)_v = w2 w_r.
// Segments are processed from the last: each is first re-solved from its checkpoint (the
// same forward code, so the same converged states), and its gradient seeds the end node of
// the previous one.  WIDE job shapes hold one node of four ICs per lane; 8-IC jobs (256
// nodes) hold the node-row layout of the forward product (a lane pair (l, l ^ 8) shares the
// components of one IC), and their lanes exchange what the Hessian product and the
// velocity rows need with their partner.
// EIH: the relativistic dynamics, whose force also depends on the velocity: J^T w is
// ((da/dr)^T w_v, w_r + (da/dv)^T w_v) (pc_eih_vjp) instead of (H w_v, w_r).
template <int PAIRS, int NP, bool EIH = false>
__device__ __attribute__((noinline)) void pc_adjoint_job(const PcAdjParams& a, const PcJobDev& job,
                                                         const PcGroupDev& g)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int NT = Sh::NT, T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ, W = Sh::W;
    PcSmem<PAIRS>& sm = pc_smem<PAIRS>();
    const PcParams& p = a.fwd;
    double* sF = sm.F;
    double* sY0 = sm.Y0;
    const int tid = threadIdx.x;
    // the products run every k step here (the bound NP folds to the compile-time count): a
    // second, shorter k loop per product costs this body registers at every node count
    const PcLane L = pc_lane_geometry<PAIRS, NP>(tid, NP);
    const int N = g.N, S = g.S, P = p.n_pert;
    const int n = job.n;
    const int64_t ic = job.ic0 + tid;
    // adjoint scratch at the top of the record area: seed Lam, estimate LamIt, partial sums
    constexpr int ADJ = 12 * T + W * 6 * 16;
    constexpr int REC_CAP = PcSmem<PAIRS>::REC - ADJ;
    double* sLam = sm.Rec + REC_CAP;
    double* sLamIt = sLam + 6 * T;
    double* sLamPart = sLamIt + 6 * T;
    const bool rec_lds = N * 3 * (P + 1) <= REC_CAP;
    const double t2a = a.adj_tol * a.adj_tol;

    if (tid < T) {
        for (int c = 0; c < 6; ++c) sLam[c * T + tid] = tid < n ? a.gbar_final[(size_t)ic * 6 + c] : 0.0;
    }
    gconst_dp kp0 = (gconst_dp)g.kfrag + (size_t)L.strip0 * NQ * 64 + L.lane;
    gconst_dp kpT = (gconst_dp)g.kfragT + (size_t)L.strip0 * NQ * 64 + L.lane;
    double yc[6][4];
    int had_notconv = 0, adj_notconv = 0, dead_any = 0;
    for (int s = S - 1; s >= 0; --s) {
        // segment s's converged iterate: the forward call's node states when given, else a
        // re-solve from its checkpoint
        if (tid < T) {
            const double* src = a.ckpt + ((size_t)(job.ic0 + (tid < n ? tid : 0)) * (a.ckpt_stride + 1) + s) * 6;
            bool fin = true;
            for (int c = 0; c < 6; ++c) {
                const double v = src[c];
                sY0[c * T + tid] = v;
                fin = fin && isfinite(v);
            }
            sm.Dead[tid] = !fin;
        }
        __syncthreads();
        const double4* grec = reinterpret_cast<const double4*>(p.recs) +
                              (size_t)(g.rec_offset + (int64_t)s * N) * (P + 1);
        const double4* erec = nullptr;
        if constexpr (EIH)
            erec = reinterpret_cast<const double4*>(p.recs_eih) + (size_t)(g.rec_offset + (int64_t)s * N) * pc_eih_rec(P);
        if (a.fwd_nodes) {
            if (!EIH && rec_lds) pc_stage_records<PAIRS>(grec, N, P, sm);
#pragma unroll
            for (int h = 0; h < Sh::H; ++h) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = pc_node(L, h, r);
                    const int m = pc_ic(L, r);
                    double v[6];
                    if (j < N && m < n) {
                        const gconst_dp y = pc_gcd(a.fwd_nodes) +
                                            (((size_t)(job.ic0 + m) * a.ckpt_stride + s) * a.nodes_stride + j) * 6;
#pragma unroll
                        for (int c = 0; c < 6; ++c) v[c] = y[c];
                    } else {   // padding node or column: any finite state (its results are unused)
#pragma unroll
                        for (int c = 0; c < 6; ++c) v[c] = sY0[c * T + m];
                    }
                    if constexpr (Sh::WIDE) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) yc[c][r] = v[c];
                    } else {
#pragma unroll
                        for (int cb = 0; cb < 3; ++cb) yc[3 * h + cb][r] = v[2 * cb + L.hi];
                    }
                }
            }
        } else {
            pc_segment_solve<PAIRS, NP, false, EIH>(p, g, n, job.ic0, s, sm, L, kp0, yc, nullptr, had_notconv,
                                                    REC_CAP);
        }
        __syncthreads();
        const double Ts = g.t0 + g.h * s, Te = g.t0 + g.h * (s + 1);
        const double w2 = 0.5 * (Te - Ts);

        // seed of this segment at the lane's nodes: the next segment's gradient at the end
        // node, plus the node seeds when given (recomputed where needed, not held)
        // the Hessian's points: WIDE, the lane's node of its four ICs; 8-IC jobs, the four
        // rows of strip hi (each lane of a pair takes one strip)
        int jr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, Sh::WIDE ? 0 : L.hi, r);
            jr[r] = j < N ? j : N - 1;
        }
        auto seed_at = [&](int c, int j, int m) -> double {
            double v = (j == N - 1) ? sLam[c * T + m] : 0.0;
            if (a.gbar_nodes && m < n && j < N)
                v += a.gbar_nodes[(((size_t)(job.ic0 + m) * a.ckpt_stride + s) * a.nodes_stride + j) * 6 + c];
            return v;
        };
        auto seed = [&](int c, int r) -> double { return seed_at(c, pc_node(L, 0, r), pc_ic(L, r)); };
        for (int i = tid; i < 6 * PAIRS; i += NT) sF[i] = 0.0;
        if (tid < T) {
            sm.Active[tid] = (tid < n) && !sm.Dead[tid];
            for (int c = 0; c < 6; ++c) sLamIt[c * T + tid] = 0.0;
        }
        __syncthreads();
        // mu^(0) = gbar
#pragma unroll
        for (int h = 0; h < Sh::H; ++h) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = pc_node(L, h, r);
                const int m = pc_ic(L, r);
                if (j < N) {
                    if constexpr (Sh::WIDE) {
#pragma unroll
                        for (int c = 0; c < 6; ++c) sF[j * ROW + c * T + pc_fcol<PAIRS, NP>(j, m)] = seed_at(c, j, m);
                    } else {
#pragma unroll
                        for (int cb = 0; cb < 3; ++cb) {
                            const int c = 2 * cb + L.hi;
                            sF[j * ROW + c * T + pc_fcol<PAIRS, NP>(j, m)] = seed_at(c, j, m);
                        }
                    }
                }
            }
        }
        __syncthreads();

        int it = 1;
        for (; it <= a.adj_max_iter; ++it) {
            f64x4 acc[6];
            pc_product_adj<PAIRS, NP>(sF, kpT, acc, L);          // w = K^T mu
            double hx[4], hy[4], hz[4];
            if constexpr (Sh::WIDE) {
                double wx[4], wy[4], wz[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    wx[r] = acc[3][r];
                    wy[r] = acc[4][r];
                    wz[r] = acc[5][r];
                }
                double gx[4] = {}, gy[4] = {}, gz[4] = {};   // (da/dv)^T w_v (relativistic)
                if constexpr (EIH)
                    pc_eih_vjp<4, true>(yc[0], yc[1], yc[2], yc[3], yc[4], yc[5], wx, wy, wz, erec, jr, N, P, p.inv_c2,
                                        hx, hy, hz, gx, gy, gz);
                else if (rec_lds)
                    pc_hess_apply<4, true>(yc[0], yc[1], yc[2], wx, wy, wz, jr, P, p.mu_sun, sm.Rec, sm.Mu, grec,
                                           hx, hy, hz);
                else
                    pc_hess_apply<4, false>(yc[0], yc[1], yc[2], wx, wy, wz, jr, P, p.mu_sun, sm.Rec, sm.Mu, grec,
                                            hx, hy, hz);
                // mu_new = gbar + J^T w, and its sum over the strip's nodes (the 16 lanes of a
                // row group hold one node each of the same four ICs)
                const bool node_ok = pc_node(L, 0, 0) < N;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double nv0 = seed(3, r) + w2 * (acc[0][r] + gx[r]);
                    const double nv1 = seed(4, r) + w2 * (acc[1][r] + gy[r]);
                    const double nv2 = seed(5, r) + w2 * (acc[2][r] + gz[r]);
                    acc[0][r] = seed(0, r) + w2 * hx[r];
                    acc[1][r] = seed(1, r) + w2 * hy[r];
                    acc[2][r] = seed(2, r) + w2 * hz[r];
                    acc[3][r] = nv0;
                    acc[4][r] = nv1;
                    acc[5][r] = nv2;
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        double part = node_ok ? acc[c][r] : 0.0;
                        part = pc_row_sum16(part);
                        if ((L.lane & 15) == 0) sLamPart[(L.wave * 6 + c) * 16 + (L.lane >> 4) + 4 * r] = part;
                    }
                }
            } else {
                // node-row layout: element (3h + cb, r) is comp 2cb + hi of node j(h, r); the
                // low lane of a pair holds comps 0, 2, 4, the high lane 1, 3, 5.  Each lane
                // forms H w_v at the four points of strip hi (position and w_v = (w3, w4, w5),
                // taking the three components it lacks from its partner)
                const int hi = L.hi;
                const int m = pc_ic(L, 0);
                double xs[4], ys[4], zs[4], wxs[4], wys[4], wzs[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double e1 = pc_dpp<0x128>(hi ? yc[0][r] : yc[3][r]);     // lo: y(0); hi: x(1)
                    const double e2 = pc_dpp<0x128>(hi ? acc[1][r] : yc[4][r]);    // lo: w3(0); hi: z(1)
                    const double e3 = pc_dpp<0x128>(hi ? acc[2][r] : acc[5][r]);   // lo: w5(0); hi: w4(1)
                    xs[r] = hi ? e1 : yc[0][r];
                    ys[r] = hi ? yc[3][r] : e1;
                    zs[r] = hi ? e2 : yc[1][r];
                    wxs[r] = hi ? acc[4][r] : e2;
                    wys[r] = hi ? e3 : acc[2][r];
                    wzs[r] = hi ? acc[5][r] : e3;
                }
                // relativistic: (da/dv)^T w_v at the same points, which also need the velocity
                // (lo: vy(0) held, vx(0) and vz(0) from hi; hi: vx(1), vz(1) held, vy(1) from lo)
                double gvx[4] = {}, gvy[4] = {}, gvz[4] = {};
                if constexpr (EIH) {
                    double vxs[4], vys[4], vzs[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double e4 = pc_dpp<0x128>(hi ? yc[1][r] : yc[5][r]);   // lo: vx(0); hi: vy(1)
                        const double e5 = pc_dpp<0x128>(yc[2][r]);                   // lo: vz(0)
                        vxs[r] = hi ? yc[4][r] : e4;
                        vys[r] = hi ? e4 : yc[2][r];
                        vzs[r] = hi ? yc[5][r] : e5;
                    }
                    pc_eih_vjp<4, false>(xs, ys, zs, vxs, vys, vzs, wxs, wys, wzs, erec, jr, N, P, p.inv_c2, hx, hy,
                                         hz, gvx, gvy, gvz);
                } else if (rec_lds) {
                    pc_hess_apply<4, true>(xs, ys, zs, wxs, wys, wzs, jr, P, p.mu_sun, sm.Rec, sm.Mu, grec, hx, hy,
                                           hz);
                } else {
                    pc_hess_apply<4, false>(xs, ys, zs, wxs, wys, wzs, jr, P, p.mu_sun, sm.Rec, sm.Mu, grec, hx, hy,
                                            hz);
                }
                // mu_new = gbar + J^T w: position rows (comp c < 3) take w2 (H w_v)_c of their
                // point, from the lane that formed it; velocity rows (comp c >= 3) take
                // w2 w_(c-3), which the partner lane holds
                double part[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double f1 = pc_dpp<0x128>(hi ? hx[r] : hy[r]);   // lo: hx(1); hi: hy(0)
                    const double f2 = pc_dpp<0x128>(hz[r]);                // lo: hz(1)
                    // relativistic velocity terms, on the lane that holds the row: comp 3
                    // (hi) gvx, comp 4 (lo) gvy, comp 5 (hi) gvz of each strip
                    double f3 = 0.0, f4 = 0.0;
                    if constexpr (EIH) {
                        f3 = pc_dpp<0x128>(hi ? gvy[r] : gvx[r]);   // lo: gvy(1); hi: gvx(0)
                        f4 = pc_dpp<0x128>(gvz[r]);                 // hi: gvz(0)
                    }
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const double g = pc_dpp<0x128>(acc[3 * h][r]);      // lo: w1(h); hi: w0(h)
                        const double k = pc_dpp<0x128>(acc[3 * h + 1][r]);  // hi: w2(h)
                        const int j = pc_node(L, h, r);
                        const double hc0 = h == 0 ? (hi ? f1 : hx[r]) : (hi ? hy[r] : f1);   // comp hi
                        const double hc2 = h == 0 ? hz[r] : f2;                              // comp 2 (lo)
                        const double gv1 = h == 0 ? f3 : gvx[r];                             // comp 3 (hi)
                        const double gv2 = hi ? (h == 0 ? f4 : gvz[r]) : (h == 0 ? gvy[r] : f3);   // comp 4 + hi
                        const double n0 = seed_at(hi, j, m) + w2 * hc0;
                        const double n1 = seed_at(2 + hi, j, m) + w2 * (hi ? g + gv1 : hc2);
                        const double n2 = seed_at(4 + hi, j, m) + w2 * ((hi ? k : g) + gv2);
                        acc[3 * h][r] = n0;
                        acc[3 * h + 1][r] = n1;
                        acc[3 * h + 2][r] = n2;
                        if (j < N) {
                            part[0] += n0;
                            part[1] += n1;
                            part[2] += n2;
                        }
                    }
                }
                // sum over the wave's 32 nodes: the four row groups of 16 lanes hold nodes
                // l / 16 + 4 r of both strips
#pragma unroll
                for (int cb = 0; cb < 3; ++cb) {
                    double v = part[cb];
                    v += __shfl_xor(v, 16);
                    v += __shfl_xor(v, 32);
                    if (L.lane < 16) sLamPart[(L.wave * 6 + 2 * cb + hi) * 16 + m] = v;
                }
            }
            int act[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) act[r] = sm.Active[pc_ic(L, r)];
            __syncthreads();   // K^T mu read by every wave; partial sums complete

            // gradient estimate lambda = sum_j mu_j per IC; stop when it no longer changes
            if (tid < T && sm.Active[tid]) {
                double ln[6], d2 = 0.0, n2 = 0.0;
                for (int c = 0; c < 6; ++c) {
                    double v = 0.0;
                    if constexpr (Sh::WIDE) {
                        for (int w = tid >> 4; w < W; w += Sh::G16) v += sLamPart[(w * 6 + c) * 16 + (tid & 15)];
                    } else {
                        for (int w = 0; w < W; ++w) v += sLamPart[(w * 6 + c) * 16 + tid];
                    }
                    ln[c] = v;
                    const double d = v - sLamIt[c * T + tid];
                    d2 += d * d;
                    n2 += v * v;
                    sLamIt[c * T + tid] = v;
                }
                int rec = 0;
                if (!isfinite(n2)) rec = -2;
                else if (it > 1 && d2 <= t2a * n2) rec = it;
                else if (it == a.adj_max_iter) rec = -1;
                if (rec != 0) {
                    sm.Active[tid] = 0;
                    if (rec == -2) sm.Dead[tid] = 1;
                    if (rec == -1) adj_notconv = 1;
                    if (tid < n && a.adj_iters) a.adj_iters[(size_t)ic * a.ckpt_stride + s] = rec;
                }
            }
            if constexpr (Sh::WIDE) {
                if (pc_node(L, 0, 0) < N) {
                    const int j = pc_node(L, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (act[r]) {
#pragma unroll
                            for (int c = 0; c < 6; ++c)
                                sF[j * ROW + c * T + pc_fcol<PAIRS, NP>(j, pc_ic(L, r))] = acc[c][r];
                        }
                    }
                }
            } else if (act[0]) {
                const int m = pc_ic(L, 0);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = pc_node(L, h, r);
                        if (j < N) {
#pragma unroll
                            for (int cb = 0; cb < 3; ++cb)
                                sF[j * ROW + (2 * cb + L.hi) * T + pc_fcol<PAIRS, NP>(j, m)] = acc[3 * h + cb][r];
                        }
                    }
                }
            }
            pc_note_active<PAIRS, NP>(sm, L);
            __syncthreads();   // mu complete; the active notes visible
            if (!pc_any_active<PAIRS, NP>(sm)) break;
        }
        // this segment's gradient seeds the end node of the previous one
        if (tid < T) {
            const bool dead = sm.Dead[tid];
            dead_any |= dead;
            for (int c = 0; c < 6; ++c) sLam[c * T + tid] = dead ? (double)NAN : sLamIt[c * T + tid];
        }
        __syncthreads();
    }
    if (tid < n) {
        for (int c = 0; c < 6; ++c) a.grad_out[(size_t)ic * 6 + c] = sLam[c * T + tid];
        if (adj_notconv || had_notconv) atomicAdd(&a.counters[0], 1);
        if (dead_any) atomicAdd(&a.counters[1], 1);
    }
    __syncthreads();
}

template <int PAIRS>
__global__ __launch_bounds__(PAIRS / 4) void pc_adjoint_kernel(const PcAdjParams* __restrict__ ap)
{
    __shared__ int sJob;
    const PcAdjParams& a = *ap;
    for (;;) {
        if (threadIdx.x == 0) sJob = atomicAdd(a.counters + 2, 1);
        __syncthreads();
        const int jb = sJob;
        __syncthreads();
        if (jb >= a.fwd.n_jobs) break;
        const PcJobDev job = a.fwd.jobs[jb];
        const PcGroupDev g = a.fwd.groups[job.group];
        const bool eih = a.fwd.inv_c2 != 0.0;
        switch (g.NP) {
        case 16: eih ? pc_adjoint_job<PAIRS, 16, true>(a, job, g) : pc_adjoint_job<PAIRS, 16>(a, job, g); break;
        case 32: eih ? pc_adjoint_job<PAIRS, 32, true>(a, job, g) : pc_adjoint_job<PAIRS, 32>(a, job, g); break;
        case 64: eih ? pc_adjoint_job<PAIRS, 64, true>(a, job, g) : pc_adjoint_job<PAIRS, 64>(a, job, g); break;
        case 128: eih ? pc_adjoint_job<PAIRS, 128, true>(a, job, g) : pc_adjoint_job<PAIRS, 128>(a, job, g); break;
        case 256: eih ? pc_adjoint_job<PAIRS, 256, true>(a, job, g) : pc_adjoint_job<PAIRS, 256>(a, job, g); break;
        default: break;
        }
    }
}

int pc_launch_adjoint(const PcAdjParams& a, const PcAdjParams* a_dev, int grid, void* stream)
{
    if (a.fwd.n_jobs <= 0) return hipSuccess;
    if (grid <= 0 || grid > a.fwd.n_jobs) grid = a.fwd.n_jobs;
    hipLaunchKernelGGL(pc_adjoint_kernel<2048>, dim3(grid), dim3(512), 0, (hipStream_t)stream, a_dev);
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
