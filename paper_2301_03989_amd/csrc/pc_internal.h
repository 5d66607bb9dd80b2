// pc_internal.h -- structures shared by the host planner and the gfx950 kernels.
//
// Layout conventions (all FP64):
//  * A "job" is one workgroup's share of one group: T consecutive ICs of the group,
//    all NP (padded) nodes, all segments.  NP * T == PAIRS, PAIRS in {1024, 2048}.
//  * Inside a workgroup the state of a job lives in LDS as [node j][comp 9][IC m]:
//    comps 0..5 = x y z vx vy vz of the current iterate, comps 6..8 = the
//    acceleration at the nodes.  Comps 3..8 are the force matrix F of Sec. 2.2
//    (velocity and acceleration), so y_new = y0 + w2 * K_N F is one product with
//    a contiguous right-hand side per node row.
//  * K_N is stored as MFMA A-operand fragments: kfrag[strip][q][lane] =
//    K_N[16*strip + lane%16][4*q + lane/16], zero-padded to NP x NP, so one wave
//    reads a 16x4 slice with one coalesced 512-byte load.
//  * Ephemeris records: for every (group, segment, node) the positions and
//    parameters of the perturbers, rec[p] = (x, y, z, mu_p), followed by the
//    indirect term rec[P] = (sum_p mu_p r_p/|r_p|^3, 0).
#pragma once
#include <stdint.h>

#define PC_VERSION 100
#define PC_MAX_NP_FOR_HOOK 256   // largest padded node count of the operator hook
#define PC_MAX_PERT_DEV 16       // perturbers per force evaluation

struct PcGroupDev {
    double t0, h, tol;         // segment s spans [t0 + (s0 + s) h, t0 + (s0 + s + 1) h]
    int64_t ic_offset, n_ic;
    int64_t rec_offset;        // first ephemeris record of the group (S * N records)
    const double* kfrag;       // [NP/16][NP/4][64]
    const float* kfrag32;      // FP32 copy in the same fragment order
    const float* kfrag32p;     // FP32 copy, rows permuted for the f32 MFMA result layout
    const double* kfragT;      // fragments of K_N^T (adjoint)
    const double* kfrag2;      // fragments of the double-integration operator K2_N (second order)
    const double* tau;         // [NP] CGL nodes, zero past N
    int32_t N, NP, T, S;
    int32_t s0;                // first segment of the group on the t0 + k h grid (a call that
                               // resumes a span at one of its segment boundaries), else 0
    int64_t thread_offset;     // flyby screen: first thread of the group (n_ic * samples each)
};

struct PcJobDev {
    int64_t ic0;               // global index of the job's first IC
    int32_t group;
    int32_t n;                 // ICs in the job: <= T, or more (refilled columns)
};

// Perturber on a Keplerian orbit, prepared on the host:
// r(t) = a (cos E - e) P + b sin E Q,  E - e sin E = M0 + n (t - epoch).
struct PcBodyDev {
    double mu, a, e, n, M0, b;
    double P[3], Q[3];
};

struct PcParams {
    const PcGroupDev* groups;
    const PcJobDev* jobs;
    int32_t n_jobs;
    int32_t n_pert;
    const double* ics;          // [n_ic][6]
    double* states_out;         // [n_ic][6]
    int32_t* iters_out;         // [n_ic][iters_stride] or null
    int32_t iters_stride;
    int32_t nodes_stride;
    double* bounds_out;         // [n_ic][iters_stride+1][6] or null
    double* nodes_out;          // [n_ic][iters_stride][nodes_stride][6] or null
    const double* recs;         // ephemeris records, (n_pert+1) double4 each
    const double* recs_eih;     // Einstein-Infeld-Hoffmann records (3 (n_pert+1) + 1 double4
                                // each, pc_ephem_kernel), or null for the point-mass model
    double inv_c2;              // 1/c^2 of the relativistic model (0: point masses)
    double mu_sun;
    int32_t max_iter, fixed_iters, tol_mode, init;
    const double* guess;        // init 2: [n_ic][iters_stride][nodes_stride][6] initial node states
    int32_t precision;          // 0 FP64; 1 FP32 sweeps, then FP64
    int32_t max_fp32;           // cap on FP32 sweeps per segment
    int32_t conv;               // PC_CONV_PER_IC or PC_CONV_GROUP_MAX (plain path only)
    int32_t order;              // 1: first-order sweeps; 2: second-order sweeps (WIDE shapes)
    int32_t feedback;           // order 2: integral error feedback
    double switch2;             // squared relative change below which a job leaves FP32
    int32_t* counters;          // [0] ICs with a not-converged segment, [1] non-finite ICs
    int32_t* queue;             // next job of the persistent kernel (starts at 0)
};

// Adjoint of a propagation (reverse sweep over segments from boundary checkpoints).
struct PcAdjParams {
    PcParams fwd;               // groups, jobs, model and forward options (outputs unused)
    const double* ckpt;         // [n_ic][ckpt_stride + 1][6] segment-boundary states
    int32_t ckpt_stride;
    int32_t nodes_stride;
    const double* gbar_final;   // [n_ic][6] dL/d(final state)
    const double* gbar_nodes;   // [n_ic][ckpt_stride][nodes_stride][6] dL/d(node states), or null
    const double* fwd_nodes;    // [n_ic][ckpt_stride][nodes_stride][6] the forward call's converged
                                // node states, or null (each segment is re-solved from ckpt)
    double adj_tol;             // relative change of the propagated gradient that stops a sweep loop
    int32_t adj_max_iter;
    double* grad_out;           // [n_ic][6] dL/d(initial state)
    int32_t* adj_iters;         // [n_ic][ckpt_stride] adjoint sweeps per segment, or null
    int32_t* counters;          // [0] not converged, [1] non-finite, [2] queue
};

struct PcEphemParams {
    const PcGroupDev* groups;
    int32_t n_groups;
    int64_t n_recs;
    const PcBodyDev* bodies;
    int32_t n_pert;
    double epoch;
    double* recs;
    double* recs_eih;           // or null
    double mu_sun;
};

// One contiguous run of 32-bit words to copy (the gathers and scatters between a call's
// arrays and the sub-calls of its refinement passes or of flyby isolation).
struct PcCopyDev {
    const void* src;
    void* dst;
    int64_t words;
};

// Launchers (pc_kernels.hip).  All return a hipError_t as int.
int pc_launch_ephem(const PcEphemParams& p, void* stream);
// The launchers take the parameter block twice: by value for its host-side fields (job
// count), and as a device copy (in the workspace, written by the call's table transfer)
// that the kernels read, so that no lane keeps a private copy of it.
int pc_launch_fused(const PcParams& p, const PcParams* p_dev, int pairs, int grid, void* stream);
int pc_fused_occupancy(int pairs, int* blocks_per_cu);
// list: device [n] copy descriptors, one workgroup each.
int pc_launch_copy_runs(const PcCopyDev* list, int64_t n, void* stream);
// Flyby screen: ratio[m] = smallest distance of IC m's two-body (mu = 1) prediction to a
// perturber, in Hill radii, over `samples` CGL points of every segment of its group; ICs
// outside the groups are left alone.  ratio: device [n_ic].
struct PcFlybyParams {
    const PcGroupDev* groups;
    int32_t n_groups;
    const PcBodyDev* bodies;
    int32_t n_pert;
    double epoch;
    const double* ics;
    double* ratio;
    int32_t samples;
    int64_t n_threads;        // sum over groups of n_ic * samples
};
int pc_launch_flyby(const PcFlybyParams& p, void* stream);
int pc_launch_adjoint(const PcAdjParams& a, const PcAdjParams* a_dev, int grid, void* stream);
int pc_launch_apply_operator(int NP, const double* kfrag, int N, int64_t n_cols, const double* F,
                             const double* y0, double scale, double* Y, void* stream);
int pc_launch_eval_force(const double* r, const double* t, int64_t n, const PcBodyDev* bodies,
                         int n_pert, double epoch, double mu_sun, double* a, void* stream);
int pc_launch_eval_kepler(const double* y0, const double* dt, int64_t n, double* y, int32_t* ok,
                          void* stream);
// On-chip ceilings (pc_ceilings.hip): out[0] FP64 matrix-core TFLOP/s, out[1] FP64 vector FMA
// TFLOP/s, out[2] device copy GB/s (bytes read + written).  buf: device scratch of buf_bytes.
int pc_ceilings_run(int n_cu, void* buf, size_t buf_bytes, void* stream, double* out);
