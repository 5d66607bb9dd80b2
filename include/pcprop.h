/*
 * pcprop.h -- C ABI of the batched Picard-Chebyshev propagator for AMD MI355X (gfx950).
 *
 * Method: Masat, Colombo, Boutonnet, "GPU-based high-precision orbital propagation of
 * large sets of initial conditions through Picard-Chebyshev augmentation"
 * (arXiv 2301.03989).  The initial value problem is dx/dt = f(x, t), x(t0) = x0
 * (Sec. 2.1, eq. ibvp); each Picard iteration evaluates the dynamics at the N
 * Chebyshev-Gauss-Lobatto nodes of a segment, refits and integrates the Chebyshev
 * coefficients and evaluates the new iterate at the nodes (Sec. 2.2, matrix form:
 * F = w2 f(y, t), B_1 = S A F + 2 y_0, B_j = A F, y = C B), until the largest change
 * between two iterates falls below a tolerance (Sec. 2.2).  Many initial conditions
 * (ICs) are stacked into one augmented system (Sec. 3.1) and groups of them with
 * different settings form the second augmentation level (Sec. 3.2).  Long spans are
 * split into segments integrated in sequence, forward or backward (Sec. 2.2).
 *
 * Conventions for every entry point:
 *   - Return PC_OK (0) or one of the PC_E* codes below; no exception crosses the ABI.
 *   - Pointers marked "device" are HIP device allocations owned by the caller,
 *     contiguous, float64 unless noted.  Pointers marked "host" are host memory owned
 *     by the caller.  No pointer is retained after a call returns.
 *   - Work is ordered on `stream` (a hipStream_t; NULL is the null stream).  Calls that
 *     report a status return only after the stream has finished their work.
 *   - Units are the caller's; the workloads use mu_Sun = 1, AU and TU = 1/k days.
 *   - ICs are rows of six values (x, y, z, vx, vy, vz); output order = input order.
 *   - tf < t0 integrates backward in time.
 *   - A pc_ctx is used by one host thread at a time.
 */
#ifndef PCPROP_H
#define PCPROP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define PC_OK          0  /* success */
#define PC_EINVAL      1  /* invalid argument (null pointer, size out of range, bad model...) */
#define PC_ENOTCONV    2  /* at least one IC hit max_iter in some segment; outputs are written */
#define PC_ENONFINITE  3  /* at least one IC became non-finite (or was given non-finite); outputs written */
#define PC_EHIP        4  /* a HIP runtime call failed */
#define PC_ENOMEM      5  /* workspace too small (see pc_workspace_bytes) */

/* Per-IC, per-segment iteration records written to iters_out:
 *   k >= 1            the segment converged after k Picard iterations
 *   PC_ITER_NOTCONV   max_iter reached; the last iterate is kept and chained on
 *   PC_ITER_NONFINITE the state became non-finite; this and every later segment  */
#define PC_ITER_NOTCONV    (-1)
#define PC_ITER_NONFINITE  (-2)

#define PC_MAX_NODES  256  /* N per segment: 3 .. 256 */
#define PC_MAX_PERT   16   /* perturbing bodies */
#define PC_MAX_STREAMS 16  /* streams of the plain path's outer level (pc_opts.streams) */

typedef struct pc_ctx pc_ctx;     /* owns the cached operators per node count */
typedef void* pc_stream_t;        /* a hipStream_t */

/* Force model: a(r, t) = -mu_sun r/|r|^3 - sum_p mu_p [(r - r_p)/|r - r_p|^3 + r_p/|r_p|^3],
 * a point-mass, heliocentric form (with the indirect term) of the restricted N-body
 * dynamics of Sec. 5.4.1, with perturber p on a two-body Keplerian orbit about the
 * central body (gravitational parameter 1).  Perturber positions are evaluated once
 * per node before the iterations, as Sec. 5.4.1 does for its ephemerides.
 * inv_c2 > 0 selects the relativistic form Sec. 5.4.1 uses, the Einstein-Infeld-Hoffmann
 * acceleration of the massless propagated body (PPN beta = gamma = 1, 1/c^2 = inv_c2 in
 * the model's units): it depends on the body's velocity and on the positions, velocities,
 * accelerations and potentials of the major bodies (the central body at rest at the
 * origin, the perturbers on their orbits, differentiated in time), all evaluated once per
 * node before the iterations; the Newtonian indirect term is kept, so inv_c2 = 0 is the
 * point-mass model.  It runs with the per-IC stopping rule, forward (fused and plain
 * paths) and in pc_adjoint; other calls with inv_c2 > 0 return PC_EINVAL.  Under PC_FP32_THEN_FP64 the
 * FP64 sweeps evaluate this acceleration and the increment sweeps linearise with the
 * point-mass gravity gradient (the relativistic terms change it by O(1/c^2), which only
 * perturbs the linearisation the FP64 sweeps correct). */
typedef struct {
    double mu_sun;        /* central body's gravitational parameter */
    int32_t n_pert;       /* 0 .. PC_MAX_PERT; 0 = two-body dynamics */
    const double* pert;   /* host [n_pert][7]: mu_p, a, e, inc, raan, argp, M0 (radians);
                             M0 is the mean anomaly at `epoch`; 0 <= e < 1, a > 0 */
    double epoch;
    double inv_c2;        /* 1/c^2: 0 = point masses (default), > 0 = Einstein-Infeld-Hoffmann */
} pc_model;

/* Initial guess of every segment (Sec. 2.1): warm (two-body Kepler from the segment's
 * initial state), cold (the initial state at every node), or the caller's node states
 * (opts.guess): a hot start from a previous propagation, e.g. of a simpler model or of
 * nearby initial conditions, which Sec. 2.1 lists as guesses closer to the solution. */
enum { PC_INIT_KEPLER = 0, PC_INIT_COLD = 1, PC_INIT_GUESS = 2 };
enum { PC_TOL_REL = 0, PC_TOL_ABS = 1 };         /* relative or absolute stopping rule, Sec. 2.2 */
/* Arithmetic of the sweeps.  PC_FP32_THEN_FP64 (fused path): every segment starts with
 * an FP32 phase, which ends once the relative change of every iterating IC of the job is
 * below switch_tol (or after max_fp32 FP32 sweeps).  Jobs of 16 or more ICs run one FP64
 * sweep and then increment sweeps, Y <- Y + w2 K_N dF, dF = (dv, G dr) the change of the
 * force matrix to first order in the last change (dr, dv) of the iterate, G the gravity
 * gradient at the iterate of the last FP64 sweep: dF, G and the product are FP32 (matrix
 * cores), no force is evaluated, and the sweeps converge at the Picard rate.  At the
 * switch one FP64 sweep re-anchors the iterate on y0 + w2 K_N F(Y); increment sweeps from
 * there carry on until no IC of the job changes by more than tol; FP64 sweeps follow, and
 * each IC stops on the first of them that changes it by less than tol (usually the
 * first).  8-IC jobs run Picard sweeps with an FP32 force and FP32 product, then FP64
 * sweeps.  The accumulation into the iterate, the stopping test and all stored states stay
 * FP64.  iters_out counts all sweeps; it is usually one more than the FP64 schedule's,
 * more for ICs whose job holds a slower IC. */
enum { PC_FP64 = 0, PC_FP32_THEN_FP64 = 1 };
enum { PC_PATH_FUSED = 0, PC_PATH_PLAIN = 1 };   /* one persistent launch / per-iteration kernels */
/* Granularity of the stopping rule (Sec. 3.2).  PC_CONV_PER_IC: every IC stops at its own
 * first sweep whose change is below tol and keeps that iterate.  PC_CONV_GROUP_MAX: one
 * decision per group, on the largest change over the group's ICs that are still finite,
 * as the paper's CUDA program does for the whole augmented system (Sec. 5.4.2): every IC
 * of the group takes the same number of sweeps per segment (iters_out holds that number,
 * or PC_ITER_NOTCONV for all of them when max_iter sweeps do not bring the maximum below
 * tol).  A non-finite IC leaves its group (PC_ITER_NONFINITE) without holding the others
 * back.  PC_CONV_GROUP_MAX runs on the plain path, whose host loop sees every sweep of
 * the whole group; the fused path and the adjoint reject it with PC_EINVAL. */
enum { PC_CONV_PER_IC = 0, PC_CONV_GROUP_MAX = 1 };

typedef struct {
    int32_t init;         /* PC_INIT_KEPLER (default), PC_INIT_COLD or PC_INIT_GUESS */
    int32_t max_iter;     /* Picard iterations per segment before PC_ITER_NOTCONV (default 64) */
    int32_t tol_mode;     /* PC_TOL_REL (default) or PC_TOL_ABS */
    int32_t precision;    /* PC_FP64 */
    int32_t path;         /* PC_PATH_FUSED (default) or PC_PATH_PLAIN */
    int32_t fixed_iters;  /* > 0: run exactly this many iterations per segment (no stopping rule) */
    int32_t tile_pairs;   /* nodes x ICs held by one workgroup: 0 = the context's table (set by
                             pc_autotune or pc_set_tile_pairs; untuned: 1024 up to 64 padded
                             nodes, else 2048), 1024 or 2048 */
    int32_t graph;        /* fused path: 1 = capture the call's device work (table copy, ephemeris,
                             propagation kernel, status copy) in a HIP graph and replay it while
                             the call's shapes, options and pointers repeat (default 0) */
    double switch_tol;    /* PC_FP32_THEN_FP64: relative change below which a job leaves FP32
                             (0 = default: 1e-6 for FP32 increment sweeps, 1e-4 for FP32
                             Picard sweeps of 8-IC jobs).  On a 262144-IC N-body ensemble
                             1e-5, 1e-6 and 1e-7 ran within 2 % of each other */
    int32_t max_fp32;     /* PC_FP32_THEN_FP64: cap on FP32 sweeps per segment (0 = default 24) */
    int32_t job_list;     /* fused FP64 forward calls: ICs per job in units of its column block
                             (the ICs one workgroup iterates at once: 2048 / padded nodes, or
                             1024 / padded nodes with tile_pairs 1024); when an IC converges,
                             its column takes the next IC of the job for the same segment.
                             0 = automatic (the longest of 1, 2, 4, 8 whose jobs fill the
                             workgroup slots within 25 % of the fewest block-times), 1 = off,
                             2, 4 or 8 = that many blocks.  Results do not depend on it. */
    int32_t conv;         /* PC_CONV_PER_IC (default) or PC_CONV_GROUP_MAX */
    int32_t streams;      /* plain path: groups run on this many streams at once (the
                             outer-level streams of Sec. 5.4; 1..PC_MAX_STREAMS, default 1),
                             all driven from the calling thread, which polls each stream's
                             per-iteration read-back and takes that stream's next loop decision
                             when it has landed; the workspace holds one plain-path state per
                             stream.  Results do not depend on it. */
    int32_t order;        /* 1 (default): the iteration of Sec. 2.2 on the first-order system,
                             y = y0 + w2 K_N F(y).  2: the second-order form that Sec. 1 cites
                             as applicable to the augmented system: the velocity and the
                             position are both obtained from the acceleration samples,
                             v = v0 + w2 K_N a and x = x0 + w2 v0 (tau + 1) + w2^2 K2_N a, with
                             K2_N the degree N-2 fit integrated twice, so the position takes
                             the new velocity instead of the previous one (about half the
                             sweeps at the same product cost per sweep).  Its fixed point is a
                             different discretisation of the same ODE (the position series
                             has degree N).  Order 2 runs on the fused FP64 path with the
                             per-IC rule and the point-mass model, for every node count (3 to
                             256, with or without the feedback); other calls with order 2
                             return PC_EINVAL. */
    int32_t feedback;     /* order 2: 1 = integral error feedback, the development Sec. 1 cites
                             with the adaptive variant of the method.  The sweep's accelerations
                             were taken at the previous position iterate; the change dx the
                             sweep makes to the position is fed back through the linear part of
                             the point-mass dynamics, da = (da/dr) dx at the previous iterate,
                             whose single and double integrals (the same operators) are added
                             to the new velocity and position.  A second product per sweep and
                             one barrier; the fixed point is the second-order one.  0 (default)
                             or 1, order 2 only */
    const double* guess;  /* init = PC_INIT_GUESS: device [n_ic][iters_stride][nodes_stride][6],
                             the node states of the initial guess of every segment, in the
                             layout of the same call's nodes_out (e.g. the nodes_out of an
                             earlier call); a non-finite row falls back to the segment's
                             initial state at that node.  NULL otherwise (default) */
    int32_t refine;       /* adaptive segment refinement, 0 (default, off) .. 8, fused path:
                             long spans are integrated piecewise because the iteration does not
                             hold over too long a piece (Sec. 2.2), and the adaptive variant of
                             the method cited in Sec. 1 sets the piece length per segment.  A
                             segment whose sweeps do not converge within max_iter is solved
                             again from its initial state as 2, then 4, ... up to 2^refine equal
                             sub-segments of the same node count (each with its own warm start
                             and sweeps) until all of them converge; its iters_out entry is then
                             the sum of their sweep counts (PC_ITER_NOTCONV, with the finest
                             split's end state, if that still fails), bounds_out and states_out
                             take the new states, and the rest of the span is run again from
                             there on the original segment grid.  Runs after the main launch,
                             in passes of up to 8192 refined ICs (one launch each).  Needs
                             iters_out and bounds_out, takes no nodes_out and no guess;
                             pc_workspace_bytes includes its region.  iters_out, bounds_out and
                             states_out of ICs that need no refinement are those of refine = 0. */
    double flyby_hill;    /* flyby isolation, 0 (default, off) or a threshold in Hill radii: the
                             outer level isolates sub-groups of trajectories that experience a
                             planetary flyby (Sec. 3.2; flyby detection, Sec. 7).  Before the
                             propagation every IC is screened (pc_flyby_ratio, 16 sample points
                             per segment); in every group, the ICs whose ratio is below
                             flyby_hill form a group of their own with the same interval, nodes,
                             segments and tolerance, and the call runs on the ICs reordered so
                             (a copy in the workspace; outputs are returned in the caller's
                             order).  Under the per-IC rule the results are those without
                             isolation; under PC_CONV_GROUP_MAX the flyby ICs no longer set the
                             sweep count of the rest of their group.  Not with nodes_out, a
                             guess, refinement, graph capture or the allocation-free call. */
} pc_opts;

/* One outer-level group of the two-level augmentation (Sec. 3.2): ICs
 * [ic_offset, ic_offset + n_ic) share the interval, node count, segment count and
 * tolerance.  Segment s spans [t0 + s h, t0 + (s+1) h], h = (tf - t0)/segments. */
typedef struct {
    int64_t ic_offset;
    int64_t n_ic;         /* >= 1 */
    double t0, tf;        /* t0 != tf, both finite */
    int32_t nodes;        /* 3 .. PC_MAX_NODES */
    int32_t segments;     /* >= 1 */
    double tol;           /* > 0, finite */
} pc_group;

/* Fill `opts` with the defaults listed above. */
void pc_default_opts(pc_opts* opts);

/* Create a context on HIP device `device`.  *out receives the context. */
int pc_ctx_create(int device, pc_ctx** out);
void pc_ctx_destroy(pc_ctx* ctx);

/* Bytes of device workspace that pc_propagate_batched needs for these groups. */
int pc_workspace_bytes(pc_ctx* ctx, const pc_group* groups /* host [n_groups] */, int32_t n_groups,
                       const pc_model* model, const pc_opts* opts, size_t* bytes /* host out */);

/* Propagate n_ic ICs over [t0, tf] in `segments` segments of `nodes` CGL nodes, each
 * iterated until max_j max(|dr_j|/|r_j|, |dv_j|/|v_j|) < tol (Sec. 2.2, Sec. 5.4.2),
 * per IC (the per-block error of Sec. 3.2 with blocks of one member).
 *   ics        device [n_ic][6]          initial states at t0
 *   states_out device [n_ic][6]          states at tf
 *   iters_out  device int32 [n_ic][segments] iteration records, or NULL
 *   workspace  device, ws_bytes >= pc_workspace_bytes(one group)
 * Equivalent to pc_propagate_batched with a single group. */
int pc_propagate(pc_ctx* ctx, const double* ics, int64_t n_ic, double t0, double tf,
                 int32_t nodes, int32_t segments, double tol,
                 const pc_model* model, const pc_opts* opts /* NULL = defaults */,
                 double* states_out, int32_t* iters_out,
                 void* workspace, size_t ws_bytes, pc_stream_t stream);

/* Two-level augmented propagation (Sec. 3.2): all groups in one call.
 *   ics          device [n_ic][6]; groups index into it and must not overlap
 *   states_out   device [n_ic][6]
 *   iters_out    device int32 [n_ic][iters_stride] or NULL; iters_stride >= every group's
 *                segment count; unused columns are left untouched
 *   bounds_out   device [n_ic][iters_stride + 1][6] segment-boundary states, or NULL
 *   nodes_out    device [n_ic][iters_stride][nodes_stride][6] final node states of every
 *                segment, or NULL; nodes_stride >= every group's node count
 * The fused path runs every group in one launch; the plain path runs each group with
 * per-iteration kernels and a host-side loop (the structure of Sec. 5.4). */
int pc_propagate_batched(pc_ctx* ctx, const double* ics, int64_t n_ic,
                         const pc_group* groups /* host */, int32_t n_groups,
                         const pc_model* model, const pc_opts* opts,
                         double* states_out, int32_t* iters_out, int32_t iters_stride,
                         double* bounds_out, double* nodes_out, int32_t nodes_stride,
                         void* workspace, size_t ws_bytes, pc_stream_t stream);

/* Bytes of device memory that pc_propagate_batched_noalloc uses as its workspace. */
#define PC_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* pc_propagate_batched for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same fused-path kernels and
 * results, with no device or host allocation in the call.  Its workspace is a static
 * device array of PC_NOALLOC_SCRATCH_BYTES (32 MiB) that the library holds on every
 * device it runs on until the process ends, its address taken once per device when a
 * context is created there.  The caller still owns ics and every output.
 *   Arguments as pc_propagate_batched without workspace and ws_bytes.
 *   Limits (PC_ENOMEM with a message naming the sizes when exceeded): the call's workspace
 *   (pc_workspace_bytes: descriptor tables, ephemeris records) must fit the scratch, e.g.
 *   up to about 110000 segment-node pairs over all groups at 8 point-mass perturbers;
 *   its job tables must fit the context's pinned staging buffer (4 MiB, or more once an
 *   earlier call has grown it).
 *   PC_EINVAL: opts->path must be PC_PATH_FUSED and opts->graph 0; every node count of the
 *   call must have been used before on this context (an earlier pc_propagate_batched
 *   builds and caches its operators), since building them allocates.
 *   Every call on one device shares that device's scratch and each call starts by copying
 *   its tables over it (work-queue head and status counters included); calls that overlap
 *   on one device, from any context or thread, race and must be serialised by the caller.
 *   The call synchronises its stream before returning, as pc_propagate_batched does. */
int pc_propagate_batched_noalloc(pc_ctx* ctx, const double* ics, int64_t n_ic,
                                 const pc_group* groups /* host */, int32_t n_groups,
                                 const pc_model* model, const pc_opts* opts,
                                 double* states_out, int32_t* iters_out, int32_t iters_stride,
                                 double* bounds_out, double* nodes_out, int32_t nodes_stride,
                                 pc_stream_t stream);

/* Gradient of a loss through the converged propagation (reverse mode, segment
 * checkpointing).  Per segment the converged node states satisfy Y = 1 y0^T + K_N G(Y)
 * (the fixed point of Sec. 2.2); with J_j = w2 df/dy at node j the loss gradient seeds
 * gbar give dL/dy0 = sum_j mu_j where mu = gbar + J^T (K_N^T mu), solved by sweeping until
 * the propagated gradient changes by less than adj_tol (relative).  Segments are taken
 * from the last: each is re-solved from its checkpoint with the forward code (or, when
 * fwd_nodes is given, its converged node states are read from there), then its gradient
 * seeds the end node of the previous one.  Fused FP64 path, any node count (3 .. 256).
 * With the relativistic model (inv_c2 > 0) the acceleration also depends on the velocity,
 * so J^T w = ((da/dr)^T w_v, w_r + (da/dv)^T w_v), both products evaluated exactly at
 * each node (the major bodies' states are the call's own, re-evaluated as forward).
 *   groups, model, opts  as in the forward pc_propagate_batched call
 *   ckpt        device [n_ic][ckpt_stride + 1][6] segment-boundary states of the forward call
 *               (its bounds_out); ckpt_stride >= every group's segment count
 *   gbar_final  device [n_ic][6] dL/d(final state)
 *   gbar_nodes  device [n_ic][ckpt_stride][nodes_stride][6] dL/d(node states), or NULL
 *   fwd_nodes   device [n_ic][ckpt_stride][nodes_stride][6] the forward call's node states
 *               (its nodes_out, same strides), or NULL: storing them costs 48 bytes per IC,
 *               node and segment and saves the re-solves
 *   grad_ics    device [n_ic][6] dL/d(initial state), output
 *   adj_iters   device int32 [n_ic][ckpt_stride] adjoint sweeps per segment, or NULL
 * Returns PC_ENOTCONV if a forward re-solve or an adjoint sweep loop hit its cap. */
int pc_adjoint(pc_ctx* ctx, int64_t n_ic, const pc_group* groups /* host */, int32_t n_groups,
               const pc_model* model, const pc_opts* opts, const double* ckpt, int32_t ckpt_stride,
               const double* gbar_final, const double* gbar_nodes, const double* fwd_nodes,
               int32_t nodes_stride,
               double adj_tol, int32_t adj_max_iter, double* grad_ics, int32_t* adj_iters,
               void* workspace, size_t ws_bytes, pc_stream_t stream);

/* Flyby screen of the outer level (Sec. 3.2, Sec. 7), the test of opts.flyby_hill: for
 * every IC of the groups, the smallest distance of its two-body (mu = 1) prediction from
 * t0 to any perturber of `model` (mu_p > 0), in units of that perturber's Hill radius
 * a_p (mu_p/3)^(1/3), over `samples` Chebyshev-Gauss-Lobatto points of each segment of
 * its group (t = w2 tau_k + w1).  An IC whose orbit is not elliptic gets 0; with no
 * massive perturber the result is +inf.
 *   ics    device [n_ic][6]
 *   ratio  device [n_ic] out; entries of ICs outside the groups are left untouched
 *   samples 2 .. 64 (opts.flyby_hill uses 16)
 *   workspace: pc_workspace_bytes of the same groups */
int pc_flyby_ratio(pc_ctx* ctx, const double* ics, int64_t n_ic, const pc_group* groups /* host */,
                   int32_t n_groups, const pc_model* model, int32_t samples, double* ratio,
                   void* workspace, size_t ws_bytes, pc_stream_t stream);

/* ---- operator and kernel-level entry points (used by the tests) ---- */

/* The N x N matrix K_N with y_j = y_0 + sum_l K_N[j][l] g_l for the w2-scaled force
 * samples g (steps F -> B -> y of Sec. 2.2 folded into one product).  K_host: host
 * [nodes][nodes], row-major. */
int pc_get_operator(pc_ctx* ctx, int32_t nodes, double* K_host);

/* Y[j][c] = y0[c] + scale * sum_l K_N[j][l] F[l][c] on the GPU's FP64 matrix cores.
 *   F device [nodes][n_cols], y0 device [n_cols], Y device [nodes][n_cols]. */
int pc_apply_operator(pc_ctx* ctx, int32_t nodes, int64_t n_cols, const double* F,
                      const double* y0, double scale, double* Y, pc_stream_t stream);

/* Accelerations of the force model at n points: r device [3][n], t device [n],
 * a_out device [3][n]. */
int pc_eval_force(pc_ctx* ctx, const double* r, const double* t, int64_t n,
                  const pc_model* model, double* a_out, pc_stream_t stream);

/* Two-body (mu = 1) propagation used by the warm start (Sec. 2.1): y0 device [6][n],
 * dt device [n] -> y device [6][n]; ok device int32 [n] (1 = elliptic orbit solved). */
int pc_eval_kepler(pc_ctx* ctx, const double* y0, const double* dt, int64_t n,
                   double* y, int32_t* ok, pc_stream_t stream);

/* On-chip ceilings for the roofline figures, measured on this device: out[0] = FP64
 * matrix-core rate (a loop of independent v_mfma_f64_16x16x4 chains on every SIMD),
 * out[1] = FP64 vector rate (a loop of independent FMA chains on every lane), both in
 * TFLOP/s, and out[2] = device copy bandwidth in GB/s (bytes read plus written, one half of
 * buf copied to the other).  Best of three timed launches each.
 *   buf  device scratch, overwritten; buf_bytes >= 16 MiB (the copy moves buf_bytes / 2)
 *   out  host [3] */
int pc_measure_ceilings(pc_ctx* ctx, void* buf, size_t buf_bytes, pc_stream_t stream, double* out);

/* Number of HIP graphs the context has captured for graph = 1 calls (test hook: a call
 * whose signature, or whose pinned staging buffer, differs from the captured one's is
 * captured again). */
int pc_graph_captures(pc_ctx* ctx, int64_t* count /* host out */);

/* Kernel timing of the next calls: when enabled, pc_propagate_batched records HIP events
 * on its stream around its propagation kernels (not the ephemeris table build or the
 * copies), and pc_last_kernel_ms returns the elapsed time of the last such call in
 * milliseconds.  Used by the benchmark for the roofline figure. */
int pc_set_timing(pc_ctx* ctx, int enable);
int pc_last_kernel_ms(pc_ctx* ctx, double* ms /* host out */);

/* Autotuner of the fused FP64 path: on the caller's batch (the whole call, default options,
 * median kernel time of three runs per candidate) it starts from the untuned rules and
 * keeps each change that makes the call faster, in coordinate order: first the job shape
 * of the call (tile_pairs 2048, or 1024 where every node count fits it; one shape per
 * launch, recorded for the batch's largest padded node count), then, for each padded node
 * count of the batch from the largest, the job length (job_list 1, 2, 4 or 8 column blocks,
 * recorded per padded node count).  Later calls with tile_pairs = 0 and job_list = 0 read
 * these tables; nothing is recorded that measured slower than the untuned rules.
 * 4 + 12 x (node counts) calls of the batch are run.
 *   scratch_states  device [n_ic][6], overwritten
 *   chosen_pairs    host out, the recorded shape
 * Other arguments as pc_propagate_batched. */
int pc_autotune(pc_ctx* ctx, const double* ics, int64_t n_ic, const pc_group* groups, int32_t n_groups,
                const pc_model* model, double* scratch_states, void* workspace, size_t ws_bytes,
                pc_stream_t stream, int32_t* chosen_pairs);

/* Set / read the tuned job shape for a padded node count (16, 32, 64, 128 or 256):
 * pairs 1024 or 2048, or 0 to clear. */
int pc_set_tile_pairs(pc_ctx* ctx, int32_t padded_nodes, int32_t pairs);
int pc_get_tile_pairs(pc_ctx* ctx, int32_t padded_nodes, int32_t* pairs);

/* Set / read the tuned job length (column blocks per job: 1, 2, 4 or 8; 0 = the untuned
 * rule) for a padded node count, used by fused FP64 calls with job_list = 0. */
int pc_set_job_list(pc_ctx* ctx, int32_t padded_nodes, int32_t blocks);
int pc_get_job_list(pc_ctx* ctx, int32_t padded_nodes, int32_t* blocks);

/* Message for a status code (static storage). */
const char* pc_strerror(int code);

/* Detail of the last error raised in this context (static per context). */
const char* pc_last_error(pc_ctx* ctx);

/* Library version, 100 * major + minor. */
int pc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PCPROP_H */
