// pc_plain.hip -- the "plain" GPU path: one group at a time, a sequence of kernels per
// Picard iteration and a host-side loop, the structure of the paper's CUDA program
// (Sec. 5.4): dynamics kernel over all stacked states, the fit/integrate/evaluate
// product (here one FP64 MFMA product with the +y0 term in its epilogue), the error
// computation and its reduction, and a host check of the result every iteration.
//
// Differences from the paper's program: by default the error is per IC (converged ICs are
// frozen and jobs whose ICs have all converged are compacted out of the next launches)
// and the host reads back one active-job count per iteration instead of block maxima.
// With PC_CONV_GROUP_MAX the paper's whole-system rule holds per group: no IC stops on
// its own, the step kernels count the jobs that still hold a change above tol, and the
// host ends the segment for the whole group when that count is zero.
//
// State in HBM, per group: Y[node][comp 9][IC] (comps 0..5 iterate, 6..8 acceleration),
// IC index fastest -- the component-major, row-by-node layout of Sec. 5.4.1.
#include "pcprop.h"
#include "pc_device.h"
#include "pc_plain.h"

namespace {

constexpr int kPlainForceBlock = 256;

// Initial states of the group's ICs (padding columns copy the job's first IC).
__global__ void pc_plain_load(PcPlainArgs a)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.Mpad) return;
    const PcJobDev job = a.jobs[m / a.T];
    const int i = (int)(m % a.T);
    const double* y = a.p.ics + (job.ic0 + (i < job.n ? i : 0)) * 6;
    bool fin = true;
    for (int c = 0; c < 6; ++c) {
        const double v = y[c];
        a.Y0[c * a.Mpad + m] = v;
        fin = fin && isfinite(v);
    }
    a.dead[m] = !fin;
    a.notconv[m] = 0;
    a.valid[m] = i < job.n;
}

// Segment start: initial guess (Kepler or cold, Sec. 2.1) at every (node, IC) pair,
// zero padding rows, flags and the full job list.
__global__ void pc_plain_init(PcPlainArgs a, int s, double w2)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)a.NP * a.Mpad;
    if (idx < a.n_jobs) a.job_list[idx] = (int32_t)idx;
    if (idx == 0) {
        a.count[0] = a.n_jobs;
        a.count[2] = 0;
    }
    if (idx >= total) return;
    const int j = (int)(idx / a.Mpad);
    const int64_t m = idx - (int64_t)j * a.Mpad;
    double* Yj = a.Y + (size_t)j * 9 * a.Mpad + m;
    if (j >= a.N) {
        for (int c = 0; c < 9; ++c) Yj[c * a.Mpad] = 0.0;
        return;
    }
    double y0[6], y[6];
    for (int c = 0; c < 6; ++c) y0[c] = a.Y0[c * a.Mpad + m];
    const bool dead = a.dead[m];
    bool have = false;
    if (a.p.init == 2 && !dead && a.valid[m]) {   // the caller's node states
        const PcJobDev job = a.jobs[m / a.T];
        const double* gp =
            a.p.guess + (((size_t)(job.ic0 + m % a.T) * a.p.iters_stride + s) * a.p.nodes_stride + j) * 6;
        have = true;
        for (int c = 0; c < 6; ++c) {
            y[c] = gp[c];
            have = have && isfinite(y[c]);
        }
    } else if (a.p.init == 0 && !dead) {
        have = pc_kepler(y0, w2 * (a.g->tau[j] + 1.0), y);
    }
    if (!have)
        for (int c = 0; c < 6; ++c) y[c] = y0[c];
    for (int c = 0; c < 6; ++c) Yj[c * a.Mpad] = y[c];
    if (j == 0) {
        a.active[m] = a.valid[m] && !dead;
        if (dead && a.valid[m] && a.p.iters_out) {
            const PcJobDev job = a.jobs[m / a.T];
            a.p.iters_out[(size_t)(job.ic0 + m % a.T) * a.p.iters_stride + s] = -2;
        }
    }
}

// Dynamics at every (node, IC) pair of the active jobs (the paper's dynamics kernel):
// one thread per pair, state read from and acceleration written to HBM.
__global__ __launch_bounds__(kPlainForceBlock) void pc_plain_force(PcPlainArgs a, int s)
{
    const int bpj = (a.NP * a.T) / kPlainForceBlock;          // blocks per job
    const int job = a.job_list[blockIdx.x / bpj];
    const int pr = (blockIdx.x % bpj) * kPlainForceBlock + threadIdx.x;
    const int j = pr / a.T;
    const int64_t m = (int64_t)job * a.T + pr % a.T;
    if (j >= a.N || !a.active[m]) return;
    const int P = a.p.n_pert;
    double* Yj = a.Y + (size_t)j * 9 * a.Mpad + m;
    if (a.p.inv_c2 != 0.0) {
        // relativistic model: the segment's records of the major bodies (slot-major)
        const double4* erec = reinterpret_cast<const double4*>(a.p.recs_eih) +
                              (size_t)(a.g->rec_offset + (int64_t)s * a.N) * pc_eih_rec(P);
        const double x[1] = {Yj[0]}, y[1] = {Yj[a.Mpad]}, z[1] = {Yj[2 * a.Mpad]};
        const double vx[1] = {Yj[3 * a.Mpad]}, vy[1] = {Yj[4 * a.Mpad]}, vz[1] = {Yj[5 * a.Mpad]};
        const int jr[1] = {j};
        double ax[1], ay[1], az[1];
        pc_force_eih<1, true>(x, y, z, vx, vy, vz, erec, jr, a.N, P, a.p.inv_c2, ax, ay, az);
        Yj[6 * a.Mpad] = ax[0];
        Yj[7 * a.Mpad] = ay[0];
        Yj[8 * a.Mpad] = az[0];
        return;
    }
    const double4* rec = reinterpret_cast<const double4*>(a.p.recs) +
                         (size_t)(a.g->rec_offset + (int64_t)s * a.N + j) * (P + 1);
    double ax, ay, az;
    pc_accel(Yj[0], Yj[a.Mpad], Yj[2 * a.Mpad], rec, P, a.p.mu_sun, ax, ay, az);
    Yj[6 * a.Mpad] = ax;
    Yj[7 * a.Mpad] = ay;
    Yj[8 * a.Mpad] = az;
}

// The product y_new = y0 + w2 K_N F for one active job per workgroup, with the error of
// every IC against the previous iterate and the stopping decision in the epilogue.  The
// job's state moves between HBM and LDS with IC-contiguous (coalesced) accesses; the
// lanes' shares of it come from LDS.
template <int PAIRS, int NP>
__global__ __launch_bounds__(PAIRS / 4) void pc_plain_step(PcPlainArgs a, int s, int it, double w2)
{
    using Sh = PcShape<PAIRS, NP>;
    constexpr int NT = Sh::NT, T = Sh::T, ROW = Sh::ROW, NQ = Sh::NQ;
    __shared__ double sF[6 * PAIRS];   // F = (v, a); after the product: the new iterate (r, v)
    __shared__ double sR[3 * PAIRS];   // positions of the current iterate, [node][3][IC]
    __shared__ double sY0[6 * T];
    __shared__ int sFlag[Sh::W * 16];
    __shared__ int sActive[T];
    __shared__ int sWas[T];
    __shared__ int sOpen;   // group-max rule: some IC of the job changed by more than tol

    const int tid = threadIdx.x;
    const int job = a.job_list[blockIdx.x];
    const int64_t m0 = (int64_t)job * T;
    const int N = a.N;
    const PcLane L = pc_lane_geometry<PAIRS, NP>(tid, N);
    const size_t row = (size_t)9 * a.Mpad;

    // stage F = (v, a) (Y comps 3..8) and r (Y comps 0..2) of the job, and its initial states
    for (int i = tid; i < 6 * PAIRS; i += NT) {
        const int j = i / ROW, c = (i % ROW) / T, k = i % T;
        sF[j * ROW + c * T + pc_fcol<PAIRS, NP>(j, k)] =
            j < N ? a.Y[(size_t)j * row + (size_t)(3 + c) * a.Mpad + m0 + k] : 0.0;
    }
    for (int i = tid; i < 3 * PAIRS; i += NT) {
        const int j = i / (3 * T), c = (i % (3 * T)) / T, k = i % T;
        sR[j * 3 * T + c * T + pc_fcol<PAIRS, NP>(j, k)] =
            j < N ? a.Y[(size_t)j * row + (size_t)c * a.Mpad + m0 + k] : 0.0;
    }
    for (int i = tid; i < 6 * T; i += NT) sY0[i] = a.Y0[(size_t)(i / T) * a.Mpad + m0 + i % T];
    if (tid < T) {
        sActive[tid] = a.active[m0 + tid];
        sWas[tid] = sActive[tid];
    }
    if (tid == 0) sOpen = 0;
    __syncthreads();
    double yc[6][4];
#pragma unroll
    for (int h = 0; h < Sh::H; ++h) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, h, r);
            const int jj = j < N ? j : N - 1;
            const int col = pc_fcol<PAIRS, NP>(jj, pc_ic(L, r));
            if constexpr (Sh::WIDE) {
#pragma unroll
                for (int c = 0; c < 3; ++c) yc[c][r] = sR[jj * 3 * T + c * T + col];
#pragma unroll
                for (int c = 0; c < 3; ++c) yc[3 + c][r] = sF[jj * ROW + c * T + col];
            } else {
#pragma unroll
                for (int cb = 0; cb < 3; ++cb) {
                    const int c = 2 * cb + L.hi;
                    yc[3 * h + cb][r] = c < 3 ? sR[jj * 3 * T + c * T + col] : sF[jj * ROW + (c - 3) * T + col];
                }
            }
        }
    }

    f64x4 acc[6];
    gconst_dp kp0 = (gconst_dp)a.g->kfrag + (size_t)L.strip0 * NQ * 64 + L.lane;
    double kpre[8];
    pc_kpre_load<PAIRS, NP>(kp0, kpre);
    const int flag = pc_product<PAIRS, NP, false, false>(sF, sY0, kp0, kpre, nullptr, yc, acc, w2,
                                                         pc_tol(a.p.tol_mode, a.t2, 0.0), N, L);
    if (L.lane < 16) sFlag[L.wave * 16 + L.lane] = flag;
    __syncthreads();   // F read by every wave, flags complete

    if (tid < T && sActive[tid]) {
        const int f = pc_gather_flags<PAIRS, NP>(sFlag, tid);
        int rec = 0;
        if (f & 2) rec = -2;
        else if (a.p.fixed_iters > 0) rec = (it == a.p.fixed_iters) ? it : 0;
        else if (a.p.conv == PC_CONV_GROUP_MAX) { if (f & 1) sOpen = 1; }   // the host decides
        else if (!(f & 1)) rec = it;
        else if (it == a.p.max_iter) rec = -1;
        if (rec != 0) {
            sActive[tid] = 0;
            a.active[m0 + tid] = 0;
            if (rec == -2) a.dead[m0 + tid] = 1;
            if (rec == -1) a.notconv[m0 + tid] = 1;
            const PcJobDev jd = a.jobs[job];
            if (tid < jd.n && a.p.iters_out)
                a.p.iters_out[(size_t)(jd.ic0 + tid) * a.p.iters_stride + s] = rec;
        }
    }
    // the new iterate into LDS (over F, now free), then out to HBM for the ICs that were
    // iterating
#pragma unroll
    for (int h = 0; h < Sh::H; ++h) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = pc_node(L, h, r);
            if (j >= N) continue;
            const int col = pc_fcol<PAIRS, NP>(j, pc_ic(L, r));
            if constexpr (Sh::WIDE) {
#pragma unroll
                for (int c = 0; c < 6; ++c) sF[j * ROW + c * T + col] = acc[c][r];
            } else {
#pragma unroll
                for (int cb = 0; cb < 3; ++cb) sF[j * ROW + (2 * cb + L.hi) * T + col] = acc[3 * h + cb][r];
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < 6 * PAIRS; i += NT) {
        const int j = i / ROW, c = (i % ROW) / T, k = i % T;
        if (j < N && sWas[k]) a.Y[(size_t)j * row + (size_t)c * a.Mpad + m0 + k] = sF[j * ROW + c * T + pc_fcol<PAIRS, NP>(j, k)];
    }
    const int any = __syncthreads_or(tid < T ? sActive[tid] : 0);
    if (tid == 0) {
        a.job_flag[job] = any;
        if (sOpen) atomicAdd(&a.count[2], 1);
    }
}

// Stream compaction of the active job list: prefix sum of the job flags (one workgroup).
__global__ __launch_bounds__(1024) void pc_plain_compact(PcPlainArgs a)
{
    __shared__ int sScan[1024];
    __shared__ int sBase;
    const int n_in = a.count[0];
    if (threadIdx.x == 0) sBase = 0;
    __syncthreads();
    for (int c0 = 0; c0 < n_in; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int job = i < n_in ? a.job_list[i] : -1;
        const int f = (job >= 0) ? (a.job_flag[job] != 0) : 0;
        sScan[threadIdx.x] = f;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {          // inclusive Hillis-Steele scan
            const int v = threadIdx.x >= off ? sScan[threadIdx.x - off] : 0;
            __syncthreads();
            sScan[threadIdx.x] += v;
            __syncthreads();
        }
        if (f) a.job_list_out[sBase + sScan[threadIdx.x] - 1] = job;
        __syncthreads();
        if (threadIdx.x == 1023) sBase += sScan[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.count[1] = sBase;
        a.count[3] = a.count[2];   // jobs with a change above tol (group-max rule)
        a.count[2] = 0;
    }
}

// Group-max rule, end of a segment's sweeps: every IC still in the group records the
// group's status (the sweep count, or -1 when max_iter sweeps did not converge).
__global__ void pc_plain_group_end(PcPlainArgs a, int s, int status)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.Mpad || !a.active[m]) return;
    a.active[m] = 0;
    if (status == -1) a.notconv[m] = 1;
    const PcJobDev job = a.jobs[m / a.T];
    const int i = (int)(m % a.T);
    if (i < job.n && a.p.iters_out) a.p.iters_out[(size_t)(job.ic0 + i) * a.p.iters_stride + s] = status;
}

// Segment end: the last node starts the next segment; optional node / boundary outputs.
__global__ void pc_plain_chain(PcPlainArgs a, int s, int last)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.Mpad) return;
    const PcJobDev job = a.jobs[m / a.T];
    const int i = (int)(m % a.T);
    const bool valid = i < job.n;
    const int64_t ic = job.ic0 + i;
    const size_t row = (size_t)9 * a.Mpad;
    if (valid && a.p.nodes_out) {
        for (int j = 0; j < a.N; ++j) {
            double* o = a.p.nodes_out + (((size_t)ic * a.p.iters_stride + s) * a.p.nodes_stride + j) * 6;
            for (int c = 0; c < 6; ++c) o[c] = a.Y[(size_t)j * row + (size_t)c * a.Mpad + m];
        }
    }
    const bool dead = a.dead[m];
    for (int c = 0; c < 6; ++c) {
        const double v = dead ? (double)NAN : a.Y[(size_t)(a.N - 1) * row + (size_t)c * a.Mpad + m];
        a.Y0[c * a.Mpad + m] = v;
        if (valid && a.p.bounds_out)
            a.p.bounds_out[((size_t)ic * (a.p.iters_stride + 1) + s + 1) * 6 + c] = v;
    }
    if (valid && last) {
        for (int c = 0; c < 6; ++c) a.p.states_out[(size_t)ic * 6 + c] = a.Y0[c * a.Mpad + m];
        if (a.notconv[m]) atomicAdd(&a.p.counters[0], 1);
        if (dead) atomicAdd(&a.p.counters[1], 1);
    }
}

__global__ void pc_plain_bounds0(PcPlainArgs a)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= a.Mpad || !a.p.bounds_out) return;
    const PcJobDev job = a.jobs[m / a.T];
    const int i = (int)(m % a.T);
    if (i >= job.n) return;
    for (int c = 0; c < 6; ++c)
        a.p.bounds_out[((size_t)(job.ic0 + i) * (a.p.iters_stride + 1)) * 6 + c] = a.Y0[c * a.Mpad + m];
}

template <int PAIRS, int NP>
void launch_step(const PcPlainArgs& a, int grid, int s, int it, double w2, hipStream_t st)
{
    hipLaunchKernelGGL((pc_plain_step<PAIRS, NP>), dim3(grid), dim3(PAIRS / 4), 0, st, a, s, it, w2);
}

int launch_step_np(const PcPlainArgs& a, int grid, int s, int it, double w2, hipStream_t st)
{
    switch (a.NP) {
    case 16: launch_step<2048, 16>(a, grid, s, it, w2, st); break;
    case 32: launch_step<2048, 32>(a, grid, s, it, w2, st); break;
    case 64: launch_step<2048, 64>(a, grid, s, it, w2, st); break;
    case 128: launch_step<2048, 128>(a, grid, s, it, w2, st); break;
    case 256: launch_step<2048, 256>(a, grid, s, it, w2, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

size_t pc_plain_bytes(int NP, int n_jobs, int T)
{
    const size_t Mpad = (size_t)n_jobs * T;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    return al(9 * (size_t)NP * Mpad * 8) + al(6 * Mpad * 8) + 4 * al(Mpad * 4) + 3 * al((size_t)n_jobs * 4) + 256;
}

namespace {

constexpr int kPlainBs = 256;

// One Picard iteration of the active jobs, then the read-back of the active-job count
// (and, for the group-max rule, of the jobs with a change above tol) that drives the
// host loop (Sec. 5.4.2).
hipError_t plain_enqueue_iteration(PcPlainRun& r)
{
    PcPlainArgs& a = r.a;
    hipStream_t st = (hipStream_t)r.stream;
    a.job_list = r.lists[r.cur];
    a.job_list_out = r.lists[1 - r.cur];
    const int bpj = a.NP * a.T / kPlainForceBlock;
    hipLaunchKernelGGL(pc_plain_force, dim3((unsigned)(r.count * bpj)), dim3(kPlainForceBlock), 0, st, a, r.s);
    hipError_t e = (hipError_t)launch_step_np(a, r.count, r.s, r.it, r.w2, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pc_plain_compact, dim3(1), dim3(1024), 0, st, a);
    e = hipMemcpyAsync(r.host, a.count + 1, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(a.count, a.count + 1, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
}

// Segment r.s: initial guess at every node, full job list, first iteration.
hipError_t plain_begin_segment(PcPlainRun& r)
{
    PcPlainArgs& a = r.a;
    hipStream_t st = (hipStream_t)r.stream;
    const double h = a.g_host.h;
    const double Ts = a.g_host.t0 + h * r.s, Te = a.g_host.t0 + h * (r.s + 1);
    r.w2 = 0.5 * (Te - Ts);
    r.cur = 0;
    a.job_list = r.lists[0];
    const int64_t total = (int64_t)a.NP * a.Mpad;
    hipLaunchKernelGGL(pc_plain_init, dim3((unsigned)((total + kPlainBs - 1) / kPlainBs)), dim3(kPlainBs), 0, st,
                       a, r.s, r.w2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    r.count = a.n_jobs;
    r.status = -1;
    r.it = 1;
    return plain_enqueue_iteration(r);
}

}  // namespace

int pc_plain_begin(PcPlainRun& r, const PcPlainArgs& args, void* workspace, int32_t* host_count, void* stream)
{
    r = PcPlainRun{};
    r.a = args;
    r.host = host_count;
    r.stream = stream;
    PcPlainArgs& a = r.a;
    hipStream_t st = (hipStream_t)stream;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    char* w = static_cast<char*>(workspace);
    a.Mpad = (int64_t)a.n_jobs * a.T;
    a.Y = reinterpret_cast<double*>(w);                w += al(9 * (size_t)a.NP * a.Mpad * 8);
    a.Y0 = reinterpret_cast<double*>(w);               w += al(6 * (size_t)a.Mpad * 8);
    a.active = reinterpret_cast<int32_t*>(w);          w += al(a.Mpad * 4);
    a.dead = reinterpret_cast<int32_t*>(w);            w += al(a.Mpad * 4);
    a.notconv = reinterpret_cast<int32_t*>(w);         w += al(a.Mpad * 4);
    a.valid = reinterpret_cast<int32_t*>(w);           w += al(a.Mpad * 4);
    r.lists[0] = reinterpret_cast<int32_t*>(w);        w += al((size_t)a.n_jobs * 4);
    r.lists[1] = reinterpret_cast<int32_t*>(w);        w += al((size_t)a.n_jobs * 4);
    a.job_flag = reinterpret_cast<int32_t*>(w);        w += al((size_t)a.n_jobs * 4);
    a.count = reinterpret_cast<int32_t*>(w);
    r.n_it = a.p.fixed_iters > 0 ? a.p.fixed_iters : a.p.max_iter;
    r.group = a.p.conv == PC_CONV_GROUP_MAX && a.p.fixed_iters == 0;

    const unsigned gm = (unsigned)((a.Mpad + kPlainBs - 1) / kPlainBs);
    hipLaunchKernelGGL(pc_plain_load, dim3(gm), dim3(kPlainBs), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pc_plain_bounds0, dim3(gm), dim3(kPlainBs), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return plain_begin_segment(r);
}

int pc_plain_advance(PcPlainRun& r)
{
    PcPlainArgs& a = r.a;
    hipStream_t st = (hipStream_t)r.stream;
    r.count = r.host[0];
    r.cur = 1 - r.cur;
    bool end = false;
    if (r.group && r.host[2] == 0) {   // group-max rule: no job holds a change above tol
        r.status = r.it;
        end = true;
    } else if (r.it >= r.n_it || r.count == 0) {
        end = true;
    }
    if (!end) {
        ++r.it;
        return plain_enqueue_iteration(r);
    }
    const unsigned gm = (unsigned)((a.Mpad + kPlainBs - 1) / kPlainBs);
    if (r.group) {
        hipLaunchKernelGGL(pc_plain_group_end, dim3(gm), dim3(kPlainBs), 0, st, a, r.s, r.status);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(pc_plain_chain, dim3(gm), dim3(kPlainBs), 0, st, a, r.s, r.s == a.S - 1 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (++r.s == a.S) {
        r.done = true;
        return hipSuccess;
    }
    return plain_begin_segment(r);
}

int pc_run_plain(PcPlainArgs a, void* workspace, int32_t* host_count, void* stream)
{
    PcPlainRun r;
    hipError_t e = (hipError_t)pc_plain_begin(r, a, workspace, host_count, stream);
    while (e == hipSuccess && !r.done) {
        e = hipStreamSynchronize((hipStream_t)stream);
        if (e == hipSuccess) e = (hipError_t)pc_plain_advance(r);
    }
    return e;
}
