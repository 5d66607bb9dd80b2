// pc_api.hip -- host side of the C ABI declared in include/pcprop.h.
//
// Plans a call (operators per node count, groups, jobs, ephemeris records), stages the
// descriptor tables in pinned host memory, copies them into the caller's workspace on
// the caller's stream and launches the kernels of pc_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "pcprop.h"
#include "pc_internal.h"
#include "pc_plain.h"

namespace {

constexpr int kMaxDevices = 64;

struct OperatorCache {
    int N = 0, NP = 0;
    double* kfrag = nullptr;   // device, [NP/16][NP/4][64]
    float* kfrag32 = nullptr;  // device, FP32 fragments in kfrag order
    float* kfrag32p = nullptr; // device, FP32 fragments with rows permuted per strip
    double* kfragT = nullptr;  // device, fragments of K_N^T
    double* kfrag2 = nullptr;  // device, fragments of K2_N
    double* tau = nullptr;     // device, [NP]
    std::vector<double> K;     // host copy, [N][N]
};

struct HostOperator {
    int N = 0, NP = 0;
    std::vector<double> K;        // [N][N]
    std::vector<double> frag;     // [NP/16][NP/4][64]
    std::vector<float> frag32;    // FP32, frag order
    std::vector<float> frag32p;   // FP32, rows permuted per strip
    std::vector<double> fragT;    // fragments of K_N^T
    std::vector<double> frag2;    // fragments of K2_N (second-order sweeps)
    std::vector<double> tau;      // [NP]
};

// Device memory of pc_propagate_batched_noalloc: the workspace of its calls (descriptor
// tables, kernel parameters, work-queue head and status counters, ephemeris records).
// Each device holds its own copy for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress returns for that device (scratch_address).
static __device__ __align__(256) char scratch[PC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mutex;
char* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

}  // namespace

struct pc_ctx {
    int device = 0;
    int n_cu = 256;
    std::map<int, OperatorCache> ops;
    std::map<int, HostOperator> host_ops;
    void* staging = nullptr;        // pinned host memory for descriptor tables
    size_t staging_bytes = 0;
    PcBodyDev* d_bodies = nullptr;  // device copy of the perturber table (test hooks)
    int32_t* pinned_count = nullptr;   // per-iteration read-back of the plain path
    // plain path on several streams (pc_opts.streams): one stream, read-back slot and
    // completion event per stream, created on first use
    hipStream_t pl_stream[PC_MAX_STREAMS] = {};
    hipEvent_t pl_done[PC_MAX_STREAMS] = {};
    hipEvent_t pl_poll[PC_MAX_STREAMS] = {};   // each stream's last read-back
    hipEvent_t pl_start = nullptr;
    int32_t* pl_count = nullptr;       // pinned, 16 ints per stream
    int pl_streams = 0;
    int tile_table[5] = {0, 0, 0, 0, 0}; // tuned job shape per padded node count 16..256 (0: default)
    int list_table[5] = {0, 0, 0, 0, 0}; // tuned job length (column blocks) per padded node count (0: default)
    hipStream_t cap_stream = nullptr;  // stream used to capture HIP graphs
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<char> graph_key;       // call signature of the captured graph
    int64_t graph_captures = 0;        // graphs captured so far (test hook)
    char* scratch = nullptr;           // this device's `scratch` (pc_propagate_batched_noalloc)
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = -1.0;
    char last_error[512] = {0};
};

namespace {

constexpr size_t kAlign = 256;
// pinned staging allocated with every context (grown by calls that need more)
constexpr size_t kStagingBytes = (size_t)4 << 20;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int set_error(pc_ctx* ctx, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int set_error(pc_ctx* ctx, int code, const char* fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->last_error, sizeof(ctx->last_error), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define PC_HIP(ctx, call)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return set_error(ctx, PC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)

// The same, for calls made after work has been queued on `sq`: the stream is drained
// first, so that no queued kernel can still write into the caller's buffers after the
// call has returned.
#define PC_HIP_DRAIN(ctx, sq, call)                                                           \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            (void)hipStreamSynchronize(sq);                                                   \
            return set_error(ctx, PC_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));  \
        }                                                                                     \
    } while (0)

int padded_nodes(int N)
{
    int np = 16;
    while (np < N) np <<= 1;
    return np;
}

// T_k at node j of the N-point CGL grid: tau_j = cos(pi (N-1-j)/(N-1)), so
// T_k(tau_j) = cos(pi k (N-1-j)/(N-1)), with the integer angle reduced exactly.
long double cheb_at_node(int k, int j, int N)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    long m = ((long)k * (long)(N - 1 - j)) % (2L * (N - 1));
    if (m > N - 1) m = 2L * (N - 1) - m;
    return cosl(pi * (long double)m / (long double)(N - 1));
}

// K_N such that y_j = y_0 + sum_l K_N[j][l] g_l (Sec. 2.2 with A, C, S folded):
// fit g with the degree N-2 Chebyshev series c_k = 2/(N-1) sum''_l g_l T_k(tau_l),
// integrate term by term, b_k = (c_{k-1} - c_{k+1})/(2k), and pin the constant so that
// y(tau = -1) = y_0, which leaves y_j - y_0 = sum_{k>=1} b_k (T_k(tau_j) - (-1)^k).
// Accumulated in long double, rounded once.
void build_operator(int N, std::vector<double>& K)
{
    std::vector<long double> D((size_t)(N + 1) * N, 0.0L);   // fit coefficients c_m per unit g_l
    for (int m = 0; m <= N - 2; ++m)
        for (int l = 0; l < N; ++l) {
            const long double w = (l == 0 || l == N - 1) ? 0.5L : 1.0L;
            D[(size_t)m * N + l] = 2.0L / (long double)(N - 1) * w * cheb_at_node(m, l, N);
        }
    std::vector<long double> Bc((size_t)N * N, 0.0L);        // integrated coefficients b_k per g_l
    for (int k = 1; k <= N - 1; ++k)
        for (int l = 0; l < N; ++l) {
            const long double lo = D[(size_t)(k - 1) * N + l];
            const long double up = (k + 1 <= N - 2) ? D[(size_t)(k + 1) * N + l] : 0.0L;
            Bc[(size_t)k * N + l] = (lo - up) / (2.0L * k);
        }
    K.assign((size_t)N * N, 0.0);
    std::vector<long double> E(N);
    for (int j = 1; j < N; ++j) {                              // row 0 is exactly zero
        for (int k = 1; k <= N - 1; ++k) E[k] = cheb_at_node(k, j, N) - ((k & 1) ? -1.0L : 1.0L);
        for (int l = 0; l < N; ++l) {
            long double s = 0.0L;
            for (int k = 1; k <= N - 1; ++k) s += E[k] * Bc[(size_t)k * N + l];
            K[(size_t)j * N + l] = (double)s;
        }
    }
}

// K2_N such that x_j = x_0 + w2 v_0 (tau_j + 1) + w2^2 sum_l K2_N[j][l] a_l for the
// accelerations a at the nodes (the second-order form of the method): the degree N-2 fit
// of build_operator, integrated once to the velocity series b (zero at tau = -1, constant
// b_0 = -2 sum_k (-1)^k b_k in the half-coefficient convention) and once more to the
// position series d_k = (b_{k-1} - b_{k+1}) / (2k), k = 1..N, pinned to zero at tau = -1.
// Accumulated in long double, rounded once.
void build_operator2(int N, std::vector<double>& K2)
{
    std::vector<long double> Tt((size_t)(N + 1) * N);   // T_k(tau_j), k = 0..N
    for (int k = 0; k <= N; ++k)
        for (int j = 0; j < N; ++j) Tt[(size_t)k * N + j] = cheb_at_node(k, j, N);
    std::vector<long double> c(N + 2), b(N + 2), d(N + 2);
    K2.assign((size_t)N * N, 0.0);
    for (int l = 0; l < N; ++l) {
        std::fill(c.begin(), c.end(), 0.0L);
        std::fill(b.begin(), b.end(), 0.0L);
        std::fill(d.begin(), d.end(), 0.0L);
        const long double w = (l == 0 || l == N - 1) ? 0.5L : 1.0L;
        for (int m = 0; m <= N - 2; ++m) c[m] = 2.0L / (long double)(N - 1) * w * Tt[(size_t)m * N + l];
        long double alt = 0.0L;
        for (int k = 1; k <= N - 1; ++k) {
            b[k] = (c[k - 1] - c[k + 1]) / (2.0L * k);
            alt += (k & 1) ? -b[k] : b[k];
        }
        b[0] = -2.0L * alt;
        for (int k = 1; k <= N; ++k) d[k] = (b[k - 1] - b[k + 1]) / (2.0L * k);
        for (int j = 1; j < N; ++j) {   // row 0 is exactly zero
            long double sx = 0.0L;
            for (int k = 1; k <= N; ++k) sx += d[k] * (Tt[(size_t)k * N + j] - ((k & 1) ? -1.0L : 1.0L));
            K2[(size_t)j * N + l] = (double)sx;
        }
    }
}

// Host copies of K_N and of its fragments in the kernels' layouts, built once per N.
const HostOperator& host_operator(pc_ctx* ctx, int N)
{
    auto it = ctx->host_ops.find(N);
    if (it != ctx->host_ops.end()) return it->second;
    HostOperator h;
    h.N = N;
    h.NP = padded_nodes(N);
    build_operator(N, h.K);
    const int NP = h.NP, NQ = NP / 4;
    h.frag.assign((size_t)NP * NP, 0.0);
    for (int strip = 0; strip < NP / 16; ++strip)
        for (int q = 0; q < NQ; ++q)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = 16 * strip + (lane & 15), col = 4 * q + (lane >> 4);
                h.frag[((size_t)strip * NQ + q) * 64 + lane] =
                    (row < N && col < N) ? h.K[(size_t)row * N + col] : 0.0;
            }
    // FP32 fragments.  frag32 has the frag order: it is the B operand of the transposed
    // product of jobs with 16 or more ICs.  frag32p serves the node-row layout of 8-IC
    // jobs: the f32 16x16x4 MFMA returns row 4(l/16) + r in element r, the f64 one row
    // l/16 + 4r, and feeding A row i from strip row perm(i) = (i/4) + 4 (i%4) puts the same
    // node in the same lane and element for both precisions.
    h.frag32.assign((size_t)NP * NP, 0.0f);
    for (size_t i = 0; i < h.frag.size(); ++i) h.frag32[i] = (float)h.frag[i];
    h.frag32p.assign((size_t)NP * NP, 0.0f);
    for (int strip = 0; strip < NP / 16; ++strip)
        for (int q = 0; q < NQ; ++q)
            for (int lane = 0; lane < 64; ++lane) {
                const int i = lane & 15;
                const int row = 16 * strip + (i / 4) + 4 * (i % 4), col = 4 * q + (lane >> 4);
                h.frag32p[((size_t)strip * NQ + q) * 64 + lane] =
                    (row < N && col < N) ? (float)h.K[(size_t)row * N + col] : 0.0f;
            }
    h.fragT.assign((size_t)NP * NP, 0.0);
    for (int strip = 0; strip < NP / 16; ++strip)
        for (int q = 0; q < NQ; ++q)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = 16 * strip + (lane & 15), col = 4 * q + (lane >> 4);   // of K_N^T
                h.fragT[((size_t)strip * NQ + q) * 64 + lane] =
                    (row < N && col < N) ? h.K[(size_t)col * N + row] : 0.0;
            }
    std::vector<double> K2;
    build_operator2(N, K2);
    h.frag2.assign((size_t)NP * NP, 0.0);
    for (int strip = 0; strip < NP / 16; ++strip)
        for (int q = 0; q < NQ; ++q)
            for (int lane = 0; lane < 64; ++lane) {
                const int row = 16 * strip + (lane & 15), col = 4 * q + (lane >> 4);
                h.frag2[((size_t)strip * NQ + q) * 64 + lane] =
                    (row < N && col < N) ? K2[(size_t)row * N + col] : 0.0;
            }
    h.tau.assign(NP, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < N; ++j) h.tau[j] = (double)(-cosl(pi * (long double)j / (long double)(N - 1)));
    return ctx->host_ops.emplace(N, std::move(h)).first->second;
}

int get_operator(pc_ctx* ctx, int N, const OperatorCache** out)
{
    auto it = ctx->ops.find(N);
    if (it != ctx->ops.end()) {
        *out = &it->second;
        return PC_OK;
    }
    const HostOperator& h = host_operator(ctx, N);
    OperatorCache oc;
    oc.N = N;
    oc.NP = h.NP;
    oc.K = h.K;
    PC_HIP(ctx, hipSetDevice(ctx->device));
    PC_HIP(ctx, hipMalloc(&oc.kfrag, h.frag.size() * sizeof(double)));
    PC_HIP(ctx, hipMalloc(&oc.tau, h.tau.size() * sizeof(double)));
    PC_HIP(ctx, hipMalloc(&oc.kfragT, h.fragT.size() * sizeof(double)));
    PC_HIP(ctx, hipMemcpy(oc.kfragT, h.fragT.data(), h.fragT.size() * sizeof(double), hipMemcpyHostToDevice));
    PC_HIP(ctx, hipMalloc(&oc.kfrag32, h.frag32.size() * sizeof(float)));
    PC_HIP(ctx, hipMemcpy(oc.kfrag32, h.frag32.data(), h.frag32.size() * sizeof(float), hipMemcpyHostToDevice));
    PC_HIP(ctx, hipMalloc(&oc.kfrag32p, h.frag32p.size() * sizeof(float)));
    PC_HIP(ctx, hipMemcpy(oc.kfrag32p, h.frag32p.data(), h.frag32p.size() * sizeof(float), hipMemcpyHostToDevice));
    PC_HIP(ctx, hipMemcpy(oc.kfrag, h.frag.data(), h.frag.size() * sizeof(double), hipMemcpyHostToDevice));
    PC_HIP(ctx, hipMemcpy(oc.tau, h.tau.data(), h.tau.size() * sizeof(double), hipMemcpyHostToDevice));
    PC_HIP(ctx, hipMalloc(&oc.kfrag2, h.frag2.size() * sizeof(double)));
    PC_HIP(ctx, hipMemcpy(oc.kfrag2, h.frag2.data(), h.frag2.size() * sizeof(double), hipMemcpyHostToDevice));
    auto res = ctx->ops.emplace(N, std::move(oc));
    *out = &res.first->second;
    return PC_OK;
}

// A captured graph copies its tables from the staging buffer it was captured with, so a
// reallocation of that buffer retires the graph (it is captured again on its next call).
void drop_graph(pc_ctx* ctx)
{
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_key.clear();
}

int ensure_staging(pc_ctx* ctx, size_t bytes)
{
    if (bytes <= ctx->staging_bytes) return PC_OK;
    drop_graph(ctx);
    if (ctx->staging) {
        PC_HIP(ctx, hipHostFree(ctx->staging));
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
    }
    size_t cap = std::max<size_t>(bytes, 1 << 20);
    PC_HIP(ctx, hipHostMalloc(&ctx->staging, cap, hipHostMallocDefault));
    ctx->staging_bytes = cap;
    return PC_OK;
}

// Streams, completion events and pinned read-back slots of the multi-stream plain path
// (default priority; created once, kept by the context).
int ensure_plain_streams(pc_ctx* ctx, int ns)
{
    if (!ctx->pl_start) PC_HIP(ctx, hipEventCreateWithFlags(&ctx->pl_start, hipEventDisableTiming));
    if (!ctx->pl_count) PC_HIP(ctx, hipHostMalloc(&ctx->pl_count, PC_MAX_STREAMS * 16 * sizeof(int32_t),
                                                  hipHostMallocDefault));
    for (; ctx->pl_streams < ns; ++ctx->pl_streams) {
        const int t = ctx->pl_streams;
        PC_HIP(ctx, hipStreamCreateWithFlags(&ctx->pl_stream[t], hipStreamNonBlocking));
        PC_HIP(ctx, hipEventCreateWithFlags(&ctx->pl_done[t], hipEventDisableTiming));
        PC_HIP(ctx, hipEventCreateWithFlags(&ctx->pl_poll[t], hipEventDisableTiming));
    }
    return PC_OK;
}

// Device address of `scratch` on the context's device (current when this runs), looked
// up once per device and kept for every later context on it.
int scratch_address(pc_ctx* ctx, char** out)
{
    *out = nullptr;
    if (ctx->device >= kMaxDevices)
        return set_error(ctx, PC_EINVAL, "device %d: the static scratch is kept for devices 0..%d",
                         ctx->device, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[ctx->device]) {
        void* p = nullptr;
        PC_HIP(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(ctx, PC_EHIP, "hipGetSymbolAddress returned no address for the scratch");
        g_scratch_ptr[ctx->device] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[ctx->device];
    return PC_OK;
}

int validate_model(pc_ctx* ctx, const pc_model* model)
{
    if (!model) return set_error(ctx, PC_EINVAL, "model is NULL");
    if (!(model->mu_sun > 0.0) || !std::isfinite(model->mu_sun))
        return set_error(ctx, PC_EINVAL, "mu_sun must be positive and finite");
    if (model->n_pert < 0 || model->n_pert > PC_MAX_PERT)
        return set_error(ctx, PC_EINVAL, "n_pert must be in [0, %d]", PC_MAX_PERT);
    if (model->n_pert > 0 && !model->pert) return set_error(ctx, PC_EINVAL, "pert is NULL");
    if (!std::isfinite(model->epoch)) return set_error(ctx, PC_EINVAL, "epoch not finite");
    if (!(model->inv_c2 >= 0.0) || !std::isfinite(model->inv_c2))
        return set_error(ctx, PC_EINVAL, "inv_c2 must be >= 0 and finite");
    for (int p = 0; p < model->n_pert; ++p) {
        const double* el = model->pert + 7 * p;
        for (int k = 0; k < 7; ++k)
            if (!std::isfinite(el[k])) return set_error(ctx, PC_EINVAL, "perturber %d: non-finite element", p);
        if (!(el[0] >= 0.0)) return set_error(ctx, PC_EINVAL, "perturber %d: mu must be >= 0", p);
        if (!(el[1] > 0.0)) return set_error(ctx, PC_EINVAL, "perturber %d: a must be > 0", p);
        if (!(el[2] >= 0.0 && el[2] < 1.0)) return set_error(ctx, PC_EINVAL, "perturber %d: e must be in [0,1)", p);
    }
    return PC_OK;
}

// Orientation of each perturber's orbit, prepared once per call (plan step).
void prepare_bodies(const pc_model* model, PcBodyDev* out)
{
    for (int p = 0; p < model->n_pert; ++p) {
        const double* el = model->pert + 7 * p;
        const double a = el[1], e = el[2], inc = el[3], raan = el[4], argp = el[5];
        PcBodyDev& B = out[p];
        B.mu = el[0];
        B.a = a;
        B.e = e;
        B.n = std::sqrt(1.0 / (a * a * a));
        B.M0 = el[6];
        B.b = a * std::sqrt(1.0 - e * e);
        const double cO = std::cos(raan), sO = std::sin(raan), cw = std::cos(argp), sw = std::sin(argp);
        const double ci = std::cos(inc), si = std::sin(inc);
        B.P[0] = cO * cw - sO * sw * ci;
        B.P[1] = sO * cw + cO * sw * ci;
        B.P[2] = sw * si;
        B.Q[0] = -cO * sw - sO * cw * ci;
        B.Q[1] = -sO * sw + cO * cw * ci;
        B.Q[2] = cw * si;
    }
}

struct JobClass {
    int np, begin, end;
};

struct Plan {
    int pairs = 2048;
    bool plain = false;
    std::vector<JobClass> classes;
    std::vector<int> group_job_begin;   // plain path: jobs of group g are [begin[g], begin[g+1])
    size_t off_plain = 0;
    std::vector<PcGroupDev> groups;
    std::vector<PcJobDev> jobs;
    int64_t n_recs = 0;
    int max_S = 0, max_N = 0;
    int list = 1;                  // job ICs in units of the job's columns (untuned node counts)
    // workspace offsets
    size_t off_counters = 0, off_params = 0, off_groups = 0, off_jobs = 0, off_bodies = 0, off_recs = 0, total = 0;
    size_t off_recs_eih = 0;   // relativistic model: per-node states of the major bodies
    size_t plain_stride = 0;   // bytes of one plain-path state (one per stream)
    int plain_streams = 1;
    size_t staged = 0;   // bytes of [counters .. bodies] copied from the staging buffer
    // adaptive refinement (opts.refine > 0): a region after the call's own, holding the
    // sub-calls' inputs and outputs, copy descriptors and workspace
    size_t off_refine = 0, ref_ics = 0, ref_states = 0, ref_iters = 0, ref_bounds = 0, ref_copies = 0,
           ref_sub = 0, ref_sub_cap = 0;
    int refine_smax = 0;          // segment stride of the sub-calls' records
    int64_t refine_budget = 0;    // ephemeris records one refinement pass may plan
    // flyby isolation (opts.flyby_hill > 0): a region after the call's own, holding the
    // screen's ratios, the reordered copy of the ICs and outputs, copy descriptors and the
    // reordered call's workspace
    size_t off_flyby = 0, fly_ratio = 0, fly_ics = 0, fly_states = 0, fly_iters = 0, fly_bounds = 0, fly_copies = 0,
           fly_sub = 0, fly_sub_cap = 0;
    int64_t fly_span = 0, fly_cov = 0;   // ICs indexed by the groups (0 .. span-1), ICs in them
};

constexpr int kFlybySamples = 16;   // screen points per segment of opts.flyby_hill

// Tasks of one refinement pass at most (the pass's buffers are sized for this many).
constexpr int64_t kRefineChunk = 8192;

int log2_index(int np)
{
    int k = 0;
    while ((16 << k) < np) ++k;
    return k;   // 16 -> 0 ... 256 -> 4
}

int choose_pairs(const pc_ctx* ctx, const pc_group* groups, int n_groups, const pc_opts& o)
{
    if (o.tile_pairs == 1024 || o.tile_pairs == 2048) return o.tile_pairs;
    int np_max = 16;
    for (int i = 0; i < n_groups; ++i) np_max = std::max(np_max, padded_nodes(groups[i].nodes));
    // untuned default: the 256-thread shape up to 64 padded nodes, where two of its
    // workgroups share a CU and overlap their jobs (about 9 % faster at 64 nodes than one
    // 512-thread workgroup per CU); the 512-thread shape above, where its transposed
    // 16-IC blocks beat the 8-IC node-row blocks of the small shape
    const int tuned = ctx->tile_table[log2_index(np_max)];
    const int pick = tuned != 0 ? tuned : (np_max <= 64 ? 1024 : 2048);
    if (pick == 1024 && np_max * 8 <= 1024) return 1024;
    return 2048;
}

// lists_ok: jobs may hold more ICs than columns (refilled columns; fused FP64 forward calls).
// A plan without lists has the most jobs, so its workspace size bounds every other plan's.
// cached_only: take the operators from the context's cache and fail where one is missing
// (the allocation-free entry point builds none).
// seg0 (or null): per group, the first segment to run on its t0 + k h grid (refinement
// passes resume a span at a segment boundary); the group then runs segments - seg0[g].
int make_plan(pc_ctx* ctx, int64_t n_ic, const pc_group* groups, int n_groups, const pc_model* model,
              const pc_opts& o, bool build_tables, Plan& plan, bool lists_ok = false, bool cached_only = false,
              const int* seg0 = nullptr)
{
    if (!groups || n_groups < 1) return set_error(ctx, PC_EINVAL, "need at least one group");
    if (o.tile_pairs != 0 && o.tile_pairs != 1024 && o.tile_pairs != 2048)
        return set_error(ctx, PC_EINVAL, "tile_pairs must be 0, 1024 or 2048");
    plan.pairs = choose_pairs(ctx, groups, n_groups, o);
    plan.plain = (o.path == PC_PATH_PLAIN);
    if (plan.plain) plan.pairs = 2048;
    if (o.order == 2) {
        // second-order sweeps need blocks of 16 or more ICs (the transposed product) up to
        // 128 nodes; 256-node groups run 8-IC node-row jobs
        for (int gi = 0; gi < n_groups; ++gi) {
            const int np = padded_nodes(std::max(3, std::min((int)groups[gi].nodes, PC_MAX_NODES)));
            if (np > 128) continue;
            if (plan.pairs / np < 16) {
                if (o.tile_pairs == 1024) return set_error(ctx, PC_EINVAL, "order 2 with %d nodes needs tile_pairs 2048", groups[gi].nodes);
                plan.pairs = 2048;
            }
        }
    }
    std::vector<std::pair<int64_t, int64_t>> spans;
    plan.groups.clear();
    plan.jobs.clear();
    plan.n_recs = 0;
    plan.max_S = plan.max_N = 0;
    for (int gi = 0; gi < n_groups; ++gi) {
        const pc_group& G = groups[gi];
        if (G.n_ic < 1) return set_error(ctx, PC_EINVAL, "group %d: n_ic < 1", gi);
        if (G.ic_offset < 0 || G.ic_offset + G.n_ic > n_ic)
            return set_error(ctx, PC_EINVAL, "group %d: ICs out of range", gi);
        if (G.nodes < 3 || G.nodes > PC_MAX_NODES)
            return set_error(ctx, PC_EINVAL, "group %d: nodes must be in [3, %d]", gi, PC_MAX_NODES);
        if (G.segments < 1) return set_error(ctx, PC_EINVAL, "group %d: segments < 1", gi);
        if (seg0 && (seg0[gi] < 0 || seg0[gi] >= G.segments))
            return set_error(ctx, PC_EINVAL, "group %d: first segment out of range", gi);
        if (!std::isfinite(G.t0) || !std::isfinite(G.tf) || G.t0 == G.tf)
            return set_error(ctx, PC_EINVAL, "group %d: need finite t0 != tf", gi);
        if (!(G.tol > 0.0) || !std::isfinite(G.tol))
            return set_error(ctx, PC_EINVAL, "group %d: tol must be positive and finite", gi);
        const int NP = padded_nodes(G.nodes);
        if (NP * 8 > plan.pairs)
            return set_error(ctx, PC_EINVAL, "group %d: %d nodes need tile_pairs >= %d", gi, G.nodes, NP * 8);
        spans.push_back({G.ic_offset, G.ic_offset + G.n_ic});
        plan.max_S = std::max(plan.max_S, G.segments - (seg0 ? seg0[gi] : 0));
        plan.max_N = std::max(plan.max_N, G.nodes);
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return set_error(ctx, PC_EINVAL, "groups overlap");

    // ICs per job in units of the job's columns (1, 2, 4 or 8 blocks).  Longer jobs refill
    // their columns for longer, so fewer columns idle in segment tails (on 16384 eccentric
    // ICs, one 8-block job per CU beat eight one-block jobs per CU by about 10 % at 256
    // nodes), but the queue hands out whole jobs: J jobs of m blocks on S workgroup slots
    // take up to ceil(J / S) m block-times.  The choice is the longest jobs whose bound is
    // within 25 % of the best one (the bound is loose when jobs of several groups, sorted
    // longest first, fill each other's gaps: on the uneven 65536-IC batch 8-block jobs,
    // 20 % above the bound of 1-, 2- and 4-block ones, ran fastest).  A rule that only
    // asked for a job per CU gave 270 two-block jobs to 256 CUs for 539 blocks (34 %
    // slower than one-block jobs) and counted one slot per CU where the 1024-pair shape
    // has two (25 % slower at 64 nodes).
    int list = 1;
    if (lists_ok && o.job_list != 1) {
        auto jobs_at = [&](int m) {
            int64_t nj = 0;
            for (int gi = 0; gi < n_groups; ++gi) {
                const int64_t cols = (int64_t)m * (plan.pairs / padded_nodes(groups[gi].nodes));
                nj += (groups[gi].n_ic + cols - 1) / cols;
            }
            return nj;
        };
        if (o.job_list > 1) list = o.job_list;
        else {
            int occ = 1;
            if (pc_fused_occupancy(plan.pairs, &occ) != 0 || occ < 1) occ = 1;
            const int64_t slots = (int64_t)ctx->n_cu * occ;
            int64_t span[4], best = 0;
            for (int k = 0; k < 4; ++k) {
                span[k] = (jobs_at(1 << k) + slots - 1) / slots * (1 << k);
                best = k == 0 ? span[0] : std::min(best, span[k]);
            }
            for (int k = 0; k < 4; ++k)
                if (4 * span[k] <= 5 * best) list = 1 << k;
        }
    }
    // per padded node count: the autotuner's job length where it has tuned one (automatic
    // calls only), else the call's
    int list_np[5];
    for (int k = 0; k < 5; ++k) {
        list_np[k] = list;
        if (lists_ok && o.job_list == 0 && ctx->list_table[k] != 0) list_np[k] = ctx->list_table[k];
    }
    plan.list = list;
    struct Cost { int np; double c; PcJobDev j; };
    std::vector<Cost> costs;
    for (int gi = 0; gi < n_groups; ++gi) {
        const pc_group& G = groups[gi];
        PcGroupDev d{};
        d.t0 = G.t0;
        d.h = (G.tf - G.t0) / (double)G.segments;
        d.tol = G.tol;
        d.ic_offset = G.ic_offset;
        d.n_ic = G.n_ic;
        d.rec_offset = plan.n_recs;
        d.N = G.nodes;
        d.NP = padded_nodes(G.nodes);
        d.T = plan.pairs / d.NP;
        d.s0 = seg0 ? seg0[gi] : 0;
        d.S = G.segments - d.s0;
        if (build_tables) {
            const OperatorCache* oc = nullptr;
            if (cached_only && ctx->ops.find(G.nodes) == ctx->ops.end())
                return set_error(ctx, PC_EINVAL,
                                 "the operators of %d nodes are not built in this context yet (a call of "
                                 "pc_propagate_batched with that node count builds them)", G.nodes);
            int rc = get_operator(ctx, G.nodes, &oc);
            if (rc != PC_OK) return rc;
            d.kfrag = oc->kfrag;
            d.kfrag32 = oc->kfrag32;
            d.kfrag32p = oc->kfrag32p;
            d.kfragT = oc->kfragT;
            d.kfrag2 = oc->kfrag2;
            d.tau = oc->tau;
        }
        plan.n_recs += (int64_t)d.S * G.nodes;
        plan.groups.push_back(d);
        // cost model of one job: segments x NP x column blocks (matrix work per iteration
        // ~ NP^2 T = NP * PAIRS per block)
        const int64_t per_job = (int64_t)list_np[log2_index(d.NP)] * d.T;
        for (int64_t i0 = 0; i0 < G.n_ic; i0 += per_job) {
            PcJobDev j{};
            j.ic0 = G.ic_offset + i0;
            j.group = gi;
            j.n = (int)std::min<int64_t>(per_job, G.n_ic - i0);
            const double c = (double)d.S * (double)d.NP * (double)((j.n + d.T - 1) / d.T);
            costs.push_back({d.NP, c, j});
        }
    }
    // fused: one queue over all jobs, longest first (the persistent workgroups then fill
    // the tail with short jobs).  plain: group-major, IC order.
    if (!plan.plain)
        std::stable_sort(costs.begin(), costs.end(), [](const Cost& a, const Cost& b) { return a.c > b.c; });
    plan.group_job_begin.assign(n_groups + 1, 0);
    for (const Cost& c : costs) plan.group_job_begin[c.j.group + 1] += plan.plain ? 1 : 0;
    for (int gi = 0; gi < n_groups; ++gi) plan.group_job_begin[gi + 1] += plan.group_job_begin[gi];
    plan.classes.clear();
    for (size_t i = 0; i < costs.size(); ++i) {
        if (plan.classes.empty() || plan.classes.back().np != costs[i].np)
            plan.classes.push_back({costs[i].np, (int)i, (int)i});
        plan.classes.back().end = (int)i + 1;
        plan.jobs.push_back(costs[i].j);
    }

    const int P = model->n_pert;
    size_t off = 0;
    plan.off_counters = off; off = align_up(off + 4 * sizeof(int32_t));   // 2 counters + queue head
    plan.off_params = off;   off = align_up(off + std::max(sizeof(PcParams), sizeof(PcAdjParams)));
    plan.off_groups = off;   off = align_up(off + plan.groups.size() * sizeof(PcGroupDev));
    plan.off_jobs = off;     off = align_up(off + plan.jobs.size() * sizeof(PcJobDev));
    plan.off_bodies = off;   off = align_up(off + std::max(1, P) * sizeof(PcBodyDev));
    plan.staged = off;
    plan.off_recs = off;     off = align_up(off + (size_t)plan.n_recs * (P + 1) * 4 * sizeof(double));
    plan.off_recs_eih = off;
    if (model->inv_c2 > 0.0) off = align_up(off + (size_t)plan.n_recs * (3 * (P + 1) + 1) * 4 * sizeof(double));
    plan.off_plain = off;
    if (plan.plain) {
        size_t mx = 0;
        for (int gi = 0; gi < n_groups; ++gi) {
            const PcGroupDev& d = plan.groups[gi];
            const int nj = plan.group_job_begin[gi + 1] - plan.group_job_begin[gi];
            mx = std::max(mx, pc_plain_bytes(d.NP, nj, d.T));
        }
        plan.plain_streams = std::min(std::max(1, (int)o.streams), n_groups);
        plan.plain_stride = align_up(mx);
        off = align_up(off + plan.plain_stride * plan.plain_streams);
    }
    plan.total = off;
    if (o.refine > 0 && !plan.plain) {
        // region of the refinement passes: up to kRefineChunk tasks per pass, each pass
        // planning at most refine_budget ephemeris records (enough for the longest single
        // task: a whole group's span, or one segment split 2^refine ways)
        const int parts = 1 << o.refine;
        plan.refine_smax = std::max(plan.max_S, parts);
        plan.refine_budget = plan.n_recs;
        for (int gi = 0; gi < n_groups; ++gi)
            plan.refine_budget = std::max<int64_t>(plan.refine_budget,
                                                   (int64_t)std::max((int)groups[gi].segments, parts) * groups[gi].nodes);
        const int64_t C = kRefineChunk;
        size_t r = 0;
        plan.ref_ics = r;    r = align_up(r + (size_t)C * 6 * sizeof(double));
        plan.ref_states = r; r = align_up(r + (size_t)C * 6 * sizeof(double));
        plan.ref_iters = r;  r = align_up(r + (size_t)C * plan.refine_smax * sizeof(int32_t));
        plan.ref_bounds = r; r = align_up(r + (size_t)C * (plan.refine_smax + 1) * 6 * sizeof(double));
        plan.ref_copies = r; r = align_up(r + (size_t)2 * C * sizeof(PcCopyDev));
        plan.ref_sub = r;
        size_t rec_bytes = (size_t)(P + 1) * 4 * sizeof(double);
        if (model->inv_c2 > 0.0) rec_bytes += (size_t)(3 * (P + 1) + 1) * 4 * sizeof(double);
        plan.ref_sub_cap = 8 * kAlign + 4 * sizeof(int32_t) + std::max(sizeof(PcParams), sizeof(PcAdjParams)) +
                           (size_t)C * (sizeof(PcGroupDev) + sizeof(PcJobDev)) + std::max(1, P) * sizeof(PcBodyDev) +
                           (size_t)plan.refine_budget * rec_bytes;
        r = align_up(r + plan.ref_sub_cap);
        plan.off_refine = plan.total;
        plan.total += r;
    }
    if (o.flyby_hill > 0.0) {
        // sizes of the reordered call: every group split at worst into two (one more group
        // and job per group, each part with its own ephemeris records)
        std::vector<pc_group> split;
        int64_t cov = 0, span = 0;
        for (int gi = 0; gi < n_groups; ++gi) {
            pc_group a = groups[gi];
            span = std::max<int64_t>(span, a.ic_offset + a.n_ic);
            a.ic_offset = cov;
            if (a.n_ic >= 2) {
                pc_group b = a;
                a.n_ic -= 1;
                b.ic_offset = cov + a.n_ic;
                b.n_ic = 1;
                split.push_back(a);
                split.push_back(b);
            } else {
                split.push_back(a);
            }
            cov += groups[gi].n_ic;
        }
        pc_opts oi = o;
        oi.flyby_hill = 0.0;
        Plan inner;
        int rc = make_plan(ctx, cov, split.data(), (int)split.size(), model, oi, false, inner, lists_ok);
        if (rc != PC_OK) return rc;
        const int S = plan.max_S;
        size_t r = 0;
        plan.fly_ratio = r;  r = align_up(r + (size_t)span * sizeof(double));
        plan.fly_ics = r;    r = align_up(r + (size_t)cov * 6 * sizeof(double));
        plan.fly_states = r; r = align_up(r + (size_t)cov * 6 * sizeof(double));
        plan.fly_iters = r;  r = align_up(r + (size_t)cov * S * sizeof(int32_t));
        plan.fly_bounds = r; r = align_up(r + (size_t)cov * (S + 1) * 6 * sizeof(double));
        plan.fly_copies = r; r = align_up(r + (size_t)3 * cov * sizeof(PcCopyDev));
        plan.fly_sub = r;
        plan.fly_sub_cap = inner.total;
        r = align_up(r + inner.total);
        plan.fly_span = span;
        plan.fly_cov = cov;
        plan.off_flyby = plan.total;
        plan.total += r;
    }
    return PC_OK;
}

// Options of a forward call.
int validate_forward(pc_ctx* ctx, const pc_opts& o, const pc_model* model)
{
    if (o.init != PC_INIT_KEPLER && o.init != PC_INIT_COLD && o.init != PC_INIT_GUESS)
        return set_error(ctx, PC_EINVAL, "bad init");
    if ((o.init == PC_INIT_GUESS) != (o.guess != nullptr))
        return set_error(ctx, PC_EINVAL, "init PC_INIT_GUESS needs a guess buffer, and only it takes one");
    if (o.tol_mode != PC_TOL_REL && o.tol_mode != PC_TOL_ABS) return set_error(ctx, PC_EINVAL, "bad tol_mode");
    if (o.precision != PC_FP64 && o.precision != PC_FP32_THEN_FP64)
        return set_error(ctx, PC_EINVAL, "unsupported precision");
    if (o.precision == PC_FP32_THEN_FP64 && o.path != PC_PATH_FUSED)
        return set_error(ctx, PC_EINVAL, "the FP32 -> FP64 schedule runs on the fused path");
    if (o.path != PC_PATH_FUSED && o.path != PC_PATH_PLAIN) return set_error(ctx, PC_EINVAL, "bad path");
    if (o.max_iter < 1 || o.max_iter > 100000) return set_error(ctx, PC_EINVAL, "max_iter out of range");
    if (!(o.switch_tol >= 0.0) || !std::isfinite(o.switch_tol) || o.max_fp32 < 0)
        return set_error(ctx, PC_EINVAL, "bad precision-schedule options");
    if (o.job_list != 0 && o.job_list != 1 && o.job_list != 2 && o.job_list != 4 && o.job_list != 8)
        return set_error(ctx, PC_EINVAL, "job_list must be 0, 1, 2, 4 or 8");
    if (o.fixed_iters < 0 || o.fixed_iters > 100000) return set_error(ctx, PC_EINVAL, "fixed_iters out of range");
    if (o.conv != PC_CONV_PER_IC && o.conv != PC_CONV_GROUP_MAX) return set_error(ctx, PC_EINVAL, "bad conv");
    if (o.conv == PC_CONV_GROUP_MAX && o.path != PC_PATH_PLAIN)
        return set_error(ctx, PC_EINVAL, "group-max convergence runs on the plain path");
    if (o.streams < 0 || o.streams > PC_MAX_STREAMS || (o.streams > 1 && o.path != PC_PATH_PLAIN))
        return set_error(ctx, PC_EINVAL, "streams must be 1..%d, and above 1 only on the plain path",
                         PC_MAX_STREAMS);
    if (model->inv_c2 > 0.0 && o.conv != PC_CONV_PER_IC)
        return set_error(ctx, PC_EINVAL, "the relativistic model runs with the per-IC stopping rule");
    if (o.order != 1 && o.order != 2) return set_error(ctx, PC_EINVAL, "order must be 1 or 2");
    if (o.feedback != 0 && o.feedback != 1) return set_error(ctx, PC_EINVAL, "feedback must be 0 or 1");
    if (o.feedback && o.order != 2) return set_error(ctx, PC_EINVAL, "feedback needs order 2");
    if (o.order == 2 && (o.path != PC_PATH_FUSED || o.precision != PC_FP64 || model->inv_c2 > 0.0 ||
                         o.conv != PC_CONV_PER_IC))
        return set_error(ctx, PC_EINVAL, "order 2 runs on the fused FP64 path, point masses, per-IC rule");
    if (o.refine < 0 || o.refine > 8) return set_error(ctx, PC_EINVAL, "refine must be 0..8");
    if (!(o.flyby_hill >= 0.0) || !std::isfinite(o.flyby_hill))
        return set_error(ctx, PC_EINVAL, "flyby_hill must be >= 0 and finite");
    if (o.flyby_hill > 0.0 && (o.refine > 0 || o.init == PC_INIT_GUESS || o.graph))
        return set_error(ctx, PC_EINVAL, "flyby isolation runs without refinement, a guess or graph capture");
    if (o.refine > 0 && (o.path != PC_PATH_FUSED || o.init == PC_INIT_GUESS))
        return set_error(ctx, PC_EINVAL, "refinement runs on the fused path and without a guess");
    return PC_OK;
}

// Stage the call's tables [counters | params | groups | jobs | bodies] in the pinned
// staging buffer (zeroed counters and queue head, so that the one host-to-device copy of
// this region also clears them) and describe the call for the kernels, whose tables live
// at device address `base` (the caller's workspace).
void stage_call(pc_ctx* ctx, const Plan& plan, const pc_model* model, const pc_opts& o, char* base,
                const double* ics, double* states_out, int32_t* iters_out, int32_t iters_stride,
                double* bounds_out, double* nodes_out, int32_t nodes_stride, PcEphemParams& ep, PcParams& pp)
{
    const bool eih = model->inv_c2 > 0.0;
    char* st = static_cast<char*>(ctx->staging);
    std::memset(st, 0, plan.staged);
    std::memcpy(st + plan.off_groups, plan.groups.data(), plan.groups.size() * sizeof(PcGroupDev));
    std::memcpy(st + plan.off_jobs, plan.jobs.data(), plan.jobs.size() * sizeof(PcJobDev));
    prepare_bodies(model, reinterpret_cast<PcBodyDev*>(st + plan.off_bodies));

    ep = PcEphemParams{};
    ep.groups = reinterpret_cast<const PcGroupDev*>(base + plan.off_groups);
    ep.n_groups = (int)plan.groups.size();
    ep.n_recs = plan.n_recs;
    ep.bodies = reinterpret_cast<const PcBodyDev*>(base + plan.off_bodies);
    ep.n_pert = model->n_pert;
    ep.epoch = model->epoch;
    ep.recs = reinterpret_cast<double*>(base + plan.off_recs);
    ep.recs_eih = eih ? reinterpret_cast<double*>(base + plan.off_recs_eih) : nullptr;
    ep.mu_sun = model->mu_sun;

    pp = PcParams{};
    pp.groups = ep.groups;
    pp.jobs = reinterpret_cast<const PcJobDev*>(base + plan.off_jobs);
    pp.n_jobs = (int)plan.jobs.size();
    pp.n_pert = model->n_pert;
    pp.ics = ics;
    pp.states_out = states_out;
    pp.iters_out = iters_out;
    pp.iters_stride = iters_stride;
    pp.nodes_stride = nodes_stride;
    pp.bounds_out = bounds_out;
    pp.nodes_out = nodes_out;
    pp.recs = ep.recs;
    pp.mu_sun = model->mu_sun;
    pp.recs_eih = ep.recs_eih;
    pp.inv_c2 = eih ? model->inv_c2 : 0.0;
    pp.max_iter = o.max_iter;
    pp.fixed_iters = o.fixed_iters;
    pp.tol_mode = o.tol_mode;
    pp.conv = o.conv;
    pp.init = o.init;
    pp.guess = o.guess;
    pp.precision = o.precision;
    pp.order = o.order;
    pp.feedback = o.feedback;
    pp.max_fp32 = o.max_fp32 > 0 ? o.max_fp32 : 24;
    pp.switch2 = o.switch_tol * o.switch_tol;   // 0: the kernel's default for the job's sweep kind
    pp.counters = reinterpret_cast<int32_t*>(base + plan.off_counters);
    pp.queue = pp.counters + 2;
    std::memcpy(st + plan.off_params, &pp, sizeof(pp));   // the device copy the kernel reads
}

// Adaptive segment refinement after a fused call (opts.refine > 0), on the call's stream.
// A segment that ended PC_ITER_NOTCONV is solved again from its initial state (its
// boundary record) as 2, then 4, ... up to 2^refine equal sub-segments, until all of them
// converge (each a complete segment solve: own warm start, own sweeps); it then records
// the sum of their sweep counts (or PC_ITER_NOTCONV with the finest split's end state).
// The rest of the span is run again from the new boundary, on the original segment grid,
// and its first failing segment, if any, is refined in turn.  Tasks of one kind, group and
// segment run as one group of a sub-call; one pass is one fused launch over up to
// kRefineChunk tasks.  iters_out and bounds_out hold the call's records and are rewritten.
// Returns the call's status from the final records.
int refine_passes(pc_ctx* ctx, const Plan& plan, const pc_group* groups, int n_groups, const pc_model* model,
                  const pc_opts& o, bool lists_ok, char* ws, int64_t n_ic, double* states_out, int32_t* iters_out,
                  int32_t stride, double* bounds_out, hipStream_t hs)
{
    struct Task {
        int64_t m;   // IC
        int g;       // group
        int s;       // segment
        int depth;   // > 0: split segment s into 2^depth parts; 0: run segments s.. to the end
    };
    const int smax = plan.refine_smax;
    char* R = ws + plan.off_refine;
    double* ics_sub = reinterpret_cast<double*>(R + plan.ref_ics);
    double* states_sub = reinterpret_cast<double*>(R + plan.ref_states);
    int32_t* iters_sub = reinterpret_cast<int32_t*>(R + plan.ref_iters);
    double* bounds_sub = reinterpret_cast<double*>(R + plan.ref_bounds);
    PcCopyDev* copies_dev = reinterpret_cast<PcCopyDev*>(R + plan.ref_copies);
    char* sub_ws = R + plan.ref_sub;

    std::vector<int32_t> it((size_t)n_ic * stride);
    PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(it.data(), iters_out, it.size() * sizeof(int32_t), hipMemcpyDeviceToHost, hs));
    PC_HIP(ctx, hipStreamSynchronize(hs));
    std::vector<Task> pending;
    // the first failing segment of every IC (none after a non-finite one)
    auto first_failure = [&](int64_t m, int gi, int from) {
        for (int s = from; s < groups[gi].segments; ++s) {
            const int32_t v = it[(size_t)m * stride + s];
            if (v == PC_ITER_NONFINITE) return;
            if (v == PC_ITER_NOTCONV) {
                pending.push_back({m, gi, s, 1});
                return;
            }
        }
    };
    for (int gi = 0; gi < n_groups; ++gi)
        for (int64_t m = groups[gi].ic_offset; m < groups[gi].ic_offset + groups[gi].n_ic; ++m) first_failure(m, gi, 0);

    pc_opts so = o;
    so.refine = 0;
    so.graph = 0;
    int occ = 0;
    std::vector<int32_t> its;
    std::vector<PcCopyDev> cp;
    while (!pending.empty()) {
        std::stable_sort(pending.begin(), pending.end(), [](const Task& a, const Task& b) {
            if (a.g != b.g) return a.g < b.g;
            if (a.s != b.s) return a.s < b.s;
            return a.depth < b.depth;
        });
        std::vector<pc_group> sg;
        std::vector<int> s0;
        std::vector<Task> pass;
        int64_t recs = 0;
        size_t take = 0;
        for (size_t i = 0; i < pending.size() && (int64_t)pass.size() < kRefineChunk; ++i) {
            const Task& t = pending[i];
            const pc_group& G = groups[t.g];
            const bool fresh = pass.empty() || t.g != pass.back().g || t.s != pass.back().s ||
                               t.depth != pass.back().depth;
            if (fresh) {
                const int segs = t.depth > 0 ? (1 << t.depth) : G.segments - t.s;
                const int64_t r = (int64_t)segs * G.nodes;
                if (!pass.empty() && recs + r > plan.refine_budget) break;
                recs += r;
                pc_group q = G;
                q.ic_offset = (int64_t)pass.size();
                q.n_ic = 0;
                if (t.depth > 0) {   // segment s alone, split; its ends as the oracle forms them
                    const double h = (G.tf - G.t0) / (double)G.segments;
                    q.t0 = G.t0 + h * t.s;
                    q.tf = G.t0 + h * (t.s + 1);
                    q.segments = segs;
                    s0.push_back(0);
                } else {             // segments s.. of the group's own grid
                    s0.push_back(t.s);
                }
                sg.push_back(q);
            }
            pass.push_back(t);
            ++sg.back().n_ic;
            take = i + 1;
        }
        pending.erase(pending.begin(), pending.begin() + take);
        const int64_t np = (int64_t)pass.size();

        Plan sub;
        int rc = make_plan(ctx, np, sg.data(), (int)sg.size(), model, so, true, sub, lists_ok, false, s0.data());
        if (rc != PC_OK) return rc;
        if (sub.total > plan.ref_sub_cap)
            return set_error(ctx, PC_EHIP, "refinement pass needs %zu bytes of %zu", sub.total, plan.ref_sub_cap);
        // gathers: each task starts from the boundary record of its segment
        cp.resize(np);
        for (int64_t k = 0; k < np; ++k)
            cp[k] = {bounds_out + ((size_t)pass[k].m * (stride + 1) + pass[k].s) * 6, ics_sub + k * 6, 12};
        const size_t dcopy = align_up(sub.staged);
        rc = ensure_staging(ctx, dcopy + 2 * kRefineChunk * sizeof(PcCopyDev) + kAlign);
        if (rc != PC_OK) return rc;
        char* st = static_cast<char*>(ctx->staging);
        std::memcpy(st + dcopy, cp.data(), np * sizeof(PcCopyDev));
        PcEphemParams ep;
        PcParams pp;
        stage_call(ctx, sub, model, so, sub_ws, ics_sub, states_sub, iters_sub, smax, bounds_sub, nullptr, 0, ep, pp);
        const PcParams* pp_dev = reinterpret_cast<const PcParams*>(sub_ws + sub.off_params);
        PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_fused_occupancy(sub.pairs, &occ));
        const int grid = std::max(1, ctx->n_cu * std::max(1, occ));
        PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(copies_dev, st + dcopy, np * sizeof(PcCopyDev), hipMemcpyHostToDevice, hs));
        PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_copy_runs(copies_dev, np, hs));
        PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(sub_ws, st, sub.staged, hipMemcpyHostToDevice, hs));
        PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_ephem(ep, hs));
        if (ctx->timing) PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->ev0, hs));
        PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_fused(pp, pp_dev, sub.pairs, grid, hs));
        if (ctx->timing) PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->ev1, hs));
        its.resize((size_t)np * smax);
        PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(its.data(), iters_sub, its.size() * sizeof(int32_t), hipMemcpyDeviceToHost, hs));
        PC_HIP(ctx, hipStreamSynchronize(hs));
        if (ctx->timing) {
            float ms = 0.0f;
            PC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
            ctx->last_ms += ms;
        }
        // results: accept or split further; scatter accepted records into the outputs
        cp.clear();
        for (int64_t k = 0; k < np; ++k) {
            const Task& t = pass[k];
            const int S = groups[t.g].segments;
            const int32_t* r = its.data() + (size_t)k * smax;
            double* brow = bounds_out + (size_t)t.m * (stride + 1) * 6;
            int32_t* irow = it.data() + (size_t)t.m * stride;
            if (t.depth > 0) {
                int32_t st_ = 0, total = 0;
                for (int q = 0; q < (1 << t.depth); ++q) {
                    if (r[q] == PC_ITER_NONFINITE) { st_ = PC_ITER_NONFINITE; break; }
                    if (r[q] == PC_ITER_NOTCONV) st_ = PC_ITER_NOTCONV;
                    else total += r[q];
                }
                const int32_t status = st_ < 0 ? st_ : total;
                if (status == PC_ITER_NOTCONV && t.depth < o.refine) {
                    pending.push_back({t.m, t.g, t.s, t.depth + 1});
                    continue;
                }
                irow[t.s] = status;
                cp.push_back({states_sub + k * 6, brow + (size_t)(t.s + 1) * 6, 12});
                if (t.s + 1 < S) pending.push_back({t.m, t.g, t.s + 1, 0});
                else cp.push_back({states_sub + k * 6, states_out + (size_t)t.m * 6, 12});
            } else {
                for (int j = 0; j < S - t.s; ++j) irow[t.s + j] = r[j];
                cp.push_back({bounds_sub + ((size_t)k * (smax + 1) + 1) * 6, brow + (size_t)(t.s + 1) * 6,
                              (int64_t)(S - t.s) * 12});
                cp.push_back({states_sub + k * 6, states_out + (size_t)t.m * 6, 12});
                first_failure(t.m, t.g, t.s);
            }
        }
        if (!cp.empty()) {
            std::memcpy(st + dcopy, cp.data(), cp.size() * sizeof(PcCopyDev));
            PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(copies_dev, st + dcopy, cp.size() * sizeof(PcCopyDev),
                                                 hipMemcpyHostToDevice, hs));
            PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_copy_runs(copies_dev, (int64_t)cp.size(), hs));
            PC_HIP(ctx, hipStreamSynchronize(hs));   // the staging buffer is written again next pass
        }
    }
    PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(iters_out, it.data(), it.size() * sizeof(int32_t), hipMemcpyHostToDevice, hs));
    PC_HIP(ctx, hipStreamSynchronize(hs));
    int notconv = 0, nonfinite = 0;
    for (int gi = 0; gi < n_groups; ++gi)
        for (int64_t m = groups[gi].ic_offset; m < groups[gi].ic_offset + groups[gi].n_ic; ++m) {
            bool nc = false, nf = false;
            for (int s = 0; s < groups[gi].segments; ++s) {
                nc = nc || it[(size_t)m * stride + s] == PC_ITER_NOTCONV;
                nf = nf || it[(size_t)m * stride + s] == PC_ITER_NONFINITE;
            }
            notconv += nc;
            nonfinite += nf;
        }
    if (nonfinite > 0) return set_error(ctx, PC_ENONFINITE, "%d initial conditions became non-finite", nonfinite);
    if (notconv > 0)
        return set_error(ctx, PC_ENOTCONV, "%d initial conditions did not converge after refinement", notconv);
    return PC_OK;
}

// Flyby screen of the groups of `plan` into ratio (device, indexed like the ICs), queued on
// hs: the plan's group table (each group with its first thread) and the perturbers staged
// and copied into the workspace's table region, the groups' entries of ratio set to +inf,
// then pc_flyby_kernel.
int flyby_screen(pc_ctx* ctx, const Plan& plan, const pc_model* model, char* ws, const double* ics, double* ratio,
                 int samples, hipStream_t hs)
{
    std::vector<PcGroupDev> gd = plan.groups;
    int64_t threads = 0, cov = 0;
    for (PcGroupDev& d : gd) {
        d.thread_offset = threads;
        threads += d.n_ic * samples;
        cov = std::max<int64_t>(cov, d.n_ic);
    }
    const size_t off_inf = align_up(plan.staged);
    int rc = ensure_staging(ctx, off_inf + (size_t)cov * sizeof(double) + kAlign);
    if (rc != PC_OK) return rc;
    char* st = static_cast<char*>(ctx->staging);
    std::memset(st, 0, plan.staged);
    std::memcpy(st + plan.off_groups, gd.data(), gd.size() * sizeof(PcGroupDev));
    prepare_bodies(model, reinterpret_cast<PcBodyDev*>(st + plan.off_bodies));
    double* inf = reinterpret_cast<double*>(st + off_inf);
    for (int64_t i = 0; i < cov; ++i) inf[i] = INFINITY;
    PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(ws, st, plan.staged, hipMemcpyHostToDevice, hs));
    for (const PcGroupDev& d : gd)
        PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(ratio + d.ic_offset, inf, (size_t)d.n_ic * sizeof(double),
                                             hipMemcpyHostToDevice, hs));
    PcFlybyParams fp{};
    fp.groups = reinterpret_cast<const PcGroupDev*>(ws + plan.off_groups);
    fp.n_groups = (int)gd.size();
    fp.bodies = reinterpret_cast<const PcBodyDev*>(ws + plan.off_bodies);
    fp.n_pert = model->n_pert;
    fp.epoch = model->epoch;
    fp.ics = ics;
    fp.ratio = ratio;
    fp.samples = samples;
    fp.n_threads = threads;
    PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_flyby(fp, hs));
    return PC_OK;
}

// Copies described by `cp`, staged and run on hs through the device descriptor array `dev`;
// returns once they are done (the staging buffer is free again).
int run_copies(pc_ctx* ctx, const std::vector<PcCopyDev>& cp, PcCopyDev* dev, hipStream_t hs)
{
    if (cp.empty()) return PC_OK;
    int rc = ensure_staging(ctx, cp.size() * sizeof(PcCopyDev) + kAlign);
    if (rc != PC_OK) return rc;
    std::memcpy(ctx->staging, cp.data(), cp.size() * sizeof(PcCopyDev));
    PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(dev, ctx->staging, cp.size() * sizeof(PcCopyDev), hipMemcpyHostToDevice, hs));
    PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_copy_runs(dev, (int64_t)cp.size(), hs));
    PC_HIP(ctx, hipStreamSynchronize(hs));
    return PC_OK;
}

pc_opts defaults()
{
    pc_opts o;
    pc_default_opts(&o);
    return o;
}

}  // namespace

extern "C" {

void pc_default_opts(pc_opts* o)
{
    if (!o) return;
    o->init = PC_INIT_KEPLER;
    o->max_iter = 64;
    o->tol_mode = PC_TOL_REL;
    o->precision = PC_FP64;
    o->path = PC_PATH_FUSED;
    o->fixed_iters = 0;
    o->tile_pairs = 0;
    o->graph = 0;
    o->switch_tol = 0.0;
    o->max_fp32 = 0;
    o->job_list = 0;
    o->conv = PC_CONV_PER_IC;
    o->streams = 1;
    o->order = 1;
    o->feedback = 0;
    o->guess = nullptr;
    o->refine = 0;
    o->flyby_hill = 0.0;
}

int pc_version(void) { return PC_VERSION; }

const char* pc_strerror(int code)
{
    switch (code) {
    case PC_OK: return "ok";
    case PC_EINVAL: return "invalid argument";
    case PC_ENOTCONV: return "some initial conditions did not converge within max_iter";
    case PC_ENONFINITE: return "some initial conditions became non-finite";
    case PC_EHIP: return "HIP runtime error";
    case PC_ENOMEM: return "workspace too small";
    default: return "unknown status";
    }
}

const char* pc_last_error(pc_ctx* ctx) { return ctx ? ctx->last_error : "no context"; }

int pc_ctx_create(int device, pc_ctx** out)
{
    if (!out) return PC_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return PC_EINVAL;
    pc_ctx* ctx = new (std::nothrow) pc_ctx();
    if (!ctx) return PC_ENOMEM;
    ctx->device = device;
    if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        ctx->n_cu = 256;
    if (hipSetDevice(device) != hipSuccess ||
        hipMalloc(&ctx->d_bodies, PC_MAX_PERT * sizeof(PcBodyDev)) != hipSuccess ||
        hipHostMalloc(&ctx->pinned_count, 64, hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        ensure_staging(ctx, kStagingBytes) != PC_OK) {
        pc_ctx_destroy(ctx);
        return PC_EHIP;
    }
    // the allocation-free entry point's device memory on this device (a failure here only
    // disables that entry point, which then reports it)
    if (scratch_address(ctx, &ctx->scratch) != PC_OK) ctx->scratch = nullptr;
    ctx->last_error[0] = 0;
    *out = ctx;
    return PC_OK;
}

void pc_ctx_destroy(pc_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->ops) {
        (void)hipFree(kv.second.kfrag);
        (void)hipFree(kv.second.tau);
        (void)hipFree(kv.second.kfrag32);
        (void)hipFree(kv.second.kfrag32p);
        (void)hipFree(kv.second.kfragT);
        (void)hipFree(kv.second.kfrag2);
    }
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->d_bodies) (void)hipFree(ctx->d_bodies);
    if (ctx->pinned_count) (void)hipHostFree(ctx->pinned_count);
    for (int t = 0; t < ctx->pl_streams; ++t) {
        if (ctx->pl_stream[t]) (void)hipStreamDestroy(ctx->pl_stream[t]);
        if (ctx->pl_done[t]) (void)hipEventDestroy(ctx->pl_done[t]);
        if (ctx->pl_poll[t]) (void)hipEventDestroy(ctx->pl_poll[t]);
    }
    if (ctx->pl_start) (void)hipEventDestroy(ctx->pl_start);
    if (ctx->pl_count) (void)hipHostFree(ctx->pl_count);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

int pc_workspace_bytes(pc_ctx* ctx, const pc_group* groups, int32_t n_groups, const pc_model* model,
                       const pc_opts* opts, size_t* bytes)
{
    if (!ctx || !bytes) return PC_EINVAL;
    int rc = validate_model(ctx, model);
    if (rc != PC_OK) return rc;
    const pc_opts o = opts ? *opts : defaults();
    int64_t n_ic = 0;
    if (groups)
        for (int i = 0; i < n_groups; ++i) n_ic = std::max<int64_t>(n_ic, groups[i].ic_offset + groups[i].n_ic);
    Plan plan;
    rc = make_plan(ctx, n_ic, groups, n_groups, model, o, false, plan);
    if (rc != PC_OK) return rc;
    *bytes = plan.total;
    return PC_OK;
}

static int isolate_flybys(pc_ctx* ctx, const Plan& plan, const double* ics, const pc_group* groups, int32_t n_groups,
                          const pc_model* model, const pc_opts& o, double* states_out, int32_t* iters_out,
                          int32_t iters_stride, double* bounds_out, char* ws, hipStream_t hs);

// The forward call.  no_alloc: the workspace is this device's static `scratch` (workspace
// and ws_bytes are ignored), the operators must already be cached, the tables must fit the
// staging buffer the context holds, and only the fused path without graph capture runs, so
// that nothing is allocated.
static int propagate_impl(pc_ctx* ctx, const double* ics, int64_t n_ic, const pc_group* groups,
                          int32_t n_groups, const pc_model* model, const pc_opts* opts,
                          double* states_out, int32_t* iters_out, int32_t iters_stride,
                          double* bounds_out, double* nodes_out, int32_t nodes_stride,
                          void* workspace, size_t ws_bytes, pc_stream_t stream, bool no_alloc)
{
    if (!ctx) return PC_EINVAL;
    ctx->last_error[0] = 0;
    if (!ics || !states_out || n_ic < 1) return set_error(ctx, PC_EINVAL, "null ics/states_out or n_ic < 1");
    int rc = validate_model(ctx, model);
    if (rc != PC_OK) return rc;
    const pc_opts o = opts ? *opts : defaults();
    rc = validate_forward(ctx, o, model);
    if (rc != PC_OK) return rc;
    if (o.refine > 0 && (!iters_out || !bounds_out || nodes_out || no_alloc))
        return set_error(ctx, PC_EINVAL, "refinement needs iters_out and bounds_out, takes no nodes_out and "
                         "does not run in the allocation-free call");
    if (no_alloc) {
        if (o.path != PC_PATH_FUSED) return set_error(ctx, PC_EINVAL, "the allocation-free call runs the fused path");
        if (o.graph) return set_error(ctx, PC_EINVAL, "the allocation-free call does not capture graphs");
        if (!ctx->scratch) return set_error(ctx, PC_EHIP, "no scratch address on device %d", ctx->device);
        workspace = ctx->scratch;
        ws_bytes = PC_NOALLOC_SCRATCH_BYTES;
    }
    const bool eih = model->inv_c2 > 0.0;
    PC_HIP(ctx, hipSetDevice(ctx->device));
    Plan plan;
    const bool lists_ok = o.path == PC_PATH_FUSED && o.precision == PC_FP64 && !eih && !o.feedback &&
                          o.init != PC_INIT_GUESS;
    rc = make_plan(ctx, n_ic, groups, n_groups, model, o, true, plan, lists_ok, no_alloc);
    if (rc != PC_OK) return rc;
    if ((iters_out || bounds_out || nodes_out) && iters_stride < plan.max_S)
        return set_error(ctx, PC_EINVAL, "iters_stride %d < %d segments", iters_stride, plan.max_S);
    if ((nodes_out || o.guess) && nodes_stride < plan.max_N)
        return set_error(ctx, PC_EINVAL, "nodes_stride %d < %d nodes", nodes_stride, plan.max_N);
    if (o.guess && iters_stride < plan.max_S)
        return set_error(ctx, PC_EINVAL, "iters_stride %d < %d segments", iters_stride, plan.max_S);
    if (no_alloc && plan.total > ws_bytes)
        return set_error(ctx, PC_ENOMEM, "the call needs %zu bytes of workspace; the static scratch of the "
                         "allocation-free call holds %zu", plan.total, ws_bytes);
    if (!workspace || ws_bytes < plan.total)
        return set_error(ctx, PC_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, plan.total);
    if (o.flyby_hill > 0.0) {
        if (nodes_out || no_alloc)
            return set_error(ctx, PC_EINVAL, "flyby isolation takes no nodes_out and does not run in the "
                             "allocation-free call");
        return isolate_flybys(ctx, plan, ics, groups, n_groups, model, o, states_out, iters_out, iters_stride,
                              bounds_out, static_cast<char*>(workspace), (hipStream_t)stream);
    }

    // stage [counters | params | groups | jobs | bodies] and copy them in one transfer
    if (no_alloc && plan.staged + kAlign > ctx->staging_bytes)
        return set_error(ctx, PC_ENOMEM, "the call's tables take %zu bytes; the context's staging buffer "
                         "holds %zu", plan.staged + kAlign, ctx->staging_bytes);
    rc = ensure_staging(ctx, plan.staged + kAlign);
    if (rc != PC_OK) return rc;
    char* st = static_cast<char*>(ctx->staging);
    char* ws = static_cast<char*>(workspace);
    hipStream_t hs = (hipStream_t)stream;
    PcEphemParams ep;
    PcParams pp;
    stage_call(ctx, plan, model, o, ws, ics, states_out, iters_out, iters_stride, bounds_out, nodes_out,
               nodes_stride, ep, pp);
    const PcParams* pp_dev = reinterpret_cast<const PcParams*>(ws + plan.off_params);
    int32_t* hc = reinterpret_cast<int32_t*>(st);   // staging is free again once the copy has run

    int grid = 1;
    if (!plan.plain) {
        int occ = 0;
        PC_HIP(ctx, (hipError_t)pc_fused_occupancy(plan.pairs, &occ));
        grid = std::max(1, ctx->n_cu * std::max(1, occ));
    }
    // the device work of a fused call: tables in, ephemeris, persistent kernel, status out
    auto enqueue_fused = [&](hipStream_t sq, bool events) -> hipError_t {
        hipError_t e = hipMemcpyAsync(ws, st, plan.staged, hipMemcpyHostToDevice, sq);
        if (e == hipSuccess) e = (hipError_t)pc_launch_ephem(ep, sq);
        if (e == hipSuccess && events) e = hipEventRecord(ctx->ev0, sq);
        if (e == hipSuccess) e = (hipError_t)pc_launch_fused(pp, pp_dev, plan.pairs, grid, sq);
        if (e == hipSuccess && events) e = hipEventRecord(ctx->ev1, sq);
        if (e == hipSuccess) e = hipMemcpyAsync(hc, pp.counters, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, sq);
        return e;
    };

    if (plan.plain) {
        PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(ws, st, plan.staged, hipMemcpyHostToDevice, hs));
        PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_ephem(ep, hs));
        if (ctx->timing) PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->ev0, hs));
        // one group at a time, kernels per iteration, host loop (the structure of Sec. 5.4)
        auto plain_args = [&](int gi) {
            PcPlainArgs a{};
            a.p = pp;
            a.g = pp.groups + gi;
            a.g_host = plan.groups[gi];
            a.jobs = pp.jobs + plan.group_job_begin[gi];
            a.n_jobs = plan.group_job_begin[gi + 1] - plan.group_job_begin[gi];
            a.N = plan.groups[gi].N;
            a.NP = plan.groups[gi].NP;
            a.T = plan.groups[gi].T;
            a.S = plan.groups[gi].S;
            a.t2 = plan.groups[gi].tol * plan.groups[gi].tol;
            return a;
        };
        const int ns = plan.plain_streams;
        if (ns <= 1) {
            for (int gi = 0; gi < n_groups; ++gi)
                PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_run_plain(plain_args(gi), ws + plan.off_plain, ctx->pinned_count, stream));
        } else {
            // the outer level on ns streams: group gi on stream gi % ns.  The calling thread
            // drives every stream: it polls each stream's last read-back with an event and
            // takes that stream's next loop decision when it has landed, so the streams' host
            // round trips overlap without any thread of ours but this one launching work.
            // The streams start after the work queued so far; the caller's stream waits for
            // all of them.
            rc = ensure_plain_streams(ctx, ns);
            if (rc != PC_OK) {
                (void)hipStreamSynchronize(hs);
                return rc;
            }
            PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->pl_start, hs));
            std::vector<PcPlainRun> runs(ns);
            std::vector<int> next(ns);      // next group of each stream
            std::vector<char> busy(ns, 0);
            hipError_t e = hipSuccess;
            auto drain = [&] {   // let every stream finish before the caller can free its buffers
                for (int t = 0; t < ns; ++t) (void)hipStreamSynchronize(ctx->pl_stream[t]);
            };
            for (int t = 0; t < ns && e == hipSuccess; ++t) {
                next[t] = t + ns;
                e = hipStreamWaitEvent(ctx->pl_stream[t], ctx->pl_start, 0);
                if (e == hipSuccess && t < n_groups) {
                    e = (hipError_t)pc_plain_begin(runs[t], plain_args(t), ws + plan.off_plain + t * plan.plain_stride,
                                                   ctx->pl_count + 16 * t, ctx->pl_stream[t]);
                    if (e == hipSuccess) e = hipEventRecord(ctx->pl_poll[t], ctx->pl_stream[t]);
                    busy[t] = 1;
                }
            }
            int running = 0;
            for (int t = 0; t < ns; ++t) running += busy[t];
            while (e == hipSuccess && running > 0) {
                bool moved = false;
                for (int t = 0; t < ns && e == hipSuccess; ++t) {
                    if (!busy[t]) continue;
                    const hipError_t q = hipEventQuery(ctx->pl_poll[t]);
                    if (q == hipErrorNotReady) continue;
                    if (q != hipSuccess) {
                        e = q;
                        break;
                    }
                    moved = true;
                    e = (hipError_t)pc_plain_advance(runs[t]);
                    if (e == hipSuccess && runs[t].done) {
                        if (next[t] < n_groups) {
                            const int gi = next[t];
                            next[t] += ns;
                            e = (hipError_t)pc_plain_begin(runs[t], plain_args(gi),
                                                           ws + plan.off_plain + t * plan.plain_stride,
                                                           ctx->pl_count + 16 * t, ctx->pl_stream[t]);
                        } else {
                            busy[t] = 0;
                            --running;
                        }
                    }
                    if (e == hipSuccess && busy[t]) e = hipEventRecord(ctx->pl_poll[t], ctx->pl_stream[t]);
                }
                if (!moved) std::this_thread::yield();
            }
            for (int t = 0; t < ns && e == hipSuccess; ++t) e = hipEventRecord(ctx->pl_done[t], ctx->pl_stream[t]);
            if (e != hipSuccess) {
                drain();
                (void)hipStreamSynchronize(hs);
                return set_error(ctx, PC_EHIP, "plain path on %d streams: %s", ns, hipGetErrorString(e));
            }
            for (int t = 0; t < ns; ++t) PC_HIP_DRAIN(ctx, hs, hipStreamWaitEvent(hs, ctx->pl_done[t], 0));
        }
        if (ctx->timing) PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->ev1, hs));
        PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(hc, pp.counters, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, hs));
    } else if (o.graph) {
        // signature of the call: a captured graph is replayed only for the same one
        std::vector<char> key;
        auto put = [&key](const void* q, size_t nb) {
            key.insert(key.end(), static_cast<const char*>(q), static_cast<const char*>(q) + nb);
        };
        const void* ptrs[8] = {ics, states_out, iters_out, bounds_out, nodes_out, workspace, stream, ctx->staging};
        put(ptrs, sizeof(ptrs));
        put(&n_ic, sizeof(n_ic));
        put(&n_groups, sizeof(n_groups));
        put(groups, sizeof(pc_group) * n_groups);
        put(&o, sizeof(o));
        put(&model->mu_sun, sizeof(double));
        put(&model->epoch, sizeof(double));
        put(&model->inv_c2, sizeof(double));
        put(&model->n_pert, sizeof(int32_t));
        if (model->n_pert > 0) put(model->pert, sizeof(double) * 7 * model->n_pert);
        put(&iters_stride, sizeof(iters_stride));
        put(&nodes_stride, sizeof(nodes_stride));
        put(&ws_bytes, sizeof(ws_bytes));
        put(&plan.pairs, sizeof(plan.pairs));
        if (!ctx->graph_exec || key != ctx->graph_key) {
            drop_graph(ctx);
            PC_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            const hipError_t e = enqueue_fused(ctx->cap_stream, false);
            hipGraph_t gr = nullptr;
            const hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &gr);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                return set_error(ctx, PC_EHIP, "graph capture failed: %s",
                                 hipGetErrorString(e != hipSuccess ? e : e2));
            }
            ctx->graph = gr;
            PC_HIP(ctx, hipGraphInstantiate(&ctx->graph_exec, ctx->graph, nullptr, nullptr, 0));
            ctx->graph_key = key;
            ++ctx->graph_captures;
        }
        // the whole graph is timed in graph mode (copies and ephemeris included)
        if (ctx->timing) PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->ev0, hs));
        PC_HIP_DRAIN(ctx, hs, hipGraphLaunch(ctx->graph_exec, hs));
        if (ctx->timing) PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->ev1, hs));
    } else {
        PC_HIP_DRAIN(ctx, hs, enqueue_fused(hs, ctx->timing));
    }
    PC_HIP(ctx, hipStreamSynchronize(hs));
    if (ctx->timing) {
        float ms = 0.0f;
        PC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->last_ms = ms;
    }
    if (o.refine > 0 && hc[0] > 0)
        return refine_passes(ctx, plan, groups, n_groups, model, o, lists_ok, ws, n_ic, states_out, iters_out,
                             iters_stride, bounds_out, hs);
    if (hc[1] > 0) return set_error(ctx, PC_ENONFINITE, "%d initial conditions became non-finite", hc[1]);
    if (hc[0] > 0) return set_error(ctx, PC_ENOTCONV, "%d initial conditions did not converge", hc[0]);
    return PC_OK;
}

// Flyby isolation (opts.flyby_hill > 0): screen every IC, split every group into its quiet
// ICs and its flyby ICs (ratio below the threshold), each part a group of its own, and
// run the call on the ICs in that order: a copy of the ICs in the workspace, the reordered
// call's outputs there too, scattered back to the caller's rows.  When no group is split
// the call runs in place.
static int isolate_flybys(pc_ctx* ctx, const Plan& plan, const double* ics, const pc_group* groups, int32_t n_groups,
                          const pc_model* model, const pc_opts& o, double* states_out, int32_t* iters_out,
                          int32_t iters_stride, double* bounds_out, char* ws, hipStream_t hs)
{
    char* F = ws + plan.off_flyby;
    double* ratio = reinterpret_cast<double*>(F + plan.fly_ratio);
    int rc = flyby_screen(ctx, plan, model, ws, ics, ratio, kFlybySamples, hs);
    if (rc != PC_OK) return rc;
    std::vector<double> hr((size_t)plan.fly_span);
    PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(hr.data(), ratio, hr.size() * sizeof(double), hipMemcpyDeviceToHost, hs));
    PC_HIP(ctx, hipStreamSynchronize(hs));
    std::vector<pc_group> ng;
    std::vector<int64_t> perm;
    std::vector<int> seg_of;   // segments of the group of each reordered IC
    bool split = false;
    for (int gi = 0; gi < n_groups; ++gi) {
        const pc_group& G = groups[gi];
        std::vector<int64_t> quiet, fly;
        for (int64_t m = G.ic_offset; m < G.ic_offset + G.n_ic; ++m)
            (hr[(size_t)m] < o.flyby_hill ? fly : quiet).push_back(m);
        for (const auto* part : {&quiet, &fly}) {
            if (part->empty()) continue;
            pc_group q = G;
            q.ic_offset = (int64_t)perm.size();
            q.n_ic = (int64_t)part->size();
            ng.push_back(q);
            perm.insert(perm.end(), part->begin(), part->end());
            seg_of.insert(seg_of.end(), part->size(), G.segments);
        }
        split = split || (!quiet.empty() && !fly.empty());
    }
    pc_opts oi = o;
    oi.flyby_hill = 0.0;
    if (!split)   // every group is all quiet or all flyby: nothing moves
        return propagate_impl(ctx, ics, plan.fly_span, groups, n_groups, model, &oi, states_out, iters_out,
                              iters_stride, bounds_out, nullptr, 0, ws, plan.off_flyby, hs, false);
    const int S = plan.max_S;
    const int64_t cov = (int64_t)perm.size();
    double* ics_p = reinterpret_cast<double*>(F + plan.fly_ics);
    double* states_p = reinterpret_cast<double*>(F + plan.fly_states);
    int32_t* iters_p = reinterpret_cast<int32_t*>(F + plan.fly_iters);
    double* bounds_p = reinterpret_cast<double*>(F + plan.fly_bounds);
    PcCopyDev* copies = reinterpret_cast<PcCopyDev*>(F + plan.fly_copies);
    std::vector<PcCopyDev> cp((size_t)cov);
    for (int64_t k = 0; k < cov; ++k) cp[k] = {ics + perm[k] * 6, ics_p + k * 6, 12};
    rc = run_copies(ctx, cp, copies, hs);
    if (rc != PC_OK) return rc;
    const int status = propagate_impl(ctx, ics_p, cov, ng.data(), (int32_t)ng.size(), model, &oi, states_p,
                                      iters_out ? iters_p : nullptr, S, bounds_out ? bounds_p : nullptr, nullptr, 0,
                                      F + plan.fly_sub, plan.fly_sub_cap, hs, false);
    if (status != PC_OK && status != PC_ENOTCONV && status != PC_ENONFINITE) return status;
    const std::string msg = ctx->last_error;
    cp.clear();
    for (int64_t k = 0; k < cov; ++k) {
        const int64_t m = perm[k];
        cp.push_back({states_p + k * 6, states_out + m * 6, 12});
        if (iters_out) cp.push_back({iters_p + k * S, iters_out + m * iters_stride, seg_of[k]});
        if (bounds_out)
            cp.push_back({bounds_p + k * (S + 1) * 6, bounds_out + m * (iters_stride + 1) * 6,
                          (int64_t)(seg_of[k] + 1) * 12});
    }
    rc = run_copies(ctx, cp, copies, hs);
    if (rc != PC_OK) return rc;
    if (status != PC_OK) set_error(ctx, status, "%s", msg.c_str());
    return status;
}

int pc_flyby_ratio(pc_ctx* ctx, const double* ics, int64_t n_ic, const pc_group* groups, int32_t n_groups,
                   const pc_model* model, int32_t samples, double* ratio, void* workspace, size_t ws_bytes,
                   pc_stream_t stream)
{
    if (!ctx) return PC_EINVAL;
    ctx->last_error[0] = 0;
    if (!ics || !ratio || n_ic < 1) return set_error(ctx, PC_EINVAL, "null ics/ratio or n_ic < 1");
    if (samples < 2 || samples > 64) return set_error(ctx, PC_EINVAL, "samples must be 2..64");
    int rc = validate_model(ctx, model);
    if (rc != PC_OK) return rc;
    PC_HIP(ctx, hipSetDevice(ctx->device));
    const pc_opts o = defaults();
    Plan plan;
    rc = make_plan(ctx, n_ic, groups, n_groups, model, o, false, plan);
    if (rc != PC_OK) return rc;
    if (!workspace || ws_bytes < plan.staged)
        return set_error(ctx, PC_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, plan.staged);
    hipStream_t hs = (hipStream_t)stream;
    rc = flyby_screen(ctx, plan, model, static_cast<char*>(workspace), ics, ratio, samples, hs);
    if (rc != PC_OK) return rc;
    PC_HIP(ctx, hipStreamSynchronize(hs));
    return PC_OK;
}

int pc_propagate_batched(pc_ctx* ctx, const double* ics, int64_t n_ic, const pc_group* groups,
                         int32_t n_groups, const pc_model* model, const pc_opts* opts,
                         double* states_out, int32_t* iters_out, int32_t iters_stride,
                         double* bounds_out, double* nodes_out, int32_t nodes_stride,
                         void* workspace, size_t ws_bytes, pc_stream_t stream)
{
    return propagate_impl(ctx, ics, n_ic, groups, n_groups, model, opts, states_out, iters_out, iters_stride,
                          bounds_out, nodes_out, nodes_stride, workspace, ws_bytes, stream, false);
}

int pc_propagate_batched_noalloc(pc_ctx* ctx, const double* ics, int64_t n_ic, const pc_group* groups,
                                 int32_t n_groups, const pc_model* model, const pc_opts* opts,
                                 double* states_out, int32_t* iters_out, int32_t iters_stride,
                                 double* bounds_out, double* nodes_out, int32_t nodes_stride,
                                 pc_stream_t stream)
{
    return propagate_impl(ctx, ics, n_ic, groups, n_groups, model, opts, states_out, iters_out, iters_stride,
                          bounds_out, nodes_out, nodes_stride, nullptr, 0, stream, true);
}

int pc_propagate(pc_ctx* ctx, const double* ics, int64_t n_ic, double t0, double tf, int32_t nodes,
                 int32_t segments, double tol, const pc_model* model, const pc_opts* opts,
                 double* states_out, int32_t* iters_out, void* workspace, size_t ws_bytes,
                 pc_stream_t stream)
{
    pc_group g;
    g.ic_offset = 0;
    g.n_ic = n_ic;
    g.t0 = t0;
    g.tf = tf;
    g.nodes = nodes;
    g.segments = segments;
    g.tol = tol;
    return pc_propagate_batched(ctx, ics, n_ic, &g, 1, model, opts, states_out, iters_out, segments,
                                nullptr, nullptr, 0, workspace, ws_bytes, stream);
}

int pc_measure_ceilings(pc_ctx* ctx, void* buf, size_t buf_bytes, pc_stream_t stream, double* out)
{
    if (!ctx || !buf || !out) return PC_EINVAL;
    if (buf_bytes < ((size_t)16 << 20)) return set_error(ctx, PC_EINVAL, "buf_bytes must be at least 16 MiB");
    PC_HIP(ctx, hipSetDevice(ctx->device));
    PC_HIP_DRAIN(ctx, (hipStream_t)stream, (hipError_t)pc_ceilings_run(ctx->n_cu, buf, buf_bytes, stream, out));
    return PC_OK;
}

int pc_graph_captures(pc_ctx* ctx, int64_t* count)
{
    if (!ctx || !count) return PC_EINVAL;
    *count = ctx->graph_captures;
    return PC_OK;
}

int pc_set_timing(pc_ctx* ctx, int enable)
{
    if (!ctx) return PC_EINVAL;
    PC_HIP(ctx, hipSetDevice(ctx->device));
    if (enable && !ctx->ev0) {
        PC_HIP(ctx, hipEventCreate(&ctx->ev0));
        PC_HIP(ctx, hipEventCreate(&ctx->ev1));
    }
    ctx->timing = enable != 0;
    ctx->last_ms = -1.0;
    return PC_OK;
}

int pc_last_kernel_ms(pc_ctx* ctx, double* ms)
{
    if (!ctx || !ms) return PC_EINVAL;
    *ms = ctx->last_ms;
    return ctx->last_ms >= 0.0 ? PC_OK : set_error(ctx, PC_EINVAL, "no timed call yet");
}

int pc_adjoint(pc_ctx* ctx, int64_t n_ic, const pc_group* groups, int32_t n_groups, const pc_model* model,
               const pc_opts* opts, const double* ckpt, int32_t ckpt_stride, const double* gbar_final,
               const double* gbar_nodes, const double* fwd_nodes, int32_t nodes_stride, double adj_tol,
               int32_t adj_max_iter,
               double* grad_ics, int32_t* adj_iters, void* workspace, size_t ws_bytes, pc_stream_t stream)
{
    if (!ctx) return PC_EINVAL;
    ctx->last_error[0] = 0;
    if (!ckpt || !gbar_final || !grad_ics || n_ic < 1)
        return set_error(ctx, PC_EINVAL, "null ckpt/gbar_final/grad_ics or n_ic < 1");
    int rc = validate_model(ctx, model);
    if (rc != PC_OK) return rc;
    pc_opts o = opts ? *opts : defaults();
    if (o.path != PC_PATH_FUSED || o.precision != PC_FP64)
        return set_error(ctx, PC_EINVAL, "the adjoint re-solves segments on the fused FP64 path");
    if (o.conv != PC_CONV_PER_IC)
        return set_error(ctx, PC_EINVAL, "the adjoint linearises the map converged per IC");
    if (o.order != 1) return set_error(ctx, PC_EINVAL, "the adjoint linearises the first-order map");
    if (o.init == PC_INIT_GUESS) return set_error(ctx, PC_EINVAL, "the adjoint re-solves with a warm or cold start");
    if (o.init != PC_INIT_KEPLER && o.init != PC_INIT_COLD) return set_error(ctx, PC_EINVAL, "bad init");
    if (o.max_iter < 1 || o.max_iter > 100000 || o.fixed_iters < 0) return set_error(ctx, PC_EINVAL, "bad iterations");
    if (!(adj_tol > 0.0) || !std::isfinite(adj_tol) || adj_max_iter < 2 || adj_max_iter > 100000)
        return set_error(ctx, PC_EINVAL, "adj_tol must be > 0 and adj_max_iter >= 2");
    o.tile_pairs = 2048;
    PC_HIP(ctx, hipSetDevice(ctx->device));
    Plan plan;
    rc = make_plan(ctx, n_ic, groups, n_groups, model, o, true, plan);
    if (rc != PC_OK) return rc;
    if (ckpt_stride < plan.max_S) return set_error(ctx, PC_EINVAL, "ckpt_stride < segments");
    if ((gbar_nodes || fwd_nodes) && nodes_stride < plan.max_N)
        return set_error(ctx, PC_EINVAL, "nodes_stride < nodes");
    if (!workspace || ws_bytes < plan.total)
        return set_error(ctx, PC_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, plan.total);
    rc = ensure_staging(ctx, plan.staged + kAlign);
    if (rc != PC_OK) return rc;
    char* st = static_cast<char*>(ctx->staging);
    std::memset(st, 0, plan.staged);
    std::memcpy(st + plan.off_groups, plan.groups.data(), plan.groups.size() * sizeof(PcGroupDev));
    std::memcpy(st + plan.off_jobs, plan.jobs.data(), plan.jobs.size() * sizeof(PcJobDev));
    prepare_bodies(model, reinterpret_cast<PcBodyDev*>(st + plan.off_bodies));
    char* ws = static_cast<char*>(workspace);
    hipStream_t hs = (hipStream_t)stream;
    PcEphemParams ep{};
    ep.groups = reinterpret_cast<const PcGroupDev*>(ws + plan.off_groups);
    ep.n_groups = (int)plan.groups.size();
    ep.n_recs = plan.n_recs;
    ep.bodies = reinterpret_cast<const PcBodyDev*>(ws + plan.off_bodies);
    ep.n_pert = model->n_pert;
    ep.epoch = model->epoch;
    ep.recs = reinterpret_cast<double*>(ws + plan.off_recs);
    const bool eih = model->inv_c2 > 0.0;
    ep.recs_eih = eih ? reinterpret_cast<double*>(ws + plan.off_recs_eih) : nullptr;
    ep.mu_sun = model->mu_sun;

    PcAdjParams a{};
    a.fwd.groups = ep.groups;
    a.fwd.jobs = reinterpret_cast<const PcJobDev*>(ws + plan.off_jobs);
    a.fwd.n_jobs = (int)plan.jobs.size();
    a.fwd.n_pert = model->n_pert;
    a.fwd.recs = ep.recs;
    a.fwd.mu_sun = model->mu_sun;
    a.fwd.recs_eih = ep.recs_eih;
    a.fwd.inv_c2 = eih ? model->inv_c2 : 0.0;
    a.fwd.max_iter = o.max_iter;
    a.fwd.fixed_iters = o.fixed_iters;
    a.fwd.tol_mode = o.tol_mode;
    a.fwd.init = o.init;
    a.fwd.precision = PC_FP64;
    a.fwd.max_fp32 = 1;
    a.fwd.switch2 = 0.0;
    a.fwd.iters_stride = ckpt_stride;
    a.ckpt = ckpt;
    a.ckpt_stride = ckpt_stride;
    a.nodes_stride = nodes_stride;
    a.gbar_final = gbar_final;
    a.gbar_nodes = gbar_nodes;
    a.fwd_nodes = fwd_nodes;
    a.adj_tol = adj_tol;
    a.adj_max_iter = adj_max_iter;
    a.grad_out = grad_ics;
    a.adj_iters = adj_iters;
    a.counters = reinterpret_cast<int32_t*>(ws + plan.off_counters);
    std::memcpy(st + plan.off_params, &a, sizeof(a));   // the device copy the kernel reads
    const PcAdjParams* a_dev = reinterpret_cast<const PcAdjParams*>(ws + plan.off_params);
    PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(ws, st, plan.staged, hipMemcpyHostToDevice, hs));
    PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_ephem(ep, hs));
    if (ctx->timing) PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->ev0, hs));
    PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_adjoint(a, a_dev, ctx->n_cu, hs));
    if (ctx->timing) PC_HIP_DRAIN(ctx, hs, hipEventRecord(ctx->ev1, hs));
    int32_t* hc = reinterpret_cast<int32_t*>(st);
    PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(hc, a.counters, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, hs));
    PC_HIP(ctx, hipStreamSynchronize(hs));
    if (ctx->timing) {
        float ms = 0.0f;
        PC_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->last_ms = ms;
    }
    if (hc[1] > 0) return set_error(ctx, PC_ENONFINITE, "%d gradients are non-finite", hc[1]);
    if (hc[0] > 0) return set_error(ctx, PC_ENOTCONV, "%d forward or adjoint sweeps did not converge", hc[0]);
    return PC_OK;
}

int pc_set_tile_pairs(pc_ctx* ctx, int32_t padded_nodes, int32_t pairs)
{
    if (!ctx) return PC_EINVAL;
    if (padded_nodes < 16 || padded_nodes > 256 || (padded_nodes & (padded_nodes - 1)))
        return set_error(ctx, PC_EINVAL, "padded_nodes must be 16, 32, 64, 128 or 256");
    if (pairs != 0 && pairs != 1024 && pairs != 2048) return set_error(ctx, PC_EINVAL, "pairs must be 0, 1024 or 2048");
    if (pairs == 1024 && padded_nodes * 8 > 1024) return set_error(ctx, PC_EINVAL, "1024 pairs need <= 128 nodes");
    ctx->tile_table[log2_index(padded_nodes)] = pairs;
    return PC_OK;
}

int pc_get_tile_pairs(pc_ctx* ctx, int32_t padded_nodes, int32_t* pairs)
{
    if (!ctx || !pairs) return PC_EINVAL;
    if (padded_nodes < 16 || padded_nodes > 256 || (padded_nodes & (padded_nodes - 1)))
        return set_error(ctx, PC_EINVAL, "padded_nodes must be 16, 32, 64, 128 or 256");
    *pairs = ctx->tile_table[log2_index(padded_nodes)];
    return PC_OK;
}

int pc_set_job_list(pc_ctx* ctx, int32_t padded_nodes, int32_t blocks)
{
    if (!ctx) return PC_EINVAL;
    if (padded_nodes < 16 || padded_nodes > 256 || (padded_nodes & (padded_nodes - 1)))
        return set_error(ctx, PC_EINVAL, "padded_nodes must be 16, 32, 64, 128 or 256");
    if (blocks != 0 && blocks != 1 && blocks != 2 && blocks != 4 && blocks != 8)
        return set_error(ctx, PC_EINVAL, "blocks must be 0, 1, 2, 4 or 8");
    ctx->list_table[log2_index(padded_nodes)] = blocks;
    return PC_OK;
}

int pc_get_job_list(pc_ctx* ctx, int32_t padded_nodes, int32_t* blocks)
{
    if (!ctx || !blocks) return PC_EINVAL;
    if (padded_nodes < 16 || padded_nodes > 256 || (padded_nodes & (padded_nodes - 1)))
        return set_error(ctx, PC_EINVAL, "padded_nodes must be 16, 32, 64, 128 or 256");
    *blocks = ctx->list_table[log2_index(padded_nodes)];
    return PC_OK;
}

int pc_autotune(pc_ctx* ctx, const double* ics, int64_t n_ic, const pc_group* groups, int32_t n_groups,
                const pc_model* model, double* scratch_states, void* workspace, size_t ws_bytes,
                pc_stream_t stream, int32_t* chosen_pairs)
{
    if (!ctx || !groups || n_groups < 1 || !scratch_states || !chosen_pairs) return PC_EINVAL;
    int np_max = 16;
    bool present[5] = {false, false, false, false, false};
    for (int i = 0; i < n_groups; ++i) {
        const int np = padded_nodes(std::max(3, std::min((int)groups[i].nodes, PC_MAX_NODES)));
        np_max = std::max(np_max, np);
        present[log2_index(np)] = true;
    }
    const int kmax = log2_index(np_max);
    // start from the untuned rules: tables cleared for the batch's node counts
    int tile_saved = ctx->tile_table[kmax], list_saved[5];
    for (int k = 0; k < 5; ++k) list_saved[k] = ctx->list_table[k];
    auto restore = [&] {
        ctx->tile_table[kmax] = tile_saved;
        for (int k = 0; k < 5; ++k) ctx->list_table[k] = list_saved[k];
    };
    ctx->tile_table[kmax] = 0;
    for (int k = 0; k < 5; ++k)
        if (present[k]) ctx->list_table[k] = 0;
    const bool was_timing = ctx->timing;
    int rc = pc_set_timing(ctx, 1);
    if (rc != PC_OK) {
        restore();
        return rc;
    }
    pc_opts o;
    pc_default_opts(&o);
    // median kernel time of three runs of the caller's batch under the current tables
    auto measure = [&](double* ms) -> int {
        double t[3];
        for (int rep = 0; rep < 3; ++rep) {
            const int r = pc_propagate_batched(ctx, ics, n_ic, groups, n_groups, model, &o, scratch_states, nullptr,
                                               0, nullptr, nullptr, 0, workspace, ws_bytes, stream);
            if (r != PC_OK && r != PC_ENOTCONV && r != PC_ENONFINITE) return r;
            t[rep] = ctx->last_ms;
        }
        std::sort(t, t + 3);
        *ms = t[1];
        return PC_OK;
    };
    auto fail = [&](int r) {
        ctx->timing = was_timing;
        restore();
        return r;
    };
    // one untimed run (operators, staging), then the untuned rules as the first incumbent
    rc = pc_propagate_batched(ctx, ics, n_ic, groups, n_groups, model, &o, scratch_states, nullptr, 0, nullptr,
                              nullptr, 0, workspace, ws_bytes, stream);
    if (rc != PC_OK && rc != PC_ENOTCONV && rc != PC_ENONFINITE) return fail(rc);
    double best_ms = 0.0, ms = 0.0;
    if ((rc = measure(&best_ms)) != PC_OK) return fail(rc);
    int best_pairs = 0;   // 0: the untuned shape rule
    // the job shape of the call (one per launch): the 1024-pair shape only fits up to 128
    // padded nodes
    const int cands[2] = {2048, 1024};
    for (int c : cands) {
        if (c == 1024 && np_max * 8 > 1024) continue;
        ctx->tile_table[kmax] = c;
        if ((rc = measure(&ms)) != PC_OK) return fail(rc);
        if (ms < best_ms) {
            best_ms = ms;
            best_pairs = c;
        }
    }
    ctx->tile_table[kmax] = best_pairs;
    // then the job length of each node count, largest first, the others held at their best
    for (int k = 4; k >= 0; --k) {
        if (!present[k]) continue;
        int best_list = 0;   // 0: the untuned rule
        for (int m : {1, 2, 4, 8}) {
            ctx->list_table[k] = m;
            if ((rc = measure(&ms)) != PC_OK) return fail(rc);
            if (ms < best_ms) {
                best_ms = ms;
                best_list = m;
            }
        }
        ctx->list_table[k] = best_list;
    }
    ctx->timing = was_timing;
    int pairs = best_pairs;
    if (pairs == 0) {   // record the shape the untuned rule picked
        pc_opts d;
        pc_default_opts(&d);
        pairs = choose_pairs(ctx, groups, n_groups, d);
    }
    ctx->tile_table[kmax] = pairs;
    *chosen_pairs = pairs;
    return PC_OK;
}

int pc_get_operator(pc_ctx* ctx, int32_t nodes, double* K_host)
{
    if (!ctx || !K_host) return PC_EINVAL;
    if (nodes < 3 || nodes > PC_MAX_NODES) return set_error(ctx, PC_EINVAL, "nodes out of range");
    const OperatorCache* oc = nullptr;
    int rc = get_operator(ctx, nodes, &oc);
    if (rc != PC_OK) return rc;
    std::memcpy(K_host, oc->K.data(), oc->K.size() * sizeof(double));
    return PC_OK;
}

int pc_apply_operator(pc_ctx* ctx, int32_t nodes, int64_t n_cols, const double* F, const double* y0,
                      double scale, double* Y, pc_stream_t stream)
{
    if (!ctx || !F || !y0 || !Y || n_cols < 1) return PC_EINVAL;
    if (nodes < 3 || nodes > PC_MAX_NODES) return set_error(ctx, PC_EINVAL, "nodes out of range");
    PC_HIP(ctx, hipSetDevice(ctx->device));
    const OperatorCache* oc = nullptr;
    int rc = get_operator(ctx, nodes, &oc);
    if (rc != PC_OK) return rc;
    PC_HIP_DRAIN(ctx, (hipStream_t)stream, (hipError_t)pc_launch_apply_operator(oc->NP, oc->kfrag, nodes, n_cols, F, y0, scale, Y, stream));
    PC_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    return PC_OK;
}

int pc_eval_force(pc_ctx* ctx, const double* r, const double* t, int64_t n, const pc_model* model,
                  double* a_out, pc_stream_t stream)
{
    if (!ctx || !r || !t || !a_out || n < 1) return PC_EINVAL;
    int rc = validate_model(ctx, model);
    if (rc != PC_OK) return rc;
    if (model->inv_c2 > 0.0)
        return set_error(ctx, PC_EINVAL, "the force hook takes positions only (point-mass model)");
    PC_HIP(ctx, hipSetDevice(ctx->device));
    rc = ensure_staging(ctx, PC_MAX_PERT * sizeof(PcBodyDev));
    if (rc != PC_OK) return rc;
    prepare_bodies(model, static_cast<PcBodyDev*>(ctx->staging));
    hipStream_t hs = (hipStream_t)stream;
    if (model->n_pert > 0)
        PC_HIP_DRAIN(ctx, hs, hipMemcpyAsync(ctx->d_bodies, ctx->staging, model->n_pert * sizeof(PcBodyDev),
                                   hipMemcpyHostToDevice, hs));
    PC_HIP_DRAIN(ctx, hs, (hipError_t)pc_launch_eval_force(r, t, n, ctx->d_bodies, model->n_pert, model->epoch,
                                                 model->mu_sun, a_out, stream));
    PC_HIP(ctx, hipStreamSynchronize(hs));
    return PC_OK;
}

int pc_eval_kepler(pc_ctx* ctx, const double* y0, const double* dt, int64_t n, double* y, int32_t* ok,
                   pc_stream_t stream)
{
    if (!ctx || !y0 || !dt || !y || !ok || n < 1) return PC_EINVAL;
    PC_HIP(ctx, hipSetDevice(ctx->device));
    PC_HIP_DRAIN(ctx, (hipStream_t)stream, (hipError_t)pc_launch_eval_kepler(y0, dt, n, y, ok, stream));
    PC_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    return PC_OK;
}

}  // extern "C"
