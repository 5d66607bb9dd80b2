// pc_ceilings.hip -- on-chip ceilings that the roofline figures are quoted against, next to
// the datasheet peaks: an FP64 matrix-core loop, an FP64 vector FMA loop and a device copy.
//
// Each kernel does a fixed, known amount of work with enough independent chains per wave to
// keep its pipe busy, and writes a value derived from every chain so that none of the work
// can be dropped.  The host function times them with HIP events on the caller's stream,
// after a warm-up.  (A sweep of the matrix loop on this chip: 4 or 8 chains per wave at one
// to four waves per SIMD all reach 75-78 TFLOP/s once warm; 16 chains per wave fall to
// 31-38.)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pcprop.h"
#include "pc_internal.h"

namespace {

typedef double f64x4c __attribute__((ext_vector_type(4)));

constexpr int kChains = 8;          // independent accumulators per wave / lane
constexpr int kMfmaBlock = 256;     // four waves, one per SIMD (two workgroups per CU)
constexpr int kFmaBlock = 256;

// kChains independent v_mfma_f64_16x16x4_f64 chains per wave: 2 * 16 * 16 * 4 flop each.
// No launch bound: with __launch_bounds__(256) the compiler kept the accumulators in VGPRs
// and copied all 64 of them into AGPRs and back around every loop iteration (128 moves per
// 8 MFMAs), which halved the measured rate (47 TFLOP/s); without it the loop is MFMAs only.
__global__ void pc_ceiling_mfma(int iters, double* sink)
{
    const double a = 1.0 + 1e-9 * (double)threadIdx.x;
    const double b = 1.0 - 1e-9 * (double)blockIdx.x;
    f64x4c acc[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc[k] = f64x4c{0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += acc[k].x + acc[k].y + acc[k].z + acc[k].w;
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// kChains independent v_fma_f64 chains per lane: 2 flop each.
__global__ __launch_bounds__(kFmaBlock) void pc_ceiling_fma(int iters, double* sink)
{
    const double a = 1.0 - 1e-12 * (double)threadIdx.x;
    const double b = 1e-9 * (double)blockIdx.x;
    double x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = (double)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) x[k] = fma(x[k], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// dst = src, 16-byte accesses, grid-stride.
__global__ __launch_bounds__(256) void pc_ceiling_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                       size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

int pc_ceilings_run(int n_cu, void* buf, size_t buf_bytes, void* stream, double* out)
{
    hipStream_t st = (hipStream_t)stream;
    double* sink = static_cast<double*>(buf);
    const int mfma_grid = n_cu * 2, fma_grid = n_cu * 8;
    const size_t sink_need = (size_t)std::max(mfma_grid * kMfmaBlock, fma_grid * kFmaBlock) * sizeof(double);
    if (buf_bytes < sink_need || buf_bytes < ((size_t)16 << 20)) return hipErrorInvalidValue;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // best of five timed launches after the pipe has run for about 50 ms untimed
    auto best_ms = [&](auto launch, double* ms) -> hipError_t {
        hipError_t r = hipEventRecord(e0, st);
        float warm = 0.0f;
        for (int rep = 0; rep < 200 && r == hipSuccess && warm < 50.0f; ++rep) {
            launch();
            r = hipGetLastError();
            if (r == hipSuccess) r = hipEventRecord(e1, st);
            if (r == hipSuccess) r = hipEventSynchronize(e1);
            if (r == hipSuccess) r = hipEventElapsedTime(&warm, e0, e1);
        }
        float best = 1e30f;
        for (int rep = 0; rep < 5 && r == hipSuccess; ++rep) {
            r = hipEventRecord(e0, st);
            if (r == hipSuccess) launch();
            if (r == hipSuccess) r = hipGetLastError();
            if (r == hipSuccess) r = hipEventRecord(e1, st);
            if (r == hipSuccess) r = hipEventSynchronize(e1);
            float t = 0.0f;
            if (r == hipSuccess) r = hipEventElapsedTime(&t, e0, e1);
            best = std::min(best, t);
        }
        *ms = best;
        return r;
    };
    double ms = 0.0;
    const int mfma_iters = 8192, fma_iters = 32768;
    if (e == hipSuccess)
        e = best_ms([&] { hipLaunchKernelGGL(pc_ceiling_mfma, dim3(mfma_grid), dim3(kMfmaBlock), 0, st, mfma_iters, sink); },
                    &ms);
    if (e == hipSuccess) {
        const double flop = (double)mfma_grid * (kMfmaBlock / 64) * mfma_iters * kChains * (2.0 * 16 * 16 * 4);
        out[0] = flop / (ms * 1e-3) / 1e12;
        e = best_ms([&] { hipLaunchKernelGGL(pc_ceiling_fma, dim3(fma_grid), dim3(kFmaBlock), 0, st, fma_iters, sink); },
                    &ms);
    }
    if (e == hipSuccess) {
        const double flop = (double)fma_grid * kFmaBlock * fma_iters * kChains * 2.0;
        out[1] = flop / (ms * 1e-3) / 1e12;
        const size_t half = (buf_bytes / 2) / sizeof(double2) * sizeof(double2);
        const size_t n = half / sizeof(double2);
        const double2* src = static_cast<const double2*>(buf);
        double2* dst = reinterpret_cast<double2*>(static_cast<char*>(buf) + half);
        const int cgrid = n_cu * 16;
        e = best_ms([&] { hipLaunchKernelGGL(pc_ceiling_copy, dim3(cgrid), dim3(256), 0, st, src, dst, n); }, &ms);
        if (e == hipSuccess) out[2] = 2.0 * (double)half / (ms * 1e-3) / 1e9;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}
