// Measured FP32 vector ceiling of the device: a register-only loop of
// independent FMA chains on every compute unit, compiled with the same flags
// as every kernel of the library (no packed FP32 instructions), so its rate is
// what the arithmetic of these kernels can reach at most.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/tm.h"
#include "tm_api_internal.h"

namespace tmsap {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 8;  // independent FMA chains per thread
constexpr int kProbeIters = 32768;

__global__ void __launch_bounds__(kProbeThreads) k_fma_probe(int iters, float a, float b, float* out) {
    float x[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) x[k] = (float)(threadIdx.x + k) * 1e-3f;
#pragma unroll 8
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) x[k] = __builtin_fmaf(x[k], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += x[k];
    // the chains stay near 1 for a = 1 - 1e-6, b = 1e-6: never true, but the compiler cannot drop them
    if (s == -1.f) out[blockIdx.x] = s;
}

}  // namespace

}  // namespace tmsap

using namespace tmsap;

extern "C" {

int tm_probe_fp32_fma(double* tflops, const tm_opts* opts) {
    int rc;
    if (!tflops) return fail(TM_ERR_ARG, "tflops is NULL");
    if ((rc = check_opts(opts))) return rc;
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ds->device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    const unsigned grid = (unsigned)std::max(1, cus) * 16;  // 16 workgroups of 4 wavefronts per compute unit
    if ((e = ds->red.ensure((size_t)grid * sizeof(float))) != hipSuccess) return hip_fail(e, "probe buffer");
    hipStream_t st = (hipStream_t)opts->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    float best_ms = 0.f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // the first launch warms up, the best of the rest counts
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_fma_probe, dim3(grid), dim3(kProbeThreads), 0, st, kProbeIters, 1.f - 1e-6f, 1e-6f,
                               static_cast<float*>(ds->red.ptr));
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0 && (best_ms == 0.f || ms < best_ms)) best_ms = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "FMA probe");
    if (!(best_ms > 0.f)) return fail(TM_ERR_HIP, "FMA probe: no timing");
    const double flops = 2.0 * kProbeChains * (double)kProbeIters * grid * kProbeThreads;
    *tflops = flops / (best_ms * 1e-3) / 1e12;
    return TM_OK;
}

}  // extern "C"
