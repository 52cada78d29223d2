// Measured VALU ceilings of the current device, for the roofline the
// benchmark reports beside the published peaks: sustained lane-operation
// rates of FP32 FMA, the FP32 transcendentals the right-hand side uses
// (v_exp_f32, v_log_f32, v_rcp_f32) and FP64 FMA.  Each kernel runs eight
// independent dependency chains per lane of one operation, enough waves to
// fill every SIMD, and one store per thread at the end.  Built with the same
// flags as the solver kernels (no packed FP32), so the FP32 FMA figure is
// the unpacked ceiling those kernels can reach.  FP32 FMA is measured twice:
// with its multiplier and addend in scalar registers (v_fma_f32, the form the
// solver's arithmetic compiles to) and with a literal multiplier
// (v_fmamk_f32), which the hardware issues at a different rate.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "rac.h"
#include "rac_internal.h"

namespace rac {
namespace {

constexpr int kChains = 8;
constexpr int kCeilThreads = 256;

enum : int { kFma = 0, kExp = 1, kLog = 2, kRcp = 3, kFmaLiteral = 4 };

template <int OP>
__global__ __launch_bounds__(kCeilThreads) void ceiling_f32(float* out, int iters, float seed, float b, float c) {
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = seed + (float)(threadIdx.x + j) * 1e-6f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            if (OP == kFma) a[j] = __builtin_fmaf(a[j], b, c);
            if (OP == kFmaLiteral) a[j] = __builtin_fmaf(a[j], 0.9999999f, 1e-7f);
            if (OP == kExp) a[j] = __builtin_amdgcn_exp2f(-a[j]);
            if (OP == kLog) a[j] = __builtin_amdgcn_logf(__builtin_fabsf(a[j]));
            if (OP == kRcp) a[j] = __builtin_amdgcn_rcpf(a[j]);
        }
    }
    float s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kCeilThreads) void ceiling_f64(double* out, int iters, double seed, double b, double c) {
    double a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = seed + (double)(threadIdx.x + j) * 1e-6;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = __builtin_fma(a[j], b, c);
    }
    double s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace rac

extern "C" rac_status rac_valu_ceilings(double* lane_ops_per_s, int32_t n) {
    using namespace rac;
    if (!lane_ops_per_s || n < 1) return fail(RAC_EINVAL, "rac_valu_ceilings: NULL or empty output");
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(RAC_EDEVICE, "rac_valu_ceilings: no device");
    // Eight waves per SIMD on every CU, each lane running kChains chains.
    const int blocks = n_cu * 8;
    const int iters = 4096;
    const double lane_ops = (double)blocks * kCeilThreads * kChains * iters;
    void* buf = nullptr;
    if (hipMalloc(&buf, (size_t)blocks * kCeilThreads * sizeof(double)) != hipSuccess)
        return fail(RAC_ENOMEM, "rac_valu_ceilings: scratch");
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rac_status st = RAC_OK;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        st = fail(RAC_EDEVICE, "rac_valu_ceilings: stream or events");
    // Each chain feeds an operation its own previous result (the negation
    // and absolute value are free source modifiers), so nothing can be
    // folded or hoisted; the rate of these operations does not depend on
    // the values.
    auto run = [&](auto launch) -> double {
        launch();  // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
        launch();
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
        return ms > 0 ? lane_ops / (ms * 1e-3) : -1.0;
    };
    constexpr int kN = 6;
    double r[kN] = {0, 0, 0, 0, 0, 0};
    if (st == RAC_OK) {
        float* f = (float*)buf;
        auto f32 = [&](auto kernel, float seed) {
            return run([&] {
                hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kCeilThreads), 0, s, f, iters, seed, 0.9999999f, 1e-7f);
            });
        };
        r[0] = f32(ceiling_f32<kFma>, 0.5f);
        r[1] = f32(ceiling_f32<kExp>, 0.5f);
        r[2] = f32(ceiling_f32<kLog>, 1.5f);
        r[3] = f32(ceiling_f32<kRcp>, 1.5f);
        r[4] = run([&] {
            hipLaunchKernelGGL(ceiling_f64, dim3(blocks), dim3(kCeilThreads), 0, s, (double*)buf, iters, 0.5,
                               0.9999999, 1e-7);
        });
        r[5] = f32(ceiling_f32<kFmaLiteral>, 0.5f);
        if (hipGetLastError() != hipSuccess) st = fail(RAC_EDEVICE, "rac_valu_ceilings: launch");
        for (double v : r)
            if (v <= 0) st = fail(RAC_EDEVICE, "rac_valu_ceilings: timing");
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(buf);
    if (st != RAC_OK) return st;
    for (int i = 0; i < n && i < kN; ++i) lane_ops_per_s[i] = r[i];
    for (int i = kN; i < n; ++i) lane_ops_per_s[i] = 0;
    return RAC_OK;
}
