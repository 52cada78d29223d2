// Registry of the compiled kernel instantiations.
#pragma once

#include "kernel_common.h"

namespace rac {

using KernelFn = void (*)(LaunchArgs);

struct KernelEntry {
    int precision;  // RAC_FP32 / RAC_FP64
    bool ts;        // time-series mode
    int epl, gpl;   // compiled slot budgets
    bool bounded;   // serving step-batch variant
    const void* fn; // __global__ function
    int method;     // RAC_DP5 / RAC_TSIT5
    bool realn = false;  // FP64 kernel for real Hill coefficients
};

// Each instantiation unit appends its entries.
int kernels_f32_ss(const KernelEntry** out);
int kernels_f32_ts(const KernelEntry** out);
int kernels_f64_ss(const KernelEntry** out);
int kernels_f64_ts(const KernelEntry** out);
int kernels_f32_serve(const KernelEntry** out);
int kernels_f32_ss_tsit5(const KernelEntry** out);
int kernels_f32_ts_tsit5(const KernelEntry** out);
int kernels_f64_ss_tsit5(const KernelEntry** out);
int kernels_f64_ts_tsit5(const KernelEntry** out);
int kernels_f64_realn(const KernelEntry** out);
int kernels_f64_realn_tsit5(const KernelEntry** out);

const KernelEntry* find_kernel(int precision, bool ts, int epl, int gpl, bool bounded = false,
                               int method = RAC_DP5, bool realn = false);

}  // namespace rac
