// Instantiations of the DP5(4) kernel: float state, time-series mode.
#include "dp5_kernel.h"
#include "kernel_table.h"
#include "rac.h"

namespace rac {

#define RAC_K(E, G) {RAC_FP32, true, E, G, false, reinterpret_cast<const void*>(&dp5_kernel<float, E, G, true>)}

static const KernelEntry kTable[] = {
    RAC_K(4, 1), RAC_K(4, 2), RAC_K(4, 3), RAC_K(4, 4), RAC_K(4, 6), RAC_K(4, 8), RAC_K(8, 1),
    RAC_K(8, 2), RAC_K(8, 3), RAC_K(8, 4), RAC_K(8, 6), RAC_K(8, 8), RAC_K(12, 1),
    RAC_K(12, 2), RAC_K(12, 3), RAC_K(12, 4), RAC_K(12, 6), RAC_K(12, 8), RAC_K(16, 1),
    RAC_K(16, 2), RAC_K(16, 3), RAC_K(16, 4), RAC_K(16, 6), RAC_K(16, 8), RAC_K(24, 1),
    RAC_K(24, 2), RAC_K(24, 3), RAC_K(24, 4), RAC_K(24, 6), RAC_K(32, 1), RAC_K(32, 2),
    RAC_K(32, 3), RAC_K(7, 3), RAC_K(11, 3), RAC_K(13, 5), RAC_K(6, 2), RAC_K(10, 4), RAC_K(6, 3),
};

int kernels_f32_ts(const KernelEntry** out) {
    *out = kTable;
    return (int)(sizeof(kTable) / sizeof(kTable[0]));
}

}  // namespace rac
