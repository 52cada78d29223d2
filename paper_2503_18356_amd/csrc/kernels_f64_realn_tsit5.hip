// Instantiations of the Tsitouras 5(4) kernel for real Hill coefficients:
// double state, steady-state and time-series modes.
#include "dp5_kernel.h"
#include "kernel_table.h"
#include "rac.h"

namespace rac {

#define RAC_KR(TS, M, E, G)                                                                          \
    {RAC_FP64, TS, E, G, false, reinterpret_cast<const void*>(&dp5_kernel<double, E, G, TS, false, M, true>), \
     M, true}
#define RAC_KR_ALL(TS, M)                                                                            \
    RAC_KR(TS, M, 4, 1), RAC_KR(TS, M, 4, 2), RAC_KR(TS, M, 4, 3), RAC_KR(TS, M, 4, 4), RAC_KR(TS, M, 4, 6), \
        RAC_KR(TS, M, 8, 1), RAC_KR(TS, M, 8, 2), RAC_KR(TS, M, 8, 3), RAC_KR(TS, M, 8, 4),           \
        RAC_KR(TS, M, 12, 1), RAC_KR(TS, M, 12, 2), RAC_KR(TS, M, 12, 3), RAC_KR(TS, M, 16, 1),       \
        RAC_KR(TS, M, 16, 2), RAC_KR(TS, M, 7, 3)

static const KernelEntry kTable[] = {
    RAC_KR_ALL(false, kTsit5), RAC_KR_ALL(true, kTsit5),
};

int kernels_f64_realn_tsit5(const KernelEntry** out) {
    *out = kTable;
    return (int)(sizeof(kTable) / sizeof(kTable[0]));
}

}  // namespace rac
