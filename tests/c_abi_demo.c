/* A plain C caller of the library's C ABI, with no Python and no C++: it
 * samples a network's parameters on the host, copies them to device memory
 * it allocates itself, integrates every (parameter set, initial condition)
 * pair to a steady state on the GPU and prints one line per trajectory:
 *   id status n_accepted x_0 ... x_{N-1}
 * Usage: c_abi_demo SEED N_SETS N_IC   (network: the toggle switch with
 * self-activation, A -| B, B -| A, A -> A, B -> B).  Exit status 0 on
 * success, 1 on any failed call (the message goes to stderr). */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "rac.h"

#define CHECK_RAC(call)                                                         \
    do {                                                                        \
        rac_status st_ = (call);                                                \
        if (st_ != RAC_OK) {                                                    \
            fprintf(stderr, "%s: %d %s\n", #call, (int)st_, rac_last_error()); \
            return 1;                                                           \
        }                                                                       \
    } while (0)
#define CHECK_HIP(call)                                                          \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));          \
            return 1;                                                            \
        }                                                                        \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 4) {
        fprintf(stderr, "usage: %s SEED N_SETS N_IC\n", argv[0]);
        return 1;
    }
    const unsigned long long seed = strtoull(argv[1], NULL, 10);
    const long long P = atoll(argv[2]);
    const int n_ic = atoi(argv[3]);
    if (P < 1 || n_ic < 1) {
        fprintf(stderr, "N_SETS and N_IC must be positive\n");
        return 1;
    }
    const int32_t src[] = {0, 1, 0, 1}, dst[] = {1, 0, 0, 1};
    const int8_t sign[] = {-1, -1, 1, 1};
    rac_topology* topo = NULL;
    CHECK_RAC(rac_create_topology(2, 4, src, dst, sign, &topo));
    int32_t N = 0, E = 0;
    CHECK_RAC(rac_topology_size(topo, &N, &E));

    /* Host parameters (Table 1 ranges) and initial-condition fractions. */
    float* hG = malloc(sizeof(float) * N * P);
    float* hk = malloc(sizeof(float) * N * P);
    float* hT = malloc(sizeof(float) * E * P);
    float* hl = malloc(sizeof(float) * E * P);
    uint8_t* hn = malloc((size_t)E * P);
    float* hic = malloc(sizeof(float) * N * n_ic);
    if (!hG || !hk || !hT || !hl || !hn || !hic) {
        fprintf(stderr, "host allocation failed\n");
        return 1;
    }
    rac_params_view hp = {hG, hk, hT, hl, hn, P, NULL};
    CHECK_RAC(rac_sample_params(topo, NULL, seed, 0, P, n_ic, &hp, hic));

    /* Device copies, owned by this program. */
    rac_params_view dp = {NULL, NULL, NULL, NULL, NULL, P, NULL};
    float* dic = NULL;
    CHECK_HIP(hipMalloc((void**)&dp.G, sizeof(float) * N * P));
    CHECK_HIP(hipMalloc((void**)&dp.k, sizeof(float) * N * P));
    CHECK_HIP(hipMalloc((void**)&dp.T, sizeof(float) * E * P));
    CHECK_HIP(hipMalloc((void**)&dp.lam, sizeof(float) * E * P));
    CHECK_HIP(hipMalloc((void**)&dp.n, (size_t)E * P));
    CHECK_HIP(hipMalloc((void**)&dic, sizeof(float) * N * n_ic));
    CHECK_HIP(hipMemcpy(dp.G, hG, sizeof(float) * N * P, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dp.k, hk, sizeof(float) * N * P, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dp.T, hT, sizeof(float) * E * P, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dp.lam, hl, sizeof(float) * E * P, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dp.n, hn, (size_t)E * P, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dic, hic, sizeof(float) * N * n_ic, hipMemcpyHostToDevice));

    const long long n_traj = P * n_ic;
    float* dx = NULL;
    int8_t* dst_ = NULL;
    int32_t* dacc = NULL;
    CHECK_HIP(hipMalloc((void**)&dx, sizeof(float) * N * n_traj));
    CHECK_HIP(hipMalloc((void**)&dst_, (size_t)n_traj));
    CHECK_HIP(hipMalloc((void**)&dacc, sizeof(int32_t) * n_traj));
    rac_traj_info info = {NULL, dst_, dacc, NULL};

    rac_solver_opts opts;
    rac_default_opts(&opts, RAC_FP32);
    CHECK_RAC(rac_steady_states(topo, &dp, dic, n_ic, &opts, dx, &info, NULL));
    CHECK_HIP(hipDeviceSynchronize());

    float* hx = malloc(sizeof(float) * N * n_traj);
    int8_t* hs = malloc((size_t)n_traj);
    int32_t* ha = malloc(sizeof(int32_t) * n_traj);
    if (!hx || !hs || !ha) {
        fprintf(stderr, "host allocation failed\n");
        return 1;
    }
    CHECK_HIP(hipMemcpy(hx, dx, sizeof(float) * N * n_traj, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(hs, dst_, (size_t)n_traj, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(ha, dacc, sizeof(int32_t) * n_traj, hipMemcpyDeviceToHost));
    for (long long t = 0; t < n_traj; ++t) {
        printf("%lld %d %d", t, (int)hs[t], (int)ha[t]);
        for (int i = 0; i < N; ++i) printf(" %.9g", (double)hx[t * N + i]);
        printf("\n");
    }

    hipFree(dx); hipFree(dst_); hipFree(dacc); hipFree(dic);
    hipFree(dp.G); hipFree(dp.k); hipFree(dp.T); hipFree(dp.lam); hipFree(dp.n);
    free(hG); free(hk); free(hT); free(hl); free(hn); free(hic); free(hx); free(hs); free(ha);
    rac_destroy_topology(topo);
    return 0;
}
