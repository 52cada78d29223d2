// Post-processing of integration results on the device: G/k normalisation,
// the global histogram of normalised values with multi-level Otsu
// thresholds, discretisation into levels and state codes, the number of
// distinct states per parameter set, and global state frequencies.
//
// Every step is HBM- or atomic-bound except the threshold search, a small
// exhaustive FP64 search over bin-index tuples in one workgroup.  Integer
// decisions taken from floating point (bins, levels, the threshold argmax)
// use fixed IEEE operations (no contraction) so that they are reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "rac.h"
#include "rac_internal.h"

namespace rac {
namespace {

constexpr uint64_t kNoState = ~0ull;
constexpr int kMaxBins = 1024;
constexpr int kMaxStatesPerSet = 4096;
constexpr int kThreads = 256;

#define RAC_PP(call, what)                                                              \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(RAC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

int grid_for(int64_t n, int per_block = kThreads) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

// Bin of a normalised value: clamp to [0, 1], floor(y B), cap at B - 1.
__device__ __forceinline__ int bin_of(float y, int n_bins) {
    const float yc = fminf(fmaxf(y, 0.0f), 1.0f);
    const int b = (int)floorf(__fmul_rn(yc, (float)n_bins));
    return b < n_bins - 1 ? b : n_bins - 1;
}

__global__ void normalize_kernel(const float* __restrict__ x, float* __restrict__ y, int64_t n_elem,
                                 int N, int64_t P, int n_ic, int n_t, const float* __restrict__ G,
                                 const float* __restrict__ k) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / N;
        const int i = (int)(e - r * N);
        const int64_t p = r / n_t / n_ic;
        y[e] = __fdiv_rn(__fmul_rn(x[e], k[i * P + p]), G[i * P + p]);
    }
}

template <typename T>
__global__ void fill_kernel(T* a, int64_t n, T v) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        a[e] = v;
}

// Block-local LDS histogram, then one atomic per bin into the global counts.
__global__ void histogram_kernel(const float* __restrict__ y, int64_t n_rows, int N,
                                 const int8_t* __restrict__ status, int n_bins,
                                 unsigned long long* __restrict__ hist) {
    __shared__ unsigned int h[kMaxBins];
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int64_t n_elem = n_rows * N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_elem;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (status && status[e / N] != RAC_CONVERGED) continue;
        atomicAdd(&h[bin_of(y[e], n_bins)], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], (unsigned long long)h[b]);
}

// Exhaustive multi-level Otsu over threshold tuples 0 < t1 < ... < t_{L-1} < B:
// maximise sum_k S_k^2 / W_k over the classes [t_k, t_{k+1}), evaluated in
// FP64 in class order; among equal maxima the lexicographically first tuple
// (smallest flattened index) wins.  One workgroup.
__global__ __launch_bounds__(1024) void otsu_kernel(const unsigned long long* __restrict__ hist, int B,
                                                    int L, int* __restrict__ thr) {
    __shared__ long long cw[kMaxBins + 1], cs[kMaxBins + 1];
    __shared__ double best_v[1024];
    __shared__ long long best_i[1024];
    if (threadIdx.x == 0) {
        long long w = 0, s = 0;
        cw[0] = 0;
        cs[0] = 0;
        for (int b = 0; b < B; ++b) {
            w += (long long)hist[b];
            s += (long long)b * (long long)hist[b];
            cw[b + 1] = w;
            cs[b + 1] = s;
        }
    }
    __syncthreads();
    const int m = L - 1;
    long long n_idx = 1;
    for (int j = 0; j < m; ++j) n_idx *= B;
    double bv = -1.0;
    long long bi = -1;
    for (long long idx = threadIdx.x; idx < n_idx; idx += blockDim.x) {
        int t[3] = {0, 0, 0};
        long long r = idx;
        for (int j = m - 1; j >= 0; --j) {
            t[j] = (int)(r % B);
            r /= B;
        }
        bool ok = t[0] >= 1;
        for (int j = 1; j < m; ++j) ok = ok && t[j] > t[j - 1];
        if (!ok) continue;
        double v = 0.0;
        int lo = 0;
        for (int kc = 0; kc <= m; ++kc) {
            const int hi = kc < m ? t[kc] : B;
            const long long W = cw[hi] - cw[lo];
            const long long S = cs[hi] - cs[lo];
            const double term = W > 0 ? __ddiv_rn(__dmul_rn((double)S, (double)S), (double)W) : 0.0;
            v = __dadd_rn(v, term);
            lo = hi;
        }
        if (v > bv) {  // indices grow along a thread's walk: first maximum kept
            bv = v;
            bi = idx;
        }
    }
    best_v[threadIdx.x] = bv;
    best_i[threadIdx.x] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double ov = best_v[threadIdx.x + s];
            const long long oi = best_i[threadIdx.x + s];
            const double cv = best_v[threadIdx.x];
            const long long ci = best_i[threadIdx.x];
            if (oi >= 0 && (ci < 0 || ov > cv || (ov == cv && oi < ci))) {
                best_v[threadIdx.x] = ov;
                best_i[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        long long r = best_i[0];
        for (int j = m - 1; j >= 0; --j) {
            thr[j] = r < 0 ? 0 : (int)(r % B);
            r = r < 0 ? r : r / B;
        }
    }
}

__global__ void discretize_kernel(const float* __restrict__ y, int64_t n_rows, int N,
                                  const int8_t* __restrict__ status, int n_bins, int L,
                                  const int* __restrict__ thr, uint8_t* __restrict__ levels,
                                  uint64_t* __restrict__ codes) {
    int t[3] = {n_bins, n_bins, n_bins};
    for (int j = 0; j < L - 1; ++j) t[j] = thr[j];
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n_rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        const bool keep = !status || status[r] == RAC_CONVERGED;
        uint64_t code = 0;
        for (int i = 0; i < N; ++i) {
            const int b = bin_of(y[r * N + i], n_bins);
            const int lv = (b >= t[0]) + (b >= t[1]) + (b >= t[2]);
            if (levels) levels[r * N + i] = keep ? (uint8_t)lv : (uint8_t)255;
            code = code * (uint64_t)L + (uint64_t)lv;
        }
        if (codes) codes[r] = keep ? code : kNoState;
    }
}

// One workgroup per parameter set: bitonic sort of its n_ic codes in LDS,
// then the distinct codes (NO_STATE excluded) in ascending order.
__global__ __launch_bounds__(kThreads) void multistability_kernel(const uint64_t* __restrict__ codes, int n_ic,
                                                                  int n_pow2, int* __restrict__ n_states,
                                                                  uint64_t* __restrict__ states) {
    __shared__ uint64_t key[kMaxStatesPerSet];
    __shared__ int cnt[kThreads + 1];
    const int64_t p = blockIdx.x;
    const uint64_t* c = codes + p * n_ic;
    for (int i = threadIdx.x; i < n_pow2; i += blockDim.x) key[i] = i < n_ic ? c[i] : kNoState;
    __syncthreads();
    for (int size = 2; size <= n_pow2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n_pow2; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const uint64_t a = key[i], b = key[j];
                    if ((a > b) == up) {
                        key[i] = b;
                        key[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // Each thread owns a contiguous chunk; count its first occurrences.
    const int chunk = (n_pow2 + blockDim.x - 1) / blockDim.x;
    const int beg = threadIdx.x * chunk;
    const int end = beg + chunk < n_pow2 ? beg + chunk : n_pow2;
    int mine = 0;
    for (int i = beg; i < end; ++i)
        mine += key[i] != kNoState && (i == 0 || key[i] != key[i - 1]);
    cnt[threadIdx.x + 1] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt[0] = 0;
        for (int t = 1; t <= (int)blockDim.x; ++t) cnt[t] += cnt[t - 1];
        n_states[p] = cnt[blockDim.x];
    }
    __syncthreads();
    uint64_t* out = states + p * n_ic;
    int pos = cnt[threadIdx.x];
    for (int i = beg; i < end; ++i)
        if (key[i] != kNoState && (i == 0 || key[i] != key[i - 1])) out[pos++] = key[i];
    const int total = cnt[blockDim.x];
    for (int i = total + threadIdx.x; i < n_ic; i += blockDim.x) out[i] = kNoState;
}

// 64-bit finaliser (splitmix64) as the hash of a state code.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Add `add` to key c in the global table (open addressing, linear probing);
// a full table raises the overflow flag.
__device__ void global_insert(uint64_t c, unsigned long long add, unsigned long long* keys,
                              unsigned long long* counts, uint64_t mask, int* overflow) {
    uint64_t h = mix64(c) & mask;
    for (uint64_t probe = 0; probe <= mask; ++probe) {
        const unsigned long long prev = atomicCAS(&keys[h], (unsigned long long)kNoState, (unsigned long long)c);
        if (prev == kNoState || prev == c) {
            atomicAdd(&counts[h], add);
            return;
        }
        h = (h + 1) & mask;
    }
    atomicExch(overflow, 1);
}

// Counts are first gathered in a per-workgroup LDS table, so that only the
// distinct states of each workgroup reach the global atomics (a few hot
// states otherwise serialise them); keys that find no LDS slot within a few
// probes go to the global table directly.
constexpr int kLocalSlots = 1024;
constexpr int kLocalProbes = 16;

__global__ __launch_bounds__(kThreads) void insert_kernel(const uint64_t* __restrict__ codes, int64_t n,
                                                          unsigned long long* keys, unsigned long long* counts,
                                                          uint64_t mask, int* overflow) {
    __shared__ unsigned long long lk[kLocalSlots];
    __shared__ unsigned int lc[kLocalSlots];
    for (int i = threadIdx.x; i < kLocalSlots; i += blockDim.x) {
        lk[i] = kNoState;
        lc[i] = 0;
    }
    __syncthreads();
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = codes[r];
        if (c == kNoState) continue;
        int h = (int)(mix64(c) & (kLocalSlots - 1));
        bool placed = false;
        for (int probe = 0; probe < kLocalProbes; ++probe) {
            const unsigned long long prev = atomicCAS(&lk[h], (unsigned long long)kNoState, (unsigned long long)c);
            if (prev == kNoState || prev == c) {
                atomicAdd(&lc[h], 1u);
                placed = true;
                break;
            }
            h = (h + 1) & (kLocalSlots - 1);
        }
        if (!placed) global_insert(c, 1ull, keys, counts, mask, overflow);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kLocalSlots; i += blockDim.x)
        if (lk[i] != kNoState) global_insert(lk[i], lc[i], keys, counts, mask, overflow);
}

__global__ void compact_kernel(const unsigned long long* keys, const unsigned long long* counts, int64_t cap,
                               uint64_t* out_keys, int64_t* out_counts, unsigned long long* n_unique) {
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < cap;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (keys[s] == kNoState) continue;
        const unsigned long long at = atomicAdd(n_unique, 1ull);
        out_keys[at] = keys[s];
        out_counts[at] = (int64_t)counts[s];
    }
}

// Bitonic sorting network over n (a power of two) (key, count) pairs,
// ascending by key.  Passes with stride < kTile run inside one LDS tile of
// kTile pairs (bitonic_tile: every size up to kTile in the first call, then
// the short strides of each larger size); longer strides are global passes.
constexpr int kTile = 2048;

__global__ __launch_bounds__(kThreads) void bitonic_tile(uint64_t* keys, int64_t* vals, int64_t n,
                                                         int64_t size_lo, int64_t size_hi) {
    __shared__ uint64_t k[kTile];
    __shared__ int64_t v[kTile];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = threadIdx.x; i < kTile; i += blockDim.x) {
        k[i] = keys[base + i];
        v[i] = vals[base + i];
    }
    __syncthreads();
    for (int64_t size = size_lo; size <= size_hi; size <<= 1) {
        for (int64_t stride = (size < kTile ? size : kTile) >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < kTile; i += blockDim.x) {
                const int j = i ^ (int)stride;
                if (j > i) {
                    const bool up = ((base + i) & size) == 0;
                    const uint64_t a = k[i], b = k[j];
                    if ((a > b) == up) {
                        k[i] = b;
                        k[j] = a;
                        const int64_t t = v[i];
                        v[i] = v[j];
                        v[j] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < kTile; i += blockDim.x) {
        keys[base + i] = k[i];
        vals[base + i] = v[i];
    }
}

__global__ void bitonic_pass(uint64_t* keys, int64_t* vals, int64_t n, int64_t size, int64_t stride) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i ^ stride;
        if (j > i) {
            const bool up = (i & size) == 0;
            const uint64_t a = keys[i], b = keys[j];
            if ((a > b) == up) {
                keys[i] = b;
                keys[j] = a;
                const int64_t t = vals[i];
                vals[i] = vals[j];
                vals[j] = t;
            }
        }
    }
}

__global__ void finish_counts_kernel(const unsigned long long* n_unique, const int* overflow, int64_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = *overflow ? -1 : (int64_t)*n_unique;
}

bool codes_fit(int n_genes, int n_levels) {
    // L^N - 1 must stay below the NO_STATE marker.
    unsigned __int128 v = 1;
    for (int i = 0; i < n_genes; ++i) {
        v *= (unsigned)n_levels;
        if (v > (unsigned __int128)kNoState) return false;
    }
    return true;
}

}  // namespace
}  // namespace rac

extern "C" {

rac_status rac_normalize(const rac_topology* topo, const rac_params_view* p, int32_t n_ic, int32_t n_t,
                         const float* dev_x, float* dev_y, void* hip_stream) {
    using namespace rac;
    if (!topo || !p || !dev_x || !dev_y || !p->G || !p->k)
        return fail(RAC_EINVAL, "rac_normalize: NULL argument");
    if (n_ic < 1 || n_t < 1 || p->n_sets < 0) return fail(RAC_EINVAL, "rac_normalize: bad sizes");
    const int N = topo->n_genes;
    const int64_t n_elem = p->n_sets * (int64_t)n_ic * n_t * N;
    if (n_elem == 0) return RAC_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(n_elem)), dim3(kThreads), 0, s, dev_x, dev_y, n_elem, N,
                       (int64_t)p->n_sets, (int)n_ic, (int)n_t, p->G, p->k);
    RAC_PP(hipGetLastError(), "rac_normalize: launch");
    return RAC_OK;
}

rac_status rac_level_thresholds(const float* dev_y, int64_t n_rows, int32_t n_genes, const int8_t* dev_status,
                                int32_t n_bins, int32_t n_levels, uint64_t* dev_hist, int32_t* dev_thresholds,
                                void* hip_stream) {
    using namespace rac;
    if (!dev_hist || !dev_thresholds || (n_rows > 0 && !dev_y))
        return fail(RAC_EINVAL, "rac_level_thresholds: NULL argument");
    if (n_rows < 0 || n_genes < 1) return fail(RAC_EINVAL, "rac_level_thresholds: bad sizes");
    if (n_bins < 2 || n_bins > kMaxBins || n_levels < 2 || n_levels > 4 || n_levels > n_bins)
        return fail(RAC_EINVAL, "rac_level_thresholds: need 2 <= n_bins <= 1024 and 2 <= n_levels <= min(4, n_bins)");
    if (n_levels == 4 && n_bins > 256)
        return fail(RAC_EUNSUPPORTED, "rac_level_thresholds: four levels need n_bins <= 256");
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(fill_kernel<unsigned long long>, dim3(grid_for(n_bins)), dim3(kThreads), 0, s,
                       (unsigned long long*)dev_hist, (int64_t)n_bins, 0ull);
    RAC_PP(hipGetLastError(), "rac_level_thresholds: clear");
    if (n_rows > 0) {
        hipLaunchKernelGGL(histogram_kernel, dim3(grid_for(n_rows * n_genes, kThreads * 16)), dim3(kThreads), 0, s,
                           dev_y, n_rows, (int)n_genes, dev_status, (int)n_bins, (unsigned long long*)dev_hist);
        RAC_PP(hipGetLastError(), "rac_level_thresholds: histogram");
    }
    hipLaunchKernelGGL(otsu_kernel, dim3(1), dim3(1024), 0, s, (const unsigned long long*)dev_hist, (int)n_bins,
                       (int)n_levels, dev_thresholds);
    RAC_PP(hipGetLastError(), "rac_level_thresholds: search");
    return RAC_OK;
}

rac_status rac_discretize(const float* dev_y, int64_t n_rows, int32_t n_genes, const int8_t* dev_status,
                          int32_t n_bins, int32_t n_levels, const int32_t* dev_thresholds, uint8_t* dev_levels,
                          uint64_t* dev_codes, void* hip_stream) {
    using namespace rac;
    if (!dev_thresholds || (n_rows > 0 && !dev_y) || (!dev_levels && !dev_codes))
        return fail(RAC_EINVAL, "rac_discretize: NULL argument");
    if (n_rows < 0 || n_genes < 1) return fail(RAC_EINVAL, "rac_discretize: bad sizes");
    if (n_bins < 2 || n_bins > kMaxBins || n_levels < 2 || n_levels > 4)
        return fail(RAC_EINVAL, "rac_discretize: need 2 <= n_bins <= 1024 and 2 <= n_levels <= 4");
    if (dev_codes && !codes_fit(n_genes, n_levels))
        return fail(RAC_EUNSUPPORTED, "rac_discretize: n_levels^n_genes does not fit a 64-bit state code");
    if (n_rows == 0) return RAC_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(discretize_kernel, dim3(grid_for(n_rows)), dim3(kThreads), 0, s, dev_y, n_rows,
                       (int)n_genes, dev_status, (int)n_bins, (int)n_levels, dev_thresholds, dev_levels,
                       dev_codes);
    RAC_PP(hipGetLastError(), "rac_discretize: launch");
    return RAC_OK;
}

rac_status rac_multistability(const uint64_t* dev_codes, int64_t n_sets, int32_t n_ic, int32_t* dev_n_states,
                              uint64_t* dev_states, void* hip_stream) {
    using namespace rac;
    if (n_sets < 0 || n_ic < 1) return fail(RAC_EINVAL, "rac_multistability: bad sizes");
    if (n_sets > 0 && (!dev_codes || !dev_n_states || !dev_states))
        return fail(RAC_EINVAL, "rac_multistability: NULL argument");
    if (n_ic > kMaxStatesPerSet) return fail(RAC_EUNSUPPORTED, "rac_multistability: n_ic above 4096");
    if (n_sets > 0x7fffffffLL) return fail(RAC_EUNSUPPORTED, "rac_multistability: too many sets");
    if (n_sets == 0) return RAC_OK;
    int n_pow2 = 1;
    while (n_pow2 < n_ic) n_pow2 <<= 1;
    hipLaunchKernelGGL(multistability_kernel, dim3((unsigned)n_sets), dim3(kThreads), 0, (hipStream_t)hip_stream,
                       dev_codes, (int)n_ic, n_pow2, dev_n_states, dev_states);
    RAC_PP(hipGetLastError(), "rac_multistability: launch");
    return RAC_OK;
}

rac_status rac_state_counts(const uint64_t* dev_codes, int64_t n_rows, int64_t capacity, uint64_t* dev_keys,
                            int64_t* dev_counts, int64_t* dev_n_unique, void* hip_stream) {
    using namespace rac;
    if (!dev_keys || !dev_counts || !dev_n_unique || (n_rows > 0 && !dev_codes))
        return fail(RAC_EINVAL, "rac_state_counts: NULL argument");
    if (n_rows < 0 || capacity < 2 || capacity > (1LL << 30) || (capacity & (capacity - 1)))
        return fail(RAC_EINVAL, "rac_state_counts: capacity must be a power of two in [2, 2^30]");
    hipStream_t s = (hipStream_t)hip_stream;
    // Workspace: hash keys and counts, the unique counter and the overflow flag.
    const size_t bytes = (size_t)capacity * 16 + 256;
    char* ws = nullptr;
    RAC_PP(hipMallocAsync((void**)&ws, bytes, s), "rac_state_counts: workspace");
    auto* tk = (unsigned long long*)ws;
    auto* tc = tk + capacity;
    auto* nu = (unsigned long long*)(ws + (size_t)capacity * 16);
    int* ovf = (int*)(nu + 1);
    const int g = grid_for(capacity);
    hipLaunchKernelGGL(fill_kernel<unsigned long long>, dim3(g), dim3(kThreads), 0, s, tk, capacity,
                       (unsigned long long)kNoState);
    hipLaunchKernelGGL(fill_kernel<unsigned long long>, dim3(g), dim3(kThreads), 0, s, tc, capacity, 0ull);
    hipLaunchKernelGGL(fill_kernel<unsigned long long>, dim3(1), dim3(64), 0, s, nu, (int64_t)2, 0ull);
    hipLaunchKernelGGL(fill_kernel<uint64_t>, dim3(g), dim3(kThreads), 0, s, dev_keys, capacity, kNoState);
    hipLaunchKernelGGL(fill_kernel<int64_t>, dim3(g), dim3(kThreads), 0, s, dev_counts, capacity, (int64_t)0);
    if (n_rows > 0)
        hipLaunchKernelGGL(insert_kernel, dim3(std::min(grid_for(n_rows), 1024)), dim3(kThreads), 0, s, dev_codes,
                           n_rows, tk, tc, (uint64_t)(capacity - 1), ovf);
    hipLaunchKernelGGL(compact_kernel, dim3(g), dim3(kThreads), 0, s, tk, tc, capacity, dev_keys, dev_counts, nu);
    if (capacity <= kTile) {
        for (int64_t size = 2; size <= capacity; size <<= 1)
            for (int64_t stride = size >> 1; stride > 0; stride >>= 1)
                hipLaunchKernelGGL(bitonic_pass, dim3(g), dim3(kThreads), 0, s, dev_keys, dev_counts, capacity,
                                   size, stride);
    } else {
        const int tiles = (int)(capacity / kTile);
        hipLaunchKernelGGL(bitonic_tile, dim3(tiles), dim3(kThreads), 0, s, dev_keys, dev_counts, capacity,
                           (int64_t)2, (int64_t)kTile);
        for (int64_t size = 2 * kTile; size <= capacity; size <<= 1) {
            for (int64_t stride = size >> 1; stride >= kTile; stride >>= 1)
                hipLaunchKernelGGL(bitonic_pass, dim3(g), dim3(kThreads), 0, s, dev_keys, dev_counts, capacity,
                                   size, stride);
            hipLaunchKernelGGL(bitonic_tile, dim3(tiles), dim3(kThreads), 0, s, dev_keys, dev_counts, capacity,
                               size, size);
        }
    }
    hipLaunchKernelGGL(finish_counts_kernel, dim3(1), dim3(64), 0, s, nu, ovf, dev_n_unique);
    hipError_t le = hipGetLastError();
    hipError_t fe = hipFreeAsync(ws, s);
    RAC_PP(le, "rac_state_counts: launch");
    RAC_PP(fe, "rac_state_counts: free");
    return RAC_OK;
}

}  // extern "C"
