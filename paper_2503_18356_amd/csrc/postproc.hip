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
#include "fastdiv.h"
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

// Element e of x[rows][N]: row e / N, gene e % N, parameter set row / (n_t n_ic).
// Index arithmetic in 32 bits when the element count allows it.  With x and y
// 16-byte aligned (VEC) each thread takes four consecutive elements (16-byte
// loads and stores) and the last one the ragged tail; otherwise one element.
template <bool WIDE>
__device__ __forceinline__ float normalized(float xv, int64_t e, int N, int64_t P, int64_t rows_per_set,
                                            const FastDiv& by_n, const FastDiv& by_set,
                                            const float* __restrict__ G, const float* __restrict__ k) {
    int64_t r, p;
    if (WIDE) {
        r = e / N;
        p = r / rows_per_set;
    } else {
        r = fastdiv((uint32_t)e, by_n);
        p = fastdiv((uint32_t)r, by_set);
    }
    const int i = (int)(e - r * N);
    return __fdiv_rn(__fmul_rn(xv, k[i * P + p]), G[i * P + p]);
}

template <bool WIDE, bool VEC>
__global__ void normalize_kernel(const float* __restrict__ x, float* __restrict__ y, int64_t n_elem,
                                 int N, int64_t P, int64_t rows_per_set, FastDiv by_n, FastDiv by_set,
                                 const float* __restrict__ G, const float* __restrict__ k) {
    if (!VEC) {
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_elem;
             e += (int64_t)gridDim.x * blockDim.x)
            y[e] = normalized<WIDE>(x[e], e, N, P, rows_per_set, by_n, by_set, G, k);
        return;
    }
    const int64_t n4 = n_elem >> 2;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q <= n4;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = q << 2;
        if (q < n4) {
            const float4 xv = reinterpret_cast<const float4*>(x)[q];
            float4 yv;
            yv.x = normalized<WIDE>(xv.x, e, N, P, rows_per_set, by_n, by_set, G, k);
            yv.y = normalized<WIDE>(xv.y, e + 1, N, P, rows_per_set, by_n, by_set, G, k);
            yv.z = normalized<WIDE>(xv.z, e + 2, N, P, rows_per_set, by_n, by_set, G, k);
            yv.w = normalized<WIDE>(xv.w, e + 3, N, P, rows_per_set, by_n, by_set, G, k);
            reinterpret_cast<float4*>(y)[q] = yv;
        } else {
            for (int64_t t = e; t < n_elem; ++t)
                y[t] = normalized<WIDE>(x[t], t, N, P, rows_per_set, by_n, by_set, G, k);
        }
    }
}

template <typename T>
__global__ void fill_kernel(T* a, int64_t n, T v) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        a[e] = v;
}

// LDS histogram per wave (values cluster in few bins, so one shared copy per
// workgroup serialises its atomics four times as much), summed per bin at
// the end with one global atomic per bin and workgroup.
template <bool WIDE, bool VEC>
__global__ __launch_bounds__(kThreads) void histogram_kernel(const float* __restrict__ y, int64_t n_rows, int N,
                                                             FastDiv by_n, const int8_t* __restrict__ status,
                                                             int n_bins, unsigned long long* __restrict__ hist) {
    __shared__ unsigned int h[kThreads / 64][kMaxBins];
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
        for (int w = 0; w < kThreads / 64; ++w) h[w][b] = 0;
    __syncthreads();
    unsigned int* const mine = h[threadIdx.x >> 6];
    const int64_t n_elem = n_rows * N;
    auto add = [&](float v, int64_t e) {
        if (status && status[WIDE ? e / N : (int64_t)fastdiv((uint32_t)e, by_n)] != RAC_CONVERGED) return;
        atomicAdd(&mine[bin_of(v, n_bins)], 1u);
    };
    // Four consecutive elements per thread (16-byte loads; y 16-byte aligned),
    // the ragged tail last; otherwise one element per thread.
    const int64_t n4 = VEC ? n_elem >> 2 : -1;
    if (!VEC)
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_elem;
             e += (int64_t)gridDim.x * blockDim.x)
            add(y[e], e);
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q <= n4;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = q << 2;
        if (q < n4) {
            const float4 v = reinterpret_cast<const float4*>(y)[q];
            add(v.x, e);
            add(v.y, e + 1);
            add(v.z, e + 2);
            add(v.w, e + 3);
        } else {
            for (int64_t t = e; t < n_elem; ++t) add(y[t], t);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x) {
        unsigned int c = 0;
        for (int w = 0; w < kThreads / 64; ++w) c += h[w][b];
        if (c) atomicAdd(&hist[b], (unsigned long long)c);
    }
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

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// One wave per parameter set, for n_ic <= 128: the set's codes sit two per
// lane (indices lane and lane + 64, NO_STATE past n_ic), a bitonic network
// over the 128 keys runs in registers (cross-lane pairs by shuffles, the
// stride-64 pairs inside a lane), first occurrences are flagged against the
// preceding key and their output positions come from lane-masked popcounts
// of the ballots.
__global__ __launch_bounds__(kThreads) void multistability_wave(const uint64_t* __restrict__ codes, int64_t n_sets,
                                                                int n_ic, int* __restrict__ n_states,
                                                                uint64_t* __restrict__ states) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (p >= n_sets) return;  // uniform over the wave
    const uint64_t* c = codes + p * n_ic;
    uint64_t a = lane < n_ic ? c[lane] : kNoState;
    uint64_t b = lane + 64 < n_ic ? c[lane + 64] : kNoState;
    for (int size = 2; size <= 128; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride == 64) {  // size 128: pairs (lane, lane + 64), ascending
                const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
                a = lo;
                b = hi;
            } else {
                const uint64_t pa = shfl_u64(a, lane ^ stride), pb = shfl_u64(b, lane ^ stride);
                const bool lower = (lane & stride) == 0;
                const bool min_a = lower == ((lane & size) == 0);
                const bool min_b = lower == (((lane + 64) & size) == 0);
                a = (min_a == (pa < a)) ? pa : a;
                b = (min_b == (pb < b)) ? pb : b;
            }
        }
    }
    // Every lane takes part in every shuffle (a shuffle reads the source lane's
    // register, which must be active); the selects come afterwards.
    const int up1 = lane == 0 ? 0 : lane - 1;
    const uint64_t prev_a = shfl_u64(a, up1);
    const uint64_t last_a = shfl_u64(a, 63);
    const uint64_t sb = shfl_u64(b, up1);
    const uint64_t prev_b = lane == 0 ? last_a : sb;
    const bool fa = a != kNoState && (lane == 0 || a != prev_a);
    const bool fb = b != kNoState && b != prev_b;
    const uint64_t ma = __ballot(fa), mb = __ballot(fb);
    const uint64_t below = (1ull << lane) - 1ull;
    const int na = __popcll(ma), total = na + __popcll(mb);
    uint64_t* out = states + p * n_ic;
    if (fa) out[__popcll(ma & below)] = a;
    if (fb) out[na + __popcll(mb & below)] = b;
    for (int i = total + lane; i < n_ic; i += 64) out[i] = kNoState;
    if (lane == 0) n_states[p] = total;
}

// One workgroup per parameter set, for larger n_ic: bitonic sort of its n_ic
// codes in LDS (n_pow2 keys, dynamic shared memory), then the distinct codes
// (NO_STATE excluded) in ascending order, placed by a block-wide scan of the
// per-thread counts.
__global__ __launch_bounds__(kThreads) void multistability_kernel(const uint64_t* __restrict__ codes, int n_ic,
                                                                  int n_pow2, int* __restrict__ n_states,
                                                                  uint64_t* __restrict__ states) {
    extern __shared__ uint64_t key[];
    __shared__ int wsum[kThreads / 64];
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
    // Exclusive scan of the counts: inside each wave by shuffles, then over
    // the wave totals.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = mine;
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        if (w < wave) before += wsum[w];
        total += wsum[w];
    }
    uint64_t* out = states + p * n_ic;
    int pos = before + incl - mine;
    for (int i = beg; i < end; ++i)
        if (key[i] != kNoState && (i == 0 || key[i] != key[i - 1])) out[pos++] = key[i];
    for (int i = total + threadIdx.x; i < n_ic; i += blockDim.x) out[i] = kNoState;
    if (threadIdx.x == 0) n_states[p] = total;
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

// Clears the hash table (keys NO_STATE, counts 0), the unique counter and
// overflow flag, and the caller's output arrays, in one pass.
__global__ void clear_tables(unsigned long long* tk, unsigned long long* tc, unsigned long long* flags,
                             uint64_t* out_keys, int64_t* out_counts, int64_t cap) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cap;
         e += (int64_t)gridDim.x * blockDim.x) {
        tk[e] = kNoState;
        tc[e] = 0;
        out_keys[e] = kNoState;
        out_counts[e] = 0;
        if (e < 2) flags[e] = 0;
    }
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

// Bitonic sorting network over the compacted (key, count) pairs, ascending
// by key.  The compacted entries fill [0, n_unique) and every later entry
// holds the largest key, so only the first m = n_unique rounded up to a
// power of two entries need sorting: stages of sizes above m would merge a
// sorted head with a constant tail and change nothing, and the kernels read
// m from the device and skip them (the launches stay fixed, so nothing waits
// for the count on the host).  Passes with stride < kTile run inside one LDS
// tile (bitonic_tile: every size up to the tile in the first call, then the
// short strides of each larger size); longer strides are global passes.
constexpr int kTile = 2048;

__device__ __forceinline__ int64_t sort_extent(const unsigned long long* n_unique) {
    int64_t m = 1;
    while ((unsigned long long)m < *n_unique) m <<= 1;
    return m;
}

// tile = min(n, kTile) pairs per workgroup.
__global__ __launch_bounds__(kThreads) void bitonic_tile(uint64_t* keys, int64_t* vals, int64_t tile,
                                                         int64_t size_lo, int64_t size_hi,
                                                         const unsigned long long* n_unique) {
    __shared__ uint64_t k[kTile];
    __shared__ int64_t v[kTile];
    const int64_t m = sort_extent(n_unique);
    const int64_t base = (int64_t)blockIdx.x * tile;
    if (base >= m || m < 2) return;
    const int lim = (int)(m - base < tile ? m - base : tile);  // a power of two
    if (size_hi > m) size_hi = m;
    if (size_lo > size_hi) return;
    for (int i = threadIdx.x; i < lim; i += blockDim.x) {
        k[i] = keys[base + i];
        v[i] = vals[base + i];
    }
    __syncthreads();
    for (int64_t size = size_lo; size <= size_hi; size <<= 1) {
        for (int64_t stride = (size < lim ? size : lim) >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < lim; i += blockDim.x) {
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
    for (int i = threadIdx.x; i < lim; i += blockDim.x) {
        keys[base + i] = k[i];
        vals[base + i] = v[i];
    }
}

__global__ void bitonic_pass(uint64_t* keys, int64_t* vals, int64_t size, int64_t stride,
                             const unsigned long long* n_unique) {
    const int64_t m = sort_extent(n_unique);
    if (size > m) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
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

// The paper's steady-state flag per trajectory: 1 unless CONVERGED.
__global__ void steady_flag_kernel(const int8_t* __restrict__ status, int64_t n, uint8_t* __restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = status[i] == RAC_CONVERGED ? 0 : 1;
}

}  // namespace
}  // namespace rac

extern "C" {

int32_t rac_not_steady_flag(int32_t status) { return status == RAC_CONVERGED ? 0 : 1; }

rac_status rac_steady_flags(const int8_t* dev_status, int64_t n, uint8_t* dev_flag, void* hip_stream) {
    using namespace rac;
    if (n < 0) return fail(RAC_EINVAL, "rac_steady_flags: n < 0");
    if (n == 0) return RAC_OK;
    if (!dev_status || !dev_flag) return fail(RAC_EINVAL, "rac_steady_flags: NULL array");
    hipLaunchKernelGGL(steady_flag_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)hip_stream,
                       dev_status, n, dev_flag);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RAC_EDEVICE, std::string("rac_steady_flags: ") + hipGetErrorString(e));
    return RAC_OK;
}

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
    const int64_t rows_per_set = (int64_t)n_ic * n_t;
    const bool vec = (((uintptr_t)dev_x | (uintptr_t)dev_y) & 15) == 0;
    const dim3 grid(grid_for(vec ? n_elem / 4 + 1 : n_elem));
    const bool narrow = n_elem <= 0xffffffffLL;
    const FastDiv by_n = narrow ? make_fastdiv((uint32_t)N) : FastDiv{1, 0, 0};
    const FastDiv by_set = narrow ? make_fastdiv((uint32_t)rows_per_set) : FastDiv{1, 0, 0};
    auto kern = narrow ? (vec ? normalize_kernel<false, true> : normalize_kernel<false, false>)
                       : (vec ? normalize_kernel<true, true> : normalize_kernel<true, false>);
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), 0, s, dev_x, dev_y, n_elem, N, (int64_t)p->n_sets, rows_per_set,
                       by_n, by_set, p->G, p->k);
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
        const int64_t n_elem = n_rows * n_genes;
        const bool vec = ((uintptr_t)dev_y & 15) == 0;
        const dim3 grid(grid_for(vec ? n_elem / 4 + 1 : n_elem, kThreads * 4));
        const bool narrow = n_elem <= 0xffffffffLL;
        auto kern = narrow ? (vec ? histogram_kernel<false, true> : histogram_kernel<false, false>)
                           : (vec ? histogram_kernel<true, true> : histogram_kernel<true, false>);
        hipLaunchKernelGGL(kern, grid, dim3(kThreads), 0, s, dev_y, n_rows, (int)n_genes,
                           narrow ? make_fastdiv((uint32_t)n_genes) : FastDiv{1, 0, 0}, dev_status, (int)n_bins,
                           (unsigned long long*)dev_hist);
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
    if (n_pow2 <= 128) {
        const int64_t per = kThreads / 64;
        hipLaunchKernelGGL(multistability_wave, dim3((unsigned)((n_sets + per - 1) / per)), dim3(kThreads), 0,
                           (hipStream_t)hip_stream, dev_codes, n_sets, (int)n_ic, dev_n_states, dev_states);
    } else {
        hipLaunchKernelGGL(multistability_kernel, dim3((unsigned)n_sets), dim3(kThreads),
                           (unsigned)(n_pow2 * sizeof(uint64_t)), (hipStream_t)hip_stream, dev_codes, (int)n_ic,
                           n_pow2, dev_n_states, dev_states);
    }
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
    hipLaunchKernelGGL(clear_tables, dim3(g), dim3(kThreads), 0, s, tk, tc, nu, dev_keys, dev_counts, capacity);
    if (n_rows > 0)
        hipLaunchKernelGGL(insert_kernel, dim3(std::min(grid_for(n_rows), 1024)), dim3(kThreads), 0, s, dev_codes,
                           n_rows, tk, tc, (uint64_t)(capacity - 1), ovf);
    hipLaunchKernelGGL(compact_kernel, dim3(g), dim3(kThreads), 0, s, tk, tc, capacity, dev_keys, dev_counts, nu);
    if (capacity <= kTile) {
        hipLaunchKernelGGL(bitonic_tile, dim3(1), dim3(kThreads), 0, s, dev_keys, dev_counts, capacity,
                           (int64_t)2, capacity, nu);
    } else {
        const int tiles = (int)(capacity / kTile);
        hipLaunchKernelGGL(bitonic_tile, dim3(tiles), dim3(kThreads), 0, s, dev_keys, dev_counts, (int64_t)kTile,
                           (int64_t)2, (int64_t)kTile, nu);
        for (int64_t size = 2 * kTile; size <= capacity; size <<= 1) {
            for (int64_t stride = size >> 1; stride >= kTile; stride >>= 1)
                hipLaunchKernelGGL(bitonic_pass, dim3(g), dim3(kThreads), 0, s, dev_keys, dev_counts, size, stride,
                                   nu);
            hipLaunchKernelGGL(bitonic_tile, dim3(tiles), dim3(kThreads), 0, s, dev_keys, dev_counts, (int64_t)kTile,
                               size, size, nu);
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
