// Boolean Ising formalism (Eq. 3) on the device: one trajectory per lane,
// states bit-packed in W 64-bit words, the coupling of each gene held as
// bit masks of its activating and inhibiting regulators in LDS.  A gene's
// signed input sum is a difference of two popcounts:
//   off = 0:   sum = a - h
//   off = -1:  sum = 2 (a - h) - (|act| - |inh|)
// where a (h) counts the activating (inhibiting) regulators that are on.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "rac.h"
#include "rac_internal.h"

namespace rac {
namespace {

constexpr int kMaxIsingGenes = 256;
constexpr int kIsingBlock = 256;

// Philox4x64-10 (Salmon et al., SC'11).
__device__ __forceinline__ void philox(uint64_t w[4], uint64_t ka, uint64_t kb) {
    const uint64_t kMulA = 0xD2E7470EE14C6C93ULL, kMulB = 0xCA5A826395121157ULL;
    const uint64_t kWeylA = 0x9E3779B97F4A7C15ULL, kWeylB = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa_hi = __umul64hi(kMulA, w[0]), pa_lo = kMulA * w[0];
        const uint64_t pb_hi = __umul64hi(kMulB, w[2]), pb_lo = kMulB * w[2];
        const uint64_t o0 = pb_hi ^ w[1] ^ ka;
        const uint64_t o2 = pa_hi ^ w[3] ^ kb;
        w[0] = o0;
        w[1] = pb_lo;
        w[2] = o2;
        w[3] = pa_lo;
        ka += kWeylA;
        kb += kWeylB;
    }
}

struct IsingArgs {
    const uint64_t* masks;  // [N][2][W]: activating, inhibiting regulators
    const int32_t* order;   // async update order or NULL
    const uint64_t* init;   // [n_traj][W] or NULL (random states)
    uint64_t* final_state;  // [n_traj][W]
    int32_t* steps;
    int8_t* status;
    unsigned long long* evals;  // optional: gene evaluations performed, summed
    int64_t n_traj;
    uint64_t seed;
    int32_t N, low, max_steps, check_every, order_len, async;
};

template <int W>
__global__ __launch_bounds__(kIsingBlock) void ising_kernel(IsingArgs a) {
    __shared__ uint64_t m_act[kMaxIsingGenes][W], m_inh[kMaxIsingGenes][W];
    __shared__ int bias[kMaxIsingGenes];  // |act| - |inh|, used when off = -1
    for (int i = threadIdx.x; i < a.N; i += blockDim.x) {
        int na = 0, nh = 0;
        for (int w = 0; w < W; ++w) {
            m_act[i][w] = a.masks[((size_t)i * 2 + 0) * W + w];
            m_inh[i][w] = a.masks[((size_t)i * 2 + 1) * W + w];
            na += __popcll(m_act[i][w]);
            nh += __popcll(m_inh[i][w]);
        }
        bias[i] = na - nh;
    }
    __syncthreads();
    const int N = a.N;
    // The state gene i moves to from s (Eq. 3); ties keep the current bit.
    auto next_bit = [&](const uint64_t (&s)[W], int i) -> uint64_t {
        int act = 0, inh = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            act += __popcll(s[w] & m_act[i][w]);
            inh += __popcll(s[w] & m_inh[i][w]);
        }
        const int sum = a.low == 0 ? act - inh : 2 * (act - inh) - bias[i];
        const uint64_t cur = (s[i >> 6] >> (i & 63)) & 1ull;
        return sum > 0 ? 1ull : (sum < 0 ? 0ull : cur);
    };
    auto sync_map = [&](const uint64_t (&s)[W], uint64_t (&out)[W]) {
#pragma unroll
        for (int w = 0; w < W; ++w) out[w] = 0;
        for (int i = 0; i < N; ++i) out[i >> 6] |= next_bit(s, i) << (i & 63);
    };
    auto same = [&](const uint64_t (&x)[W], const uint64_t (&y)[W]) {
        bool eq = true;
#pragma unroll
        for (int w = 0; w < W; ++w) eq = eq && x[w] == y[w];
        return eq;
    };
    // Persistent lanes: a lane takes trajectories t, t + stride, ... and
    // starts the next as soon as one ends, so a wave no longer waits for
    // the slowest of its 64 trajectories before any lane moves on.
    uint64_t lane_evals = 0;  // gene evaluations this lane performed
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint64_t s[W], nxt[W], ref[W];
    uint64_t blk[4] = {0, 0, 0, 0};
    int st = 1, steps = 0, step = 0, ref_at = 0, save_at = 1, left = -1, u = 0;
    bool have = false, wait = false;
    auto start = [&]() {
        have = t < a.n_traj;
        if (!have) return;
        if (a.init) {
#pragma unroll
            for (int w = 0; w < W; ++w) s[w] = a.init[t * W + w];
        } else {
            // Gene i on when the top bit of word i % 4 of block (t, i / 4, 9, 0)
            // is set (its 53-bit uniform is >= 1/2).
#pragma unroll
            for (int w = 0; w < W; ++w) s[w] = 0;
            for (int i = 0; i < N; i += 4) {
                uint64_t b[4] = {(uint64_t)t, (uint64_t)(i >> 2), 9, 0};
                philox(b, a.seed, 0);
                for (int j = 0; j < 4 && i + j < N; ++j) s[(i + j) >> 6] |= (b[j] >> 63) << ((i + j) & 63);
            }
        }
        st = 1;
        steps = a.max_steps;
        step = 0;
        u = 0;
        left = -1;
#pragma unroll
        for (int w = 0; w < W; ++w) ref[w] = s[w];
        ref_at = 0;
        save_at = 1;
    };
    auto finish = [&]() {
#pragma unroll
        for (int w = 0; w < W; ++w) a.final_state[t * W + w] = s[w];
        if (a.steps) a.steps[t] = steps;
        if (a.status) a.status[t] = (int8_t)st;
        t += stride;
        start();
    };
    start();
    if (!a.async) {
        // One map evaluation per lane per iteration.  The map is
        // deterministic, so a state seen before means the trajectory is
        // periodic from there on: its state after max_steps updates is
        // reached by stepping only the remainder (`left`) of the updates
        // left modulo the period.  States are compared with a checkpoint
        // taken after 1, 2, 4, 8, ... updates, which finds a cycle of period
        // p after a transient of length m within 2 max(m, p) + p updates
        // (Brent's cycle detection).
        while (__ballot(have) != 0) {
            if (!have) continue;
            sync_map(s, nxt);
            lane_evals += N;
            if (left > 0) {
#pragma unroll
                for (int w = 0; w < W; ++w) s[w] = nxt[w];
                if (--left == 0) finish();
            } else if (same(nxt, s)) {
                st = 0;
                steps = step;
                finish();
            } else if (step == a.max_steps) {
                finish();
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w) s[w] = nxt[w];
                const int done = ++step;  // updates applied to s
                if (same(s, ref)) {
                    left = (a.max_steps - done) % (done - ref_at);
                    if (left == 0) finish();
                } else if (done == save_at) {
#pragma unroll
                    for (int w = 0; w < W; ++w) ref[w] = s[w];
                    ref_at = done;
                    save_at = done < (1 << 29) ? 2 * done : done;
                }
            }
        }
    } else {
        // Rounds of `every` updates.  Every lane's fixed-point tests fall on
        // a round start (u % every == 0), so the wave runs the test's full
        // map evaluation once per round for all lanes; a trajectory started
        // in a round's test phase waits for the next round's test.
        const int every = a.check_every > 0 ? a.check_every : N;
        while (__ballot(have) != 0) {
            if (have) {
                if (u % every == 0) {
                    sync_map(s, nxt);
                    lane_evals += N;
                    if (same(nxt, s)) {
                        st = 0;
                        steps = u;
                        finish();
                        wait = true;
                    } else if (u == a.max_steps) {
                        finish();
                        wait = true;
                    }
                } else if (u == a.max_steps) {
                    finish();
                    wait = true;
                }
            }
            for (int k = 0; k < every; ++k) {
                const bool busy = have && !wait && u < a.max_steps;
                if (__ballot(busy) == 0) break;  // bounded by the updates left, not by `every`
                if (!busy) continue;
                int i;
                if (a.order) {
                    i = a.order[u % a.order_len];
                } else {
                    // Eight gene choices per Philox block: the 32-bit halves of
                    // its words, scaled to [0, N) by a multiply-shift.
                    if ((u & 7) == 0) {
                        blk[0] = (uint64_t)t;
                        blk[1] = (uint64_t)(u >> 3);
                        blk[2] = 8;
                        blk[3] = 0;
                        philox(blk, a.seed, 0);
                    }
                    const uint64_t w64 = blk[(u & 7) >> 1];
                    const uint64_t h = (u & 1) ? (w64 >> 32) : (w64 & 0xFFFFFFFFull);
                    i = (int)((h * (uint64_t)N) >> 32);
                }
                const uint64_t b = next_bit(s, i);
                ++lane_evals;
                s[i >> 6] = (s[i >> 6] & ~(1ull << (i & 63))) | (b << (i & 63));
                ++u;
            }
            wait = false;
        }
    }
    if (a.evals) {
        // One atomic per wave: the wave's sum gathered by shuffles.
        for (int off = 32; off > 0; off >>= 1) lane_evals += __shfl_xor(lane_evals, off);
        if ((threadIdx.x & 63) == 0) atomicAdd(a.evals, (unsigned long long)lane_evals);
    }
}

}  // namespace
}  // namespace rac

extern "C" {

void rac_default_ising_opts(rac_ising_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = RAC_ISING_SYNC;
    o->low = 0;
    o->max_steps = 1000;
    o->check_every = 0;
    o->seed = 0;
    o->order = nullptr;
    o->order_len = 0;
    o->dev_evals = nullptr;
}

rac_status rac_ising(const rac_topology* topo, const rac_ising_opts* o, int64_t n_traj, const uint64_t* dev_init,
                     uint64_t* dev_final, int32_t* dev_steps, int8_t* dev_status, void* hip_stream) {
    using namespace rac;
    if (!topo || !o) return fail(RAC_EINVAL, "rac_ising: NULL argument");
    if (n_traj < 0) return fail(RAC_EINVAL, "rac_ising: n_traj < 0");
    if (n_traj > 0 && !dev_final) return fail(RAC_EINVAL, "rac_ising: NULL final-state array");
    if (o->mode != RAC_ISING_SYNC && o->mode != RAC_ISING_ASYNC)
        return fail(RAC_EINVAL, "rac_ising: mode must be RAC_ISING_SYNC or RAC_ISING_ASYNC");
    if (o->low != 0 && o->low != -1) return fail(RAC_EINVAL, "rac_ising: low must be 0 or -1");
    if (o->max_steps < 0 || o->check_every < 0) return fail(RAC_EINVAL, "rac_ising: negative step counts");
    if (o->order && o->order_len < 1) return fail(RAC_EINVAL, "rac_ising: order_len < 1");
    const int N = topo->n_genes;
    if (N > kMaxIsingGenes) return fail(RAC_EUNSUPPORTED, "rac_ising: more than 256 genes");
    if (o->order)
        for (int k = 0; k < o->order_len; ++k)
            if (o->order[k] < 0 || o->order[k] >= N) return fail(RAC_EINVAL, "rac_ising: gene index in order out of range");
    if (n_traj == 0) return RAC_OK;
    const int W = (N + 63) / 64;
    hipStream_t s = (hipStream_t)hip_stream;
    // Grid: synchronous calls take a lane per trajectory up to 256 blocks per
    // CU; asynchronous ones at most 16 blocks (64 waves) per CU, past which
    // each lane works through several trajectories and refills as each ends.
    // Refill pays off where trajectories are long and uneven (asynchronous,
    // 10^7 states: 349 against 457 ms) and costs where they are short
    // (synchronous, 10^7 states: 20.5 against 13.3 ms: a random initial
    // state takes six Philox blocks, which the whole wave waits for whenever
    // one of its lanes starts a trajectory).
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
        return fail(RAC_EDEVICE, "rac_ising: device query failed");
    const int per_cu = o->mode == RAC_ISING_ASYNC ? 16 : 256;
    const int blocks = (int)std::min<int64_t>((n_traj + kIsingBlock - 1) / kIsingBlock, (int64_t)n_cu * per_cu);
    // Regulator masks per gene, uploaded stream-ordered; a host callback frees
    // the staging copy once the copy has run.
    const size_t n_mask = (size_t)N * 2 * W;
    const size_t n_order = o->order ? ((size_t)o->order_len + 1) / 2 : 0;  // two i32 per u64
    auto* host = new std::vector<uint64_t>(n_mask + n_order, 0);
    for (int e = 0; e < topo->n_edges; ++e) {
        const int i = topo->dst[e], j = topo->src[e];
        (*host)[((size_t)i * 2 + (topo->sign[e] > 0 ? 0 : 1)) * W + (j >> 6)] |= 1ull << (j & 63);
    }
    if (o->order) std::memcpy(host->data() + n_mask, o->order, sizeof(int32_t) * (size_t)o->order_len);
    uint64_t* dev_masks = nullptr;
    const size_t bytes = host->size() * sizeof(uint64_t);
    hipError_t e = hipMallocAsync((void**)&dev_masks, bytes, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dev_masks, host->data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipLaunchHostFunc(s, [](void* p) { delete static_cast<std::vector<uint64_t>*>(p); }, host);
    else
        delete host;
    if (e != hipSuccess) return fail(RAC_EDEVICE, std::string("rac_ising: upload: ") + hipGetErrorString(e));
    IsingArgs a;
    std::memset(&a, 0, sizeof(a));
    a.masks = dev_masks;
    a.order = o->order ? (const int32_t*)(dev_masks + n_mask) : nullptr;
    a.init = dev_init;
    a.final_state = dev_final;
    a.steps = dev_steps;
    a.status = dev_status;
    a.evals = o->dev_evals;
    a.n_traj = n_traj;
    a.seed = o->seed;
    a.N = N;
    a.low = o->low;
    a.max_steps = o->max_steps;
    a.check_every = o->check_every;
    a.order_len = o->order_len;
    a.async = o->mode == RAC_ISING_ASYNC;

    if (W == 1)
        hipLaunchKernelGGL(ising_kernel<1>, dim3(blocks), dim3(kIsingBlock), 0, s, a);
    else if (W == 2)
        hipLaunchKernelGGL(ising_kernel<2>, dim3(blocks), dim3(kIsingBlock), 0, s, a);
    else if (W == 3)
        hipLaunchKernelGGL(ising_kernel<3>, dim3(blocks), dim3(kIsingBlock), 0, s, a);
    else
        hipLaunchKernelGGL(ising_kernel<4>, dim3(blocks), dim3(kIsingBlock), 0, s, a);
    e = hipGetLastError();
    hipError_t fe = hipFreeAsync(dev_masks, s);
    if (e == hipSuccess) e = fe;
    if (e != hipSuccess) return fail(RAC_EDEVICE, std::string("rac_ising: launch: ") + hipGetErrorString(e));
    return RAC_OK;
}

}  // extern "C"
