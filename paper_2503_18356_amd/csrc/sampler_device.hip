// Device-side parameter and initial-condition sampling: the same counter-based
// draws and the same FP64 range mappings as rac_sample_params, one thread per
// (set, parameter slot), so a request can be sampled where it is integrated.
// Results equal the host sampler bit for bit: every step is an exactly
// rounded IEEE operation (no contraction into fused multiply-adds).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rac_internal.h"

namespace rac {
namespace {

// Philox4x64-10 (Salmon et al., SC'11), as on the host.
__device__ __forceinline__ void philox_block(uint64_t w[4], uint64_t ka, uint64_t kb) {
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

__device__ __forceinline__ double draw(uint64_t seed, uint64_t index, uint64_t slot, uint64_t domain) {
    uint64_t w[4] = {index, slot >> 2, domain, 0};
    philox_block(w, seed, 0);
    return (double)(w[slot & 3] >> 11) * (1.0 / 9007199254740992.0);
}

// a + b * c with separate roundings (never fused).
__device__ __forceinline__ double lin(double a, double b, double c) { return __dadd_rn(a, __dmul_rn(b, c)); }

struct SampleArgs {
    const int8_t* sign;  // [E] device
    uint64_t seed;
    int64_t set_begin, n_sets;
    int32_t N, E, n_ic;
    double g_min, g_span, k_min, k_span, la_min, la_span, inv_lo, inv_span;
    double M, t_lo, t_span;
    int32_t n_min, n_span;
    int32_t n_continuous;
    double nc_span;  // n_max - n_min (continuous option)
    float *G, *k, *T, *lam, *ic, *nf;
    uint8_t* n;
    // Generator tables (device; NULL for uniform draws with one threshold scale).
    int32_t method;
    const double* scale;      // [E] threshold scale per edge, or NULL: all M
    const uint32_t* sobol_v;  // [dims][32]
    const uint32_t* shift0;   // [2N + 3E]
    const uint32_t* shift1;   // [N]
    const uint64_t* key0;     // [2N + 3E][4]
    const uint64_t* key1;     // [N][4]
    int64_t lhs_n0, lhs_n1;
    int32_t lhs_w0, lhs_w1;
};

__device__ uint64_t lhs_cell(uint64_t x, const uint64_t* key, int w, uint64_t n) {
    const uint64_t mask = w >= 64 ? ~0ull : (1ull << w) - 1;
    const int sh = w / 2 > 0 ? w / 2 : 1;
    do {
        for (int r = 0; r < 4; ++r) {
            x = (x ^ key[r]) & mask;
            x = (x * 0x9E3779B97F4A7C15ull) & mask;
            x ^= x >> sh;
        }
    } while (x >= n);
    return x;
}

// The unit-cube coordinate of slot q for item a (domain 0 parameter sets,
// 1 initial conditions), as on the host.
__device__ double unit(const SampleArgs& a, uint64_t item, uint64_t q, int domain) {
    if (a.method == RAC_SAMPLE_SOBOL) {
        uint32_t x = 0;
        const uint32_t* v = a.sobol_v + q * 32;
        for (int b = 0; b < 32; ++b)
            if ((item >> b) & 1) x ^= v[b];
        x ^= domain ? a.shift1[q] : a.shift0[q];
        return (double)x * (1.0 / 4294967296.0);
    }
    if (a.method == RAC_SAMPLE_LHS) {
        const uint64_t* key = (domain ? a.key1 : a.key0) + 4 * q;
        const int64_t n = domain ? a.lhs_n1 : a.lhs_n0;
        const uint64_t cell = lhs_cell(item, key, domain ? a.lhs_w1 : a.lhs_w0, (uint64_t)n);
        return __ddiv_rn(__dadd_rn((double)cell, draw(a.seed, item, q, 6 + domain)), (double)n);
    }
    return draw(a.seed, item, q, domain);
}

__global__ __launch_bounds__(256) void sample_kernel(SampleArgs a) {
    const int64_t slots = 2 * (int64_t)a.N + 3 * (int64_t)a.E;
    const int64_t total = slots * a.n_sets;
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * blockDim.x) {
        // Set index fastest, so each parameter row is written coalesced.
        const int64_t j = id % a.n_sets;
        const int64_t q = id / a.n_sets;
        const uint64_t p = (uint64_t)(a.set_begin + j);
        const double u = unit(a, p, (uint64_t)q, 0);
        if (q < a.N) {
            a.G[q * a.n_sets + j] = (float)lin(a.g_min, a.g_span, u);
        } else if (q < 2 * a.N) {
            a.k[(q - a.N) * a.n_sets + j] = (float)lin(a.k_min, a.k_span, u);
        } else {
            const int64_t r = q - 2 * a.N, e = r / 3, which = r % 3;
            if (which == 0) {
                a.T[e * a.n_sets + j] = (float)__dmul_rn(a.scale ? a.scale[e] : a.M, lin(a.t_lo, a.t_span, u));
            } else if (which == 1) {
                if (a.n_continuous) {
                    a.nf[e * a.n_sets + j] = (float)lin((double)a.n_min, a.nc_span, u);
                } else {
                    int32_t kk = (int32_t)floor(__dmul_rn(u, (double)a.n_span));
                    if (kk > a.n_span - 1) kk = a.n_span - 1;
                    a.n[e * a.n_sets + j] = (uint8_t)(a.n_min + kk);
                    if (a.nf) a.nf[e * a.n_sets + j] = (float)(a.n_min + kk);
                }
            } else {
                const double l = a.sign[e] > 0 ? lin(a.la_min, a.la_span, u)
                                               : __ddiv_rn(1.0, lin(a.inv_lo, a.inv_span, u));
                a.lam[e * a.n_sets + j] = (float)l;
            }
        }
    }
    if (a.ic) {
        const int64_t nic = (int64_t)a.n_ic * a.N;
        for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < nic;
             id += (int64_t)gridDim.x * blockDim.x) {
            const int64_t c = id / a.N, i = id % a.N;
            a.ic[id] = (float)unit(a, (uint64_t)c, (uint64_t)i, 1);
        }
    }
}

}  // namespace

// Shared with the host sampler: validity check and the median of G/k.
bool sample_ranges_ok(const rac_ranges& r);
double sample_ratio_median(const rac_ranges& r);

}  // namespace rac

extern "C" rac_status rac_sample_params_device(const rac_topology* topo, const rac_ranges* ranges,
                                               uint64_t seed, int64_t set_begin, int64_t n_sets,
                                               int32_t n_ic, rac_params_view* dev_out,
                                               float* dev_ic_frac, void* hip_stream) {
    using namespace rac;
    if (!topo) return fail(RAC_EINVAL, "rac_sample_params_device: NULL topology");
    if (!dev_out) return fail(RAC_EINVAL, "rac_sample_params_device: NULL output view");
    if (n_sets < 0 || n_ic < 0 || set_begin < 0)
        return fail(RAC_EINVAL, "rac_sample_params_device: negative count or offset");
    if (dev_out->n_sets != n_sets) return fail(RAC_EINVAL, "rac_sample_params_device: out->n_sets != n_sets");
    const int64_t N = topo->n_genes, E = topo->n_edges;
    rac_ranges r;
    if (ranges)
        r = *ranges;
    else
        rac_default_ranges(&r);
    if (!sample_ranges_ok(r)) return fail(RAC_EINVAL, "rac_sample_params_device: invalid ranges");
    if (n_sets > 0 && (!dev_out->G || !dev_out->k ||
                       (E > 0 && (!dev_out->T || !dev_out->lam || (r.n_continuous ? !dev_out->nf : !dev_out->n)))))
        return fail(RAC_EINVAL, "rac_sample_params_device: NULL parameter array");
    if (n_sets == 0 && (n_ic == 0 || !dev_ic_frac)) return RAC_OK;
    const DevicePlan* dp = nullptr;
    rac_status st = get_device_plan(topo, 1, &dp);  // carries the device copy of the signs
    if (st != RAC_OK) return st;
    SampleArgs a;
    std::memset(&a, 0, sizeof(a));
    a.sign = dp->sign;
    a.seed = seed;
    a.set_begin = set_begin;
    a.n_sets = n_sets;
    a.N = (int32_t)N;
    a.E = (int32_t)E;
    a.n_ic = n_ic;
    a.g_min = r.g_min;
    a.g_span = r.g_max - r.g_min;
    a.k_min = r.k_min;
    a.k_span = r.k_max - r.k_min;
    a.la_min = r.lam_act_min;
    a.la_span = r.lam_act_max - r.lam_act_min;
    a.inv_lo = 1.0 / r.lam_inh_max;
    a.inv_span = 1.0 / r.lam_inh_min - a.inv_lo;
    a.M = sample_ratio_median(r);
    a.t_lo = r.t_lo;
    a.t_span = r.t_hi - r.t_lo;
    a.n_min = r.n_min;
    a.n_span = r.n_max - r.n_min + 1;
    a.n_continuous = r.n_continuous;
    a.nc_span = (double)(r.n_max - r.n_min);
    a.nf = dev_out->nf;
    a.G = dev_out->G;
    a.k = dev_out->k;
    a.T = dev_out->T;
    a.lam = dev_out->lam;
    a.n = dev_out->n;
    a.ic = dev_ic_frac;
    a.method = r.method;
    hipStream_t stream = (hipStream_t)hip_stream;
    SampleTables tb;
    st = make_sample_tables(topo, r, seed, set_begin, n_sets, n_ic, &tb);
    if (st != RAC_OK) return st;
    bool one_scale = true;
    for (double v : tb.scale) one_scale = one_scale && v == a.M;
    char* dev_block = nullptr;
    if (r.method != RAC_SAMPLE_UNIFORM || !one_scale) {
        // One upload of every table the kernel reads; the staging copy is
        // freed by a host callback once the copy has run.
        const int64_t D = 2 * N + 3 * E;
        const int64_t dims = r.method == RAC_SAMPLE_SOBOL ? std::max(D, N) : 0;
        auto* host = new std::vector<char>();
        auto put = [&](const void* src, size_t bytes) {
            const size_t off = (host->size() + 15) / 16 * 16;
            host->resize(off + bytes);
            if (bytes) std::memcpy(host->data() + off, src, bytes);
            return off;
        };
        const size_t o_scale = put(tb.scale.data(), tb.scale.size() * sizeof(double));
        const size_t o_v = put(tb.sobol_v, (size_t)dims * 32 * sizeof(uint32_t));
        const size_t o_s0 = put(tb.shift0.data(), tb.shift0.size() * sizeof(uint32_t));
        const size_t o_s1 = put(tb.shift1.data(), tb.shift1.size() * sizeof(uint32_t));
        const size_t o_k0 = put(tb.lhs_key0.data(), tb.lhs_key0.size() * sizeof(uint64_t));
        const size_t o_k1 = put(tb.lhs_key1.data(), tb.lhs_key1.size() * sizeof(uint64_t));
        hipError_t he = hipMallocAsync((void**)&dev_block, std::max<size_t>(host->size(), 16), stream);
        if (he == hipSuccess)
            he = hipMemcpyAsync(dev_block, host->data(), host->size(), hipMemcpyHostToDevice, stream);
        if (he == hipSuccess)
            he = hipLaunchHostFunc(stream, [](void* p) { delete static_cast<std::vector<char>*>(p); }, host);
        else
            delete host;
        if (he != hipSuccess)
            return fail(RAC_EDEVICE, std::string("sampler table upload: ") + hipGetErrorString(he));
        a.scale = (const double*)(dev_block + o_scale);
        a.sobol_v = (const uint32_t*)(dev_block + o_v);
        a.shift0 = (const uint32_t*)(dev_block + o_s0);
        a.shift1 = (const uint32_t*)(dev_block + o_s1);
        a.key0 = (const uint64_t*)(dev_block + o_k0);
        a.key1 = (const uint64_t*)(dev_block + o_k1);
        a.lhs_n0 = tb.lhs_n0;
        a.lhs_n1 = tb.lhs_n1;
        a.lhs_w0 = tb.lhs_w0;
        a.lhs_w1 = tb.lhs_w1;
    }
    const int64_t work = std::max<int64_t>((2 * N + 3 * E) * n_sets, (int64_t)n_ic * N);
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 65536));
    hipLaunchKernelGGL(sample_kernel, dim3(blocks), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (dev_block) {
        hipError_t fe = hipFreeAsync(dev_block, stream);
        if (e == hipSuccess) e = fe;
    }
    if (e != hipSuccess) return fail(RAC_EDEVICE, std::string("sample kernel launch: ") + hipGetErrorString(e));
    return RAC_OK;
}
