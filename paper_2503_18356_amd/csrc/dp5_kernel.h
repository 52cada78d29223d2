// The persistent Runge-Kutta 5(4) ensemble kernel, templated on the state
// precision R, the compiled edge-slot and gene-slot budgets (EPL, GPL), the
// output mode (steady state or time series), the serving variant and the
// method (Dormand-Prince or Tsitouras pair).  Included by the translation
// units that instantiate it.
#pragma once

#include <type_traits>

#include "kernel_common.h"

namespace rac {

enum : int { kDP5 = RAC_DP5, kTsit5 = RAC_TSIT5 };

// Dormand & Prince (1980) 5(4) tableau (Hairer, Norsett, Wanner I, Table 5.2).
// Row s holds the weights of k_1..k_s in the input of stage s+1; row 6 is the
// fifth-order solution (first same as last).
__device__ constexpr double kA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84},
};
// Fifth- minus fourth-order weights (the embedded error estimate).
__device__ constexpr double kErr[7] = {
    35.0 / 384 - 5179.0 / 57600,     0.0,
    500.0 / 1113 - 7571.0 / 16695,   125.0 / 192 - 393.0 / 640,
    -2187.0 / 6784 + 92097.0 / 339200, 11.0 / 84 - 187.0 / 2100,
    -1.0 / 40};
// Dense output (continuous extension of order 4, Hairer, Norsett, Wanner I,
// Sec. II.6): weights of k_1, k_3..k_7 in the fifth interpolation coefficient.
__device__ constexpr double kDense[7] = {
    -12715105075.0 / 11282082432.0, 0.0,
    87487479700.0 / 32700410799.0,  -10690763975.0 / 1880347072.0,
    701980252875.0 / 199316789632.0, -1453857185.0 / 822651844.0,
    69997945.0 / 29380423.0};

// Tsitouras (2011) 5(4) pair, the method of the paper's library: stage
// weights (row 6 is the fifth-order solution, first same as last) and the
// fifth- minus fourth-order weights.
__device__ constexpr double kTsA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {0.161, 0, 0, 0, 0, 0},
    {-0.008480655492356989, 0.335480655492357, 0, 0, 0, 0},
    {2.897153057105493, -6.359448489975075, 4.3622954328695815, 0, 0, 0},
    {5.325864828439257, -11.748883564062828, 7.4955393428898365, -0.09249506636175525, 0, 0},
    {5.86145544294642, -12.92096931784711, 8.159367898576159, -0.071584973281401,
     -0.028269050394068383, 0},
    {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742, -3.290069515436081,
     2.324710524099774},
};
__device__ constexpr double kTsErr[7] = {-0.00178001105222577714, -0.0008164344596567469,
                                         0.007880878010261995,    -0.1447110071732629,
                                         0.5823571654525552,      -0.45808210592918697,
                                         0.015151515151515152};

// Continuous extension for Tsit5 time series: x(t + th h) = x + h sum_i b_i(th)
// k_i with b_i(th) = sum_p kTsDense[i][p] th^(p+1).  The weights satisfy the
// order conditions of orders 1..4 as identities in th, equal the step's
// weights at th = 1 and match f at both ends (local error O(h^5)); the one
// remaining freedom is the minimum-norm choice (tsit5_dense.py derives them
// from kTsA).
__device__ constexpr double kTsDense[7][4] = {
    {1.0, -2.631639750604532, 2.649122568481329, -0.9210220510587314},
    {0.0, 0.1922746789549526, -0.3445493579099373, 0.16227467895497885},
    {0.0, 3.345581016079935, -4.771603430501868, 1.9059120648364314},
    {0.0, -1.6743637698306488, 8.864761836076259, -5.811389492141867},
    {0.0, -5.698194445881719, -1.7638891699808519, 4.172014100426498},
    {0.0, 6.090496396744703, -2.8821506970903297, -0.8836351755546025},
    {0.0, 0.3758458745373101, -1.7516917490746, 1.3758458745372943},
};

template <int M>
__device__ constexpr double tab_a(int s, int l) { return M == kTsit5 ? kTsA[s][l] : kA[s][l]; }
template <int M>
__device__ constexpr double tab_e(int l) { return M == kTsit5 ? kTsErr[l] : kErr[l]; }

// Transcendentals: hardware v_log/v_exp/v_rcp for FP32; exact routines and
// an integer power for FP64.
template <typename R>
struct Ops;

template <>
struct Ops<float> {
    using NType = float;
    __device__ static float to_n(float n) { return n; }
    // Sources publish log2 of their level once per evaluation and edges keep
    // n log2 T, so an edge costs one fma, one exp2 and one reciprocal:
    //   factor = b + d / (1 + 2^(n log2 x - n log2 T)),
    // with (b, d) = (sqrt(lam), 1/sqrt(lam) - sqrt(lam)) in the symmetric
    // form, or b = 1, d = D >= 0 and, for activation, n and n log2 T negated
    // in the base-free form (the kernel body picks the form per shape).
    // x = 0 publishes -inf, giving the limit H^S = 1 in both forms.  The
    // clamp at 0 is an integer max on the bits (a negative float is a
    // negative int), one instruction instead of a canonicalised float max.
    __device__ static float publish(float v) {
        const int b = __builtin_bit_cast(int, v);
        return __builtin_amdgcn_logf(__builtin_bit_cast(float, b > 0 ? b : 0));
    }
    __device__ static float edge_t(float T, float n) { return n * __builtin_amdgcn_logf(T); }
    __device__ static float hill(float lx, float nlT, float n, float b, float d) {
        const float r = __builtin_amdgcn_exp2f(__builtin_fmaf(n, lx, -nlT));
        return __builtin_fmaf(d, __builtin_amdgcn_rcpf(1.0f + r), b);
    }
    __device__ static float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
    __device__ static float abs(float v) { return __builtin_fabsf(v); }
    __device__ static float sqrt(float v) { return __builtin_sqrtf(v); }
    __device__ static float max(float a, float b) { return __builtin_fmaxf(a, b); }
    // Step factor 0.9 err^(-1/5) from the mean square err^2 = err2 (finite),
    // clamped to [0.2, fmax]; FP32 is ample for a controller factor (err2 = 0
    // gives +inf, clamped to fmax).
    __device__ static double step_factor(double err2, double fmax) {
        const float f = 0.9f * __builtin_amdgcn_exp2f(-0.1f * __builtin_amdgcn_logf((float)err2));
        return (double)__builtin_amdgcn_fmed3f(f, 0.2f, (float)fmax);
    }
    // v^(1/5) for the starting step (v > 0).
    __device__ static float root5(float v) { return __builtin_amdgcn_exp2f(0.2f * __builtin_amdgcn_logf(v)); }
};

template <>
struct Ops<double> {
    using NType = int;
    __device__ static int to_n(float n) { return (int)n; }
    // Sources publish their level, edges keep 1/T; (x/T)^n by squaring, the
    // three low bits of n (Table 1's 1..6) by selects without a branch and
    // any higher bits in a loop that lanes with n < 8 skip.
    __device__ static double publish(double v) { return v > 0.0 ? v : 0.0; }
    __device__ static double edge_t(double T, float) { return 1.0 / T; }
    __device__ static double hill(double xs, double invT, int n, double b, double d) {
        const double q = xs * invT;
        const double q2 = q * q, q4 = q2 * q2;
        double r = (n & 1) ? q : 1.0;
        r = (n & 2) ? r * q2 : r;
        r = (n & 4) ? r * q4 : r;
        if (n >= 8) {
            double base = q4 * q4;
            for (int e = n >> 3; e > 0; e >>= 1) {
                if (e & 1) r *= base;
                base *= base;
            }
        }
        return fma(d, recip(1.0 + r), b);
    }
    // 1/v for v >= 1: the hardware estimate and two Newton steps (each
    // squares the relative error; the estimate's is far below 2^-13, so two
    // reach the last bit up to rounding).  v is capped at 2^1000 first, so
    // an infinite v gives 2^-1000 (a factor b to double precision) instead
    // of the NaN the Newton step would make of 0 * inf.
    __device__ static double recip(double v) {
        v = __builtin_fmin(v, 0x1p1000);
        double y = __builtin_amdgcn_rcp(v);
        y = fma(y, fma(-v, y, 1.0), y);
        return fma(y, fma(-v, y, 1.0), y);
    }
    __device__ static double rcp(double v) { return 1.0 / v; }
    __device__ static double abs(double v) { return __builtin_fabs(v); }
    __device__ static double sqrt(double v) { return ::sqrt(v); }
    __device__ static double max(double a, double b) { return a > b ? a : b; }
    __device__ static double step_factor(double err2, double fmax) {
        const double f = err2 > 0 ? 0.9 * ::pow(err2, -0.1) : 10.0;
        return f < 0.2 ? 0.2 : (f > fmax ? fmax : f);
    }
    __device__ static double root5(double v) { return ::pow(v, 0.2); }
};

// FP64 kernels for real Hill coefficients (the nf array): (x/T)^n as
// exp(n log(x/T)).  A separate instantiation, so that the integer kernels
// carry no exp/log code and no extra registers.
struct OpsRealN : Ops<double> {
    using NType = float;
    __device__ static float to_n(float n) { return n; }
    __device__ static double hill(double xs, double invT, float n, double b, double d) {
        const double r = ::exp((double)n * ::log(xs * invT));
        return fma(d, recip(1.0 + r), b);
    }
};
template <typename R, bool REALN>
struct OpsFor {
    using type = Ops<R>;
};
template <>
struct OpsFor<double, true> {
    using type = OpsRealN;
};

// Wave-level ordering of LDS writes before reads by other lanes of the wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane moves inside a row of 16 lanes (DPP): quad butterflies for
// masks 1 and 2, the half-row and row mirrors pair groups of 4 and 8 lanes.
enum : int { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };
// Every pattern used reads a lane of the same row, so no lane takes the
// bound-control default.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// A value every lane of the wave holds, moved to scalar registers.
__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Sum over the aligned group of lpt lanes (a power of two); every lane of
// the group gets the same bits, since each level adds two equal partial sums
// in either order.  Called from wave-uniform control flow only; the levels
// nest so that a small group tests only the levels it takes plus one.
template <typename T>
__device__ __forceinline__ T group_reduce(T v, int lpt) {
    if (lpt >= 2) {
        v += dpp_mov<kDppXor1>(v);
        if (lpt >= 4) {
            v += dpp_mov<kDppXor2>(v);
            if (lpt >= 8) {
                v += dpp_mov<kDppHalfMirror>(v);
                if (lpt >= 16) {
                    v += dpp_mov<kDppMirror>(v);
                    if (lpt >= 32) {
                        v += __shfl_xor(v, 16);
                        if (lpt >= 64) v += __shfl_xor(v, 32);
                    }
                }
            }
        }
    }
    return v;
}

enum : int { kRunning = -1 };
// Steps after which a trajectory counts as long for wave priority (a little
// above the typical count of a Table 1 steady-state solve; priority rises
// again at four times this).
constexpr int kLongSteps = 100;

// LDS use per wave, in elements of R (P = kPubStride * GPL):
//   [0, P)                      source levels: gene i = r + q * lpt (slot q of
//                               group lane r) of group g at q * kPubStride +
//                               r * S + g, S = kPubStride / lpt (1 at 64 lanes);
//                               padding gene slots write levels nobody reads
//   [P, P + 64*(EPL+1))         running products, index slot * 64 + lane
//   [P + 64*(EPL+1), +64)       one sink per lane, read by padding edge slots
//   [P + 64*(EPL+2), +128*GPL)  (G', k) of gene slot q of each lane, pair index
//                               q * 64 + lane (private to the lane: loaded with
//                               the trajectory, read by every right-hand side)
//   then 16 bytes per lane      the group's network record (1/N, N, network
//   (32 in time-series mode)    index; in time-series mode also the address
//                               of the trajectory's output rows), private to
//                               the lane, read once a step
// Every address a lane uses is precomputed as an absolute LDS byte offset.
// The level stride S = 96 / lpt spreads the sources that the lanes of a half
// wave read in one edge slot over the 32 LDS banks: group g's copies of one
// gene are consecutive, and genes whose index differs by 1, 2 or 3 modulo 4
// start at banks 24, 16 or 8 apart (S = 24 at 4 lanes; the levels written by
// one half wave fall on 32 distinct banks).
constexpr int kPubStride = 96;
template <bool TS>
struct alignas(16) GroupRec {
    double inv_n;  // 1 / N of the group's network
    int32_t n_genes, net;
};
template <>
struct alignas(16) GroupRec<true> {
    double inv_n;
    int32_t n_genes, net;
    void* xo;      // first output row of the group's trajectory
    int64_t pad;
};

template <typename R, int EPL, int GPL, bool TS>
struct LdsLayout {
    static constexpr int kPub = kPubStride * GPL;
    static constexpr int kRec = kPub + 64 * (EPL + 2 + 2 * GPL);  // start of the network records
    static constexpr int kWaveElems = kRec + 64 * (int)sizeof(GroupRec<TS>) / (int)sizeof(R);
};

template <typename R>
struct alignas(2 * sizeof(R)) RatePair {
    R G, k;
};

// Waves per SIMD the compiler is asked to fit (1: no request), for the FP32
// shapes that sit a few VGPRs above an occupancy step.  Asked, the compiler
// fits them below it with no spill, or (the Tsitouras series shapes and
// its (4, 8) steady-state shape) with three dwords of spill, whose reloads
// cost less than the extra wave gains at two waves per SIMD: the Tsitouras
// 22-gene series runs 24 % faster at three waves than at two, the DP5
// 22-gene steady states 9.6 % faster at four than at three.  Shapes that
// would spill more are not asked: their reloads inside the step loop cost
// more than the wave (the DP5 22-gene series at four waves with 120 bytes of
// spill runs 20 % slower).
template <typename R, int EPL, int GPL, bool TS, bool BOUNDED, int M, bool REALN>
constexpr int requested_waves() {
    // FP64: two waves per SIMD (the (12, 3) series shape and the 16-slot
    // shapes compile to a few registers over 256 unasked, which leaves one
    // wave per SIMD to hide every FP64 latency alone; asked, they spill
    // 12-76 bytes).  Real-n kernels carry exp/log and would spill 36-204
    // bytes, so they are left to the compiler.
    if (sizeof(R) != 4) return REALN ? 1 : 2;
    if (BOUNDED) {  // serving step batches (DP5, steady states)
        if (EPL == 4 && GPL == 2) return 5;
        // (8, 4) and (11, 3) fit four waves with 12 bytes of spill, (10, 4)
        // with 52, all outside the step loop (saturated serving 1.7 % faster).
        if ((EPL == 12 && GPL == 2) || (EPL == 8 && GPL == 4) || (EPL == 10 && GPL == 4) ||
            (EPL == 11 && GPL == 3))
            return 4;
        if ((EPL == 13 && GPL == 5) || (EPL == 16 && GPL == 4)) return 3;
        return 1;
    }
    if (!TS) {
        // (11, 3) fits four waves with no spill, (10, 4) with 28 bytes whose
        // reloads stay outside the step loop (the uneven 64-network batch
        // 1.5 % faster than at three).
        if ((EPL == 11 && GPL == 3) || (EPL == 10 && GPL == 4)) return 4;
        if (EPL == 4 && GPL == 8) return 3;
        if (M == kTsit5 && EPL == 13 && GPL == 5) return 3;
        return 1;
    }
    if (M == kDP5) {
        // The 22-gene series shape (11, 3) fits four waves with 56 bytes of
        // spill and runs 8.5 % faster than at three (25.6 -> 23.4 ms);
        // (8, 3) takes 12 bytes.
        if ((EPL == 11 || EPL == 8) && GPL == 3) return 4;
        return (EPL == 16 && GPL == 8) ? 2 : 1;
    }
    if ((EPL == 11 && GPL == 3) || (EPL == 8 && GPL == 4) || (EPL == 12 && GPL == 3) || (EPL == 16 && GPL == 2))
        return 3;
    return (EPL == 12 && GPL == 8) ? 2 : 1;
}

template <typename R, int EPL, int GPL, bool TS, bool BOUNDED = false, int M = kDP5, bool REALN = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(requested_waves<R, EPL, GPL, TS, BOUNDED, M, REALN>(), 8)))
void dp5_kernel(LaunchArgs a) {
    static_assert(!(TS && BOUNDED), "serving step batches run in steady-state mode");
    static_assert(!REALN || sizeof(R) == 8, "FP32 kernels take real coefficients natively");
    using O = typename OpsFor<R, REALN>::type;
    using NT = typename O::NType;
    using Lay = LdsLayout<R, EPL, GPL, TS>;
    using Rec = GroupRec<TS>;
    static_assert(EPL >= 1, "at least one edge slot");
    __shared__ R lds[(kBlock / 64) * Lay::kWaveElems];
    char* const lb = reinterpret_cast<char*>(lds);
    auto ld = [&](uint32_t addr) -> R { return *reinterpret_cast<const R*>(lb + addr); };
    auto st = [&](uint32_t addr, R v) { *reinterpret_cast<R*>(lb + addr) = v; };
    constexpr uint32_t SZ = sizeof(R);

    const int lane = threadIdx.x & 63;
    const uint32_t wave_elem = (threadIdx.x >> 6) * Lay::kWaveElems;
    const uint32_t pre_base = (wave_elem + Lay::kPub + lane) * SZ;        // prefix[0] of this lane
    const uint32_t sink = (wave_elem + Lay::kPub + 64 * (EPL + 1) + lane) * SZ;

    const int lpt = a.lpt;
    const int sh = __builtin_ctz(lpt);
    const int n_groups = 64 >> sh;
    const int g = lane >> sh;         // group within the wave
    const int r = lane & (lpt - 1);   // lane within the group
    const int gshift = g * lpt;
    const uint64_t glow = lpt == 64 ? ~0ull : ((1ull << lpt) - 1);
    // Level of gene slot q: pub_base + q * kPubStride elements.
    const int pub_s = __builtin_amdgcn_readfirstlane(lpt == 64 ? 1 : kPubStride / lpt);
    auto level_index = [&](int gene) {  // element index of a gene's level in this group
        return (uint32_t)((gene >> sh) * kPubStride + (gene & (lpt - 1)) * pub_s + g);
    };
    const uint32_t pub_base = (wave_elem + (uint32_t)(r * pub_s + g)) * SZ;
    // Rates (G', k) of gene slot q: rate_base + q * 128 elements.
    const uint32_t rate_base = (wave_elem + Lay::kPub + 64 * (EPL + 2) + 2 * lane) * SZ;
    auto rate = [&](int q) -> RatePair<R> {
        return *reinterpret_cast<const RatePair<R>*>(lb + rate_base + (uint32_t)q * 128 * SZ);
    };
    const Controls& c = a.c;

    st(pre_base, (R)1);  // prefix[0] = 1, never overwritten
    // Padding edge slots read the sink; give it a finite value so that their
    // factor is exactly 1 even for lanes that hold no padding gene slot.
    st(sink, (R)0);
    // Lanes that never hold a trajectory still evaluate right-hand sides.
#pragma unroll
    for (int q = 0; q < GPL; ++q)
        *reinterpret_cast<RatePair<R>*>(lb + rate_base + (uint32_t)q * 128 * SZ) = RatePair<R>{(R)0, (R)0};

    // Edge slots: source address, threshold term (O::edge_t), n, sqrt(lam),
    // 1/sqrt(lam) - sqrt(lam).
    // FP32 shapes of up to 16 edge slots use factors 1 + D / (1 + 2^z) (no
    // base term; with Table 1's lambdas D >= 0 and every factor lies in
    // [1, 1 + D], D < 100).  Wider and FP64 shapes keep the symmetric form
    // sqrt(lam) + (1/sqrt(lam) - sqrt(lam)) / (1 + r), whose factors lie in
    // [0.1, 10] for Table 1.
    constexpr bool kUnitBase = std::is_same<R, float>::value && EPL <= kUnitBaseMaxEpl;
    // FP32 range, for any lambdas: with l_s = log2 of slot s's extreme factor
    // (1 + D), a base-free lane's running product lies in an interval of
    // width A = sum |l_s| (log2) centred on 2^(sum l_s / 2); it starts at
    // 2^-round(sum l_s / 2) instead of 1, which centres it on 1.  The start
    // lives in prefix[0] and cancels in every row's prefix ratio (a power of
    // two: no rounding changes).  Reading it costs each evaluation one LDS
    // read and one multiply (0.7 % on the 10-gene and 22-gene workloads);
    // a read skipped by a wave-uniform branch where no lane needs it measured
    // slower (1.5-2.5 %).  A trajectory FP32 still cannot hold (A >
    // 250, or 126 in the symmetric form, or a production rate that the row's
    // factors can push out of the normal range) starts with x = NaN and so
    // ends NONFINITE at t0: that needs lambdas far outside Table 1, and FP64
    // solves it.
    constexpr bool kRangeCheck = std::is_same<R, float>::value;
    uint32_t e_xa[EPL];
    R e_invT[EPL], e_b[kUnitBase ? 1 : EPL], e_d[EPL];
    NT e_n[EPL];
    // Gene slots: state, stages, G', k and LDS addresses (publish, prefix end/begin).
    R x[GPL], y[GPL], kk[7][GPL];
    uint32_t g_pe[GPL], g_pb[GPL];
#pragma unroll
    for (int s = 0; s < EPL; ++s) {
        e_xa[s] = sink; e_invT[s] = 0; e_d[s] = 0; e_n[s] = O::to_n(1.0f);
        if constexpr (!kUnitBase) e_b[s] = 1;
    }
    auto base_of = [&](int s) -> R {
        if constexpr (kUnitBase) return (R)1;
        else return e_b[s];
    };
#pragma unroll
    for (int q = 0; q < GPL; ++q) {
        x[q] = 0; y[q] = 0;
        g_pe[q] = pre_base; g_pb[q] = pre_base;
#pragma unroll
        for (int l = 0; l < 7; ++l) kk[l][q] = 0;
    }

    // Per-group scalars (replicated over the group's lanes).
    int64_t traj = -1;
    int kout = 0, nacc = 0, nrej = 0;
    bool fresh = false, last_rej = false;
    double t = 0, h = 0;
    const double t_stop = TS ? a.t_out[a.n_t - 1] : c.t_end;  // the same for every trajectory
    bool exhausted = false;   // queue drained and no claimed index left
    bool drained = false;     // the shared queue has nothing left to pop
    // Sub-queue this wave pops from (persistent launches): its XCD's range
    // first, then the following ones; tried counts the ranges found empty.
    const int home = (int)(blockIdx.x % kSubQueues);
    int q = home, tried = 0;
    // Sub-queue x holds the granules g of kGranule consecutive trajectories
    // with g % kSubQueues == x; positions count within a sub-queue.
    auto q_count = [&](int x) -> uint64_t {
        const uint64_t n = (uint64_t)a.total, ng = n / kGranule, rem = n % kGranule;
        return (ng / kSubQueues + ((uint64_t)x < ng % kSubQueues ? 1 : 0)) * kGranule +
               ((uint64_t)x == ng % kSubQueues ? rem : 0);
    };
    auto q_index = [&](int x, uint64_t pos) -> int64_t {
        return (int64_t)(((pos / kGranule) * kSubQueues + (uint64_t)x) * kGranule + pos % kGranule);
    };
    uint64_t popped = 0;      // queue position after this wave's last pop
    // Positions this wave has claimed but not started: [claim_next, claim_end)
    // of sub-queue claim_q.
    uint64_t claim_next = 0, claim_end = 0;
    int claim_q = home;
    // The group's network (index, N, 1/N), kept in LDS rather than registers.
    Rec* const rec = reinterpret_cast<Rec*>(lb + (wave_elem + Lay::kRec) * SZ + sizeof(Rec) * lane);
    rec->inv_n = 1.0;
    rec->n_genes = 1;
    rec->net = 0;
    // Gene slot q of this lane holds gene r + q * lpt; slots past N pad.
    auto gene_of = [&](int q) { return r + q * lpt; };
    auto is_real = [&](int q) { return r + q * lpt < rec->n_genes; };

    // One right-hand-side evaluation f(yv) for every lane of the wave: no
    // branches, padding slots evaluate factors of exactly 1.
    auto rhs = [&](const R (&yv)[GPL], R (&f)[GPL]) {
#pragma unroll
        for (int q = 0; q < GPL; ++q) st(pub_base + (uint32_t)q * kPubStride * SZ, O::publish(yv[q]));
        wave_sync();
        R run = kUnitBase ? ld(pre_base) : (R)1;
        // Chunks of up to four independent factors, then their running products.
#pragma unroll
        for (int c0 = 0; c0 < EPL; c0 += 4) {
            R hv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c0 + j < EPL)
                    hv[j] = O::hill(ld(e_xa[c0 + j]), e_invT[c0 + j], e_n[c0 + j], base_of(c0 + j), e_d[c0 + j]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (c0 + j < EPL) {
                    run *= hv[j];
                    st(pre_base + (uint32_t)(c0 + j + 1) * 64 * SZ, run);
                }
            }
        }
        wave_sync();
#pragma unroll
        for (int q = 0; q < GPL; ++q) {
            const RatePair<R> gr = rate(q);
            f[q] = gr.G * (ld(g_pe[q]) * O::rcp(ld(g_pb[q]))) - gr.k * yv[q];
        }
    };

    auto group_sum = [&](double v) { return group_reduce(v, lpt); };
    // Steady-state test |f_i| <= ss_atol + ss_rtol k_i |x_i|, compared in FP64.
    auto is_steady = [&](R f, R kv, R xv) {
        return __builtin_fabs((double)f) <= c.ss_atol + c.ss_rtol * (double)kv * __builtin_fabs((double)xv);
    };
    auto group_sumr = [&](R v) { return group_reduce(v, lpt); };
    auto group_all = [&](bool p) { return ((__ballot(p) >> gshift) & glow) == glow; };

    // Write the end-of-trajectory record and free the group.
    auto finish = [&](int status) {
        const NetDesc* dp = a.nets + rec->net;
        const int N = dp->n_genes;
        const int64_t local = traj - dp->traj_begin;
        if constexpr (!TS) {
            R* const xo = (R*)dp->x_out + local * N;
#pragma unroll
            for (int q = 0; q < GPL; ++q)
                if (is_real(q)) xo[gene_of(q)] = x[q];
        } else {
            // Steady before the last output: the remaining outputs hold x_ss.
            R* const xo = (R*)rec->xo;
            for (int k = kout; k < a.n_t; ++k)
#pragma unroll
                for (int q = 0; q < GPL; ++q)
                    if (is_real(q)) xo[k * N + gene_of(q)] = x[q];
        }
        if (r == 0) {
            double* tf = dp->t_final;
            int8_t* sp = dp->status;
            int32_t* na = dp->n_acc;
            int32_t* nr = dp->n_rej;
            if (tf) tf[local] = t;
            if (sp) sp[local] = (int8_t)status;
            if (na) na[local] = nacc;
            if (nr) nr[local] = nrej;
            int32_t* dn = dp->done;
            if (dn) atomicAdd(dn, 1);
        }
        traj = -1;
        fresh = false;
    };

    // Saved state of a wave between serving step batches, lane fastest:
    // x[GPL], k1[GPL] (R); t, h (f64); trajectory id (i64); accepted,
    // rejected, flags (i32; bit 0 last step rejected, bit 1 not yet started).
    constexpr size_t kOffK = (size_t)64 * GPL * SZ, kOffT = 2 * kOffK, kOffH = kOffT + 512,
                     kOffTraj = kOffH + 512, kOffAcc = kOffTraj + 512, kOffRej = kOffAcc + 256,
                     kOffFlags = kOffRej + 256, kSlotBytes = kOffFlags + 256;
    static_assert(kSlotBytes == serve_slot_bytes(GPL, SZ), "slot layout");
    char* const sbase =
        BOUNDED ? a.slots + (size_t)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * kSlotBytes : nullptr;

    // Start trajectory idx (a global queue index) in this lane's group: find
    // its network, load and derive its parameters, set x0.
    auto load_traj = [&](int64_t idx) {
            // Which network: binary search over first queue indices.
            int lo = 0, hi = (BOUNDED ? __hip_atomic_load(&a.ctl->n_nets, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT)
                                      : a.n_nets) - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.nets[mid].traj_begin <= idx) lo = mid; else hi = mid - 1;
            }
            const int net = lo;
            // Loads go one slot at a time (the memory clobbers stop
            // the scheduler from hoisting them all), which keeps
            // this rarely taken path from setting the kernel's
            // register peak next to the live trajectory state.
            const NetDesc* dp = a.nets + net;
            traj = idx;
            const int64_t local = idx - dp->traj_begin;
            const int n_ic = dp->n_ic;
            int64_t p = (int64_t)((double)local * dp->inv_n_ic);
            if (p * n_ic > local) --p;
            if ((p + 1) * n_ic <= local) ++p;
            const int ci = (int)(local - p * n_ic);
            const int64_t P = dp->n_sets;
            const int n_genes = dp->n_genes;
            rec->inv_n = 1.0 / n_genes;
            rec->n_genes = n_genes;
            rec->net = net;
            if constexpr (TS) rec->xo = (R*)dp->x_out + local * (int64_t)a.n_t * n_genes;
            const int stride = dp->stride;
            const int32_t* lane_edge = dp->lane_edge + r * stride;
            const float* Tp = dp->T + p;
            const float* Lp = dp->lam + p;
            // Hill coefficients: real ones when given, else the integer array.
            const float* NFp = dp->nf ? dp->nf + p : nullptr;
            const uint8_t* Np = dp->nf ? nullptr : dp->n + p;
            // log2 range of this lane's running product: the sum and the
            // sum of magnitudes of log2 of the slots' extreme factors.
            float lane_s2 = 0.0f, lane_a2 = 0.0f;
            // Only the loads are conditional: padding slots take T = lam = n = 1,
            // an inhibiting sign and the sink, which the same formulas turn
            // into a factor of exactly 1 (every array element is written on
            // one path, which keeps the arrays in registers).
#pragma unroll
            for (int s = 0; s < EPL; ++s) {
                asm volatile("" ::: "memory");
                const int pk = s < stride ? lane_edge[s] : -1;
                float Tv = 1.0f, Lv = 1.0f, nv = 1.0f;
                bool act = false;
                uint32_t xa = sink;
                if (pk >= 0) {
                    const int e = pk & 0x7fff, src = pk >> 16;
                    act = (pk & 0x8000) != 0;
                    Tv = Tp[e * P];
                    Lv = Lp[e * P];
                    nv = NFp ? NFp[e * P] : (float)Np[e * P];
                    xa = (wave_elem + level_index(src)) * SZ;
                }
                e_xa[s] = xa;
                if constexpr (kUnitBase) {
                    // Activation: H^S = 1 + (lam - 1) / (1 + (T/x)^n), the
                    // exponent negated; inhibition: H^S = lam (1 + (1/lam - 1)
                    // / (1 + (x/T)^n)), the lam folded into the gene below.
                    const float nn = act ? -nv : nv;
                    e_n[s] = nn;
                    e_invT[s] = nn * __builtin_amdgcn_logf(Tv);
                    e_d[s] = act ? Lv - 1.0f : 1.0f / Lv - 1.0f;
                    const float l2 = __builtin_amdgcn_logf(1.0f + e_d[s]);
                    lane_s2 += l2;
                    lane_a2 += __builtin_fabsf(l2);
                } else {
                    const R sl = O::sqrt((R)Lv);
                    e_invT[s] = O::edge_t((R)Tv, nv);
                    e_n[s] = O::to_n(nv);
                    e_b[s] = sl;
                    e_d[s] = (R)1 / sl - sl;
                    if constexpr (kRangeCheck) lane_a2 += 0.5f * __builtin_fabsf(__builtin_amdgcn_logf(Lv));
                }
            }
            // Symmetric-form products range over [2^-A, 2^A]; base-free ones
            // over an interval of width A that the start centres on 1.
            bool out_of_range = kRangeCheck && !(lane_a2 <= (kUnitBase ? 250.0f : 126.0f));
            if constexpr (kUnitBase)
                st(pre_base, out_of_range ? 1.0f : __builtin_amdgcn_ldexpf(1.0f, -(int)__builtin_rintf(0.5f * lane_s2)));
            const float* Gp = dp->G + p;
            const float* Kp = dp->k + p;
            const float* icp = dp->ic + (int64_t)ci * n_genes;
            const int32_t* row_ptr = dp->row_ptr;
            const int32_t* gene_row = dp->gene_row;
            const int8_t* sign = dp->sign;
            // As for edges: conditional loads, one unconditional write per
            // element; padding genes get G = k = 0 and the sink.
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                asm volatile("" ::: "memory");
                const int gene = r + q * lpt;
                const bool real = gene < n_genes;
                R Gv = 0, kv = 1, gf = 0, u = 0;
                int row = 0;
                if (real) {
                    Gv = (R)Gp[gene * P];
                    kv = (R)Kp[gene * P];
                    // Fold the edge factors' constant parts into the
                    // production rate: lam per inhibiting edge and, for
                    // activation over lambda, 1/lam per activating edge
                    // (or sqrt(lam) and 1/sqrt(lam) in the symmetric form).
                    gf = Gv;
                    // log2 of the row's smallest and largest factor products.
                    float row_lo2 = 0.0f, row_hi2 = 0.0f;
                    for (int e = row_ptr[gene]; e < row_ptr[gene + 1]; ++e) {
                        const R lv = (R)Lp[e * P];
                        if constexpr (kUnitBase) {
                            gf *= sign[e] > 0 ? (c.divide ? (R)1 / lv : (R)1) : lv;
                            // log2 (1 + D): log2 lam for activation, -log2 lam for inhibition.
                            const float l2 = (sign[e] > 0 ? 1.0f : -1.0f) * __builtin_amdgcn_logf((float)lv);
                            row_lo2 += l2 < 0.0f ? l2 : 0.0f;
                            row_hi2 += l2 > 0.0f ? l2 : 0.0f;
                        } else {
                            const R sl = O::sqrt(lv);
                            gf *= (sign[e] > 0 && c.divide) ? (R)1 / sl : sl;
                            if constexpr (kRangeCheck) {
                                const float l2 = 0.5f * __builtin_fabsf(__builtin_amdgcn_logf((float)lv));
                                row_lo2 -= l2;
                                row_hi2 += l2;
                            }
                        }
                    }
                    // G' times the row's factors must stay normal and finite.
                    if constexpr (kRangeCheck) {
                        const float lg = __builtin_amdgcn_logf((float)gf);
                        if (Gv != (R)0 && !(lg + row_lo2 >= -125.0f && lg + row_hi2 <= 126.0f))
                            out_of_range = true;
                    }
                    row = gene_row[gene];
                    u = (R)icp[gene];
                }
                const int rl = row & 0xff, pb = (row >> 8) & 0xff, pe = (row >> 16) & 0xff;
                const uint32_t rowlane = (uint32_t)(gshift + rl);
                g_pb[q] = real ? (wave_elem + Lay::kPub + (uint32_t)pb * 64 + rowlane) * SZ : pre_base;
                g_pe[q] = real ? (wave_elem + Lay::kPub + (uint32_t)pe * 64 + rowlane) * SZ : pre_base;
                *reinterpret_cast<RatePair<R>*>(lb + rate_base + (uint32_t)q * 128 * SZ) =
                    RatePair<R>{gf, real ? kv : (R)0};
                // Padding slots hold x = 1 with G = k = 0: their derivative,
                // error and steady test are exactly 0, 0 and true, and their
                // error scale atol + rtol is positive.
                x[q] = real ? (c.ic_absolute ? u : u * Gv / kv) : (R)1;
            }
            if constexpr (kRangeCheck) {
                if (((__ballot(out_of_range) >> gshift) & glow) != 0) {
#pragma unroll
                    for (int q = 0; q < GPL; ++q) x[q] = __builtin_nanf("");
                }
            }
            t = c.t0;
            nacc = 0; nrej = 0; kout = 0; last_rej = false;
            fresh = true;
    };

    auto save = [&]() {
        reinterpret_cast<int64_t*>(sbase + kOffTraj)[lane] = traj;
#pragma unroll
        for (int q = 0; q < GPL; ++q) {
            reinterpret_cast<R*>(sbase)[q * 64 + lane] = x[q];
            reinterpret_cast<R*>(sbase + kOffK)[q * 64 + lane] = kk[0][q];
        }
        reinterpret_cast<double*>(sbase + kOffT)[lane] = t;
        reinterpret_cast<double*>(sbase + kOffH)[lane] = h;
        reinterpret_cast<int32_t*>(sbase + kOffAcc)[lane] = nacc;
        reinterpret_cast<int32_t*>(sbase + kOffRej)[lane] = nrej;
        reinterpret_cast<int32_t*>(sbase + kOffFlags)[lane] = (last_rej ? 1 : 0) | (fresh ? 2 : 0);
    };

    if (BOUNDED) {
        // Resume the trajectories this wave held when the previous batch ended.
        const int64_t saved = reinterpret_cast<const int64_t*>(sbase + kOffTraj)[lane];
        if (saved >= 0) {
            load_traj(saved);
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                x[q] = reinterpret_cast<const R*>(sbase)[q * 64 + lane];
                kk[0][q] = reinterpret_cast<const R*>(sbase + kOffK)[q * 64 + lane];
            }
            t = reinterpret_cast<const double*>(sbase + kOffT)[lane];
            h = reinterpret_cast<const double*>(sbase + kOffH)[lane];
            nacc = reinterpret_cast<const int32_t*>(sbase + kOffAcc)[lane];
            nrej = reinterpret_cast<const int32_t*>(sbase + kOffRej)[lane];
            const int32_t fl = reinterpret_cast<const int32_t*>(sbase + kOffFlags)[lane];
            last_rej = (fl & 1) != 0;
            fresh = (fl & 2) != 0;
        }
    }

    for (int iter = 0;; ++iter) {
        if (BOUNDED && iter >= a.batch_steps) {
            save();
            return;
        }
        // ---- refill free groups from the work queue --------------------
        if (!exhausted) {
            const uint64_t free_lead = __ballot(traj < 0 && r == 0);
            const int nfree = __popcll(free_lead);
            const uint64_t busy_lead = __ballot(traj >= 0 && r == 0);
            // End of the range popped from: the serving queue's tail, or the
            // current sub-queue's end.
            const uint64_t total =
                BOUNDED ? __hip_atomic_load(&a.ctl->total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : q_count(q);
            // Refill in batches (each refill costs the wave two extra right-hand
            // sides), but take single items once the range is nearly drained.
            const uint64_t n_waves = (uint64_t)gridDim.x * (kBlock / 64) / (BOUNDED ? 1 : kSubQueues) + 1;
            const bool near_end = popped >= total || total - popped < n_waves * 64;
            if (nfree > 0 && (nfree >= c.refill_min || busy_lead == 0 || near_end)) {
                // Serve from this wave's claimed indices first; pop the rest
                // from the shared queue.  While the queue is long, one pop
                // claims a whole chunk (one atomic per chunk instead of per
                // refill); near its end, and in step batches (whose waves
                // keep no claims between batches), a pop takes exactly what
                // is needed.
                const uint64_t local_n = claim_end - claim_next < (uint64_t)nfree ? claim_end - claim_next
                                                                                 : (uint64_t)nfree;
                const uint64_t need = (uint64_t)nfree - local_n;
                unsigned long long base = 0, got = 0;
                int pop_q = q;
                if (need > 0 && !drained) {
                    const bool claim = !BOUNDED && total - popped > n_waves * (uint64_t)c.chunk * 2 &&
                                       popped < total;
                    const uint64_t want = claim && need < (uint64_t)c.chunk ? (uint64_t)c.chunk : need;
                    if (BOUNDED) {
                        if (lane == 0) {
                            // One atomic per wave.  In step batches head may run
                            // past total; the batch's last graph node clamps it
                            // back before the host appends more, so appended
                            // indices are served.
                            base = atomicAdd(a.counter, (unsigned long long)want);
                            got = base >= total ? 0ull
                                                : (base + (unsigned long long)want <= total ? (unsigned long long)want
                                                                                           : total - base);
                        }
                        base = uniform64(__shfl(base, 0));
                        got = uniform64(__shfl(got, 0));
                        popped = base + got;
                        if (base + want >= total || got < want) drained = true;
                    } else {
                        // Pop from sub-queue q; a range found exhausted sends
                        // the wave on to the next one (at most kSubQueues
                        // attempts per pop, one atomic each).
                        for (;;) {
                            const uint64_t q_end = q_count(q);
                            pop_q = q;
                            if (lane == 0) {
                                base = atomicAdd(a.counter + q * kCounterStride, (unsigned long long)want);
                                got = base >= q_end ? 0ull
                                                    : (base + (unsigned long long)want <= q_end ? (unsigned long long)want
                                                                                                : q_end - base);
                            }
                            base = uniform64(__shfl(base, 0));
                            got = uniform64(__shfl(got, 0));
                            popped = base + got;
                            if (base + want >= q_end || got < want) {
                                if (++tried >= kSubQueues) {
                                    drained = true;
                                } else {
                                    q = q + 1 == kSubQueues ? 0 : q + 1;
                                    popped = 0;
                                }
                            }
                            if (got > 0 || drained) break;
                        }
                    }
                }
                if (traj < 0) {
                    const uint64_t rank = (uint64_t)__popcll(free_lead & ((1ull << gshift) - 1ull));
                    if (rank < local_n) {
                        load_traj(BOUNDED ? (int64_t)(claim_next + rank) : q_index(claim_q, claim_next + rank));
                    } else if (rank - local_n < (uint64_t)got) {
                        const uint64_t pos = (uint64_t)base + (rank - local_n);
                        load_traj(BOUNDED ? (int64_t)pos : q_index(pop_q, pos));
                    }
                }
                claim_next += local_n;
                if (got > need) {
                    claim_next = (uint64_t)base + need;
                    claim_end = (uint64_t)base + got;
                    claim_q = pop_q;
                }
                if (drained && claim_next >= claim_end) exhausted = true;
            }
        }
        // Waves that hold an unusually long trajectory (oscillating parameter
        // sets run to t_end in several times the typical step count) issue
        // ahead of the others, so that a long trajectory started late in the
        // queue does not run on alone after every other wave has finished;
        // the work is the same, only its order changes.  Re-evaluated every
        // eighth iteration.
        if ((iter & 7) == 0) {
            const int steps = nacc + nrej;
            if (__ballot(traj >= 0 && steps >= kLongSteps) == 0) __builtin_amdgcn_s_setprio(0);
            else if (__ballot(traj >= 0 && steps >= 4 * kLongSteps) == 0) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(3);
        }
        if (__ballot(traj >= 0) == 0) {
            if (exhausted) {
                if (BOUNDED) save();
                break;
            }
            continue;
        }

        // ---- start new trajectories: f(x0), steady test at t0, first step -
        // (Hairer, Norsett, Wanner I, Sec. II.4 starting step, in the state
        // precision R.)
        if (__ballot(fresh) != 0) {
#pragma unroll
            for (int q = 0; q < GPL; ++q) y[q] = x[q];
            rhs(y, kk[1]);
            bool fin = true, steady = true;
            R s0 = 0, s1 = 0;
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                if (fresh) kk[0][q] = kk[1][q];
                if (is_real(q)) {
                    const R xv = x[q], fv = kk[1][q];
                    fin = fin && __builtin_isfinite(xv) && __builtin_isfinite(fv);
                    const R isc = (R)1 / ((R)c.atol + (R)c.rtol * O::abs(xv));
                    s0 += (xv * isc) * (xv * isc);
                    s1 += (fv * isc) * (fv * isc);
                    steady = steady && is_steady(kk[1][q], rate(q).k, x[q]);
                }
            }
            const bool all_fin = group_all(fin);
            const bool all_steady = group_all(steady);
            const int n_genes = rec->n_genes;
            const R d0 = O::sqrt(group_sumr(s0) / (R)n_genes), d1 = O::sqrt(group_sumr(s1) / (R)n_genes);
            if constexpr (TS) {
                if (fresh) {
                    R* const xo = (R*)rec->xo;
                    while (kout < a.n_t && a.t_out[kout] <= t) {
#pragma unroll
                        for (int q = 0; q < GPL; ++q)
                            if (is_real(q)) xo[kout * n_genes + gene_of(q)] = x[q];
                        ++kout;
                    }
                }
            }
            const R hmax = (R)(t_stop - c.t0);
            // Either norm below 1e-5: no usable scale, take 1e-6.
            R hg = (d0 < (R)1e-5 || d1 < (R)1e-5) ? (R)1e-6 : (R)0.01 * d0 / d1;
            hg = hg < hmax ? hg : hmax;
#pragma unroll
            for (int q = 0; q < GPL; ++q) y[q] = x[q] + hg * kk[0][q];
            rhs(y, kk[2]);
            R s2 = 0;
#pragma unroll
            for (int q = 0; q < GPL; ++q)
                if (is_real(q)) {
                    const R dv = (kk[2][q] - kk[0][q]) / ((R)c.atol + (R)c.rtol * O::abs(x[q]));
                    s2 += dv * dv;
                }
            const R d2 = O::sqrt(group_sumr(s2) / (R)n_genes) / hg;
            if (fresh) {
                if (!all_fin) {
                    finish(RAC_NONFINITE);
                } else if ((!TS || c.stop_at_steady) && all_steady) {
                    finish(RAC_CONVERGED);
                } else if (t >= t_stop) {
                    finish(RAC_T_END);
                } else {
                    const double hm = t_stop - c.t0;
                    if (c.h0 > 0) {
                        h = c.h0 < hm ? c.h0 : hm;
                    } else {
                        const R der = d1 > d2 ? d1 : d2;
                        const R h1 = der <= (R)1e-15 ? (hg * (R)1e-3 > (R)1e-6 ? hg * (R)1e-3 : (R)1e-6)
                                                     : O::root5((R)0.01 / der);
                        const double hh = (double)((R)100 * hg < h1 ? (R)100 * hg : h1);
                        h = hh <= hm ? hh : hm;
                    }
                    fresh = false;
                }
            }
            continue;
        }

        // ---- one DP5 attempt for every running group ---------------------
        const bool running = traj >= 0;
        int stop_status = kRunning;
        if (running) {
            const double tmag = fabs(t) > 1.0 ? fabs(t) : 1.0;
            if ((int64_t)nacc + nrej >= c.max_steps) stop_status = RAC_MAX_STEPS;
            else if (h < 16.0 * 2.220446049250313e-16 * tmag) stop_status = RAC_STEP_UNDERFLOW;
        }
        if (__ballot(running && stop_status != kRunning) != 0) {
            if (running && stop_status != kRunning) finish(stop_status);
            continue;
        }
        double hs = h;
        bool clipped = false;
        if (t + hs >= t_stop) {
            hs = t_stop - t;
            clipped = true;
        }
        const R hR = (R)hs;
        R epart[GPL];  // error combination of k1..k6, formed before the last stage
#pragma unroll
        for (int st_ = 1; st_ < 7; ++st_) {
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                R acc = (R)tab_a<M>(st_, 0) * kk[0][q];
#pragma unroll
                for (int l = 1; l < st_; ++l)
                    if (tab_a<M>(st_, l) != 0.0) acc += (R)tab_a<M>(st_, l) * kk[l][q];
                y[q] = x[q] + hR * acc;
            }
            if (st_ == 6) {
                // Summing k1..k6 into the error now (same order as one pass
                // over k1..k7) frees them during the last right-hand side
                // unless dense output still needs them.
#pragma unroll
                for (int q = 0; q < GPL; ++q) {
                    R e = (R)tab_e<M>(0) * kk[0][q];
#pragma unroll
                    for (int l = 1; l < 6; ++l)
                        if (tab_e<M>(l) != 0.0) e += (R)tab_e<M>(l) * kk[l][q];
                    epart[q] = e;
                }
            }
            rhs(y, kk[st_]);
        }
        // y now holds the fifth-order solution, kk[6] its derivative.
        double serr = 0;
        bool fin = true;
#pragma unroll
        for (int q = 0; q < GPL; ++q) {
            R e = epart[q];
            if (tab_e<M>(6) != 0.0) e += (R)tab_e<M>(6) * kk[6][q];
            // Scaled error e_i / (atol + rtol max(|x_i|, |x_new,i|)); the ratio
            // in R, its square accumulated in FP64.
            const R sc = (R)c.atol + (R)c.rtol * O::max(O::abs(x[q]), O::abs(y[q]));
            const double rq = (double)(hR * e * O::rcp(sc));
            serr += rq * rq;
            fin = fin && __builtin_isfinite(y[q]);
        }
        // Accept iff the RMS error is <= 1, i.e. its square is; one factor
        // 0.9 err^(-1/5), clamped to [0.2, 10] after an accepted step that did
        // not follow a rejection and to [0.2, 1] otherwise.
        const double err2 = group_sum(serr) * rec->inv_n;
        const bool all_fin = group_all(fin);  // collective: evaluated by every lane
        const bool accept = running && all_fin && err2 <= 1.0;
        const double fmax = (accept && !last_rej) ? 10.0 : 1.0;
        const double fac = __builtin_isfinite(err2) ? O::step_factor(err2, fmax) : 0.2;
        if (running) {
            h = hs * fac;
            nrej += accept ? 0 : 1;
            last_rej = !accept;
        }
        // Dense output for every output time inside the accepted step.
        if constexpr (TS) if (accept && kout < a.n_t && a.t_out[kout] <= (clipped ? t_stop : t + hs)) {
            R* const xo = (R*)rec->xo;
            const int N = rec->n_genes;
            const double t_new = clipped ? t_stop : t + hs;
            const R ih = O::rcp(hR);  // theta in the state precision
            while (kout < a.n_t && a.t_out[kout] <= t_new) {
                const R th = (R)(a.t_out[kout] - t) * ih;
                if constexpr (M == kTsit5) {
                    R bt[7];
#pragma unroll
                    for (int l = 0; l < 7; ++l)
                        bt[l] = th * ((R)kTsDense[l][0] +
                                      th * ((R)kTsDense[l][1] + th * ((R)kTsDense[l][2] + th * (R)kTsDense[l][3])));
#pragma unroll
                    for (int q = 0; q < GPL; ++q) {
                        if (is_real(q)) {
                            R acc = bt[0] * kk[0][q];
#pragma unroll
                            for (int l = 1; l < 7; ++l) acc += bt[l] * kk[l][q];
                            xo[kout * N + gene_of(q)] = x[q] + hR * acc;
                        }
                    }
                } else {
                    // Continuous extension of order 4 (Hairer, Norsett,
                    // Wanner I, Sec. II.6).
                    const R th1 = (R)1 - th;
#pragma unroll
                    for (int q = 0; q < GPL; ++q) {
                        if (is_real(q)) {
                            const R ydiff = y[q] - x[q];
                            const R bspl = hR * kk[0][q] - ydiff;
                            const R c4 = ydiff - hR * kk[6][q] - bspl;
                            R c5 = (R)kDense[0] * kk[0][q];
#pragma unroll
                            for (int l = 2; l < 7; ++l) c5 += (R)kDense[l] * kk[l][q];
                            c5 *= hR;
                            xo[kout * N + gene_of(q)] =
                                x[q] + th * (ydiff + th1 * (bspl + th * (c4 + th1 * c5)));
                        }
                    }
                }
                ++kout;
            }
        }
        if (accept) {
            ++nacc;
            t = clipped ? t_stop : t + hs;
#pragma unroll
            for (int q = 0; q < GPL; ++q) {
                x[q] = y[q];
                kk[0][q] = kk[6][q];
            }
        }
        // Steady test after an accepted step (uniform branch: time series stop
        // only with stop_at_steady).
        bool all_steady = false;
        if (!TS || c.stop_at_steady) {
            bool steady = accept;
#pragma unroll
            for (int q = 0; q < GPL; ++q) steady = steady && is_steady(kk[0][q], rate(q).k, x[q]);
            all_steady = group_all(steady);
        }
        if (accept) {
            if (all_steady) finish(RAC_CONVERGED);
            else if (t >= t_stop) finish(RAC_T_END);
        }
    }
}

}  // namespace rac
