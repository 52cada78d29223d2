// Host-side parameter and initial-condition sampling (GRiNS Sec. 2.1.2,
// Table 1) from a counter-based generator, so that any parameter set can be
// regenerated from (seed, set index) alone.
#include <cmath>
#include <cstdint>

#include "rac_internal.h"

namespace rac {
namespace {

// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): each round
// multiplies two counter words by fixed odd constants, swaps the 128-bit
// halves across lanes and xors in the key; the key is bumped by the Weyl
// constants between rounds.
struct Philox4x64 {
    static constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ULL;
    static constexpr uint64_t kMulB = 0xCA5A826395121157ULL;
    static constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ULL;
    static constexpr uint64_t kWeylB = 0xBB67AE8584CAA73BULL;

    static void block(uint64_t w[4], uint64_t key_a, uint64_t key_b) {
        for (int r = 0; r < 10; ++r) {
            const unsigned __int128 pa = (unsigned __int128)kMulA * w[0];
            const unsigned __int128 pb = (unsigned __int128)kMulB * w[2];
            const uint64_t pa_hi = (uint64_t)(pa >> 64), pa_lo = (uint64_t)pa;
            const uint64_t pb_hi = (uint64_t)(pb >> 64), pb_lo = (uint64_t)pb;
            const uint64_t out0 = pb_hi ^ w[1] ^ key_a;
            const uint64_t out2 = pa_hi ^ w[3] ^ key_b;
            w[0] = out0;
            w[1] = pb_lo;
            w[2] = out2;
            w[3] = pa_lo;
            key_a += kWeylA;
            key_b += kWeylB;
        }
    }
};

// Uniform in [0, 1) from the top 53 bits of word (slot % 4) of the block at
// counter (index, slot / 4, domain, 0) under key (seed, 0).
double draw(uint64_t seed, uint64_t index, uint64_t slot, uint64_t domain) {
    uint64_t w[4] = {index, slot >> 2, domain, 0};
    Philox4x64::block(w, seed, 0);
    return (double)(w[slot & 3] >> 11) * (1.0 / 9007199254740992.0);
}

// Fraction of (G, k) pairs with G/k <= m, for G ~ U[a, b] and k ~ U[c, d]:
// the mean over k of the clipped linear ramp (m k - a) / (b - a).
double ratio_cdf(double a, double b, double c, double d, double m) {
    auto clamp01 = [](double v) { return v < 0 ? 0.0 : (v > 1 ? 1.0 : v); };
    if (d <= c && b <= a) return m * c >= a ? 1.0 : 0.0;
    if (d <= c) return clamp01((m * c - a) / (b - a));
    if (b <= a) return clamp01((d - a / m) / (d - c));
    auto clampk = [&](double k) { return k < c ? c : (k > d ? d : k); };
    const double lo = clampk(a / m), hi = clampk(b / m);
    const double ramp = (0.5 * m * (hi * hi - lo * lo) - a * (hi - lo)) / (b - a);
    return (ramp + (d - hi)) / (d - c);
}

double ratio_median(const rac_ranges& r) {
    if (r.t_median > 0) return r.t_median;
    const double a = r.g_min, b = r.g_max, c = r.k_min, d = r.k_max;
    // When the ramp spans every k, the CDF is linear in m: median (a+b)/(c+d).
    const double lin = (a + b) / (c + d);
    if (lin * c >= a && lin * d <= b) return lin;
    double lo = a / d, hi = b / c;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        (ratio_cdf(a, b, c, d, mid) < 0.5 ? lo : hi) = mid;
    }
    return 0.5 * (lo + hi);
}

bool ranges_ok(const rac_ranges& r) {
    return r.g_min >= 0 && r.g_max >= r.g_min && r.k_min > 0 && r.k_max >= r.k_min &&
           r.lam_act_min > 0 && r.lam_act_max >= r.lam_act_min && r.lam_inh_min > 0 &&
           r.lam_inh_max >= r.lam_inh_min && r.n_min >= 1 && r.n_max >= r.n_min && r.n_max <= 255 &&
           r.t_lo > 0 && r.t_hi >= r.t_lo && std::isfinite(r.g_max) && std::isfinite(r.lam_act_max) &&
           (r.g_max > 0 || r.t_median > 0);
}

}  // namespace

bool sample_ranges_ok(const rac_ranges& r) { return ranges_ok(r); }
double sample_ratio_median(const rac_ranges& r) { return ratio_median(r); }

}  // namespace rac

extern "C" {

void rac_default_ranges(rac_ranges* r) {
    if (!r) return;
    r->g_min = 1.0;
    r->g_max = 100.0;
    r->k_min = 0.1;
    r->k_max = 1.0;
    r->lam_act_min = 1.0;
    r->lam_act_max = 100.0;
    r->lam_inh_min = 0.01;
    r->lam_inh_max = 1.0;
    r->n_min = 1;
    r->n_max = 6;
    r->t_lo = 0.02;
    r->t_hi = 1.98;
    r->t_median = 0.0;
}

rac_status rac_sample_params(const rac_topology* topo, const rac_ranges* ranges, uint64_t seed,
                             int64_t set_begin, int64_t n_sets, int32_t n_ic, rac_params_view* out,
                             float* ic_frac) {
    using rac::fail;
    if (!topo) return fail(RAC_EINVAL, "rac_sample_params: NULL topology");
    if (!out) return fail(RAC_EINVAL, "rac_sample_params: NULL output view");
    if (n_sets < 0 || n_ic < 0 || set_begin < 0)
        return fail(RAC_EINVAL, "rac_sample_params: negative count or offset");
    if (out->n_sets != n_sets) return fail(RAC_EINVAL, "rac_sample_params: out->n_sets != n_sets");
    const int64_t N = topo->n_genes, E = topo->n_edges;
    if (n_sets > 0 && (!out->G || !out->k || (E > 0 && (!out->T || !out->lam || !out->n))))
        return fail(RAC_EINVAL, "rac_sample_params: NULL parameter array");
    rac_ranges r;
    if (ranges)
        r = *ranges;
    else
        rac_default_ranges(&r);
    if (!rac::ranges_ok(r)) return fail(RAC_EINVAL, "rac_sample_params: invalid ranges");
    const double M = rac::ratio_median(r);
    const double inv_lo = 1.0 / r.lam_inh_max, inv_hi = 1.0 / r.lam_inh_min;
    const int32_t n_span = r.n_max - r.n_min + 1;
    for (int64_t j = 0; j < n_sets; ++j) {
        const uint64_t p = (uint64_t)(set_begin + j);
        for (int64_t i = 0; i < N; ++i) {
            out->G[i * n_sets + j] = (float)(r.g_min + (r.g_max - r.g_min) * rac::draw(seed, p, i, 0));
            out->k[i * n_sets + j] = (float)(r.k_min + (r.k_max - r.k_min) * rac::draw(seed, p, N + i, 0));
        }
        for (int64_t e = 0; e < E; ++e) {
            const uint64_t slot = 2 * N + 3 * e;
            const double ut = rac::draw(seed, p, slot, 0);
            out->T[e * n_sets + j] = (float)(M * (r.t_lo + (r.t_hi - r.t_lo) * ut));
            const double un = rac::draw(seed, p, slot + 1, 0);
            int32_t k = (int32_t)std::floor(un * n_span);
            if (k > n_span - 1) k = n_span - 1;
            out->n[e * n_sets + j] = (uint8_t)(r.n_min + k);
            const double ul = rac::draw(seed, p, slot + 2, 0);
            double lam;
            if (topo->sign[e] > 0)
                lam = r.lam_act_min + (r.lam_act_max - r.lam_act_min) * ul;
            else  // uniform in the inverse range, then inverted
                lam = 1.0 / (inv_lo + (inv_hi - inv_lo) * ul);
            out->lam[e * n_sets + j] = (float)lam;
        }
    }
    if (ic_frac)
        for (int64_t c = 0; c < n_ic; ++c)
            for (int64_t i = 0; i < N; ++i) ic_frac[c * N + i] = (float)rac::draw(seed, c, i, 1);
    return RAC_OK;
}

}  // extern "C"
