// Host-side parameter and initial-condition sampling (GRiNS Sec. 2.1.2,
// Table 1) from a counter-based generator, so that any parameter set can be
// regenerated from (seed, set index) alone.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

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
           (r.g_max > 0 || r.t_median > 0) &&
           (r.method == RAC_SAMPLE_UNIFORM || r.method == RAC_SAMPLE_SOBOL || r.method == RAC_SAMPLE_LHS) &&
           (r.threshold_rule == RAC_THRESHOLD_PRIOR_MEDIAN || r.threshold_rule == RAC_THRESHOLD_HALF_FUNCTIONAL) &&
           r.hf_samples >= 1 && r.lhs_total >= 0 && (r.n_continuous == 0 || r.n_continuous == 1);
}

// ---- Sobol' direction numbers ---------------------------------------------
// GF(2) polynomials as bit masks (bit j = coefficient of x^j).
uint64_t gf2_mul_mod(uint64_t a, uint64_t b, uint64_t poly, int deg) {
    uint64_t acc = 0;
    for (; b; b >>= 1) {
        if (b & 1) acc ^= a;
        a <<= 1;
        if ((a >> deg) & 1) a ^= poly;
    }
    return acc;
}

// x^e modulo poly.
uint64_t gf2_x_pow(uint64_t e, uint64_t poly, int deg) {
    uint64_t acc = 1, base = deg == 1 ? 1 : 2;
    for (; e; e >>= 1) {
        if (e & 1) acc = gf2_mul_mod(acc, base, poly, deg);
        base = gf2_mul_mod(base, base, poly, deg);
    }
    return acc;
}

bool primitive(uint64_t poly, int deg) {
    const uint64_t ord = (1ull << deg) - 1;
    if (gf2_x_pow(ord, poly, deg) != 1) return false;
    uint64_t rest = ord;
    for (uint64_t f = 2; f * f <= rest; ++f) {
        if (rest % f) continue;
        while (rest % f == 0) rest /= f;
        if (gf2_x_pow(ord / f, poly, deg) == 1) return false;
    }
    if (rest > 1 && rest < ord && gf2_x_pow(ord / rest, poly, deg) == 1) return false;
    return true;
}

const uint32_t* sobol_table() {
    static std::vector<uint32_t> v;
    static std::once_flag once;
    std::call_once(once, [] {
        v.assign((size_t)kSobolDims * 32, 0);
        for (int b = 0; b < 32; ++b) v[b] = 1u << (31 - b);
        int dim = 1;
        for (int deg = 1; deg <= 18 && dim < kSobolDims; ++deg) {
            for (uint64_t poly = (1ull << deg) + 1; poly < (2ull << deg) && dim < kSobolDims; poly += 2) {
                if (!primitive(poly, deg)) continue;
                uint64_t m[33] = {0};
                for (int k = 1; k <= deg; ++k) {
                    uint64_t w[4] = {(uint64_t)dim, (uint64_t)k, 0, 0};
                    Philox4x64::block(w, 0x536F626F6C2D6D6Bull, 0);
                    m[k] = 2 * (w[0] % (1ull << (k - 1))) + 1;
                }
                for (int k = deg + 1; k <= 32; ++k) {
                    uint64_t next = m[k - deg] ^ (m[k - deg] << deg);
                    for (int j = 1; j < deg; ++j)
                        if ((poly >> (deg - j)) & 1) next ^= m[k - j] << j;
                    m[k] = next;
                }
                for (int b = 0; b < 32; ++b) v[(size_t)dim * 32 + b] = (uint32_t)(m[b + 1] << (31 - b));
                ++dim;
            }
        }
    });
    return v.data();
}

uint32_t sobol_point(const uint32_t* V, uint64_t i, int q) {
    uint32_t x = 0;
    for (int b = 0; i; ++b, i >>= 1)
        if (i & 1) x ^= V[(size_t)q * 32 + b];
    return x;
}

// ---- Latin hypercube permutations ------------------------------------------
uint64_t lhs_round_mix(uint64_t x, const uint64_t* key, int w) {
    const uint64_t mask = w >= 64 ? ~0ull : (1ull << w) - 1;
    const int sh = w / 2 > 0 ? w / 2 : 1;
    for (int r = 0; r < 4; ++r) {
        x = (x ^ key[r]) & mask;
        x = (x * 0x9E3779B97F4A7C15ull) & mask;
        x ^= x >> sh;
    }
    return x;
}

uint64_t lhs_cell(uint64_t i, const uint64_t* key, int w, uint64_t n) {
    do {
        i = lhs_round_mix(i, key, w);
    } while (i >= n);
    return i;
}

double unit(const SampleTables& t, uint64_t seed, uint64_t item, uint64_t q, int domain) {
    if (t.method == RAC_SAMPLE_SOBOL) {
        const uint32_t sh = domain ? t.shift1[q] : t.shift0[q];
        return (double)(sobol_point(t.sobol_v, item, (int)q) ^ sh) * (1.0 / 4294967296.0);
    }
    if (t.method == RAC_SAMPLE_LHS) {
        const uint64_t* key = domain ? &t.lhs_key1[4 * q] : &t.lhs_key0[4 * q];
        const int64_t n = domain ? t.lhs_n1 : t.lhs_n0;
        const uint64_t cell = lhs_cell(item, key, domain ? t.lhs_w1 : t.lhs_w0, (uint64_t)n);
        return ((double)cell + draw(seed, item, q, 6 + domain)) / (double)n;
    }
    return draw(seed, item, q, domain);
}

// ---- Half-functional threshold scale ---------------------------------------
double shifted_hill(double B, double B0, double n, double lam) {
    const double a = std::pow(B0, n), b = std::pow(B, n);
    return a / (a + b) + lam * b / (a + b);
}

double hf_draw(uint64_t na, uint64_t nh, uint64_t s, uint64_t d) {
    uint64_t w[4] = {na, nh, s, d >> 2};
    Philox4x64::block(w, 0x48616C662D66756Eull, 0);
    return (double)(w[d & 3] >> 11) * (1.0 / 9007199254740992.0);
}

double hf_median(const rac_ranges& r, int na, int nh) {
    const double M0 = ratio_median(r);
    if (na + nh == 0) return M0;
    // Cached per (ranges, class): the estimate is a pure function of both.
    static std::mutex mu;
    static std::map<std::string, double> cache;
    std::string key((const char*)&r, sizeof(r));
    key.append((const char*)&na, sizeof(na));
    key.append((const char*)&nh, sizeof(nh));
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const double inv_lo = 1.0 / r.lam_inh_max, inv_hi = 1.0 / r.lam_inh_min;
    const int32_t span = r.n_max - r.n_min + 1;
    std::vector<double> level((size_t)r.hf_samples);
    for (int s = 0; s < r.hf_samples; ++s) {
        uint64_t d = 0;
        const double G = r.g_min + (r.g_max - r.g_min) * hf_draw(na, nh, s, d++);
        const double k = r.k_min + (r.k_max - r.k_min) * hf_draw(na, nh, s, d++);
        double x = G / k;
        for (int e = 0; e < na + nh; ++e) {
            const double Gs = r.g_min + (r.g_max - r.g_min) * hf_draw(na, nh, s, d++);
            const double ks = r.k_min + (r.k_max - r.k_min) * hf_draw(na, nh, s, d++);
            const double T = M0 * (r.t_lo + (r.t_hi - r.t_lo) * hf_draw(na, nh, s, d++));
            const double un = hf_draw(na, nh, s, d++);
            double n;
            if (r.n_continuous) {
                n = (double)(float)((double)r.n_min + (double)(r.n_max - r.n_min) * un);
            } else {
                int32_t off = (int32_t)std::floor(un * span);
                if (off > span - 1) off = span - 1;
                n = (double)(r.n_min + off);
            }
            const double u = hf_draw(na, nh, s, d++);
            const bool act = e < na;
            const double lam = act ? r.lam_act_min + (r.lam_act_max - r.lam_act_min) * u
                                   : 1.0 / (inv_lo + (inv_hi - inv_lo) * u);
            double h = shifted_hill(Gs / ks, T, n, lam);
            if (act && r.hf_act_over_lambda) h = h / lam;
            x *= h;
        }
        level[(size_t)s] = x;
    }
    std::sort(level.begin(), level.end());
    const size_t S = level.size();
    const double med = (S % 2) ? level[S / 2] : 0.5 * (level[S / 2 - 1] + level[S / 2]);
    const double out = (double)(float)med;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = out;
    return out;
}

int width_for(int64_t n) {
    int w = 1;
    while (w < 63 && (1ll << w) < n) ++w;
    return w;
}

}  // namespace

bool sample_ranges_ok(const rac_ranges& r) { return ranges_ok(r); }
double sample_ratio_median(const rac_ranges& r) { return ratio_median(r); }

rac_status make_sample_tables(const rac_topology* t, const rac_ranges& r, uint64_t seed, int64_t set_begin,
                              int64_t n_sets, int32_t n_ic, SampleTables* out) {
    const int64_t N = t->n_genes, E = t->n_edges, D = 2 * N + 3 * E;
    SampleTables& tb = *out;
    tb.method = r.method;
    // Threshold scale per edge.
    const double M0 = ratio_median(r);
    tb.scale.assign((size_t)E, M0);
    if (r.t_median <= 0 && r.threshold_rule == RAC_THRESHOLD_HALF_FUNCTIONAL) {
        std::vector<int> na((size_t)N, 0), nh((size_t)N, 0);
        for (int64_t e = 0; e < E; ++e) (t->sign[e] > 0 ? na : nh)[(size_t)t->dst[e]]++;
        for (int64_t e = 0; e < E; ++e) {
            const int s = t->src[e];
            tb.scale[(size_t)e] = hf_median(r, na[(size_t)s], nh[(size_t)s]);
        }
    }
    if (r.method == RAC_SAMPLE_SOBOL) {
        if (D > kSobolDims || N > kSobolDims || set_begin + n_sets > (1ll << 32) || n_ic > (1ll << 32))
            return fail(RAC_EUNSUPPORTED, "Sobol' sampling supports at most 4096 dimensions and 2^32 points");
        tb.sobol_v = sobol_table();
        auto shifts = [&](int domain, int64_t dims, std::vector<uint32_t>& v) {
            v.resize((size_t)dims);
            for (int64_t q = 0; q < dims; ++q) {
                uint64_t w[4] = {(uint64_t)q, 0, (uint64_t)(2 + domain), 0};
                Philox4x64::block(w, seed, 0);
                v[(size_t)q] = (uint32_t)(w[0] >> 32);
            }
        };
        shifts(0, D, tb.shift0);
        shifts(1, N, tb.shift1);
    } else if (r.method == RAC_SAMPLE_LHS) {
        tb.lhs_n0 = r.lhs_total > 0 ? r.lhs_total : set_begin + n_sets;
        if (tb.lhs_n0 < set_begin + n_sets)
            return fail(RAC_EINVAL, "lhs_total is below set_begin + n_sets");
        tb.lhs_n1 = n_ic;
        tb.lhs_w0 = width_for(tb.lhs_n0);
        tb.lhs_w1 = width_for(tb.lhs_n1);
        auto keys = [&](int domain, int64_t dims, std::vector<uint64_t>& v) {
            v.resize((size_t)dims * 4);
            for (int64_t q = 0; q < dims; ++q) {
                uint64_t w[4] = {(uint64_t)q, 0, (uint64_t)(4 + domain), 0};
                Philox4x64::block(w, seed, 0);
                for (int j = 0; j < 4; ++j) v[(size_t)q * 4 + j] = w[j];
            }
        };
        keys(0, D, tb.lhs_key0);
        keys(1, N, tb.lhs_key1);
    }
    return RAC_OK;
}

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
    r->method = RAC_SAMPLE_UNIFORM;
    r->threshold_rule = RAC_THRESHOLD_PRIOR_MEDIAN;
    r->hf_samples = 65536;
    r->hf_act_over_lambda = 1;
    r->lhs_total = 0;
    r->n_continuous = 0;
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
    rac_ranges r;
    if (ranges)
        r = *ranges;
    else
        rac_default_ranges(&r);
    if (!rac::ranges_ok(r)) return fail(RAC_EINVAL, "rac_sample_params: invalid ranges");
    if (n_sets > 0 && (!out->G || !out->k ||
                       (E > 0 && (!out->T || !out->lam || (r.n_continuous ? !out->nf : !out->n)))))
        return fail(RAC_EINVAL, "rac_sample_params: NULL parameter array");
    rac::SampleTables tb;
    rac_status st = rac::make_sample_tables(topo, r, seed, set_begin, n_sets, n_ic, &tb);
    if (st != RAC_OK) return st;
    const double inv_lo = 1.0 / r.lam_inh_max, inv_hi = 1.0 / r.lam_inh_min;
    const int32_t n_span = r.n_max - r.n_min + 1;
    for (int64_t j = 0; j < n_sets; ++j) {
        const uint64_t p = (uint64_t)(set_begin + j);
        for (int64_t i = 0; i < N; ++i) {
            out->G[i * n_sets + j] = (float)(r.g_min + (r.g_max - r.g_min) * rac::unit(tb, seed, p, i, 0));
            out->k[i * n_sets + j] = (float)(r.k_min + (r.k_max - r.k_min) * rac::unit(tb, seed, p, N + i, 0));
        }
        for (int64_t e = 0; e < E; ++e) {
            const uint64_t slot = 2 * N + 3 * e;
            const double ut = rac::unit(tb, seed, p, slot, 0);
            out->T[e * n_sets + j] = (float)(tb.scale[(size_t)e] * (r.t_lo + (r.t_hi - r.t_lo) * ut));
            const double un = rac::unit(tb, seed, p, slot + 1, 0);
            if (r.n_continuous) {
                out->nf[e * n_sets + j] = (float)((double)r.n_min + (double)(r.n_max - r.n_min) * un);
            } else {
                int32_t k = (int32_t)std::floor(un * n_span);
                if (k > n_span - 1) k = n_span - 1;
                out->n[e * n_sets + j] = (uint8_t)(r.n_min + k);
                if (out->nf) out->nf[e * n_sets + j] = (float)(r.n_min + k);
            }
            const double ul = rac::unit(tb, seed, p, slot + 2, 0);
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
            for (int64_t i = 0; i < N; ++i) ic_frac[c * N + i] = (float)rac::unit(tb, seed, c, i, 1);
    return RAC_OK;
}

}  // extern "C"
