/*
 * RACIPE CPU oracle -- TEST INFRASTRUCTURE ONLY (tests, smoke check and the
 * benchmark's CPU baseline).  Plain FP64 C, no blocking or fusion, written
 * for readability against the GRiNS paper (arXiv 2503.18356).  Shares no
 * code with the GPU library.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Ten rounds of two 64x64->128 multiplies with   */
/* the published multipliers and Weyl key increments.                        */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The q-th uniform of stream (a, domain): counter (a, q/4, domain, 0), key
 * (seed, 0), word q%4, top 53 bits scaled to [0, 1). */
static double orc_uniform(uint64_t seed, uint64_t a, uint64_t q, uint64_t domain) {
    uint64_t ctr[4] = {a, q / 4, domain, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return (double)(out[q % 4] >> 11) * 0x1.0p-53;
}

/* ------------------------------------------------------------------------ */
/* Topology: canonical edge order sorted by (dst, src).                      */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t s, d; int8_t g; } orc_edge;

static int orc_edge_cmp(const void* a, const void* b) {
    const orc_edge* x = (const orc_edge*)a;
    const orc_edge* y = (const orc_edge*)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    return 0;
}

int orc_canonicalize(int n_genes, int n_edges, const int32_t* src, const int32_t* dst,
                     const int8_t* sign, int32_t* out_src, int32_t* out_dst, int8_t* out_sign) {
    if (n_genes < 1 || n_edges < 0) return -1;
    orc_edge* e = (orc_edge*)malloc(sizeof(orc_edge) * (size_t)(n_edges > 0 ? n_edges : 1));
    for (int i = 0; i < n_edges; ++i) {
        if (src[i] < 0 || src[i] >= n_genes || dst[i] < 0 || dst[i] >= n_genes ||
            (sign[i] != 1 && sign[i] != -1)) {
            free(e);
            return -1;
        }
        e[i].s = src[i]; e[i].d = dst[i]; e[i].g = sign[i];
    }
    qsort(e, (size_t)n_edges, sizeof(orc_edge), orc_edge_cmp);
    for (int i = 1; i < n_edges; ++i)
        if (e[i].s == e[i - 1].s && e[i].d == e[i - 1].d) { free(e); return -1; }
    for (int i = 0; i < n_edges; ++i) { out_src[i] = e[i].s; out_dst[i] = e[i].d; out_sign[i] = e[i].g; }
    free(e);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sampling (Sec. 2.1.2, Table 1).                                           */
/* ------------------------------------------------------------------------ */
void orc_default_ranges(orc_ranges* r) {
    /* Table 1 defaults. */
    r->g_min = 1.0;  r->g_max = 100.0;
    r->k_min = 0.1;  r->k_max = 1.0;
    r->lam_act_min = 1.0;  r->lam_act_max = 100.0;
    r->lam_inh_min = 0.01; r->lam_inh_max = 1.0;
    r->n_min = 1; r->n_max = 6;
    /* Half-functional window: 0.02 .. 1.98 times the median. */
    r->t_lo = 0.02; r->t_hi = 1.98;
    r->t_median = 0.0;
    r->method = ORC_UNIFORM;
    r->threshold_rule = ORC_T_PRIOR_MEDIAN;
    r->hf_samples = 65536;
    r->hf_act_over_lambda = 1;
    r->lhs_total = 0;
    r->n_continuous = 0;
}

/* CDF of G/k for independent G ~ U[a,b], k ~ U[c,d]:
 *   F(m) = (1/(d-c)) * integral_c^d clip((m*k - a)/(b - a), 0, 1) dk. */
static double orc_gk_cdf(const orc_ranges* r, double m) {
    double a = r->g_min, b = r->g_max, c = r->k_min, d = r->k_max;
    if (d <= c) { /* k fixed */
        if (b <= a) return (m * c >= a) ? 1.0 : 0.0;
        double v = (m * c - a) / (b - a);
        return v < 0 ? 0 : (v > 1 ? 1 : v);
    }
    if (b <= a) { /* G fixed: P(a/k <= m) = P(k >= a/m) */
        double kk = a / m;
        double v = (d - kk) / (d - c);
        return v < 0 ? 0 : (v > 1 ? 1 : v);
    }
    double k1 = a / m, k2 = b / m; /* the ramp runs for k in [k1, k2] */
    double lo = k1 < c ? c : (k1 > d ? d : k1);
    double hi = k2 < c ? c : (k2 > d ? d : k2);
    double ramp = (m * (hi * hi - lo * lo) / 2.0 - a * (hi - lo)) / (b - a);
    double flat = d - hi; /* k above k2: the clip is 1 */
    return (ramp + flat) / (d - c);
}

double orc_gk_median(const orc_ranges* r) {
    if (r->t_median > 0) return r->t_median;
    /* Interior case: the ramp covers all k, so F is linear in m and
     * F(m) = (m*E[k] - a)/(b - a) = 1/2 gives m = (a + b)/(c + d). */
    double m = (r->g_min + r->g_max) / (r->k_min + r->k_max);
    if (m * r->k_min >= r->g_min && m * r->k_max <= r->g_max) return m;
    /* Otherwise bisection on the CDF. */
    double lo = r->g_min / r->k_max, hi = r->g_max / r->k_min;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (orc_gk_cdf(r, mid) < 0.5) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------ */
/* Sobol' sequence: primitive polynomials over GF(2) by increasing degree    */
/* (then value); dimension q >= 1 uses the (q-1)-th.  Initial direction      */
/* numbers m_1..m_s are odd and below 2^k, drawn once from Philox with a     */
/* fixed key; later ones follow Bratley and Fox's recurrence.  Points are    */
/* generated directly from the binary digits of the index.                   */
/* ------------------------------------------------------------------------ */
#define ORC_SOBOL_MAX_DEG 18
#define ORC_SOBOL_MAX_DIM 4096

static uint64_t orc_gf2_mulmod(uint64_t a, uint64_t b, uint64_t poly, int s) {
    uint64_t r = 0;
    while (b) {
        if (b & 1) r ^= a;
        b >>= 1;
        a <<= 1;
        if (a >> s & 1) a ^= poly;
    }
    return r;
}

static uint64_t orc_gf2_xpow(uint64_t e, uint64_t poly, int s) {
    uint64_t result = 1, base = 2 % (1ull << s);
    if (s == 1) base = 1; /* x = 1 mod (x + 1) */
    while (e) {
        if (e & 1) result = orc_gf2_mulmod(result, base, poly, s);
        base = orc_gf2_mulmod(base, base, poly, s);
        e >>= 1;
    }
    return result;
}

/* Primitive iff x has multiplicative order 2^s - 1 modulo the polynomial. */
static int orc_is_primitive(uint64_t poly, int s) {
    uint64_t order = (1ull << s) - 1;
    if (orc_gf2_xpow(order, poly, s) != 1) return 0;
    uint64_t m = order;
    for (uint64_t f = 2; f * f <= m; ++f) {
        if (m % f) continue;
        while (m % f == 0) m /= f;
        if (orc_gf2_xpow(order / f, poly, s) == 1) return 0;
    }
    if (m > 1 && m != order && orc_gf2_xpow(order / m, poly, s) == 1) return 0;
    return 1;
}

static uint32_t orc_sobol_v[ORC_SOBOL_MAX_DIM][32];
static int orc_sobol_ready = 0;
static int orc_prim_count[ORC_SOBOL_MAX_DEG + 1];
static pthread_once_t orc_sobol_once = PTHREAD_ONCE_INIT;

static void orc_sobol_init(void) {
    for (int b = 0; b < 32; ++b) orc_sobol_v[0][b] = 1u << (31 - b);
    int q = 1;
    for (int s = 1; s <= ORC_SOBOL_MAX_DEG; ++s) {
        for (uint64_t poly = (1ull << s) | 1; poly < (2ull << s); poly += 2) {
            if (!orc_is_primitive(poly, s)) continue;
            orc_prim_count[s]++;
            if (q >= ORC_SOBOL_MAX_DIM) continue;
            uint64_t m[33];
            for (int k = 1; k <= s && k <= 32; ++k) {
                uint64_t ctr[4] = {(uint64_t)q, (uint64_t)k, 0, 0};
                uint64_t key[2] = {0x536F626F6C2D6D6Bull, 0};
                uint64_t out[4];
                orc_philox4x64_10(ctr, key, out);
                m[k] = (out[0] % (1ull << (k - 1))) * 2 + 1; /* odd, < 2^k */
            }
            for (int k = s + 1; k <= 32; ++k) {
                uint64_t v = m[k - s] ^ (m[k - s] << s);
                for (int j = 1; j < s; ++j)
                    if (poly >> (s - j) & 1) v ^= m[k - j] << j;
                m[k] = v;
            }
            for (int b = 0; b < 32; ++b) orc_sobol_v[q][b] = (uint32_t)(m[b + 1] << (31 - b));
            ++q;
        }
    }
    orc_sobol_ready = q;
}

int orc_sobol_u32(int64_t i, int32_t q, uint32_t* out) {
    pthread_once(&orc_sobol_once, orc_sobol_init);
    if (q < 0 || q >= orc_sobol_ready || i < 0 || i >= (1ll << 32)) return -1;
    uint32_t x = 0;
    for (int b = 0; b < 32; ++b)
        if (((uint64_t)i >> b) & 1) x ^= orc_sobol_v[q][b];
    *out = x;
    return 0;
}

int orc_primitive_count(int32_t s) {
    pthread_once(&orc_sobol_once, orc_sobol_init);
    return (s >= 1 && s <= ORC_SOBOL_MAX_DEG) ? orc_prim_count[s] : -1;
}

/* Digital shift of dimension q in a domain (0 parameters, 1 initial
 * conditions), keyed by the seed. */
static uint32_t orc_sobol_shift(uint64_t seed, int32_t domain, int32_t q) {
    uint64_t ctr[4] = {(uint64_t)q, 0, (uint64_t)(2 + domain), 0};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return (uint32_t)(out[0] >> 32);
}

/* ------------------------------------------------------------------------ */
/* Latin hypercube: in dimension q item i falls in stratum perm_q(i), with   */
/* a uniform offset inside it.  perm_q is a keyed bijection of [0, n): an     */
/* invertible mix of w-bit words (2^w >= n) applied until the value lands    */
/* in [0, n) (cycle walking).                                                */
/* ------------------------------------------------------------------------ */
static uint64_t orc_lhs_mix(uint64_t x, const uint64_t k[4], int w) {
    const uint64_t mask = w >= 64 ? ~0ull : ((1ull << w) - 1);
    const int sh = w / 2 > 0 ? w / 2 : 1;
    for (int r = 0; r < 4; ++r) {
        x = (x ^ k[r]) & mask;
        x = (x * 0x9E3779B97F4A7C15ull) & mask;  /* odd multiplier: bijective */
        x ^= x >> sh;                            /* xorshift: bijective */
    }
    return x;
}

int64_t orc_lhs_perm(uint64_t seed, int32_t domain, int32_t q, int64_t n, int64_t i) {
    if (n < 1 || i < 0 || i >= n) return -1;
    int w = 1;
    while ((1ll << w) < n) ++w;
    uint64_t ctr[4] = {(uint64_t)q, 0, (uint64_t)(4 + domain), 0};
    uint64_t key[2] = {seed, 0};
    uint64_t k[4];
    orc_philox4x64_10(ctr, key, k);
    uint64_t x = (uint64_t)i;
    do {
        x = orc_lhs_mix(x, k, w);
    } while (x >= (uint64_t)n);
    return (int64_t)x;
}

/* The unit-cube coordinate of dimension q for item a (a parameter set or an
 * initial condition) under the configured generator. */
static double orc_unit(const orc_ranges* r, uint64_t seed, uint64_t a, uint64_t q, int domain,
                       int64_t lhs_n) {
    if (r->method == ORC_SOBOL) {
        uint32_t v = 0;
        orc_sobol_u32((int64_t)a, (int32_t)q, &v);
        return (double)(v ^ orc_sobol_shift(seed, domain, (int32_t)q)) * 0x1.0p-32;
    }
    if (r->method == ORC_LHS) {
        int64_t cell = orc_lhs_perm(seed, domain, (int32_t)q, lhs_n, (int64_t)a);
        double jitter = orc_uniform(seed, a, q, (uint64_t)(6 + domain));
        return ((double)cell + jitter) / (double)lhs_n;
    }
    return orc_uniform(seed, a, q, (uint64_t)domain);
}

/* ------------------------------------------------------------------------ */
/* Half-functional rule (Sec. 2.1.2): the threshold scale of an edge is the  */
/* median level of its source.  For a source with n_act activating and      */
/* n_inh inhibitory regulators that level is taken one step deep: its own    */
/* G/k times the Hill terms of its in-edges, each regulator at an            */
/* unregulated level G'/k' and each in-edge with prior T, n and lambda; the  */
/* median over hf_samples Monte Carlo draws (Philox, fixed key), rounded to  */
/* FP32.  Unregulated sources use the prior median of G/k.                   */
/* ------------------------------------------------------------------------ */
static double orc_shifted_hill(double B, double B0, double n, double lam);

static int orc_cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static double orc_hf_draw(uint64_t na, uint64_t nh, uint64_t s, uint64_t d) {
    uint64_t ctr[4] = {na, nh, s, d / 4};
    uint64_t key[2] = {0x48616C662D66756Eull, 0};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return (double)(out[d % 4] >> 11) * 0x1.0p-53;
}

double orc_hf_median(const orc_ranges* r, int32_t n_act, int32_t n_inh) {
    const double M0 = orc_gk_median(r);
    if (n_act + n_inh == 0 || r->hf_samples < 1) return M0;
    const int S = r->hf_samples;
    double* v = (double*)malloc(sizeof(double) * (size_t)S);
    for (int s = 0; s < S; ++s) {
        uint64_t d = 0;
        double G = r->g_min + (r->g_max - r->g_min) * orc_hf_draw(n_act, n_inh, s, d++);
        double k = r->k_min + (r->k_max - r->k_min) * orc_hf_draw(n_act, n_inh, s, d++);
        double x = G / k;
        for (int e = 0; e < n_act + n_inh; ++e) {
            double Gs = r->g_min + (r->g_max - r->g_min) * orc_hf_draw(n_act, n_inh, s, d++);
            double ks = r->k_min + (r->k_max - r->k_min) * orc_hf_draw(n_act, n_inh, s, d++);
            double T = M0 * (r->t_lo + (r->t_hi - r->t_lo) * orc_hf_draw(n_act, n_inh, s, d++));
            double un = orc_hf_draw(n_act, n_inh, s, d++), n;
            if (r->n_continuous) {
                n = (double)(float)((double)r->n_min + (double)(r->n_max - r->n_min) * un);
            } else {
                int32_t span = r->n_max - r->n_min + 1;
                int32_t off = (int32_t)floor(un * span);
                if (off > span - 1) off = span - 1;
                n = (double)(r->n_min + off);
            }
            double u = orc_hf_draw(n_act, n_inh, s, d++);
            double lam;
            if (e < n_act) {
                lam = r->lam_act_min + (r->lam_act_max - r->lam_act_min) * u;
            } else {
                double inv_lo = 1.0 / r->lam_inh_max, inv_hi = 1.0 / r->lam_inh_min;
                lam = 1.0 / (inv_lo + (inv_hi - inv_lo) * u);
            }
            double h = orc_shifted_hill(Gs / ks, T, n, lam);
            if (e < n_act && r->hf_act_over_lambda) h = h / lam;
            x *= h;
        }
        v[s] = x;
    }
    qsort(v, (size_t)S, sizeof(double), orc_cmp_double);
    double med = (S % 2) ? v[S / 2] : 0.5 * (v[S / 2 - 1] + v[S / 2]);
    free(v);
    return (double)(float)med;
}

int orc_sample(int n_genes, int n_edges, const int32_t* src, const int32_t* dst, const int8_t* sign,
               const orc_ranges* r, uint64_t seed, int64_t set_begin, int64_t n_sets, int32_t n_ic,
               float* G, float* k, float* T, float* lam, uint8_t* n, float* ic, float* nf) {
    if (n_genes < 1 || n_edges < 0 || n_sets < 0 || n_ic < 0) return -1;
    if (r->n_continuous ? !nf : !n) return -1;
    if (r->method != ORC_UNIFORM && r->method != ORC_SOBOL && r->method != ORC_LHS) return -1;
    if (r->threshold_rule != ORC_T_PRIOR_MEDIAN && r->threshold_rule != ORC_T_HALF_FUNCTIONAL) return -1;
    const int64_t N = n_genes, E = n_edges;
    if (r->method == ORC_SOBOL && (2 * N + 3 * E > ORC_SOBOL_MAX_DIM || set_begin + n_sets > (1ll << 32)))
        return -1;
    const int64_t lhs_n = r->lhs_total > 0 ? r->lhs_total : set_begin + n_sets;
    if (r->method == ORC_LHS && lhs_n < set_begin + n_sets) return -1;
    /* Threshold scale per edge: the fixed value, the prior median, or the
     * half-functional median of the edge's source. */
    double* scale = (double*)malloc(sizeof(double) * (size_t)(E > 0 ? E : 1));
    const double M0 = orc_gk_median(r);
    for (int64_t e = 0; e < E; ++e) {
        scale[e] = M0;
        if (r->t_median <= 0 && r->threshold_rule == ORC_T_HALF_FUNCTIONAL) {
            int32_t na = 0, nh = 0;
            for (int64_t f = 0; f < E; ++f)
                if (dst[f] == src[e]) {
                    if (sign[f] > 0) ++na; else ++nh;
                }
            scale[e] = orc_hf_median(r, na, nh);
        }
    }
    for (int64_t j = 0; j < n_sets; ++j) {
        const uint64_t p = (uint64_t)(set_begin + j);
        for (int64_t i = 0; i < N; ++i) {
            double u = orc_unit(r, seed, p, (uint64_t)i, 0, lhs_n);
            G[i * n_sets + j] = (float)(r->g_min + (r->g_max - r->g_min) * u);
            u = orc_unit(r, seed, p, (uint64_t)(N + i), 0, lhs_n);
            k[i * n_sets + j] = (float)(r->k_min + (r->k_max - r->k_min) * u);
        }
        for (int64_t e = 0; e < E; ++e) {
            uint64_t base = (uint64_t)(2 * N + 3 * e);
            /* Threshold: uniform in [t_lo, t_hi] times the source's scale. */
            double u = orc_unit(r, seed, p, base, 0, lhs_n);
            T[e * n_sets + j] = (float)(scale[e] * (r->t_lo + (r->t_hi - r->t_lo) * u));
            /* Hill coefficient: integer, uniform over n_min..n_max; or, in the
             * continuous option, real and uniform on [n_min, n_max]. */
            u = orc_unit(r, seed, p, base + 1, 0, lhs_n);
            if (r->n_continuous) {
                nf[e * n_sets + j] = (float)((double)r->n_min + (double)(r->n_max - r->n_min) * u);
            } else {
                int32_t span = r->n_max - r->n_min + 1;
                int32_t off = (int32_t)floor(u * span);
                if (off > span - 1) off = span - 1;
                n[e * n_sets + j] = (uint8_t)(r->n_min + off);
                if (nf) nf[e * n_sets + j] = (float)(r->n_min + off);
            }
            /* Fold change: activation uniform in its range; inhibition uniform
             * in the inverse range, then inverted. */
            u = orc_unit(r, seed, p, base + 2, 0, lhs_n);
            double l;
            if (sign[e] > 0) {
                l = r->lam_act_min + (r->lam_act_max - r->lam_act_min) * u;
            } else {
                double inv_lo = 1.0 / r->lam_inh_max, inv_hi = 1.0 / r->lam_inh_min;
                l = 1.0 / (inv_lo + (inv_hi - inv_lo) * u);
            }
            lam[e * n_sets + j] = (float)l;
        }
    }
    free(scale);
    if (ic) {
        /* Initial conditions: fractions of each node's range, shared by all
         * sets; a Latin hypercube over the n_ic conditions. */
        for (int64_t c = 0; c < n_ic; ++c)
            for (int64_t i = 0; i < N; ++i)
                ic[c * N + i] = (float)orc_unit(r, seed, (uint64_t)c, (uint64_t)i, 1, n_ic);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. 1 and Eq. 2, literally.                                               */
/* ------------------------------------------------------------------------ */
void orc_default_opts(orc_opts* o) {
    o->t0 = 0.0; o->t_end = 200.0; o->rtol = 1e-6; o->atol = 1e-9;
    o->ss_atol = 1e-6; o->ss_rtol = 0.0; o->h0 = 0.0; o->max_steps = 100000;
    o->divide_act_by_lambda = 1; o->stop_at_steady = 0; o->ic_absolute = 0;
    o->method = ORC_DP5;
}

/* Shifted Hill function H^S(B, B0, n, lambda), Eq. 2. */
static double orc_shifted_hill(double B, double B0, double n, double lam) {
    double a = pow(B0, n);
    double b = pow(B, n);
    return a / (a + b) + lam * b / (a + b);
}

void orc_rhs(const orc_problem* pb, int64_t p, int32_t divide, const double* x, double* f) {
    const int64_t P = pb->n_sets;
    int e = 0;
    for (int i = 0; i < pb->n_genes; ++i) {
        double prod = 1.0;
        /* Canonical order groups the in-edges of gene i together. */
        while (e < pb->n_edges && pb->dst[e] == i) {
            int j = pb->src[e];
            double B = x[j] > 0.0 ? x[j] : 0.0;
            double lam = pb->lam[e * P + p];
            /* Hill coefficient: the integer array, or the real-valued one when given. */
            double n = pb->nf ? (double)pb->nf[e * P + p] : (double)pb->n[e * P + p];
            double hs = orc_shifted_hill(B, pb->T[e * P + p], n, lam);
            if (pb->sign[e] > 0 && divide) hs = hs / lam; /* activating term over lambda */
            prod *= hs;
            ++e;
        }
        f[i] = (double)pb->G[i * P + p] * prod - (double)pb->k[i * P + p] * x[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Dormand-Prince 5(4) tableau (Dormand & Prince 1980; Hairer, Norsett,       */
/* Wanner, Solving ODEs I, Table 5.2).                                       */
/* ------------------------------------------------------------------------ */
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84},
};
/* 5th-order weights (equal to the last row of A) and 4th-order weights. */
static const double DP_B[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
static const double DP_BH[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

/* ------------------------------------------------------------------------ */
/* Tsitouras 5(4) tableau (Ch. Tsitouras, Comput. Math. Appl. 62 (2011),      */
/* Table 1), the solver the paper's library uses (Sec. 2.1.3).  Nodes c2..c5  */
/* are 0.161, 0.327, 0.9 and 0.98002554...; c6 = c7 = 1.  The last row is the */
/* fifth-order solution; the differences b - bh are the published error      */
/* weights.                                                                  */
/* ------------------------------------------------------------------------ */
static const double TS_A[7][6] = {
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
static const double TS_E[7] = {-0.00178001105222577714, -0.0008164344596567469, 0.007880878010261995,
                               -0.1447110071732629,     0.5823571654525552,     -0.45808210592918697,
                               0.015151515151515152};

typedef struct {
    double a[7][7];
    double b[7], bh[7], c[7];
} orc_rk;

static void orc_rk_get(int32_t method, orc_rk* t) {
    memset(t, 0, sizeof(*t));
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j < 6; ++j) t->a[i][j] = method == ORC_TSIT5 ? TS_A[i][j] : DP_A[i][j];
        double ci = 0.0;
        for (int j = 0; j < i; ++j) ci += t->a[i][j];
        t->c[i] = ci;
    }
    for (int j = 0; j < 7; ++j) {
        if (method == ORC_TSIT5) {
            t->b[j] = j < 6 ? TS_A[6][j] : 0.0;
            t->bh[j] = t->b[j] - TS_E[j];
        } else {
            t->b[j] = DP_B[j];
            t->bh[j] = DP_BH[j];
        }
    }
}

int orc_tableau(int32_t method, double* a, double* b, double* bh, double* c) {
    if (method != ORC_DP5 && method != ORC_TSIT5) return -1;
    orc_rk t;
    orc_rk_get(method, &t);
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j < 7; ++j) a[i * 7 + j] = t.a[i][j];
        b[i] = t.b[i];
        bh[i] = t.bh[i];
        c[i] = t.c[i];
    }
    return 0;
}

typedef struct {
    const orc_problem* pb;
    const orc_opts* o;
    int64_t p;
    int N;
    orc_rk rk;
    double* k[7];
    double* y;
    double* xn;
} orc_stepper;

static void orc_stepper_init(orc_stepper* s, const orc_problem* pb, const orc_opts* o, int64_t p) {
    s->pb = pb; s->o = o; s->p = p; s->N = pb->n_genes;
    orc_rk_get(o->method, &s->rk);
    for (int i = 0; i < 7; ++i) s->k[i] = (double*)calloc((size_t)s->N, sizeof(double));
    s->y = (double*)calloc((size_t)s->N, sizeof(double));
    s->xn = (double*)calloc((size_t)s->N, sizeof(double));
}

static void orc_stepper_free(orc_stepper* s) {
    for (int i = 0; i < 7; ++i) free(s->k[i]);
    free(s->y);
    free(s->xn);
}

/* One attempt of the 5(4) pair from (x, f=k1) with step h.  Writes the
 * 5th-order result to s->xn, its derivative to s->k[6] (FSAL), and returns
 * the RMS error norm. */
static double orc_rk_attempt(orc_stepper* s, const double* x, const double* f, double h) {
    const int N = s->N;
    memcpy(s->k[0], f, sizeof(double) * (size_t)N);
    for (int st = 1; st < 7; ++st) {
        for (int i = 0; i < N; ++i) {
            double acc = 0.0;
            for (int l = 0; l < st; ++l) acc += s->rk.a[st][l] * s->k[l][i];
            s->y[i] = x[i] + h * acc;
        }
        orc_rhs(s->pb, s->p, s->o->divide_act_by_lambda, s->y, s->k[st]);
    }
    /* Stage 7 input is the 5th-order solution (first-same-as-last). */
    memcpy(s->xn, s->y, sizeof(double) * (size_t)N);
    double sum = 0.0;
    for (int i = 0; i < N; ++i) {
        double e = 0.0;
        for (int l = 0; l < 7; ++l) e += (s->rk.b[l] - s->rk.bh[l]) * s->k[l][i];
        e *= h;
        double ax = fabs(x[i]), an = fabs(s->xn[i]);
        double sc = s->o->atol + s->o->rtol * (ax > an ? ax : an);
        sum += (e / sc) * (e / sc);
    }
    return sqrt(sum / N);
}

static int orc_all_finite(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* Steady when every |dx_i/dt| <= ss_atol + ss_rtol * k_i * |x_i|. */
static int orc_is_steady(const orc_stepper* s, const double* x, const double* f) {
    const int64_t P = s->pb->n_sets;
    for (int i = 0; i < s->N; ++i) {
        double tol = s->o->ss_atol + s->o->ss_rtol * (double)s->pb->k[i * P + s->p] * fabs(x[i]);
        if (!(fabs(f[i]) <= tol)) return 0;
    }
    return 1;
}

static double orc_rms_scaled(const double* v, const double* x, int N, const orc_opts* o) {
    double sum = 0.0;
    for (int i = 0; i < N; ++i) {
        double sc = o->atol + o->rtol * fabs(x[i]);
        sum += (v[i] / sc) * (v[i] / sc);
    }
    return sqrt(sum / N);
}

/* Starting step size (Hairer, Norsett, Wanner I, Sec. II.4), order 5. */
static double orc_initial_step(orc_stepper* s, const double* x, const double* f, double hmax) {
    const int N = s->N;
    const orc_opts* o = s->o;
    double d0 = orc_rms_scaled(x, x, N, o);
    double d1 = orc_rms_scaled(f, x, N, o);
    /* Either norm below 1e-5: no usable scale, take 1e-6. */
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    if (h0 > hmax) h0 = hmax;
    for (int i = 0; i < N; ++i) s->y[i] = x[i] + h0 * f[i];
    orc_rhs(s->pb, s->p, o->divide_act_by_lambda, s->y, s->k[1]);
    double sum = 0.0;
    for (int i = 0; i < N; ++i) {
        double sc = o->atol + o->rtol * fabs(x[i]);
        double dv = (s->k[1][i] - f[i]) / sc;
        sum += dv * dv;
    }
    double d2 = sqrt(sum / N) / h0;
    double der = d1 > d2 ? d1 : d2;
    double h1 = (der <= 1e-15) ? (1e-6 > h0 * 1e-3 ? 1e-6 : h0 * 1e-3) : pow(0.01 / der, 1.0 / 5.0);
    double h = 100.0 * h0 < h1 ? 100.0 * h0 : h1;
    if (!(h <= hmax)) h = hmax;
    return h;
}

typedef struct {
    double t_final;
    int8_t status;
    int32_t n_acc, n_rej;
} orc_result;

/* Adaptive DP5(4) run of one trajectory.  With n_t == 0 it integrates to a
 * steady state or t_end; otherwise it clips steps onto every t_out[k] and
 * records x there (xs[k*N + i]).  x holds the initial state on entry and the
 * final state on exit. */
static orc_result orc_integrate_one(const orc_problem* pb, const orc_opts* o, int64_t p,
                                    double* x, const double* t_out, int32_t n_t, double* xs) {
    orc_result res = {o->t0, ORC_T_END, 0, 0};
    const int N = pb->n_genes;
    const int ts_mode = n_t > 0;
    const int use_steady = ts_mode ? o->stop_at_steady : 1;
    const double t_stop = ts_mode ? t_out[n_t - 1] : o->t_end;
    orc_stepper s;
    orc_stepper_init(&s, pb, o, p);
    double* f = (double*)calloc((size_t)N, sizeof(double));
    double t = o->t0;
    int kout = 0;
    orc_rhs(pb, p, o->divide_act_by_lambda, x, f);
    /* Record output times that coincide with the start. */
    while (ts_mode && kout < n_t && t_out[kout] <= t) {
        memcpy(xs + (int64_t)kout * N, x, sizeof(double) * (size_t)N);
        ++kout;
    }
    if (!orc_all_finite(x, N) || !orc_all_finite(f, N)) {
        res.status = ORC_NONFINITE;
        goto done;
    }
    if (use_steady && orc_is_steady(&s, x, f)) {
        res.status = ORC_CONVERGED;
        goto done;
    }
    if (t >= t_stop) {
        res.status = ORC_T_END;
        goto done;
    }
    double hmax = t_stop - o->t0;
    double h = o->h0 > 0 ? o->h0 : orc_initial_step(&s, x, f, hmax);
    if (h > hmax) h = hmax;
    int last_rejected = 0;
    for (;;) {
        if ((int64_t)res.n_acc + res.n_rej >= o->max_steps) { res.status = ORC_MAX_STEPS; break; }
        double tmag = fabs(t) > 1.0 ? fabs(t) : 1.0;
        if (h < 16.0 * DBL_EPSILON * tmag) { res.status = ORC_STEP_UNDERFLOW; break; }
        /* Land exactly on the next output time (time series) or on t_end. */
        double t_next = ts_mode ? t_out[kout] : t_stop;
        int clipped = 0;
        double hs = h;
        if (t + hs >= t_next) { hs = t_next - t; clipped = 1; }
        double err = orc_rk_attempt(&s, x, f, hs);
        int ok = isfinite(err) && err <= 1.0 && orc_all_finite(s.xn, N);
        if (ok) {
            res.n_acc++;
            t = clipped ? t_next : t + hs;
            memcpy(x, s.xn, sizeof(double) * (size_t)N);
            memcpy(f, s.k[6], sizeof(double) * (size_t)N);
            double fac = err > 0 ? 0.9 * pow(err, -1.0 / 5.0) : 10.0;
            double facmax = last_rejected ? 1.0 : 10.0;
            if (fac > facmax) fac = facmax;
            if (fac < 0.2) fac = 0.2;
            double hn = hs * fac;
            /* A step shortened only to hit an output time does not shrink h. */
            h = (clipped && hn < h) ? h : hn;
            last_rejected = 0;
            if (ts_mode) {
                while (kout < n_t && t_out[kout] <= t) {
                    memcpy(xs + (int64_t)kout * N, x, sizeof(double) * (size_t)N);
                    ++kout;
                }
            }
            if (use_steady && orc_is_steady(&s, x, f)) {
                res.status = ORC_CONVERGED;
                break;
            }
            if (t >= t_stop) { res.status = ORC_T_END; break; }
        } else {
            res.n_rej++;
            double fac = isfinite(err) ? 0.9 * pow(err, -1.0 / 5.0) : 0.2;
            if (fac < 0.2) fac = 0.2;
            if (fac > 1.0) fac = 1.0;
            h = hs * fac;
            last_rejected = 1;
        }
    }
done:
    /* Steady before the last output time: the remaining outputs hold x_ss. */
    while (ts_mode && kout < n_t) {
        memcpy(xs + (int64_t)kout * N, x, sizeof(double) * (size_t)N);
        ++kout;
    }
    res.t_final = t;
    free(f);
    orc_stepper_free(&s);
    return res;
}

/* Initial state of trajectory (p, c): fraction u of G/k, or an absolute value. */
static void orc_initial_state(const orc_problem* pb, const orc_opts* o, int64_t p, int64_t c,
                              double* x) {
    const int64_t P = pb->n_sets;
    for (int i = 0; i < pb->n_genes; ++i) {
        double u = (double)pb->ic[c * pb->n_genes + i];
        x[i] = o->ic_absolute ? u : u * (double)pb->G[i * P + p] / (double)pb->k[i * P + p];
    }
}

/* ------------------------------------------------------------------------ */
/* Thread pool driver.                                                       */
/* ------------------------------------------------------------------------ */
enum { ORC_JOB_STEADY, ORC_JOB_TS, ORC_JOB_RK4 };

typedef struct {
    int kind;
    const orc_problem* pb;
    const orc_opts* o;
    const int64_t* ids;
    int64_t n_traj;
    const double* t_out;
    int32_t n_t;
    double h_rk4;
    double* x_out;
    double* t_final;
    int8_t* status;
    int32_t* n_acc;
    int32_t* n_rej;
    int64_t next;
    pthread_mutex_t mu;
} orc_job;

static void orc_rk4_one(const orc_problem* pb, const orc_opts* o, int64_t p, double* x, double h,
                        const double* t_out, int32_t n_t, double* xs) {
    const int N = pb->n_genes;
    double* k1 = (double*)calloc((size_t)N, sizeof(double));
    double* k2 = (double*)calloc((size_t)N, sizeof(double));
    double* k3 = (double*)calloc((size_t)N, sizeof(double));
    double* k4 = (double*)calloc((size_t)N, sizeof(double));
    double* y = (double*)calloc((size_t)N, sizeof(double));
    double t = o->t0;
    for (int kk = 0; kk < n_t; ++kk) {
        while (t < t_out[kk]) {
            double hs = h;
            int clip = 0;
            if (t + hs >= t_out[kk]) { hs = t_out[kk] - t; clip = 1; }
            orc_rhs(pb, p, o->divide_act_by_lambda, x, k1);
            for (int i = 0; i < N; ++i) y[i] = x[i] + 0.5 * hs * k1[i];
            orc_rhs(pb, p, o->divide_act_by_lambda, y, k2);
            for (int i = 0; i < N; ++i) y[i] = x[i] + 0.5 * hs * k2[i];
            orc_rhs(pb, p, o->divide_act_by_lambda, y, k3);
            for (int i = 0; i < N; ++i) y[i] = x[i] + hs * k3[i];
            orc_rhs(pb, p, o->divide_act_by_lambda, y, k4);
            for (int i = 0; i < N; ++i) x[i] += hs / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
            t = clip ? t_out[kk] : t + hs;
        }
        memcpy(xs + (int64_t)kk * N, x, sizeof(double) * (size_t)N);
    }
    free(k1); free(k2); free(k3); free(k4); free(y);
}

static void orc_run_one(orc_job* jb, int64_t idx) {
    const orc_problem* pb = jb->pb;
    const int N = pb->n_genes;
    int64_t traj = jb->ids ? jb->ids[idx] : idx;
    int64_t p = traj / pb->n_ic, c = traj % pb->n_ic;
    double* x = (double*)calloc((size_t)N, sizeof(double));
    orc_initial_state(pb, jb->o, p, c, x);
    if (jb->kind == ORC_JOB_RK4) {
        orc_rk4_one(pb, jb->o, p, x, jb->h_rk4, jb->t_out, jb->n_t, jb->x_out + idx * jb->n_t * N);
    } else {
        orc_result r;
        if (jb->kind == ORC_JOB_STEADY) {
            r = orc_integrate_one(pb, jb->o, p, x, NULL, 0, NULL);
            memcpy(jb->x_out + idx * N, x, sizeof(double) * (size_t)N);
        } else {
            r = orc_integrate_one(pb, jb->o, p, x, jb->t_out, jb->n_t, jb->x_out + idx * jb->n_t * N);
        }
        if (jb->t_final) jb->t_final[idx] = r.t_final;
        if (jb->status) jb->status[idx] = r.status;
        if (jb->n_acc) jb->n_acc[idx] = r.n_acc;
        if (jb->n_rej) jb->n_rej[idx] = r.n_rej;
    }
    free(x);
}

static void* orc_worker(void* arg) {
    orc_job* jb = (orc_job*)arg;
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        int64_t i = jb->next;
        jb->next += 16;
        pthread_mutex_unlock(&jb->mu);
        if (i >= jb->n_traj) break;
        int64_t end = i + 16 < jb->n_traj ? i + 16 : jb->n_traj;
        for (; i < end; ++i) orc_run_one(jb, i);
    }
    return NULL;
}

static int orc_run_job(orc_job* jb, int32_t n_threads) {
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 512) n_threads = 512;
    jb->next = 0;
    pthread_mutex_init(&jb->mu, NULL);
    pthread_t th[512];
    int started = 0;
    for (int i = 1; i < n_threads; ++i)
        if (pthread_create(&th[started], NULL, orc_worker, jb) == 0) ++started;
    orc_worker(jb);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&jb->mu);
    return 0;
}

static int orc_check_problem(const orc_problem* pb) {
    if (!pb || pb->n_genes < 1 || pb->n_edges < 0 || pb->n_ic < 1 || pb->n_sets < 0) return -1;
    return 0;
}

static int orc_check_method(const orc_opts* o) {
    return (o->method == ORC_DP5 || o->method == ORC_TSIT5) ? 0 : -1;
}

int orc_steady_states(const orc_problem* pb, const orc_opts* o, const int64_t* traj_ids,
                      int64_t n_traj, int32_t n_threads, double* x_out, double* t_final,
                      int8_t* status, int32_t* n_acc, int32_t* n_rej) {
    if (orc_check_problem(pb) || orc_check_method(o)) return -1;
    orc_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.kind = ORC_JOB_STEADY; jb.pb = pb; jb.o = o; jb.ids = traj_ids;
    jb.n_traj = traj_ids ? n_traj : pb->n_sets * pb->n_ic;
    jb.x_out = x_out; jb.t_final = t_final; jb.status = status; jb.n_acc = n_acc; jb.n_rej = n_rej;
    return orc_run_job(&jb, n_threads);
}

static int orc_check_times(const orc_opts* o, const double* t_out, int32_t n_t) {
    if (n_t < 1 || !t_out) return -1;
    for (int i = 0; i < n_t; ++i) {
        if (t_out[i] < o->t0) return -1;
        if (i > 0 && !(t_out[i] > t_out[i - 1])) return -1;
    }
    return 0;
}

int orc_time_series(const orc_problem* pb, const orc_opts* o, const double* t_out, int32_t n_t,
                    const int64_t* traj_ids, int64_t n_traj, int32_t n_threads, double* x_out,
                    double* t_final, int8_t* status, int32_t* n_acc, int32_t* n_rej) {
    if (orc_check_problem(pb) || orc_check_method(o) || orc_check_times(o, t_out, n_t)) return -1;
    orc_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.kind = ORC_JOB_TS; jb.pb = pb; jb.o = o; jb.ids = traj_ids;
    jb.n_traj = traj_ids ? n_traj : pb->n_sets * pb->n_ic;
    jb.t_out = t_out; jb.n_t = n_t;
    jb.x_out = x_out; jb.t_final = t_final; jb.status = status; jb.n_acc = n_acc; jb.n_rej = n_rej;
    return orc_run_job(&jb, n_threads);
}

int orc_rk4(const orc_problem* pb, const orc_opts* o, double h, const double* t_out, int32_t n_t,
            const int64_t* traj_ids, int64_t n_traj, int32_t n_threads, double* x_out) {
    if (orc_check_problem(pb) || orc_check_times(o, t_out, n_t) || !(h > 0)) return -1;
    orc_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.kind = ORC_JOB_RK4; jb.pb = pb; jb.o = o; jb.ids = traj_ids;
    jb.n_traj = traj_ids ? n_traj : pb->n_sets * pb->n_ic;
    jb.t_out = t_out; jb.n_t = n_t; jb.h_rk4 = h; jb.x_out = x_out;
    return orc_run_job(&jb, n_threads);
}

int orc_dp5_fixed(const orc_problem* pb, const orc_opts* o, int64_t traj, int64_t n_steps,
                  double* x_out, double* err_last) {
    if (orc_check_problem(pb) || orc_check_method(o) || n_steps < 1) return -1;
    const int N = pb->n_genes;
    int64_t p = traj / pb->n_ic, c = traj % pb->n_ic;
    orc_stepper s;
    orc_stepper_init(&s, pb, o, p);
    double* x = (double*)calloc((size_t)N, sizeof(double));
    double* f = (double*)calloc((size_t)N, sizeof(double));
    orc_initial_state(pb, o, p, c, x);
    double h = (o->t_end - o->t0) / (double)n_steps;
    double err = 0.0;
    for (int64_t st = 0; st < n_steps; ++st) {
        orc_rhs(pb, p, o->divide_act_by_lambda, x, f);
        err = orc_rk_attempt(&s, x, f, h);
        memcpy(x, s.xn, sizeof(double) * (size_t)N);
    }
    memcpy(x_out, x, sizeof(double) * (size_t)N);
    if (err_last) *err_last = err;
    free(x); free(f);
    orc_stepper_free(&s);
    return 0;
}
