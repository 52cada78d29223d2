/*
 * RACIPE CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 reference for what the GPU path computes.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * What it implements (GRiNS paper, arXiv 2503.18356):
 *   - the RACIPE node ODE (Eq. 1) with the shifted Hill function (Eq. 2),
 *     evaluated literally with pow();
 *   - parameter and initial-condition sampling with the default ranges of
 *     Table 1, the inverted inhibitory fold change (Sec. 2.1.2) and the
 *     threshold window 0.02..1.98 x median of the source's G/k (Sec. 2.1.2,
 *     simplified to the prior median of G/k);
 *   - an adaptive Dormand-Prince 5(4) integrator run to a steady state or to
 *     a list of output times (Sec. 2.1.3), fixed-step RK4 and fixed-step DP5
 *     for cross-checks;
 *   - Philox4x64-10 (Salmon et al., SC'11) as the counter-based generator.
 *
 * Parameter layout is set-index fastest: G[i*P + p], T[e*P + p], ...
 * Edges are in canonical order, sorted by (dst, src).
 */
#ifndef RACIPE_ORACLE_H
#define RACIPE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x64 with 10 rounds. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Sort an edge list into canonical (dst, src) order.  Returns 0, or -1 on a
 * bad index / duplicate edge / bad sign. */
int orc_canonicalize(int n_genes, int n_edges, const int32_t* src, const int32_t* dst,
                     const int8_t* sign, int32_t* out_src, int32_t* out_dst, int8_t* out_sign);

/* Sampling configuration: Table 1 ranges, the threshold rule and the
 * generator of the unit-cube points (Sec. 2.1.2).  t_median > 0 fixes the
 * threshold scale of every edge; otherwise it follows threshold_rule. */
typedef struct {
    double g_min, g_max, k_min, k_max;
    double lam_act_min, lam_act_max, lam_inh_min, lam_inh_max;
    int32_t n_min, n_max;
    double t_lo, t_hi, t_median;
    int32_t method;          /* ORC_UNIFORM, ORC_SOBOL or ORC_LHS */
    int32_t threshold_rule;  /* ORC_T_PRIOR_MEDIAN or ORC_T_HALF_FUNCTIONAL */
    int32_t hf_samples;      /* Monte Carlo samples per in-degree class (> 0) */
    int32_t hf_act_over_lambda; /* activating terms over lambda in the estimate */
    int64_t lhs_total;       /* sets in the Latin hypercube (0: set_begin + n_sets) */
    int32_t n_continuous;    /* 1: real Hill coefficients, uniform on [n_min, n_max] */
} orc_ranges;

enum { ORC_UNIFORM = 0, ORC_SOBOL = 1, ORC_LHS = 2 };
enum { ORC_T_PRIOR_MEDIAN = 0, ORC_T_HALF_FUNCTIONAL = 1 };

/* Threshold scale of edges leaving a gene with n_act activating and n_inh
 * inhibitory regulators under the half-functional rule (its median level). */
double orc_hf_median(const orc_ranges* r, int32_t n_act, int32_t n_inh);

/* The q-th coordinate of Sobol' point i before any shift, as a 32-bit
 * fraction (dimension 0 is van der Corput).  Returns -1 beyond the supported
 * dimensions. */
int orc_sobol_u32(int64_t i, int32_t q, uint32_t* out);

/* Number of primitive polynomials of degree s found by the enumeration. */
int orc_primitive_count(int32_t s);

/* The Latin-hypercube permutation of dimension q over n items. */
int64_t orc_lhs_perm(uint64_t seed, int32_t domain, int32_t q, int64_t n, int64_t i);

void orc_default_ranges(orc_ranges* r);
double orc_gk_median(const orc_ranges* r);

/* Sample sets [set_begin, set_begin+n_sets) into arrays of stride n_sets, and
 * n_ic initial-condition fractions ic[c*N + i] (ic may be NULL).  Integer Hill
 * coefficients go to n (required) and, when nf is not NULL, also to nf as
 * floats; with r->n_continuous they are real, uniform on [n_min, n_max] (the
 * same draw), go to nf (required) and n is not written. */
int orc_sample(int n_genes, int n_edges, const int32_t* src_canon, const int32_t* dst_canon,
               const int8_t* sign_canon, const orc_ranges* r,
               uint64_t seed, int64_t set_begin, int64_t n_sets, int32_t n_ic,
               float* G, float* k, float* T, float* lam, uint8_t* n, float* ic, float* nf);

typedef struct {
    double t0, t_end, rtol, atol, ss_atol, ss_rtol, h0;
    int64_t max_steps;
    int32_t divide_act_by_lambda; /* 1 = Eq. 1 as printed */
    int32_t stop_at_steady;       /* time-series mode only */
    int32_t ic_absolute;          /* ic holds absolute values, not fractions of G/k */
    int32_t method;               /* ORC_DP5 or ORC_TSIT5 */
} orc_opts;

/* Embedded explicit Runge-Kutta 5(4) pairs with 7 stages, first same as last. */
enum { ORC_DP5 = 0, ORC_TSIT5 = 1 };

/* The tableau of a method: a[7*7] (row i holds the weights of k_1..k_i in the
 * input of stage i+1), b[7] fifth-order weights, bh[7] fourth-order
 * weights, c[7] nodes.  Returns -1 for an unknown method. */
int orc_tableau(int32_t method, double* a, double* b, double* bh, double* c);

void orc_default_opts(orc_opts* o);

/* A network with its parameters.  src/dst/sign are canonical. */
typedef struct {
    int32_t n_genes, n_edges;
    const int32_t* src;
    const int32_t* dst;
    const int8_t* sign;
    const float* G;
    const float* k;
    const float* T;
    const float* lam;
    const uint8_t* n;
    int64_t n_sets; /* stride of the parameter arrays */
    const float* ic;
    int32_t n_ic;
    const float* nf; /* real Hill coefficients [E][P], used instead of n when not NULL */
} orc_problem;

enum { ORC_CONVERGED = 0, ORC_T_END = 1, ORC_MAX_STEPS = 2, ORC_STEP_UNDERFLOW = 3, ORC_NONFINITE = 4 };

/* Right-hand side of Eq. 1 for parameter set p at state x. */
void orc_rhs(const orc_problem* pb, int64_t p, int32_t divide, const double* x, double* f);

/* Steady-state solve of the trajectories traj_ids[0..n_traj) (traj = p*n_ic + c);
 * traj_ids NULL means all P*n_ic.  x_out[n_traj][N]. */
int orc_steady_states(const orc_problem* pb, const orc_opts* o, const int64_t* traj_ids,
                      int64_t n_traj, int32_t n_threads, double* x_out, double* t_final,
                      int8_t* status, int32_t* n_acc, int32_t* n_rej);

/* Time series at t_out[0..n_t), step-clipped so each t_k is hit exactly.
 * x_out[n_traj][n_t][N]. */
int orc_time_series(const orc_problem* pb, const orc_opts* o, const double* t_out, int32_t n_t,
                    const int64_t* traj_ids, int64_t n_traj, int32_t n_threads, double* x_out,
                    double* t_final, int8_t* status, int32_t* n_acc, int32_t* n_rej);

/* Fixed-step classical RK4 to every t_k (steps clipped at each t_k). */
int orc_rk4(const orc_problem* pb, const orc_opts* o, double h, const double* t_out, int32_t n_t,
            const int64_t* traj_ids, int64_t n_traj, int32_t n_threads, double* x_out);

/* Fixed-step run of o->method (no control) from t0 to t_end with n_steps
 * equal steps, for one trajectory; also returns the embedded error estimate
 * of the last step. */
int orc_dp5_fixed(const orc_problem* pb, const orc_opts* o, int64_t traj, int64_t n_steps,
                  double* x_out, double* err_last);

#ifdef __cplusplus
}
#endif
#endif
