/*
 * rac.h -- C ABI of the MI355X RACIPE ensemble integrator.
 *
 * RACIPE (GRiNS, arXiv 2503.18356, Sec. 2.1) turns a signed directed gene
 * regulatory network into the ODE system of Eq. 1,
 *
 *   dx_i/dt = G_i * prod_{act e=(j->i)} H^S(x_j; T_e, n_e, lam_e) / lam_e
 *                 * prod_{inh e=(j->i)} H^S(x_j; T_e, n_e, lam_e)  -  k_i * x_i,
 *
 * with the shifted Hill function of Eq. 2,
 *
 *   H^S(B; B0, n, lam) = B0^n / (B0^n + B^n) + lam * B^n / (B0^n + B^n),
 *
 * samples 2N + 3E parameters per parameter set (Sec. 2.1.2, Table 1) and
 * integrates every (parameter set, initial condition) pair to a steady state
 * or to a list of output times (Sec. 2.1.3).  This library does the sampling
 * on the host and the integration on the GPU with hand-written HIP kernels:
 * an adaptive Dormand-Prince 5(4) stepper with per-trajectory step control.
 *
 * Conventions for every entry point:
 *   - Every call returns rac_status.  Argument errors are detected before any
 *     work is enqueued; rac_last_error() then returns a thread-local message.
 *   - Numerical failures of single trajectories are never return codes: they
 *     are reported per trajectory in rac_traj_info.status.
 *   - "dev" pointers are device memory owned by the caller (e.g. torch
 *     tensors); "host" pointers are host memory owned by the caller.  The
 *     library keeps no reference to caller memory after a call returns,
 *     except that enqueued kernels read and write the dev buffers until they
 *     complete on the given stream.
 *   - Integration calls are stream-ordered and asynchronous: they enqueue on
 *     hip_stream (a hipStream_t, NULL = the null stream) and return.  The
 *     caller synchronises the stream before reading results.
 *   - Trajectory id = p * n_ic + c for parameter set p and initial condition
 *     c (the initial condition index runs fastest), the paper's (parameter,
 *     initial condition) identifiers (Sec. 2.1.3).
 *   - Edges are held in canonical order, sorted by (dst, src).  Parameter
 *     arrays index edges in that order; rac_topology_edges() returns it.
 */
#ifndef RAC_H
#define RAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RAC_OK = 0,
    RAC_EINVAL = -1,       /* bad argument; nothing was enqueued */
    RAC_ENOMEM = -2,       /* host or device allocation failed */
    RAC_EDEVICE = -3,      /* a HIP call failed */
    RAC_EUNSUPPORTED = -4  /* valid input outside what the compiled kernels cover */
} rac_status;

/* Per-trajectory termination status. */
typedef enum {
    RAC_CONVERGED = 0,      /* steady-state test passed (at t0 or after a step) */
    RAC_T_END = 1,          /* reached t_end (or the last output time) */
    RAC_MAX_STEPS = 2,      /* more than max_steps attempted steps */
    RAC_STEP_UNDERFLOW = 3, /* step size fell below 16 * 2^-52 * max(|t|, 1) */
    RAC_NONFINITE = 4       /* initial state or its derivative not finite; in FP32
                               also a trajectory whose Hill-factor products FP32
                               cannot hold (lambdas far outside Table 1: a lane's
                               factors spanning over 2^250, or a production rate
                               they push out of the normal range), ended at t0
                               with x = NaN; FP64 solves it */
} rac_traj_status;

/* The paper's steady-state flag of a status (Sec. 2.1.3 and 3.1 report a flag
 * that is one when no steady state was reached): 0 for RAC_CONVERGED, 1 for
 * every other status. */
int32_t rac_not_steady_flag(int32_t status);

/* The same flag for n trajectories on the device: dev_flag[i] (u8) =
 * rac_not_steady_flag(dev_status[i]).  Stream-ordered and asynchronous;
 * EINVAL for n < 0 or a NULL array with n > 0. */
rac_status rac_steady_flags(const int8_t* dev_status, int64_t n, uint8_t* dev_flag, void* hip_stream);

typedef enum { RAC_FP32 = 0, RAC_FP64 = 1 } rac_precision;

/* Embedded Runge-Kutta 5(4) pair of the integrator.  RAC_DP5: Dormand-Prince
 * (Hairer, Norsett, Wanner I, Table 5.2).  RAC_TSIT5: Tsitouras (2011), the
 * solver the paper's library uses (Sec. 2.1.3). */
typedef enum { RAC_DP5 = 0, RAC_TSIT5 = 1 } rac_method;

/* Message for the last failing call on this thread ("" if none). */
const char* rac_last_error(void);

/* Library version string. */
const char* rac_version(void);

/* ------------------------------------------------------------------------ */
/* Topology (Sec. 2.1.1): signed directed network; sign +1 = activation,     */
/* -1 = inhibition.  Self-loops are allowed (Sec. 3.1, 3.2).                 */
/* ------------------------------------------------------------------------ */
typedef struct rac_topology rac_topology;

/* Copies the edge list (host arrays of length n_edges) and sorts it into
 * canonical (dst, src) order.  EINVAL: n_genes < 1, n_edges < 0, an index out
 * of [0, n_genes), a sign other than +-1, a duplicate (src, dst) pair, or a
 * NULL array with n_edges > 0.  EUNSUPPORTED: n_genes > 4096 or n_edges >
 * 32767.  The handle is immutable and safe to share across threads; device
 * copies of its lane plans are made lazily and cached in it.  Free it with
 * rac_destroy_topology. */
rac_status rac_create_topology(int32_t n_genes, int32_t n_edges, const int32_t* src,
                               const int32_t* dst, const int8_t* sign, rac_topology** out);

/* Frees the handle and its device copies.  The caller must ensure no enqueued
 * work still uses it.  NULL is a no-op. */
void rac_destroy_topology(rac_topology* topo);

/* Sizes of a topology. */
rac_status rac_topology_size(const rac_topology* topo, int32_t* n_genes, int32_t* n_edges);

/* Canonical edge order: host arrays of length n_edges (any may be NULL). */
rac_status rac_topology_edges(const rac_topology* topo, int32_t* src, int32_t* dst, int8_t* sign);

/* ------------------------------------------------------------------------ */
/* Sampling (Sec. 2.1.2, Table 1).                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    double g_min, g_max;          /* production rate G: Table 1 [1, 100] */
    double k_min, k_max;          /* degradation rate k: [0.1, 1] */
    double lam_act_min, lam_act_max; /* activating fold change: [1, 100] */
    double lam_inh_min, lam_inh_max; /* inhibiting fold change: [0.01, 1],
                                        sampled uniformly in the inverse range
                                        [1/max, 1/min] and inverted */
    int32_t n_min, n_max;         /* integer Hill coefficient: [1, 6] */
    double t_lo, t_hi;            /* threshold window: [0.02, 1.98] x median */
    double t_median;              /* > 0: fixed threshold scale of every edge;
                                     <= 0: follow threshold_rule */
    int32_t method;               /* unit-cube generator: RAC_SAMPLE_UNIFORM
                                     (default), RAC_SAMPLE_SOBOL, RAC_SAMPLE_LHS */
    int32_t threshold_rule;       /* RAC_THRESHOLD_PRIOR_MEDIAN (default) or
                                     RAC_THRESHOLD_HALF_FUNCTIONAL */
    int32_t hf_samples;           /* Monte Carlo draws per in-degree class of the
                                     half-functional rule (default 65536) */
    int32_t hf_act_over_lambda;   /* 1 (default): activating terms over lambda in
                                     that estimate, as in Eq. 1 */
    int64_t lhs_total;            /* sets in the Latin hypercube; 0 = set_begin +
                                     n_sets (a design over exactly this call) */
    int32_t n_continuous;         /* 0 (default): integer Hill coefficients,
                                     uniform over n_min..n_max, written to n
                                     (and to nf as floats when nf is given);
                                     1: real Hill coefficients, uniform on
                                     [n_min, n_max] (Table 1 gives the range
                                     without a type), written to nf only */
} rac_ranges;

/* Unit-cube generators (Sec. 2.1.2).  Parameter set p is point p of the
 * generator in 2N + 3E dimensions (slot order: G_i, k_i for i < N, then T_e,
 * n_e, lambda_e for each canonical edge); initial condition c is point c of a
 * second design in N dimensions.
 *  UNIFORM: Philox4x64-10 draws as described at rac_sample_params.
 *  SOBOL: a Sobol' sequence indexed directly by p (p < 2^32, at most 4096
 *   dimensions).  Dimension 0 is van der Corput; dimension q >= 1 takes the
 *   (q-1)-th primitive polynomial over GF(2) in order of degree, then value,
 *   with initial direction numbers m_k = 2 (w mod 2^(k-1)) + 1, w = word 0 of
 *   Philox at counter (q, k, 0, 0), key (0x536F626F6C2D6D6B, 0), and Bratley
 *   and Fox's recurrence after them; 32-bit points XOR a digital shift (the top
 *   half of word 0 of Philox at counter (q, 0, 2 + domain, 0), key (seed, 0);
 *   domain 0 parameters, 1 initial conditions), scaled by 2^-32.
 *  LHS: u = (perm_q(p) + v) / n with v a Philox draw at counter (p, q / 4,
 *   6 + domain, 0) and perm_q a bijection of [0, n): starting from p, apply
 *   four rounds of (xor key word r, multiply by 0x9E3779B97F4A7C15, xor with
 *   itself shifted right by max(1, w / 2)) on w-bit words (2^w >= n, keys = the Philox
 *   block at counter (q, 0, 4 + domain, 0), key (seed, 0)) until the value
 *   falls below n.  n = lhs_total for parameters and n_ic for initial
 *   conditions. */
typedef enum { RAC_SAMPLE_UNIFORM = 0, RAC_SAMPLE_SOBOL = 1, RAC_SAMPLE_LHS = 2 } rac_sample_method;

/* Threshold rules (Sec. 2.1.2).  PRIOR_MEDIAN: T_e = U[t_lo, t_hi] times the
 * prior median of G/k.  HALF_FUNCTIONAL: T_e = U[t_lo, t_hi] times the median
 * level of the edge's source gene given its in-degree (a activating, h
 * inhibitory regulators): unregulated sources use the prior median of G/k;
 * otherwise the level is estimated one step deep, x = (G/k) times the
 * product over its in-edges of H^S(B; T, n, lambda) (over lambda for
 * activation when hf_act_over_lambda), with B = G'/k' an unregulated level
 * and T, n, lambda from their priors (T with the prior median), by
 * hf_samples Monte Carlo draws (Philox counter (a, h, s, d / 4), key
 * (0x48616C662D66756E, 0), word d % 4, draws in the order G, k, then per
 * in-edge G', k', T, n, lambda, activating in-edges first); the median of the
 * draws rounded to FP32. */
typedef enum { RAC_THRESHOLD_PRIOR_MEDIAN = 0, RAC_THRESHOLD_HALF_FUNCTIONAL = 1 } rac_threshold_rule;

/* Table 1 defaults. */
void rac_default_ranges(rac_ranges* r);

/* Caller-owned parameter arrays, set index fastest (SoA), stride n_sets:
 *   G[i * n_sets + p], k[i * n_sets + p]            for genes i < N,
 *   T[e * n_sets + p], lam[e * n_sets + p], n[...]  for canonical edges e < E.
 * lam is the fold change of Table 1 (activation >= 1, inhibition <= 1).  n is
 * the integer Hill coefficient (u8); nf, when not NULL, holds real Hill
 * coefficients (f32, > 0, same layout) and is used instead of n, which may
 * then be NULL (Eq. 2 with a non-integer exponent).  The same struct
 * describes host arrays (rac_sample_params) and device arrays (integration
 * calls). */
typedef struct {
    float* G;
    float* k;
    float* T;
    float* lam;
    uint8_t* n;
    int64_t n_sets;
    float* nf;
} rac_params_view;

/* Deterministic, index-addressable sampling on the host: set p depends only
 * on (seed, p), so sets [set_begin, set_begin + n_sets) come out the same
 * whatever the batch.  Each parameter is drawn from Philox4x64-10 (Salmon et
 * al. 2011; counter (p, slot / 4, 0, 0), key (seed, 0), word slot % 4, top 53
 * bits scaled to [0, 1); slots G_i = i, k_i = N + i, T_e = 2N + 3e,
 * n_e = 2N + 3e + 1, lam_e = 2N + 3e + 2), mapped to its range in FP64 and
 * rounded to FP32.  Thresholds are uniform in [t_lo, t_hi] times the median
 * of G/k (the half-functional window of Sec. 2.1.2 with the prior median).
 * Initial-condition fractions ic_frac[c * N + i] (host, may be NULL) in
 * [0, 1) use counter (c, i / 4, 1, 0): they are shared by all parameter sets
 * (Sec. 3.1).  out->n_sets must equal n_sets.  ranges NULL = Table 1 with
 * uniform draws and the prior-median threshold rule; other generators and the
 * half-functional rule are chosen in the ranges.
 * EINVAL: NULL arrays, n_sets < 0, n_ic < 0, inverted/non-positive ranges,
 * unknown method or rule, hf_samples < 1, lhs_total below set_begin + n_sets.
 * EUNSUPPORTED: Sobol' beyond 4096 dimensions or 2^32 points. */
rac_status rac_sample_params(const rac_topology* topo, const rac_ranges* ranges, uint64_t seed,
                             int64_t set_begin, int64_t n_sets, int32_t n_ic,
                             rac_params_view* out, float* ic_frac);

/* The same sampling on the GPU, bit-identical to rac_sample_params: dev_out
 * and dev_ic_frac (may be NULL) are device arrays; the work is enqueued on
 * hip_stream (asynchronous).  Argument errors as rac_sample_params. */
rac_status rac_sample_params_device(const rac_topology* topo, const rac_ranges* ranges,
                                    uint64_t seed, int64_t set_begin, int64_t n_sets,
                                    int32_t n_ic, rac_params_view* dev_out, float* dev_ic_frac,
                                    void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Integration (Sec. 2.1.3).                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double t0;          /* start time (default 0) */
    double t_end;       /* hard stop even if not steady (default 200) */
    double rtol, atol;  /* error control (defaults 1e-6, 1e-9) */
    double ss_atol;     /* steady when every |dx_i/dt| <= ss_atol + ss_rtol * k_i * |x_i| */
    double ss_rtol;     /* default 0 for FP64, 1e-5 for FP32 (FP32 rounding floor of f) */
    double h0;          /* first step; <= 0 picks it automatically */
    int64_t max_steps;  /* attempted steps per trajectory (default 100000) */
    int32_t precision;  /* RAC_FP32: FP32 state and right-hand side, FP64 time,
                           error norm and steady test.  RAC_FP64: all FP64. */
    int32_t activation_divides_by_lambda; /* 1 (default) = Eq. 1 as printed */
    int32_t stop_at_steady; /* time series only: stop once steady and fill the
                               remaining output times with x_ss (default 0) */
    int32_t ic_absolute;    /* 1: ic holds absolute levels instead of fractions
                               of G_i/k_i, e.g. to pin input nodes (Sec. 3.2) */
    int32_t lanes_per_traj; /* 0 = automatic; else 1, 2, 4, ..., 64 */
    int32_t refill_min;     /* 0 = automatic: a wave pulls new trajectories from
                               the work queue once this many of its trajectory
                               groups are free (each refill costs the wave two
                               right-hand sides); always 1 near the queue end */
    int32_t method;         /* RAC_DP5 (default) or RAC_TSIT5.  Both use the same
                               step control; time series interpolate inside a step
                               with a continuous extension of order 4 (DP5: Hairer,
                               Norsett, Wanner I, Sec. II.6; Tsit5: quartic weights
                               solving the order conditions, C1 at both ends) */
} rac_solver_opts;

/* Defaults for a precision. */
void rac_default_opts(rac_solver_opts* o, int32_t precision);

/* Per-trajectory outputs, device arrays of length P * n_ic (any may be NULL). */
typedef struct {
    double* t_final;     /* time at termination */
    int8_t* status;      /* rac_traj_status */
    int32_t* n_accepted; /* accepted steps */
    int32_t* n_rejected; /* rejected steps */
} rac_traj_info;

/* Integrates all P * n_ic trajectories (P = dev_params->n_sets) from
 * x0_i = ic[c][i] * G_i / k_i (or ic[c][i] with ic_absolute) to a steady state
 * or t_end.  dev_ic: device [n_ic][N] f32.  dev_x_out: device
 * [P * n_ic][N], f32 for RAC_FP32 and f64 for RAC_FP64.  A single combination
 * (Sec. 2.1.3) is P = n_ic = 1.  P * n_ic = 0 enqueues nothing.
 * EINVAL: NULL handle/opts/arrays, n_ic < 1, t_end <= t0, rtol < 0, atol < 0,
 * rtol + atol == 0, ss_atol < 0, max_steps < 1, bad precision.
 * EUNSUPPORTED: the network does not fit the compiled lane plans. */
rac_status rac_steady_states(const rac_topology* topo, const rac_params_view* dev_params,
                             const float* dev_ic, int32_t n_ic, const rac_solver_opts* opts,
                             void* dev_x_out, const rac_traj_info* dev_info, void* hip_stream);

/* rac_steady_states for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, bit for bit, but no
 * device allocation or free.  The work-queue counters (one per XCD) and the
 * network descriptor live in a library-owned device scratch array of 4096
 * bytes per GPU (the counters and one descriptor: one network per call), kept
 * until the process
 * ends and cleared by a kernel at the start of every call.  Calls that
 * overlap on one GPU (concurrent streams or threads) share that scratch and
 * race: order them on one stream.  The network's lane plan for the lane count
 * the options select must already be on the current device, which any
 * earlier rac_steady_states call with the same options leaves there.  Kernel
 * shapes that keep a few registers in per-lane scratch (the four-wave
 * (10, 4) shape) use the HIP runtime's private segment for them, which the
 * runtime provides at dispatch; this call allocates nothing itself.
 * EINVAL as rac_steady_states, and when the lane plan is not on the device;
 * EUNSUPPORTED as rac_steady_states; EDEVICE if the scratch address cannot be
 * found. */
rac_status rac_steady_states_noalloc(const rac_topology* topo, const rac_params_view* dev_params,
                                     const float* dev_ic, int32_t n_ic, const rac_solver_opts* opts,
                                     void* dev_x_out, const rac_traj_info* dev_info, void* hip_stream);

/* Time series at host_t_out[0..n_t) (strictly increasing, >= t0; Sec. 2.1.3):
 * integrates to the last output time; each output is the DP5 continuous
 * extension (Hairer, Norsett, Wanner I, Sec. II.6) at that time.
 * dev_x_out: device [P * n_ic][n_t][N] (f32 or f64 by precision).  opts->t_end
 * is ignored.  Status T_END means the last output time was reached.
 * EINVAL as rac_steady_states, plus n_t < 1 or unordered / early times. */
rac_status rac_integrate(const rac_topology* topo, const rac_params_view* dev_params,
                         const float* dev_ic, int32_t n_ic, const rac_solver_opts* opts,
                         const double* host_t_out, int32_t n_t, void* dev_x_out,
                         const rac_traj_info* dev_info, void* hip_stream);

/* One work item of a fused multi-network launch. */
typedef struct {
    const rac_topology* topo;
    rac_params_view params;  /* device arrays */
    const float* ic;         /* device [n_ic][N] */
    int32_t n_ic;
    void* x_out;             /* device [P * n_ic][N] */
    rac_traj_info info;      /* device arrays */
    int32_t lanes_per_traj;  /* 0: as opts; else this network's lane count
                                (a power of two <= 64, e.g. an autotuner's) */
    int32_t refill_min;      /* 0: as opts; else the refill batch of the launch
                                that takes this network (the largest asked by
                                the networks sharing a launch) */
} rac_batch_item;

/* Steady states of several networks of uneven size in persistent launches
 * that pull trajectories from one device work queue (networks sharing a lane
 * count and kernel shape go into the same launch; lanes freed by converged
 * trajectories are refilled from the queue; launches overlap on side streams
 * forked from and joined into hip_stream).  Results per item are as
 * rac_steady_states with the same opts and the item's lane count.  EINVAL as
 * rac_steady_states for any item, or a lane count that is not 0 or a power
 * of two <= 64, or refill_min < 0. */
rac_status rac_steady_states_batch(const rac_batch_item* items, int32_t n_items,
                                   const rac_solver_opts* opts, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Serving step batches (continuous batching of simulation requests).        */
/* ------------------------------------------------------------------------ */
/* A server owns a device work queue, a table of admitted requests and a slot
 * table holding the state of in-flight trajectories between batches.  Each
 * rac_server_step enqueues one step batch: a persistent launch of the
 * bounded DP5 kernel (RAC_FP32, lanes_per_traj lanes per trajectory, kernel
 * shape (epl, gpl)) that resumes the parked trajectories, pulls new ones
 * from the queue as lanes free up, runs at most batch_steps loop iterations
 * per wave and parks what is unfinished.  The launch has fixed arguments
 * and is captured into a hipGraph on the first call and replayed after.
 * Requests submitted while others are in flight join the queue and share
 * the same launches; each trajectory's result is the same as from
 * rac_steady_states with the same opts and lane count.
 * Ownership: the server owns its device memory (request table of
 * max_requests entries, slot table sized for one full grid); submitted
 * arrays stay caller-owned and must stay valid until the request's done
 * count reaches P * n_ic.  One server is used from one stream at a time:
 * submits and step batches must be ordered on it (a batch's last graph node
 * resets a queue head that the batch left past the tail). */
typedef struct rac_server rac_server;

/* EINVAL: bad opts, lanes_per_traj < 1, max_requests < 1, batch_steps < 1.
 * EUNSUPPORTED: precision other than RAC_FP32, method other than RAC_DP5, or
 * no compiled (epl, gpl).
 * ENOMEM: device allocation failed. */
rac_status rac_server_create(const rac_solver_opts* opts, int32_t epl, int32_t gpl,
                             int32_t max_requests, int32_t batch_steps, rac_server** out);
void rac_server_destroy(rac_server* s);

/* Admit a request (arguments as rac_steady_states); enqueues two small
 * uploads on hip_stream and returns its id (0, 1, ...).  EUNSUPPORTED if the
 * network's lane plan does not fit the server's shape; ENOMEM if the request
 * table is full. */
rac_status rac_server_submit(rac_server* s, const rac_topology* topo,
                             const rac_params_view* dev_params, const float* dev_ic,
                             int32_t n_ic, void* dev_x_out, const rac_traj_info* dev_info,
                             void* hip_stream, int32_t* request_id);

/* Enqueue one step batch on hip_stream (graph replay).  EINVAL for the null
 * stream, which cannot be captured. */
rac_status rac_server_step(rac_server* s, void* hip_stream);

/* Enqueue a copy of the finished-trajectory counts of requests
 * [first, first + count) into host_out (host); valid after the stream syncs. */
rac_status rac_server_done_counts(rac_server* s, int32_t first, int32_t count, int32_t* host_out,
                                  void* hip_stream);

/* Submitted requests, queued trajectories in total, waves per step batch and
 * slot-table bytes (any pointer may be NULL). */
rac_status rac_server_info(const rac_server* s, int32_t* n_requests, int64_t* total_trajectories,
                           int32_t* grid_waves, int64_t* slot_bytes);

/* ------------------------------------------------------------------------ */
/* Post-processing of results (the analysis functions of Sec. 2.1.4 and their */
/* use in Sec. 3.1), on the device.                                           */
/* ------------------------------------------------------------------------ */
/* A row is one state vector of N genes: row r = p * n_ic + c of a steady-state
 * result, or (p * n_ic + c) * n_t + j of a time series.  All arrays are
 * caller-owned device memory; every call is stream-ordered and asynchronous
 * and returns argument errors before enqueueing anything. */
#define RAC_NO_STATE 0xFFFFFFFFFFFFFFFFull /* state code of an excluded row */

/* G/k normalisation: y[r][i] = (x[r][i] * k_i) / G_i of the row's parameter
 * set, each operation rounded to FP32, so that 1 is the gene's maximal level
 * (Sec. 2.1.4).  x and y are [P * n_ic * n_t][N] f32 (y may be x).
 * EINVAL: NULL pointers, n_ic < 1, n_t < 1. */
rac_status rac_normalize(const rac_topology* topo, const rac_params_view* dev_params, int32_t n_ic,
                         int32_t n_t, const float* dev_x, float* dev_y, void* hip_stream);

/* Level thresholds from the global distribution of normalised values
 * (Sec. 2.1.4; the paper does not state the method, this is the library's
 * reading).  Bins: b = min(floor(clamp(y, 0, 1) * n_bins), n_bins - 1) in FP32
 * (NaN counts as 0); dev_hist[n_bins] (u64) receives the counts over all
 * genes of the rows whose dev_status is RAC_CONVERGED (all rows if
 * dev_status is NULL).  dev_thresholds[n_levels - 1] receives the bin indices
 * 0 < t_1 < ... < t_{L-1} < n_bins maximising sum_k S_k^2 / W_k over the
 * classes [t_k, t_{k+1}) (W = count, S = sum of bin indices; Otsu's
 * between-class variance up to constants), evaluated in FP64 in class order;
 * the lexicographically first maximum wins.  EINVAL: n_bins outside
 * [2, 1024], n_levels outside [2, 4], NULL pointers.  EUNSUPPORTED: four
 * levels with n_bins > 256. */
rac_status rac_level_thresholds(const float* dev_y, int64_t n_rows, int32_t n_genes,
                                const int8_t* dev_status, int32_t n_bins, int32_t n_levels,
                                uint64_t* dev_hist, int32_t* dev_thresholds, void* hip_stream);

/* Levels and state codes: level = number of thresholds <= the value's bin;
 * dev_levels[n_rows][N] (u8, 255 for excluded rows; may be NULL) and
 * dev_codes[n_rows] = sum_i level_i * n_levels^(N-1-i), gene 0 most
 * significant (the concatenated levels of Sec. 3.1; RAC_NO_STATE for rows
 * whose status is not RAC_CONVERGED; may be NULL).  EUNSUPPORTED when codes
 * are asked for and n_levels^N exceeds 64 bits. */
rac_status rac_discretize(const float* dev_y, int64_t n_rows, int32_t n_genes,
                          const int8_t* dev_status, int32_t n_bins, int32_t n_levels,
                          const int32_t* dev_thresholds, uint8_t* dev_levels, uint64_t* dev_codes,
                          void* hip_stream);

/* Multistability of each parameter set (Sec. 3.1): the number of distinct
 * states over its n_ic initial conditions (RAC_NO_STATE rows excluded) in
 * dev_n_states[n_sets] (i32), and those states in ascending order in
 * dev_states[n_sets][n_ic] (u64), padded with RAC_NO_STATE.  Input codes are
 * [n_sets][n_ic].  EUNSUPPORTED: n_ic > 4096. */
rac_status rac_multistability(const uint64_t* dev_codes, int64_t n_sets, int32_t n_ic,
                              int32_t* dev_n_states, uint64_t* dev_states, void* hip_stream);

/* State frequencies over all rows (Sec. 3.1): the distinct codes in ascending
 * order in dev_keys[capacity] with their counts in dev_counts[capacity]
 * (unused entries RAC_NO_STATE / 0), and their number in *dev_n_unique, or -1
 * when more than `capacity` distinct states occur (a hash table of that many
 * slots; the library allocates it stream-ordered).  EINVAL: capacity not a
 * power of two in [2, 2^30], NULL pointers. */
rac_status rac_state_counts(const uint64_t* dev_codes, int64_t n_rows, int64_t capacity,
                            uint64_t* dev_keys, int64_t* dev_counts, int64_t* dev_n_unique,
                            void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Boolean Ising formalism (Eq. 3).                                           */
/* ------------------------------------------------------------------------ */
/* Gene i's next state is on when sum_j J_ij s_j > 0, off when < 0 and
 * unchanged when 0, with J_ij = +1 for an activating edge j -> i, -1 for an
 * inhibiting one; an off gene counts as `low` (0 or -1) in the sums.
 * States are bit-packed, [n_traj][W] u64 with W = ceil(N / 64) and gene i in
 * bit i % 64 of word i / 64 (N <= 256).
 *  SYNC: every gene updates at once; a trajectory stops at the first state
 *   that maps to itself (steps = updates done) or after max_steps updates.
 *   A trajectory that revisits a state is periodic; the library then steps
 *   only the remainder of the updates left modulo the period, so its final
 *   state, steps and status are those of max_steps updates (Brent's cycle
 *   detection; dev_evals counts the updates actually done).
 *  ASYNC: one gene per update, cycled from `order` (host array of order_len
 *   gene indices) or chosen at random: update u of trajectory t takes the
 *   low (u even) or high (u odd) 32-bit half h of word (u % 8) / 2 of Philox
 *   at counter (t, u / 8, 8, 0), key (seed, 0), and picks gene (h N) >> 32.
 *   The state is tested for being a fixed point of the synchronous map at
 *   the start and every check_every updates (0: N); the first pass stops it.
 * Without dev_init, gene i of trajectory t starts on when the top bit of word
 * i % 4 of Philox at counter (t, i / 4, 9, 0), key (seed, 0) is set.
 * Outputs: dev_final[n_traj][W]; dev_steps[n_traj] (i32) and dev_status
 * [n_traj] (i8: 0 fixed point reached, 1 max_steps) may be NULL.
 * EINVAL: bad mode or low, negative counts, order entries outside [0, N),
 * NULL outputs.  EUNSUPPORTED: N > 256. */
typedef enum { RAC_ISING_SYNC = 0, RAC_ISING_ASYNC = 1 } rac_ising_mode;

typedef struct {
    int32_t mode;           /* RAC_ISING_SYNC (default) or RAC_ISING_ASYNC */
    int32_t low;            /* value of an off gene in the sums: 0 (default) or -1 */
    int32_t max_steps;      /* updates per trajectory (default 1000) */
    int32_t check_every;    /* asynchronous fixed-point test interval; 0 = N */
    uint64_t seed;          /* random gene choices and random initial states */
    const int32_t* order;   /* asynchronous update order (host), or NULL */
    int32_t order_len;
    unsigned long long* dev_evals; /* optional device counter, or NULL: the gene
                               evaluations the call performs are added to it
                               (stream-ordered; the caller zeroes it) */
} rac_ising_opts;

void rac_default_ising_opts(rac_ising_opts* o);

rac_status rac_ising(const rac_topology* topo, const rac_ising_opts* opts, int64_t n_traj,
                     const uint64_t* dev_init, uint64_t* dev_final, int32_t* dev_steps,
                     int8_t* dev_status, void* hip_stream);

/* The lanes-per-trajectory choice the library would make for a network
 * (0 if none fits), and whether a given choice fits the compiled kernels.
 * rac_auto_lanes is the cost model's choice for a call that fills the GPU;
 * rac_auto_lanes_for is what a call of n_traj trajectories in all (every
 * network of a batch call) takes when its options give no lane count: the
 * same, unless the call is too small to fill the GPU at that choice, then
 * more lanes per trajectory (shorter trajectories, more issue work). */
int32_t rac_auto_lanes(const rac_topology* topo, int32_t precision);
int32_t rac_auto_lanes_for(const rac_topology* topo, int32_t precision, int64_t n_traj);
int32_t rac_lanes_supported(const rac_topology* topo, int32_t precision, int32_t lanes);

/* The compiled kernel shape (edge slots, gene slots per lane) a network uses
 * at a lane count.  EUNSUPPORTED if none fits. */
rac_status rac_plan_shape(const rac_topology* topo, int32_t precision, int32_t lanes, int32_t* epl,
                          int32_t* gpl);

/* Measurement support, not part of the method: the sustained lane-operation
 * rates (operations per second summed over all lanes) of the current device
 * for, in this order, FP32 FMA with register operands (v_fma_f32),
 * v_exp_f32, v_log_f32, v_rcp_f32, FP64 FMA and FP32 FMA with a literal
 * multiplier (v_fmamk_f32), written to lane_ops_per_s[0..min(n, 6)) (entries
 * past 6 are set to 0).  Synchronous: allocates a scratch buffer and a
 * stream of its own, runs six short kernels compiled like the solver kernels
 * (no packed FP32), and returns when they are timed.  EINVAL for a NULL
 * pointer or n < 1; EDEVICE or ENOMEM when the device calls fail. */
rac_status rac_valu_ceilings(double* lane_ops_per_s, int32_t n);

/* Which algebraic form of the Hill factor (Eq. 2) kernels of a precision and
 * edge-slot count use: 1 for 1 + D / (1 + 2^z) with D >= 0 and the constant
 * lam (inhibition) or 1/lam (activation over lambda) folded into the
 * production rate, 0 for sqrt(lam) + (1/sqrt(lam) - sqrt(lam)) / (1 + r).
 * Both are Eq. 2 rearranged; kernels of the same form and lane count give
 * bit-identical results whatever their slot counts, kernels of different
 * forms agree to rounding.  -1 for a bad precision or epl < 1. */
int32_t rac_factor_form(int32_t precision, int32_t epl);

#ifdef __cplusplus
}
#endif
#endif
