// Device-side structures and the persistent Dormand-Prince 5(4) kernel body.
//
// Mapping (CDNA4, wave64): a wave holds 64 / L trajectory groups of L lanes.
// Each lane owns ceil(N / L) genes (their DP5 state lives in its VGPRs) and a
// balanced set of whole in-edge rows (their per-trajectory edge parameters
// live in its VGPRs).  One right-hand-side evaluation is
//   1. owners publish their level max(y_i, 0) (FP32: its log2) to LDS,
//   2. every lane walks its edge slots: read the source level from LDS,
//      evaluate the shifted Hill factor, keep a running product in LDS,
//   3. owners read prefix[end] / prefix[begin] of their row and form
//      f_i = G_i' * P_i - k_i * y_i.
// Step control, the error norm and the steady test are per group; groups
// that finish are refilled from a device work queue (each wave claims chunks
// of queue indices with one atomic per chunk).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rac.h"
#include "rac_internal.h"

namespace rac {

struct NetDesc {
    const int32_t* lane_edge;  // [lpt][stride] packed (edge | activating << 15 | src << 16), -1 empty
    const int32_t* gene_row;   // [N] packed row lane | begin << 8 | end << 16
    const int32_t* row_ptr;    // [N + 1]
    const int8_t* sign;        // [E]
    const float* G;
    const float* k;
    const float* T;
    const float* lam;
    const uint8_t* n;
    const float* nf;           // real Hill coefficients [E][P], or nullptr: use n
    const float* ic;           // [n_ic][N]
    void* x_out;
    double* t_final;
    int8_t* status;
    int32_t* n_acc;
    int32_t* n_rej;
    int32_t* done;             // finished-trajectory counter (serving), or nullptr
    int64_t n_sets;            // parameter array stride P
    int64_t traj_begin;        // first queue index of this network
    int64_t n_traj;            // P * n_ic
    double inv_n_ic;           // 1 / n_ic
    int32_t n_genes, n_edges, n_ic, stride;
};

struct Controls {
    double t0, t_end, rtol, atol, ss_atol, ss_rtol, h0;
    int64_t max_steps;
    int32_t divide, ic_absolute, stop_at_steady, refill_min;
    int32_t chunk;  // queue indices a wave claims per pop while the queue is long
    int32_t pad;
};

// Device-resident queue control of a serving step batch: the kernel pops
// [head, total); the host appends work by raising total and n_nets between
// batches and never writes head.
struct ServeCtl {
    unsigned long long head;
    unsigned long long total;
    int32_t n_nets;
    int32_t pad;
};

struct LaunchArgs {
    // Device array of the launch's networks, also for a single one: the
    // kernel reads descriptors from memory on its rare paths (trajectory
    // start and end) instead of holding them in scalar registers.
    const NetDesc* nets;
    int32_t n_nets;
    int64_t total;        // trajectories over all networks
    unsigned long long* counter;  // kSubQueues counters (serving: one, the queue head)
    int32_t lpt, epl, gpl;  // lanes per trajectory; runtime slot bounds
    const double* t_out;    // device, time-series mode
    int32_t n_t;
    Controls c;
    // Serving step batches only.
    ServeCtl* ctl;          // queue control in device memory
    char* slots;            // per-wave saved trajectory state
    int32_t batch_steps;    // loop iterations per launch
};

constexpr int kBlock = 256;  // 4 independent waves per block

// Persistent launches split their work queue into one sub-queue per XCD
// (workgroups go to the 8 XCDs of an MI355X round robin, so block b runs on
// XCD b % 8): sub-queue x serves the granules of kGranule consecutive
// trajectories whose index is x modulo 8, so the parameter rows a granule
// reads stay in one XCD's L2 while every sub-queue holds a fair sample of the
// work; a wave pops from its own XCD's sub-queue and then steals from the
// following ones.  The counters count positions within their sub-queue.
constexpr int kSubQueues = 8;
constexpr uint64_t kGranule = 2048;
// Each counter has a 256-byte line of its own (atomics from different XCDs on
// one line would contend); the counters take kCounterBytes.
constexpr int kCounterStride = 32;  // in u64
constexpr size_t kCounterBytes = (size_t)kSubQueues * kCounterStride * 8;

// Bytes of saved state per wave between serving step batches (x and k1 per
// gene slot, then t, h, trajectory id, step counts and flags per lane).
constexpr size_t serve_slot_bytes(int gpl, size_t elem) { return (size_t)128 * gpl * elem + 2304; }

}  // namespace rac
