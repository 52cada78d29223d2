// Internal declarations shared by the host code and the HIP kernels.
#pragma once

#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "rac.h"

namespace rac {

// Largest network the lane plans address: src gene and edge id are packed in
// 16 bits each.
constexpr int kMaxGenes = 4096;
constexpr int kMaxEdges = 32767;
constexpr int kWave = 64;

// Compiled kernel shapes: edge slots per lane (EPL) and gene slots per lane
// (GPL) are compile-time register budgets; the counts actually used are
// runtime bounds <= these.
struct Shape {
    int epl, gpl;
};
// FP32 kernels with at most this many edge slots per lane evaluate each Hill
// factor as 1 + D / (1 + 2^z), D >= 0; others use the symmetric form with a
// base term.  The two agree to rounding, not bit for bit.
constexpr int kUnitBaseMaxEpl = 16;
constexpr Shape kShapesF32[] = {
    {4, 1}, {4, 2}, {4, 3}, {4, 4}, {4, 6}, {4, 8}, {8, 1}, {8, 2}, {8, 3}, {8, 4}, {8, 6},
    {8, 8}, {12, 1}, {12, 2}, {12, 3}, {12, 4}, {12, 6}, {12, 8}, {16, 1}, {16, 2}, {16, 3},
    {16, 4}, {16, 6}, {16, 8}, {24, 1}, {24, 2}, {24, 3}, {24, 4}, {24, 6}, {32, 1}, {32, 2},
    {32, 3}, {7, 3}, {11, 3}, {13, 5}, {6, 2}, {10, 4}, {6, 3}};
constexpr Shape kShapesF64[] = {
    {4, 1}, {4, 2}, {4, 3}, {4, 4}, {4, 6}, {8, 1}, {8, 2}, {8, 3}, {8, 4}, {12, 1}, {12, 2},
    {12, 3}, {16, 1}, {16, 2}, {7, 3}};

// How one network is spread over the lanes of a trajectory group.
struct LanePlan {
    int lpt = 0;      // lanes per trajectory (power of two, <= 64)
    int epl = 0;      // edge slots used per lane (max over lanes)
    int stride = 1;   // row stride of lane_edge = max(epl, 1)
    int gpl = 0;      // gene slots used per lane = ceil(N / lpt)
    // [lpt][epl]: (edge id) | (activating << 15) | (src gene << 16), or -1 for
    // an empty slot (edge ids stay below 2^15).
    std::vector<int32_t> lane_edge;
    // [N]: row lane | (first prefix index << 8) | (end prefix index << 16).
    std::vector<int32_t> gene_row;
};

struct DevicePlan {
    int device = -1;
    int lpt = 0;
    int32_t* lane_edge = nullptr;  // [lpt][stride]
    int32_t* gene_row = nullptr;   // [N]
    int32_t* row_ptr = nullptr;    // [N + 1]
    int8_t* sign = nullptr;        // [E]
    void* block = nullptr;         // single allocation holding the above
};

}  // namespace rac

struct rac_topology {
    int32_t n_genes = 0;
    int32_t n_edges = 0;
    std::vector<int32_t> src, dst;   // canonical (dst, src) order
    std::vector<int8_t> sign;
    std::vector<int32_t> row_ptr;    // [N + 1] CSR by target
    mutable std::mutex mu;
    // Deques keep element addresses stable while new plans are appended.
    mutable std::deque<rac::LanePlan> plans;        // by lpt, built lazily
    mutable std::deque<rac::DevicePlan> dev_plans;  // by (device, lpt)
};

namespace rac {

void set_error(const std::string& msg);
rac_status fail(rac_status st, const std::string& msg);

// Host-side lane plan (built once per (topology, lpt), cached).
const LanePlan* get_plan(const rac_topology* t, int lpt);
int max_in_degree(const rac_topology* t);
// Cheapest compiled shape covering (epl, gpl); {0, 0} if none.
Shape pick_shape(int epl, int gpl, int precision);
bool plan_fits(const rac_topology* t, int lpt, int precision);
int auto_lanes(const rac_topology* t, int precision);
// auto_lanes adjusted for a call too small to fill the GPU.
int auto_lanes_for(const rac_topology* t, int precision, double n_traj);
// Estimated issue cost of one trajectory step at a lane count and kernel shape
// (lanes x per-lane slot work / latency-hiding efficiency of the shape).
double shape_cost(int lpt, const Shape& s, int precision);

// Per-call tables of the sampler (host and device use the same ones).
struct SampleTables {
    int method = RAC_SAMPLE_UNIFORM;
    std::vector<double> scale;                // per edge: threshold scale
    const uint32_t* sobol_v = nullptr;        // [kSobolDims][32] direction numbers
    std::vector<uint32_t> shift0, shift1;     // Sobol' shifts per dimension
    std::vector<uint64_t> lhs_key0, lhs_key1; // 4 LHS round keys per dimension
    int64_t lhs_n0 = 0, lhs_n1 = 0;           // Latin hypercube sizes
    int lhs_w0 = 1, lhs_w1 = 1;               // their word widths
};
constexpr int kSobolDims = 4096;
rac_status make_sample_tables(const rac_topology* t, const rac_ranges& r, uint64_t seed, int64_t set_begin,
                              int64_t n_sets, int32_t n_ic, SampleTables* out);

// Device copy of a plan on the current device (cached in the handle).
rac_status get_device_plan(const rac_topology* t, int lpt, const DevicePlan** out);
void free_device_plans(rac_topology* t);

}  // namespace rac
