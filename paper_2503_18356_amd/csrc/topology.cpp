// Topology handle, error reporting and the lane plans that spread one network
// over the lanes of a trajectory group.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>

#include "rac_internal.h"

namespace rac {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

rac_status fail(rac_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

int max_in_degree(const rac_topology* t) {
    int m = 0;
    for (int i = 0; i < t->n_genes; ++i) m = std::max(m, t->row_ptr[i + 1] - t->row_ptr[i]);
    return m;
}

Shape pick_shape(int epl, int gpl, int precision) {
    Shape best{0, 0};
    auto consider = [&](const Shape& s) {
        if (s.epl < epl || s.gpl < gpl) return;
        if (best.epl == 0 || 14 * s.epl + 25 * s.gpl < 14 * best.epl + 25 * best.gpl) best = s;
    };
    if (precision == RAC_FP64)
        for (const Shape& s : kShapesF64) consider(s);
    else
        for (const Shape& s : kShapesF32) consider(s);
    return best;
}

// Build the plan for `lpt` lanes per trajectory.
//  - Gene i is owned (its DP5 state lives) in lane i % lpt, slot i / lpt.
//  - Whole in-edge rows are packed into lanes, largest in-degree first, each
//    into the currently least loaded lane.  A lane evaluates its edge slots
//    in order and keeps running products, so the production term of gene i is
//    prefix[end] / prefix[begin] of the lane that holds its row.
static LanePlan build_plan(const rac_topology* t, int lpt) {
    LanePlan p;
    p.lpt = lpt;
    const int N = t->n_genes;
    p.gpl = (N + lpt - 1) / lpt;
    std::vector<int> order(N);
    std::iota(order.begin(), order.end(), 0);
    auto deg = [&](int i) { return t->row_ptr[i + 1] - t->row_ptr[i]; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return deg(a) > deg(b); });
    std::vector<std::vector<int>> lane_rows(lpt);
    std::vector<int> load(lpt, 0);
    for (int i : order) {
        if (deg(i) == 0) continue;
        int best = 0;
        for (int l = 1; l < lpt; ++l)
            if (load[l] < load[best]) best = l;
        lane_rows[best].push_back(i);
        load[best] += deg(i);
    }
    p.epl = *std::max_element(load.begin(), load.end());
    p.stride = std::max(p.epl, 1);
    p.lane_edge.assign((size_t)lpt * p.stride, -1);
    p.gene_row.assign(N, 0);  // empty rows: lane 0, prefix [0, 0) -> product 1
    for (int l = 0; l < lpt; ++l) {
        int s = 0;
        for (int i : lane_rows[l]) {
            int begin = s;
            for (int e = t->row_ptr[i]; e < t->row_ptr[i + 1]; ++e) {
                p.lane_edge[(size_t)l * p.stride + s] = e | (t->sign[e] > 0 ? 0x8000 : 0) | (t->src[e] << 16);
                ++s;
            }
            p.gene_row[i] = l | (begin << 8) | (s << 16);
        }
    }
    return p;
}

const LanePlan* get_plan(const rac_topology* t, int lpt) {
    std::lock_guard<std::mutex> lk(t->mu);
    for (auto& p : t->plans)
        if (p.lpt == lpt) return &p;
    t->plans.push_back(build_plan(t, lpt));
    return &t->plans.back();
}

bool plan_fits(const rac_topology* t, int lpt, int precision) {
    if (lpt < 1 || lpt > kWave || (lpt & (lpt - 1))) return false;
    const LanePlan* p = get_plan(t, lpt);
    return pick_shape(std::max(p->epl, 1), p->gpl, precision).epl != 0;
}

// Heuristic lane count when the caller gives none: minimise estimated issue
// work per trajectory step, lanes x (edge slots x 14 + gene slots x 25 + 40),
// divided by a latency-hiding efficiency that falls with the shape's register
// footprint (waves per SIMD).  The constants come from timing the kernel
// shapes on MI355X; the autotuner measures instead of estimating.
static double shape_efficiency(const Shape& s, int precision) {
    // Fitted to the compiled kernels' VGPR counts (FP32 edges cost one
    // register less in the base-free factor form).
    const double vgpr = precision == RAC_FP64 ? 105.0 + 8.0 * s.epl + 18.0 * s.gpl
                                              : 55.0 + (s.epl <= kUnitBaseMaxEpl ? 4.0 : 5.0) * s.epl + 12.0 * s.gpl;
    const int waves = vgpr > 256 ? 1 : std::min(8, (int)(512.0 / (8.0 * std::ceil(vgpr / 8.0))));
    static const double eff[] = {0.0, 0.30, 0.54, 0.71, 0.88, 1.0, 1.0, 1.0, 1.0};
    return eff[waves];
}

double shape_cost(int lpt, const Shape& s, int precision) {
    return lpt * (14.0 * s.epl + 25.0 * s.gpl + 40.0) / shape_efficiency(s, precision);
}

// Lane count for a call of n_traj trajectories.  A call that cannot fill the
// GPU at the cost model's choice finishes sooner with more lanes per
// trajectory: each trajectory's steps are shorter although the issue work
// grows.  Estimated time = cost per trajectory step / utilisation, with the
// utilisation u = x / (x + 2.6) of x = n_traj x lanes / (lanes resident on
// an MI355X at four waves per SIMD), a form fitted to timings of 10^3 to
// 10^6 trajectories of 2-, 10-, 22- and 50-gene networks (it keeps the
// model's choice for 10^6 trajectories of a 10-gene network and moves 10^4
// of them from 4 to 16 lanes, 36 % faster).  Calls with x >= 8 at the
// model's choice keep it unchanged, and a move needs an estimated gain of
// 15 % (the register model behind the costs is approximate: the 22-gene
// network's 10^4 trajectories, estimated 14 % faster at 16 lanes than at 8,
// measured 9 % slower).
int auto_lanes_for(const rac_topology* t, int precision, double n_traj) {
    const int base = auto_lanes(t, precision);
    constexpr double kResidentLanes = 256.0 * 4 * 4 * kWave;
    auto fill = [&](int lpt) {
        const double x = n_traj * lpt / kResidentLanes;
        return x / (x + 2.6);
    };
    if (base == 0 || n_traj * base >= 8.0 * kResidentLanes) return base;
    auto est = [&](int lpt) {
        const LanePlan* p = get_plan(t, lpt);
        const Shape s = pick_shape(std::max(p->epl, 1), p->gpl, precision);
        return shape_cost(lpt, s, precision) / fill(lpt);
    };
    int best = base;
    double best_t = 0.85 * est(base);
    for (int lpt = 2 * base; lpt <= kWave; lpt *= 2) {
        if (!plan_fits(t, lpt, precision)) continue;
        const double tt = est(lpt);
        if (tt < best_t) {
            best = lpt;
            best_t = tt;
        }
    }
    return best;
}

int auto_lanes(const rac_topology* t, int precision) {
    int best = 0;
    double best_cost = 0;
    for (int lpt = 1; lpt <= kWave; lpt *= 2) {
        if (!plan_fits(t, lpt, precision)) continue;
        const LanePlan* p = get_plan(t, lpt);
        // Padded slots are evaluated too, so cost the compiled shape.
        const Shape s = pick_shape(std::max(p->epl, 1), p->gpl, precision);
        const double cost = shape_cost(lpt, s, precision);
        if (best == 0 || cost < best_cost) {
            best = lpt;
            best_cost = cost;
        }
    }
    return best;
}

}  // namespace rac

extern "C" {

const char* rac_last_error(void) { return rac::g_last_error.c_str(); }

const char* rac_version(void) { return "racipe-mi355x 0.1"; }

rac_status rac_create_topology(int32_t n_genes, int32_t n_edges, const int32_t* src,
                               const int32_t* dst, const int8_t* sign, rac_topology** out) {
    using rac::fail;
    if (!out) return fail(RAC_EINVAL, "rac_create_topology: out is NULL");
    *out = nullptr;
    if (n_genes < 1) return fail(RAC_EINVAL, "rac_create_topology: n_genes < 1");
    if (n_edges < 0) return fail(RAC_EINVAL, "rac_create_topology: n_edges < 0");
    if (n_edges > 0 && (!src || !dst || !sign))
        return fail(RAC_EINVAL, "rac_create_topology: NULL edge array");
    if (n_genes > rac::kMaxGenes || n_edges > rac::kMaxEdges)
        return fail(RAC_EUNSUPPORTED, "rac_create_topology: network larger than 4096 genes / 32767 edges");
    struct E { int32_t s, d; int8_t g; };
    std::vector<E> e(n_edges);
    for (int i = 0; i < n_edges; ++i) {
        if (src[i] < 0 || src[i] >= n_genes || dst[i] < 0 || dst[i] >= n_genes)
            return fail(RAC_EINVAL, "rac_create_topology: edge " + std::to_string(i) + " index out of range");
        if (sign[i] != 1 && sign[i] != -1)
            return fail(RAC_EINVAL, "rac_create_topology: edge " + std::to_string(i) + " sign not +-1");
        e[i] = {src[i], dst[i], sign[i]};
    }
    std::sort(e.begin(), e.end(), [](const E& a, const E& b) {
        return a.d != b.d ? a.d < b.d : a.s < b.s;
    });
    for (int i = 1; i < n_edges; ++i)
        if (e[i].s == e[i - 1].s && e[i].d == e[i - 1].d)
            return fail(RAC_EINVAL, "rac_create_topology: duplicate edge " + std::to_string(e[i].s) +
                                        " -> " + std::to_string(e[i].d));
    auto* t = new (std::nothrow) rac_topology;
    if (!t) return fail(RAC_ENOMEM, "rac_create_topology: out of host memory");
    t->n_genes = n_genes;
    t->n_edges = n_edges;
    t->src.resize(n_edges);
    t->dst.resize(n_edges);
    t->sign.resize(n_edges);
    t->row_ptr.assign(n_genes + 1, 0);
    for (int i = 0; i < n_edges; ++i) {
        t->src[i] = e[i].s;
        t->dst[i] = e[i].d;
        t->sign[i] = e[i].g;
        t->row_ptr[e[i].d + 1]++;
    }
    for (int i = 0; i < n_genes; ++i) t->row_ptr[i + 1] += t->row_ptr[i];
    *out = t;
    return RAC_OK;
}

void rac_destroy_topology(rac_topology* topo) {
    if (!topo) return;
    rac::free_device_plans(topo);
    delete topo;
}

rac_status rac_topology_size(const rac_topology* topo, int32_t* n_genes, int32_t* n_edges) {
    if (!topo) return rac::fail(RAC_EINVAL, "rac_topology_size: NULL topology");
    if (n_genes) *n_genes = topo->n_genes;
    if (n_edges) *n_edges = topo->n_edges;
    return RAC_OK;
}

rac_status rac_topology_edges(const rac_topology* topo, int32_t* src, int32_t* dst, int8_t* sign) {
    if (!topo) return rac::fail(RAC_EINVAL, "rac_topology_edges: NULL topology");
    const size_t E = topo->n_edges;
    if (src && E) std::memcpy(src, topo->src.data(), E * sizeof(int32_t));
    if (dst && E) std::memcpy(dst, topo->dst.data(), E * sizeof(int32_t));
    if (sign && E) std::memcpy(sign, topo->sign.data(), E * sizeof(int8_t));
    return RAC_OK;
}

int32_t rac_auto_lanes(const rac_topology* topo, int32_t precision) {
    if (!topo || (precision != RAC_FP32 && precision != RAC_FP64)) return 0;
    return rac::auto_lanes(topo, precision);
}

int32_t rac_auto_lanes_for(const rac_topology* topo, int32_t precision, int64_t n_traj) {
    if (!topo || (precision != RAC_FP32 && precision != RAC_FP64) || n_traj < 0) return 0;
    return rac::auto_lanes_for(topo, precision, (double)n_traj);
}

rac_status rac_plan_shape(const rac_topology* topo, int32_t precision, int32_t lanes, int32_t* epl,
                          int32_t* gpl) {
    if (!topo || (precision != RAC_FP32 && precision != RAC_FP64))
        return rac::fail(RAC_EINVAL, "rac_plan_shape: bad topology or precision");
    if (!rac::plan_fits(topo, lanes, precision))
        return rac::fail(RAC_EUNSUPPORTED, "rac_plan_shape: no compiled shape for this lane count");
    const rac::LanePlan* p = rac::get_plan(topo, lanes);
    const rac::Shape s = rac::pick_shape(std::max(p->epl, 1), p->gpl, precision);
    if (epl) *epl = s.epl;
    if (gpl) *gpl = s.gpl;
    return RAC_OK;
}

int32_t rac_lanes_supported(const rac_topology* topo, int32_t precision, int32_t lanes) {
    if (!topo || (precision != RAC_FP32 && precision != RAC_FP64)) return 0;
    return rac::plan_fits(topo, lanes, precision) ? 1 : 0;
}

}  // extern "C"
