// Host side of the integration calls: option checks, device copies of the
// lane plans, kernel selection, persistent-grid sizing and launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "kernel_table.h"
#include "rac_internal.h"

namespace rac {

#define RAC_HIP(call, what)                                                             \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(RAC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

const KernelEntry* find_kernel(int precision, bool ts, int epl, int gpl, bool bounded, int method, bool realn) {
    static std::vector<KernelEntry> all = [] {
        std::vector<KernelEntry> v;
        for (auto fn : {kernels_f32_ss, kernels_f32_ts, kernels_f64_ss, kernels_f64_ts, kernels_f32_serve,
                        kernels_f32_ss_tsit5, kernels_f32_ts_tsit5, kernels_f64_ss_tsit5,
                        kernels_f64_ts_tsit5, kernels_f64_realn, kernels_f64_realn_tsit5}) {
            const KernelEntry* t = nullptr;
            int n = fn(&t);
            v.insert(v.end(), t, t + n);
        }
        return v;
    }();
    for (const KernelEntry& k : all)
        if (k.precision == precision && k.ts == ts && k.epl == epl && k.gpl == gpl && k.bounded == bounded &&
            k.method == method && k.realn == realn)
            return &k;
    return nullptr;
}

// Side streams per device (default priority) on which run_jobs overlaps the
// launches of one call; created on first use and kept for the process.
static const std::vector<hipStream_t>& side_streams(int dev) {
    static std::mutex m;
    static std::map<int, std::vector<hipStream_t>> all;
    std::lock_guard<std::mutex> lk(m);
    auto it = all.find(dev);
    if (it != all.end()) return it->second;
    std::vector<hipStream_t> v;
    for (int i = 0; i < 3; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) break;
        v.push_back(s);
    }
    return all[dev] = v;
}

// A library-owned non-blocking stream per device for small uploads, so that
// building a plan never waits for (or serialises with) work on user streams.
static hipStream_t lib_stream(int dev) {
    static std::mutex m;
    static std::map<int, hipStream_t> streams;
    std::lock_guard<std::mutex> lk(m);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    streams[dev] = s;
    return s;
}

// The device copy of a plan made earlier on the current device, without
// building or uploading anything (nullptr if there is none).
static const DevicePlan* find_device_plan(const rac_topology* t, int lpt, int dev) {
    std::lock_guard<std::mutex> lk(t->mu);
    for (auto& d : t->dev_plans)
        if (d.device == dev && d.lpt == lpt) return &d;
    return nullptr;
}

rac_status get_device_plan(const rac_topology* t, int lpt, const DevicePlan** out) {
    int dev = 0;
    RAC_HIP(hipGetDevice(&dev), "hipGetDevice");
    const LanePlan* lp = get_plan(t, lpt);
    std::lock_guard<std::mutex> lk(t->mu);
    for (auto& d : t->dev_plans)
        if (d.device == dev && d.lpt == lpt) {
            *out = &d;
            return RAC_OK;
        }
    const size_t n_le = lp->lane_edge.size(), N = t->n_genes, E = t->n_edges;
    const size_t bytes = 4 * (n_le + N + N + 1) + std::max<size_t>(E, 1);
    hipStream_t ls = lib_stream(dev);
    if (!ls) return fail(RAC_EDEVICE, "device plan: no upload stream");
    void* block = nullptr;
    if (hipMallocAsync(&block, bytes, ls) != hipSuccess) return fail(RAC_ENOMEM, "device plan: allocation failed");
    std::vector<char> host(bytes, 0);
    char* h = host.data();
    std::memcpy(h, lp->lane_edge.data(), 4 * n_le);
    std::memcpy(h + 4 * n_le, lp->gene_row.data(), 4 * N);
    std::memcpy(h + 4 * (n_le + N), t->row_ptr.data(), 4 * (N + 1));
    if (E) std::memcpy(h + 4 * (n_le + 2 * N + 1), t->sign.data(), E);
    if (hipMemcpyAsync(block, h, bytes, hipMemcpyHostToDevice, ls) != hipSuccess ||
        hipStreamSynchronize(ls) != hipSuccess) {
        (void)hipFreeAsync(block, ls);
        return fail(RAC_EDEVICE, "device plan: upload failed");
    }
    DevicePlan d;
    d.device = dev;
    d.lpt = lpt;
    d.block = block;
    char* b = (char*)block;
    d.lane_edge = (int32_t*)b;
    d.gene_row = (int32_t*)(b + 4 * n_le);
    d.row_ptr = (int32_t*)(b + 4 * (n_le + N));
    d.sign = (int8_t*)(b + 4 * (n_le + 2 * N + 1));
    t->dev_plans.push_back(d);
    *out = &t->dev_plans.back();
    return RAC_OK;
}

// Plans are released on the upload stream without a device-wide
// synchronisation; the caller guarantees no enqueued work still reads them.
void free_device_plans(rac_topology* t) {
    for (auto& d : t->dev_plans) {
        hipStream_t ls = lib_stream(d.device);
        if (ls) (void)hipFreeAsync(d.block, ls);
    }
    t->dev_plans.clear();
}

namespace {

// Zero the sub-queue counters and, for a single network, store its
// descriptor (a kernel, not a memset: no memset node in captured graphs, and
// no host copy for the common one-network launch).
__global__ void setup_launch(unsigned long long* counter, NetDesc* table, NetDesc one) {
    if (blockIdx.x == 0 && threadIdx.x < kSubQueues) counter[threadIdx.x * kCounterStride] = 0ull;
    if (threadIdx.x == 0 && blockIdx.x == 0 && table) *table = one;
}

rac_status check_opts(const rac_solver_opts* o, const char* who) {
    std::string w(who);
    if (!o) return fail(RAC_EINVAL, w + ": NULL opts");
    if (o->precision != RAC_FP32 && o->precision != RAC_FP64)
        return fail(RAC_EINVAL, w + ": precision must be RAC_FP32 or RAC_FP64");
    if (!std::isfinite(o->t0) || !std::isfinite(o->t_end))
        return fail(RAC_EINVAL, w + ": t0 and t_end must be finite");
    if (!(o->rtol >= 0) || !(o->atol >= 0) || !(o->rtol + o->atol > 0))
        return fail(RAC_EINVAL, w + ": need rtol >= 0, atol >= 0, rtol + atol > 0");
    if (!(o->ss_atol >= 0) || !(o->ss_rtol >= 0))
        return fail(RAC_EINVAL, w + ": steady tolerances must be >= 0");
    if (o->max_steps < 1) return fail(RAC_EINVAL, w + ": max_steps < 1");
    if (!(o->h0 <= 0 || std::isfinite(o->h0))) return fail(RAC_EINVAL, w + ": h0 not finite");
    if (o->lanes_per_traj < 0 || o->lanes_per_traj > kWave ||
        (o->lanes_per_traj & (o->lanes_per_traj - 1)))
        return fail(RAC_EINVAL, w + ": lanes_per_traj must be 0 or a power of two <= 64");
    if (o->refill_min < 0) return fail(RAC_EINVAL, w + ": refill_min < 0");
    if (o->method != RAC_DP5 && o->method != RAC_TSIT5)
        return fail(RAC_EINVAL, w + ": method must be RAC_DP5 or RAC_TSIT5");
    return RAC_OK;
}

rac_status check_item(const rac_topology* topo, const rac_params_view* p, const float* ic,
                      int32_t n_ic, const void* x_out, const char* who) {
    std::string w(who);
    if (!topo) return fail(RAC_EINVAL, w + ": NULL topology");
    if (!p) return fail(RAC_EINVAL, w + ": NULL params");
    if (p->n_sets < 0) return fail(RAC_EINVAL, w + ": n_sets < 0");
    if (n_ic < 1) return fail(RAC_EINVAL, w + ": n_ic < 1");
    if (p->n_sets > 0) {
        if (!p->G || !p->k || (topo->n_edges > 0 && (!p->T || !p->lam || (!p->n && !p->nf))))
            return fail(RAC_EINVAL, w + ": NULL parameter array");
        if (!ic) return fail(RAC_EINVAL, w + ": NULL initial conditions");
        if (!x_out) return fail(RAC_EINVAL, w + ": NULL x_out");
        if (p->n_sets > (int64_t)1 << 40) return fail(RAC_EUNSUPPORTED, w + ": n_sets too large");
    }
    return RAC_OK;
}

struct Job {
    const rac_topology* topo;
    rac_params_view params;
    const float* ic;
    int32_t n_ic;
    void* x_out;
    rac_traj_info info;
    int32_t lanes = 0;   // 0: from the options
    int32_t refill = 0;  // 0: from the options
};

// The options' lane count, else the cost model's choice for a call of
// n_traj trajectories in all (more lanes when the call cannot fill the GPU).
int pick_lanes(const rac_topology* t, const rac_solver_opts* o, double n_traj) {
    return o->lanes_per_traj > 0 ? o->lanes_per_traj : auto_lanes_for(t, o->precision, n_traj);
}

Controls make_controls(const rac_solver_opts* o, int n_groups) {
    Controls c;
    c.t0 = o->t0;
    c.t_end = o->t_end;
    c.rtol = o->rtol;
    c.atol = o->atol;
    c.ss_atol = o->ss_atol;
    c.ss_rtol = o->ss_rtol;
    c.h0 = o->h0;
    c.max_steps = o->max_steps;
    c.divide = o->activation_divides_by_lambda ? 1 : 0;
    c.ic_absolute = o->ic_absolute ? 1 : 0;
    c.stop_at_steady = o->stop_at_steady ? 1 : 0;
    // A wave pulls new work once a quarter of its groups are free, or half of
    // them when it holds eight or fewer (each refill costs the whole wave a
    // start-up iteration of two right-hand sides; measured on the 22-gene
    // network at 8 groups per wave: refill at 4 free groups 24.7 ms, at 2
    // 25.2 ms, at 1 25.8 ms).
    c.refill_min = o->refill_min > 0 ? o->refill_min : std::max(1, n_groups <= 8 ? n_groups / 2 : n_groups / 4);
    c.chunk = n_groups;
    c.pad = 0;
    return c;
}

std::map<std::tuple<int, const void*>, int>& occupancy_cache() {
    static std::map<std::tuple<int, const void*>, int> m;
    return m;
}

// Launch one persistent kernel over the given networks (all with lane count
// lpt) in a shared work queue.
// With fixed_block (a single steady-state network only), the queue counter
// and the network descriptor go to that device block instead of a per-call
// allocation, and the lane plan must already be on the device: nothing is
// allocated.
rac_status launch_group(const std::vector<Job>& jobs, int lpt, const rac_solver_opts* o, bool ts,
                        const double* host_t_out, int32_t n_t, hipStream_t stream,
                        char* fixed_block = nullptr) {
    int epl = 0, gpl = 0, max_n = 0;
    int64_t total = 0;
    std::vector<NetDesc> descs;
    if (fixed_block && (ts || jobs.size() != 1))
        return fail(RAC_EINVAL, "launch without allocation: one steady-state network only");
    int cur_dev = 0;
    RAC_HIP(hipGetDevice(&cur_dev), "hipGetDevice");
    for (const Job& j : jobs) {
        const DevicePlan* dp = nullptr;
        if (fixed_block) {
            dp = find_device_plan(j.topo, lpt, cur_dev);
            if (!dp)
                return fail(RAC_EINVAL, "the network's lane plan for " + std::to_string(lpt) +
                                            " lanes is not on this device yet: solve it once with "
                                            "rac_steady_states (same options) before the call without allocation");
        } else {
            rac_status st = get_device_plan(j.topo, lpt, &dp);
            if (st != RAC_OK) return st;
        }
        const LanePlan* lp = get_plan(j.topo, lpt);
        NetDesc d;
        std::memset(&d, 0, sizeof(d));
        d.lane_edge = dp->lane_edge;
        d.gene_row = dp->gene_row;
        d.row_ptr = dp->row_ptr;
        d.sign = dp->sign;
        d.G = j.params.G;
        d.k = j.params.k;
        d.T = j.params.T;
        d.lam = j.params.lam;
        d.n = j.params.n;
        d.nf = j.params.nf;
        d.ic = j.ic;
        d.x_out = j.x_out;
        d.t_final = j.info.t_final;
        d.status = j.info.status;
        d.n_acc = j.info.n_accepted;
        d.n_rej = j.info.n_rejected;
        d.n_sets = j.params.n_sets;
        d.traj_begin = total;
        d.n_traj = j.params.n_sets * j.n_ic;
        d.n_genes = j.topo->n_genes;
        d.n_edges = j.topo->n_edges;
        d.n_ic = j.n_ic;
        d.inv_n_ic = 1.0 / j.n_ic;
        d.stride = lp->stride;
        total += d.n_traj;
        epl = std::max(epl, lp->epl);
        gpl = std::max(gpl, lp->gpl);
        max_n = std::max(max_n, j.topo->n_genes);
        descs.push_back(d);
    }
    if (total == 0) return RAC_OK;
    const Shape shape = pick_shape(std::max(epl, 1), gpl, o->precision);
    // FP64 launches with real Hill coefficients in any network take the
    // exp/log kernels (integer coefficients of the other networks are read as
    // floats there); FP32 kernels handle both.
    bool realn = false;
    for (const NetDesc& d : descs) realn = realn || d.nf != nullptr;
    realn = realn && o->precision == RAC_FP64;
    const KernelEntry* ke =
        shape.epl ? find_kernel(o->precision, ts, shape.epl, shape.gpl, false, o->method, realn) : nullptr;
    if (!ke) return fail(RAC_EUNSUPPORTED, "no compiled kernel for this network size and lane count");

    int dev = 0, n_cu = 0;
    RAC_HIP(hipGetDevice(&dev), "hipGetDevice");
    RAC_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
    int per_cu = 0;
    {
        static std::mutex m;
        std::lock_guard<std::mutex> lk(m);
        auto key = std::make_tuple(dev, ke->fn);
        auto it = occupancy_cache().find(key);
        if (it == occupancy_cache().end()) {
            RAC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ke->fn, kBlock, 0),
                    "hipOccupancyMaxActiveBlocksPerMultiprocessor");
            occupancy_cache()[key] = per_cu;
        } else {
            per_cu = it->second;
        }
    }
    per_cu = std::max(per_cu, 1);
    const int n_groups = kWave / lpt;
    const int64_t waves_needed = (total + n_groups - 1) / n_groups;
    const int64_t blocks_needed = (waves_needed + kBlock / kWave - 1) / (kBlock / kWave);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * n_cu, blocks_needed));

    LaunchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_nets = (int32_t)descs.size();
    a.total = total;
    a.lpt = lpt;
    a.epl = epl;
    a.gpl = gpl;
    a.n_t = ts ? n_t : 0;
    a.c = make_controls(o, n_groups);
    int refill = 0;
    for (const Job& j : jobs) refill = std::max(refill, j.refill);
    if (refill > 0) a.c.refill_min = refill;

    // Per-call device block: queue counters, network table, output times.
    const size_t off_nets = kCounterBytes;
    const size_t off_t = off_nets + (descs.size() * sizeof(NetDesc) + 255) / 256 * 256;
    const size_t bytes = off_t + (ts ? sizeof(double) * n_t : 0);
    void* blk = fixed_block;
    if (!fixed_block) RAC_HIP(hipMallocAsync(&blk, bytes, stream), "hipMallocAsync");
    char* b = (char*)blk;
    a.counter = (unsigned long long*)b;
    a.nets = (const NetDesc*)(b + off_nets);
    if (descs.size() > 1)
        RAC_HIP(hipMemcpyAsync(b + off_nets, descs.data(), descs.size() * sizeof(NetDesc),
                               hipMemcpyHostToDevice, stream), "hipMemcpyAsync(nets)");
    if (ts) {
        a.t_out = (const double*)(b + off_t);
        RAC_HIP(hipMemcpyAsync(b + off_t, host_t_out, sizeof(double) * n_t, hipMemcpyHostToDevice, stream),
                "hipMemcpyAsync(t_out)");
    }
    hipLaunchKernelGGL(setup_launch, dim3(1), dim3(64), 0, stream, a.counter,
                       descs.size() == 1 ? (NetDesc*)(b + off_nets) : nullptr, descs[0]);
    RAC_HIP(hipGetLastError(), "setup_launch");
    void* args[] = {&a};
    RAC_HIP(hipLaunchKernel(ke->fn, dim3(grid), dim3(kBlock), args, 0, stream), "dp5 kernel launch");
    if (!fixed_block) RAC_HIP(hipFreeAsync(blk, stream), "hipFreeAsync");
    return RAC_OK;
}

using ClassKey = std::tuple<int, int, int>;  // lanes per trajectory, edge slots, gene slots

// Merge launch classes: a class moves into a larger shape of the same lane
// count and factor form (results stay bit-identical) when the work its padded
// slots add, trajectories x the cost difference per step, is below what one
// more launch wastes while it drains, taken as half a residency of the
// target's trajectories (4096 waves of 64 / lanes each) at the target's cost.
// Smallest classes first, into the target that adds least, until none moves.
void merge_classes(std::map<ClassKey, std::vector<Job>>& groups, int precision) {
    constexpr double kResidentWaves = 4096.0;
    auto traj_of = [](const std::vector<Job>& js) {
        double n = 0;
        for (const Job& j : js) n += (double)j.params.n_sets * j.n_ic;
        return n;
    };
    for (bool moved = true; moved && groups.size() > 1;) {
        moved = false;
        std::vector<std::pair<double, ClassKey>> by_work;
        for (auto& kv : groups) {
            const auto& [l, e, g] = kv.first;
            by_work.push_back({traj_of(kv.second) * shape_cost(l, Shape{e, g}, precision), kv.first});
        }
        std::sort(by_work.begin(), by_work.end());
        for (const auto& bw : by_work) {
            const auto& [l, e, g] = bw.second;
            const double n = traj_of(groups[bw.second]);
            const double c_src = shape_cost(l, Shape{e, g}, precision);
            const ClassKey* best = nullptr;
            double best_add = 0;
            for (auto& kv : groups) {
                const auto& [l2, e2, g2] = kv.first;
                if (kv.first == bw.second || l2 != l || e2 < e || g2 < g ||
                    rac_factor_form(precision, e2) != rac_factor_form(precision, e))
                    continue;
                const double c_dst = shape_cost(l, Shape{e2, g2}, precision);
                const double add = n * (c_dst - c_src);
                const double drain = 0.5 * kResidentWaves * (kWave / l) * c_dst;
                if (add <= drain && (best == nullptr || add < best_add)) {
                    best = &kv.first;
                    best_add = add;
                }
            }
            if (best) {
                std::vector<Job>& dst = groups[*best];
                for (Job& j : groups[bw.second]) dst.push_back(j);
                groups.erase(bw.second);
                moved = true;
                break;
            }
        }
    }
}

rac_status run_jobs(std::vector<Job>& jobs, const rac_solver_opts* o, bool ts,
                    const double* host_t_out, int32_t n_t, void* stream) {
    // Group networks by (lane count, kernel shape): one persistent launch each.
    std::map<ClassKey, std::vector<Job>> groups;
    double call_traj = 0;
    for (const Job& j : jobs) call_traj += (double)j.params.n_sets * j.n_ic;
    for (const Job& j : jobs) {
        if (j.params.n_sets == 0) continue;
        const int lpt = j.lanes > 0 ? j.lanes : pick_lanes(j.topo, o, call_traj);
        if (lpt == 0 || !plan_fits(j.topo, lpt, o->precision))
            return fail(RAC_EUNSUPPORTED, "network (N=" + std::to_string(j.topo->n_genes) + ", E=" +
                                              std::to_string(j.topo->n_edges) +
                                              ") does not fit the compiled kernels at this lane count");
        const LanePlan* lp = get_plan(j.topo, lpt);
        const Shape s = pick_shape(std::max(lp->epl, 1), lp->gpl, o->precision);
        groups[std::make_tuple(lpt, s.epl, s.gpl)].push_back(j);
    }
    merge_classes(groups, o->precision);
    hipStream_t main = (hipStream_t)stream;
    if (groups.size() <= 1) {
        for (auto& kv : groups) {
            rac_status st = launch_group(kv.second, std::get<0>(kv.first), o, ts, host_t_out, n_t, main);
            if (st != RAC_OK) return st;
        }
        return RAC_OK;
    }
    // Several launches, spread over the caller's stream and the library's
    // side streams (forked from and joined back into the caller's stream), so
    // that the tail of one persistent launch, when few of its trajectories
    // remain, is filled by the waves of another.  Largest estimated work
    // first, each onto the stream with the least work so far (longest
    // processing time first); a launch's work is its trajectories times the
    // per-step cost of its lane count and shape.
    std::vector<std::pair<double, const std::tuple<int, int, int>*>> order;
    for (auto& kv : groups) {
        double n_traj = 0;
        for (const Job& j : kv.second) n_traj += (double)j.params.n_sets * j.n_ic;
        const Shape s{std::get<1>(kv.first), std::get<2>(kv.first)};
        order.push_back({n_traj * shape_cost(std::get<0>(kv.first), s, o->precision), &kv.first});
    }
    std::sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    int dev = 0;
    RAC_HIP(hipGetDevice(&dev), "hipGetDevice");
    const std::vector<hipStream_t>& side = side_streams(dev);
    if (side.empty()) return fail(RAC_EDEVICE, "side stream creation failed");
    hipEvent_t fork = nullptr;
    RAC_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming), "hipEventCreate");
    RAC_HIP(hipEventRecord(fork, main), "hipEventRecord");
    for (hipStream_t sd : side) RAC_HIP(hipStreamWaitEvent(sd, fork, 0), "hipStreamWaitEvent");
    rac_status st = RAC_OK;
    std::vector<double> load(side.size() + 1, 0.0);  // [0]: the caller's stream
    for (size_t k = 0; k < order.size() && st == RAC_OK; ++k) {
        const auto& key = *order[k].second;
        const size_t i = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
        load[i] += order[k].first;
        hipStream_t sk = i == 0 ? main : side[i - 1];
        st = launch_group(groups[key], std::get<0>(key), o, ts, host_t_out, n_t, sk);
    }
    // Join: the caller's stream waits for everything enqueued on the side streams.
    for (hipStream_t sd : side) {
        hipEvent_t done = nullptr;
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(done, sd) != hipSuccess || hipStreamWaitEvent(main, done, 0) != hipSuccess)
            st = fail(RAC_EDEVICE, "joining side streams failed");
        if (done) (void)hipEventDestroy(done);
    }
    (void)hipEventDestroy(fork);
    return st;
}

// Device scratch of the call without allocation: the queue counters in the
// first kCounterBytes, the network descriptor after them.  Each device holds its
// own copy for the life of the process; in host code the array's name is
// only a stand-in, so its device address is looked up once per device and
// used everywhere instead.
constexpr size_t kNoAllocScratchBytes = 4096;
static_assert(kCounterBytes + sizeof(NetDesc) <= kNoAllocScratchBytes, "scratch holds the counters and one descriptor");
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

rac_status scratch_address(int dev, char** out) {
    static std::mutex m;
    static std::map<int, char*> addr;
    std::lock_guard<std::mutex> lk(m);
    auto it = addr.find(dev);
    if (it != addr.end()) {
        *out = it->second;
        return RAC_OK;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(RAC_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    addr[dev] = (char*)p;
    *out = (char*)p;
    return RAC_OK;
}

}  // namespace

rac_status check_opts_public(const rac_solver_opts* o, const char* who) { return check_opts(o, who); }
rac_status check_item_public(const rac_topology* topo, const rac_params_view* p, const float* ic,
                             int32_t n_ic, const void* x_out, const char* who) {
    return check_item(topo, p, ic, n_ic, x_out, who);
}
Controls make_controls_public(const rac_solver_opts* o, int n_groups) { return make_controls(o, n_groups); }

}  // namespace rac

extern "C" {

void rac_default_opts(rac_solver_opts* o, int32_t precision) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->t0 = 0.0;
    o->t_end = 200.0;
    o->rtol = 1e-6;
    o->atol = 1e-9;
    o->ss_atol = 1e-6;
    o->ss_rtol = precision == RAC_FP64 ? 0.0 : 1e-5;
    o->h0 = 0.0;
    o->max_steps = 100000;
    o->precision = precision;
    o->activation_divides_by_lambda = 1;
    o->stop_at_steady = 0;
    o->ic_absolute = 0;
    o->lanes_per_traj = 0;
    o->refill_min = 0;
    o->method = RAC_DP5;
}

rac_status rac_steady_states(const rac_topology* topo, const rac_params_view* dev_params,
                             const float* dev_ic, int32_t n_ic, const rac_solver_opts* opts,
                             void* dev_x_out, const rac_traj_info* dev_info, void* hip_stream) {
    using namespace rac;
    rac_status st = check_opts(opts, "rac_steady_states");
    if (st != RAC_OK) return st;
    if (!(opts->t_end > opts->t0)) return fail(RAC_EINVAL, "rac_steady_states: t_end <= t0");
    st = check_item(topo, dev_params, dev_ic, n_ic, dev_x_out, "rac_steady_states");
    if (st != RAC_OK) return st;
    std::vector<Job> jobs{{topo, *dev_params, dev_ic, n_ic, dev_x_out,
                           dev_info ? *dev_info : rac_traj_info{nullptr, nullptr, nullptr, nullptr}}};
    return run_jobs(jobs, opts, false, nullptr, 0, hip_stream);
}

rac_status rac_steady_states_noalloc(const rac_topology* topo, const rac_params_view* dev_params,
                                     const float* dev_ic, int32_t n_ic, const rac_solver_opts* opts,
                                     void* dev_x_out, const rac_traj_info* dev_info, void* hip_stream) {
    using namespace rac;
    rac_status st = check_opts(opts, "rac_steady_states_noalloc");
    if (st != RAC_OK) return st;
    if (!(opts->t_end > opts->t0)) return fail(RAC_EINVAL, "rac_steady_states_noalloc: t_end <= t0");
    st = check_item(topo, dev_params, dev_ic, n_ic, dev_x_out, "rac_steady_states_noalloc");
    if (st != RAC_OK) return st;
    if (dev_params->n_sets == 0) return RAC_OK;
    const int lpt = pick_lanes(topo, opts, (double)dev_params->n_sets * n_ic);
    if (lpt == 0 || !plan_fits(topo, lpt, opts->precision))
        return fail(RAC_EUNSUPPORTED, "rac_steady_states_noalloc: network does not fit the compiled kernels");
    int dev = 0;
    const hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return fail(RAC_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(he));
    char* block = nullptr;
    st = scratch_address(dev, &block);
    if (st != RAC_OK) return st;
    std::vector<Job> jobs{{topo, *dev_params, dev_ic, n_ic, dev_x_out,
                           dev_info ? *dev_info : rac_traj_info{nullptr, nullptr, nullptr, nullptr}}};
    return launch_group(jobs, lpt, opts, false, nullptr, 0, (hipStream_t)hip_stream, block);
}

rac_status rac_integrate(const rac_topology* topo, const rac_params_view* dev_params,
                         const float* dev_ic, int32_t n_ic, const rac_solver_opts* opts,
                         const double* host_t_out, int32_t n_t, void* dev_x_out,
                         const rac_traj_info* dev_info, void* hip_stream) {
    using namespace rac;
    rac_status st = check_opts(opts, "rac_integrate");
    if (st != RAC_OK) return st;
    st = check_item(topo, dev_params, dev_ic, n_ic, dev_x_out, "rac_integrate");
    if (st != RAC_OK) return st;
    if (n_t < 1 || !host_t_out) return fail(RAC_EINVAL, "rac_integrate: need n_t >= 1 output times");
    if ((int64_t)n_t * topo->n_genes >= ((int64_t)1 << 31))
        return fail(RAC_EUNSUPPORTED, "rac_integrate: n_t x N must stay below 2^31 (one trajectory's series)");
    for (int i = 0; i < n_t; ++i) {
        if (!std::isfinite(host_t_out[i]) || host_t_out[i] < opts->t0)
            return fail(RAC_EINVAL, "rac_integrate: output time before t0 or not finite");
        if (i > 0 && !(host_t_out[i] > host_t_out[i - 1]))
            return fail(RAC_EINVAL, "rac_integrate: output times must be strictly increasing");
    }
    std::vector<Job> jobs{{topo, *dev_params, dev_ic, n_ic, dev_x_out,
                           dev_info ? *dev_info : rac_traj_info{nullptr, nullptr, nullptr, nullptr}}};
    return run_jobs(jobs, opts, true, host_t_out, n_t, hip_stream);
}

rac_status rac_steady_states_batch(const rac_batch_item* items, int32_t n_items,
                                   const rac_solver_opts* opts, void* hip_stream) {
    using namespace rac;
    rac_status st = check_opts(opts, "rac_steady_states_batch");
    if (st != RAC_OK) return st;
    if (!(opts->t_end > opts->t0)) return fail(RAC_EINVAL, "rac_steady_states_batch: t_end <= t0");
    if (n_items < 0 || (n_items > 0 && !items)) return fail(RAC_EINVAL, "rac_steady_states_batch: bad items");
    std::vector<Job> jobs;
    for (int i = 0; i < n_items; ++i) {
        const rac_batch_item& it = items[i];
        st = check_item(it.topo, &it.params, it.ic, it.n_ic, it.x_out, "rac_steady_states_batch");
        if (st != RAC_OK) return st;
        if (it.lanes_per_traj < 0 || it.lanes_per_traj > kWave || (it.lanes_per_traj & (it.lanes_per_traj - 1)))
            return fail(RAC_EINVAL, "rac_steady_states_batch: item lanes_per_traj must be 0 or a power of two <= 64");
        if (it.refill_min < 0) return fail(RAC_EINVAL, "rac_steady_states_batch: item refill_min < 0");
        Job j{it.topo, it.params, it.ic, it.n_ic, it.x_out, it.info};
        j.lanes = it.lanes_per_traj;
        j.refill = it.refill_min;
        jobs.push_back(j);
    }
    return run_jobs(jobs, opts, false, nullptr, 0, hip_stream);
}

int32_t rac_factor_form(int32_t precision, int32_t epl) {
    if ((precision != RAC_FP32 && precision != RAC_FP64) || epl < 1) return -1;
    return precision == RAC_FP32 && epl <= rac::kUnitBaseMaxEpl ? 1 : 0;
}

}  // extern "C"
