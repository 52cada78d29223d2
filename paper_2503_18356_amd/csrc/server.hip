// Serving step batches: a fixed grid of the bounded DP5 kernel advances every
// in-flight trajectory of every admitted request by a bounded number of loop
// iterations, parks unfinished trajectories in a device slot table, and pulls
// new trajectories from a device queue that the host extends between batches.
// The launch has fixed arguments, so it is captured once into a hipGraph and
// replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "kernel_table.h"
#include "rac_internal.h"

namespace rac {
// Defined in solver.hip.
rac_status check_opts_public(const rac_solver_opts* o, const char* who);
rac_status check_item_public(const rac_topology* topo, const rac_params_view* p, const float* ic,
                             int32_t n_ic, const void* x_out, const char* who);
Controls make_controls_public(const rac_solver_opts* o, int n_groups);
}  // namespace rac

struct rac_server {
    rac_solver_opts opts;
    int lpt = 0, epl = 0, gpl = 0;
    int device = 0;
    int grid = 0;
    int max_requests = 0;
    int batch_steps = 0;
    const rac::KernelEntry* ke = nullptr;
    char* block = nullptr;
    rac::ServeCtl* ctl = nullptr;
    rac::NetDesc* nets = nullptr;
    int32_t* done = nullptr;
    char* slots = nullptr;
    size_t slot_bytes = 0;
    // Host copies that the stream-ordered uploads read from (never reused).
    std::vector<rac::NetDesc> host_nets;
    std::vector<rac::ServeCtl> host_ctl;
    int32_t n_requests = 0;
    int64_t total = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    rac::LaunchArgs args;
    std::mutex mu;
};

namespace rac {
namespace {

// Undo a queue head that ran past the tail during a batch (claims beyond the
// tail were never served).  Last node of every step batch, so it runs before
// a later submit moves the tail.
__global__ void clamp_head(ServeCtl* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && c->head > c->total) c->head = c->total;
}

#define RAC_SHIP(call, what)                                                            \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(RAC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace
}  // namespace rac

extern "C" {

rac_status rac_server_create(const rac_solver_opts* opts, int32_t epl, int32_t gpl,
                             int32_t max_requests, int32_t batch_steps, rac_server** out) {
    using namespace rac;
    if (!out) return fail(RAC_EINVAL, "rac_server_create: out is NULL");
    *out = nullptr;
    rac_status st = check_opts_public(opts, "rac_server_create");
    if (st != RAC_OK) return st;
    if (!(opts->t_end > opts->t0)) return fail(RAC_EINVAL, "rac_server_create: t_end <= t0");
    if (opts->precision != RAC_FP32)
        return fail(RAC_EUNSUPPORTED, "rac_server_create: serving step batches are compiled for RAC_FP32");
    if (opts->method != RAC_DP5)
        return fail(RAC_EUNSUPPORTED, "rac_server_create: serving step batches are compiled for RAC_DP5");
    if (opts->lanes_per_traj < 1) return fail(RAC_EINVAL, "rac_server_create: lanes_per_traj must be set");
    if (max_requests < 1 || batch_steps < 1)
        return fail(RAC_EINVAL, "rac_server_create: need max_requests >= 1 and batch_steps >= 1");
    const KernelEntry* ke = find_kernel(RAC_FP32, false, epl, gpl, true);
    if (!ke) return fail(RAC_EUNSUPPORTED, "rac_server_create: no compiled kernel shape (epl, gpl)");
    auto* s = new (std::nothrow) rac_server;
    if (!s) return fail(RAC_ENOMEM, "rac_server_create: out of host memory");
    s->opts = *opts;
    s->lpt = opts->lanes_per_traj;
    s->epl = epl;
    s->gpl = gpl;
    s->max_requests = max_requests;
    s->batch_steps = batch_steps;
    s->ke = ke;
    int n_cu = 0, per_cu = 0;
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ke->fn, kBlock, 0) != hipSuccess) {
        delete s;
        return fail(RAC_EDEVICE, "rac_server_create: device query failed");
    }
    s->grid = std::max(1, per_cu) * n_cu;
    s->slot_bytes = serve_slot_bytes(gpl, sizeof(float)) * (size_t)s->grid * (kBlock / kWave);
    const size_t off_nets = 256;
    const size_t off_done = off_nets + sizeof(NetDesc) * (size_t)max_requests;
    const size_t off_slots = (off_done + sizeof(int32_t) * (size_t)max_requests + 255) / 256 * 256;
    const size_t bytes = off_slots + s->slot_bytes;
    if (hipMalloc(&s->block, bytes) != hipSuccess) {
        delete s;
        return fail(RAC_ENOMEM, "rac_server_create: hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    s->ctl = (ServeCtl*)s->block;
    s->nets = (NetDesc*)(s->block + off_nets);
    s->done = (int32_t*)(s->block + off_done);
    s->slots = s->block + off_slots;
    // Empty queue, zero counters, every slot free (trajectory id -1).
    if (hipMemset(s->block, 0, off_slots) != hipSuccess ||
        hipMemset(s->slots, 0xff, s->slot_bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(s->block);
        delete s;
        return fail(RAC_EDEVICE, "rac_server_create: initialisation failed");
    }
    s->host_nets.resize(max_requests);
    s->host_ctl.resize(max_requests);
    std::memset(&s->args, 0, sizeof(s->args));
    s->args.nets = s->nets;
    s->args.n_nets = 0;
    s->args.lpt = s->lpt;
    s->args.epl = epl;
    s->args.gpl = gpl;
    s->args.c = make_controls_public(opts, kWave / s->lpt);
    s->args.ctl = s->ctl;
    s->args.counter = &s->ctl->head;
    s->args.slots = s->slots;
    s->args.batch_steps = batch_steps;
    *out = s;
    return RAC_OK;
}

void rac_server_destroy(rac_server* s) {
    if (!s) return;
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->block) (void)hipFree(s->block);
    delete s;
}

rac_status rac_server_submit(rac_server* s, const rac_topology* topo, const rac_params_view* dev_params,
                             const float* dev_ic, int32_t n_ic, void* dev_x_out,
                             const rac_traj_info* dev_info, void* hip_stream, int32_t* request_id) {
    using namespace rac;
    if (!s) return fail(RAC_EINVAL, "rac_server_submit: NULL server");
    rac_status st = check_item_public(topo, dev_params, dev_ic, n_ic, dev_x_out, "rac_server_submit");
    if (st != RAC_OK) return st;
    if (!plan_fits(topo, s->lpt, RAC_FP32)) return fail(RAC_EUNSUPPORTED, "rac_server_submit: network does not fit");
    const LanePlan* lp = get_plan(topo, s->lpt);
    if (std::max(lp->epl, 1) > s->epl || lp->gpl > s->gpl)
        return fail(RAC_EUNSUPPORTED, "rac_server_submit: network needs a larger kernel shape than this server's");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->n_requests >= s->max_requests) return fail(RAC_ENOMEM, "rac_server_submit: request table full");
    const DevicePlan* dp = nullptr;
    st = get_device_plan(topo, s->lpt, &dp);
    if (st != RAC_OK) return st;
    const int32_t id = s->n_requests;
    NetDesc& d = s->host_nets[id];
    std::memset(&d, 0, sizeof(d));
    d.lane_edge = dp->lane_edge;
    d.gene_row = dp->gene_row;
    d.row_ptr = dp->row_ptr;
    d.sign = dp->sign;
    d.G = dev_params->G;
    d.k = dev_params->k;
    d.T = dev_params->T;
    d.lam = dev_params->lam;
    d.n = dev_params->n;
    d.nf = dev_params->nf;
    d.ic = dev_ic;
    d.x_out = dev_x_out;
    if (dev_info) {
        d.t_final = dev_info->t_final;
        d.status = dev_info->status;
        d.n_acc = dev_info->n_accepted;
        d.n_rej = dev_info->n_rejected;
    }
    d.done = s->done + id;
    d.n_sets = dev_params->n_sets;
    d.traj_begin = s->total;
    d.n_traj = dev_params->n_sets * n_ic;
    d.inv_n_ic = 1.0 / n_ic;
    d.n_genes = topo->n_genes;
    d.n_edges = topo->n_edges;
    d.n_ic = n_ic;
    d.stride = lp->stride;
    ServeCtl& c = s->host_ctl[id];
    c.head = 0;
    c.total = (unsigned long long)(s->total + d.n_traj);
    c.n_nets = id + 1;
    c.pad = 0;
    hipStream_t stream = (hipStream_t)hip_stream;
    RAC_SHIP(hipMemcpyAsync(s->nets + id, &d, sizeof(NetDesc), hipMemcpyHostToDevice, stream),
             "rac_server_submit: table upload");
    RAC_SHIP(hipMemcpyAsync(&s->ctl->total, &c.total, sizeof(c.total) + sizeof(c.n_nets),
                            hipMemcpyHostToDevice, stream),
             "rac_server_submit: queue upload");
    s->total += d.n_traj;
    s->n_requests = id + 1;
    if (request_id) *request_id = id;
    return RAC_OK;
}

rac_status rac_server_step(rac_server* s, void* hip_stream) {
    using namespace rac;
    if (!s) return fail(RAC_EINVAL, "rac_server_step: NULL server");
    if (!hip_stream) return fail(RAC_EINVAL, "rac_server_step: needs a created stream (the null stream cannot be captured)");
    std::lock_guard<std::mutex> lk(s->mu);
    hipStream_t stream = (hipStream_t)hip_stream;
    if (!s->exec) {
        // Capture the step-batch launch once; its arguments never change.
        RAC_SHIP(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed), "rac_server_step: begin capture");
        void* args[] = {&s->args};
        hipError_t le = hipLaunchKernel(s->ke->fn, dim3(s->grid), dim3(kBlock), args, 0, stream);
        if (le == hipSuccess) {
            hipLaunchKernelGGL(clamp_head, dim3(1), dim3(64), 0, stream, s->ctl);
            le = hipGetLastError();
        }
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(stream, &g);
        if (le != hipSuccess || ce != hipSuccess)
            return fail(RAC_EDEVICE, std::string("rac_server_step: capture failed: ") +
                                         hipGetErrorString(le != hipSuccess ? le : ce));
        s->graph = g;
        RAC_SHIP(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0), "rac_server_step: instantiate");
    }
    RAC_SHIP(hipGraphLaunch(s->exec, stream), "rac_server_step: graph launch");
    return RAC_OK;
}

rac_status rac_server_done_counts(rac_server* s, int32_t first, int32_t count, int32_t* host_out,
                                  void* hip_stream) {
    using namespace rac;
    if (!s || !host_out || first < 0 || count < 0) return fail(RAC_EINVAL, "rac_server_done_counts: bad argument");
    if (count == 0) return RAC_OK;
    if (first + count > s->n_requests) return fail(RAC_EINVAL, "rac_server_done_counts: range beyond submitted requests");
    RAC_SHIP(hipMemcpyAsync(host_out, s->done + first, sizeof(int32_t) * count, hipMemcpyDeviceToHost,
                            (hipStream_t)hip_stream),
             "rac_server_done_counts: copy");
    return RAC_OK;
}

rac_status rac_server_info(const rac_server* s, int32_t* n_requests, int64_t* total_trajectories,
                           int32_t* grid_waves, int64_t* slot_bytes) {
    if (!s) return rac::fail(RAC_EINVAL, "rac_server_info: NULL server");
    if (n_requests) *n_requests = s->n_requests;
    if (total_trajectories) *total_trajectories = s->total;
    if (grid_waves) *grid_waves = s->grid * (rac::kBlock / rac::kWave);
    if (slot_bytes) *slot_bytes = (int64_t)s->slot_bytes;
    return RAC_OK;
}

}  // extern "C"
