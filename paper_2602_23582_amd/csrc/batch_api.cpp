// C ABI of the batched form: many systems per launch, optional HIP-graph
// replay of the step's launches, and an autotuner over launch options that
// leave every result unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "rbsog_impl.hpp"

using rbsog::Batch;
using rbsog::System;

struct rbsog_batch {
    std::vector<std::unique_ptr<System>> systems;
    std::vector<int64_t> off;  // first atom of each system in the caller's arrays
    int64_t ntot = 0;
    Batch batch;
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;  // private stream the graph is captured on
    std::string err;
    // a batch of contexts (rbsog_batch_create): admitted by device memory
    bool of_contexts = false;
    int64_t budget = 0, used = 0;
    std::vector<rbsog_ctx *> ctxs;
    std::vector<int64_t> ctx_bytes;  // bytes each admitted context was charged
};

namespace {

#define HIP_TRY(b, call)                                                       \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            (b)->err = std::string(#call) + ": " + hipGetErrorString(e_);     \
            return RBSOG_EDEVICE;                                              \
        }                                                                      \
    } while (0)

#define RB_TRY(call)                   \
    do {                               \
        int r_ = (call);               \
        if (r_ != RBSOG_OK) return r_; \
    } while (0)

int fail(rbsog_batch *b, int code, const char *msg)
{
    b->err = msg;
    return code;
}

bool is_device_ptr(const void *p)
{
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

void destroy(rbsog_batch *b)
{
    bool any = !b->ctxs.empty();
    for (auto &s : b->systems) any = any || s->atom_mem;
    if (any) (void)hipStreamSynchronize(b->batch.stream);
    for (rbsog_ctx *c : b->ctxs) {
        c->in_batch = nullptr;
        c->staged = false;
    }
    for (auto &s : b->systems) rbsog::system_free(*s);
    rbsog::batch_free(b->batch);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

// the device work of one step after the uploads
hipError_t launch_step(Batch &bt)
{
    // the sampler's fence first, then the binning launches, then the sampler
    // (on the second stream): the binning does not wait for the host's
    // cross-stream calls
    hipError_t e = rbsog::record_sample_fence(bt);
    if (e == hipSuccess) e = rbsog::launch_bin_and_sort(bt);
    if (e == hipSuccess) e = rbsog::launch_sample_fenced(bt);
    if (e == hipSuccess) e = rbsog::launch_pair(bt);
    if (e == hipSuccess) e = rbsog::launch_kspace(bt);
    return e;
}

std::vector<int64_t> graph_key(const Batch &bt)
{
    std::vector<int64_t> k(bt.plan_len, bt.plan_len + rbsog::kNumPlans);
    k.push_back(bt.pair_schedule);
    k.push_back(bt.pair_wg_per_cu);
    k.push_back(bt.precision);
    k.push_back(reinterpret_cast<intptr_t>(bt.d_desc));
    k.push_back(reinterpret_cast<intptr_t>(bt.d_step));
    k.push_back(reinterpret_cast<intptr_t>(bt.d_plan));
    k.push_back(static_cast<int64_t>(bt.sys.size()));
    for (int g = 0; g <= rbsog::kNumPairGroups; ++g) k.push_back(bt.pair_split[g]);
    k.push_back(bt.want_energy);
    return k;
}

// launches of the step as a graph, captured on a private stream and replayed
// on the batch's stream; captured again whenever a launch shape changes
int run_graph(rbsog_batch *b)
{
    Batch &bt = b->batch;
    const std::vector<int64_t> key = graph_key(bt);
    if (!bt.graph_exec || key != bt.graph_key) {
        if (bt.graph_exec) (void)hipGraphExecDestroy(bt.graph_exec);
        if (bt.graph) (void)hipGraphDestroy(bt.graph);
        bt.graph_exec = nullptr;
        bt.graph = nullptr;
        if (!b->cap_stream) HIP_TRY(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        hipStream_t user = bt.stream;
        bt.stream = b->cap_stream;
        hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        hipError_t e2 = e == hipSuccess ? launch_step(bt) : e;
        hipError_t e3 = e == hipSuccess ? hipStreamEndCapture(b->cap_stream, &bt.graph) : e;
        bt.stream = user;
        HIP_TRY(b, e);
        HIP_TRY(b, e2);
        HIP_TRY(b, e3);
        HIP_TRY(b, hipGraphInstantiate(&bt.graph_exec, bt.graph, nullptr, nullptr, 0));
        bt.graph_key = key;
    }
    HIP_TRY(b, hipGraphLaunch(bt.graph_exec, bt.stream));
    return RBSOG_OK;
}

// One step of every admitted context from its staged inputs; the results go
// to each context (read back with rbsog_pressure, rbsog_step_info).
int step_contexts(rbsog_batch *b, double *host_P, double *host_energy, int64_t *host_info)
{
    Batch &bt = b->batch;
    if (b->ctxs.empty()) return fail(b, RBSOG_ESTATE, "no context admitted");
    for (rbsog_ctx *c : b->ctxs)
        if (!c->staged) return fail(b, RBSOG_ESTATE, "an admitted context has no staged step (rbsog_stage)");
    for (rbsog_ctx *c : b->ctxs) {
        if (c->desc_moved) bt.desc_dirty = true;
        c->desc_moved = false;
    }
    bt.want_energy = host_energy != nullptr;
    RB_TRY(rbsog::batch_upload(bt, b->err));
    if (b->use_graph && !bt.timing) {
        RB_TRY(run_graph(b));
    } else {
        HIP_TRY(b, launch_step(bt));
    }
    RB_TRY(rbsog::batch_fetch_results(bt, b->err));
    const size_t S = b->ctxs.size();
    int rc = RBSOG_OK;
    for (size_t s = 0; s < S; ++s) {
        rbsog_ctx *c = b->ctxs[s];
        const rbsog::StepResults &r = bt.h_res[s];
        c->batch.h_res[0] = r;
        c->res_from_batch = true;
        c->staged = false;
        c->state = 2;
        if (r.status != 0 && rc == RBSOG_OK) rc = fail(b, RBSOG_EDEVICE, "sampler: no start draw accepted");
        if (r.bad_input && rc == RBSOG_OK) rc = fail(b, RBSOG_EINVAL, "positions have NaN/Inf");
        if (host_P)
            for (int k = 0; k < 9; ++k) host_P[9 * s + k] = r.Ptot[k];
        if (host_energy) {
            host_energy[3 * s] = r.UN;
            host_energy[3 * s + 1] = r.UF;
            host_energy[3 * s + 2] = r.Uself;
        }
        if (host_info) {
            host_info[4 * s] = r.nd;
            host_info[4 * s + 1] = r.acc_r;
            host_info[4 * s + 2] = r.acc_nr;
            host_info[4 * s + 3] = static_cast<int64_t>(std::llround(r.npairs));
        }
    }
    return rc;
}

int step_impl(rbsog_batch *b, const int64_t *host_steps, const double *host_boxes, const double *x, const double *y,
              const double *z, double *fx, double *fy, double *fz, double *host_P, double *host_energy,
              int64_t *host_info)
{
    if (b->of_contexts) {
        if (host_steps || host_boxes || x || y || z || fx || fy || fz)
            return fail(b, RBSOG_EINVAL, "a batch of contexts takes its inputs from rbsog_stage (pass NULL)");
        return step_contexts(b, host_P, host_energy, host_info);
    }
    if (!host_steps || !host_boxes || !x || !y || !z || !fx || !fy || !fz)
        return fail(b, RBSOG_EINVAL, "null argument");
    if (!(is_device_ptr(x) && is_device_ptr(y) && is_device_ptr(z) && is_device_ptr(fx) && is_device_ptr(fy) &&
          is_device_ptr(fz)))
        return fail(b, RBSOG_EINVAL, "batch position and force arrays must be device memory");
    Batch &bt = b->batch;
    const size_t S = b->systems.size();
    for (size_t s = 0; s < S; ++s) {
        if (host_steps[s] < 0 || (host_steps[s] >> 32)) return fail(b, RBSOG_EINVAL, "step must be in [0, 2^32)");
        RB_TRY(rbsog::check_box(host_boxes + 3 * s, b->systems[s]->prm.rc, b->err));
    }
    for (size_t s = 0; s < S; ++s) {
        System &y_ = *b->systems[s];
        rbsog::system_set_box(y_, host_boxes + 3 * s);
        bool recarved = false;
        RB_TRY(rbsog::system_ensure_cells(y_, b->err, &recarved));
        if (recarved) bt.desc_dirty = true;
        rbsog::SysStep &t = y_.stp;
        t.step = static_cast<uint32_t>(host_steps[s]);
        t.x = x + b->off[s];
        t.y = y + b->off[s];
        t.z = z + b->off[s];
        t.fx = fx + b->off[s];
        t.fy = fy + b->off[s];
        t.fz = fz + b->off[s];
    }
    bt.want_energy = host_energy != nullptr;
    RB_TRY(rbsog::batch_upload(bt, b->err));
    if (b->use_graph && !bt.timing) {
        RB_TRY(run_graph(b));
    } else {
        HIP_TRY(b, launch_step(bt));
    }
    if (host_P || host_energy || host_info) {
        RB_TRY(rbsog::batch_fetch_results(bt, b->err));
        for (size_t s = 0; s < S; ++s) {
            const rbsog::StepResults &r = bt.h_res[s];
            if (r.status != 0) return fail(b, RBSOG_EDEVICE, "sampler: no start draw accepted");
            if (r.bad_input) return fail(b, RBSOG_EINVAL, "positions have NaN/Inf");
            if (host_P)
                for (int k = 0; k < 9; ++k) host_P[9 * s + k] = r.Ptot[k];
            if (host_energy) {
                host_energy[3 * s] = r.UN;
                host_energy[3 * s + 1] = r.UF;
                host_energy[3 * s + 2] = r.Uself;
            }
            if (host_info) {
                host_info[4 * s] = r.nd;
                host_info[4 * s + 1] = r.acc_r;
                host_info[4 * s + 2] = r.acc_nr;
                host_info[4 * s + 3] = static_cast<int64_t>(std::llround(r.npairs));
            }
        }
    }
    return RBSOG_OK;
}

}  // namespace

extern "C" {

int rbsog_batch_setup(const rbsog_params *params, int32_t nsys, const int64_t *n, const double *host_q,
                      const double *host_boxes, void *hip_stream, rbsog_batch **out)
{
    if (!out) return RBSOG_EINVAL;
    *out = nullptr;
    if (!params || !n || !host_q || !host_boxes || nsys < 1 || nsys > 65536) return RBSOG_EINVAL;
    for (int32_t s = 1; s < nsys; ++s)
        if (params[s].precision != params[0].precision) return RBSOG_EINVAL;
    rbsog_batch *b = new (std::nothrow) rbsog_batch;
    if (!b) return RBSOG_ENOMEM;
    int rc = RBSOG_OK;
    b->off.resize(nsys);
    for (int32_t s = 0; s < nsys && rc == RBSOG_OK; ++s) {
        b->off[s] = b->ntot;
        b->systems.emplace_back(new System);
        rc = rbsog::system_init(*b->systems[s], params[s], n[s], host_q + b->ntot, host_boxes + 3 * s, b->err);
        b->ntot += n[s];
    }
    if (rc == RBSOG_OK)
        rc = rbsog::batch_init(b->batch, static_cast<hipStream_t>(hip_stream), params[0].precision, b->err);
    for (int32_t s = 0; s < nsys && rc == RBSOG_OK; ++s) {
        rc = rbsog::system_alloc(*b->systems[s], b->err);
        if (rc == RBSOG_OK) rc = rbsog::system_upload_q(*b->systems[s], host_q + b->off[s], b->batch.stream, b->err);
    }
    if (rc == RBSOG_OK) {
        std::vector<System *> ptrs;
        for (auto &s : b->systems) ptrs.push_back(s.get());
        rc = rbsog::batch_set_systems(b->batch, ptrs, b->err);
    }
    if (rc != RBSOG_OK) {
        destroy(b);
        return rc;
    }
    *out = b;
    return RBSOG_OK;
}

int rbsog_batch_create(int64_t mem_budget_bytes, void *hip_stream, rbsog_batch **out)
{
    if (!out) return RBSOG_EINVAL;
    *out = nullptr;
    if (mem_budget_bytes <= 0) return RBSOG_EINVAL;
    rbsog_batch *b = new (std::nothrow) rbsog_batch;
    if (!b) return RBSOG_ENOMEM;
    b->of_contexts = true;
    b->budget = mem_budget_bytes;
    const int rc = rbsog::batch_init(b->batch, static_cast<hipStream_t>(hip_stream), RBSOG_PREC_FP32C, b->err);
    if (rc != RBSOG_OK) {
        destroy(b);
        return rc;
    }
    *out = b;
    return RBSOG_OK;
}

int rbsog_batch_admit(rbsog_batch *b, rbsog_ctx *ctx)
{
    if (!b || !ctx) return RBSOG_EINVAL;
    b->err.clear();
    if (!b->of_contexts) return fail(b, RBSOG_EINVAL, "this batch was set up with its own systems");
    if (ctx->in_batch) return fail(b, RBSOG_ESTATE, "the context is already admitted to a batch");
    if (!b->ctxs.empty() && ctx->sys.prm.precision != b->batch.precision)
        return fail(b, RBSOG_EINVAL, "every context of a batch uses one precision");
    const int64_t bytes = static_cast<int64_t>(rbsog::system_device_bytes(ctx->sys));
    if (b->ctxs.size() >= 65536 || bytes > b->budget - b->used)
        return fail(b, RBSOG_EAGAIN, "memory budget or slots of the batch are full");
    // the context's own queued work finishes before the batch's stream uses its buffers
    HIP_TRY(b, hipStreamSynchronize(ctx->batch.stream));
    if (b->ctxs.empty()) b->batch.precision = ctx->sys.prm.precision;
    b->ctxs.push_back(ctx);
    b->ctx_bytes.push_back(bytes);
    std::vector<System *> sys;
    for (rbsog_ctx *c : b->ctxs) sys.push_back(&c->sys);
    const int rc = rbsog::batch_set_systems(b->batch, sys, b->err);
    if (rc != RBSOG_OK) {
        b->ctxs.pop_back();
        b->ctx_bytes.pop_back();
        return rc;
    }
    b->used += bytes;
    ctx->in_batch = b;
    ctx->staged = false;
    ctx->desc_moved = false;
    ctx->res_from_batch = false;
    return RBSOG_OK;
}

int rbsog_batch_release(rbsog_batch *b, rbsog_ctx *ctx)
{
    if (!b || !ctx) return RBSOG_EINVAL;
    b->err.clear();
    if (ctx->in_batch != b) return fail(b, RBSOG_EINVAL, "the context is not admitted to this batch");
    HIP_TRY(b, hipStreamSynchronize(b->batch.stream));
    for (size_t s = 0; s < b->ctxs.size(); ++s)
        if (b->ctxs[s] == ctx) {
            b->used -= b->ctx_bytes[s];
            b->ctxs.erase(b->ctxs.begin() + static_cast<std::ptrdiff_t>(s));
            b->ctx_bytes.erase(b->ctx_bytes.begin() + static_cast<std::ptrdiff_t>(s));
            break;
        }
    ctx->in_batch = nullptr;
    ctx->staged = false;
    // the context's own batch re-uploads its descriptor (the batch wrote other result slots)
    ctx->batch.desc_dirty = true;
    std::vector<System *> sys;
    for (rbsog_ctx *c : b->ctxs) sys.push_back(&c->sys);
    return rbsog::batch_set_systems(b->batch, sys, b->err);
}

int rbsog_batch_step(rbsog_batch *b, const int64_t *host_steps, const double *host_boxes, const double *x,
                     const double *y, const double *z, double *fx, double *fy, double *fz, double *host_P,
                     double *host_energy, int64_t *host_info)
{
    if (!b) return RBSOG_EINVAL;
    b->err.clear();
    return step_impl(b, host_steps, host_boxes, x, y, z, fx, fy, fz, host_P, host_energy, host_info);
}

int rbsog_batch_rescale(rbsog_batch *b, const double *host_mu, double *x, double *y, double *z, double *host_boxes)
{
    if (!b) return RBSOG_EINVAL;
    b->err.clear();
    if (b->of_contexts) return fail(b, RBSOG_ESTATE, "a batch of contexts is rescaled per context");
    if (!host_mu || !host_boxes || !x || !y || !z) return fail(b, RBSOG_EINVAL, "null argument");
    if (!(is_device_ptr(x) && is_device_ptr(y) && is_device_ptr(z)))
        return fail(b, RBSOG_EINVAL, "rbsog_batch_rescale needs device position arrays");
    const size_t S = b->systems.size();
    for (size_t s = 0; s < 3 * S; ++s)
        if (!std::isfinite(host_mu[s]) || host_mu[s] <= 0)
            return fail(b, RBSOG_EINVAL, "scale factors must be positive and finite");
    for (size_t s = 0; s < S; ++s) {
        rbsog::SysStep &t = b->systems[s]->stp;
        for (int d = 0; d < 3; ++d) t.mu[d] = host_mu[3 * s + d];
        t.x = x + b->off[s];
        t.y = y + b->off[s];
        t.z = z + b->off[s];
    }
    RB_TRY(rbsog::batch_upload(b->batch, b->err));
    HIP_TRY(b, rbsog::launch_rescale(b->batch));
    for (size_t s = 0; s < 3 * S; ++s) host_boxes[s] *= host_mu[s];
    return RBSOG_OK;
}

int rbsog_batch_set_options(rbsog_batch *b, int32_t schedule, int32_t wg_per_cu, int32_t use_graph)
{
    if (!b) return RBSOG_EINVAL;
    if ((schedule != RBSOG_SCHED_STATIC && schedule != RBSOG_SCHED_PERSISTENT) || wg_per_cu < 1 || wg_per_cu > 64)
        return fail(b, RBSOG_EINVAL, "bad launch options");
    b->batch.pair_schedule = schedule;
    b->batch.pair_wg_per_cu = wg_per_cu;
    b->use_graph = use_graph != 0;
    return RBSOG_OK;
}

int rbsog_batch_autotune(rbsog_batch *b, const int64_t *host_steps, const double *host_boxes, const double *x,
                         const double *y, const double *z, double *fx, double *fy, double *fz, int32_t reps,
                         double *host_ms, int32_t *host_choice)
{
    if (!b) return RBSOG_EINVAL;
    b->err.clear();
    if (reps < 1 || reps > 1000) return fail(b, RBSOG_EINVAL, "reps must be in [1, 1000]");
    struct Cand {
        int schedule, wg;
    };
    const Cand cands[] = {{RBSOG_SCHED_STATIC, 1}, {RBSOG_SCHED_PERSISTENT, 4}, {RBSOG_SCHED_PERSISTENT, 8},
                          {RBSOG_SCHED_PERSISTENT, 16}, {RBSOG_SCHED_PERSISTENT, 32}};
    const int nc = sizeof(cands) / sizeof(cands[0]);
    hipEvent_t e0, e1;
    HIP_TRY(b, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(b, RBSOG_EDEVICE, "event creation failed");
    }
    double best = 1e300;
    int choice = 0;
    int rc = RBSOG_OK;
    for (int c = 0; c < nc && rc == RBSOG_OK; ++c) {
        b->batch.pair_schedule = cands[c].schedule;
        b->batch.pair_wg_per_cu = cands[c].wg;
        rc = step_impl(b, host_steps, host_boxes, x, y, z, fx, fy, fz, nullptr, nullptr, nullptr);
        if (rc == RBSOG_OK && hipStreamSynchronize(b->batch.stream) != hipSuccess) rc = RBSOG_EDEVICE;
        if (rc != RBSOG_OK) break;
        (void)hipEventRecord(e0, b->batch.stream);
        for (int r = 0; r < reps && rc == RBSOG_OK; ++r)
            rc = step_impl(b, host_steps, host_boxes, x, y, z, fx, fy, fz, nullptr, nullptr, nullptr);
        (void)hipEventRecord(e1, b->batch.stream);
        float ms = 0.f;
        if (rc == RBSOG_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = RBSOG_EDEVICE;
        const double mean = ms / reps;
        if (host_ms) host_ms[c] = mean;
        if (mean < best) {
            best = mean;
            choice = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != RBSOG_OK) {
        if (b->err.empty()) b->err = "autotune step failed";
        return rc;
    }
    b->batch.pair_schedule = cands[choice].schedule;
    b->batch.pair_wg_per_cu = cands[choice].wg;
    if (host_choice) *host_choice = choice;
    return RBSOG_OK;
}

namespace {

// The cached autotuner's candidates: the pair kernel's schedule and the step's
// graph replay.  None changes an operation or the order of any sum, so every
// candidate gives the same bits.
struct TuneCand {
    int schedule, wg, graph;
};
constexpr TuneCand kTuneCands[] = {
    {RBSOG_SCHED_STATIC, 1, 0},      {RBSOG_SCHED_PERSISTENT, 4, 0},  {RBSOG_SCHED_PERSISTENT, 8, 0},
    {RBSOG_SCHED_PERSISTENT, 16, 0}, {RBSOG_SCHED_PERSISTENT, 32, 0}, {RBSOG_SCHED_STATIC, 1, 1},
    {RBSOG_SCHED_PERSISTENT, 4, 1},  {RBSOG_SCHED_PERSISTENT, 8, 1},  {RBSOG_SCHED_PERSISTENT, 16, 1},
    {RBSOG_SCHED_PERSISTENT, 32, 1}};
constexpr int kNumTuneCands = sizeof(kTuneCands) / sizeof(kTuneCands[0]);
static_assert(kNumTuneCands == RBSOG_TUNE_CANDIDATES, "candidate count of the header");

std::mutex g_tune_mu;  // one reader or writer of a cache file at a time in this process

// The cache key: the device (architecture and compute units), the batch's
// atoms rounded down to a power of two and its largest batch size P rounded
// up to one.
int tune_key(rbsog_batch *b, std::string &key)
{
    int dev = 0;
    hipDeviceProp_t prop;
    HIP_TRY(b, hipGetDevice(&dev));
    HIP_TRY(b, hipGetDeviceProperties(&prop, dev));
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    int nb = 0;
    while ((int64_t{2} << nb) <= b->ntot) ++nb;
    int pmax = 1;
    for (const auto &s : b->systems) pmax = std::max(pmax, static_cast<int>(s->prm.P));
    int pb = 1;
    while (pb < pmax) pb <<= 1;
    key = arch + " cu" + std::to_string(prop.multiProcessorCount) + " n2^" + std::to_string(nb) + " P" +
          std::to_string(pb);
    return RBSOG_OK;
}

// the last line of the file for this key: candidate index and its step time
bool tune_lookup(const char *path, const std::string &key, int &choice, double &ms)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        const char *bar = std::strchr(line, '|');
        if (!bar || std::string(line, bar - line) != key) continue;
        int c = -1;
        double m = 0.0;
        if (std::sscanf(bar + 1, "%d %lf", &c, &m) == 2 && c >= 0 && c < kNumTuneCands) {
            choice = c;
            ms = m;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

}  // namespace

int rbsog_batch_autotune_cached(rbsog_batch *b, const char *cache_path, int32_t force, const int64_t *host_steps,
                                const double *host_boxes, const double *x, const double *y, const double *z,
                                double *fx, double *fy, double *fz, int32_t reps, double *host_ms,
                                int32_t *host_choice, int32_t *host_cached)
{
    if (!b || !cache_path) return RBSOG_EINVAL;
    b->err.clear();
    if (b->of_contexts) return fail(b, RBSOG_EINVAL, "the autotuner times batches built by rbsog_batch_setup");
    if (reps < 1 || reps > 1000) return fail(b, RBSOG_EINVAL, "reps must be in [1, 1000]");
    std::string key;
    RB_TRY(tune_key(b, key));
    if (host_ms)
        for (int c = 0; c < kNumTuneCands; ++c) host_ms[c] = 0.0;
    int choice = 0;
    double best = 0.0;
    bool hit = false;
    if (!force) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        hit = tune_lookup(cache_path, key, choice, best);
    }
    if (!hit) {
        hipEvent_t e0, e1;
        HIP_TRY(b, hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(b, RBSOG_EDEVICE, "event creation failed");
        }
        best = 1e300;
        int rc = RBSOG_OK;
        for (int c = 0; c < kNumTuneCands && rc == RBSOG_OK; ++c) {
            b->batch.pair_schedule = kTuneCands[c].schedule;
            b->batch.pair_wg_per_cu = kTuneCands[c].wg;
            b->use_graph = kTuneCands[c].graph != 0;
            // one untimed step (it captures the graph when one is replayed)
            rc = step_impl(b, host_steps, host_boxes, x, y, z, fx, fy, fz, nullptr, nullptr, nullptr);
            if (rc == RBSOG_OK && hipStreamSynchronize(b->batch.stream) != hipSuccess) rc = RBSOG_EDEVICE;
            if (rc != RBSOG_OK) break;
            (void)hipEventRecord(e0, b->batch.stream);
            for (int r = 0; r < reps && rc == RBSOG_OK; ++r)
                rc = step_impl(b, host_steps, host_boxes, x, y, z, fx, fy, fz, nullptr, nullptr, nullptr);
            (void)hipEventRecord(e1, b->batch.stream);
            float ms = 0.f;
            if (rc == RBSOG_OK &&
                (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = RBSOG_EDEVICE;
            const double mean = ms / reps;
            if (host_ms) host_ms[c] = mean;
            if (mean < best) {
                best = mean;
                choice = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != RBSOG_OK) {
            if (b->err.empty()) b->err = "autotune step failed";
            return rc;
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        FILE *f = std::fopen(cache_path, "a");
        if (!f) return fail(b, RBSOG_EINVAL, (std::string("cannot append to the tuning cache ") + cache_path).c_str());
        const bool ok = std::fprintf(f, "%s|%d %.6f schedule=%s wg_per_cu=%d graph=%d\n", key.c_str(), choice, best,
                                     kTuneCands[choice].schedule == RBSOG_SCHED_STATIC ? "static" : "persistent",
                                     kTuneCands[choice].wg, kTuneCands[choice].graph) > 0;
        if (std::fclose(f) != 0 || !ok)
            return fail(b, RBSOG_EINVAL, (std::string("cannot write the tuning cache ") + cache_path).c_str());
    } else if (host_ms) {
        host_ms[choice] = best;
    }
    b->batch.pair_schedule = kTuneCands[choice].schedule;
    b->batch.pair_wg_per_cu = kTuneCands[choice].wg;
    b->use_graph = kTuneCands[choice].graph != 0;
    if (host_choice) *host_choice = choice;
    if (host_cached) *host_cached = hit ? 1 : 0;
    return RBSOG_OK;
}

int rbsog_batch_set_timing(rbsog_batch *b, int on)
{
    if (!b) return RBSOG_EINVAL;
    rbsog::batch_set_timing(b->batch, on);
    return RBSOG_OK;
}

int rbsog_batch_get_timing(rbsog_batch *b, int32_t cap, int32_t *host_nk, char *host_names, double *host_ms,
                           int64_t *host_count)
{
    if (!b) return RBSOG_EINVAL;
    return rbsog::batch_get_timing(b->batch, cap, host_nk, host_names, host_ms, host_count, b->err);
}

int rbsog_batch_destroy(rbsog_batch *b)
{
    if (!b) return RBSOG_OK;
    destroy(b);
    return RBSOG_OK;
}

const char *rbsog_batch_last_error(const rbsog_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
