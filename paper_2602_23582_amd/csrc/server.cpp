// Served form: a request loop on a worker thread with continuous batching.
//
// A request is one system and a number of steps.  Admission is first come,
// first served: the head of the queue is admitted when a slot is free and its
// device state (positions, forces and every per-system buffer, sized for the
// largest cell grid its box schedule reaches) fits first-fit into the
// server's memory pool.  Every tick runs one batched step over all admitted
// requests, each at its own step index; a request that completes releases its
// memory, and requests that arrived meanwhile join the next tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rbsog_impl.hpp"

using rbsog::Batch;
using rbsog::System;
using Clock = std::chrono::steady_clock;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Pinned staging for the uploads of admitted requests: copies from it run
// behind a step in flight without holding the host, where copies from the
// requests' pageable buffers would wait for the stream.  Refilled every tick;
// a tick that admits more than it holds uploads the rest from pageable memory.
constexpr size_t kStageBytes = size_t(64) << 20;

// First-fit allocator over offsets of one device allocation.
class Pool {
public:
    void reset(size_t bytes)
    {
        free_.clear();
        free_[0] = bytes;
        used_ = 0;
        peak_ = 0;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t peak() const { return peak_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0, peak_ = 0;
};

struct Request {
    int64_t ticket = 0;
    int64_t n = 0;
    int nsteps = 1;
    double growth = 0.0;
    std::vector<double> q, x, y, z;  // inputs, freed once uploaded
    std::vector<float> q32;          // FP32C charges in flight to the device
    std::vector<double> boxes;       // box of every step (3 nsteps)
    std::vector<double> mus;         // scale factor before every step (1 at k = 0)
    int64_t max_cells = 0;
    size_t bytes = 0, off = 0;
    System sys;
    double *d_pos = nullptr, *d_frc = nullptr;
    int k = 0;  // next step
    int box_step = -1;  // the step whose box the host-side System holds (set_box done)
    std::vector<double> P, U, fx, fy, fz;
    Clock::time_point t_submit, t_admit, t_done;
    int shared_ticks = 0;
    bool done = false;
    int status = RBSOG_OK;
};

}  // namespace

struct rbsog_server {
    int precision = RBSOG_PREC_FP32C;
    size_t pool_bytes = 0;
    int max_active = 1;
    bool energy = true;  // every tick sums the energies
    int device = 0;
    hipStream_t stream = nullptr;
    char *pool_mem = nullptr;
    char *stage = nullptr;  // pinned, kStageBytes (null if it could not be allocated)
    size_t stage_used = 0;
    // pinned, two slots of kStageBytes (one per tick in flight or being
    // read): the forces of requests a tick completes, copied there behind the
    // step and handed to the requests while the next tick runs (null if it
    // could not be allocated)
    char *dstage = nullptr;
    // pinned results of the two ticks in flight or being read, and the
    // events that mark each tick's end
    rbsog::StepResults *h_tres[2] = {nullptr, nullptr};
    size_t res_cap[2] = {0, 0};
    hipEvent_t tick_ev[2] = {nullptr, nullptr};
    Pool pool;
    Batch batch;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::unordered_map<int64_t, std::unique_ptr<Request>> requests;
    int64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    // statistics
    int64_t submitted = 0, completed = 0, ticks = 0, peak_active = 0;
    double atom_steps = 0.0, busy_s = 0.0;
    double phase_s[3] = {};  // admission; set-up and launch; results and forces back
    std::string err, worker_err;
};

namespace {

size_t request_bytes(const rbsog_params &p, int64_t n, int64_t max_cells)
{
    return align_up(rbsog::system_atom_bytes(p, n)) + align_up(rbsog::system_cell_bytes(n, max_cells)) +
           2 * align_up(3 * n * sizeof(double));
}

// Queue the upload of an admitted request's state into its pool memory; the
// host copies stay alive until a synchronisation of the stream has covered it.
int admit(rbsog_server *sv, Request *r, std::string &err)
{
    char *base = sv->pool_mem + r->off;
    System &s = r->sys;
    s.own_mem = false;
    rbsog::system_carve_atoms(s, base);
    base += align_up(rbsog::system_atom_bytes(s.prm, s.n));
    rbsog::system_carve_cells(s, base, r->max_cells);
    base += align_up(rbsog::system_cell_bytes(s.n, r->max_cells));
    r->d_pos = reinterpret_cast<double *>(base);
    base += align_up(3 * r->n * sizeof(double));
    r->d_frc = reinterpret_cast<double *>(base);
    const int64_t n = r->n;
    const bool f64 = s.prm.precision == RBSOG_PREC_FP64;
    const size_t qb = align_up(n * (f64 ? sizeof(double) : sizeof(float))), pb = 3 * n * sizeof(double);
    if (sv->stage && sv->stage_used + qb + pb <= kStageBytes) {
        char *p = sv->stage + sv->stage_used;
        sv->stage_used += align_up(qb + pb);
        if (f64) {
            std::memcpy(p, r->q.data(), n * sizeof(double));
        } else {
            float *q32 = reinterpret_cast<float *>(p);
            for (int64_t i = 0; i < n; ++i) q32[i] = static_cast<float>(r->q[i]);
        }
        double *xyz = reinterpret_cast<double *>(p + qb);
        std::memcpy(xyz, r->x.data(), n * sizeof(double));
        std::memcpy(xyz + n, r->y.data(), n * sizeof(double));
        std::memcpy(xyz + 2 * n, r->z.data(), n * sizeof(double));
        hipError_t e = hipMemcpyAsync(const_cast<void *>(s.desc.q), p, n * (f64 ? sizeof(double) : sizeof(float)),
                                      hipMemcpyHostToDevice, sv->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(r->d_pos, xyz, pb, hipMemcpyHostToDevice, sv->stream);
        if (e != hipSuccess) {
            err = std::string("request upload: ") + hipGetErrorString(e);
            return RBSOG_EDEVICE;
        }
        return RBSOG_OK;
    }
    int rc = rbsog::system_upload_q(s, r->q.data(), sv->stream, err, &r->q32);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(r->d_pos, r->x.data(), n * sizeof(double), hipMemcpyHostToDevice, sv->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->d_pos + n, r->y.data(), n * sizeof(double), hipMemcpyHostToDevice, sv->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->d_pos + 2 * n, r->z.data(), n * sizeof(double), hipMemcpyHostToDevice, sv->stream);
    if (e != hipSuccess) {
        err = std::string("request upload: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    return RBSOG_OK;
}

// The host copies of requests whose uploads a stream synchronisation has
// covered are no longer needed.
void uploads_done(const std::vector<Request *> &admitted, Clock::time_point t)
{
    for (Request *r : admitted) {
        std::vector<double>().swap(r->q);
        std::vector<double>().swap(r->x);
        std::vector<double>().swap(r->y);
        std::vector<double>().swap(r->z);
        std::vector<float>().swap(r->q32);
        r->t_admit = t;
    }
}

// Queued requests, first come first served, while slots (busy of them taken)
// and pool memory allow.  The caller holds the lock.
void take_admissions(rbsog_server *sv, size_t busy, std::vector<Request *> &out)
{
    while (!sv->pending.empty() && static_cast<int>(busy + out.size()) < sv->max_active) {
        Request *r = sv->pending.front();
        size_t off = 0;
        if (!sv->pool.alloc(r->bytes, off)) break;
        r->off = off;
        sv->pending.pop_front();
        out.push_back(r);
    }
}

// Launch one batched step over every active request.
int tick_launch(rbsog_server *sv, std::string &err)
{
    Batch &bt = sv->batch;
    // rescale before step k >= 1 (mu = 1 at k = 0 leaves positions unchanged)
    for (Request *r : sv->active) {
        rbsog::SysStep &t = r->sys.stp;
        for (int d = 0; d < 3; ++d) t.mu[d] = r->mus[r->k];
        t.x = r->d_pos;
        t.y = r->d_pos + r->n;
        t.z = r->d_pos + 2 * r->n;
    }
    int rc = rbsog::batch_upload(bt, err);
    if (rc) return rc;
    hipError_t e = rbsog::launch_rescale(bt);
    if (e != hipSuccess) {
        err = std::string("rescale: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    for (Request *r : sv->active) {
        System &s = r->sys;
        if (r->box_step != r->k) {
            rbsog::system_set_box(s, &r->boxes[3 * r->k]);
            r->box_step = r->k;
        }
        if (s.ncells > s.ncells_cap) {
            err = "cell grid outgrew its reservation";
            return RBSOG_EBOX;
        }
        rbsog::SysStep &t = s.stp;
        t.step = static_cast<uint32_t>(r->k);
        t.fx = r->d_frc;
        t.fy = r->d_frc + r->n;
        t.fz = r->d_frc + 2 * r->n;
    }
    bt.want_energy = sv->energy;
    rc = rbsog::batch_upload(bt, err);
    if (rc) return rc;
    e = rbsog::launch_sample(bt);
    if (e == hipSuccess) e = rbsog::launch_bin_and_sort(bt);
    if (e == hipSuccess) e = rbsog::launch_pair(bt);
    if (e == hipSuccess) e = rbsog::launch_kspace(bt);
    if (e != hipSuccess) {
        err = std::string("step launch: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    return RBSOG_OK;
}

// A launched tick whose results the worker has not read yet.
struct Tick {
    std::vector<Request *> reqs;   // batch order: request i's results are slot entry i
    std::vector<int> steps;        // each request's step index in this tick
    std::vector<Request *> finished;  // completed by it, forces copied into their own buffers
    std::vector<std::pair<Request *, size_t>> outbox;  // completed by it, forces in its download staging slot
    int slot = 0;                  // results and download staging slot
};

// Make reqs the batch and launch their step (each at its own step index).
int start_tick(rbsog_server *sv, const std::vector<Request *> &reqs, int slot, Tick &t, std::string &err)
{
    std::vector<System *> sys;
    for (Request *r : reqs) sys.push_back(&r->sys);
    bool same = sv->batch.sys.size() == sys.size();
    for (size_t i = 0; same && i < sys.size(); ++i) same = sv->batch.sys[i] == sys[i];
    if (!same) {
        const int rc = rbsog::batch_set_systems(sv->batch, sys, err);
        if (rc) return rc;
    }
    sv->active = reqs;
    t = Tick{};
    t.reqs = reqs;
    for (Request *r : reqs) t.steps.push_back(r->k);
    t.slot = slot;
    return tick_launch(sv, err);
}

// Queue behind the tick the copies of the forces of the requests it completes
// (into its pinned download staging slot while that has room, else into the
// requests' pageable buffers) and of its results, then mark the tick's end.
int queue_tick_outputs(rbsog_server *sv, Tick &t, std::string &err)
{
    char *stage = sv->dstage ? sv->dstage + t.slot * kStageBytes : nullptr;
    size_t used = 0;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < t.reqs.size() && e == hipSuccess; ++i) {
        Request *r = t.reqs[i];
        if (t.steps[i] + 1 < r->nsteps) continue;
        const int64_t n = r->n;
        const size_t bytes = 3 * n * sizeof(double);
        if (stage && used + bytes <= kStageBytes) {
            e = hipMemcpyAsync(stage + used, r->d_frc, bytes, hipMemcpyDeviceToHost, sv->stream);
            t.outbox.emplace_back(r, used);
            used += align_up(bytes);
            continue;
        }
        r->fx.resize(n);
        r->fy.resize(n);
        r->fz.resize(n);
        e = hipMemcpyAsync(r->fx.data(), r->d_frc, n * sizeof(double), hipMemcpyDeviceToHost, sv->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->fy.data(), r->d_frc + n, n * sizeof(double), hipMemcpyDeviceToHost, sv->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->fz.data(), r->d_frc + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost,
                               sv->stream);
        t.finished.push_back(r);
    }
    // the slot's last copy ran before the tick that used it was read
    if (e == hipSuccess && sv->res_cap[t.slot] < t.reqs.size()) {
        if (sv->h_tres[t.slot]) (void)hipHostFree(sv->h_tres[t.slot]);
        sv->h_tres[t.slot] = nullptr;
        sv->res_cap[t.slot] = 0;
        const size_t cap = std::max<size_t>(2 * t.reqs.size(), 64);
        e = hipHostMalloc(reinterpret_cast<void **>(&sv->h_tres[t.slot]), cap * sizeof(rbsog::StepResults));
        if (e == hipSuccess) sv->res_cap[t.slot] = cap;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(sv->h_tres[t.slot], sv->batch.d_res, t.reqs.size() * sizeof(rbsog::StepResults),
                           hipMemcpyDeviceToHost, sv->stream);
    if (e == hipSuccess) e = hipEventRecord(sv->tick_ev[t.slot], sv->stream);
    if (e != hipSuccess) {
        err = std::string("tick outputs: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    return RBSOG_OK;
}

// Wait for the tick's end and record its results.
int record_tick(rbsog_server *sv, const Tick &t, double &atom_steps, std::string &err)
{
    const hipError_t e = hipEventSynchronize(sv->tick_ev[t.slot]);
    if (e != hipSuccess) {
        err = std::string("tick: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    const bool shared = t.reqs.size() > 1;
    for (size_t i = 0; i < t.reqs.size(); ++i) {
        Request *r = t.reqs[i];
        const int k = t.steps[i];
        const rbsog::StepResults &res = sv->h_tres[t.slot][i];
        if (res.status != 0) {
            err = "sampler found no nonzero initial state";
            return RBSOG_EDEVICE;
        }
        for (int c = 0; c < 9; ++c) r->P[9 * k + c] = res.Ptot[c];
        if (sv->energy) {
            r->U[3 * k] = res.UN;
            r->U[3 * k + 1] = res.UF;
            r->U[3 * k + 2] = res.Uself;
        }
        r->shared_ticks += shared;
        atom_steps += static_cast<double>(r->n);
    }
    return RBSOG_OK;
}

// Hand forces staged in download slot `slot` to their requests and complete them.
void deliver(rbsog_server *sv, std::vector<std::pair<Request *, size_t>> &outbox, int slot)
{
    if (outbox.empty()) return;
    const char *stage = sv->dstage + slot * kStageBytes;
    for (auto &[r, off] : outbox) {
        const double *f = reinterpret_cast<const double *>(stage + off);
        const int64_t n = r->n;
        r->fx.assign(f, f + n);
        r->fy.assign(f + n, f + 2 * n);
        r->fz.assign(f + 2 * n, f + 3 * n);
    }
    const Clock::time_point t = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto &[r, off] : outbox) {
            r->t_done = t;
            r->done = true;
            sv->completed += 1;
        }
    }
    outbox.clear();
    sv->cv_done.notify_all();
}

// Ticks are pipelined: while tick k runs, the worker hands over the forces
// tick k - 1 completed, admits the requests that arrived (their uploads
// queued behind tick k), queues tick k's force and result copies, and
// launches tick k + 1 (the requests that continue, at their next step, and
// the admitted ones) before it waits for tick k's end.  The device thus
// always has the next tick queued while the host reads the last one.  Only
// an idle server admits before launching.
void worker_main(rbsog_server *sv)
{
    (void)hipSetDevice(sv->device);
    std::string err;
    Tick cur;              // the tick in flight, when running
    bool running = false;
    std::vector<std::pair<Request *, size_t>> handover;  // forces staged by the last read tick
    int handover_slot = 0, next_slot = 0;
    for (;;) {
        const Clock::time_point t0 = Clock::now();
        int rc = RBSOG_OK;
        double admit_s = 0.0, launch_s = 0.0, wait_s = 0.0, atom_steps = 0.0;
        std::vector<Request *> admitted;
        if (!running) {
            deliver(sv, handover, handover_slot);
            sv->stage_used = 0;  // nothing is in flight
            cur = Tick{};
            {
                std::unique_lock<std::mutex> lk(sv->mu);
                sv->cv_work.wait(lk, [&] { return sv->stop || !sv->pending.empty(); });
                if (sv->stop) break;
                take_admissions(sv, 0, admitted);
            }
            if (admitted.empty()) continue;  // (an empty pool holds the queue's head)
            for (Request *r : admitted)
                if (rc == RBSOG_OK) rc = admit(sv, r, err);  // stream order puts the uploads before the step
            const Clock::time_point ta = Clock::now();
            admit_s += std::chrono::duration<double>(ta - t0).count();
            if (rc == RBSOG_OK) rc = start_tick(sv, admitted, next_slot, cur, err);
            launch_s += std::chrono::duration<double>(Clock::now() - ta).count();
            next_slot ^= 1;
            running = rc == RBSOG_OK;
        }
        Tick nxt;
        bool launched = false;
        std::vector<Request *> next;
        if (rc == RBSOG_OK) {
            const Clock::time_point tb = Clock::now();
            deliver(sv, handover, handover_slot);  // while the tick runs
            size_t completing = 0;
            for (size_t i = 0; i < cur.reqs.size(); ++i) completing += cur.steps[i] + 1 >= cur.reqs[i]->nsteps;
            bool stopping = false;
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                stopping = sv->stop;  // finish the tick in flight, launch and admit nothing more
                if (!stopping) take_admissions(sv, cur.reqs.size() - completing, next);
            }
            for (Request *r : next)
                if (rc == RBSOG_OK) rc = admit(sv, r, err);  // behind the tick in flight
            // the next step's box, cell grid, normalisation sums and start
            // bounds of every request that continues (the tick's SysStep is
            // already in its upload buffer, so the host copy is free to change)
            for (size_t i = 0; i < cur.reqs.size(); ++i) {
                Request *r = cur.reqs[i];
                if (cur.steps[i] + 1 < r->nsteps) {
                    rbsog::system_set_box(r->sys, &r->boxes[3 * (cur.steps[i] + 1)]);
                    r->box_step = cur.steps[i] + 1;
                }
            }
            if (rc == RBSOG_OK) rc = queue_tick_outputs(sv, cur, err);
            const Clock::time_point tl = Clock::now();
            admit_s += std::chrono::duration<double>(tl - tb).count();
            // the next tick: continuing requests at their next step, then the admitted ones
            std::vector<Request *> reqs;
            for (size_t i = 0; i < cur.reqs.size(); ++i)
                if (cur.steps[i] + 1 < cur.reqs[i]->nsteps) {
                    cur.reqs[i]->k = cur.steps[i] + 1;
                    reqs.push_back(cur.reqs[i]);
                }
            reqs.insert(reqs.end(), next.begin(), next.end());
            if (rc == RBSOG_OK && !reqs.empty() && !stopping) {
                rc = start_tick(sv, reqs, next_slot, nxt, err);
                launched = rc == RBSOG_OK;
            }
            const Clock::time_point tw = Clock::now();
            launch_s += std::chrono::duration<double>(tw - tl).count();
            if (rc == RBSOG_OK) rc = record_tick(sv, cur, atom_steps, err);
            wait_s = std::chrono::duration<double>(Clock::now() - tw).count();
        }
        const Clock::time_point t1 = Clock::now();
        if (rc == RBSOG_OK) {
            // the tick's end covers the uploads queued before and behind it
            // (and every copy out of the upload staging)
            sv->stage_used = 0;
            uploads_done(admitted, t1);
            uploads_done(next, t1);
            for (Request *r : cur.finished) sv->pool.release(r->off, r->bytes);
            for (auto &ro : cur.outbox) sv->pool.release(ro.first->off, ro.first->bytes);
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->busy_s += std::chrono::duration<double>(t1 - t0).count();
        sv->phase_s[0] += admit_s;
        sv->phase_s[1] += launch_s;
        sv->phase_s[2] += wait_s;
        sv->atom_steps += atom_steps;
        sv->ticks += 1;
        sv->peak_active = std::max<int64_t>(sv->peak_active, static_cast<int64_t>(cur.reqs.size()));
        if (rc != RBSOG_OK) {
            // a failed tick fails every request it held, launched or had
            // admitted; the worker stops once nothing queued still reads
            // their host copies
            (void)hipStreamSynchronize(sv->stream);
            sv->worker_err = err;
            for (const std::vector<Request *> *v : {&cur.reqs, &nxt.reqs, &admitted, &next})
                for (Request *r : *v) {
                    r->status = rc;
                    r->done = true;
                }
            sv->active.clear();
            sv->cv_done.notify_all();
            break;
        }
        for (Request *r : cur.finished) {
            r->t_done = t1;
            r->done = true;
            sv->completed += 1;
        }
        if (!cur.finished.empty()) sv->cv_done.notify_all();
        handover.swap(cur.outbox);  // handed over while the next tick runs, or before waiting for work
        handover_slot = cur.slot;
        if (launched) {
            cur = std::move(nxt);
            next_slot ^= 1;
        } else {
            sv->active.clear();
        }
        running = launched;
    }
    deliver(sv, handover, handover_slot);
}

}  // namespace

extern "C" {

int rbsog_server_create(int32_t precision, int64_t pool_bytes, int32_t max_active, void *hip_stream,
                        rbsog_server **out)
{
    if (!out) return RBSOG_EINVAL;
    *out = nullptr;
    if ((precision != RBSOG_PREC_FP32C && precision != RBSOG_PREC_FP64) || pool_bytes <= 0 || max_active < 1 ||
        max_active > 65536)
        return RBSOG_EINVAL;
    rbsog_server *sv = new (std::nothrow) rbsog_server;
    if (!sv) return RBSOG_ENOMEM;
    sv->precision = precision;
    sv->pool_bytes = static_cast<size_t>(pool_bytes);
    sv->max_active = max_active;
    sv->stream = static_cast<hipStream_t>(hip_stream);
    std::string err;
    int rc = rbsog::batch_init(sv->batch, sv->stream, precision, err);
    if (rc == RBSOG_OK && hipGetDevice(&sv->device) != hipSuccess) rc = RBSOG_EDEVICE;
    if (rc == RBSOG_OK && hipMalloc(reinterpret_cast<void **>(&sv->pool_mem), sv->pool_bytes) != hipSuccess) {
        (void)hipGetLastError();
        rc = RBSOG_ENOMEM;
    }
    if (rc == RBSOG_OK && hipHostMalloc(reinterpret_cast<void **>(&sv->stage), kStageBytes) != hipSuccess) {
        (void)hipGetLastError();  // uploads then come from the requests' own buffers
        sv->stage = nullptr;
    }
    if (rc == RBSOG_OK && hipHostMalloc(reinterpret_cast<void **>(&sv->dstage), 2 * kStageBytes) != hipSuccess) {
        (void)hipGetLastError();  // forces then go straight to the requests' own buffers
        sv->dstage = nullptr;
    }
    for (hipEvent_t &e : sv->tick_ev)
        if (rc == RBSOG_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = RBSOG_EDEVICE;
    if (rc != RBSOG_OK) {
        rbsog::batch_free(sv->batch);
        delete sv;
        return rc;
    }
    sv->pool.reset(sv->pool_bytes);
    sv->worker = std::thread(worker_main, sv);
    *out = sv;
    return RBSOG_OK;
}

int rbsog_server_set_energy(rbsog_server *sv, int32_t on)
{
    if (!sv) return RBSOG_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->submitted > 0) {
        sv->err = "the energy setting is fixed once a request was submitted";
        return RBSOG_ESTATE;
    }
    sv->energy = on != 0;
    return RBSOG_OK;
}

int rbsog_server_submit(rbsog_server *sv, const rbsog_params *params, int64_t n, const double *host_q,
                        const double *host_x, const double *host_y, const double *host_z, const double host_box[3],
                        int32_t nsteps, double growth, int64_t *ticket)
{
    if (!sv) return RBSOG_EINVAL;
    if (!params || !host_q || !host_x || !host_y || !host_z || !host_box || !ticket || nsteps < 1 ||
        !std::isfinite(growth)) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->err = "null argument or bad step count";
        return RBSOG_EINVAL;
    }
    if (params->precision != sv->precision) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->err = "request precision differs from the server's";
        return RBSOG_EINVAL;
    }
    std::unique_ptr<Request> r(new (std::nothrow) Request);
    if (!r) return RBSOG_ENOMEM;
    std::string err;
    int rc = rbsog::system_init(r->sys, *params, n, host_q, host_box, err);
    // boxes of every step: L_k = L_{k-1} mu_k, mu_k = (1 + g k)/(1 + g (k - 1))
    if (rc == RBSOG_OK) {
        r->boxes.resize(3 * static_cast<size_t>(nsteps));
        r->mus.resize(nsteps);
        double L[3] = {host_box[0], host_box[1], host_box[2]};
        for (int k = 0; k < nsteps && rc == RBSOG_OK; ++k) {
            const double m = k == 0 ? 1.0 : (1.0 + growth * k) / (1.0 + growth * (k - 1));
            if (!(m > 0.0) || !std::isfinite(m)) {
                err = "box law gives a non-positive scale factor";
                rc = RBSOG_EINVAL;
                break;
            }
            r->mus[k] = m;
            for (int d = 0; d < 3; ++d) {
                if (k > 0) L[d] *= m;
                r->boxes[3 * k + d] = L[d];
            }
            rc = rbsog::check_box(L, params->rc, err);
            r->max_cells = std::max(r->max_cells, rbsog::cells_for_box(L, params->rc));
        }
    }
    if (rc == RBSOG_OK) {
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(host_x[i]) || !std::isfinite(host_y[i]) || !std::isfinite(host_z[i])) {
                err = "positions have NaN/Inf";
                rc = RBSOG_EINVAL;
                break;
            }
    }
    if (rc == RBSOG_OK) {
        r->bytes = request_bytes(r->sys.prm, n, r->max_cells);
        if (r->bytes > sv->pool_bytes) {
            err = "request needs more device memory than the pool holds";
            rc = RBSOG_EAGAIN;
        }
    }
    if (rc != RBSOG_OK) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->err = err;
        return rc;
    }
    r->n = n;
    r->nsteps = nsteps;
    r->growth = growth;
    r->q.assign(host_q, host_q + n);
    r->x.assign(host_x, host_x + n);
    r->y.assign(host_y, host_y + n);
    r->z.assign(host_z, host_z + n);
    r->P.assign(9 * static_cast<size_t>(nsteps), 0.0);
    r->U.assign(3 * static_cast<size_t>(nsteps), 0.0);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop || !sv->worker_err.empty()) {
        sv->err = "server is stopped: " + sv->worker_err;
        return RBSOG_ESTATE;
    }
    r->ticket = sv->next_ticket++;
    r->t_submit = Clock::now();
    *ticket = r->ticket;
    sv->pending.push_back(r.get());
    sv->requests.emplace(r->ticket, std::move(r));
    sv->submitted += 1;
    sv->cv_work.notify_one();
    return RBSOG_OK;
}

int rbsog_server_wait(rbsog_server *sv, int64_t ticket, double timeout_s, double *host_fx, double *host_fy,
                      double *host_fz, double *host_P, double *host_energy, double *host_times)
{
    if (!sv) return RBSOG_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) {
        sv->err = "unknown ticket";
        return RBSOG_EINVAL;
    }
    Request *r = it->second.get();
    auto ready = [&] { return r->done; };
    if (timeout_s < 0) {
        sv->cv_done.wait(lk, ready);
    } else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return RBSOG_EAGAIN;
    }
    if (r->status != RBSOG_OK) {
        sv->err = "request failed: " + sv->worker_err;
        const int st = r->status;
        sv->requests.erase(it);
        return st;
    }
    const int64_t n = r->n;
    if (host_fx) std::memcpy(host_fx, r->fx.data(), n * sizeof(double));
    if (host_fy) std::memcpy(host_fy, r->fy.data(), n * sizeof(double));
    if (host_fz) std::memcpy(host_fz, r->fz.data(), n * sizeof(double));
    if (host_P) std::memcpy(host_P, r->P.data(), r->P.size() * sizeof(double));
    if (host_energy) std::memcpy(host_energy, r->U.data(), r->U.size() * sizeof(double));
    if (host_times) {
        host_times[0] = std::chrono::duration<double>(r->t_admit - r->t_submit).count();
        host_times[1] = std::chrono::duration<double>(r->t_done - r->t_submit).count();
        host_times[2] = r->shared_ticks;
    }
    sv->requests.erase(it);
    return RBSOG_OK;
}

int rbsog_server_stats(rbsog_server *sv, double *host_stats)
{
    if (!sv || !host_stats) return RBSOG_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    host_stats[0] = static_cast<double>(sv->submitted);
    host_stats[1] = static_cast<double>(sv->completed);
    host_stats[2] = static_cast<double>(sv->ticks);
    host_stats[3] = sv->atom_steps;
    host_stats[4] = sv->busy_s;
    host_stats[5] = static_cast<double>(sv->peak_active);
    host_stats[6] = static_cast<double>(sv->pool.peak());
    host_stats[7] = static_cast<double>(sv->pending.size());
    host_stats[8] = sv->phase_s[0];
    host_stats[9] = sv->phase_s[1];
    host_stats[10] = sv->phase_s[2];
    return RBSOG_OK;
}

int rbsog_server_destroy(rbsog_server *sv)
{
    if (!sv) return RBSOG_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    (void)hipStreamSynchronize(sv->stream);
    rbsog::batch_free(sv->batch);
    if (sv->pool_mem) (void)hipFree(sv->pool_mem);
    if (sv->stage) (void)hipHostFree(sv->stage);
    if (sv->dstage) (void)hipHostFree(sv->dstage);
    for (int k = 0; k < 2; ++k) {
        if (sv->h_tres[k]) (void)hipHostFree(sv->h_tres[k]);
        if (sv->tick_ev[k]) (void)hipEventDestroy(sv->tick_ev[k]);
    }
    delete sv;
    return RBSOG_OK;
}

const char *rbsog_server_last_error(const rbsog_server *sv) { return sv ? sv->err.c_str() : "null server"; }

}  // extern "C"
