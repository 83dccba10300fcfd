// C ABI of the RBSOG library, single-system entry points: a context is one
// system evaluated as a batch of one, so it runs exactly the kernels (and
// gives exactly the results) of the batched and served forms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "rbsog_impl.hpp"

using rbsog::Batch;
using rbsog::System;

namespace {

// Table 1, row 2 (r_c = 9 A): the parameter set used in all of the paper's runs.
constexpr double kRow2B = 1.62976708826776469;
constexpr double kRow2Sigma9 = 3.270345668108471;
constexpr double kRow2Omega = 1.007806979343806;

int fail(rbsog_ctx *c, int code, const char *msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(rbsog_ctx *c, hipError_t e, const char *where)
{
    if (c) c->err = std::string(where) + ": " + hipGetErrorString(e);
    return RBSOG_EDEVICE;
}

#define HIP_TRY(c, call)                                     \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
    } while (0)

#define RB_TRY(call)              \
    do {                          \
        int r_ = (call);          \
        if (r_ != RBSOG_OK) return r_; \
    } while (0)

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

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

void destroy(rbsog_ctx *c)
{
    if (c->sys.atom_mem) (void)hipStreamSynchronize(c->batch.stream);
    rbsog::system_free(c->sys);
    rbsog::batch_free(c->batch);
    if (c->d_stage) (void)hipFree(c->d_stage);
    if (c->h_ring) (void)hipHostFree(c->h_ring);
    for (hipEvent_t e : c->ring_ev)
        if (e) (void)hipEventDestroy(e);
    for (double *p : {c->npt.d_mass, c->npt.d_F, c->npt.d_part, c->npt.d_kin})
        if (p) (void)hipFree(p);
    delete c;
}

// grid for the current box: more cells than allocated re-carve the cell part
int refresh_cells(rbsog_ctx *c)
{
    bool recarved = false;
    RB_TRY(rbsog::system_ensure_cells(c->sys, c->err, &recarved));
    if (recarved) {
        c->batch.desc_dirty = true;
        c->desc_moved = true;
    }
    return RBSOG_OK;
}

// results of the last evaluation on the host: the context's own, or those a
// batch of contexts left for it
int fetch(rbsog_ctx *c)
{
    if (c->res_from_batch) return RBSOG_OK;
    return rbsog::batch_fetch_results(c->batch, c->err);
}

// calls that launch the context's own work are refused while it is admitted
int own_work(rbsog_ctx *c)
{
    if (c->in_batch) return fail(c, RBSOG_ESTATE, "the context is admitted to a batch (rbsog_stage, rbsog_batch_step)");
    c->res_from_batch = false;
    return RBSOG_OK;
}

}  // namespace

extern "C" {

int rbsog_version(void) { return 10100; }

const char *rbsog_strerror(int code)
{
    switch (code) {
    case RBSOG_OK: return "ok";
    case RBSOG_EINVAL: return "invalid argument";
    case RBSOG_ENEUTRAL: return "charges are not neutral";
    case RBSOG_EBOX: return "invalid box for the cutoff";
    case RBSOG_ENOMEM: return "out of memory";
    case RBSOG_EDEVICE: return "HIP device error";
    case RBSOG_ESTATE: return "call out of order";
    case RBSOG_EAGAIN: return "admission refused";
    default: return "unknown error";
    }
}

const char *rbsog_last_error(const rbsog_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int rbsog_params_init(rbsog_params *p, double rc)
{
    if (!p || !(rc > 0) || !std::isfinite(rc)) return RBSOG_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->b = kRow2B;
    p->sigma = kRow2Sigma9 * rc / 9.0;
    p->omega = kRow2Omega;
    p->M = 10;
    p->rc = rc;
    p->P = 100;
    p->seed = 0;
    p->system_id = 0;
    p->coulomb_k = 1.0;
    p->precision = RBSOG_PREC_FP32C;
    p->recalibration = RBSOG_RECAL_EXCHANGE;
    return RBSOG_OK;
}

int rbsog_setup(const rbsog_params *params, int64_t n, const double *host_q, const double host_box[3],
                void *hip_stream, rbsog_ctx **out)
{
    if (!out) return RBSOG_EINVAL;
    *out = nullptr;
    if (!params || !host_q || !host_box) return RBSOG_EINVAL;
    rbsog_ctx *c = new (std::nothrow) rbsog_ctx;
    if (!c) return RBSOG_ENOMEM;
    int rc = rbsog::system_init(c->sys, *params, n, host_q, host_box, c->err);
    if (rc == RBSOG_OK)
        rc = rbsog::batch_init(c->batch, static_cast<hipStream_t>(hip_stream), params->precision, c->err);
    if (rc == RBSOG_OK) rc = rbsog::system_alloc(c->sys, c->err);
    if (rc == RBSOG_OK) rc = rbsog::system_upload_q(c->sys, host_q, c->batch.stream, c->err);
    if (rc == RBSOG_OK) rc = rbsog::batch_set_systems(c->batch, {&c->sys}, c->err);
    if (rc != RBSOG_OK) {
        destroy(c);
        return rc;
    }
    *out = c;
    return RBSOG_OK;
}

static int sample_tail(rbsog_ctx *c, int64_t step, int32_t *host_m_r, int32_t *host_m_nr, double host_S[2]);

int rbsog_sample_modes(rbsog_ctx *c, int64_t step, const double host_box[3], int32_t *host_m_r,
                       int32_t *host_m_nr, double host_S[2])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    RB_TRY(own_work(c));
    if (step < 0 || (step >> 32)) return fail(c, RBSOG_EINVAL, "step must be in [0, 2^32)");
    RB_TRY(rbsog::check_box(host_box, c->sys.prm.rc, c->err));
    rbsog::system_set_box(c->sys, host_box);
    return sample_tail(c, step, host_m_r, host_m_nr, host_S);
}

int rbsog_sample_modes_cell(rbsog_ctx *c, int64_t step, const double host_h[9], int32_t *host_m_r,
                            int32_t *host_m_nr, double host_S[2])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    RB_TRY(own_work(c));
    if (!host_h) return fail(c, RBSOG_EINVAL, "cell tensor is NULL");
    if (step < 0 || (step >> 32)) return fail(c, RBSOG_EINVAL, "step must be in [0, 2^32)");
    const bool had_table = c->sys.gl_mem != nullptr;
    RB_TRY(rbsog::system_set_cell(c->sys, host_h, c->err));
    if (c->sys.gl_mem && !had_table) c->batch.desc_dirty = true;  // the descriptor now points at the table
    return sample_tail(c, step, host_m_r, host_m_nr, host_S);
}

static int sample_tail(rbsog_ctx *c, int64_t step, int32_t *host_m_r, int32_t *host_m_nr, double host_S[2])
{
    RB_TRY(refresh_cells(c));
    c->sys.stp.step = static_cast<uint32_t>(step);
    RB_TRY(rbsog::batch_upload(c->batch, c->err));
    HIP_TRY(c, rbsog::launch_sample(c->batch));
    if (host_m_r || host_m_nr) {
        const int64_t P = c->sys.prm.P;
        RB_TRY(rbsog::batch_fetch_results(c->batch, c->err));
        if (host_m_r)
            HIP_TRY(c, hipMemcpy(host_m_r, c->sys.desc.mraw, 3 * P * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (host_m_nr)
            HIP_TRY(c, hipMemcpy(host_m_nr, c->sys.desc.mraw + 3 * P, 3 * P * sizeof(int32_t),
                                 hipMemcpyDeviceToHost));
        if (c->batch.h_res[0].status != 0) return fail(c, RBSOG_EDEVICE, "sampler: no start draw accepted");
    }
    if (host_S) {
        host_S[0] = c->sys.Sr;
        host_S[1] = c->sys.Snr;
    }
    c->state = 1;
    return RBSOG_OK;
}

int rbsog_force_virial(rbsog_ctx *c, const double *x, const double *y, const double *z, double *fx, double *fy,
                       double *fz, double host_energy[3], double host_vir[6])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    RB_TRY(own_work(c));
    if (!x || !y || !z || !fx || !fy || !fz) return fail(c, RBSOG_EINVAL, "null position or force array");
    if (c->state < 1) return fail(c, RBSOG_ESTATE, "rbsog_sample_modes must precede rbsog_force_virial");
    const int64_t n = c->sys.n;
    hipStream_t st = c->batch.stream;
    const int din = is_device_ptr(x) + is_device_ptr(y) + is_device_ptr(z);
    const int dout = is_device_ptr(fx) + is_device_ptr(fy) + is_device_ptr(fz);
    if (din % 3 || dout % 3)
        return fail(c, RBSOG_EINVAL, "x, y, z (and fx, fy, fz) must be all host or all device arrays");
    const bool dev_in = din == 3, dev_out = dout == 3;
    const double *px = x, *py = y, *pz = z;
    double *gx = fx, *gy = fy, *gz = fz;
    if ((!dev_in || !dev_out) && !c->d_stage) HIP_TRY(c, hipMalloc(&c->d_stage, 6 * n * sizeof(double)));
    if (!dev_in) {
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(z[i]))
                return fail(c, RBSOG_EINVAL, "positions have NaN/Inf");
        HIP_TRY(c, hipMemcpyAsync(c->d_stage, x, n * sizeof(double), hipMemcpyHostToDevice, st));
        HIP_TRY(c, hipMemcpyAsync(c->d_stage + n, y, n * sizeof(double), hipMemcpyHostToDevice, st));
        HIP_TRY(c, hipMemcpyAsync(c->d_stage + 2 * n, z, n * sizeof(double), hipMemcpyHostToDevice, st));
        px = c->d_stage;
        py = c->d_stage + n;
        pz = c->d_stage + 2 * n;
    }
    if (!dev_out) {
        gx = c->d_stage + 3 * n;
        gy = c->d_stage + 4 * n;
        gz = c->d_stage + 5 * n;
    }
    rbsog::SysStep &t = c->sys.stp;
    t.x = px;
    t.y = py;
    t.z = pz;
    t.fx = gx;
    t.fy = gy;
    t.fz = gz;
    c->batch.want_energy = host_energy != nullptr;
    RB_TRY(rbsog::batch_upload(c->batch, c->err));
    HIP_TRY(c, rbsog::launch_bin_and_sort(c->batch));
    HIP_TRY(c, rbsog::launch_pair(c->batch));
    HIP_TRY(c, rbsog::launch_kspace(c->batch));
    if (!dev_out) {
        HIP_TRY(c, hipMemcpyAsync(fx, gx, n * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipMemcpyAsync(fy, gy, n * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipMemcpyAsync(fz, gz, n * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    c->state = 2;
    if (host_energy || host_vir || !dev_out) {
        RB_TRY(rbsog::batch_fetch_results(c->batch, c->err));
        const rbsog::StepResults &r = c->batch.h_res[0];
        if (r.status != 0) return fail(c, RBSOG_EDEVICE, "sampler: no start draw accepted");
        if (r.bad_input) return fail(c, RBSOG_EINVAL, "positions have NaN/Inf");
        if (host_energy) {
            host_energy[0] = r.UN;
            host_energy[1] = r.UF;
            host_energy[2] = r.Uself;
        }
        if (host_vir)
            for (int k = 0; k < 6; ++k) host_vir[k] = r.vir[k];
    }
    return RBSOG_OK;
}

int rbsog_pressure(rbsog_ctx *c, double host_P[9], double host_parts[27])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (!host_P) return fail(c, RBSOG_EINVAL, "null pressure output");
    if (c->state < 2) return fail(c, RBSOG_ESTATE, "rbsog_force_virial must precede rbsog_pressure");
    RB_TRY(fetch(c));
    const rbsog::StepResults &r = c->batch.h_res[0];
    if (r.status != 0) return fail(c, RBSOG_EDEVICE, "sampler: no start draw accepted");
    if (r.bad_input) return fail(c, RBSOG_EINVAL, "positions have NaN/Inf");
    for (int k = 0; k < 9; ++k) host_P[k] = r.Ptot[k];
    if (host_parts)
        for (int k = 0; k < 9; ++k) {
            host_parts[k] = r.PN[k];
            host_parts[9 + k] = r.Pr[k];
            host_parts[18 + k] = r.Pnr[k];
        }
    return RBSOG_OK;
}

int rbsog_rescale(rbsog_ctx *c, const double host_mu[3], double *x, double *y, double *z, double host_box[3])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    RB_TRY(own_work(c));
    if (!host_mu || !host_box || !x || !y || !z) return fail(c, RBSOG_EINVAL, "null argument");
    if (!finite3(host_mu) || host_mu[0] <= 0 || host_mu[1] <= 0 || host_mu[2] <= 0)
        return fail(c, RBSOG_EINVAL, "scale factors must be positive and finite");
    if (!(is_device_ptr(x) && is_device_ptr(y) && is_device_ptr(z)))
        return fail(c, RBSOG_EINVAL, "rbsog_rescale needs device position arrays");
    if (c->sys.tri)
        return fail(c, RBSOG_ESTATE, "rbsog_rescale scales a box; a general cell is passed to rbsog_sample_modes_cell");
    rbsog::SysStep &t = c->sys.stp;
    for (int d = 0; d < 3; ++d) t.mu[d] = host_mu[d];
    t.x = x;
    t.y = y;
    t.z = z;
    RB_TRY(rbsog::batch_upload(c->batch, c->err));
    HIP_TRY(c, rbsog::launch_rescale(c->batch));
    for (int d = 0; d < 3; ++d) host_box[d] *= host_mu[d];
    return RBSOG_OK;
}

// The work of rbsog_step up to its last launch (no synchronisation).
static int step_queue(rbsog_ctx *c, int64_t step, const double host_mu[3], double host_box[3], double *x, double *y,
                      double *z, double *fx, double *fy, double *fz, bool energy)
{
    RB_TRY(own_work(c));
    if (!host_box || !x || !y || !z || !fx || !fy || !fz) return fail(c, RBSOG_EINVAL, "null argument");
    if (step < 0 || (step >> 32)) return fail(c, RBSOG_EINVAL, "step must be in [0, 2^32)");
    if (c->sys.tri)
        return fail(c, RBSOG_ESTATE, "rbsog_step takes a box; a general cell is passed to rbsog_sample_modes_cell");
    if (!(is_device_ptr(x) && is_device_ptr(y) && is_device_ptr(z) && is_device_ptr(fx) && is_device_ptr(fy) &&
          is_device_ptr(fz)))
        return fail(c, RBSOG_EINVAL, "rbsog_step needs device position and force arrays");
    double box[3] = {host_box[0], host_box[1], host_box[2]};
    if (host_mu) {
        if (!finite3(host_mu) || host_mu[0] <= 0 || host_mu[1] <= 0 || host_mu[2] <= 0)
            return fail(c, RBSOG_EINVAL, "scale factors must be positive and finite");
        for (int d = 0; d < 3; ++d) box[d] *= host_mu[d];
    }
    RB_TRY(rbsog::check_box(box, c->sys.prm.rc, c->err));
    rbsog::SysStep &t = c->sys.stp;
    if (host_mu)
        for (int d = 0; d < 3; ++d) t.mu[d] = host_mu[d];
    rbsog::system_set_box(c->sys, box);
    RB_TRY(refresh_cells(c));
    t.step = static_cast<uint32_t>(step);
    t.x = x;
    t.y = y;
    t.z = z;
    t.fx = fx;
    t.fy = fy;
    t.fz = fz;
    c->batch.want_energy = energy;
    // one upload; the rescale and the binning are queued before the sampler
    // (second stream), which waits only for the upload
    RB_TRY(rbsog::batch_upload(c->batch, c->err));
    HIP_TRY(c, rbsog::record_sample_fence(c->batch));
    if (host_mu) HIP_TRY(c, rbsog::launch_rescale(c->batch));
    HIP_TRY(c, rbsog::launch_bin_and_sort(c->batch));
    HIP_TRY(c, rbsog::launch_sample_fenced(c->batch));
    HIP_TRY(c, rbsog::launch_pair(c->batch));
    HIP_TRY(c, rbsog::launch_kspace(c->batch));
    for (int d = 0; d < 3; ++d) host_box[d] = box[d];
    c->state = 2;
    return RBSOG_OK;
}

int rbsog_step(rbsog_ctx *c, int64_t step, const double host_mu[3], double host_box[3], double *x, double *y,
               double *z, double *fx, double *fy, double *fz, double host_P[9], double host_energy[3])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    RB_TRY(step_queue(c, step, host_mu, host_box, x, y, z, fx, fy, fz, host_energy != nullptr));
    if (host_P || host_energy) {
        RB_TRY(rbsog::batch_fetch_results(c->batch, c->err));
        const rbsog::StepResults &r = c->batch.h_res[0];
        if (r.status != 0) return fail(c, RBSOG_EDEVICE, "sampler: no start draw accepted");
        if (r.bad_input) return fail(c, RBSOG_EINVAL, "positions have NaN/Inf");
        if (host_P)
            for (int k = 0; k < 9; ++k) host_P[k] = r.Ptot[k];
        if (host_energy) {
            host_energy[0] = r.UN;
            host_energy[1] = r.UF;
            host_energy[2] = r.Uself;
        }
    }
    return RBSOG_OK;
}

int rbsog_step_async(rbsog_ctx *c, int64_t step, const double host_mu[3], double host_box[3], double *x,
                     double *y, double *z, double *fx, double *fy, double *fz, int32_t energy, int64_t *ticket)
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (!ticket) return fail(c, RBSOG_EINVAL, "null ticket");
    if (!c->h_ring) {
        HIP_TRY(c, hipHostMalloc(reinterpret_cast<void **>(&c->h_ring),
                                 rbsog_ctx::kResRing * sizeof(rbsog::StepResults)));
        for (hipEvent_t &e : c->ring_ev) HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    // the slot this step's results go to: its last copy must have run
    const int slot = static_cast<int>(c->next_ticket % rbsog_ctx::kResRing);
    if (c->ring_ticket[slot] >= 0) HIP_TRY(c, hipEventSynchronize(c->ring_ev[slot]));
    c->ring_ticket[slot] = -1;
    RB_TRY(step_queue(c, step, host_mu, host_box, x, y, z, fx, fy, fz, energy != 0));
    HIP_TRY(c, hipMemcpyAsync(c->h_ring + slot, c->batch.d_res, sizeof(rbsog::StepResults), hipMemcpyDeviceToHost,
                              c->batch.stream));
    HIP_TRY(c, hipEventRecord(c->ring_ev[slot], c->batch.stream));
    c->ring_ticket[slot] = c->next_ticket;
    *ticket = c->next_ticket++;
    return RBSOG_OK;
}

int rbsog_step_wait(rbsog_ctx *c, int64_t ticket, double host_P[9], double host_energy[3])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (ticket < 0) return fail(c, RBSOG_EINVAL, "negative ticket");
    const int slot = static_cast<int>(ticket % rbsog_ctx::kResRing);
    if (c->ring_ticket[slot] != ticket)
        return fail(c, RBSOG_EINVAL, "no results for this ticket (unknown, or more than 4 steps ago)");
    HIP_TRY(c, hipEventSynchronize(c->ring_ev[slot]));
    const rbsog::StepResults &r = c->h_ring[slot];
    if (r.status != 0) return fail(c, RBSOG_EDEVICE, "sampler: no start draw accepted");
    if (r.bad_input) return fail(c, RBSOG_EINVAL, "positions have NaN/Inf");
    if (host_P)
        for (int k = 0; k < 9; ++k) host_P[k] = r.Ptot[k];
    if (host_energy) {
        host_energy[0] = r.UN;
        host_energy[1] = r.UF;
        host_energy[2] = r.Uself;
    }
    return RBSOG_OK;
}

int rbsog_destroy(rbsog_ctx *c)
{
    if (!c) return RBSOG_OK;
    if (c->in_batch) (void)rbsog_batch_release(c->in_batch, c);
    destroy(c);
    return RBSOG_OK;
}

int rbsog_stage(rbsog_ctx *c, int64_t step, const double host_box[3], const double *x, const double *y,
                const double *z, double *fx, double *fy, double *fz)
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (!c->in_batch) return fail(c, RBSOG_ESTATE, "rbsog_stage needs a context admitted to a batch");
    if (step < 0 || (step >> 32)) return fail(c, RBSOG_EINVAL, "step must be in [0, 2^32)");
    if (!x || !y || !z || !fx || !fy || !fz) return fail(c, RBSOG_EINVAL, "null position or force array");
    if (!(is_device_ptr(x) && is_device_ptr(y) && is_device_ptr(z) && is_device_ptr(fx) && is_device_ptr(fy) &&
          is_device_ptr(fz)))
        return fail(c, RBSOG_EINVAL, "staged position and force arrays must be device memory");
    RB_TRY(rbsog::check_box(host_box, c->sys.prm.rc, c->err));
    rbsog::system_set_box(c->sys, host_box);
    RB_TRY(refresh_cells(c));
    rbsog::SysStep &t = c->sys.stp;
    t.step = static_cast<uint32_t>(step);
    t.x = x;
    t.y = y;
    t.z = z;
    t.fx = fx;
    t.fy = fy;
    t.fz = fz;
    c->staged = true;
    return RBSOG_OK;
}

int rbsog_debug_cells(rbsog_ctx *c, int32_t *host_cell, int32_t host_ncell[3])
{
    if (!c) return RBSOG_EINVAL;
    if (c->in_batch) return fail(c, RBSOG_ESTATE, "the context is admitted to a batch");
    if (c->state < 2) return fail(c, RBSOG_ESTATE, "no evaluation yet");
    HIP_TRY(c, hipStreamSynchronize(c->batch.stream));
    if (host_cell) {
        HIP_TRY(c, hipMemcpy(host_cell, c->sys.desc.cell, c->sys.n * sizeof(int32_t), hipMemcpyDeviceToHost));
        // the device numbers cells z fastest; the interface reports x fastest
        const int nx = c->sys.nc[0], ny = c->sys.nc[1], nz = c->sys.nc[2];
        for (int64_t i = 0; i < c->sys.n; ++i) {
            const int id = host_cell[i];
            const int cz = id % nz, cy = (id / nz) % ny, cx = id / (nz * ny);
            host_cell[i] = cx + nx * (cy + ny * cz);
        }
    }
    if (host_ncell)
        for (int d = 0; d < 3; ++d) host_ncell[d] = c->sys.nc[d];
    return RBSOG_OK;
}

int rbsog_debug_long_range_force(rbsog_ctx *c, double *fx, double *fy, double *fz)
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (c->in_batch) return fail(c, RBSOG_ESTATE, "the context is admitted to a batch");
    if (c->state < 2) return fail(c, RBSOG_ESTATE, "no evaluation yet");
    if (!(is_device_ptr(fx) && is_device_ptr(fy) && is_device_ptr(fz)))
        return fail(c, RBSOG_EINVAL, "rbsog_debug_long_range_force needs device arrays");
    HIP_TRY(c, rbsog::launch_long_range_force(c->batch, fx, fy, fz));
    HIP_TRY(c, hipStreamSynchronize(c->batch.stream));
    return RBSOG_OK;
}

int rbsog_debug_modes(rbsog_ctx *c, int32_t cap, int32_t *host_nd, int32_t *host_modes, int32_t *host_counts,
                      double *host_rho)
{
    if (!c) return RBSOG_EINVAL;
    if (c->in_batch) return fail(c, RBSOG_ESTATE, "the context is admitted to a batch");
    if (c->state < 1) return fail(c, RBSOG_ESTATE, "no sampled modes yet");
    if (cap < 0) return fail(c, RBSOG_EINVAL, "negative capacity");
    RB_TRY(fetch(c));
    const int nd = c->batch.h_res[0].nd;
    const int mcap = c->sys.desc.mcap;
    if (host_nd) *host_nd = nd;
    const int k = std::min(nd, cap);
    if (host_modes && k > 0) {
        std::vector<int4> m(k);
        HIP_TRY(c, hipMemcpy(m.data(), c->sys.desc.modes, k * sizeof(int4), hipMemcpyDeviceToHost));
        for (int d = 0; d < k; ++d) {
            host_modes[3 * d] = m[d].x;
            host_modes[3 * d + 1] = m[d].y;
            host_modes[3 * d + 2] = m[d].z;
        }
    }
    if (host_counts && k > 0) {
        std::vector<int32_t> cn(2 * mcap);
        HIP_TRY(c, hipMemcpy(cn.data(), c->sys.desc.cnt, 2 * mcap * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int d = 0; d < k; ++d) {
            host_counts[2 * d] = cn[d];
            host_counts[2 * d + 1] = cn[mcap + d];
        }
    }
    if (host_rho && k > 0) {
        if (c->state < 2) return fail(c, RBSOG_ESTATE, "rho needs rbsog_force_virial");
        HIP_TRY(c, hipMemcpy(host_rho, c->sys.desc.rho, 2 * k * sizeof(double), hipMemcpyDeviceToHost));
    }
    return RBSOG_OK;
}

int rbsog_step_info(rbsog_ctx *c, int64_t host_info[4])
{
    if (!c || !host_info) return RBSOG_EINVAL;
    if (c->state < 1) return fail(c, RBSOG_ESTATE, "no sampled modes yet");
    RB_TRY(fetch(c));
    const rbsog::StepResults &r = c->batch.h_res[0];
    host_info[0] = r.nd;
    host_info[1] = r.acc_r;
    host_info[2] = r.acc_nr;
    host_info[3] = c->state >= 2 ? static_cast<int64_t>(std::llround(r.npairs)) : 0;
    return RBSOG_OK;
}

int rbsog_set_timing(rbsog_ctx *c, int on)
{
    if (!c) return RBSOG_EINVAL;
    rbsog::batch_set_timing(c->batch, on);
    return RBSOG_OK;
}

int rbsog_get_timing(rbsog_ctx *c, int32_t cap, int32_t *host_nk, char *host_names, double *host_ms,
                     int64_t *host_count)
{
    if (!c) return RBSOG_EINVAL;
    return rbsog::batch_get_timing(c->batch, cap, host_nk, host_names, host_ms, host_count, c->err);
}

}  // extern "C"
