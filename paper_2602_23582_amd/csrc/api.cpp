// C ABI of the RBSOG library: validation, context and buffer management, and
// the per-step entry points declared in include/rbsog.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "rbsog_impl.hpp"

using rbsog::kMaxModes;
using rbsog::kMaxP;
using rbsog::kPairWave;
using rbsog::kSkChunk;

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
    if (c) {
        c->err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return RBSOG_EDEVICE;
}

#define HIP_TRY(c, call)                                 \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
    } while (0)

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

int check_box(rbsog_ctx *c, const double *box, double rc)
{
    if (!box) return fail(c, RBSOG_EINVAL, "box is NULL");
    if (!finite3(box)) return fail(c, RBSOG_EINVAL, "box has NaN/Inf");
    if (box[0] <= 0 || box[1] <= 0 || box[2] <= 0) return fail(c, RBSOG_EBOX, "box edges must be positive");
    const double lmin = std::min(box[0], std::min(box[1], box[2]));
    if (rc > 0.5 * lmin) return fail(c, RBSOG_EBOX, "cutoff exceeds half the shortest box edge");
    return RBSOG_OK;
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

template <class T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T));
}

void free_buffers(rbsog_ctx *c)
{
    void *bufs[] = {c->d_tab, c->d_q, c->d_u, c->d_cell, c->d_count, c->d_cursor, c->d_start, c->d_nblk,
                    c->d_bstart, c->d_scan_tmp, c->d_blocks, c->d_perm_tmp, c->d_perm, c->d_rec, c->d_fsr,
                    c->d_pair_part, c->d_mraw, c->d_modes, c->d_cnt, c->d_rho_part, c->d_rho, c->d_coef,
                    c->d_res, c->d_stage};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (c->h_res) (void)hipHostFree(c->h_res);
    for (auto &t : c->timers) {
        for (auto &e : t.pending) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        for (auto &e : t.pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
    c->timers.clear();
}

// (re)size the per-cell and pair-block buffers for the current grid
int ensure_cells(rbsog_ctx *c)
{
    if (c->ncells > (int64_t)1024 * 1024) return fail(c, RBSOG_EBOX, "more than 2^20 cells: box too large for rc");
    if (c->ncells <= c->ncells_cap) return RBSOG_OK;
    int32_t **arrs[] = {&c->d_count, &c->d_cursor, &c->d_start, &c->d_nblk, &c->d_bstart};
    for (auto a : arrs) {
        if (*a) (void)hipFree(*a);
        *a = nullptr;
        HIP_TRY(c, dalloc(a, c->ncells + 1));
    }
    if (c->d_blocks) (void)hipFree(c->d_blocks);
    if (c->d_pair_part) (void)hipFree(c->d_pair_part);
    c->d_blocks = nullptr;
    c->d_pair_part = nullptr;
    const int64_t pair_grid = (c->n + kPairWave - 1) / kPairWave + c->ncells;
    HIP_TRY(c, dalloc(&c->d_blocks, pair_grid));
    HIP_TRY(c, dalloc(&c->d_pair_part, 8 * pair_grid));
    c->ncells_cap = c->ncells;
    return RBSOG_OK;
}

}  // namespace

namespace rbsog {

void timer_begin(rbsog_ctx *c, const char *name)
{
    if (!c->timing) return;
    Timer *t = nullptr;
    for (auto &x : c->timers)
        if (x.name == name) t = &x;
    if (!t) {
        if (c->timers.size() >= static_cast<size_t>(kMaxTimed)) return;
        c->timers.push_back(Timer{});
        t = &c->timers.back();
        t->name = name;
    }
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!t->pool.empty()) {
        ev = t->pool.back();
        t->pool.pop_back();
    } else {
        (void)hipEventCreate(&ev.first);
        (void)hipEventCreate(&ev.second);
    }
    (void)hipEventRecord(ev.first, c->stream);
    t->pending.push_back(ev);
}

void timer_end(rbsog_ctx *c, const char *name)
{
    if (!c->timing) return;
    for (auto &x : c->timers)
        if (x.name == name && !x.pending.empty()) {
            (void)hipEventRecord(x.pending.back().second, c->stream);
            return;
        }
}

}  // namespace rbsog

extern "C" {

int rbsog_version(void) { return 10000; }

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
    p->recalibration = RBSOG_RECAL_PRINTED;
    return RBSOG_OK;
}

int rbsog_setup(const rbsog_params *params, int64_t n, const double *host_q, const double host_box[3],
                void *hip_stream, rbsog_ctx **out)
{
    if (!out) return RBSOG_EINVAL;
    *out = nullptr;
    if (!params || !host_q || !host_box) return RBSOG_EINVAL;
    if (n <= 0 || n > (int64_t)1 << 30) return RBSOG_EINVAL;
    const rbsog_params &p = *params;
    if (!(p.b > 1.0) || !(p.sigma > 0.0) || !std::isfinite(p.b) || !std::isfinite(p.sigma) ||
        !std::isfinite(p.omega))
        return RBSOG_EINVAL;
    if (p.M < 1 || p.M > RBSOG_MAX_M || p.P < 1 || p.P > kMaxP) return RBSOG_EINVAL;
    if (!(p.rc > 0.0) || !std::isfinite(p.rc) || !std::isfinite(p.coulomb_k)) return RBSOG_EINVAL;
    if (p.precision != RBSOG_PREC_FP64 && p.precision != RBSOG_PREC_FP32C) return RBSOG_EINVAL;
    if (p.recalibration != RBSOG_RECAL_PRINTED && p.recalibration != RBSOG_RECAL_EXCHANGE) return RBSOG_EINVAL;
    if (p.system_id >> 32) return RBSOG_EINVAL;
    double qs = 0.0, qa = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(host_q[i])) return RBSOG_EINVAL;
        qs += host_q[i];
        qa += std::fabs(host_q[i]);
    }
    if (std::fabs(qs) > 1e-10 * qa) return RBSOG_ENEUTRAL;
    rbsog_ctx *c = new (std::nothrow) rbsog_ctx;
    if (!c) return RBSOG_ENOMEM;
    int rc = check_box(c, host_box, p.rc);
    if (rc) {
        delete c;
        return rc;
    }
    c->prm = p;
    c->n = n;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return RBSOG_EDEVICE;
    }
    if (c->prm.omega <= 0.0) c->prm.omega = rbsog::omega_c0(p.b, p.sigma, p.rc, p.M);
    rbsog::sog_tables(c->prm, c->w, c->wt, c->s);
    double wsum = 0.0;
    for (int l = 0; l < p.M; ++l) wsum += c->w[l];
    for (int64_t i = 0; i < n; ++i) c->q2sum += host_q[i] * host_q[i];
    // U_self = (1/2) F(0) sum q^2 (App. A)
    c->Uself = p.coulomb_k * 0.5 * wsum * c->q2sum;
    for (int d = 0; d < 3; ++d) c->L[d] = host_box[d];
    rbsog::cell_grid(c->L, p.rc, c->nc);
    c->ncells = (int64_t)c->nc[0] * c->nc[1] * c->nc[2];

    auto cleanup = [&](int code) {
        free_buffers(c);
        delete c;
        return code;
    };
    const bool f64 = p.precision == RBSOG_PREC_FP64;
    const size_t rsz = f64 ? sizeof(double) : sizeof(float);
    const size_t fsz = f64 ? sizeof(uint64_t) : sizeof(uint32_t);
    const size_t recsz = f64 ? 32 : 16;
    if (dalloc(&c->d_tab, 1) != hipSuccess || hipMalloc(&c->d_q, n * rsz) != hipSuccess ||
        hipMalloc(&c->d_u, 3 * n * fsz) != hipSuccess || dalloc(&c->d_cell, n) != hipSuccess ||
        dalloc(&c->d_perm_tmp, n) != hipSuccess || dalloc(&c->d_perm, n) != hipSuccess ||
        hipMalloc(&c->d_rec, n * recsz) != hipSuccess || hipMalloc(&c->d_fsr, 3 * n * rsz) != hipSuccess ||
        dalloc(&c->d_scan_tmp, 2 * 1024 + 2) != hipSuccess || dalloc(&c->d_mraw, 6 * (int64_t)p.P) != hipSuccess ||
        dalloc(&c->d_modes, kMaxModes) != hipSuccess || dalloc(&c->d_cnt, 2 * kMaxModes) != hipSuccess ||
        dalloc(&c->d_rho, 2 * kMaxModes) != hipSuccess || hipMalloc(&c->d_coef, kMaxModes * 64) != hipSuccess ||
        dalloc(&c->d_res, 1) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&c->h_res), sizeof(rbsog::StepResults)) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(RBSOG_ENOMEM);
    }
    c->sk_blocks = (n + kSkChunk - 1) / kSkChunk;
    if (dalloc(&c->d_rho_part, 2 * c->sk_blocks * kMaxModes) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(RBSOG_ENOMEM);
    }
    if (ensure_cells(c) != RBSOG_OK) return cleanup(RBSOG_ENOMEM);

    rbsog::SogTables tab{};
    tab.M = p.M;
    tab.rc2 = p.rc * p.rc;
    tab.rc2_32 = static_cast<float>(p.rc * p.rc);
    const double log2e = 1.4426950408889634073599246810018921;
    for (int l = 0; l < p.M; ++l) {
        tab.w[l] = c->w[l];
        tab.wt[l] = c->wt[l];
        tab.s[l] = c->s[l];
        tab.inv_s2[l] = 1.0 / (c->s[l] * c->s[l]);
        tab.s5[l] = std::pow(c->s[l], 5);
        tab.s7[l] = std::pow(c->s[l], 7);
        tab.w32[l] = static_cast<float>(c->w[l]);
        tab.wt32[l] = static_cast<float>(c->wt[l]);
        tab.c32[l] = static_cast<float>(-log2e / (c->s[l] * c->s[l]));
    }
    if (hipMemcpyAsync(c->d_tab, &tab, sizeof(tab), hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return cleanup(RBSOG_EDEVICE);
    if (f64) {
        if (hipMemcpyAsync(c->d_q, host_q, n * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return cleanup(RBSOG_EDEVICE);
    } else {
        std::vector<float> q32(n);
        for (int64_t i = 0; i < n; ++i) q32[i] = static_cast<float>(host_q[i]);
        if (hipMemcpyAsync(c->d_q, q32.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return cleanup(RBSOG_EDEVICE);
        if (hipStreamSynchronize(c->stream) != hipSuccess) return cleanup(RBSOG_EDEVICE);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return cleanup(RBSOG_EDEVICE);
    *out = c;
    return RBSOG_OK;
}

int rbsog_sample_modes(rbsog_ctx *c, int64_t step, const double host_box[3], int32_t *host_m_r,
                       int32_t *host_m_nr, double host_S[2])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (step < 0 || (step >> 32)) return fail(c, RBSOG_EINVAL, "step must be in [0, 2^32)");
    int rc = check_box(c, host_box, c->prm.rc);
    if (rc) return rc;
    for (int d = 0; d < 3; ++d) c->L[d] = host_box[d];
    rbsog::cell_grid(c->L, c->prm.rc, c->nc);
    c->ncells = (int64_t)c->nc[0] * c->nc[1] * c->nc[2];
    rc = ensure_cells(c);
    if (rc) return rc;
    rbsog::norm_consts(c->L, c->prm.M, c->wt, c->s, &c->Sr, &c->Snr);
    c->step = step;
    HIP_TRY(c, rbsog::launch_sample(c, static_cast<uint32_t>(step)));
    if (host_m_r || host_m_nr) {
        const int64_t P = c->prm.P;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (host_m_r) HIP_TRY(c, hipMemcpy(host_m_r, c->d_mraw, 3 * P * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (host_m_nr)
            HIP_TRY(c, hipMemcpy(host_m_nr, c->d_mraw + 3 * P, 3 * P * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemcpy(c->h_res, c->d_res, sizeof(rbsog::StepResults), hipMemcpyDeviceToHost));
        if (c->h_res->status != 0) return fail(c, RBSOG_EDEVICE, "sampler found no nonzero initial state");
    }
    if (host_S) {
        host_S[0] = c->Sr;
        host_S[1] = c->Snr;
    }
    c->state = 1;
    return RBSOG_OK;
}

int rbsog_force_virial(rbsog_ctx *c, const double *x, const double *y, const double *z, double *fx, double *fy,
                       double *fz, double host_energy[3], double host_vir[6])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (!x || !y || !z || !fx || !fy || !fz) return fail(c, RBSOG_EINVAL, "null position or force array");
    if (c->state < 1) return fail(c, RBSOG_ESTATE, "rbsog_sample_modes must precede rbsog_force_virial");
    const int64_t n = c->n;
    const bool dev_in = is_device_ptr(x) && is_device_ptr(y) && is_device_ptr(z);
    const bool dev_out = is_device_ptr(fx) && is_device_ptr(fy) && is_device_ptr(fz);
    const double *px = x, *py = y, *pz = z;
    double *gx = fx, *gy = fy, *gz = fz;
    if (!dev_in || !dev_out) {
        if (!c->d_stage) HIP_TRY(c, hipMalloc(&c->d_stage, 6 * n * sizeof(double)));
    }
    if (!dev_in) {
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(z[i]))
                return fail(c, RBSOG_EINVAL, "positions have NaN/Inf");
        HIP_TRY(c, hipMemcpyAsync(c->d_stage, x, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_stage + n, y, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_stage + 2 * n, z, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        px = c->d_stage;
        py = c->d_stage + n;
        pz = c->d_stage + 2 * n;
    }
    if (!dev_out) {
        gx = c->d_stage + 3 * n;
        gy = c->d_stage + 4 * n;
        gz = c->d_stage + 5 * n;
    }
    HIP_TRY(c, rbsog::launch_bin_and_sort(c, px, py, pz));
    HIP_TRY(c, rbsog::launch_pair(c));
    HIP_TRY(c, rbsog::launch_kspace(c, gx, gy, gz));
    if (!dev_out) {
        HIP_TRY(c, hipMemcpyAsync(fx, gx, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(fy, gy, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(fz, gz, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    c->state = 2;
    if (host_energy || host_vir || !dev_out) {
        HIP_TRY(c, hipMemcpyAsync(c->h_res, c->d_res, sizeof(rbsog::StepResults), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (c->h_res->status != 0) return fail(c, RBSOG_EDEVICE, "sampler found no nonzero initial state");
        if (host_energy) {
            host_energy[0] = c->h_res->UN;
            host_energy[1] = c->h_res->UF;
            host_energy[2] = c->h_res->Uself;
        }
        if (host_vir)
            for (int k = 0; k < 6; ++k) host_vir[k] = c->h_res->vir[k];
    }
    return RBSOG_OK;
}

int rbsog_pressure(rbsog_ctx *c, double host_P[9], double host_parts[27])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (!host_P) return fail(c, RBSOG_EINVAL, "null pressure output");
    if (c->state < 2) return fail(c, RBSOG_ESTATE, "rbsog_force_virial must precede rbsog_pressure");
    HIP_TRY(c, hipMemcpyAsync(c->h_res, c->d_res, sizeof(rbsog::StepResults), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const rbsog::StepResults &r = *c->h_res;
    if (r.status != 0) return fail(c, RBSOG_EDEVICE, "sampler found no nonzero initial state");
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
    if (!host_mu || !host_box || !x || !y || !z) return fail(c, RBSOG_EINVAL, "null argument");
    if (!finite3(host_mu) || host_mu[0] <= 0 || host_mu[1] <= 0 || host_mu[2] <= 0)
        return fail(c, RBSOG_EINVAL, "scale factors must be positive and finite");
    if (!(is_device_ptr(x) && is_device_ptr(y) && is_device_ptr(z)))
        return fail(c, RBSOG_EINVAL, "rbsog_rescale needs device position arrays");
    HIP_TRY(c, rbsog::launch_rescale(c, host_mu, x, y, z));
    for (int d = 0; d < 3; ++d) host_box[d] *= host_mu[d];
    return RBSOG_OK;
}

int rbsog_destroy(rbsog_ctx *c)
{
    if (!c) return RBSOG_OK;
    (void)hipStreamSynchronize(c->stream);
    free_buffers(c);
    delete c;
    return RBSOG_OK;
}

int rbsog_debug_cells(rbsog_ctx *c, int32_t *host_cell, int32_t host_ncell[3])
{
    if (!c) return RBSOG_EINVAL;
    if (c->state < 2) return fail(c, RBSOG_ESTATE, "no evaluation yet");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (host_cell) HIP_TRY(c, hipMemcpy(host_cell, c->d_cell, c->n * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (host_ncell)
        for (int d = 0; d < 3; ++d) host_ncell[d] = c->nc[d];
    return RBSOG_OK;
}

int rbsog_debug_modes(rbsog_ctx *c, int32_t cap, int32_t *host_nd, int32_t *host_modes, int32_t *host_counts,
                      double *host_rho)
{
    if (!c) return RBSOG_EINVAL;
    if (c->state < 1) return fail(c, RBSOG_ESTATE, "no sampled modes yet");
    if (cap < 0) return fail(c, RBSOG_EINVAL, "negative capacity");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(c->h_res, c->d_res, sizeof(rbsog::StepResults), hipMemcpyDeviceToHost));
    const int nd = c->h_res->nd;
    if (host_nd) *host_nd = nd;
    const int k = std::min(nd, cap);
    if (host_modes && k > 0) {
        std::vector<int4> m(k);
        HIP_TRY(c, hipMemcpy(m.data(), c->d_modes, k * sizeof(int4), hipMemcpyDeviceToHost));
        for (int d = 0; d < k; ++d) {
            host_modes[3 * d] = m[d].x;
            host_modes[3 * d + 1] = m[d].y;
            host_modes[3 * d + 2] = m[d].z;
        }
    }
    if (host_counts && k > 0) {
        std::vector<int32_t> cn(2 * kMaxModes);
        HIP_TRY(c, hipMemcpy(cn.data(), c->d_cnt, 2 * kMaxModes * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int d = 0; d < k; ++d) {
            host_counts[2 * d] = cn[d];
            host_counts[2 * d + 1] = cn[kMaxModes + d];
        }
    }
    if (host_rho && k > 0) {
        if (c->state < 2) return fail(c, RBSOG_ESTATE, "rho needs rbsog_force_virial");
        HIP_TRY(c, hipMemcpy(host_rho, c->d_rho, 2 * k * sizeof(double), hipMemcpyDeviceToHost));
    }
    return RBSOG_OK;
}

int rbsog_step_info(rbsog_ctx *c, int64_t host_info[4])
{
    if (!c || !host_info) return RBSOG_EINVAL;
    if (c->state < 1) return fail(c, RBSOG_ESTATE, "no sampled modes yet");
    HIP_TRY(c, hipMemcpyAsync(c->h_res, c->d_res, sizeof(rbsog::StepResults), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    host_info[0] = c->h_res->nd;
    host_info[1] = c->h_res->acc_r;
    host_info[2] = c->h_res->acc_nr;
    host_info[3] = c->state >= 2 ? static_cast<int64_t>(std::llround(c->h_res->npairs)) : 0;
    return RBSOG_OK;
}

int rbsog_set_timing(rbsog_ctx *c, int on)
{
    if (!c) return RBSOG_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    for (auto &t : c->timers) {
        for (auto &e : t.pending) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        for (auto &e : t.pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
    c->timers.clear();
    c->timing = on != 0;
    return RBSOG_OK;
}

int rbsog_get_timing(rbsog_ctx *c, int32_t cap, int32_t *host_nk, char *host_names, double *host_ms,
                     int64_t *host_count)
{
    if (!c) return RBSOG_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto &t : c->timers) {
        for (auto &e : t.pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
                t.ms += ms;
                t.count += 1;
            }
            t.pool.push_back(e);
        }
        t.pending.clear();
    }
    const int nk = static_cast<int>(c->timers.size());
    if (host_nk) *host_nk = nk;
    for (int k = 0; k < std::min(nk, cap); ++k) {
        if (host_names) {
            std::memset(host_names + 32 * k, 0, 32);
            std::strncpy(host_names + 32 * k, c->timers[k].name.c_str(), 31);
        }
        if (host_ms) host_ms[k] = c->timers[k].ms;
        if (host_count) host_count[k] = c->timers[k].count;
    }
    return RBSOG_OK;
}

}  // extern "C"
