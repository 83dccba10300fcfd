// Internal declarations of the RBSOG HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rbsog.h"

namespace rbsog {

constexpr int kMaxP = 1024;        // samples per chain handled by the one-workgroup sampler
constexpr int kMaxModes = kMaxP + 1; // distinct modes: accepted proposals plus the initial state
constexpr int kPairWave = 64;      // i-atoms per pair-kernel wavefront
constexpr int kSkChunk = 1024;     // atoms per structure-factor workgroup
constexpr int kMaxTimed = 24;

// SOG tables read by the kernels (device memory, uniform loads).
struct SogTables {
    int M;
    int pad;
    double rc2;
    // energy kernel F(r) = sum w_l exp(-r^2/s_l^2); force/pressure kernel F~ with wt_l
    double w[RBSOG_MAX_M], wt[RBSOG_MAX_M], inv_s2[RBSOG_MAX_M];
    // exp(-r^2/s^2) = exp2(r^2 * c_l) with c_l = -log2(e)/s_l^2 (FP32 kernel)
    float w32[RBSOG_MAX_M], wt32[RBSOG_MAX_M], c32[RBSOG_MAX_M];
    float rc2_32;
    float pad32;
    // sampler: s_l^2/4, wt_l s_l^5, wt_l s_l^7 are formed inside the sampler from these
    double s[RBSOG_MAX_M], s5[RBSOG_MAX_M], s7[RBSOG_MAX_M];
};

// Results of one step, written on the device, read by the host.
struct StepResults {
    double UN, UF, Uself, pad0;
    double vir[6];        // short-range virial sum (xx yy zz xy xz yz)
    double PN[9], Pr[9], Pnr[9], Ptot[9];
    double Sr, Snr;
    int32_t nd, status;
    int64_t acc_r, acc_nr;
    double npairs;  // unordered in-cutoff pairs of the last evaluation
};

struct Timer {
    std::string name;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    double ms = 0.0;
    int64_t count = 0;
};

}  // namespace rbsog

struct rbsog_ctx {
    rbsog_params prm{};
    int64_t n = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;

    // host copies of the splitting tables and constants
    double w[RBSOG_MAX_M]{}, wt[RBSOG_MAX_M]{}, s[RBSOG_MAX_M]{};
    double q2sum = 0.0, Uself = 0.0;

    // current box and derived quantities
    double L[3]{};
    double Sr = 0.0, Snr = 0.0;
    int nc[3]{1, 1, 1};
    int64_t ncells = 0, ncells_cap = 0;
    int state = 0;  // 0: set up, 1: modes sampled, 2: forces computed
    int64_t step = 0;

    // device buffers
    rbsog::SogTables *d_tab = nullptr;
    void *d_q = nullptr;          // charges, caller order (float or double)
    void *d_u = nullptr;          // fixed-point fractional coordinates, caller order (3 SoA planes)
    int32_t *d_cell = nullptr;    // cell of each atom, caller order
    int32_t *d_count = nullptr;   // atoms per cell        [ncells_cap + 1]
    int32_t *d_cursor = nullptr;  // scatter cursors       [ncells_cap + 1]
    int32_t *d_start = nullptr;   // first slot per cell   [ncells_cap + 1]
    int32_t *d_nblk = nullptr;    // pair blocks per cell  [ncells_cap + 1]
    int32_t *d_bstart = nullptr;  // first pair block per cell [ncells_cap + 1]
    int32_t *d_scan_tmp = nullptr;
    int2 *d_blocks = nullptr;     // pair block table (cell, sub-block)
    int64_t pair_grid_cap = 0;
    int32_t *d_perm_tmp = nullptr;
    int32_t *d_perm = nullptr;    // sorted slot -> caller index
    void *d_rec = nullptr;        // sorted records (fixed-point position + charge)
    void *d_fsr = nullptr;        // short-range force, sorted order (3 SoA planes)
    double *d_pair_part = nullptr;  // 8 doubles per pair workgroup
    // sampler and modes
    int32_t *d_mraw = nullptr;    // m_r then m_nr, P x 3 each
    int4 *d_modes = nullptr;      // distinct modes
    int32_t *d_cnt = nullptr;     // multiplicities: r-chain [kMaxModes], nr-chain [kMaxModes]
    double *d_rho_part = nullptr; // [sk blocks][kMaxModes] x (re, im)
    double *d_rho = nullptr;      // [kMaxModes] x (re, im)
    void *d_coef = nullptr;       // per-mode force coefficients
    rbsog::StepResults *d_res = nullptr;
    rbsog::StepResults *h_res = nullptr;  // pinned
    int64_t sk_blocks = 0;
    // host staging for host-memory positions and forces
    double *d_stage = nullptr;

    // timing
    bool timing = false;
    std::vector<rbsog::Timer> timers;
};

namespace rbsog {

// host-side setup helpers (setup.cpp)
void sog_tables(const rbsog_params &p, double *w, double *wt, double *s);
double omega_c0(double b, double sigma, double rc, int M);
void norm_consts(const double L[3], int M, const double *wt, const double *s, double *Sr, double *Snr);
void cell_grid(const double L[3], double rc, int nc[3]);

// kernel launchers (kernels.hip); each returns a hipError_t
hipError_t launch_sample(rbsog_ctx *c, uint32_t step);
hipError_t launch_bin_and_sort(rbsog_ctx *c, const double *x, const double *y, const double *z);
hipError_t launch_pair(rbsog_ctx *c);
hipError_t launch_kspace(rbsog_ctx *c, double *fx, double *fy, double *fz);
hipError_t launch_rescale(rbsog_ctx *c, const double mu[3], double *x, double *y, double *z);

// timing hooks used by the launchers
void timer_begin(rbsog_ctx *c, const char *name);
void timer_end(rbsog_ctx *c, const char *name);

}  // namespace rbsog
