// Internal declarations of the RBSOG HIP library (not part of the C ABI).
//
// Every kernel works on a batch of independent systems.  A system is described
// by a SysDesc (splitting tables, sizes, device buffers; written when the
// system joins a batch or its buffers move) and a SysStep (box, scale factors,
// normalisation constants, cell grid, step index and the caller's position and
// force arrays; written every step).  Kernels find their system and their
// block within it through a launch plan: one (system, block) entry per
// workgroup, built on the host from sizes it knows.  A system's arithmetic
// never depends on the other systems in the batch, so one system alone and the
// same system in any batch give bitwise identical results.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rbsog.h"

namespace rbsog {

constexpr int kMaxP = 1024;        // samples per chain handled by the one-workgroup sampler
constexpr int kMaxModes = kMaxP + 2; // distinct modes: accepted proposals plus the start states of both chains
constexpr int kPairWave = 64;      // i-atoms per pair-kernel wavefront
constexpr int kSkChunk = 1024;     // atoms per structure-factor workgroup
constexpr int kPairRed = 64;       // workgroups reducing a system's pair-block partials (then summed in order)
constexpr int kAtomBlock = 256;    // atoms per workgroup of the per-atom kernels
constexpr int kCellBlock = 256;    // cells per workgroup of the per-cell kernels
constexpr int kScanBlock = 1024;   // cells per workgroup of the local scan
constexpr int64_t kMaxCells = int64_t(1024) * kScanBlock;  // cells per system (two-level scan)
constexpr int kMaxTimed = 24;
constexpr int kPolyDeg = 10;       // degree of the FP32C polynomial form of the SOG sums
constexpr int kSuperCells = 4;     // most cells stacked in z into one pair-block segment
constexpr int kOrderPart = 1024;   // keys one ordering workgroup ranks in a single-cell system
constexpr int kHrngStride = 24;    // ints per pair block of the half-shell neighbourhood table
// Half-shell partial buffer: forward candidates per block are estimated at this
// density (atoms per A^3, above condensed matter's 0.1) and margin; a block
// with more runs its system on the full shell for that step.
constexpr double kHalfRefDensity = 0.15;
constexpr double kHalfMargin = 1.25;
// General cells: Gauss-Legendre points per axis of the proposal pmf's
// integral over the unit cube (eq. proposal), and the size of the per-system
// table of w_i w_j w_k exp(-pi^2 s^2 d^T C d) for the two proposal widths.
constexpr int kGl = 24;
constexpr int kGlTab = 2 * kGl * kGl * kGl;

// Distinct modes a step can visit: the r-chain's start state and proposals;
// the exchange form adds the non-radial chain's start state, the independent
// non-radial chain its start state and its own proposals.
inline int mode_cap(const rbsog_params &p)
{
    if (p.recalibration == RBSOG_RECAL_INDEPENDENT) return 2 * p.P + 2;
    if (p.recalibration == RBSOG_RECAL_EXCHANGE) return p.P + 2;
    return p.P + 1;
}

// SOG tables read by the kernels (device memory, uniform loads).
struct SogTables {
    int M;                // Gaussians of the force, virial and sampling
    int Me;               // Gaussians of the energy (>= M; wt_l = 0 for M <= l < Me)
    double rc2;
    // energy kernel F(r) = sum w_l exp(-r^2/s_l^2); force/pressure kernel F~ with wt_l
    double w[RBSOG_MAX_M], wt[RBSOG_MAX_M], inv_s2[RBSOG_MAX_M];
    // exp(-r^2/s^2) = exp2(r^2 * c_l) with c_l = -log2(e)/s_l^2 (FP32 kernel)
    float w32[RBSOG_MAX_M], wt32[RBSOG_MAX_M], c32[RBSOG_MAX_M];
    float rc2_32;
    // FP32C polynomial form on r^2 in [0, rc^2]: with t = pa r^2 - 1,
    // sum_l wt_l e_l = sum_k pg[k] t^k and sum_l w_l e_l = sum_k pf[k] t^k
    // (Chebyshev interpolants, truncation error checked at set-up)
    float pa;
    float pg[kPolyDeg + 1], pf[kPolyDeg + 1];
    int poly;             // 1: the polynomial form is used (FP32C only)
    float poly_err;       // max |p - sum| / sum(0) of the fit, both sums
    // sampler: s_l, and wt_l s_l^5, wt_l s_l^7 are formed from s5, s7
    double s[RBSOG_MAX_M], s5[RBSOG_MAX_M], s7[RBSOG_MAX_M];
    // Gauss-Legendre nodes and weights on [-1/2, 1/2] (general cells)
    double glx[kGl], glw[kGl];
};

// Results of one step of one system, written on the device, read by the host.
struct StepResults {
    double UN, UF, Uself, pad0;
    double vir[6];        // short-range virial sum (xx yy zz xy xz yz)
    double PN[9], Pr[9], Pnr[9], Ptot[9];
    double Sr, Snr;
    int32_t nd, status;
    int64_t acc_r, acc_nr;
    double npairs;  // unordered in-cutoff pairs of the last evaluation
    int32_t bad_input;  // nonzero: a position was NaN or infinite (set by k_fix)
    int32_t pad1;
};

// Static description of one system (device copy read by every kernel).
struct SysDesc {
    SogTables tab;
    int64_t n;            // atoms
    int64_t pair_cap;     // pair-block slots allocated: ceil(n/64) + ncells_cap
    int64_t sk_blocks;    // structure-factor workgroups: ceil(n/kSkChunk)
    int64_t ncells_cap;   // cells allocated
    int32_t P, M, variant, mcap;  // mcap = mode_cap(params): stride of the per-mode arrays
    uint32_t key0, key1, sys, pad;
    double ck, Uself;
    // internal device buffers
    const void *q;        // charges, system order (float or double)
    void *u;              // fixed-point fractional coordinates (3 SoA planes of n)
    int32_t *cell;        // cell of each atom
    int32_t *slot;        // each atom's place among its cell's atoms (binned slot = start + slot)
    int32_t *count, *start, *nblk, *bstart;  // per cell [ncells_cap + 1]
    int32_t *scan_tmp;    // [2 * 1024 + 2] block sums of the two-level scan
    int2 *blocks;         // pair-block table (cell, sub-block) [pair_cap]
    uint64_t *keys;       // binned slot -> (z sort key << 32) | system atom index
    void *urec;           // binned slot -> the atom's record (fixed-point position + charge), unsorted within its cell
    int32_t *perm;        // sorted slot -> system atom index
    void *rec;            // sorted records (fixed-point position + charge)
    void *fsr;            // short-range force, sorted order (3 SoA planes)
    double *pair_part;    // 8 doubles per pair block
    int32_t *mraw;        // m_r then m_nr, P x 3 each
    int4 *modes;          // distinct modes [mcap]
    int32_t *cnt;         // multiplicities: r-chain [mcap], nr-chain [mcap]
    double *rho_part;     // [sk_blocks][mcap] x (re, im)
    double *rho;          // [mcap] x (re, im)
    double *pair_red;     // [kPairRed][8] slice sums of the pair-block partials
    void *coef;           // per-mode force coefficients [mcap]
    StepResults *res;     // this system's slot of the batch results
    // half-shell pair kernel (FP32C fast path): reactions on forward candidates
    float *hpart;         // [pair_cap][3][hcap] FP32 partials, by position in the block's neighbourhood
    int32_t *hrng;        // [pair_cap][kHrngStride]: range starts, flattened prefixes, chunk count
    int32_t *hflag;       // [1] set when a block's neighbourhood exceeds hcap (full shell this step)
    int32_t hcap, pad2;   // candidates per block the partial buffer holds
    double *gltab;        // general cells: [2][kGl^3] quadrature table of the proposal pmf (null otherwise)
};

// Per-step data of one system (rewritten by the host every step).
struct SysStep {
    double L[3];
    double iL[3];         // 1/L, rounded once on the host
    double mu[3];         // scale factors of the next rescale
    double Sr, Snr;
    double Bstart[2];     // bounds of g_2/q' and g_4/q' for the exact start draws of the chains
    int32_t nc[3];        // cells per edge; cell id = cz + nc[2] (cy + nc[1] cx), z fastest
    int32_t ncells;
    uint32_t step;
    int32_t g;            // cells per pair-block segment along z (a column's cells cz = 0, g, 2g, ... start one)
    int32_t fast;         // FP32 relative-coordinate filter over whole neighbour columns (4+ cells per edge, nz >= 2g + 2)
    uint32_t thr16;       // FP32 exact filter: bound on sum (d_d / u_d)^2 of a pair inside rc, u_d = L_d / 2^16
    int32_t half;         // fast path with Newton's third law (half-shell pair kernel, partials, gather)
    int32_t tri;          // general cell: h below is not diagonal (exact path with d = h ds, sampler by quadrature)
    double h[9], hi[9];   // cell tensor (row-major, columns the cell vectors) and its inverse
    double V;             // det h
    const double *x, *y, *z;  // positions (device, system order)
    double *fx, *fy, *fz;     // forces (device, system order)
};

// Plans: one entry (system index, block index within the system) per workgroup.
enum PlanKind { kPlanAtoms, kPlanCells, kPlanScan, kPlanPair, kPlanSk, kPlanReduce, kPlanCell1, kNumPlans };

struct Timer {
    std::string name;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    double ms = 0.0;
    int64_t count = 0;
};

// Pair-kernel forms of the SOG kernels, chosen per system.
enum PairForm {
    kFormPoly = 0,   // FP32C: degree-kPolyDeg polynomials in r^2
    kFormExp10 = 1,  // M = 10 exponentials, weights in registers
    kFormExpM = 2,   // runtime M exponentials
    kNumForms = 3,
};
// Pair launches: one per (form, path); path 0 is the exact filter, path 1 the
// FP32 relative-coordinate filter over whole neighbour columns (SysStep::fast)
// with the full shell, path 2 the same with the half shell (SysStep::half),
// path 3 a general cell (SysStep::tri): the relative-coordinate filter when
// SysStep::fast (FP32, four or more cells per edge), else the exact one.
constexpr int kNumPaths = 4;
constexpr int kNumPairGroups = kNumPaths * kNumForms;

// Pair-kernel schedules (none changes any result).
enum PairSchedule {
    kPairStatic = 0,      // one workgroup per pair-block slot
    kPairPersistent = 1,  // workgroups pull pair blocks from a global counter
};

// One system on the host: parameters, splitting tables, box state and buffers.
struct System {
    rbsog_params prm{};
    int64_t n = 0;
    double w[RBSOG_MAX_M]{}, wt[RBSOG_MAX_M]{}, s[RBSOG_MAX_M]{};
    double q2sum = 0.0, Uself = 0.0;
    SogTables tab{};
    // box state (a general cell keeps h; L holds its diagonal)
    double L[3]{};
    bool tri = false;
    double h[9]{};
    void *gl_mem = nullptr;  // general cells: the pmf quadrature table (allocated on first use)
    double Sr = 0.0, Snr = 0.0;
    int nc[3]{1, 1, 1};
    int64_t ncells = 0;
    // device memory: atom-sized part (fixed) and cell-sized part (grows with the grid)
    void *atom_mem = nullptr;
    size_t atom_bytes = 0;
    void *cell_mem = nullptr;
    size_t cell_bytes = 0;
    int64_t ncells_cap = 0;
    bool own_mem = true;  // false: the memory belongs to a pool
    // half-shell buffers (own memory only): partials, neighbourhood table, flag
    void *half_mem = nullptr;
    int64_t half_blocks = 0;  // pair-block slots they cover
    int32_t half_hcap = 0;    // candidates per block
    int pair_form = kFormExpM;
    SysDesc desc{};       // host copy of the device descriptor
    SysStep stp{};        // host copy of the per-step data
};

// A batch of systems sharing one stream and one set of launches.
struct Batch {
    hipStream_t stream = nullptr;
    // The sampler and the structure factors run on a second stream, beside
    // binning and the pair kernel (default priority, joined by events):
    //   stream: upload -+-> bin -+-> pair ----------+-> reduce, estimators, force
    //                   |        |                  |
    //   aux:            +-> sampler -> (bin done) sk -+
    hipStream_t aux = nullptr;
    hipEvent_t ev_up = nullptr, ev_bin = nullptr, ev_sk = nullptr;
    int device = 0;
    int precision = RBSOG_PREC_FP32C;
    std::vector<System *> sys;
    // device arrays and their pinned host mirrors
    SysDesc *d_desc = nullptr, *h_desc = nullptr;
    SysStep *d_step = nullptr;
    static constexpr int kStepRing = 4;        // pinned per-step buffers used in turn
    SysStep *h_step[kStepRing] = {};
    std::vector<SysStep> step_last;           // what d_step holds once the queued copies have run
    hipEvent_t step_ev[kStepRing] = {};
    bool step_ev_used[kStepRing] = {};
    int step_slot = 0;
    StepResults *d_res = nullptr, *h_res = nullptr;
    int2 *d_plan = nullptr, *h_plan = nullptr;
    int32_t *d_ctrl = nullptr;  // [0 .. kNumPairGroups): work-queue counters of the pair launches
    int64_t cap_sys = 0, cap_plan = 0;
    int64_t plan_off[kNumPlans]{}, plan_len[kNumPlans]{};
    int64_t pair_split[kNumPairGroups + 1]{};  // pair-plan entries of launch group g = 2 form + path: [split[g], split[g+1])
    bool want_energy = true;              // the pair kernel sums U^N
    bool desc_dirty = true, plan_dirty = true;
    std::vector<int64_t> plan_key;  // sizes the plans were built for
    // event that guards the pinned descriptor and plan mirrors
    hipEvent_t up_done = nullptr;
    bool up_pending = false;
    // options
    int pair_schedule = kPairStatic;
    int pair_wg_per_cu = 8;
    int num_cu = 256;
    // graph of the whole step (batch form)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<int64_t> graph_key;
    // timing
    int timing = 0;  // 0 off, 1 every kernel group, 2 the pair kernel only
    std::vector<Timer> timers;
};

// ---------------------------------------------------------------------------
// host-side set-up helpers (setup.cpp)
void sog_tables(const rbsog_params &p, double *w, double *wt, double *s);
double omega_c0(double b, double sigma, double rc, int M);
void norm_consts(const double L[3], int M, const double *wt, const double *s, double *Sr, double *Snr);
double start_bound(const double L[3], int M, const double *wt, const double *s, int power);
void cell_grid(const double L[3], double rc, int nc[3]);
// General cells (row-major h, columns the cell vectors): S^r, S^nr, the start
// bound, the perpendicular widths, and the Gauss-Legendre rule on [-1/2, 1/2].
void norm_consts_cell(const double h[9], int M, const double *wt, const double *s, double *Sr, double *Snr);
double start_bound_cell(const double h[9], int M, const double *wt, const double *s, int power);
double cell_inverse(const double h[9], double hi[9]);
void cell_widths(const double hi[9], double w[3]);
void gauss_legendre_unit(int n, double *x, double *w);

// ---------------------------------------------------------------------------
// systems and batches (system.cpp)

// Validate parameters and charges, fill the tables; no device work.
int system_init(System &s, const rbsog_params &p, int64_t n, const double *host_q, const double box[3],
                std::string &err);
// Check a box against the cutoff.
int check_box(const double *box, double rc, std::string &err);
// Bytes of the atom-sized and cell-sized device parts of a system.
size_t system_atom_bytes(const rbsog_params &p, int64_t n);
size_t system_cell_bytes(int64_t n, int64_t ncells_cap);
// Device bytes a system holds now (atom, cell and half-shell parts).
size_t system_device_bytes(const System &s);
// Point the descriptor into memory the caller provides (aligned to 256 bytes).
void system_carve_atoms(System &s, void *mem);
void system_carve_cells(System &s, void *mem, int64_t ncells_cap);
// Allocate (own_mem) or re-carve the buffers; grows the cell part to the grid.
int system_alloc(System &s, std::string &err);
// Grows the cell part when the grid outgrows it; *recarved tells whether the
// cell arrays moved (the device descriptor must then be uploaded again: the
// allocator may hand back the old address, so comparing addresses is not enough).
int system_ensure_cells(System &s, std::string &err, bool *recarved = nullptr);
void system_free(System &s);
// Upload the charges (FP32 or FP64 copy) on the stream.
// Charges to the device (FP32C: rounded to float).  With a stage, the copy is
// left in flight: the caller keeps host_q and *stage until the stream is synchronised.
int system_upload_q(System &s, const double *host_q, hipStream_t stream, std::string &err,
                    std::vector<float> *stage = nullptr);
// New box: grid, S^r, S^nr, the pair path.
void system_set_box(System &s, const double box[3]);
// New general cell (row-major h); a diagonal h is the box of its diagonal.
// RBSOG_EBOX unless r_c is at most half the smallest perpendicular width.
int system_set_cell(System &s, const double h[9], std::string &err);
// Whether the system takes the half-shell pair kernel on the fast path, and
// the forward candidates per block its partial buffer holds for the grid.
bool wants_half_shell(const System &s);
int32_t half_hcap(const System &s);
// Cells needed by a box.
int64_t cells_for_box(const double box[3], double rc);

int batch_init(Batch &b, hipStream_t stream, int precision, std::string &err);
void batch_free(Batch &b);
// Replace the batch's systems (descriptors and plans are rebuilt on the next upload).
int batch_set_systems(Batch &b, const std::vector<System *> &sys, std::string &err);
// Copy descriptors (if changed), per-step data and plans (if sizes changed) to the device.
int batch_upload(Batch &b, std::string &err);
// Whether the next batch_upload would allocate (more systems or plan entries than held).
bool batch_upload_allocates(const Batch &b);
// Results of every system to the host (synchronises).
int batch_fetch_results(Batch &b, std::string &err);
// Per-kernel HIP-event timing of the batch's launches.
void batch_set_timing(Batch &b, int level);
int batch_get_timing(Batch &b, int32_t cap, int32_t *host_nk, char *host_names, double *host_ms,
                     int64_t *host_count, std::string &err);

// ---------------------------------------------------------------------------
// kernel launchers (kernels.hip); each returns a hipError_t
hipError_t launch_sample(Batch &b);
// launch_sample in two parts: the fence on the first stream (the sampler waits
// for what that stream held at it) and the sampler itself, launched later
hipError_t record_sample_fence(Batch &b);
hipError_t launch_sample_fenced(Batch &b);
hipError_t launch_bin_and_sort(Batch &b);
hipError_t launch_pair(Batch &b);
hipError_t launch_kspace(Batch &b);
hipError_t launch_rescale(Batch &b);
hipError_t launch_long_range_force(Batch &b, double *fx, double *fy, double *fz);

// timing hooks used by the launchers (system.cpp)
void timer_begin(Batch &b, const char *name, hipStream_t s);
void timer_end(Batch &b, const char *name, hipStream_t s);

// ---------------------------------------------------------------------------
// NPT integration (npt.cpp, kernels in kernels.hip)
struct NptState {
    bool ready = false;
    rbsog_npt_params prm{};
    double *d_mass = nullptr;  // [n] masses, caller order
    double *d_F = nullptr;     // [3n] force of the last evaluation (SoA)
    double *d_part = nullptr;  // [6 * kinetic blocks] partial sums of p p^T / m
    double *d_kin = nullptr;   // [6] their fixed-order total
    int64_t kin_blocks = 0;
};
constexpr int kNptBlock = 256;
// p += c F (three planes)
hipError_t launch_npt_kick(hipStream_t s, int64_t n, double c, const double *F, double *px, double *py, double *pz);
// per axis: r <- a r + b p/m, p <- p / a
hipError_t launch_npt_drift(hipStream_t s, int64_t n, const double a[3], const double b[3], const double *mass,
                            double *x, double *y, double *z, double *px, double *py, double *pz);
// p <- c p + sqrt(m) sc xi, xi standard normals from Philox (atom, 16|17, step, sys) keyed by seed
hipError_t launch_npt_ou(hipStream_t s, int64_t n, double c, double sc, const double *mass, double *px, double *py,
                         double *pz, uint64_t seed, uint32_t step, uint32_t sys);
// sum_i p_i p_i^T / m_i (xx, yy, zz, xy, xz, yz) into kin[6], fixed order
hipError_t launch_npt_kinetic(hipStream_t s, int64_t n, const double *mass, const double *px, const double *py,
                              const double *pz, double *part, int64_t nblocks, double *kin);

}  // namespace rbsog

// A single-system context: one system evaluated as a batch of one.  It can
// also be admitted to a batch of contexts (rbsog_batch_create); while
// admitted its step inputs are staged and the batch evaluates them.
struct rbsog_ctx {
    rbsog::System sys;
    rbsog::Batch batch;
    int state = 0;  // 0: set up, 1: modes sampled, 2: forces computed
    double *d_stage = nullptr;  // host-array staging (6 n doubles), allocated on first use
    rbsog::NptState npt;
    std::string err;
    rbsog_batch *in_batch = nullptr;  // the batch of contexts it is admitted to
    bool staged = false;              // inputs of the next batched step are set
    bool desc_moved = false;          // its buffers were re-carved since the batch last uploaded them
    bool res_from_batch = false;      // batch.h_res[0] holds the results of the last batched step
    // results of queued steps (rbsog_step_async): pinned slots, each filled by
    // a copy queued behind its step and marked by an event
    static constexpr int kResRing = 4;
    rbsog::StepResults *h_ring = nullptr;
    hipEvent_t ring_ev[kResRing] = {};
    int64_t ring_ticket[kResRing] = {-1, -1, -1, -1};  // the ticket each slot holds, -1 for none
    static_assert(kResRing == 4, "ring_ticket's initialiser and the error message name four slots");
    int64_t next_ticket = 0;
};
