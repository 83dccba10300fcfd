/*
 * rbsog.h - C ABI of the MI355X (gfx950) random batch sum-of-Gaussians (RBSOG)
 * electrostatics library: forces, energy and the Coulomb pressure tensor of a
 * periodic, charge-neutral point-charge system, one evaluation per MD step.
 *
 * Method: Jiang, Liang, Zhou, "Random batch sum-of-Gaussians method for
 * molecular dynamics simulation of particle systems in the NPT ensemble",
 * arXiv:2602.23582.  One step is Algorithm 1, steps 2-6:
 *   rbsog_sample_modes  - steps 2-3: Metropolis-Hastings sampling of P Fourier
 *                         modes from the radial proposal (App. D, eq.
 *                         samplingP) and their measure recalibration to the
 *                         non-radial target (Sec. 3.2, eq. samplingPnr);
 *   rbsog_force_virial  - steps 4-6: short-range SOG force, virial and energy
 *                         by cell lists (eqs. force_SOG, P_short, U_short),
 *                         structure factors of the distinct modes (eq. rho_k),
 *                         random-batch long-range force (eq. f_approx) and the
 *                         long-range estimators (eqs. P_approx_r, P_approx_nr);
 *   rbsog_pressure      - step 6: the total Coulomb pressure tensor
 *                         P^N + P^{F,r*} + P^{F,nr*}.
 *
 * Conventions
 *  - Orthorhombic cells h = diag(Lx, Ly, Lz) (Sec. 2.1 with a diagonal h).
 *  - Units: lengths in Angstrom, charges in e; every energy, force and
 *    pressure is multiplied by params.coulomb_k (1.0 = Gaussian units as in
 *    the paper).  Tinfoil boundary conditions (Theorem 1).
 *  - Positions may lie anywhere; they are wrapped into the cell internally.
 *  - Arrays named host_* are host memory.  Position and force arrays may be
 *    host or device memory (detected per call); device arrays give the fast
 *    path.  The caller owns every array passed in or out; the context owns
 *    its device buffers, which it allocates in rbsog_setup and frees in
 *    rbsog_destroy.
 *  - Every call returns RBSOG_OK (0) or a negative error code; on error the
 *    outputs are undefined and rbsog_last_error() describes the failure.
 *  - A context is not thread-safe; contexts are independent of each other.
 *  - Order per step: rbsog_sample_modes -> rbsog_force_virial -> rbsog_pressure.
 *    Work is queued on the stream given to rbsog_setup; calls that return host
 *    values synchronise that stream.
 */
#ifndef RBSOG_H
#define RBSOG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBSOG_OK 0
#define RBSOG_EINVAL (-1)   /* null pointer, bad size or count, NaN/Inf input       */
#define RBSOG_ENEUTRAL (-2) /* |sum q| > 1e-10 sum |q| (charge neutrality, Sec. 2.2) */
#define RBSOG_EBOX (-3)     /* non-positive box or rc > min(L)/2                     */
#define RBSOG_ENOMEM (-4)   /* device or host allocation failed                      */
#define RBSOG_EDEVICE (-5)  /* a HIP call failed (its message is kept)               */
#define RBSOG_ESTATE (-6)   /* call out of order                                     */
#define RBSOG_EAGAIN (-7)   /* batch admission refused (memory budget or slots)      */

#define RBSOG_PREC_FP64 0  /* every kernel in double precision                     */
#define RBSOG_PREC_FP32C 1 /* FP32 arithmetic, FP64 partial sums and reductions     */

#define RBSOG_RECAL_PRINTED 0  /* recalibration chain as printed in Sec. 3.2 (biased, see below) */
#define RBSOG_RECAL_EXCHANGE 1 /* swap of the two chain states on acceptance (the default)      */
/* The samplers the recalibration is weighed against (Sec. 3.2): */
#define RBSOG_RECAL_SHARED 2      /* no recalibration: the r-chain's modes, weighted by P^nr/P^r */
#define RBSOG_RECAL_INDEPENDENT 3 /* a second MH chain for P^nr: up to 2P+2 modes, P <= 512      */

#define RBSOG_MAX_M 64

#define RBSOG_FLAG_EXP_FORM 1  /* FP32C: evaluate the M exponentials, not the polynomial form   */
#define RBSOG_FLAG_FULL_SHELL 2 /* FP32C: the full-shell pair kernel (the default)                */
#define RBSOG_FLAG_HALF_SHELL 4 /* FP32C: the half-shell pair kernel (each unordered pair once)   */

typedef struct rbsog_ctx rbsog_ctx;

/*
 * Splitting and sampling parameters (Algorithm 1, "Require").
 *  b, sigma, omega  SOG base b = b~ > 1, width sigma = sigma~ > 0 and the
 *                   narrowest-Gaussian factor omega = omega~ (Sec. 2.2 and
 *                   3.1; Theorem 2).  omega <= 0 asks for the C0 root of the
 *                   1/r^3 split at rc (eq. continuity).
 *  M                Gaussians kept, M = M~ (Theorem 2), 1..RBSOG_MAX_M.
 *  rc               short-range cutoff, 0 < rc <= min(L)/2.
 *  P                samples per chain (Sec. 3.2: P^r = P^nr = P), 1..1024.
 *  seed, system_id  key and stream of the counter-based generator; one step is
 *                   a pure function of (seed, system_id, step, box, positions).
 *                   system_id and step must be < 2^32.
 *  coulomb_k        prefactor applied to every energy, force and pressure.
 *  precision        RBSOG_PREC_FP64 or RBSOG_PREC_FP32C.
 *  recalibration    how the non-radial modes of eq. P_approx_nr are drawn.
 *                   Every chain starts each step from an exact draw of its
 *                   own target (rejection from the rounded Gaussian sqrt(2)
 *                   wider than App. D's, under a proven bound; Philox
 *                   streams 3, 4, 7, 8, 9), so each recorded state has its
 *                   target's law.
 *                   RBSOG_RECAL_EXCHANGE (default) recalibrates the r-chain's
 *                   states (Sec. 3.2) by swapping the two chains' states when
 *                   the recalibration ratio accepts: both marginals stay
 *                   exact and the estimators are unbiased at any P; up to
 *                   P + 2 distinct modes.
 *                   RBSOG_RECAL_PRINTED is the recalibration chain as
 *                   printed: it treats the repeating r-chain states as
 *                   independent proposals and its non-radial pressure is
 *                   biased by a P-independent amount (+7% and +13% of two
 *                   diagonal components of P^F on a 64-charge test box).
 *                   RBSOG_RECAL_SHARED uses the r-chain's modes themselves,
 *                   each weighted by P^nr/P^r (times S^r/S^nr);
 *                   RBSOG_RECAL_INDEPENDENT draws a second independence MH
 *                   chain for P^nr (Philox streams 5, 6; a rounded Gaussian
 *                   proposal sqrt(2) times wider than the radial one), so
 *                   up to 2P + 2 distinct modes and P <= 512.  The radial
 *                   estimator, the force and the energy always use the r-chain.
 *  flags            0, or RBSOG_FLAG_EXP_FORM.  In FP32C the short-range
 *                   sums sum_l wt_l exp(-r^2/s_l^2) and sum_l w_l exp(-r^2/s_l^2)
 *                   are evaluated as degree-10 polynomials in r^2 on
 *                   [0, rc^2] (Chebyshev interpolants fitted in FP64 at set-up,
 *                   used when their truncation error is below 5e-8 of the sum
 *                   at r = 0, else the exponentials); RBSOG_FLAG_EXP_FORM asks
 *                   for the M exponentials of eqs. force_SOG and U_short.
 *                   The FP32C pair kernel evaluates each pair from both of
 *                   its atoms (the full shell; RBSOG_FLAG_FULL_SHELL states
 *                   it explicitly).  RBSOG_FLAG_HALF_SHELL asks FP32C systems
 *                   with four or more cells per edge to evaluate each
 *                   unordered pair once (Newton's third law; the reactions
 *                   meet in a fixed-order gather, so results stay bitwise
 *                   reproducible) at about 1.2 KB per atom of extra device
 *                   memory; on MI355X it is slower than the full shell (the
 *                   reactions collide in LDS), so it is not the default.
 *                   A step whose neighbourhoods outgrow the half shell's
 *                   buffer (densities above 0.15 atoms/A^3) runs the full
 *                   shell.  The two shells agree to FP32 rounding.
 *  M_energy         0 (= M), or M..RBSOG_MAX_M: Gaussians of the energy
 *                   kernel only (Table 1 asks 25 for the energy of row 2).
 *                   U^N (eq. U_short), U_self and U^{F*} then use M_energy
 *                   terms (w_l for l < M_energy); forces, virial, pressure
 *                   and the sampling keep M.  U^{F*} stays the
 *                   importance-sampled energy under the radial proposal:
 *                   each mode carries the ratio of the M_energy-term energy
 *                   kernel to the M-term one.
 */
typedef struct rbsog_params {
    double b;
    double sigma;
    double omega;
    int32_t M;
    double rc;
    int32_t P;
    uint64_t seed;
    uint64_t system_id;
    double coulomb_k;
    int32_t precision;
    int32_t recalibration;
    int32_t flags;
    int32_t M_energy;
    int32_t reserved[4];
} rbsog_params;

/*
 * Fill *p with Table 1, row 2 (b~ = 1.62976708826776469, sigma~ =
 * 3.270345668108471, omega~ = 1.007806979343806 at r_c = 9 A; the row the
 * paper uses in all runs) rescaled to the cutoff rc by sigma = sigma9 * rc / 9
 * (the split is scale covariant), M = 10 (the pressure column's M~), P = 100,
 * seed 0, system 0, coulomb_k 1, FP32C, exchange recalibration, flags 0,
 * M_energy 0 (= M).
 * Returns RBSOG_EINVAL if p is NULL or rc <= 0.
 */
int rbsog_params_init(rbsog_params *p, double rc);

/*
 * Create a context for one system of n point charges.
 *  host_q[n]    charges (copied; must sum to zero, Sec. 2.2).
 *  host_box[3]  initial box edges (validated against rc).
 *  hip_stream   hipStream_t on which all work of this context is queued
 *               (NULL = the null stream).
 *  out          receives the context.
 * Allocates the context's device buffers (about 120 bytes per atom in FP32C,
 * 200 in FP64, plus per-cell and per-mode arrays).
 */
int rbsog_setup(const rbsog_params *params, int64_t n, const double *host_q,
                const double host_box[3], void *hip_stream, rbsog_ctx **out);

/*
 * Algorithm 1 steps 2-3 for this step and box: computes S^r and S^nr (eqs. Sr,
 * Snr; Poisson forms of Prop. 1 where they converge faster) on the host, then
 * runs both Metropolis-Hastings chains on the device (one workgroup) and
 * builds the set of distinct modes with their multiplicities.
 *  step             step index (< 2^32), part of the generator counter.
 *  host_box[3]      box of this step.
 *  host_m_r[3P], host_m_nr[3P]  optional (NULL): the sampled integer modes of
 *                   both chains, row per sample (forces a stream sync).
 *  host_S[2]        optional (NULL): S^r, S^nr.
 */
int rbsog_sample_modes(rbsog_ctx *ctx, int64_t step, const double host_box[3],
                       int32_t *host_m_r, int32_t *host_m_nr, double host_S[2]);

/*
 * rbsog_sample_modes for a general (triclinic) cell, Sec. 2.1:
 * host_h[9] is the cell tensor h = [h_1, h_2, h_3] row-major, its columns the
 * cell vectors (h[3 i + j] = component i of h_j), det h > 0, and positions
 * are r = h s with s the fractional coordinates.  Modes are k = 2 pi h^-T m;
 * S^r and S^nr are the lattice sums of eqs. Sr, Snr (Prop. 1 forms per
 * Gaussian); the r-chain's proposal is round(h^T u) (App. D) and its pmf, eq.
 * proposal, a Gaussian integral over the unit cube with no closed form, is
 * taken by a 24-point tensor Gauss-Legendre rule.  The following
 * rbsog_force_virial and rbsog_pressure use this cell: short-range pairs by
 * the component-wise fractional minimum image, exact while r_c is at most half
 * the smallest perpendicular width of the cell (RBSOG_EBOX otherwise), on the
 * exact pair path (FP32C and FP64); the pressure tensor is full, shear
 * components included.  A diagonal h is the box of its diagonal.  The first
 * call with a non-diagonal h allocates a 221 KB quadrature table.  General
 * cells are a single-context form: rbsog_rescale refuses them (pass the next
 * cell here) and the batched and served forms take boxes.
 */
int rbsog_sample_modes_cell(rbsog_ctx *ctx, int64_t step, const double host_h[9],
                            int32_t *host_m_r, int32_t *host_m_nr, double host_S[2]);

/*
 * Algorithm 1 steps 4-6 for the positions x, y, z (n each, FP64, the caller's
 * atom order, any periodic image) in the box of the last rbsog_sample_modes:
 * writes the total force F = F^N + F^{F*} into fx, fy, fz (n each, FP64,
 * overwritten).  host_energy[3] (optional) receives U^N, U^{F*}, U_self
 * (U = U^N + U^{F*} - U_self, eq. couldecomp); host_vir[6] (optional) the
 * short-range virial sum (xx, yy, zz, xy, xz, yz), i.e. V P^N.  Requesting
 * either synchronises the stream; with both NULL the call only queues work.
 */
int rbsog_force_virial(rbsog_ctx *ctx, const double *x, const double *y, const double *z,
                       double *fx, double *fy, double *fz, double host_energy[3],
                       double host_vir[6]);

/*
 * Coulomb pressure tensor of the last rbsog_force_virial (Algorithm 1 step 6):
 * host_P[9] (row-major) = P^N + P^{F,r*} + P^{F,nr*}; host_parts[27]
 * (optional) = P^N, P^{F,r*}, P^{F,nr*}, each row-major.  Synchronises.
 */
int rbsog_pressure(rbsog_ctx *ctx, double host_P[9], double host_parts[27]);

/*
 * rbsog_force_virial for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, same kernels and bitwise the same results as
 * rbsog_force_virial; x, y, z and fx, fy, fz must be device arrays.  The
 * step's partial results (structure-factor partials per block and mode, pair
 * sums per pair block) go to a fixed 32 MiB device array of the library, one
 * per GPU, held until the process ends; everything else is the context's.
 * The call allocates nothing, so what rbsog_force_virial would allocate must
 * exist already: after rbsog_setup, and after a box change that grows the
 * cell grid, run rbsog_force_virial once.  Returns RBSOG_ESTATE when the
 * grid, the half-shell buffers or the launch plans would have to grow, and
 * RBSOG_EINVAL (message naming the scratch) when the partials exceed 32 MiB:
 * 16 B per mode and structure-factor block (a block per 1,024 atoms) plus
 * 64 B per pair block.  Calls on one GPU share the array: calls that overlap
 * on one GPU (other streams, other threads, other contexts) race, so a
 * caller serialises them.
 */
int rbsog_force_virial_noalloc(rbsog_ctx *ctx, const double *x, const double *y, const double *z,
                               double *fx, double *fy, double *fz, double host_energy[3],
                               double host_vir[6]);

/*
 * Isotropic or anisotropic box rescale in FP64 on the device (NPT update of
 * Algorithm 1 step 7 for a diagonal h): r <- mu r for the n positions (device
 * arrays) and host_box <- mu host_box.  Fractional coordinates, hence the
 * structure factors, are unchanged (Theorem 1).
 */
int rbsog_rescale(rbsog_ctx *ctx, const double host_mu[3], double *x, double *y, double *z,
                  double host_box[3]);

/*
 * One whole step of Algorithm 1 for a box in one call: the rescale of
 * rbsog_rescale (skipped when host_mu is NULL), the mode sampling of
 * rbsog_sample_modes at the box after it, the forces of rbsog_force_virial
 * and the pressure of rbsog_pressure.  Same kernels, same results, bitwise,
 * as those four calls; the step's data goes to the device in one upload and
 * the binning is queued before the sampler, so fewer host calls sit between
 * the kernels.
 *   step         step index k in [0, 2^32) (the sampler's random stream)
 *   host_mu      scale factors (positive, finite) or NULL
 *   host_box     in: the box before the rescale; out: the box after it
 *   x, y, z      positions (device arrays, n each, FP64), rescaled in place
 *   fx, fy, fz   forces out (device arrays, n each, FP64)
 *   host_P       pressure tensor out (row-major, as rbsog_pressure) or NULL
 *   host_energy  U^N, U^F*, U_self out (as rbsog_force_virial) or NULL;
 *                the energy sum runs only when it is given
 * With host_P or host_energy the call synchronises the stream; with both
 * NULL it only queues work (rbsog_pressure reads the pressure later).
 * Errors: RBSOG_EINVAL for NULL or host arrays, a bad step or bad scale
 * factors; RBSOG_EBOX for a box the cut-off does not fit; RBSOG_ESTATE for a
 * context holding a general cell or admitted to a batch; RBSOG_EDEVICE for a
 * HIP error or a sampler without an accepted start.  An error found before
 * any work is queued leaves host_box and the positions unchanged.
 */
int rbsog_step(rbsog_ctx *ctx, int64_t step, const double host_mu[3], double host_box[3], double *x,
               double *y, double *z, double *fx, double *fy, double *fz, double host_P[9],
               double host_energy[3]);

/*
 * rbsog_step without waiting for its results: queues the step (arguments as
 * rbsog_step; energy nonzero runs the energy sum) and, behind it on the same
 * stream, the copy of its results into one of four pinned slots of the
 * context, and returns a ticket in *ticket (0, 1, 2, ... per context).  The
 * host is then free to queue the next step while the device works, so a
 * stepping loop that reads each step's pressure one step later keeps the
 * device busy across step boundaries.  A fifth queued step reuses the slot
 * of the first: the call then waits for that slot's copy, and that ticket's
 * results are gone.  host_box is updated when the call returns, as in
 * rbsog_step; the forces are in fx, fy, fz once the step has run.
 */
int rbsog_step_async(rbsog_ctx *ctx, int64_t step, const double host_mu[3], double host_box[3], double *x,
                     double *y, double *z, double *fx, double *fy, double *fz, int32_t energy,
                     int64_t *ticket);

/*
 * Waits for the step of a ticket from rbsog_step_async and returns its
 * pressure tensor (host_P, row-major, as rbsog_pressure) and energies
 * (host_energy, as rbsog_force_virial; zeros unless that step ran the energy
 * sum); either may be NULL.  RBSOG_EINVAL for a ticket that was never issued
 * or whose slot a later step has taken (more than four steps ago);
 * RBSOG_EDEVICE and RBSOG_EINVAL as rbsog_pressure for that step's sampler
 * and input checks.  A ticket may be waited on more than once.
 */
int rbsog_step_wait(rbsog_ctx *ctx, int64_t ticket, double host_P[9], double host_energy[3]);

/* Free the context and its device buffers (NULL is a no-op). */
int rbsog_destroy(rbsog_ctx *ctx);

/* Static message for an error code. */
const char *rbsog_strerror(int code);

/* Message of the context's last failure ("" if none); valid until the next call. */
const char *rbsog_last_error(const rbsog_ctx *ctx);

/*
 * Inspection (tests and tools).
 *  rbsog_debug_cells: cell id of every atom (caller order) from the last
 *    rbsog_force_virial, cell = cx + nx (cy + ny cz) with cx = (u nx) >> 32
 *    and u the 32-bit fixed-point fractional coordinate; host_ncell[3] gets
 *    (nx, ny, nz).  host_cell may be NULL.
 *  rbsog_debug_modes: number of distinct modes; host_modes[3*cap] their
 *    integer vectors, host_counts[2*cap] their multiplicities in the r- and
 *    nr-chains, host_rho[2*cap] (after rbsog_force_virial) Re, Im of rho.
 *    Any output may be NULL; at most cap entries are written.
 */
int rbsog_debug_cells(rbsog_ctx *ctx, int32_t *host_cell, int32_t host_ncell[3]);
/*
 *  rbsog_debug_long_range_force: the random-batch long-range force F^{F*} of
 *    the last rbsog_force_virial alone (eq. f_approx, times coulomb_k), into
 *    device arrays fx, fy, fz (n each, caller order).  Synchronises.
 */
int rbsog_debug_long_range_force(rbsog_ctx *ctx, double *fx, double *fy, double *fz);
int rbsog_debug_modes(rbsog_ctx *ctx, int32_t cap, int32_t *host_nd, int32_t *host_modes,
                      int32_t *host_counts, double *host_rho);

/*
 * Counters of the last evaluation (synchronises): host_info[0] = number of
 * distinct sampled modes (structure factors evaluated), [1] and [2] =
 * accepted moves of the r-chain and of the recalibration chain, [3] = number
 * of unordered pairs inside r_c.
 */
int rbsog_step_info(rbsog_ctx *ctx, int64_t host_info[4]);

/*
 * Per-kernel device timing with HIP events on the context's stream.
 * rbsog_set_timing(ctx, 1) starts recording every kernel launch of
 * rbsog_sample_modes and rbsog_force_virial, rbsog_set_timing(ctx, 2) the
 * pair kernel's launches only (each recorded event can delay the next
 * launch by a few microseconds); rbsog_get_timing writes, for
 * each kernel k < cap, its name into host_names[k] (up to 31 chars + NUL,
 * 32 bytes per entry), total milliseconds into host_ms[k] and launch count
 * into host_count[k], returning the number of kernels through *host_nk.
 * Reading synchronises; rbsog_set_timing(ctx, 0) stops and clears.
 */
int rbsog_set_timing(rbsog_ctx *ctx, int on);
int rbsog_get_timing(rbsog_ctx *ctx, int32_t cap, int32_t *host_nk, char *host_names,
                     double *host_ms, int64_t *host_count);

/* Library version: major * 10000 + minor * 100 + patch. */
int rbsog_version(void);

/* ========================================================================
 * NPT integration around the evaluation (Algorithm 1 step 7): the Langevin
 * equations of motion of eq. Langevin_NPT for a diagonal h, with the
 * random-batch force and the instantaneous pressure
 * P_ins = P_coul (this library) + sum_i p_i (x) p_i / (m_i V) (eq.
 * K_U_Pins_re; the caller's other interactions are not included).
 *
 * One step of length dt is the symmetric splitting
 *   B_h(dt/2) B(dt/2) A(dt/2) O(dt) A(dt/2) [evaluate F, P] B(dt/2) B_h(dt/2)
 *   B_h: p^h_g += t G_g,  G_g = (V / L_g) sum_{mu in g} (P_ins,mumu - p_ext)
 *                               - n_g kT / L_g
 *   B:   p_i += t F_i
 *   A:   L_g += t p^h_g / (n_g M); per axis a = L_new/L_old,
 *        r_i <- a r_i + t p_i/m_i,  p_i <- p_i / a
 *        (the exact flow of r' = p/m + (L'/L) r, p' = -(L'/L) p, L' = p^h/M
 *        with p^h held fixed)
 *   O:   p_i <- c p_i + sqrt((1 - c^2) kT m_i) xi_i,  c = exp(-gamma dt);
 *        p^h_g <- c_h p^h_g + sqrt((1 - c_h^2) kT n_g M) xi_g,
 *        c_h = exp(-gamma_box dt)
 * where the box degrees of freedom g are the axes (RBSOG_COUPLE_ANISO), x+y
 * and z (RBSOG_COUPLE_SEMI, needs Lx = Ly) or all three (RBSOG_COUPLE_ISO,
 * needs a cube); coupled axes share one momentum and keep equal lengths.  The
 * normals xi are Philox4x32-10 draws keyed by (seed, system_id) of the
 * context with counter (atom, 16|17, step, system_id) for atoms and
 * (0|1, 18, step, system_id) for the box.  Units are the caller's: F and P
 * carry coulomb_k, kT is in the same energy unit, masses and dt consistent.
 * ======================================================================== */

#define RBSOG_COUPLE_ANISO 0 /* each axis its own box momentum               */
#define RBSOG_COUPLE_SEMI 1  /* x and y share one (Lx = Ly), z its own        */
#define RBSOG_COUPLE_ISO 2   /* one for all three axes (cubic box)            */

typedef struct {
    double dt;          /* time step                                              */
    double kT;          /* thermal energy                                         */
    double gamma;       /* particle friction (1 / time)                           */
    double gamma_box;   /* box friction (1 / time)                                */
    double box_mass;    /* M per box axis                                         */
    double p_ext;       /* external pressure (energy / length^3)                  */
    int32_t coupling;   /* RBSOG_COUPLE_*                                         */
    int32_t reserved[7];
} rbsog_npt_params;

/*
 * Attach the integrator to a context: parameters and the n masses
 * (host_mass, caller order, all > 0).  Device memory: 56 B per atom.
 * Errors: EINVAL for bad parameters or masses.
 */
int rbsog_npt_init(rbsog_ctx *ctx, const rbsog_npt_params *params, const double *host_mass);

/*
 * Advance nsteps steps from the state (x, y, z, px, py, pz; device arrays,
 * caller order, updated in place; host_box[3], host_pbox[3] box lengths and
 * momenta per axis, updated in place).  The forces and pressure are
 * evaluated at the starting state first; the evaluation after step k samples
 * its modes with step index first_step + k, and step k draws its noise with
 * step index first_step + k.  host_P_ins[9] (optional) receives the
 * instantaneous pressure tensor at the end (row-major), host_P_kin[9]
 * (optional) its kinetic part.  Synchronises twice per step.
 * Errors: ESTATE before rbsog_npt_init; EINVAL for host arrays or a coupled
 * group with unequal lengths; EBOX if the box shrinks below the cutoff rule.
 */
int rbsog_npt_run(rbsog_ctx *ctx, double *x, double *y, double *z, double *px, double *py, double *pz,
                  int64_t first_step, int32_t nsteps, double host_box[3], double host_pbox[3],
                  double host_P_ins[9], double host_P_kin[9]);

/* ========================================================================
 * Batched form: many independent systems of uneven size evaluated by one set
 * of launches per step.  Each launch covers every system; workgroups find
 * their (system, block) in a launch plan, and every reduction runs over one
 * system's partials in a fixed order, so a system's results are bitwise the
 * same alone (rbsog_setup, or a batch of one) and in any batch.  One step of
 * one system is the same computation as the single-system calls above
 * (Algorithm 1, steps 2-6).
 * ======================================================================== */

typedef struct rbsog_batch rbsog_batch;

#define RBSOG_SCHED_STATIC 0     /* one workgroup per pair block                     */
#define RBSOG_SCHED_PERSISTENT 1 /* a fixed grid takes pair blocks from a work queue */

/*
 * Create a batch of nsys systems (1..65536).
 *  params[nsys]       per-system parameters (as for rbsog_setup); every system
 *                     must use the same precision.
 *  n[nsys]            atoms per system.
 *  host_q[sum n]      charges, system after system (each system neutral).
 *  host_boxes[3 nsys] initial box edges.
 *  hip_stream         stream for all work of the batch (NULL = null stream).
 * Device memory: one allocation per system, about what rbsog_setup takes.
 */
int rbsog_batch_setup(const rbsog_params *params, int32_t nsys, const int64_t *n, const double *host_q,
                      const double *host_boxes, void *hip_stream, rbsog_batch **out);

/*
 * One full step of every system: mode sampling, binning, pair kernel,
 * structure factors, estimators, forces (Algorithm 1 steps 2-6).
 *  host_steps[nsys]   step index of each system (< 2^32, generator counter).
 *  host_boxes[3 nsys] box of each system for this step.
 *  x, y, z            device arrays of sum n positions, system after system.
 *  fx, fy, fz         device arrays of sum n forces (overwritten).
 *  host_P[9 nsys]     optional: total pressure tensor of each system.
 *  host_energy[3 nsys] optional: U^N, U^{F*}, U_self of each system.
 *  host_info[4 nsys]  optional: the counters of rbsog_step_info per system.
 * Asking for any host output synchronises the stream.
 */
int rbsog_batch_step(rbsog_batch *b, const int64_t *host_steps, const double *host_boxes, const double *x,
                     const double *y, const double *z, double *fx, double *fy, double *fz, double *host_P,
                     double *host_energy, int64_t *host_info);

/*
 * r <- mu_s r for the positions of each system s (device arrays laid out as
 * in rbsog_batch_step) and host_boxes[3 s + d] <- mu[3 s + d] host_boxes[3 s + d].
 */
int rbsog_batch_rescale(rbsog_batch *b, const double *host_mu, double *x, double *y, double *z,
                        double *host_boxes);

/*
 * Launch options; none changes any result.
 *  schedule      RBSOG_SCHED_STATIC or RBSOG_SCHED_PERSISTENT (pair kernel).
 *  wg_per_cu     workgroups per compute unit of the persistent grid (1..64).
 *  use_graph     nonzero: rbsog_batch_step replays a captured HIP graph of
 *                the step's launches (captured again when sizes change).
 */
int rbsog_batch_set_options(rbsog_batch *b, int32_t schedule, int32_t wg_per_cu, int32_t use_graph);

/*
 * Autotuner: times rbsog_batch_step on the given arrays for each launch
 * option in a fixed candidate list (static; persistent with 4, 8, 16, 32
 * workgroups per CU), reps steps each after one warm-up, and keeps the
 * fastest.  host_ms[5] (optional) receives the mean step time of each
 * candidate, *host_choice (optional) the index chosen.  The forces and the
 * step's results are those of a regular step.
 */
int rbsog_batch_autotune(rbsog_batch *b, const int64_t *host_steps, const double *host_boxes, const double *x,
                         const double *y, const double *z, double *fx, double *fy, double *fz, int32_t reps,
                         double *host_ms, int32_t *host_choice);

/*
 * Cached autotuner.  The candidates are the pair kernel's schedules of
 * rbsog_batch_autotune, each with and without graph replay of the step
 * (RBSOG_TUNE_CANDIDATES = 10: index c < 5 is schedule c of that list
 * without, c + 5 the same with graph replay).  None changes any operation or
 * the order of any sum, so results are bitwise the same under every choice.
 * The key is the device (architecture and number of compute units), the
 * batch's total atoms rounded down to a power of two and its largest P
 * rounded up to one.
 *  cache_path    a text file, one line per tuning: "<key>|<index> <ms> ..."
 *                (created when missing; the last line of a key counts).
 *  force         nonzero: time the candidates even when the key is cached.
 * When the key is found (and force is 0) its choice is applied without a
 * step; otherwise every candidate is timed as in rbsog_batch_autotune (one
 * untimed step, then reps timed steps on the given arrays) and the fastest
 * is applied and appended to the file.  host_ms[RBSOG_TUNE_CANDIDATES]
 * (optional) receives the mean step time of each timed candidate (on a hit,
 * only the chosen one's, from the file; the others 0), *host_choice the index
 * applied and *host_cached 1 on a hit.  RBSOG_EINVAL when the file cannot be
 * written or for a batch of contexts.  Calls within one process read and
 * write the file one at a time; several processes sharing a file may each
 * append a line for the same key.
 */
#define RBSOG_TUNE_CANDIDATES 10
int rbsog_batch_autotune_cached(rbsog_batch *b, const char *cache_path, int32_t force, const int64_t *host_steps,
                                const double *host_boxes, const double *x, const double *y, const double *z,
                                double *fx, double *fy, double *fz, int32_t reps, double *host_ms,
                                int32_t *host_choice, int32_t *host_cached);

/*
 * A batch of existing contexts, admitted by device memory.
 *  rbsog_batch_create   an empty batch whose admitted contexts may hold at most
 *                       mem_budget_bytes of device memory together; work is
 *                       queued on hip_stream (NULL = the null stream).
 *  rbsog_batch_admit    adds a context (the contexts of one batch share one
 *                       precision).  RBSOG_EAGAIN if its device memory (the
 *                       buffers rbsog_setup allocated, grown to its current
 *                       grid) exceeds what the budget has left or 65,536
 *                       contexts are admitted; RBSOG_ESTATE if it is admitted
 *                       elsewhere.  Waits for the context's own queued work.
 *  rbsog_stage          the next step of an admitted context: step index, box
 *                       and device arrays of positions and forces (n each,
 *                       caller order), kept by the caller until the batched
 *                       step has run.
 *  rbsog_batch_step     with every array argument NULL, one step of every
 *                       admitted context from its staged inputs (the launches
 *                       of rbsog_batch_step below, one set for all contexts),
 *                       then synchronises; host_P, host_energy, host_info as
 *                       below, in admission order.  Each context's
 *                       rbsog_pressure and rbsog_step_info then report its
 *                       own results.  RBSOG_ESTATE if a context has no staged
 *                       step.
 *  rbsog_batch_release  removes a context (waits for the batch's queued work);
 *                       rbsog_destroy of an admitted context releases it first.
 * While admitted, a context's own evaluation calls (sample, force, rescale,
 * debug, NPT) return RBSOG_ESTATE.  A context's results are bitwise the same
 * alone and in any batch.  rbsog_batch_rescale and rbsog_batch_autotune's
 * array arguments do not apply to a batch of contexts.
 */
int rbsog_batch_create(int64_t mem_budget_bytes, void *hip_stream, rbsog_batch **out);
int rbsog_batch_admit(rbsog_batch *b, rbsog_ctx *ctx);
int rbsog_stage(rbsog_ctx *ctx, int64_t step, const double host_box[3], const double *x, const double *y,
                const double *z, double *fx, double *fy, double *fz);
int rbsog_batch_release(rbsog_batch *b, rbsog_ctx *ctx);

/* Per-kernel HIP-event timing of the batch's launches (as rbsog_set_timing). */
int rbsog_batch_set_timing(rbsog_batch *b, int on);
int rbsog_batch_get_timing(rbsog_batch *b, int32_t cap, int32_t *host_nk, char *host_names, double *host_ms,
                           int64_t *host_count);

int rbsog_batch_destroy(rbsog_batch *b);
const char *rbsog_batch_last_error(const rbsog_batch *b);

/* ========================================================================
 * Served form: a request loop on a worker thread.  A request is one system
 * and a number of steps under the box law L_k = L_0 (1 + g k) (positions
 * rescaled by mu_k = (1 + g k)/(1 + g (k - 1)) before step k, k >= 1); it is
 * admitted when a slot and device memory from the server's pool are free,
 * its state stays on the device until it completes, and every tick runs one
 * batched step over all admitted requests, so requests that arrive while
 * others run join the next tick (continuous batching).  Results are bitwise
 * those of the same request alone.
 * ======================================================================== */

typedef struct rbsog_server rbsog_server;

/*
 * precision      RBSOG_PREC_FP32C or RBSOG_PREC_FP64 (all requests).
 * pool_bytes     device memory for request state (> 0); admission allocates
 *                from it first-fit.
 * max_active     requests per tick (>= 1); 1 serves one request at a time.
 */
int rbsog_server_create(int32_t precision, int64_t pool_bytes, int32_t max_active, void *hip_stream,
                        rbsog_server **out);

/*
 * Whether the server's steps sum the energies (on: the default).  Off, the
 * pair kernel skips the energy sum and rbsog_server_wait returns zeros for
 * them; the forces then take the relative-coordinate displacements of the
 * call without energy (they differ from the energy-on forces by rounding).
 * One setting holds for every request, so a request's results never depend
 * on its neighbours in a tick: RBSOG_ESTATE once a request was submitted.
 */
int rbsog_server_set_energy(rbsog_server *s, int32_t on);

/*
 * Queue a request (copies every input; returns at once).
 *  params         parameters of the system (params->precision must match).
 *  n, host_q[n]   charges; host_x, host_y, host_z[n] initial positions.
 *  host_box[3]    initial box; nsteps >= 1 steps; growth g (L_k = L_0 (1 + g k)).
 *  *ticket        receives the request's ticket.
 * Returns RBSOG_EAGAIN if the request can never fit the pool.
 */
int rbsog_server_submit(rbsog_server *s, const rbsog_params *params, int64_t n, const double *host_q,
                        const double *host_x, const double *host_y, const double *host_z,
                        const double host_box[3], int32_t nsteps, double growth, int64_t *ticket);

/*
 * Wait up to timeout_s seconds (< 0: forever) for a request; RBSOG_EAGAIN if
 * it has not completed.  On completion copies out (each optional)
 *  host_fx, host_fy, host_fz[n]  forces of the last step,
 *  host_P[9 nsteps]              pressure tensor of every step,
 *  host_energy[3 nsteps]         U^N, U^{F*}, U_self of every step,
 *  host_times[3]                 seconds from submission to admission, from
 *                                submission to completion, and the number of
 *                                ticks the request shared with others,
 * and releases the ticket.
 */
int rbsog_server_wait(rbsog_server *s, int64_t ticket, double timeout_s, double *host_fx, double *host_fy,
                      double *host_fz, double *host_P, double *host_energy, double *host_times);

/*
 * host_stats[11]: requests submitted, completed, ticks run, atom-steps done,
 * seconds the worker spent in ticks, peak active requests, peak pool bytes
 * in use, requests waiting now, and the ticks' seconds split three ways:
 * handing over completed requests' forces, admitting and uploading requests
 * and queuing a tick's copies (while a tick runs); setting up and launching
 * the batched steps; waiting for a tick's end.
 */
int rbsog_server_stats(rbsog_server *s, double *host_stats);

/* Stop the worker (finishing the tick in flight) and free everything. */
int rbsog_server_destroy(rbsog_server *s);
const char *rbsog_server_last_error(const rbsog_server *s);

#ifdef __cplusplus
}
#endif

#endif /* RBSOG_H */
