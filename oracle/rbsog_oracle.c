/*
 * FP64 CPU oracle for the random batch sum-of-Gaussians (RBSOG) electrostatic
 * force and pressure evaluation of Jiang, Liang and Zhou, "Random batch
 * sum-of-Gaussians method for molecular dynamics simulation of particle systems
 * in the NPT ensemble" (arXiv:2602.23582).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no source,
 * header, table, constant or helper with the HIP library: every formula here
 * is written out again from the paper, in plain double-precision loops, with
 * no blocking, fusion or reordering beyond what the formula itself states.
 *
 * Orthorhombic cells h = diag(Lx, Ly, Lz) throughout, and general (triclinic)
 * cells in the orc_tri_* functions at the end.  Gaussian units (prefactor 1).
 *
 * Parity status per function is given in its comment; "parity unpinned" marks
 * a function that no test pins to anything but itself.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------- */
/* SOG splitting parameters                                                  */
/* ------------------------------------------------------------------------- */

/*
 * u-series weights of 1/r (Sec. 2.2, eq. long):
 *     w_l = (pi/2)^(-1/2) sigma^-1 b^-l log b,   s_l = sqrt(2) b^l sigma,
 * weights of the 1/r^3 split (Sec. 3.1, definition after eq. approxerror):
 *     wt_l = (pi/2)^(-1/2) log b b^(-3l) sigma^-3, with st_l = s_l,
 * and the narrowest Gaussian rescaled by omega in both (Sec. 2.2 w_0 update,
 * eq. omega0; omega = omega~ by Theorem 2).
 * Pinned by: Table 1 continuity residuals and the self-energy closed form.
 */
void orc_sog_params(double b, double sigma, double omega, int M,
                    double *w, double *wt, double *s)
{
    const double c = sqrt(2.0 / ORC_PI) * log(b);
    for (int l = 0; l < M; ++l) {
        const double bl = pow(b, (double)l);
        w[l] = c / (sigma * bl);
        wt[l] = c / (bl * bl * bl * sigma * sigma * sigma);
        s[l] = sqrt(2.0) * bl * sigma;
    }
    w[0] *= omega;
    wt[0] *= omega;
}

/* F(r) = sum_l w_l exp(-r^2/s_l^2)   (eq. long) */
double orc_F(int M, const double *w, const double *s, double r)
{
    double acc = 0.0;
    for (int l = 0; l < M; ++l) acc += w[l] * exp(-r * r / (s[l] * s[l]));
    return acc;
}

/* F~(r) = sum_l wt_l exp(-r^2/s_l^2)   (eq. pressure_split) */
double orc_Ft(int M, const double *wt, const double *s, double r)
{
    double acc = 0.0;
    for (int l = 0; l < M; ++l) acc += wt[l] * exp(-r * r / (s[l] * s[l]));
    return acc;
}

/*
 * omega~ from C0 continuity of the 1/r^3 split at rc (eq. continuity):
 * 1/rc^3 - F~(rc) = 0 is linear in the factor applied to wt_0 (eq. omega0).
 * Pinned by: reproduces the omega column of Table 1 for M >= 20.
 */
double orc_omega_c0(double b, double sigma, double rc, int M)
{
    double *w = malloc(sizeof(double) * M), *wt = malloc(sizeof(double) * M),
           *s = malloc(sizeof(double) * M);
    orc_sog_params(b, sigma, 1.0, M, w, wt, s);
    double rest = 0.0;
    for (int l = 1; l < M; ++l) rest += wt[l] * exp(-rc * rc / (s[l] * s[l]));
    const double omega = (1.0 / (rc * rc * rc) - rest) / (wt[0] * exp(-rc * rc / (s[0] * s[0])));
    free(w); free(wt); free(s);
    return omega;
}

/*
 * Bilateral series approximation of 1/r^beta (eq. BSA_beta), summed over
 * l in [lmin, lmax]:
 *   2 log b / ((sqrt2 sigma)^beta Gamma(beta/2)) sum_l b^(-beta l) exp(-(r/(b^l sigma))^2 / 2).
 * Pinned by: the error bound of eq. BSA_err.
 */
double orc_bsa(double beta, double b, double sigma, double r, int lmin, int lmax)
{
    double acc = 0.0;
    for (int l = lmax; l >= lmin; --l) {
        const double bl = pow(b, (double)l);
        const double t = r / (bl * sigma);
        acc += pow(b, -beta * l) * exp(-0.5 * t * t);
    }
    return 2.0 * log(b) / (pow(sqrt(2.0) * sigma, beta) * tgamma(0.5 * beta)) * acc;
}

/* right-hand side of eq. BSA_err */
double orc_bsa_bound(double beta, double b)
{
    const double lb = log(b);
    return 2.0 * sqrt(2.0 * ORC_PI) / tgamma(0.5 * beta) *
           pow(0.25 * beta * beta + ORC_PI * ORC_PI / (lb * lb), 0.25 * (beta - 1.0)) *
           exp(-ORC_PI * ORC_PI / (2.0 * lb));
}

/* ------------------------------------------------------------------------- */
/* Normalisation constants S^r, S^nr                                          */
/* ------------------------------------------------------------------------- */

/* exponent at which lattice sums are truncated: exp(-60) ~ 1e-26 */
#define ORC_TRUNC 60.0

/*
 * One Gaussian's H^r_l and H^nr_l by the direct reciprocal-lattice sums of
 * eqs. Sr and Snr, k = 2 pi h^-T m:
 *   H^r  = sum_m pi^(3/2) wt s^5 |k|^2 exp(-s^2 |k|^2 / 4)
 *   H^nr = sum_m pi^(3/2) wt s^7 |k|^4 exp(-s^2 |k|^2 / 4)
 * Pinned by: equality with the Poisson forms (Prop. 1) and the large-box limit
 * H^r -> 6 V wt, H^nr -> 60 V wt (integral approximation, Theorem 4 proof).
 */
void orc_H_direct(const double L[3], double wt, double s, double *Hr, double *Hnr)
{
    int mmax[3];
    for (int d = 0; d < 3; ++d)
        mmax[d] = (int)ceil(L[d] * sqrt(4.0 * ORC_TRUNC) / (2.0 * ORC_PI * s)) + 1;
    const double pre = pow(ORC_PI, 1.5) * wt;
    double ar = 0.0, anr = 0.0;
    for (int mx = -mmax[0]; mx <= mmax[0]; ++mx)
        for (int my = -mmax[1]; my <= mmax[1]; ++my)
            for (int mz = -mmax[2]; mz <= mmax[2]; ++mz) {
                const double kx = 2.0 * ORC_PI * mx / L[0];
                const double ky = 2.0 * ORC_PI * my / L[1];
                const double kz = 2.0 * ORC_PI * mz / L[2];
                const double k2 = kx * kx + ky * ky + kz * kz;
                const double e = exp(-s * s * k2 / 4.0);
                ar += pow(s, 5) * k2 * e;
                anr += pow(s, 7) * k2 * k2 * e;
            }
    *Hr = pre * ar;
    *Hnr = pre * anr;
}

/*
 * Poisson-summation forms of Prop. 1 (eqs. H2, H2r):
 *   H^r  = V wt [6 A0 - 4 A2 / s^2]
 *   H^nr = V wt [60 A0 - 80 A2 / s^2 + 16 A4 / s^4]
 *   A_j  = sum_n |h n|^j exp(-|h n|^2 / s^2)
 * Pinned by: equality with the direct sums.
 */
void orc_H_poisson(const double L[3], double wt, double s, double *Hr, double *Hnr)
{
    int nmax[3];
    for (int d = 0; d < 3; ++d) nmax[d] = (int)ceil(s * sqrt(ORC_TRUNC) / L[d]) + 1;
    double A0 = 0.0, A2 = 0.0, A4 = 0.0;
    for (int nx = -nmax[0]; nx <= nmax[0]; ++nx)
        for (int ny = -nmax[1]; ny <= nmax[1]; ++ny)
            for (int nz = -nmax[2]; nz <= nmax[2]; ++nz) {
                const double rx = L[0] * nx, ry = L[1] * ny, rz = L[2] * nz;
                const double r2 = rx * rx + ry * ry + rz * rz;
                const double e = exp(-r2 / (s * s));
                A0 += e;
                A2 += r2 * e;
                A4 += r2 * r2 * e;
            }
    const double V = L[0] * L[1] * L[2];
    *Hr = V * wt * (6.0 * A0 - 4.0 * A2 / (s * s));
    *Hnr = V * wt * (60.0 * A0 - 80.0 * A2 / (s * s) + 16.0 * A4 / (s * s * s * s));
}

/*
 * S^r = sum_l H^r_l (eq. Sr) and S^nr = sum_l H^nr_l (eq. Snr).  Per Gaussian
 * the Poisson form is used when s_l < min L (it converges in few terms and has
 * no cancellation there) and the direct form otherwise (the choice of Sec. 3.2
 * after eq. Snr, read as "the sum with the shorter truncation").
 * form: 0 = per-Gaussian choice, 1 = all direct, 2 = all Poisson.
 */
void orc_norm_consts(const double L[3], int M, const double *wt, const double *s, int form,
                     double *Sr, double *Snr)
{
    const double Lmin = fmin(L[0], fmin(L[1], L[2]));
    double sr = 0.0, snr = 0.0;
    for (int l = 0; l < M; ++l) {
        double hr, hnr;
        const int poisson = (form == 2) || (form == 0 && s[l] < Lmin);
        if (poisson) orc_H_poisson(L, wt[l], s[l], &hr, &hnr);
        else orc_H_direct(L, wt[l], s[l], &hr, &hnr);
        sr += hr;
        snr += hnr;
    }
    *Sr = sr;
    *Snr = snr;
}

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers                                              */
/* ------------------------------------------------------------------------- */

/*
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications by
 * 0xD2511F53 and 0xCD9E8D57, key bumped by the Weyl constants 0x9E3779B9 and
 * 0xBB67AE85 between rounds.  The paper leaves the generator open; this is the
 * reading taken for it.  Pinned by: the generator's published known-answer
 * vectors.
 */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in (0,1) from two 32-bit words: the top 52 bits of (a:b), centred */
static double orc_uniform(uint32_t a, uint32_t b)
{
    const uint64_t w = ((uint64_t)a << 32) | (uint64_t)b;
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

/* The draws of one sampling step.  Counter (t, stream, step, system id), key = seed. */
static void orc_draw(uint64_t seed, uint64_t sys, uint64_t step, uint32_t t, uint32_t stream,
                     double *ua, double *ub)
{
    const uint32_t ctr[4] = {t, stream, (uint32_t)step, (uint32_t)sys};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    *ua = orc_uniform(o[0], o[1]);
    *ub = orc_uniform(o[2], o[3]);
}

/*
 * Raw inputs of one proposal, exposed for tests: three standard normals by the
 * Box-Muller transform of four uniforms (streams sxy and sz), and two
 * acceptance uniforms (stream 2).
 */
void orc_draw_proposal(uint64_t seed, uint64_t sys, uint64_t step, uint32_t t,
                       uint32_t sxy, uint32_t sz, double z[3], double uacc[2])
{
    double u1, u2, u3, u4;
    orc_draw(seed, sys, step, t, sxy, &u1, &u2);
    orc_draw(seed, sys, step, t, sz, &u3, &u4);
    const double r1 = sqrt(-2.0 * log(u1));
    const double r2 = sqrt(-2.0 * log(u3));
    z[0] = r1 * cos(2.0 * ORC_PI * u2);
    z[1] = r1 * sin(2.0 * ORC_PI * u2);
    z[2] = r2 * cos(2.0 * ORC_PI * u4);
    if (uacc) orc_draw(seed, sys, step, t, 2u, &uacc[0], &uacc[1]);
}

/*
 * Standard normals of the Langevin noise of one integration step (eq.
 * Langevin_NPT): atom i gets three from the draws with counter (i, 16, step,
 * sys) and (i, 17, step, sys) (Box-Muller, as for a proposal); the box gets
 * three from (0, 18, step, sys) and (1, 18, step, sys).  A reading: the paper
 * leaves the noise generator open.
 */
void orc_npt_normals(uint64_t seed, uint64_t sys, uint64_t step, int64_t n, double *z_atoms, double z_box[3])
{
    for (int64_t i = 0; i < n; ++i) orc_draw_proposal(seed, sys, step, (uint32_t)i, 16u, 17u, z_atoms + 3 * i, NULL);
    double u1, u2, u3, u4;
    orc_draw(seed, sys, step, 0u, 18u, &u1, &u2);
    orc_draw(seed, sys, step, 1u, 18u, &u3, &u4);
    z_box[0] = sqrt(-2.0 * log(u1)) * cos(2.0 * ORC_PI * u2);
    z_box[1] = sqrt(-2.0 * log(u1)) * sin(2.0 * ORC_PI * u2);
    z_box[2] = sqrt(-2.0 * log(u3)) * cos(2.0 * ORC_PI * u4);
}

/* ------------------------------------------------------------------------- */
/* Mode sampling: App. D (r-chain) and Sec. 3.2 (measure recalibration)       */
/* ------------------------------------------------------------------------- */

static double orc_k2(const int32_t m[3], const double L[3])
{
    double k2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double k = 2.0 * ORC_PI * m[d] / L[d];
        k2 += k * k;
    }
    return k2;
}

/*
 * Unnormalised radial target of eq. samplingP on the integer lattice (App. D):
 *   g(m) = |k|^2 sum_l wt_l s_l^5 exp(-s_l^2 |k|^2 / 4),  k = 2 pi h^-T m.
 * The constant pi^(3/2)/S^r cancels in every acceptance ratio.
 */
double orc_target_r(const int32_t m[3], const double L[3], int M, const double *wt, const double *s)
{
    const double k2 = orc_k2(m, L);
    double acc = 0.0;
    for (int l = 0; l < M; ++l) acc += wt[l] * pow(s[l], 5) * exp(-s[l] * s[l] * k2 / 4.0);
    return k2 * acc;
}

/*
 * Ratio P^nr / P^r of eqs. samplingPnr and samplingP up to the constant
 * S^r/S^nr (which cancels in the recalibration acceptance ratio):
 *   R(m) = |k|^2 sum_l wt_l s_l^7 e_l / sum_l wt_l s_l^5 e_l.
 */
double orc_ratio_nr(const int32_t m[3], const double L[3], int M, const double *wt, const double *s)
{
    const double k2 = orc_k2(m, L);
    double a7 = 0.0, a5 = 0.0;
    for (int l = 0; l < M; ++l) {
        const double e = exp(-s[l] * s[l] * k2 / 4.0);
        a7 += wt[l] * pow(s[l], 7) * e;
        a5 += wt[l] * pow(s[l], 5) * e;
    }
    return k2 * a7 / a5;
}

/*
 * Proposal pmf of eq. proposal for h = diag(L): the Gaussian integral over the
 * unit cell around m factorises into one-dimensional normal probabilities with
 * standard deviation sig_xi = L_xi / (sqrt2 pi s0); per dimension
 *   q1(m) = Phi((m+1/2)/sig) - Phi((m-1/2)/sig),
 * written through erf/erfc so that no tail probability cancels.
 */
static double orc_q1(int32_t m, double sig)
{
    const double a = 1.0 / (sqrt(2.0) * sig);
    if (m == 0) return erf(0.5 * a);
    const double am = fabs((double)m);
    return 0.5 * (erfc((am - 0.5) * a) - erfc((am + 0.5) * a));
}

double orc_proposal_pmf(const int32_t m[3], const double L[3], double s0)
{
    double q = 1.0;
    for (int d = 0; d < 3; ++d) q *= orc_q1(m[d], L[d] / (sqrt(2.0) * ORC_PI * s0));
    return q;
}

/* m* = round(h^T u), u_xi ~ N(0, 1/(2 pi^2 s0^2)): m*_xi = round(sig_xi z_xi), half away from zero */
static void orc_round_proposal(const double z[3], const double L[3], double s0, int32_t m[3])
{
    for (int d = 0; d < 3; ++d) {
        const double sig = L[d] / (sqrt(2.0) * ORC_PI * s0);
        double v = round(sig * z[d]);
        if (v > 1073741824.0) v = 1073741824.0;
        if (v < -1073741824.0) v = -1073741824.0;
        m[d] = (int32_t)v;
    }
}

/* importance weight of a lattice point: target / proposal (0 at m = 0) */
static double orc_weight(const int32_t m[3], const double L[3], int M, const double *wt, const double *s)
{
    if (m[0] == 0 && m[1] == 0 && m[2] == 0) return 0.0;
    return orc_target_r(m, L, M, wt, s) / orc_proposal_pmf(m, L, s[0]);
}

/*
 * Importance weight of the independent non-radial chain: unnormalised P^nr,
 * |k|^2 g(m) R(m) = |k|^4 sum_l wt_l s_l^7 e_l, over the pmf of a rounded
 * Gaussian proposal ORC_NR_WIDEN^-1 times wider than the radial one (width
 * parameter s_0 ORC_NR_WIDEN), so that the weight stays bounded in the tail
 * where P^nr decays like |k|^4 e^{-s_0^2 |k|^2/4}.  0 at m = 0.
 */
#define ORC_NR_WIDEN 0.70710678118654752440
static double orc_weight_nr(const int32_t m[3], const double L[3], int M, const double *wt, const double *s)
{
    if (m[0] == 0 && m[1] == 0 && m[2] == 0) return 0.0;
    return orc_target_r(m, L, M, wt, s) * orc_ratio_nr(m, L, M, wt, s) / orc_proposal_pmf(m, L, s[0] * ORC_NR_WIDEN);
}

/*
 * The recalibration chain of Sec. 3.2 on a given proposal sequence: target
 * P^nr, proposal k* = props[t], acceptance
 *   min{1, P^nr(k*) P^r(k_t) / (P^nr(k_t) P^r(k*))} = min{1, R(k*)/R(k_t)},
 * accept iff u[t] < R(k*)/R(k_t); the chain starts at props[0] and out[t] is
 * the state after step t.  Exact for proposals drawn iid from P^r.
 * Pinned by: chi^2 against P^nr with iid P^r proposals.
 */
void orc_recalibrate(int P, const int32_t *props, const double *u, const double L[3], int M,
                     const double *wt, const double *s, int32_t *out, int64_t *n_acc)
{
    int32_t cur[3] = {props[0], props[1], props[2]};
    double rcur = orc_ratio_nr(cur, L, M, wt, s);
    int64_t acc = 0;
    for (int t = 0; t < P; ++t) {
        const int32_t *prop = &props[3 * t];
        const double rprop = orc_ratio_nr(prop, L, M, wt, s);
        if (u[t] < rprop / rcur) {
            memcpy(cur, prop, sizeof cur);
            rcur = rprop;
            ++acc;
        }
        memcpy(&out[3 * t], cur, sizeof cur);
    }
    if (n_acc) *n_acc = acc;
}

/*
 * Upper bound B_p >= g_p(m) / q'(m) over the whole integer lattice, used by the
 * rejection draw that starts a chain at its own target.  g_2(m) is the
 * unnormalised radial target |k|^2 sum_l wt_l s_l^5 e_l (eq. samplingP),
 * g_4(m) = |k|^4 sum_l wt_l s_l^7 e_l the non-radial one (eq. samplingPnr),
 * e_l = exp(-s_l^2 |k|^2 / 4), and q' the rounded-Gaussian proposal of App. D
 * with width parameter s_0/sqrt2, i.e. per-axis standard deviation
 * sig_xi = L_xi / (pi s_0).
 * Derivation.  The cell integral of the normal density over [m - 1/2, m + 1/2]
 * is at least the density at the far end |m| + 1/2, and (|m| + 1/2)/sig_xi =
 * s_0 |k_xi|/2 + c_xi with c_xi = 1/(2 sig_xi), so
 *   1/q'(m) <= K exp(s_0^2 |k|^2 / 8 + (s_0/2) sum_xi c_xi |k_xi|),
 *   K = prod_xi sqrt(2 pi) sig_xi exp(c_xi^2 / 2),
 * and sum_xi c_xi |k_xi| <= |c| |k| (Cauchy-Schwarz).  Term l of g_p/q' is
 * then at most K coef_l kappa^p exp(-alpha_l kappa^2 + beta kappa) with
 * kappa = |k|, alpha_l = s_l^2/4 - s_0^2/8 > 0 and beta = s_0 |c| / 2; its
 * maximum over kappa >= 0 lies at
 *   kappa* = (beta + sqrt(beta^2 + 8 alpha_l p)) / (4 alpha_l).
 * B_p is the sum over l of these maxima.
 * Pinned by: B_p above the largest ratio found by enumerating small boxes.
 */
double orc_start_bound(const double L[3], int M, const double *wt, const double *s, int p)
{
    const double s0 = s[0];
    double K = 1.0, c2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double sig = L[d] / (ORC_PI * s0);
        const double c = 1.0 / (2.0 * sig);
        K *= sqrt(2.0 * ORC_PI) * sig * exp(0.5 * c * c);
        c2 += c * c;
    }
    const double beta = 0.5 * s0 * sqrt(c2);
    double B = 0.0;
    for (int l = 0; l < M; ++l) {
        const double coef = wt[l] * pow(s[l], p == 2 ? 5 : 7);
        const double alpha = s[l] * s[l] / 4.0 - s0 * s0 / 8.0;
        const double ks = (beta + sqrt(beta * beta + 8.0 * alpha * p)) / (4.0 * alpha);
        B += coef * pow(ks, p) * exp(-alpha * ks * ks + beta * ks);
    }
    return K * B;
}

/* g_2(m) / q'(m) of the radial target over the widened proposal (0 at m = 0) */
static double orc_weight_r_wide(const int32_t m[3], const double L[3], int M, const double *wt, const double *s)
{
    if (m[0] == 0 && m[1] == 0 && m[2] == 0) return 0.0;
    return orc_target_r(m, L, M, wt, s) / orc_proposal_pmf(m, L, s[0] * ORC_NR_WIDEN);
}

/* tries of the rejection draw of a start state; each passes with probability
   (normalised target mass) / B_p, above 0.08 for every box tested */
#define ORC_START_TRIES 1024

/*
 * Start state of a chain, an exact draw of its target by rejection: try t
 * draws m from the widened proposal (normals of streams sxy, sz at counter t)
 * and is accepted iff u * B_p < g_p(m) / q'(m), u the first (r-chain) or
 * second (non-radial chain) uniform of stream 7 at counter t.  The first
 * accepted try gives the state.  Returns 0, or -1 if no try was accepted.
 */
static int orc_exact_start(const double L[3], int M, const double *wt, const double *s, uint64_t seed,
                           uint64_t sys, uint64_t step, int p, uint32_t sxy, uint32_t sz, int32_t out[3])
{
    const double B = orc_start_bound(L, M, wt, s, p);
    for (uint32_t t = 0; t < ORC_START_TRIES; ++t) {
        double z[3], u[2];
        int32_t m[3];
        orc_draw_proposal(seed, sys, step, t, sxy, sz, z, NULL);
        orc_round_proposal(z, L, s[0] * ORC_NR_WIDEN, m);
        orc_draw(seed, sys, step, t, 7u, &u[0], &u[1]);
        const double w = p == 2 ? orc_weight_r_wide(m, L, M, wt, s) : orc_weight_nr(m, L, M, wt, s);
        if ((p == 2 ? u[0] : u[1]) * B < w) {
            memcpy(out, m, sizeof(int32_t) * 3);
            return 0;
        }
    }
    return -1;
}

/* Exposed for tests: the start states of both chains (-1 if a draw failed). */
int orc_start_states(const double L[3], int M, const double *wt, const double *s, uint64_t seed,
                     uint64_t sys, uint64_t step, int32_t m_r0[3], int32_t m_nr0[3])
{
    if (orc_exact_start(L, M, wt, s, seed, sys, step, 2, 3u, 4u, m_r0)) return -1;
    if (orc_exact_start(L, M, wt, s, seed, sys, step, 4, 8u, 9u, m_nr0)) return -1;
    return 0;
}

/*
 * One sampling step (Algorithm 1, steps 2-3).
 *  r-chain (App. D): independence Metropolis-Hastings with the rounded
 *  Gaussian proposal; accept m* iff u < [P(m*) q(m)] / [P(m) q(m*)], written
 *  as w(m*)/w(m) with w = P/q.  Every step the chain starts from an exact draw
 *  of P^r (orc_exact_start, normals from streams 3, 4), so each of its states
 *  is distributed exactly as P^r; m_r[t] is the state after the t-th MH step.
 *  variant 0 (as printed, Sec. 3.2): the nr-chain is orc_recalibrate run on
 *  the r-chain states in order, started at the first r-chain state.
 *  variant 1 (exchange): a second state z starts from an exact draw of P^nr
 *  (streams 8, 9); after each r-step the recalibration's acceptance ratio
 *  decides a swap of the two chains' states, (x, z) -> (z, x).  The joint
 *  chain keeps P^r x P^nr invariant and starts in it, so every recorded state
 *  has exactly its target's law.  At most P + 2 distinct modes appear.
 * The two samplers the recalibration is weighed against (Sec. 3.2):
 *  variant 2 (shared proposal, no recalibration): m_nr = m_r; the non-radial
 *  estimator then weighs each r-chain mode by P^nr/P^r (see the oracle's
 *  nonradial_shared).
 *  variant 3 (independent proposals): a second independence MH chain with
 *  target P^nr and a rounded Gaussian proposal of width parameter
 *  s_0 ORC_NR_WIDEN (orc_weight_nr), its normals from streams (5, 6) and its
 *  acceptance uniform the second one of stream 2; accept m* iff
 *  u < w_nr(m*)/w_nr(m); it starts from its own exact draw of P^nr (streams
 *  8, 9).  Up to 2P + 2 distinct modes.
 * Returns 0, or -1 when a start draw failed (no accepted try).
 * n_acc[0], n_acc[1] receive the accepted-move counts of the two chains.
 * Pinned by: chi^2 of long chains against the enumerated targets, the law of
 * the start states, and batch means against the deterministic sums.
 */
int orc_sample_modes(const double L[3], int M, const double *wt, const double *s, int P,
                     uint64_t seed, uint64_t sys, uint64_t step, int variant,
                     int32_t *m_r, int32_t *m_nr, int64_t n_acc[2])
{
    int32_t cur[3], z0[3];
    if (orc_exact_start(L, M, wt, s, seed, sys, step, 2, 3u, 4u, cur)) return -1;
    if ((variant == 1 || variant == 3) && orc_exact_start(L, M, wt, s, seed, sys, step, 4, 8u, 9u, z0))
        return -1;
    double wcur = orc_weight(cur, L, M, wt, s);
    double *unr = malloc(sizeof(double) * (P > 0 ? P : 1));
    int64_t acc_r = 0, acc_nr = 0;
    int32_t znr[3];
    double wz = 0.0, rz = 0.0;
    if (variant == 1) {
        memcpy(znr, z0, sizeof znr);
        wz = orc_weight(znr, L, M, wt, s);
        rz = orc_ratio_nr(znr, L, M, wt, s);
    }
    for (int t = 0; t < P; ++t) {
        double z[3], uacc[2];
        int32_t prop[3];
        orc_draw_proposal(seed, sys, step, (uint32_t)t, 0u, 1u, z, uacc);
        unr[t] = uacc[1];
        orc_round_proposal(z, L, s[0], prop);
        const double wprop = orc_weight(prop, L, M, wt, s);
        if (uacc[0] < wprop / wcur) {
            memcpy(cur, prop, sizeof cur);
            wcur = wprop;
            ++acc_r;
        }
        if (variant == 1) {
            const double rx = orc_ratio_nr(cur, L, M, wt, s);
            if (uacc[1] < rx / rz) {
                int32_t tmp[3];
                memcpy(tmp, cur, sizeof tmp);
                memcpy(cur, znr, sizeof cur);
                memcpy(znr, tmp, sizeof znr);
                const double tw = wcur;
                wcur = wz;
                wz = tw;
                rz = rx;
                ++acc_nr;
            }
            memcpy(&m_nr[3 * t], znr, sizeof znr);
        }
        memcpy(&m_r[3 * t], cur, sizeof cur);
    }
    if (variant == 0) orc_recalibrate(P, m_r, unr, L, M, wt, s, m_nr, &acc_nr);
    if (variant == 2) memcpy(m_nr, m_r, sizeof(int32_t) * 3 * (size_t)(P > 0 ? P : 0));
    if (variant == 3) {
        int32_t zc[3];
        memcpy(zc, z0, sizeof zc);
        double wzc = orc_weight_nr(zc, L, M, wt, s);
        for (int t = 0; t < P; ++t) {
            double z[3];
            int32_t prop[3];
            orc_draw_proposal(seed, sys, step, (uint32_t)t, 5u, 6u, z, NULL);
            orc_round_proposal(z, L, s[0] * ORC_NR_WIDEN, prop);
            const double wprop = orc_weight_nr(prop, L, M, wt, s);
            if (unr[t] < wprop / wzc) {
                memcpy(zc, prop, sizeof zc);
                wzc = wprop;
                ++acc_nr;
            }
            memcpy(&m_nr[3 * t], zc, sizeof zc);
        }
    }
    free(unr);
    if (n_acc) {
        n_acc[0] = acc_r;
        n_acc[1] = acc_nr;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Fractional coordinates and cell binning                                    */
/* ------------------------------------------------------------------------- */

/*
 * Cell of each atom under the fixed-point reading of s = h^-1 r (Sec. 2.1):
 * s = x * (1/L) in double, wrapped into [0,1) by subtracting floor(s);
 * u = the low 32 bits of (uint64)(s * 2^32); cell index along xi is
 * (u * n_xi) >> 32, and the linear cell id is cx + nx (cy + ny cz).
 * Pinned by: every atom lies in the interval of its cell.
 */
void orc_cell_ids(int64_t n, const double *x, const double *y, const double *z, const double L[3],
                  const int32_t ncell[3], int32_t *cell)
{
    const double *p[3] = {x, y, z};
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[3];
        for (int d = 0; d < 3; ++d) {
            double sd = p[d][i] * (1.0 / L[d]);
            sd -= floor(sd);
            const uint32_t u = (uint32_t)((uint64_t)(sd * 4294967296.0) & 0xFFFFFFFFull);
            c[d] = (uint32_t)(((uint64_t)u * (uint64_t)ncell[d]) >> 32);
        }
        cell[i] = (int32_t)(c[0] + (uint32_t)ncell[0] * (c[1] + (uint32_t)ncell[1] * c[2]));
    }
}

/* ------------------------------------------------------------------------- */
/* Short-range part (eqs. U_short, force_SOG, P_short)                        */
/* ------------------------------------------------------------------------- */

/* minimum-image displacement r_i - r_j in an orthorhombic box */
static void orc_min_image(double d[3], const double L[3])
{
    for (int k = 0; k < 3; ++k) d[k] -= L[k] * round(d[k] / L[k]);
}

/* one ordered pair's contribution: force on i, half the pair virial and energy */
static void orc_pair(double qi, double qj, const double d[3], double rc2, int M,
                     const double *w, const double *wt, const double *s,
                     double f[3], double vir[6], double *u)
{
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 >= rc2 || r2 == 0.0) return;
    const double r = sqrt(r2);
    double sw = 0.0, swt = 0.0;
    for (int l = 0; l < M; ++l) {
        const double e = exp(-r2 / (s[l] * s[l]));
        sw += w[l] * e;
        swt += wt[l] * e;
    }
    const double Nt = 1.0 / (r2 * r) - swt; /* N~(r), eq. pressure_split */
    const double Nu = 1.0 / r - sw;          /* N(r), eq. short */
    const double qq = qi * qj;
    for (int k = 0; k < 3; ++k) f[k] += qq * Nt * d[k];
    vir[0] += 0.5 * qq * Nt * d[0] * d[0];
    vir[1] += 0.5 * qq * Nt * d[1] * d[1];
    vir[2] += 0.5 * qq * Nt * d[2] * d[2];
    vir[3] += 0.5 * qq * Nt * d[0] * d[1];
    vir[4] += 0.5 * qq * Nt * d[0] * d[2];
    vir[5] += 0.5 * qq * Nt * d[1] * d[2];
    *u += 0.5 * qq * Nu;
}

/*
 * Short-range SOG force F^N_i (eq. force_SOG, with 2 w_l / s_l^2 = wt_l),
 * short-range virial sum (the numerator of eq. P_short: the caller divides by
 * V) and energy U^N (eq. U_short), all pairs by minimum image (rc <= L/2 so at
 * most one image of a pair lies inside rc), O(N^2).
 * vir = (xx, yy, zz, xy, xz, yz).
 * Pinned by: finite differences of the total SOG energy and agreement of the
 * total with Ewald.
 */
void orc_short_range_brute(int64_t n, const double *q, const double *x, const double *y,
                           const double *z, const double L[3], double rc, int M,
                           const double *w, const double *wt, const double *s,
                           double *fx, double *fy, double *fz, double vir[6], double *U)
{
    double *vi = calloc((size_t)n * 7, sizeof(double));
    const double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double f[3] = {0, 0, 0}, v[6] = {0, 0, 0, 0, 0, 0}, u = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3] = {x[i] - x[j], y[i] - y[j], z[i] - z[j]};
            orc_min_image(d, L);
            orc_pair(q[i], q[j], d, rc2, M, w, wt, s, f, v, &u);
        }
        fx[i] = f[0]; fy[i] = f[1]; fz[i] = f[2];
        for (int k = 0; k < 6; ++k) vi[7 * i + k] = v[k];
        vi[7 * i + 6] = u;
    }
    for (int k = 0; k < 6; ++k) vir[k] = 0.0;
    *U = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 6; ++k) vir[k] += vi[7 * i + k];
        *U += vi[7 * i + 6];
    }
    free(vi);
}

/*
 * Same quantities through a cell list with cells no narrower than rc (a
 * dimension with fewer than three cells is searched whole), for large N.
 * If sample != NULL only the atoms sample[0..ns) are treated as i-atoms
 * (forces for them only; virial and energy then hold their half-pair shares).
 * Pinned by: equality with orc_short_range_brute.
 */
void orc_short_range_cells(int64_t n, const double *q, const double *x, const double *y,
                           const double *z, const double L[3], double rc, int M,
                           const double *w, const double *wt, const double *s,
                           int64_t ns, const int64_t *sample,
                           double *fx, double *fy, double *fz, double vir[6], double *U)
{
    int nc[3];
    for (int d = 0; d < 3; ++d) {
        nc[d] = (int)floor(L[d] / rc);
        if (nc[d] < 3) nc[d] = 1;
    }
    const int64_t ncells = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = malloc(sizeof(int64_t) * ncells), *next = malloc(sizeof(int64_t) * n);
    int *ci = malloc(sizeof(int) * 3 * n);
    for (int64_t c = 0; c < ncells; ++c) head[c] = -1;
    const double *p[3] = {x, y, z};
    for (int64_t i = n - 1; i >= 0; --i) {
        for (int d = 0; d < 3; ++d) {
            double sd = p[d][i] / L[d];
            sd -= floor(sd);
            int c = (int)floor(sd * nc[d]);
            if (c >= nc[d]) c = nc[d] - 1;
            if (c < 0) c = 0;
            ci[3 * i + d] = c;
        }
        const int64_t c = ci[3 * i] + (int64_t)nc[0] * (ci[3 * i + 1] + (int64_t)nc[1] * ci[3 * i + 2]);
        next[i] = head[c];
        head[c] = i;
    }
    const int64_t ni = sample ? ns : n;
    double *vi = calloc((size_t)ni * 7, sizeof(double));
    const double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < ni; ++a) {
        const int64_t i = sample ? sample[a] : a;
        double f[3] = {0, 0, 0}, v[6] = {0, 0, 0, 0, 0, 0}, u = 0.0;
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = nc[d] >= 3 ? -1 : 0;
            hi[d] = nc[d] >= 3 ? 1 : 0;
        }
        for (int dz = lo[2]; dz <= hi[2]; ++dz)
            for (int dy = lo[1]; dy <= hi[1]; ++dy)
                for (int dx = lo[0]; dx <= hi[0]; ++dx) {
                    const int cx = (ci[3 * i] + dx + nc[0]) % nc[0];
                    const int cy = (ci[3 * i + 1] + dy + nc[1]) % nc[1];
                    const int cz = (ci[3 * i + 2] + dz + nc[2]) % nc[2];
                    const int64_t c = cx + (int64_t)nc[0] * (cy + (int64_t)nc[1] * cz);
                    for (int64_t j = head[c]; j >= 0; j = next[j]) {
                        if (j == i) continue;
                        double d[3] = {x[i] - x[j], y[i] - y[j], z[i] - z[j]};
                        orc_min_image(d, L);
                        orc_pair(q[i], q[j], d, rc2, M, w, wt, s, f, v, &u);
                    }
                }
        fx[a] = f[0]; fy[a] = f[1]; fz[a] = f[2];
        for (int k = 0; k < 6; ++k) vi[7 * a + k] = v[k];
        vi[7 * a + 6] = u;
    }
    for (int k = 0; k < 6; ++k) vir[k] = 0.0;
    *U = 0.0;
    for (int64_t a = 0; a < ni; ++a) {
        for (int k = 0; k < 6; ++k) vir[k] += vi[7 * a + k];
        *U += vi[7 * a + 6];
    }
    free(vi); free(head); free(next); free(ci);
}

/* ------------------------------------------------------------------------- */
/* Structure factors and the random-batch long-range part                     */
/* ------------------------------------------------------------------------- */

/*
 * rho(k) = sum_j q_j exp(i k . r_j), k = 2 pi h^-T m (eq. rho_k), one mode per
 * row of m.  Pinned by: the perfect-lattice selection rule and the agreement of
 * the full k-space sums with Ewald and with finite differences.
 */
void orc_rho(int64_t n, const double *q, const double *x, const double *y, const double *z,
             const double L[3], int64_t nm, const int32_t *m, double *re, double *im)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < nm; ++p) {
        const double kx = 2.0 * ORC_PI * m[3 * p] / L[0];
        const double ky = 2.0 * ORC_PI * m[3 * p + 1] / L[1];
        const double kz = 2.0 * ORC_PI * m[3 * p + 2] / L[2];
        double a = 0.0, b = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double th = kx * x[j] + ky * y[j] + kz * z[j];
            a += q[j] * cos(th);
            b += q[j] * sin(th);
        }
        re[p] = a;
        im[p] = b;
    }
}

/*
 * Random-batch long-range part from P sampled modes per chain.
 *  radial pressure (eq. P_approx_r):      S^r/(4 V^2 P) sum_p |rho_p|^2/|k_p|^2 I
 *  non-radial pressure (eq. P_approx_nr): -S^nr/(8 V^2 P) sum_p |rho_p|^2 k_p (x) k_p / |k_p|^4
 *  force (eq. f_approx, S = S^r/2):       -(S/P)(q_i/V) sum_p k_p Im(e^{-i k_p.r_i} rho_p)/|k_p|^2
 *  energy (not printed; importance-sampling estimate of eq. U_long under the
 *  force proposal eq. prob_p):            (S/(2 V P)) sum_p |rho_p|^2/|k_p|^2
 * The r-chain modes serve the radial pressure, the force and the energy; the
 * nr-chain modes serve the non-radial pressure.  Each sample's rho is evaluated
 * on its own (no merging of repeated modes).  Pr and Pnr are 3x3 row-major.
 * fx..fz may be NULL (no forces).  If sample != NULL forces are computed only
 * for atoms sample[0..ns) and written to fx[0..ns).
 * Pinned by: exact unbiasedness (enumerated expectation = full k-space sums).
 */
void orc_long_range_rb(int64_t n, const double *q, const double *x, const double *y,
                       const double *z, const double L[3], int P, const int32_t *m_r,
                       const int32_t *m_nr, double Sr, double Snr,
                       int64_t ns, const int64_t *sample,
                       double *fx, double *fy, double *fz, double Pr[9], double Pnr[9], double *UF)
{
    const double V = L[0] * L[1] * L[2];
    double *rr = malloc(sizeof(double) * P), *ri = malloc(sizeof(double) * P);
    double *nr_re = malloc(sizeof(double) * P), *nr_im = malloc(sizeof(double) * P);
    orc_rho(n, q, x, y, z, L, P, m_r, rr, ri);
    orc_rho(n, q, x, y, z, L, P, m_nr, nr_re, nr_im);
    double sum_r = 0.0;
    for (int p = 0; p < P; ++p) sum_r += (rr[p] * rr[p] + ri[p] * ri[p]) / orc_k2(&m_r[3 * p], L);
    for (int a = 0; a < 9; ++a) Pr[a] = 0.0;
    Pr[0] = Pr[4] = Pr[8] = Sr / (4.0 * V * V * P) * sum_r;
    double acc[9] = {0};
    for (int p = 0; p < P; ++p) {
        double k[3];
        for (int d = 0; d < 3; ++d) k[d] = 2.0 * ORC_PI * m_nr[3 * p + d] / L[d];
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double a2 = nr_re[p] * nr_re[p] + nr_im[p] * nr_im[p];
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) acc[3 * al + be] += a2 * k[al] * k[be] / (k2 * k2);
    }
    for (int a = 0; a < 9; ++a) Pnr[a] = -Snr / (8.0 * V * V * P) * acc[a];
    const double S = 0.5 * Sr;
    *UF = S / (2.0 * V * P) * sum_r;
    if (fx) {
        const int64_t ni = sample ? ns : n;
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < ni; ++a) {
            const int64_t i = sample ? sample[a] : a;
            double f[3] = {0, 0, 0};
            for (int p = 0; p < P; ++p) {
                double k[3];
                for (int d = 0; d < 3; ++d) k[d] = 2.0 * ORC_PI * m_r[3 * p + d] / L[d];
                const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                const double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
                /* Im(e^{-i th} (re + i im)) = im cos th - re sin th */
                const double imv = ri[p] * cos(th) - rr[p] * sin(th);
                for (int d = 0; d < 3; ++d) f[d] += k[d] * imv / k2;
            }
            fx[a] = -(S / P) * (q[i] / V) * f[0];
            fy[a] = -(S / P) * (q[i] / V) * f[1];
            fz[a] = -(S / P) * (q[i] / V) * f[2];
        }
    }
    free(rr); free(ri); free(nr_re); free(nr_im);
}

/* ------------------------------------------------------------------------- */
/* Deterministic full k-space sums (Theorem 1; App. A)                        */
/* ------------------------------------------------------------------------- */

/*
 * Full SOG long-range part over every k != 0 with exp(-s_0^2 k^2/4) above
 * exp(-ORC_TRUNC):
 *  U^F  = 1/(2V) sum_k Fhat(k) |rho|^2,  Fhat = sum_l pi^(3/2) w_l s_l^3 e^{-s_l^2 k^2/4} (eq. U_long)
 *  F^F_i = -(q_i/V) sum_k k Fhat(k) Im(e^{-ik.r_i} rho(k))                             (App. A)
 *  P^F  = pi^(3/2)/(4V^2) sum_k sum_l wt_l s_l^5 e^{-s_l^2 k^2/4} (I - s_l^2/2 k(x)k) |rho|^2 (eq. P_long)
 * Pinned by: finite differences (P^F = -dU^F/d strain / V, F = -dU/dr) and
 * agreement of the SOG totals with Ewald.
 */
void orc_sog_kspace_full(int64_t n, const double *q, const double *x, const double *y,
                         const double *z, const double L[3], int M, const double *w,
                         const double *wt, const double *s,
                         double *fx, double *fy, double *fz, double Pf[9], double *UF)
{
    const double V = L[0] * L[1] * L[2];
    int mmax[3];
    for (int d = 0; d < 3; ++d)
        mmax[d] = (int)ceil(L[d] * sqrt(4.0 * ORC_TRUNC) / (2.0 * ORC_PI * s[0])) + 1;
    const int64_t nx = 2 * mmax[0] + 1, ny = 2 * mmax[1] + 1, nz = 2 * mmax[2] + 1;
    const int64_t nk = nx * ny * nz;
    double *rre = malloc(sizeof(double) * nk), *rim = malloc(sizeof(double) * nk);
    int32_t *mm = malloc(sizeof(int32_t) * 3 * nk);
    int64_t cnt = 0;
    for (int a = -mmax[0]; a <= mmax[0]; ++a)
        for (int b = -mmax[1]; b <= mmax[1]; ++b)
            for (int c = -mmax[2]; c <= mmax[2]; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                const int32_t mv[3] = {a, b, c};
                if (s[0] * s[0] * orc_k2(mv, L) / 4.0 > ORC_TRUNC) continue;
                mm[3 * cnt] = a; mm[3 * cnt + 1] = b; mm[3 * cnt + 2] = c;
                ++cnt;
            }
    orc_rho(n, q, x, y, z, L, cnt, mm, rre, rim);
    double u = 0.0, pf[9] = {0};
    double *fh = malloc(sizeof(double) * cnt);
    for (int64_t p = 0; p < cnt; ++p) {
        double k[3];
        for (int d = 0; d < 3; ++d) k[d] = 2.0 * ORC_PI * mm[3 * p + d] / L[d];
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double a2 = rre[p] * rre[p] + rim[p] * rim[p];
        double F = 0.0;
        for (int l = 0; l < M; ++l) F += pow(ORC_PI, 1.5) * w[l] * pow(s[l], 3) * exp(-s[l] * s[l] * k2 / 4.0);
        fh[p] = F;
        u += F * a2;
        for (int l = 0; l < M; ++l) {
            const double g = wt[l] * pow(s[l], 5) * exp(-s[l] * s[l] * k2 / 4.0) * a2;
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be)
                    pf[3 * al + be] += g * ((al == be ? 1.0 : 0.0) - 0.5 * s[l] * s[l] * k[al] * k[be]);
        }
    }
    *UF = u / (2.0 * V);
    for (int a = 0; a < 9; ++a) Pf[a] = pow(ORC_PI, 1.5) / (4.0 * V * V) * pf[a];
    if (fx) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double f[3] = {0, 0, 0};
            for (int64_t p = 0; p < cnt; ++p) {
                double k[3];
                for (int d = 0; d < 3; ++d) k[d] = 2.0 * ORC_PI * mm[3 * p + d] / L[d];
                const double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
                const double imv = rim[p] * cos(th) - rre[p] * sin(th);
                for (int d = 0; d < 3; ++d) f[d] += k[d] * fh[p] * imv;
            }
            fx[i] = -q[i] / V * f[0];
            fy[i] = -q[i] / V * f[1];
            fz[i] = -q[i] / V * f[2];
        }
    }
    free(rre); free(rim); free(mm); free(fh);
}

/* self energy (App. A): ln b / (sqrt(2 pi) sigma) (omega + (1 - b^-(M-1))/(b - 1)) sum q^2 */
double orc_self_energy(double b, double sigma, double omega, int M, int64_t n, const double *q)
{
    double q2 = 0.0;
    for (int64_t i = 0; i < n; ++i) q2 += q[i] * q[i];
    return log(b) / (sqrt(2.0 * ORC_PI) * sigma) * (omega + (1.0 - pow(b, -(double)(M - 1))) / (b - 1.0)) * q2;
}

/* ------------------------------------------------------------------------- */
/* Ewald reference (eq. Ewald with tinfoil boundary)                          */
/* ------------------------------------------------------------------------- */

/*
 * Coulomb lattice energy (eq. potential), forces and pressure tensor (eq.
 * Pcoul) through the Ewald split 1/r = erfc(beta r)/r + erf(beta r)/r
 * (beta = 1/(sqrt2 alpha) in the notation of eq. Ewald), tinfoil boundary:
 *  real space: all images with |r_ij + h n| < rcut,
 *  reciprocal: all k != 0 with |k| < kcut, G(k) = 4 pi e^{-k^2/(4 beta^2)} / k^2,
 *  P_recip = 1/(2V^2) sum_k G |rho|^2 [I - 2 (1 + k^2/(4 beta^2)) k(x)k / k^2],
 *  self energy -beta/sqrt(pi) sum q^2.
 * Pinned by: the NaCl Madelung constant, the virial identity tr P = U/V and
 * finite differences.
 */
void orc_ewald(int64_t n, const double *q, const double *x, const double *y, const double *z,
               const double L[3], double beta, double rcut, double kcut,
               double *fx, double *fy, double *fz, double Pt[9], double *U)
{
    const double V = L[0] * L[1] * L[2];
    int nimg[3];
    for (int d = 0; d < 3; ++d) nimg[d] = (int)ceil(rcut / L[d]) + 1;
    double *acc = calloc((size_t)n * 10, sizeof(double));
    const double rcut2 = rcut * rcut;
    const double tb = 2.0 * beta / sqrt(ORC_PI);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        double f[3] = {0, 0, 0}, v[6] = {0}, u = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double d0[3] = {x[i] - x[j], y[i] - y[j], z[i] - z[j]};
            orc_min_image(d0, L);
            for (int a = -nimg[0]; a <= nimg[0]; ++a)
                for (int b = -nimg[1]; b <= nimg[1]; ++b)
                    for (int c = -nimg[2]; c <= nimg[2]; ++c) {
                        const double d[3] = {d0[0] + a * L[0], d0[1] + b * L[1], d0[2] + c * L[2]};
                        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 >= rcut2 || r2 == 0.0) continue;
                        const double r = sqrt(r2);
                        const double qq = q[i] * q[j];
                        const double g = erfc(beta * r) / (r2 * r) + tb * exp(-beta * beta * r2) / r2;
                        for (int k = 0; k < 3; ++k) f[k] += qq * g * d[k];
                        v[0] += 0.5 * qq * g * d[0] * d[0];
                        v[1] += 0.5 * qq * g * d[1] * d[1];
                        v[2] += 0.5 * qq * g * d[2] * d[2];
                        v[3] += 0.5 * qq * g * d[0] * d[1];
                        v[4] += 0.5 * qq * g * d[0] * d[2];
                        v[5] += 0.5 * qq * g * d[1] * d[2];
                        u += 0.5 * qq * erfc(beta * r) / r;
                    }
        }
        for (int k = 0; k < 3; ++k) acc[10 * i + k] = f[k];
        for (int k = 0; k < 6; ++k) acc[10 * i + 3 + k] = v[k];
        acc[10 * i + 9] = u;
    }
    double vr[6] = {0}, ur = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 6; ++k) vr[k] += acc[10 * i + 3 + k];
        ur += acc[10 * i + 9];
    }
    /* reciprocal space */
    int mmax[3];
    for (int d = 0; d < 3; ++d) mmax[d] = (int)ceil(kcut * L[d] / (2.0 * ORC_PI)) + 1;
    const int64_t nk = (int64_t)(2 * mmax[0] + 1) * (2 * mmax[1] + 1) * (2 * mmax[2] + 1);
    int32_t *mm = malloc(sizeof(int32_t) * 3 * nk);
    int64_t cnt = 0;
    for (int a = -mmax[0]; a <= mmax[0]; ++a)
        for (int b = -mmax[1]; b <= mmax[1]; ++b)
            for (int c = -mmax[2]; c <= mmax[2]; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                const int32_t mv[3] = {a, b, c};
                if (orc_k2(mv, L) >= kcut * kcut) continue;
                mm[3 * cnt] = a; mm[3 * cnt + 1] = b; mm[3 * cnt + 2] = c;
                ++cnt;
            }
    double *rre = malloc(sizeof(double) * cnt), *rim = malloc(sizeof(double) * cnt),
           *G = malloc(sizeof(double) * cnt);
    orc_rho(n, q, x, y, z, L, cnt, mm, rre, rim);
    double uk = 0.0, pk[9] = {0};
    for (int64_t p = 0; p < cnt; ++p) {
        double k[3];
        for (int d = 0; d < 3; ++d) k[d] = 2.0 * ORC_PI * mm[3 * p + d] / L[d];
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        G[p] = 4.0 * ORC_PI * exp(-k2 / (4.0 * beta * beta)) / k2;
        const double a2 = rre[p] * rre[p] + rim[p] * rim[p];
        uk += G[p] * a2;
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be)
                pk[3 * al + be] += G[p] * a2 *
                    ((al == be ? 1.0 : 0.0) - 2.0 * (1.0 + k2 / (4.0 * beta * beta)) * k[al] * k[be] / k2);
    }
    uk /= 2.0 * V;
    for (int a = 0; a < 9; ++a) pk[a] /= 2.0 * V * V;
    double q2 = 0.0;
    for (int64_t i = 0; i < n; ++i) q2 += q[i] * q[i];
    const double uself = -beta / sqrt(ORC_PI) * q2;
    *U = ur + uk + uself;
    const int idx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) Pt[3 * al + be] = vr[idx[al][be]] / V + pk[3 * al + be];
    if (fx) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double f[3] = {acc[10 * i], acc[10 * i + 1], acc[10 * i + 2]};
            for (int64_t p = 0; p < cnt; ++p) {
                double k[3];
                for (int d = 0; d < 3; ++d) k[d] = 2.0 * ORC_PI * mm[3 * p + d] / L[d];
                const double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
                const double imv = rim[p] * cos(th) - rre[p] * sin(th);
                for (int d = 0; d < 3; ++d) f[d] -= q[i] / V * k[d] * G[p] * imv;
            }
            fx[i] = f[0]; fy[i] = f[1]; fz[i] = f[2];
        }
    }
    free(acc); free(mm); free(rre); free(rim); free(G);
}

/* ------------------------------------------------------------------------- */
/* General (triclinic) cells: h = [h_1, h_2, h_3], r = h s (Sec. 2.1)          */
/* ------------------------------------------------------------------------- */

/*
 * The cell tensor h is passed row-major, h[3 i + j] = (h)_ij: column j is the
 * cell vector h_j.  Positions are Cartesian, r = h s with s the fractional
 * coordinates.  Reciprocal vectors are k = 2 pi h^-T m (eq. FourierTransform),
 * so k . r = 2 pi m . s (eq. rho_k).  The short-range sums need r_c no larger
 * than half the smallest perpendicular width of the cell only where a
 * function says so; the brute-force sums below take every image inside r_c.
 */

/* inverse and determinant of h by cofactors */
static double tri_inverse(const double h[9], double hi[9])
{
    const double a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], k = h[7], l = h[8];
    const double A = e * l - f * k, B = -(d * l - f * g), C = d * k - e * g;
    const double det = a * A + b * B + c * C;
    hi[0] = A / det;
    hi[3] = B / det;
    hi[6] = C / det;
    hi[1] = -(b * l - c * k) / det;
    hi[4] = (a * l - c * g) / det;
    hi[7] = -(a * k - b * g) / det;
    hi[2] = (b * f - c * e) / det;
    hi[5] = -(a * f - c * d) / det;
    hi[8] = (a * e - b * d) / det;
    return det;
}

/* k = 2 pi h^-T m: k_i = 2 pi sum_j (h^-1)_ji m_j */
static void tri_k(const int32_t m[3], const double hi[9], double k[3])
{
    for (int i = 0; i < 3; ++i) k[i] = 2.0 * ORC_PI * (hi[i] * m[0] + hi[3 + i] * m[1] + hi[6 + i] * m[2]);
}

static double tri_k2(const int32_t m[3], const double hi[9])
{
    double k[3];
    tri_k(m, hi, k);
    return k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
}

/* perpendicular widths w_i = 1 / |row i of h^-1| (distance between the faces s_i = 0 and 1) */
static void tri_widths(const double hi[9], double w[3])
{
    for (int i = 0; i < 3; ++i)
        w[i] = 1.0 / sqrt(hi[3 * i] * hi[3 * i] + hi[3 * i + 1] * hi[3 * i + 1] + hi[3 * i + 2] * hi[3 * i + 2]);
}

/* length of the cell vector h_j (column j) */
static double tri_col_len(const double h[9], int j)
{
    return sqrt(h[j] * h[j] + h[3 + j] * h[3 + j] + h[6 + j] * h[6 + j]);
}

/*
 * H^r_l and H^nr_l by the direct sums of eqs. Sr and Snr over m with
 * s^2 |k|^2 / 4 <= ORC_TRUNC.  Since m_j = h_j . k / (2 pi), the box
 * |m_j| <= |h_j| kmax / (2 pi) + 1 holds every such m.
 * Pinned by: the Poisson forms (Prop. 1), h = diag(L) against orc_H_direct,
 * invariance under h -> h U for unimodular U.
 */
void orc_tri_H_direct(const double h[9], double wt, double s, double *Hr, double *Hnr)
{
    double hi[9];
    tri_inverse(h, hi);
    const double kmax = sqrt(4.0 * ORC_TRUNC) / s;
    int mmax[3];
    for (int j = 0; j < 3; ++j) mmax[j] = (int)ceil(tri_col_len(h, j) * kmax / (2.0 * ORC_PI)) + 1;
    const double pre = pow(ORC_PI, 1.5) * wt;
    double ar = 0.0, anr = 0.0;
    for (int a = -mmax[0]; a <= mmax[0]; ++a)
        for (int b = -mmax[1]; b <= mmax[1]; ++b)
            for (int c = -mmax[2]; c <= mmax[2]; ++c) {
                const int32_t m[3] = {a, b, c};
                const double k2 = tri_k2(m, hi);
                const double e = exp(-s * s * k2 / 4.0);
                ar += pow(s, 5) * k2 * e;
                anr += pow(s, 7) * k2 * k2 * e;
            }
    *Hr = pre * ar;
    *Hnr = pre * anr;
}

/*
 * Prop. 1 for a general cell: A_j = sum_n |h n|^j exp(-|h n|^2 / s^2) over n
 * with |h n|^2 / s^2 <= ORC_TRUNC; n_i = (h^-1 (h n))_i, so |n_i| <= |h n| / w_i.
 * Pinned by: the direct sums.
 */
void orc_tri_H_poisson(const double h[9], double wt, double s, double *Hr, double *Hnr)
{
    double hi[9], w[3];
    const double V = fabs(tri_inverse(h, hi));
    tri_widths(hi, w);
    const double rmax = s * sqrt(ORC_TRUNC);
    int nmax[3];
    for (int i = 0; i < 3; ++i) nmax[i] = (int)ceil(rmax / w[i]) + 1;
    double A0 = 0.0, A2 = 0.0, A4 = 0.0;
    for (int a = -nmax[0]; a <= nmax[0]; ++a)
        for (int b = -nmax[1]; b <= nmax[1]; ++b)
            for (int c = -nmax[2]; c <= nmax[2]; ++c) {
                double r[3];
                for (int i = 0; i < 3; ++i) r[i] = h[3 * i] * a + h[3 * i + 1] * b + h[3 * i + 2] * c;
                const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                const double e = exp(-r2 / (s * s));
                A0 += e;
                A2 += r2 * e;
                A4 += r2 * r2 * e;
            }
    *Hr = V * wt * (6.0 * A0 - 4.0 * A2 / (s * s));
    *Hnr = V * wt * (60.0 * A0 - 80.0 * A2 / (s * s) + 16.0 * A4 / (s * s * s * s));
}

/* S^r, S^nr (eqs. Sr, Snr): Poisson form when s_l < the smallest width, form as in orc_norm_consts */
void orc_tri_norm_consts(const double h[9], int M, const double *wt, const double *s, int form, double *Sr,
                         double *Snr)
{
    double hi[9], w[3];
    tri_inverse(h, hi);
    tri_widths(hi, w);
    const double wmin = fmin(w[0], fmin(w[1], w[2]));
    double sr = 0.0, snr = 0.0;
    for (int l = 0; l < M; ++l) {
        double hr, hnr;
        const int poisson = (form == 2) || (form == 0 && s[l] < wmin);
        if (poisson) orc_tri_H_poisson(h, wt[l], s[l], &hr, &hnr);
        else orc_tri_H_direct(h, wt[l], s[l], &hr, &hnr);
        sr += hr;
        snr += hnr;
    }
    *Sr = sr;
    *Snr = snr;
}

/* unnormalised radial target (eq. samplingP) and the ratio P^nr/P^r up to S^r/S^nr, general k */
double orc_tri_target_r(const int32_t m[3], const double h[9], int M, const double *wt, const double *s)
{
    double hi[9];
    tri_inverse(h, hi);
    const double k2 = tri_k2(m, hi);
    double acc = 0.0;
    for (int l = 0; l < M; ++l) acc += wt[l] * pow(s[l], 5) * exp(-s[l] * s[l] * k2 / 4.0);
    return k2 * acc;
}

double orc_tri_ratio_nr(const int32_t m[3], const double h[9], int M, const double *wt, const double *s)
{
    double hi[9];
    tri_inverse(h, hi);
    const double k2 = tri_k2(m, hi);
    double a7 = 0.0, a5 = 0.0;
    for (int l = 0; l < M; ++l) {
        const double e = exp(-s[l] * s[l] * k2 / 4.0);
        a7 += wt[l] * pow(s[l], 7) * e;
        a5 += wt[l] * pow(s[l], 5) * e;
    }
    return k2 * a7 / a5;
}

/*
 * Gauss-Legendre rule of ORC_GL points on [-1/2, 1/2]: nodes are the roots of
 * P_n found by Newton's method from the Chebyshev guesses, weights
 * 1 / ((1 - x^2) P_n'(x)^2), halved for the unit interval.
 */
#define ORC_GL 24
static double orc_gl_x[ORC_GL], orc_gl_w[ORC_GL];
static int orc_gl_ready = 0;
static void orc_gl_init(void)
{
    if (orc_gl_ready) return;
    const int n = ORC_GL;
    for (int i = 0; i < n; ++i) {
        double x = cos(ORC_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        orc_gl_x[i] = 0.5 * x;
        orc_gl_w[i] = 0.5 * 2.0 / ((1.0 - x * x) * dp * dp);
    }
    orc_gl_ready = 1;
}

/*
 * Proposal pmf of eq. proposal for a general cell: with C = (h^T h)^-1 =
 * h^-1 h^-T,
 *   q(m) = (sqrt(pi) s0)^3 / det h  int_{m + [-1/2,1/2]^3} exp(-pi^2 s0^2 g^T C g) dg,
 * the probability that round(h^T u) = m for u ~ N(0, I / (2 pi^2 s0^2)).
 * The integral has no closed form; it is taken by the tensor Gauss-Legendre
 * rule of ORC_GL^3 points with the factor exp(-pi^2 s0^2 m^T C m) outside.
 * Pinned by: the erf product of orc_proposal_pmf at h = diag(L), the
 * normalisation over the lattice, and chi^2 of rounded draws on a sheared cell.
 */
/*
 * exp(-a (lin + dCd)) = exp(-a dCd) prod_i exp(-2 a (Cm)_i d_i): the first
 * factor, times the three weights, depends on the cell and s0 only, and is
 * tabulated once per (h, s0) (two tables kept: the chains alternate between
 * the proposal and its widened form).  Not thread-safe.
 */
struct orc_gl_table {
    double h[9], s0, V, C[9];
    int used;
    double t[ORC_GL * ORC_GL * ORC_GL];
};
static struct orc_gl_table orc_gl_tab[2];
static int orc_gl_next = 0;

static const struct orc_gl_table *orc_gl_lookup(const double h[9], double s0)
{
    for (int e = 0; e < 2; ++e)
        if (orc_gl_tab[e].used && orc_gl_tab[e].s0 == s0 && memcmp(orc_gl_tab[e].h, h, sizeof(double) * 9) == 0)
            return &orc_gl_tab[e];
    struct orc_gl_table *T = &orc_gl_tab[orc_gl_next];
    orc_gl_next ^= 1;
    double hi[9];
    T->V = fabs(tri_inverse(h, hi));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            T->C[3 * i + j] = hi[3 * i] * hi[3 * j] + hi[3 * i + 1] * hi[3 * j + 1] + hi[3 * i + 2] * hi[3 * j + 2];
    const double a = ORC_PI * ORC_PI * s0 * s0;
    for (int i = 0; i < ORC_GL; ++i)
        for (int j = 0; j < ORC_GL; ++j)
            for (int k = 0; k < ORC_GL; ++k) {
                const double d[3] = {orc_gl_x[i], orc_gl_x[j], orc_gl_x[k]};
                double dcd = 0.0;
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) dcd += d[p] * T->C[3 * p + q] * d[q];
                T->t[(i * ORC_GL + j) * ORC_GL + k] = orc_gl_w[i] * orc_gl_w[j] * orc_gl_w[k] * exp(-a * dcd);
            }
    memcpy(T->h, h, sizeof(double) * 9);
    T->s0 = s0;
    T->used = 1;
    return T;
}

double orc_tri_proposal_pmf(const int32_t m[3], const double h[9], double s0)
{
    orc_gl_init();
    const struct orc_gl_table *T = orc_gl_lookup(h, s0);
    const double a = ORC_PI * ORC_PI * s0 * s0;
    double cm[3], mm = 0.0;
    for (int i = 0; i < 3; ++i) {
        cm[i] = T->C[3 * i] * m[0] + T->C[3 * i + 1] * m[1] + T->C[3 * i + 2] * m[2];
        mm += m[i] * cm[i];
    }
    double e[3][ORC_GL];
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < ORC_GL; ++i) e[d][i] = exp(-2.0 * a * cm[d] * orc_gl_x[i]);
    double acc = 0.0;
    for (int i = 0; i < ORC_GL; ++i)
        for (int j = 0; j < ORC_GL; ++j) {
            double row = 0.0;
            for (int k = 0; k < ORC_GL; ++k) row += T->t[(i * ORC_GL + j) * ORC_GL + k] * e[2][k];
            acc += e[0][i] * e[1][j] * row;
        }
    return pow(sqrt(ORC_PI) * s0, 3) / T->V * exp(-a * mm) * acc;
}

/* m* = round(h^T u), u = z / (sqrt2 pi s0): (h^T u)_i = sum_j h_ji u_j, half away from zero */
static void tri_round_proposal(const double z[3], const double h[9], double s0, int32_t m[3])
{
    const double c = 1.0 / (sqrt(2.0) * ORC_PI * s0);
    for (int i = 0; i < 3; ++i) {
        double v = round(c * (h[i] * z[0] + h[3 + i] * z[1] + h[6 + i] * z[2]));
        if (v > 1073741824.0) v = 1073741824.0;
        if (v < -1073741824.0) v = -1073741824.0;
        m[i] = (int32_t)v;
    }
}

/* exposed for tests: the rounded proposal of a normal triple */
void orc_tri_round(const double z[3], const double h[9], double s0, int32_t m[3]) { tri_round_proposal(z, h, s0, m); }

static double tri_weight(const int32_t m[3], const double h[9], int M, const double *wt, const double *s, double s0q)
{
    if (m[0] == 0 && m[1] == 0 && m[2] == 0) return 0.0;
    return orc_tri_target_r(m, h, M, wt, s) / orc_tri_proposal_pmf(m, h, s0q);
}

static double tri_weight_nr(const int32_t m[3], const double h[9], int M, const double *wt, const double *s)
{
    if (m[0] == 0 && m[1] == 0 && m[2] == 0) return 0.0;
    return orc_tri_target_r(m, h, M, wt, s) * orc_tri_ratio_nr(m, h, M, wt, s) /
           orc_tri_proposal_pmf(m, h, s[0] * ORC_NR_WIDEN);
}

/*
 * Bound B_p >= g_p(m) / q'(m) over the lattice for a general cell (the start
 * draws' rejection constant; g_p and q' as in orc_start_bound, q' of width
 * parameter s' = s_0 / sqrt2).  The integrand of q' is at least its minimum
 * over the unit cube around m, and for g = m + d with |d| <= sqrt3/2,
 * |h^-T g| <= |k|/(2 pi) + c, c = ||h^-T||_F sqrt3/2 (Frobenius above the
 * spectral norm), so
 *   1/q'(m) <= V / (sqrt(pi) s')^3 exp(s'^2 |k|^2/4 + pi s'^2 c |k| + pi^2 s'^2 c^2).
 * Term l of g_p/q' is then at most K coef_l kappa^p exp(-alpha_l kappa^2 + beta kappa)
 * with alpha_l = (s_l^2 - s'^2)/4 > 0, beta = pi s'^2 c, K = V/(sqrt(pi) s')^3
 * exp(pi^2 s'^2 c^2); its maximum over kappa lies at
 * kappa* = (beta + sqrt(beta^2 + 8 alpha_l p)) / (4 alpha_l).
 * Pinned by: B_p above every ratio found by enumeration on sheared cells.
 */
double orc_tri_start_bound(const double h[9], int M, const double *wt, const double *s, int p)
{
    double hi[9];
    const double V = fabs(tri_inverse(h, hi));
    double fro = 0.0;
    for (int i = 0; i < 9; ++i) fro += hi[i] * hi[i];
    const double c = sqrt(fro) * sqrt(3.0) / 2.0;
    const double sp = s[0] * ORC_NR_WIDEN;
    const double K = V / pow(sqrt(ORC_PI) * sp, 3) * exp(ORC_PI * ORC_PI * sp * sp * c * c);
    const double beta = ORC_PI * sp * sp * c;
    double B = 0.0;
    for (int l = 0; l < M; ++l) {
        const double coef = wt[l] * pow(s[l], p == 2 ? 5 : 7);
        const double alpha = (s[l] * s[l] - sp * sp) / 4.0;
        const double ks = (beta + sqrt(beta * beta + 8.0 * alpha * p)) / (4.0 * alpha);
        B += coef * pow(ks, p) * exp(-alpha * ks * ks + beta * ks);
    }
    return K * B;
}

/* start state by rejection from the widened proposal (as orc_exact_start, general cell) */
static int tri_exact_start(const double h[9], int M, const double *wt, const double *s, uint64_t seed, uint64_t sys,
                           uint64_t step, int p, uint32_t sxy, uint32_t sz, int32_t out[3])
{
    const double B = orc_tri_start_bound(h, M, wt, s, p);
    for (uint32_t t = 0; t < ORC_START_TRIES; ++t) {
        double z[3], u[2];
        int32_t m[3];
        orc_draw_proposal(seed, sys, step, t, sxy, sz, z, NULL);
        tri_round_proposal(z, h, s[0] * ORC_NR_WIDEN, m);
        orc_draw(seed, sys, step, t, 7u, &u[0], &u[1]);
        const double w = p == 2 ? tri_weight(m, h, M, wt, s, s[0] * ORC_NR_WIDEN) : tri_weight_nr(m, h, M, wt, s);
        if ((p == 2 ? u[0] : u[1]) * B < w) {
            memcpy(out, m, sizeof(int32_t) * 3);
            return 0;
        }
    }
    return -1;
}

int orc_tri_start_states(const double h[9], int M, const double *wt, const double *s, uint64_t seed, uint64_t sys,
                         uint64_t step, int32_t m_r0[3], int32_t m_nr0[3])
{
    if (tri_exact_start(h, M, wt, s, seed, sys, step, 2, 3u, 4u, m_r0)) return -1;
    if (tri_exact_start(h, M, wt, s, seed, sys, step, 4, 8u, 9u, m_nr0)) return -1;
    return 0;
}

/*
 * One sampling step on a general cell: orc_sample_modes with k = 2 pi h^-T m,
 * the proposal round(h^T u) and its pmf by quadrature; the same draws,
 * streams and variants (0 as printed, 1 exchange, 2 shared, 3 independent).
 * Pinned by: equality with orc_sample_modes at h = diag(L), chi^2 of the
 * start states and batch means on a sheared cell.
 */
/* the chains of one step from given start states (start_nr read by variants 1 and 3) */
void orc_tri_chains(const double h[9], int M, const double *wt, const double *s, int P, uint64_t seed, uint64_t sys,
                    uint64_t step, int variant, const int32_t start_r[3], const int32_t start_nr[3], int32_t *m_r,
                    int32_t *m_nr, int64_t n_acc[2])
{
    int32_t cur[3] = {start_r[0], start_r[1], start_r[2]};
    int32_t z0[3] = {start_nr[0], start_nr[1], start_nr[2]};
    double wcur = tri_weight(cur, h, M, wt, s, s[0]);
    double *unr = malloc(sizeof(double) * (P > 0 ? P : 1));
    int64_t acc_r = 0, acc_nr = 0;
    int32_t znr[3];
    double wz = 0.0, rz = 0.0;
    if (variant == 1) {
        memcpy(znr, z0, sizeof znr);
        wz = tri_weight(znr, h, M, wt, s, s[0]);
        rz = orc_tri_ratio_nr(znr, h, M, wt, s);
    }
    for (int t = 0; t < P; ++t) {
        double z[3], uacc[2];
        int32_t prop[3];
        orc_draw_proposal(seed, sys, step, (uint32_t)t, 0u, 1u, z, uacc);
        unr[t] = uacc[1];
        tri_round_proposal(z, h, s[0], prop);
        const double wprop = tri_weight(prop, h, M, wt, s, s[0]);
        if (uacc[0] < wprop / wcur) {
            memcpy(cur, prop, sizeof cur);
            wcur = wprop;
            ++acc_r;
        }
        if (variant == 1) {
            const double rx = orc_tri_ratio_nr(cur, h, M, wt, s);
            if (uacc[1] < rx / rz) {
                int32_t tmp[3];
                memcpy(tmp, cur, sizeof tmp);
                memcpy(cur, znr, sizeof cur);
                memcpy(znr, tmp, sizeof znr);
                const double tw = wcur;
                wcur = wz;
                wz = tw;
                rz = rx;
                ++acc_nr;
            }
            memcpy(&m_nr[3 * t], znr, sizeof znr);
        }
        memcpy(&m_r[3 * t], cur, sizeof cur);
    }
    if (variant == 0) {
        int32_t c0[3] = {m_r[0], m_r[1], m_r[2]};
        double rc = orc_tri_ratio_nr(c0, h, M, wt, s);
        for (int t = 0; t < P; ++t) {
            const double rp = orc_tri_ratio_nr(&m_r[3 * t], h, M, wt, s);
            if (unr[t] < rp / rc) {
                memcpy(c0, &m_r[3 * t], sizeof c0);
                rc = rp;
                ++acc_nr;
            }
            memcpy(&m_nr[3 * t], c0, sizeof c0);
        }
    }
    if (variant == 2) memcpy(m_nr, m_r, sizeof(int32_t) * 3 * (size_t)(P > 0 ? P : 0));
    if (variant == 3) {
        int32_t zc[3];
        memcpy(zc, z0, sizeof zc);
        double wzc = tri_weight_nr(zc, h, M, wt, s);
        for (int t = 0; t < P; ++t) {
            double z[3];
            int32_t prop[3];
            orc_draw_proposal(seed, sys, step, (uint32_t)t, 5u, 6u, z, NULL);
            tri_round_proposal(z, h, s[0] * ORC_NR_WIDEN, prop);
            const double wprop = tri_weight_nr(prop, h, M, wt, s);
            if (unr[t] < wprop / wzc) {
                memcpy(zc, prop, sizeof zc);
                wzc = wprop;
                ++acc_nr;
            }
            memcpy(&m_nr[3 * t], zc, sizeof zc);
        }
    }
    free(unr);
    if (n_acc) {
        n_acc[0] = acc_r;
        n_acc[1] = acc_nr;
    }
}

int orc_tri_sample_modes(const double h[9], int M, const double *wt, const double *s, int P, uint64_t seed,
                         uint64_t sys, uint64_t step, int variant, int32_t *m_r, int32_t *m_nr, int64_t n_acc[2])
{
    int32_t cur[3], z0[3] = {0, 0, 0};
    if (tri_exact_start(h, M, wt, s, seed, sys, step, 2, 3u, 4u, cur)) return -1;
    if ((variant == 1 || variant == 3) && tri_exact_start(h, M, wt, s, seed, sys, step, 4, 8u, 9u, z0)) return -1;
    orc_tri_chains(h, M, wt, s, P, seed, sys, step, variant, cur, z0, m_r, m_nr, n_acc);
    return 0;
}

/* rho(k) = sum_j q_j exp(i k . r_j), k = 2 pi h^-T m (eq. rho_k) */
void orc_tri_rho(int64_t n, const double *q, const double *x, const double *y, const double *z, const double h[9],
                 int64_t nm, const int32_t *m, double *re, double *im)
{
    double hi[9];
    tri_inverse(h, hi);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < nm; ++p) {
        double k[3];
        tri_k(&m[3 * p], hi, k);
        double a = 0.0, b = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double th = k[0] * x[j] + k[1] * y[j] + k[2] * z[j];
            a += q[j] * cos(th);
            b += q[j] * sin(th);
        }
        re[p] = a;
        im[p] = b;
    }
}

/* the random-batch long-range part of orc_long_range_rb for a general cell (V = det h) */
void orc_tri_long_range_rb(int64_t n, const double *q, const double *x, const double *y, const double *z,
                           const double h[9], int P, const int32_t *m_r, const int32_t *m_nr, double Sr, double Snr,
                           double *fx, double *fy, double *fz, double Pr[9], double Pnr[9], double *UF)
{
    double hi[9];
    const double V = fabs(tri_inverse(h, hi));
    double *rr = malloc(sizeof(double) * P), *ri = malloc(sizeof(double) * P);
    double *nr_re = malloc(sizeof(double) * P), *nr_im = malloc(sizeof(double) * P);
    orc_tri_rho(n, q, x, y, z, h, P, m_r, rr, ri);
    orc_tri_rho(n, q, x, y, z, h, P, m_nr, nr_re, nr_im);
    double sum_r = 0.0;
    for (int p = 0; p < P; ++p) sum_r += (rr[p] * rr[p] + ri[p] * ri[p]) / tri_k2(&m_r[3 * p], hi);
    for (int a = 0; a < 9; ++a) Pr[a] = 0.0;
    Pr[0] = Pr[4] = Pr[8] = Sr / (4.0 * V * V * P) * sum_r;
    double acc[9] = {0};
    for (int p = 0; p < P; ++p) {
        double k[3];
        tri_k(&m_nr[3 * p], hi, k);
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double a2 = nr_re[p] * nr_re[p] + nr_im[p] * nr_im[p];
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) acc[3 * al + be] += a2 * k[al] * k[be] / (k2 * k2);
    }
    for (int a = 0; a < 9; ++a) Pnr[a] = -Snr / (8.0 * V * V * P) * acc[a];
    const double S = 0.5 * Sr;
    *UF = S / (2.0 * V * P) * sum_r;
    if (fx) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double f[3] = {0, 0, 0};
            for (int p = 0; p < P; ++p) {
                double k[3];
                tri_k(&m_r[3 * p], hi, k);
                const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                const double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
                const double imv = ri[p] * cos(th) - rr[p] * sin(th);
                for (int d = 0; d < 3; ++d) f[d] += k[d] * imv / k2;
            }
            fx[i] = -(S / P) * (q[i] / V) * f[0];
            fy[i] = -(S / P) * (q[i] / V) * f[1];
            fz[i] = -(S / P) * (q[i] / V) * f[2];
        }
    }
    free(rr); free(ri); free(nr_re); free(nr_im);
}

/*
 * Short-range force, virial sum and energy (eqs. force_SOG, P_short,
 * U_short) over every image r_i - r_j + h n inside r_c (no minimum-image
 * assumption), O(N^2 x images).  Pinned by: orc_short_range_brute at
 * h = diag(L), invariance under h -> h U, and the SOG totals against Ewald.
 */
void orc_tri_short_range(int64_t n, const double *q, const double *x, const double *y, const double *z,
                         const double h[9], double rc, int M, const double *w, const double *wt, const double *s,
                         double *fx, double *fy, double *fz, double vir[6], double *U)
{
    double hi[9], wd[3];
    tri_inverse(h, hi);
    tri_widths(hi, wd);
    int nimg[3];
    for (int i = 0; i < 3; ++i) nimg[i] = (int)ceil(rc / wd[i]) + 1;
    double *vi = calloc((size_t)n * 7, sizeof(double));
    const double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; ++i) {
        double f[3] = {0, 0, 0}, v[6] = {0, 0, 0, 0, 0, 0}, u = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            /* the fractional difference wrapped to [-1/2, 1/2), then every image near it */
            const double dr[3] = {x[i] - x[j], y[i] - y[j], z[i] - z[j]};
            double ds[3];
            for (int a = 0; a < 3; ++a) {
                ds[a] = hi[3 * a] * dr[0] + hi[3 * a + 1] * dr[1] + hi[3 * a + 2] * dr[2];
                ds[a] -= round(ds[a]);
            }
            for (int a = -nimg[0]; a <= nimg[0]; ++a)
                for (int b = -nimg[1]; b <= nimg[1]; ++b)
                    for (int c = -nimg[2]; c <= nimg[2]; ++c) {
                        const double t[3] = {ds[0] + a, ds[1] + b, ds[2] + c};
                        double d[3];
                        for (int e = 0; e < 3; ++e) d[e] = h[3 * e] * t[0] + h[3 * e + 1] * t[1] + h[3 * e + 2] * t[2];
                        orc_pair(q[i], q[j], d, rc2, M, w, wt, s, f, v, &u);
                    }
        }
        fx[i] = f[0]; fy[i] = f[1]; fz[i] = f[2];
        for (int k = 0; k < 6; ++k) vi[7 * i + k] = v[k];
        vi[7 * i + 6] = u;
    }
    for (int k = 0; k < 6; ++k) vir[k] = 0.0;
    *U = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 6; ++k) vir[k] += vi[7 * i + k];
        *U += vi[7 * i + 6];
    }
    free(vi);
}

/* every m != 0 with s0^2 |k|^2 / 4 <= ORC_TRUNC, k = 2 pi h^-T m; returns the count, *out malloc'd */
static int64_t tri_modes(const double h[9], const double hi[9], double kmax, int32_t **out)
{
    int mmax[3];
    for (int j = 0; j < 3; ++j) mmax[j] = (int)ceil(tri_col_len(h, j) * kmax / (2.0 * ORC_PI)) + 1;
    const int64_t nk = (int64_t)(2 * mmax[0] + 1) * (2 * mmax[1] + 1) * (2 * mmax[2] + 1);
    int32_t *mm = malloc(sizeof(int32_t) * 3 * nk);
    int64_t cnt = 0;
    for (int a = -mmax[0]; a <= mmax[0]; ++a)
        for (int b = -mmax[1]; b <= mmax[1]; ++b)
            for (int c = -mmax[2]; c <= mmax[2]; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                const int32_t mv[3] = {a, b, c};
                if (tri_k2(mv, hi) > kmax * kmax) continue;
                mm[3 * cnt] = a; mm[3 * cnt + 1] = b; mm[3 * cnt + 2] = c;
                ++cnt;
            }
    *out = mm;
    return cnt;
}

/* the full k-space sums of orc_sog_kspace_full (Theorem 1) for a general cell */
void orc_tri_sog_kspace_full(int64_t n, const double *q, const double *x, const double *y, const double *z,
                             const double h[9], int M, const double *w, const double *wt, const double *s,
                             double *fx, double *fy, double *fz, double Pf[9], double *UF)
{
    double hi[9];
    const double V = fabs(tri_inverse(h, hi));
    int32_t *mm;
    const int64_t cnt = tri_modes(h, hi, sqrt(4.0 * ORC_TRUNC) / s[0], &mm);
    double *rre = malloc(sizeof(double) * (cnt + 1)), *rim = malloc(sizeof(double) * (cnt + 1));
    double *fh = malloc(sizeof(double) * (cnt + 1));
    orc_tri_rho(n, q, x, y, z, h, cnt, mm, rre, rim);
    double u = 0.0, pf[9] = {0};
    for (int64_t p = 0; p < cnt; ++p) {
        double k[3];
        tri_k(&mm[3 * p], hi, k);
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double a2 = rre[p] * rre[p] + rim[p] * rim[p];
        double F = 0.0;
        for (int l = 0; l < M; ++l) F += pow(ORC_PI, 1.5) * w[l] * pow(s[l], 3) * exp(-s[l] * s[l] * k2 / 4.0);
        fh[p] = F;
        u += F * a2;
        for (int l = 0; l < M; ++l) {
            const double g = wt[l] * pow(s[l], 5) * exp(-s[l] * s[l] * k2 / 4.0) * a2;
            for (int al = 0; al < 3; ++al)
                for (int be = 0; be < 3; ++be)
                    pf[3 * al + be] += g * ((al == be ? 1.0 : 0.0) - 0.5 * s[l] * s[l] * k[al] * k[be]);
        }
    }
    *UF = u / (2.0 * V);
    for (int a = 0; a < 9; ++a) Pf[a] = pow(ORC_PI, 1.5) / (4.0 * V * V) * pf[a];
    if (fx) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double f[3] = {0, 0, 0};
            for (int64_t p = 0; p < cnt; ++p) {
                double k[3];
                tri_k(&mm[3 * p], hi, k);
                const double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
                const double imv = rim[p] * cos(th) - rre[p] * sin(th);
                for (int d = 0; d < 3; ++d) f[d] += k[d] * fh[p] * imv;
            }
            fx[i] = -q[i] / V * f[0];
            fy[i] = -q[i] / V * f[1];
            fz[i] = -q[i] / V * f[2];
        }
    }
    free(rre); free(rim); free(mm); free(fh);
}

/*
 * Ewald energy, forces and pressure tensor of orc_ewald for a general cell:
 * real space over every image inside rcut, reciprocal space over k = 2 pi
 * h^-T m with |k| < kcut.  Pinned by: the rock-salt Madelung constant in a
 * primitive (rhombohedral) fcc cell and orc_ewald at h = diag(L).
 */
void orc_tri_ewald(int64_t n, const double *q, const double *x, const double *y, const double *z, const double h[9],
                   double beta, double rcut, double kcut, double *fx, double *fy, double *fz, double Pt[9], double *U)
{
    double hi[9], wd[3];
    const double V = fabs(tri_inverse(h, hi));
    tri_widths(hi, wd);
    int nimg[3];
    for (int i = 0; i < 3; ++i) nimg[i] = (int)ceil(rcut / wd[i]) + 1;
    double *acc = calloc((size_t)n * 10, sizeof(double));
    const double rcut2 = rcut * rcut;
    const double tb = 2.0 * beta / sqrt(ORC_PI);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) {
        double f[3] = {0, 0, 0}, v[6] = {0}, u = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double dr[3] = {x[i] - x[j], y[i] - y[j], z[i] - z[j]};
            double ds[3];
            for (int a = 0; a < 3; ++a) {
                ds[a] = hi[3 * a] * dr[0] + hi[3 * a + 1] * dr[1] + hi[3 * a + 2] * dr[2];
                ds[a] -= round(ds[a]);
            }
            for (int a = -nimg[0]; a <= nimg[0]; ++a)
                for (int b = -nimg[1]; b <= nimg[1]; ++b)
                    for (int c = -nimg[2]; c <= nimg[2]; ++c) {
                        const double t[3] = {ds[0] + a, ds[1] + b, ds[2] + c};
                        double d[3];
                        for (int e = 0; e < 3; ++e) d[e] = h[3 * e] * t[0] + h[3 * e + 1] * t[1] + h[3 * e + 2] * t[2];
                        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 >= rcut2 || r2 == 0.0) continue;
                        const double r = sqrt(r2);
                        const double qq = q[i] * q[j];
                        const double g = erfc(beta * r) / (r2 * r) + tb * exp(-beta * beta * r2) / r2;
                        for (int k = 0; k < 3; ++k) f[k] += qq * g * d[k];
                        v[0] += 0.5 * qq * g * d[0] * d[0];
                        v[1] += 0.5 * qq * g * d[1] * d[1];
                        v[2] += 0.5 * qq * g * d[2] * d[2];
                        v[3] += 0.5 * qq * g * d[0] * d[1];
                        v[4] += 0.5 * qq * g * d[0] * d[2];
                        v[5] += 0.5 * qq * g * d[1] * d[2];
                        u += 0.5 * qq * erfc(beta * r) / r;
                    }
        }
        for (int k = 0; k < 3; ++k) acc[10 * i + k] = f[k];
        for (int k = 0; k < 6; ++k) acc[10 * i + 3 + k] = v[k];
        acc[10 * i + 9] = u;
    }
    double vr[6] = {0}, ur = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 6; ++k) vr[k] += acc[10 * i + 3 + k];
        ur += acc[10 * i + 9];
    }
    int32_t *mm;
    const int64_t cnt = tri_modes(h, hi, kcut, &mm);
    double *rre = malloc(sizeof(double) * (cnt + 1)), *rim = malloc(sizeof(double) * (cnt + 1)),
           *G = malloc(sizeof(double) * (cnt + 1));
    orc_tri_rho(n, q, x, y, z, h, cnt, mm, rre, rim);
    double uk = 0.0, pk[9] = {0};
    for (int64_t p = 0; p < cnt; ++p) {
        double k[3];
        tri_k(&mm[3 * p], hi, k);
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        G[p] = 4.0 * ORC_PI * exp(-k2 / (4.0 * beta * beta)) / k2;
        const double a2 = rre[p] * rre[p] + rim[p] * rim[p];
        uk += G[p] * a2;
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be)
                pk[3 * al + be] += G[p] * a2 *
                    ((al == be ? 1.0 : 0.0) - 2.0 * (1.0 + k2 / (4.0 * beta * beta)) * k[al] * k[be] / k2);
    }
    uk /= 2.0 * V;
    for (int a = 0; a < 9; ++a) pk[a] /= 2.0 * V * V;
    double q2 = 0.0;
    for (int64_t i = 0; i < n; ++i) q2 += q[i] * q[i];
    *U = ur + uk - beta / sqrt(ORC_PI) * q2;
    const int idx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) Pt[3 * al + be] = vr[idx[al][be]] / V + pk[3 * al + be];
    if (fx) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double f[3] = {acc[10 * i], acc[10 * i + 1], acc[10 * i + 2]};
            for (int64_t p = 0; p < cnt; ++p) {
                double k[3];
                tri_k(&mm[3 * p], hi, k);
                const double th = k[0] * x[i] + k[1] * y[i] + k[2] * z[i];
                const double imv = rim[p] * cos(th) - rre[p] * sin(th);
                for (int d = 0; d < 3; ++d) f[d] -= q[i] / V * k[d] * G[p] * imv;
            }
            fx[i] = f[0]; fy[i] = f[1]; fz[i] = f[2];
        }
    }
    free(acc); free(mm); free(rre); free(rim); free(G);
}

/* number of OpenMP threads the oracle runs on (1 without OpenMP) */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the oracle's parallel loops from now on (timing on one core) */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
