// Host-side set-up of the RBSOG splitting: SOG weights, the omega~ root, the
// normalisation constants S^r and S^nr, and the cell grid.  FP64, O(M) work per
// box, recomputed whenever the box changes.
#include <cmath>

#include "rbsog_impl.hpp"

namespace rbsog {

namespace {
constexpr double kPi = 3.141592653589793238462643383279502884;
// lattice sums stop once the Gaussian factor falls below exp(-kCut)
constexpr double kCut = 60.0;
}  // namespace

// Sec. 2.2 (u-series) and Sec. 3.1 (1/r^3 split), with b = b~, sigma = sigma~,
// M = M~ (Theorem 2): w_l = sqrt(2/pi) log b / (sigma b^l), wt_l = sqrt(2/pi)
// log b / (sigma b^l)^3, s_l = sqrt(2) sigma b^l; omega multiplies l = 0.
void sog_tables(const rbsog_params &p, double *w, double *wt, double *s)
{
    const double lead = std::sqrt(2.0 / kPi) * std::log(p.b);
    double width = p.sigma;  // sigma b^l
    for (int l = 0; l < p.M; ++l) {
        w[l] = lead / width;
        wt[l] = lead / (width * width * width);
        s[l] = std::sqrt(2.0) * width;
        width *= p.b;
    }
    w[0] *= p.omega;
    wt[0] *= p.omega;
}

// C0 continuity of the 1/r^3 split at rc (eq. continuity) fixes the factor on
// the narrowest Gaussian (eq. omega0): it is linear in that factor.
double omega_c0(double b, double sigma, double rc, int M)
{
    rbsog_params p{};
    p.b = b;
    p.sigma = sigma;
    p.omega = 1.0;
    p.M = M;
    double w[RBSOG_MAX_M], wt[RBSOG_MAX_M], s[RBSOG_MAX_M];
    sog_tables(p, w, wt, s);
    double tail = 0.0;
    for (int l = M - 1; l >= 1; --l) tail += wt[l] * std::exp(-(rc * rc) / (s[l] * s[l]));
    return (1.0 / (rc * rc * rc) - tail) / (wt[0] * std::exp(-(rc * rc) / (s[0] * s[0])));
}

namespace {

// One-dimensional moments sum_n g^j exp(-g^2/a2) over the lattice g = step*n,
// j = 0, 2, 4.  Every three-dimensional sum below factorises over the axes of
// an orthorhombic cell.
void moments_1d(double step, double a2, double mom[3])
{
    const int nmax = static_cast<int>(std::ceil(std::sqrt(kCut * a2) / step)) + 1;
    double m0 = 1.0, m2 = 0.0, m4 = 0.0;  // n = 0 term
    for (int k = nmax; k >= 1; --k) {
        const double g2 = (step * k) * (step * k);
        const double e = std::exp(-g2 / a2);
        m0 += 2.0 * e;
        m2 += 2.0 * g2 * e;
        m4 += 2.0 * g2 * g2 * e;
    }
    mom[0] = m0;
    mom[1] = m2;
    mom[2] = m4;
}

// sum over the 3D lattice of (sum_xi g_xi^2)^p exp(-sum g_xi^2 / a2) for
// p = 0, 1, 2, from the per-axis moments
void lattice_sums(const double mom[3][3], double out[3])
{
    const double a0 = mom[0][0] * mom[1][0] * mom[2][0];
    double a2 = 0.0, a4 = 0.0;
    for (int x = 0; x < 3; ++x) {
        const int y = (x + 1) % 3, z = (x + 2) % 3;
        a2 += mom[x][1] * mom[y][0] * mom[z][0];
        a4 += mom[x][2] * mom[y][0] * mom[z][0];
        a4 += 2.0 * mom[x][1] * mom[y][1] * mom[z][0];
    }
    out[0] = a0;
    out[1] = a2;
    out[2] = a4;
}

}  // namespace

// S^r = sum_l H^r_l, S^nr = sum_l H^nr_l (eqs. Sr, Snr).  Per Gaussian the
// real-space (Poisson, Prop. 1: V wt [6 A0 - 4 A2/s^2] and V wt [60 A0 -
// 80 A2/s^2 + 16 A4/s^4]) form is used for s_l below the shortest edge, where
// it needs only a few images and has no cancellation; wider Gaussians use the
// reciprocal-space sums of |k|^2 and |k|^4 under exp(-s^2 k^2/4) directly.
void norm_consts(const double L[3], int M, const double *wt, const double *s, double *Sr, double *Snr)
{
    const double V = L[0] * L[1] * L[2];
    const double lmin = std::fmin(L[0], std::fmin(L[1], L[2]));
    double sr = 0.0, snr = 0.0;
    for (int l = 0; l < M; ++l) {
        const double s2 = s[l] * s[l];
        double mom[3][3], A[3];
        if (s[l] < lmin) {
            for (int d = 0; d < 3; ++d) moments_1d(L[d], s2, mom[d]);
            lattice_sums(mom, A);
            sr += V * wt[l] * (6.0 * A[0] - 4.0 * A[1] / s2);
            snr += V * wt[l] * (60.0 * A[0] - 80.0 * A[1] / s2 + 16.0 * A[2] / (s2 * s2));
        } else {
            // exp(-s^2 k^2/4) = exp(-k^2/a2) with a2 = 4/s^2, k on the lattice 2 pi m / L
            for (int d = 0; d < 3; ++d) moments_1d(2.0 * kPi / L[d], 4.0 / s2, mom[d]);
            lattice_sums(mom, A);
            const double c = std::pow(kPi, 1.5) * wt[l];
            const double s5 = s2 * s2 * s[l];
            sr += c * s5 * A[1];
            snr += c * s5 * s2 * A[2];
        }
    }
    *Sr = sr;
    *Snr = snr;
}

// Bound of g_p(m) / q'(m) over the lattice for the rejection draws that start
// the chains (App. D proposal with width parameter s_0/sqrt2, per-axis
// deviation sig = L/(pi s_0); g_2 = |k|^2 sum wt s^5 e, g_4 = |k|^4 sum wt s^7 e,
// e = exp(-s^2 |k|^2/4)).  A cell of the rounded normal holds at least the
// density at its far end, so 1/q' <= prod_d sqrt(2 pi) sig_d exp((s_0 |k_d|/2 +
// c_d)^2/2), c_d = 1/(2 sig_d); with sum_d c_d |k_d| <= |c||k| every Gaussian's
// term is at most K coef kappa^p exp(-alpha kappa^2 + beta kappa) in kappa =
// |k|, alpha = s^2/4 - s_0^2/8, beta = s_0|c|/2, largest at the positive root
// of 2 alpha kappa^2 - beta kappa - p = 0.  The bound sums those maxima.
double start_bound(const double L[3], int M, const double *wt, const double *s, int power)
{
    const double s0 = s[0];
    double K = 1.0, csq = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double sig = L[d] / (kPi * s0);
        const double c = 1.0 / (2.0 * sig);
        K *= std::sqrt(2.0 * kPi) * sig * std::exp(0.5 * c * c);
        csq += c * c;
    }
    const double beta = 0.5 * s0 * std::sqrt(csq);
    double B = 0.0;
    for (int l = 0; l < M; ++l) {
        const double coef = wt[l] * std::pow(s[l], power == 2 ? 5 : 7);
        const double alpha = s[l] * s[l] / 4.0 - s0 * s0 / 8.0;
        const double kap = (beta + std::sqrt(beta * beta + 8.0 * alpha * power)) / (4.0 * alpha);
        B += coef * std::pow(kap, power) * std::exp(-alpha * kap * kap + beta * kap);
    }
    return K * B;
}

// Cells no narrower than rc (so all partners of an atom lie in the 27 cells
// around it); a dimension with fewer than three cells is searched whole.
void cell_grid(const double L[3], double rc, int nc[3])
{
    for (int d = 0; d < 3; ++d) {
        int k = static_cast<int>(std::floor(L[d] / rc));
        nc[d] = k >= 3 ? k : 1;
    }
}

// ---------------------------------------------------------------------------
// General cells h = [h_1, h_2, h_3] (row-major, columns the cell vectors)

double cell_inverse(const double h[9], double hi[9])
{
    // adjugate over the determinant
    const double c00 = h[4] * h[8] - h[5] * h[7], c01 = h[5] * h[6] - h[3] * h[8], c02 = h[3] * h[7] - h[4] * h[6];
    const double det = h[0] * c00 + h[1] * c01 + h[2] * c02;
    hi[0] = c00 / det;
    hi[1] = (h[2] * h[7] - h[1] * h[8]) / det;
    hi[2] = (h[1] * h[5] - h[2] * h[4]) / det;
    hi[3] = c01 / det;
    hi[4] = (h[0] * h[8] - h[2] * h[6]) / det;
    hi[5] = (h[2] * h[3] - h[0] * h[5]) / det;
    hi[6] = c02 / det;
    hi[7] = (h[1] * h[6] - h[0] * h[7]) / det;
    hi[8] = (h[0] * h[4] - h[1] * h[3]) / det;
    return det;
}

// Distance between the faces s_i = 0 and s_i = 1: 1 / |row i of h^-1|.
void cell_widths(const double hi[9], double w[3])
{
    for (int i = 0; i < 3; ++i)
        w[i] = 1.0 / std::sqrt(hi[3 * i] * hi[3 * i] + hi[3 * i + 1] * hi[3 * i + 1] + hi[3 * i + 2] * hi[3 * i + 2]);
}

// S^r and S^nr (eqs. Sr, Snr) for a general cell: the lattice sums no longer
// factor over axes.  Per Gaussian, the real-space form of Prop. 1 (sums over
// h n) when s_l is below the smallest width, else the reciprocal sums over
// k = 2 pi h^-T m; each truncated where the Gaussian factor falls below
// exp(-60).
void norm_consts_cell(const double h[9], int M, const double *wt, const double *s, double *Sr, double *Snr)
{
    double hi[9], wd[3];
    const double V = std::fabs(cell_inverse(h, hi));
    cell_widths(hi, wd);
    const double wmin = std::fmin(wd[0], std::fmin(wd[1], wd[2]));
    const double T = 60.0;
    double sr = 0.0, snr = 0.0;
    for (int l = 0; l < M; ++l) {
        const double s2 = s[l] * s[l];
        if (s[l] < wmin) {
            int nm[3];
            for (int i = 0; i < 3; ++i) nm[i] = static_cast<int>(std::ceil(s[l] * std::sqrt(T) / wd[i])) + 1;
            double a0 = 0.0, a2 = 0.0, a4 = 0.0;
            for (int n0 = -nm[0]; n0 <= nm[0]; ++n0)
                for (int n1 = -nm[1]; n1 <= nm[1]; ++n1)
                    for (int n2 = -nm[2]; n2 <= nm[2]; ++n2) {
                        double r2 = 0.0;
                        for (int i = 0; i < 3; ++i) {
                            const double r = h[3 * i] * n0 + h[3 * i + 1] * n1 + h[3 * i + 2] * n2;
                            r2 += r * r;
                        }
                        const double e = std::exp(-r2 / s2);
                        a0 += e;
                        a2 += r2 * e;
                        a4 += r2 * r2 * e;
                    }
            sr += V * wt[l] * (6.0 * a0 - 4.0 * a2 / s2);
            snr += V * wt[l] * (60.0 * a0 - 80.0 * a2 / s2 + 16.0 * a4 / (s2 * s2));
        } else {
            const double kmax = std::sqrt(4.0 * T) / s[l];
            int mm[3];
            for (int j = 0; j < 3; ++j) {
                const double len = std::sqrt(h[j] * h[j] + h[3 + j] * h[3 + j] + h[6 + j] * h[6 + j]);
                mm[j] = static_cast<int>(std::ceil(len * kmax / (2.0 * kPi))) + 1;
            }
            double b2 = 0.0, b4 = 0.0;
            for (int m0 = -mm[0]; m0 <= mm[0]; ++m0)
                for (int m1 = -mm[1]; m1 <= mm[1]; ++m1)
                    for (int m2 = -mm[2]; m2 <= mm[2]; ++m2) {
                        double k2 = 0.0;
                        for (int i = 0; i < 3; ++i) {
                            const double k = 2.0 * kPi * (hi[i] * m0 + hi[3 + i] * m1 + hi[6 + i] * m2);
                            k2 += k * k;
                        }
                        const double e = std::exp(-s2 * k2 / 4.0);
                        b2 += k2 * e;
                        b4 += k2 * k2 * e;
                    }
            const double c = std::pow(kPi, 1.5) * wt[l] * s2 * s2 * s[l];
            sr += c * b2;
            snr += c * s2 * b4;
        }
    }
    *Sr = sr;
    *Snr = snr;
}

// Bound of g_p(m)/q'(m) for a general cell.  The integrand of q' (width
// parameter s' = s_0/sqrt2) over the unit cube around m is at least its
// value where |h^-T g| is largest, and |h^-T g| <= |k|/(2 pi) + c with
// c = sqrt3/2 ||h^-T||_F, so 1/q' <= V/(sqrt(pi) s')^3 exp(pi^2 s'^2 (|k|/(2 pi) + c)^2);
// term l of g_p/q' is then K coef_l kappa^p exp(-alpha_l kappa^2 + beta kappa)
// with alpha_l = (s_l^2 - s'^2)/4, beta = pi s'^2 c, K = V/(sqrt(pi) s')^3
// exp(pi^2 s'^2 c^2), largest at kappa = (beta + sqrt(beta^2 + 8 alpha_l p))/(4 alpha_l).
double start_bound_cell(const double h[9], int M, const double *wt, const double *s, int power)
{
    double hi[9];
    const double V = std::fabs(cell_inverse(h, hi));
    double f2 = 0.0;
    for (int i = 0; i < 9; ++i) f2 += hi[i] * hi[i];
    const double c = std::sqrt(f2) * std::sqrt(3.0) / 2.0;
    const double sp = s[0] * 0.70710678118654752440;
    const double K = V / std::pow(std::sqrt(kPi) * sp, 3) * std::exp(kPi * kPi * sp * sp * c * c);
    const double beta = kPi * sp * sp * c;
    double B = 0.0;
    for (int l = 0; l < M; ++l) {
        const double coef = wt[l] * std::pow(s[l], power == 2 ? 5 : 7);
        const double alpha = (s[l] * s[l] - sp * sp) / 4.0;
        const double kap = (beta + std::sqrt(beta * beta + 8.0 * alpha * power)) / (4.0 * alpha);
        B += coef * std::pow(kap, power) * std::exp(-alpha * kap * kap + beta * kap);
    }
    return K * B;
}

// n-point Gauss-Legendre rule on [-1/2, 1/2]: the roots of P_n by Newton
// steps from x = cos(pi (i + 3/4) / (n + 1/2)), weights 2/((1 - x^2) P_n'(x)^2),
// both mapped to the unit interval.
void gauss_legendre_unit(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double r = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double deriv = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pm = 1.0, pc = r;  // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double pn = ((2 * k - 1) * r * pc - (k - 1) * pm) / k;
                pm = pc;
                pc = pn;
            }
            deriv = n * (r * pc - pm) / (r * r - 1.0);
            const double step = pc / deriv;
            r -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        x[i] = 0.5 * r;
        w[i] = 1.0 / ((1.0 - r * r) * deriv * deriv);
    }
}

}  // namespace rbsog
