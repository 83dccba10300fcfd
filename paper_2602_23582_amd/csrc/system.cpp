// Systems and batches on the host: validation, splitting tables, device
// buffer layout, descriptors, launch plans and their uploads, event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "rbsog_impl.hpp"

namespace rbsog {

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_fp64(const rbsog_params &p) { return p.precision == RBSOG_PREC_FP64; }

// byte sizes of the per-atom and per-mode buffers, in carving order
struct AtomLayout {
    size_t q, u, cell, slot, keys, urec, perm, rec, fsr, mraw, modes, cnt, rho_part, rho, pair_red, coef, scan_tmp;
    size_t total() const
    {
        return q + u + cell + slot + keys + urec + perm + rec + fsr + mraw + modes + cnt + rho_part + rho + pair_red + coef +
               scan_tmp;
    }
};

AtomLayout atom_layout(const rbsog_params &p, int64_t n)
{
    const bool f64 = is_fp64(p);
    const size_t rsz = f64 ? 8 : 4, fsz = f64 ? 8 : 4, recsz = f64 ? 32 : 16;
    const size_t mcap = static_cast<size_t>(mode_cap(p));
    const size_t skb = static_cast<size_t>((n + kSkChunk - 1) / kSkChunk);
    AtomLayout a{};
    a.q = align_up(n * rsz);
    a.u = align_up(3 * n * fsz);
    a.cell = align_up(n * 4);
    a.slot = align_up(n * 4);
    a.keys = align_up(n * 8);
    a.urec = align_up(n * recsz);
    a.perm = align_up(n * 4);
    a.rec = align_up(n * recsz);
    a.fsr = align_up(3 * n * rsz);
    a.mraw = align_up(6 * static_cast<size_t>(p.P) * 4);
    a.modes = align_up(mcap * sizeof(int4));
    a.cnt = align_up(2 * mcap * 4);
    a.rho_part = align_up(skb * mcap * 16);
    a.rho = align_up(mcap * 16);
    a.pair_red = align_up(kPairRed * 8 * sizeof(double));
    a.coef = align_up(mcap * 64);
    a.scan_tmp = align_up((2 * 1024 + 2) * 4);
    return a;
}

// Chebyshev interpolant of degree kPolyDeg of g(x) = sum_l c_l exp(-x/s_l^2)
// on x in [0, X], returned as monomial coefficients in t = 2x/X - 1; *err is
// the largest |p - g| on a fine grid divided by g(0).
void poly_fit(const double *c, const double *s, int M, double X, double mono[kPolyDeg + 1], double *err)
{
    constexpr int N = kPolyDeg + 1;
    constexpr double pi = 3.141592653589793238462643383279502884;
    auto g = [&](double x) {
        double v = 0.0;
        for (int l = 0; l < M; ++l) v += c[l] * std::exp(-x / (s[l] * s[l]));
        return v;
    };
    double f[N], cheb[N];
    for (int k = 0; k < N; ++k) f[k] = g(0.5 * X * (1.0 + std::cos(pi * (k + 0.5) / N)));
    for (int j = 0; j < N; ++j) {
        double a = 0.0;
        for (int k = 0; k < N; ++k) a += f[k] * std::cos(pi * j * (k + 0.5) / N);
        cheb[j] = (j == 0 ? 1.0 : 2.0) * a / N;
    }
    // T_j in monomials: T_0 = 1, T_1 = t, T_{j+1} = 2 t T_j - T_{j-1}
    double Tm[N][N] = {};
    Tm[0][0] = 1.0;
    if (N > 1) Tm[1][1] = 1.0;
    for (int j = 1; j + 1 < N; ++j)
        for (int k = 0; k < N; ++k) Tm[j + 1][k] = (k > 0 ? 2.0 * Tm[j][k - 1] : 0.0) - Tm[j - 1][k];
    for (int k = 0; k < N; ++k) {
        mono[k] = 0.0;
        for (int j = 0; j < N; ++j) mono[k] += cheb[j] * Tm[j][k];
    }
    double e = 0.0;
    const int grid = 8192;
    for (int q = 0; q <= grid; ++q) {
        const double x = X * q / grid, t = 2.0 * x / X - 1.0;
        double p = 0.0;
        for (int k = kPolyDeg; k >= 0; --k) p = p * t + mono[k];
        e = std::max(e, std::fabs(p - g(x)));
    }
    *err = e / g(0.0);
}

// largest accepted truncation error of the polynomial form (FP32 rounding is ~1e-7)
constexpr double kPolyTol = 5e-8;

// The fit and its error check cost about a millisecond; systems set up with
// the same weights, widths and cutoff (a served stream's, a batch's) share
// one.  A cached fit is the fit the same inputs give, bit for bit.
void poly_fit_cached(const double *c, const double *s, int M, double X, double mono[kPolyDeg + 1], double *err)
{
    struct Fit {
        double mono[kPolyDeg + 1];
        double err;
    };
    static std::mutex mu;
    static std::map<std::vector<double>, Fit> cache;
    std::vector<double> key;
    key.reserve(2 * M + 2);
    key.push_back(M);
    key.push_back(X);
    key.insert(key.end(), c, c + M);
    key.insert(key.end(), s, s + M);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            std::memcpy(mono, it->second.mono, sizeof(it->second.mono));
            *err = it->second.err;
            return;
        }
    }
    Fit f;
    poly_fit(c, s, M, X, f.mono, &f.err);
    std::memcpy(mono, f.mono, sizeof(f.mono));
    *err = f.err;
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() >= 1024) cache.clear();
    cache.emplace(std::move(key), f);
}

}  // namespace

int check_box(const double *box, double rc, std::string &err)
{
    if (!box) {
        err = "box is NULL";
        return RBSOG_EINVAL;
    }
    if (!std::isfinite(box[0]) || !std::isfinite(box[1]) || !std::isfinite(box[2])) {
        err = "box has NaN/Inf";
        return RBSOG_EINVAL;
    }
    if (box[0] <= 0 || box[1] <= 0 || box[2] <= 0) {
        err = "box edges must be positive";
        return RBSOG_EBOX;
    }
    const double lmin = std::min(box[0], std::min(box[1], box[2]));
    if (rc > 0.5 * lmin) {
        err = "cutoff exceeds half the shortest box edge";
        return RBSOG_EBOX;
    }
    int nc[3];
    cell_grid(box, rc, nc);
    if (static_cast<int64_t>(nc[0]) * nc[1] * nc[2] > kMaxCells) {
        err = "more than 2^20 cells: box too large for rc";
        return RBSOG_EBOX;
    }
    return RBSOG_OK;
}

int64_t cells_for_box(const double box[3], double rc)
{
    int nc[3];
    cell_grid(box, rc, nc);
    return static_cast<int64_t>(nc[0]) * nc[1] * nc[2];
}

int system_init(System &s, const rbsog_params &p, int64_t n, const double *host_q, const double box[3],
                std::string &err)
{
    if (n <= 0 || n > (int64_t)1 << 30) {
        err = "atom count must be in [1, 2^30]";
        return RBSOG_EINVAL;
    }
    if (!host_q) {
        err = "charges are NULL";
        return RBSOG_EINVAL;
    }
    if (!(p.b > 1.0) || !(p.sigma > 0.0) || !std::isfinite(p.b) || !std::isfinite(p.sigma) ||
        !std::isfinite(p.omega)) {
        err = "bad SOG parameters";
        return RBSOG_EINVAL;
    }
    if (p.M < 1 || p.M > RBSOG_MAX_M || p.P < 1 || p.P > kMaxP) {
        err = "M or P out of range";
        return RBSOG_EINVAL;
    }
    if (p.M_energy != 0 && (p.M_energy < p.M || p.M_energy > RBSOG_MAX_M)) {
        err = "M_energy must be 0 or in [M, 64]";
        return RBSOG_EINVAL;
    }
    if (!(p.rc > 0.0) || !std::isfinite(p.rc) || !std::isfinite(p.coulomb_k)) {
        err = "bad cutoff or prefactor";
        return RBSOG_EINVAL;
    }
    if (p.precision != RBSOG_PREC_FP64 && p.precision != RBSOG_PREC_FP32C) {
        err = "unknown precision";
        return RBSOG_EINVAL;
    }
    if (p.recalibration < RBSOG_RECAL_PRINTED || p.recalibration > RBSOG_RECAL_INDEPENDENT) {
        err = "unknown recalibration";
        return RBSOG_EINVAL;
    }
    if (mode_cap(p) > kMaxModes) {
        err = "the independent non-radial chain takes P <= 512";
        return RBSOG_EINVAL;
    }
    if (p.system_id >> 32) {
        err = "system_id must be < 2^32";
        return RBSOG_EINVAL;
    }
    if (p.flags & ~(RBSOG_FLAG_EXP_FORM | RBSOG_FLAG_FULL_SHELL | RBSOG_FLAG_HALF_SHELL)) {
        err = "unknown flags";
        return RBSOG_EINVAL;
    }
    if ((p.flags & RBSOG_FLAG_FULL_SHELL) && (p.flags & RBSOG_FLAG_HALF_SHELL)) {
        err = "full-shell and half-shell flags together";
        return RBSOG_EINVAL;
    }
    double qs = 0.0, qa = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(host_q[i])) {
            err = "charges have NaN/Inf";
            return RBSOG_EINVAL;
        }
        qs += host_q[i];
        qa += std::fabs(host_q[i]);
    }
    if (std::fabs(qs) > 1e-10 * qa) {
        err = "charges are not neutral";
        return RBSOG_ENEUTRAL;
    }
    int rc = check_box(box, p.rc, err);
    if (rc) return rc;

    s.prm = p;
    s.n = n;
    if (s.prm.omega <= 0.0) s.prm.omega = omega_c0(p.b, p.sigma, p.rc, p.M);
    // the energy's Gaussians extend the force's (R1): Me terms of w, M of wt
    const int Me = p.M_energy > 0 ? p.M_energy : p.M;
    {
        rbsog_params pe = s.prm;
        pe.M = Me;
        sog_tables(pe, s.w, s.wt, s.s);
        for (int l = p.M; l < Me; ++l) s.wt[l] = 0.0;
    }
    double wsum = 0.0;
    for (int l = 0; l < Me; ++l) wsum += s.w[l];
    s.q2sum = 0.0;
    for (int64_t i = 0; i < n; ++i) s.q2sum += host_q[i] * host_q[i];
    // U_self = (1/2) F(0) sum q^2 (App. A)
    s.Uself = p.coulomb_k * 0.5 * wsum * s.q2sum;

    SogTables &tab = s.tab;
    tab = SogTables{};
    tab.M = p.M;
    tab.Me = Me;
    tab.rc2 = p.rc * p.rc;
    tab.rc2_32 = static_cast<float>(p.rc * p.rc);
    gauss_legendre_unit(kGl, tab.glx, tab.glw);
    const double log2e = 1.4426950408889634073599246810018921;
    for (int l = 0; l < Me; ++l) {
        tab.w[l] = s.w[l];
        tab.wt[l] = s.wt[l];
        tab.s[l] = s.s[l];
        tab.inv_s2[l] = 1.0 / (s.s[l] * s.s[l]);
        tab.s5[l] = std::pow(s.s[l], 5);
        tab.s7[l] = std::pow(s.s[l], 7);
        tab.w32[l] = static_cast<float>(s.w[l]);
        tab.wt32[l] = static_cast<float>(s.wt[l]);
        tab.c32[l] = static_cast<float>(-log2e / (s.s[l] * s.s[l]));
    }
    // FP32C: the SOG sums as polynomials in r^2 when the fit is within
    // kPolyTol of the exponential form; otherwise the M exponentials
    s.pair_form = p.M == 10 && Me == p.M ? kFormExp10 : kFormExpM;
    if (p.precision == RBSOG_PREC_FP32C) {
        const double X = p.rc * p.rc;
        double mg[kPolyDeg + 1], mf[kPolyDeg + 1], eg = 1.0, ef = 1.0;
        poly_fit_cached(s.wt, s.s, p.M, X, mg, &eg);
        poly_fit_cached(s.w, s.s, Me, X, mf, &ef);
        tab.poly_err = static_cast<float>(std::max(eg, ef));
        if (eg <= kPolyTol && ef <= kPolyTol && !(p.flags & RBSOG_FLAG_EXP_FORM)) {
            tab.poly = 1;
            tab.pa = static_cast<float>(2.0 / X);
            for (int k = 0; k <= kPolyDeg; ++k) {
                tab.pg[k] = static_cast<float>(mg[k]);
                tab.pf[k] = static_cast<float>(mf[k]);
            }
            s.pair_form = kFormPoly;
        }
    }

    SysDesc &d = s.desc;
    d = SysDesc{};
    d.tab = tab;
    d.n = n;
    d.sk_blocks = (n + kSkChunk - 1) / kSkChunk;
    d.P = p.P;
    d.M = p.M;
    d.variant = p.recalibration;
    d.mcap = mode_cap(p);
    d.key0 = static_cast<uint32_t>(p.seed);
    d.key1 = static_cast<uint32_t>(p.seed >> 32);
    d.sys = static_cast<uint32_t>(p.system_id);
    d.ck = p.coulomb_k;
    d.Uself = s.Uself;
    s.stp = SysStep{};
    for (int k = 0; k < 3; ++k) s.stp.mu[k] = 1.0;
    system_set_box(s, box);
    return RBSOG_OK;
}

bool wants_half_shell(const System &s)
{
    if (is_fp64(s.prm) || !s.own_mem || (s.prm.flags & RBSOG_FLAG_FULL_SHELL)) return false;
    return (s.prm.flags & RBSOG_FLAG_HALF_SHELL) != 0;
}

// Forward candidates a half-shell block can hold.  A full block of 64 atoms in
// a column of cross-section A spans 64/(rho A) in z, so each of its four
// neighbour columns contributes about 64 + 2 rho A rc atoms to its window and
// its own column 64 + rho A rc; A is at most rc^2 (n_x+1)/n_x (n_y+1)/n_y for
// the grid, and rho the reference density.  The margin and a last chunk for
// rounding go on top.
int32_t half_hcap(const System &s)
{
    const double rc = s.prm.rc + 1e-3;
    const double A = s.prm.rc * s.prm.rc * (s.nc[0] + 1.0) / s.nc[0] * (s.nc[1] + 1.0) / s.nc[1];
    const double rhoA = kHalfRefDensity * A;
    const double est = 4.0 * (kPairWave + 2.0 * rhoA * rc) + (kPairWave + rhoA * rc);
    const int64_t c = static_cast<int64_t>(std::ceil(kHalfMargin * est / 128.0)) + 1;
    return static_cast<int32_t>(std::min<int64_t>(c * 128, int64_t(1) << 24));
}

void system_set_box(System &s, const double box[3])
{
    s.tri = false;
    s.stp.tri = 0;
    for (int d = 0; d < 9; ++d) {
        s.h[d] = 0.0;
        s.stp.h[d] = 0.0;
        s.stp.hi[d] = 0.0;
    }
    for (int d = 0; d < 3; ++d) {
        s.h[4 * d] = box[d];
        s.stp.h[4 * d] = box[d];
        s.stp.hi[4 * d] = 1.0 / box[d];
    }
    s.stp.V = box[0] * box[1] * box[2];
    for (int d = 0; d < 3; ++d) s.L[d] = box[d];
    cell_grid(s.L, s.prm.rc, s.nc);
    s.ncells = static_cast<int64_t>(s.nc[0]) * s.nc[1] * s.nc[2];
    norm_consts(s.L, s.prm.M, s.wt, s.s, &s.Sr, &s.Snr);
    SysStep &t = s.stp;
    t.Bstart[0] = start_bound(s.L, s.prm.M, s.wt, s.s, 2);
    t.Bstart[1] = start_bound(s.L, s.prm.M, s.wt, s.s, 4);
    for (int d = 0; d < 3; ++d) {
        t.L[d] = s.L[d];
        t.iL[d] = 1.0 / s.L[d];
        t.nc[d] = s.nc[d];
    }
    t.ncells = static_cast<int32_t>(s.ncells);
    // Pair blocks are 64-atom z-slabs of segments of g cells of one column.
    // The FP32 filter takes coordinates relative to a block's first atom o.
    // A neighbour of a block atom lies less than two cells from o along x and
    // y, and less than g + 1 cells along z; that is under half the box when
    // nx, ny >= 4 and nz >= 2 g + 2 (g = 1 for nz < 7), so the relative
    // coordinates of every pair inside rc are minimum-image offsets and their
    // difference is the displacement.  The other paths use single cells.
    const bool fast = !is_fp64(s.prm) && s.nc[0] >= 4 && s.nc[1] >= 4 && s.nc[2] >= 4;
    t.fast = fast ? 1 : 0;
    // Newton's third law on the fast path for systems that own their memory
    // (the served pool's requests keep the full shell and its smaller footprint)
    t.half = fast && wants_half_shell(s) ? 1 : 0;
    t.g = fast ? std::max(1, std::min(kSuperCells, (s.nc[2] - 3) / 2)) : 1;
    // The FP32 exact filter compares 16-bit wrapped differences of the
    // fixed-point coordinates, in units u_d = L_d / 2^16 truncated (under one
    // unit per axis): a pair inside rc has sum (d_d/u_d)^2 < (rc/u_min + sqrt 3)^2,
    // at most (2^15 + 2)^2 since rc <= L/2.
    const double umin = std::min(s.L[0], std::min(s.L[1], s.L[2])) * 0x1.0p-16;
    const double tr = static_cast<double>(static_cast<float>(s.prm.rc * s.prm.rc));
    const double tb = std::sqrt(tr) / umin + 2.0;
    t.thr16 = static_cast<uint32_t>(tb * tb) + 1u;
    t.Sr = s.Sr;
    t.Snr = s.Snr;
}

int system_set_cell(System &s, const double h[9], std::string &err)
{
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(h[i])) {
            err = "cell tensor has NaN/Inf";
            return RBSOG_EINVAL;
        }
    const bool diag = h[1] == 0.0 && h[2] == 0.0 && h[3] == 0.0 && h[5] == 0.0 && h[6] == 0.0 && h[7] == 0.0;
    if (diag) {
        const double box[3] = {h[0], h[4], h[8]};
        const int rc = check_box(box, s.prm.rc, err);
        if (rc != RBSOG_OK) return rc;
        system_set_box(s, box);
        return RBSOG_OK;
    }
    double hi[9], wd[3];
    const double det = cell_inverse(h, hi);
    if (!(det > 0.0)) {
        err = "the cell tensor must have a positive determinant";
        return RBSOG_EBOX;
    }
    cell_widths(hi, wd);
    const double wmin = std::min(wd[0], std::min(wd[1], wd[2]));
    if (2.0 * s.prm.rc > wmin) {
        err = "rc must be at most half the smallest perpendicular width of the cell";
        return RBSOG_EBOX;
    }
    s.tri = true;
    SysStep &t = s.stp;
    t.tri = 1;
    for (int i = 0; i < 9; ++i) {
        s.h[i] = h[i];
        t.h[i] = h[i];
        t.hi[i] = hi[i];
    }
    t.V = det;
    // cells no thinner than rc between their faces: every partner of an atom
    // lies in the 27 cells around it; fewer than three cells: one, searched whole
    for (int d = 0; d < 3; ++d) {
        s.L[d] = h[4 * d];
        const int k = static_cast<int>(std::floor(wd[d] / s.prm.rc));
        s.nc[d] = k >= 3 ? k : 1;
    }
    s.ncells = static_cast<int64_t>(s.nc[0]) * s.nc[1] * s.nc[2];
    norm_consts_cell(h, s.prm.M, s.wt, s.s, &s.Sr, &s.Snr);
    t.Bstart[0] = start_bound_cell(h, s.prm.M, s.wt, s.s, 2);
    t.Bstart[1] = start_bound_cell(h, s.prm.M, s.wt, s.s, 4);
    for (int d = 0; d < 3; ++d) {
        t.L[d] = s.L[d];
        t.iL[d] = 1.0 / s.L[d];
        t.nc[d] = s.nc[d];
    }
    t.ncells = static_cast<int32_t>(s.ncells);
    // The FP32 relative-coordinate path of a box holds for the fractional
    // grid too (every partner of a block atom within two cells of its first
    // atom along each fractional axis, under half the cell): offsets from
    // that atom are wrapped fractional differences, times h.
    const bool fast = !is_fp64(s.prm) && s.nc[0] >= 4 && s.nc[1] >= 4 && s.nc[2] >= 4;
    t.fast = fast ? 1 : 0;
    t.half = 0;
    t.g = fast ? std::max(1, std::min(kSuperCells, (s.nc[2] - 3) / 2)) : 1;
    t.thr16 = 0;
    t.Sr = s.Sr;
    t.Snr = s.Snr;
    if (!s.gl_mem) {
        const hipError_t e = hipMalloc(&s.gl_mem, kGlTab * sizeof(double));
        if (e != hipSuccess) {
            s.gl_mem = nullptr;
            err = std::string("hipMalloc (proposal quadrature table): ") + hipGetErrorString(e);
            return RBSOG_EDEVICE;
        }
    }
    s.desc.gltab = static_cast<double *>(s.gl_mem);
    return RBSOG_OK;
}

size_t system_atom_bytes(const rbsog_params &p, int64_t n) { return atom_layout(p, n).total(); }

size_t system_device_bytes(const System &s)
{
    size_t b = s.atom_bytes + s.cell_bytes;
    if (s.half_mem)
        b += align_up(static_cast<size_t>(s.half_blocks) * 3 * s.half_hcap * sizeof(float)) +
             align_up(static_cast<size_t>(s.half_blocks) * kHrngStride * sizeof(int32_t)) + kAlign;
    if (s.gl_mem) b += kGlTab * sizeof(double);
    return b;
}

size_t system_cell_bytes(int64_t n, int64_t ncells_cap)
{
    const size_t pair_cap = static_cast<size_t>((n + kPairWave - 1) / kPairWave + ncells_cap);
    return 4 * align_up((ncells_cap + 1) * 4) + align_up(pair_cap * sizeof(int2)) + align_up(pair_cap * 8 * 8);
}

void system_carve_atoms(System &s, void *mem)
{
    const AtomLayout a = atom_layout(s.prm, s.n);
    char *p = static_cast<char *>(mem);
    SysDesc &d = s.desc;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += bytes;
        return static_cast<void *>(r);
    };
    d.q = take(a.q);
    d.u = take(a.u);
    d.cell = static_cast<int32_t *>(take(a.cell));
    d.slot = static_cast<int32_t *>(take(a.slot));
    d.keys = static_cast<uint64_t *>(take(a.keys));
    d.urec = take(a.urec);
    d.perm = static_cast<int32_t *>(take(a.perm));
    d.rec = take(a.rec);
    d.fsr = take(a.fsr);
    d.mraw = static_cast<int32_t *>(take(a.mraw));
    d.modes = static_cast<int4 *>(take(a.modes));
    d.cnt = static_cast<int32_t *>(take(a.cnt));
    d.rho_part = static_cast<double *>(take(a.rho_part));
    d.rho = static_cast<double *>(take(a.rho));
    d.pair_red = static_cast<double *>(take(a.pair_red));
    d.coef = take(a.coef);
    d.scan_tmp = static_cast<int32_t *>(take(a.scan_tmp));
    s.atom_mem = mem;
    s.atom_bytes = a.total();
}

void system_carve_cells(System &s, void *mem, int64_t ncells_cap)
{
    char *p = static_cast<char *>(mem);
    SysDesc &d = s.desc;
    const size_t cb = align_up((ncells_cap + 1) * 4);
    int32_t **arrs[] = {&d.count, &d.start, &d.nblk, &d.bstart};
    for (auto a : arrs) {
        *a = reinterpret_cast<int32_t *>(p);
        p += cb;
    }
    d.pair_cap = (s.n + kPairWave - 1) / kPairWave + ncells_cap;
    d.blocks = reinterpret_cast<int2 *>(p);
    p += align_up(d.pair_cap * sizeof(int2));
    d.pair_part = reinterpret_cast<double *>(p);
    d.ncells_cap = ncells_cap;
    s.cell_mem = mem;
    s.cell_bytes = system_cell_bytes(s.n, ncells_cap);
    s.ncells_cap = ncells_cap;
}

int system_alloc(System &s, std::string &err)
{
    void *am = nullptr;
    const size_t ab = system_atom_bytes(s.prm, s.n);
    if (hipMalloc(&am, ab) != hipSuccess) {
        (void)hipGetLastError();
        err = "device allocation failed";
        return RBSOG_ENOMEM;
    }
    s.own_mem = true;
    system_carve_atoms(s, am);
    s.ncells_cap = 0;
    return system_ensure_cells(s, err);
}

// Half-shell buffers for the current grid: partials [pair_cap][3][hcap] FP32,
// the neighbourhood table and the overflow flag, reallocated when the grid
// needs more slots or candidates per block than they hold.
static int ensure_half(System &s, std::string &err, bool *recarved)
{
    if (!s.stp.half) return RBSOG_OK;
    const int64_t blocks = s.desc.pair_cap;
    const int32_t hcap = half_hcap(s);
    if (s.half_mem && blocks <= s.half_blocks && hcap <= s.half_hcap) return RBSOG_OK;
    if (s.half_mem) {
        (void)hipFree(s.half_mem);  // synchronises the device
        s.half_mem = nullptr;
    }
    const int64_t nb = std::max(blocks, s.half_blocks);
    const int32_t hc = std::max(hcap, s.half_hcap);
    const size_t part = align_up(static_cast<size_t>(nb) * 3 * hc * sizeof(float));
    const size_t rng = align_up(static_cast<size_t>(nb) * kHrngStride * sizeof(int32_t));
    void *m = nullptr;
    if (hipMalloc(&m, part + rng + kAlign) != hipSuccess) {
        (void)hipGetLastError();
        err = "device allocation failed (half-shell partials)";
        return RBSOG_ENOMEM;
    }
    s.half_mem = m;
    s.half_blocks = nb;
    s.half_hcap = hc;
    char *p = static_cast<char *>(m);
    s.desc.hpart = reinterpret_cast<float *>(p);
    s.desc.hrng = reinterpret_cast<int32_t *>(p + part);
    s.desc.hflag = reinterpret_cast<int32_t *>(p + part + rng);
    s.desc.hcap = hc;
    if (recarved) *recarved = true;
    return RBSOG_OK;
}

int system_ensure_cells(System &s, std::string &err, bool *recarved)
{
    if (recarved) *recarved = false;
    if (s.ncells <= s.ncells_cap) return ensure_half(s, err, recarved);
    if (!s.own_mem && s.cell_mem) {
        err = "cell grid outgrew the memory reserved at admission";
        return RBSOG_EBOX;
    }
    if (s.cell_mem) {
        (void)hipFree(s.cell_mem);  // synchronises the device
        s.cell_mem = nullptr;
    }
    void *cm = nullptr;
    if (hipMalloc(&cm, system_cell_bytes(s.n, s.ncells)) != hipSuccess) {
        (void)hipGetLastError();
        err = "device allocation failed";
        return RBSOG_ENOMEM;
    }
    system_carve_cells(s, cm, s.ncells);
    if (recarved) *recarved = true;
    return ensure_half(s, err, recarved);
}

void system_free(System &s)
{
    if (s.own_mem) {
        if (s.atom_mem) (void)hipFree(s.atom_mem);
        if (s.cell_mem) (void)hipFree(s.cell_mem);
    }
    if (s.half_mem) (void)hipFree(s.half_mem);
    if (s.gl_mem) (void)hipFree(s.gl_mem);
    s.atom_mem = s.cell_mem = s.half_mem = s.gl_mem = nullptr;
}

int system_upload_q(System &s, const double *host_q, hipStream_t stream, std::string &err,
                    std::vector<float> *stage)
{
    const int64_t n = s.n;
    hipError_t e;
    if (is_fp64(s.prm)) {
        e = hipMemcpyAsync(const_cast<void *>(s.desc.q), host_q, n * sizeof(double), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && !stage) e = hipStreamSynchronize(stream);
    } else {
        std::vector<float> q32;
        std::vector<float> &buf = stage ? *stage : q32;
        buf.resize(n);
        for (int64_t i = 0; i < n; ++i) buf[i] = static_cast<float>(host_q[i]);
        e = hipMemcpyAsync(const_cast<void *>(s.desc.q), buf.data(), n * sizeof(float), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && !stage) e = hipStreamSynchronize(stream);  // q32 leaves scope
    }
    if (e != hipSuccess) {
        err = std::string("charge upload: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    return RBSOG_OK;
}

// ---------------------------------------------------------------------------
// Batches

int batch_init(Batch &b, hipStream_t stream, int precision, std::string &err)
{
    b.stream = stream;
    b.precision = precision;
    if (hipGetDevice(&b.device) != hipSuccess) {
        err = "no HIP device";
        return RBSOG_EDEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b.device) == hipSuccess && ncu > 0)
        b.num_cu = ncu;
    bool ok = hipMalloc(&b.d_ctrl, 64) == hipSuccess &&
              hipEventCreateWithFlags(&b.up_done, hipEventDisableTiming) == hipSuccess &&
              hipStreamCreateWithFlags(&b.aux, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&b.ev_up, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b.ev_bin, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b.ev_sk, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < Batch::kStepRing; ++k)
        ok = hipEventCreateWithFlags(&b.step_ev[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        err = "device allocation failed";
        return RBSOG_ENOMEM;
    }
    return RBSOG_OK;
}

static void free_timers(Batch &b)
{
    for (auto &t : b.timers) {
        for (auto &e : t.pending) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        for (auto &e : t.pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
    b.timers.clear();
}

void batch_free(Batch &b)
{
    if (b.graph_exec) (void)hipGraphExecDestroy(b.graph_exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.graph_exec = nullptr;
    b.graph = nullptr;
    void *dev[] = {b.d_desc, b.d_step, b.d_res, b.d_plan, b.d_ctrl};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    void *host[] = {b.h_desc, b.h_res, b.h_plan};
    for (void *p : host)
        if (p) (void)hipHostFree(p);
    for (int k = 0; k < Batch::kStepRing; ++k) {
        if (b.h_step[k]) (void)hipHostFree(b.h_step[k]);
        if (b.step_ev[k]) (void)hipEventDestroy(b.step_ev[k]);
        b.h_step[k] = nullptr;
        b.step_ev[k] = nullptr;
    }
    if (b.up_done) (void)hipEventDestroy(b.up_done);
    if (b.aux) {
        (void)hipStreamSynchronize(b.aux);
        (void)hipStreamDestroy(b.aux);
    }
    hipEvent_t evs[] = {b.ev_up, b.ev_bin, b.ev_sk};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    b.aux = nullptr;
    b.ev_up = b.ev_bin = b.ev_sk = nullptr;
    b.d_desc = nullptr;
    b.d_step = nullptr;
    b.step_last.clear();
    b.d_res = nullptr;
    b.d_plan = nullptr;
    b.d_ctrl = nullptr;
    b.h_desc = nullptr;
    b.h_res = nullptr;
    b.h_plan = nullptr;
    b.up_done = nullptr;
    free_timers(b);
}

// the pinned mirrors may be rewritten only after the last upload has run
static int wait_uploads(Batch &b, std::string &err)
{
    if (!b.up_pending) return RBSOG_OK;
    const hipError_t e = hipEventSynchronize(b.up_done);
    if (e != hipSuccess) {
        err = std::string("upload wait: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    b.up_pending = false;
    return RBSOG_OK;
}

int batch_set_systems(Batch &b, const std::vector<System *> &sys, std::string &err)
{
    int rc = wait_uploads(b, err);
    if (rc) return rc;
    const int64_t S = static_cast<int64_t>(sys.size());
    if (S > b.cap_sys) {
        // the old buffers may still be read by queued work
        if (hipStreamSynchronize(b.stream) != hipSuccess) {
            err = "stream synchronisation failed";
            return RBSOG_EDEVICE;
        }
        const int64_t cap = std::max<int64_t>(S, 2 * b.cap_sys);
        if (b.d_desc) (void)hipFree(b.d_desc);
        if (b.d_step) (void)hipFree(b.d_step);
        if (b.d_res) (void)hipFree(b.d_res);
        if (b.h_desc) (void)hipHostFree(b.h_desc);
        if (b.h_res) (void)hipHostFree(b.h_res);
        for (int k = 0; k < Batch::kStepRing; ++k) {
            if (b.h_step[k]) (void)hipHostFree(b.h_step[k]);
            b.h_step[k] = nullptr;
            b.step_ev_used[k] = false;
        }
        b.d_desc = nullptr;
        b.d_step = nullptr;
        b.step_last.clear();
        b.d_res = nullptr;
        b.h_desc = nullptr;
        b.h_res = nullptr;
        b.cap_sys = 0;
        bool ok = hipMalloc(&b.d_desc, cap * sizeof(SysDesc)) == hipSuccess &&
                  hipMalloc(&b.d_step, cap * sizeof(SysStep)) == hipSuccess &&
                  hipMalloc(&b.d_res, cap * sizeof(StepResults)) == hipSuccess &&
                  hipHostMalloc(reinterpret_cast<void **>(&b.h_desc), cap * sizeof(SysDesc)) == hipSuccess &&
                  hipHostMalloc(reinterpret_cast<void **>(&b.h_res), cap * sizeof(StepResults)) == hipSuccess;
        for (int k = 0; ok && k < Batch::kStepRing; ++k)
            ok = hipHostMalloc(reinterpret_cast<void **>(&b.h_step[k]), cap * sizeof(SysStep)) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            err = "batch allocation failed";
            return RBSOG_ENOMEM;
        }
        b.cap_sys = cap;
    }
    b.sys = sys;
    b.desc_dirty = true;
    b.plan_dirty = true;
    return RBSOG_OK;
}

static std::vector<int64_t> plan_sizes(const Batch &b)
{
    std::vector<int64_t> k;
    k.reserve(3 * b.sys.size());
    for (const System *s : b.sys) {
        k.push_back(s->n);
        k.push_back(s->ncells);
        k.push_back(s->prm.P);
        k.push_back(s->pair_form);
        k.push_back(s->stp.fast);
        k.push_back(s->stp.half);
        k.push_back(s->stp.tri);
    }
    return k;
}

// Ordering workgroups of a system: one per cell; a single-cell system (the
// whole box within reach) splits its one cell into parts of kOrderPart keys.
static int64_t order_parts(const System &s)
{
    return s.ncells == 1 ? (s.n + kOrderPart - 1) / kOrderPart : s.ncells;
}

static int build_plans(Batch &b, std::string &err)
{
    int64_t len[kNumPlans] = {};
    for (const System *s : b.sys) {
        len[kPlanAtoms] += (s->n + kAtomBlock - 1) / kAtomBlock;
        len[kPlanCells] += (s->ncells + 1 + kCellBlock - 1) / kCellBlock;
        len[kPlanScan] += (s->ncells + kScanBlock - 1) / kScanBlock;
        len[kPlanPair] += (s->n + kPairWave - 1) / kPairWave + s->ncells;
        len[kPlanSk] += (s->n + kSkChunk - 1) / kSkChunk;
        len[kPlanReduce] += mode_cap(s->prm) + kPairRed;
        len[kPlanCell1] += order_parts(*s);
    }
    int64_t total = 0;
    for (int k = 0; k < kNumPlans; ++k) {
        b.plan_off[k] = total;
        b.plan_len[k] = len[k];
        total += len[k];
    }
    if (total > INT32_MAX) {
        err = "batch too large for one launch";
        return RBSOG_EINVAL;
    }
    if (total > b.cap_plan) {
        const int64_t cap = std::max<int64_t>(total, 2 * b.cap_plan);
        // a step still queued (a queued context step, a pipelined served
        // tick) may read the old plans: let both streams drain first
        (void)hipStreamSynchronize(b.aux);
        (void)hipStreamSynchronize(b.stream);
        if (b.d_plan) (void)hipFree(b.d_plan);
        if (b.h_plan) (void)hipHostFree(b.h_plan);
        b.d_plan = nullptr;
        b.h_plan = nullptr;
        b.cap_plan = 0;
        if (hipMalloc(&b.d_plan, cap * sizeof(int2)) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&b.h_plan), cap * sizeof(int2)) != hipSuccess) {
            (void)hipGetLastError();
            err = "plan allocation failed";
            return RBSOG_ENOMEM;
        }
        b.cap_plan = cap;
    }
    int64_t pos[kNumPlans];
    for (int k = 0; k < kNumPlans; ++k) pos[k] = b.plan_off[k];
    auto put = [&](PlanKind k, int s, int64_t nblocks) {
        for (int64_t i = 0; i < nblocks; ++i) b.h_plan[pos[k]++] = make_int2(s, static_cast<int>(i));
    };
    const int S = static_cast<int>(b.sys.size());
    for (int s = 0; s < S; ++s) {
        const System *y = b.sys[s];
        put(kPlanAtoms, s, (y->n + kAtomBlock - 1) / kAtomBlock);
        put(kPlanCells, s, (y->ncells + 1 + kCellBlock - 1) / kCellBlock);
        put(kPlanScan, s, (y->ncells + kScanBlock - 1) / kScanBlock);
        put(kPlanSk, s, (y->n + kSkChunk - 1) / kSkChunk);
        put(kPlanReduce, s, mode_cap(y->prm) + kPairRed);
        put(kPlanCell1, s, order_parts(*y));
    }
    // pair blocks grouped by the form of the SOG kernels and the filter path
    // (one launch per group, each compiled for its path alone)
    for (int g = 0; g < kNumPairGroups; ++g) {
        b.pair_split[g] = pos[kPlanPair] - b.plan_off[kPlanPair];
        for (int s = 0; s < S; ++s) {
            const System *y = b.sys[s];
            const int path = y->stp.tri ? 3 : (y->stp.half ? 2 : (y->stp.fast ? 1 : 0));
            if (kNumPaths * y->pair_form + path == g)
                put(kPlanPair, s, (y->n + kPairWave - 1) / kPairWave + y->ncells);
        }
    }
    b.pair_split[kNumPairGroups] = pos[kPlanPair] - b.plan_off[kPlanPair];
    return RBSOG_OK;
}

bool batch_upload_allocates(const Batch &b)
{
    if (static_cast<int64_t>(b.sys.size()) > b.cap_sys) return true;
    if (!b.plan_dirty && plan_sizes(b) == b.plan_key) return false;
    int64_t total = 0;
    for (const System *s : b.sys) {
        total += (s->n + kAtomBlock - 1) / kAtomBlock + (s->ncells + 1 + kCellBlock - 1) / kCellBlock +
                 (s->ncells + kScanBlock - 1) / kScanBlock + (s->n + kPairWave - 1) / kPairWave + s->ncells +
                 (s->n + kSkChunk - 1) / kSkChunk + mode_cap(s->prm) + kPairRed + order_parts(*s);
    }
    return total > b.cap_plan;
}

int batch_upload(Batch &b, std::string &err)
{
    if (b.sys.empty()) return RBSOG_OK;
    const int64_t S = static_cast<int64_t>(b.sys.size());
    const std::vector<int64_t> key = plan_sizes(b);
    const bool plans = b.plan_dirty || key != b.plan_key;
    // the pinned descriptor and plan buffers are rewritten only once the copies
    // that last read them have run; a step that rewrites neither does not wait
    int rc = RBSOG_OK;
    if (b.desc_dirty || plans) rc = wait_uploads(b, err);
    if (rc) return rc;
    hipError_t e = hipSuccess;
    bool queued = false;
    if (b.desc_dirty) {
        for (int64_t s = 0; s < S; ++s) {
            b.h_desc[s] = b.sys[s]->desc;
            b.h_desc[s].res = b.d_res + s;
        }
        e = hipMemcpyAsync(b.d_desc, b.h_desc, S * sizeof(SysDesc), hipMemcpyHostToDevice, b.stream);
        b.desc_dirty = false;
        queued = true;
    }
    if (e == hipSuccess && plans) {
        rc = build_plans(b, err);
        if (rc) return rc;
        int64_t total = 0;
        for (int k = 0; k < kNumPlans; ++k) total += b.plan_len[k];
        e = hipMemcpyAsync(b.d_plan, b.h_plan, total * sizeof(int2), hipMemcpyHostToDevice, b.stream);
        b.plan_key = key;
        b.plan_dirty = false;
        queued = true;
    }
    if (e == hipSuccess && queued) {
        e = hipEventRecord(b.up_done, b.stream);
        b.up_pending = true;
    }
    // per-step data: the next pinned buffer of the ring, reused once the copy
    // that last read it has run; nothing when the device already holds it
    bool step_same = e == hipSuccess && b.step_last.size() == static_cast<size_t>(S);
    for (int64_t s = 0; step_same && s < S; ++s)
        step_same = std::memcmp(&b.step_last[s], &b.sys[s]->stp, sizeof(SysStep)) == 0;
    if (e == hipSuccess && !step_same) {
        const int k = b.step_slot;
        b.step_slot = (k + 1) % Batch::kStepRing;
        if (b.step_ev_used[k]) e = hipEventSynchronize(b.step_ev[k]);
        if (e == hipSuccess) {
            for (int64_t s = 0; s < S; ++s) b.h_step[k][s] = b.sys[s]->stp;
            e = hipMemcpyAsync(b.d_step, b.h_step[k], S * sizeof(SysStep), hipMemcpyHostToDevice, b.stream);
        }
        if (e == hipSuccess) e = hipEventRecord(b.step_ev[k], b.stream);
        b.step_ev_used[k] = true;
        b.step_last.resize(S);
        for (int64_t s = 0; s < S; ++s) b.step_last[s] = b.sys[s]->stp;
    }
    if (e != hipSuccess) {
        err = std::string("batch upload: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    return RBSOG_OK;
}

int batch_fetch_results(Batch &b, std::string &err)
{
    if (b.sys.empty()) return RBSOG_OK;
    // work on the second stream (a sampler not yet joined) finishes first
    hipError_t e = hipStreamSynchronize(b.aux);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.h_res, b.d_res, b.sys.size() * sizeof(StepResults), hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) {
        err = std::string("result copy: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    b.up_pending = false;
    return RBSOG_OK;
}

static bool timed(const Batch &b, const char *name)
{
    return b.timing == 1 || (b.timing == 2 && std::strcmp(name, "pair") == 0);
}

void timer_begin(Batch &b, const char *name, hipStream_t stream)
{
    if (!timed(b, name)) return;
    Timer *t = nullptr;
    for (auto &x : b.timers)
        if (x.name == name) t = &x;
    if (!t) {
        if (b.timers.size() >= static_cast<size_t>(kMaxTimed)) return;
        b.timers.push_back(Timer{});
        t = &b.timers.back();
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
    (void)hipEventRecord(ev.first, stream);
    t->pending.push_back(ev);
}

void timer_end(Batch &b, const char *name, hipStream_t stream)
{
    if (!timed(b, name)) return;
    for (auto &x : b.timers)
        if (x.name == name && !x.pending.empty()) {
            (void)hipEventRecord(x.pending.back().second, stream);
            return;
        }
}

void batch_set_timing(Batch &b, int level)
{
    (void)hipStreamSynchronize(b.aux);
    (void)hipStreamSynchronize(b.stream);
    free_timers(b);
    b.timing = level == 1 || level == 2 ? level : 0;
}

int batch_get_timing(Batch &b, int32_t cap, int32_t *host_nk, char *host_names, double *host_ms,
                     int64_t *host_count, std::string &err)
{
    hipError_t e = hipStreamSynchronize(b.aux);
    if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) {
        err = std::string("timing: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    for (auto &t : b.timers) {
        for (auto &ev : t.pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) {
                t.ms += ms;
                t.count += 1;
            }
            t.pool.push_back(ev);
        }
        t.pending.clear();
    }
    const int nk = static_cast<int>(b.timers.size());
    if (host_nk) *host_nk = nk;
    for (int k = 0; k < std::min(nk, static_cast<int>(cap)); ++k) {
        if (host_names) {
            std::memset(host_names + 32 * k, 0, 32);
            std::strncpy(host_names + 32 * k, b.timers[k].name.c_str(), 31);
        }
        if (host_ms) host_ms[k] = b.timers[k].ms;
        if (host_count) host_count[k] = b.timers[k].count;
    }
    return RBSOG_OK;
}

}  // namespace rbsog
