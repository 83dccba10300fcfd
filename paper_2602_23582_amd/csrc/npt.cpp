// NPT integration around the force and pressure evaluation (Algorithm 1 step
// 7): the Langevin equations of eq. Langevin_NPT for a diagonal h, advanced by
// the symmetric splitting B_h B A O A [evaluate] B B_h declared in rbsog.h.
// Particle updates run on the device in FP64; the box degrees of freedom are a
// few doubles advanced on the host in FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "rbsog_impl.hpp"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

int fail(rbsog_ctx *c, int code, const char *msg)
{
    c->err = msg;
    return code;
}

#define NPT_HIP(c, call)                                                  \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) {                                           \
            (c)->err = std::string(#call) + ": " + hipGetErrorString(e_); \
            return RBSOG_EDEVICE;                                         \
        }                                                                 \
    } while (0)

#define NPT_TRY(call)                 \
    do {                              \
        int r_ = (call);              \
        if (r_ != RBSOG_OK) return r_; \
    } while (0)

// Philox4x32-10 (Salmon et al., SC'11) on the host: the box noise
void philox(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c[0];
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c[2];
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = static_cast<uint32_t>(p1);
        c[2] = n2;
        c[3] = static_cast<uint32_t>(p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

double unit_open(uint32_t hi, uint32_t lo)
{
    const uint64_t w = (static_cast<uint64_t>(hi) << 32) | lo;
    return (static_cast<double>(w >> 12) + 0.5) * 0x1.0p-52;
}

// three standard normals for the box at this step: Box-Muller of the draws
// (0, 18, step, sys) and (1, 18, step, sys)
void box_normals(uint64_t seed, uint32_t step, uint32_t sys, double z[3])
{
    uint32_t a[4] = {0u, 18u, step, sys}, b[4] = {1u, 18u, step, sys};
    philox(a, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    philox(b, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const double u1 = unit_open(a[0], a[1]), u2 = unit_open(a[2], a[3]);
    const double u3 = unit_open(b[0], b[1]), u4 = unit_open(b[2], b[3]);
    const double r1 = std::sqrt(-2.0 * std::log(u1)), r2 = std::sqrt(-2.0 * std::log(u3));
    z[0] = r1 * std::cos(kTwoPi * u2);
    z[1] = r1 * std::sin(kTwoPi * u2);
    z[2] = r2 * std::cos(kTwoPi * u4);
}

// Box degrees of freedom: group g of each axis, and the axes of each group.
struct Groups {
    int ng = 3;
    int of[3] = {0, 1, 2};
    int size[3] = {1, 1, 1};
};

Groups groups_for(int coupling)
{
    Groups g;
    if (coupling == RBSOG_COUPLE_SEMI) {
        g.ng = 2;
        g.of[0] = g.of[1] = 0;
        g.of[2] = 1;
        g.size[0] = 2;
        g.size[1] = 1;
    } else if (coupling == RBSOG_COUPLE_ISO) {
        g.ng = 1;
        g.of[0] = g.of[1] = g.of[2] = 0;
        g.size[0] = 3;
    }
    return g;
}

struct BoxState {
    double L[3];
    double ph[3];  // per group
};

// B_h: p^h_g += t [(V/L_g) sum_{mu in g} (P_mumu - p_ext) - n_g kT / L_g]
void kick_box(const rbsog_npt_params &p, const Groups &g, BoxState &b, const double P[9], double t)
{
    const double V = b.L[0] * b.L[1] * b.L[2];
    double drive[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) drive[g.of[d]] += P[4 * d] - p.p_ext;
    for (int k = 0; k < g.ng; ++k) {
        int d0 = 0;
        while (g.of[d0] != k) ++d0;
        const double Lg = b.L[d0];
        b.ph[k] += t * ((V / Lg) * drive[k] - g.size[k] * p.kT / Lg);
    }
}

}  // namespace

extern "C" {

int rbsog_npt_init(rbsog_ctx *c, const rbsog_npt_params *prm, const double *host_mass)
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (!prm || !host_mass) return fail(c, RBSOG_EINVAL, "null argument");
    const rbsog_npt_params &p = *prm;
    const bool ok = std::isfinite(p.dt) && p.dt > 0 && std::isfinite(p.kT) && p.kT >= 0 && std::isfinite(p.gamma) &&
                    p.gamma >= 0 && std::isfinite(p.gamma_box) && p.gamma_box >= 0 && std::isfinite(p.box_mass) &&
                    p.box_mass > 0 && std::isfinite(p.p_ext) &&
                    (p.coupling == RBSOG_COUPLE_ANISO || p.coupling == RBSOG_COUPLE_SEMI ||
                     p.coupling == RBSOG_COUPLE_ISO);
    if (!ok) return fail(c, RBSOG_EINVAL, "bad NPT parameters");
    const int64_t n = c->sys.n;
    for (int64_t i = 0; i < n; ++i)
        if (!(host_mass[i] > 0) || !std::isfinite(host_mass[i])) return fail(c, RBSOG_EINVAL, "masses must be > 0");
    rbsog::NptState &s = c->npt;
    const int64_t nb = (n + rbsog::kNptBlock - 1) / rbsog::kNptBlock;
    if (!s.d_mass) {
        NPT_HIP(c, hipMalloc(&s.d_mass, n * sizeof(double)));
        NPT_HIP(c, hipMalloc(&s.d_F, 3 * n * sizeof(double)));
        NPT_HIP(c, hipMalloc(&s.d_part, 6 * nb * sizeof(double)));
        NPT_HIP(c, hipMalloc(&s.d_kin, 6 * sizeof(double)));
    }
    s.kin_blocks = nb;
    NPT_HIP(c, hipMemcpyAsync(s.d_mass, host_mass, n * sizeof(double), hipMemcpyHostToDevice, c->batch.stream));
    NPT_HIP(c, hipStreamSynchronize(c->batch.stream));
    s.prm = p;
    s.ready = true;
    return RBSOG_OK;
}

}  // extern "C"

namespace {

bool is_device(const void *p)
{
    hipPointerAttribute_t a;
    if (!p || hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// forces (into the integrator's buffer) and Coulomb pressure at the state
int evaluate(rbsog_ctx *c, const double *x, const double *y, const double *z, const double L[3], int64_t step,
             double P[9])
{
    const int64_t n = c->sys.n;
    double *F = c->npt.d_F;
    // sampling, forces and pressure in one call (no rescale: x, y, z are only read)
    double box[3] = {L[0], L[1], L[2]};
    return rbsog_step(c, step, nullptr, box, const_cast<double *>(x), const_cast<double *>(y), const_cast<double *>(z),
                      F, F + n, F + 2 * n, P, nullptr);
}

// kinetic tensor sum p p^T / m (row-major 3x3)
int kinetic(rbsog_ctx *c, const double *px, const double *py, const double *pz, double K[9])
{
    rbsog::NptState &s = c->npt;
    NPT_HIP(c, rbsog::launch_npt_kinetic(c->batch.stream, c->sys.n, s.d_mass, px, py, pz, s.d_part, s.kin_blocks,
                                         s.d_kin));
    double k6[6];
    NPT_HIP(c, hipMemcpyAsync(k6, s.d_kin, sizeof(k6), hipMemcpyDeviceToHost, c->batch.stream));
    NPT_HIP(c, hipStreamSynchronize(c->batch.stream));
    const double v[9] = {k6[0], k6[3], k6[4], k6[3], k6[1], k6[5], k6[4], k6[5], k6[2]};
    std::memcpy(K, v, sizeof(v));
    return RBSOG_OK;
}

// A over t: the box lengths move linearly (p^h fixed); the exact flow of the
// particles is then r <- a r + t p/m, p <- p/a with a = L_new/L_old per axis
int drift(rbsog_ctx *c, const Groups &g, BoxState &b, double t, double *x, double *y, double *z, double *px,
          double *py, double *pz)
{
    const rbsog_npt_params &p = c->npt.prm;
    double a[3], bb[3];
    for (int d = 0; d < 3; ++d) {
        const int k = g.of[d];
        const double Lnew = b.L[d] + t * b.ph[k] / (g.size[k] * p.box_mass);
        if (!(Lnew > 0) || !std::isfinite(Lnew)) return fail(c, RBSOG_EBOX, "box collapsed");
        a[d] = Lnew / b.L[d];
        bb[d] = t;
        b.L[d] = Lnew;
    }
    NPT_HIP(c, rbsog::launch_npt_drift(c->batch.stream, c->sys.n, a, bb, c->npt.d_mass, x, y, z, px, py, pz));
    return RBSOG_OK;
}

}  // namespace

extern "C" {

int rbsog_npt_run(rbsog_ctx *c, double *x, double *y, double *z, double *px, double *py, double *pz,
                  int64_t first_step, int32_t nsteps, double host_box[3], double host_pbox[3], double host_P_ins[9],
                  double host_P_kin[9])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (!c->npt.ready) return fail(c, RBSOG_ESTATE, "rbsog_npt_init must precede rbsog_npt_run");
    if (!x || !y || !z || !px || !py || !pz || !host_box || !host_pbox) return fail(c, RBSOG_EINVAL, "null argument");
    if (nsteps < 0 || first_step < 0 || ((first_step + nsteps) >> 32)) return fail(c, RBSOG_EINVAL, "bad step range");
    for (const void *q : {(const void *)x, (const void *)y, (const void *)z, (const void *)px, (const void *)py,
                          (const void *)pz})
        if (!is_device(q)) return fail(c, RBSOG_EINVAL, "rbsog_npt_run needs device position and momentum arrays");
    const rbsog_npt_params &p = c->npt.prm;
    const Groups g = groups_for(p.coupling);
    BoxState b;
    for (int d = 0; d < 3; ++d) {
        if (!(host_box[d] > 0) || !std::isfinite(host_box[d]) || !std::isfinite(host_pbox[d]))
            return fail(c, RBSOG_EINVAL, "bad box or box momentum");
        b.L[d] = host_box[d];
    }
    for (int d = 0; d < 3; ++d)
        if (b.L[d] != b.L[0] && g.of[d] == g.of[0]) return fail(c, RBSOG_EINVAL, "coupled axes need equal lengths");
    if (p.coupling == RBSOG_COUPLE_SEMI && host_pbox[0] != host_pbox[1])
        return fail(c, RBSOG_EINVAL, "coupled axes need equal box momenta");
    if (p.coupling == RBSOG_COUPLE_ISO && (host_pbox[0] != host_pbox[1] || host_pbox[0] != host_pbox[2]))
        return fail(c, RBSOG_EINVAL, "coupled axes need equal box momenta");
    for (int d = 0; d < 3; ++d) b.ph[g.of[d]] = host_pbox[d];

    const int64_t n = c->sys.n;
    const double *F = c->npt.d_F;
    hipStream_t st = c->batch.stream;
    const double h = 0.5 * p.dt;
    const double c1 = std::exp(-p.gamma * p.dt), c1h = std::exp(-p.gamma_box * p.dt);
    const double sc = std::sqrt((1.0 - c1 * c1) * p.kT);
    const uint32_t sys = static_cast<uint32_t>(c->sys.prm.system_id);
    const uint64_t seed = c->sys.prm.seed;

    double PU[9], K[9], P[9];
    auto pins = [&]() {
        const double V = b.L[0] * b.L[1] * b.L[2];
        for (int k = 0; k < 9; ++k) P[k] = PU[k] + K[k] / V;
    };
    NPT_TRY(evaluate(c, x, y, z, b.L, first_step, PU));
    NPT_TRY(kinetic(c, px, py, pz, K));
    pins();
    for (int32_t s = 1; s <= nsteps; ++s) {
        const uint32_t step = static_cast<uint32_t>(first_step + s);
        kick_box(p, g, b, P, h);                                            // B_h
        NPT_HIP(c, rbsog::launch_npt_kick(st, n, h, F, px, py, pz));         // B
        NPT_TRY(drift(c, g, b, h, x, y, z, px, py, pz));                      // A
        NPT_HIP(c, rbsog::launch_npt_ou(st, n, c1, sc, c->npt.d_mass, px, py, pz, seed, step, sys));  // O
        double zb[3];
        box_normals(seed, step, sys, zb);
        for (int k = 0; k < g.ng; ++k)
            b.ph[k] = c1h * b.ph[k] + std::sqrt((1.0 - c1h * c1h) * p.kT * g.size[k] * p.box_mass) * zb[k];
        NPT_TRY(drift(c, g, b, h, x, y, z, px, py, pz));                      // A
        NPT_TRY(evaluate(c, x, y, z, b.L, static_cast<int64_t>(step), PU));  // F, P at the new state
        NPT_HIP(c, rbsog::launch_npt_kick(st, n, h, F, px, py, pz));         // B
        NPT_TRY(kinetic(c, px, py, pz, K));
        pins();
        kick_box(p, g, b, P, h);                                            // B_h
    }
    for (int d = 0; d < 3; ++d) {
        host_box[d] = b.L[d];
        host_pbox[d] = b.ph[g.of[d]];
    }
    if (host_P_ins) std::memcpy(host_P_ins, P, sizeof(P));
    if (host_P_kin) {
        const double V = b.L[0] * b.L[1] * b.L[2];
        for (int k = 0; k < 9; ++k) host_P_kin[k] = K[k] / V;
    }
    return RBSOG_OK;
}

}  // extern "C"
