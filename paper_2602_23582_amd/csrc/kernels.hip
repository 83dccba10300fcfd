// HIP kernels of the RBSOG library for gfx950 (CDNA4, wave64).
//
// One force/pressure evaluation (Algorithm 1, steps 2-6) of a batch of
// systems runs as
//   k_sampler                       - both MH chains and the distinct-mode set (one workgroup per system, FP64)
//   k_zero, k_fix, k_scan_*, k_scatter, k_order
//                                   - fixed-point fractional coordinates, cell binning, stable sort
//   k_pair                          - short-range SOG force, virial and energy over cell lists
//   k_sk                            - structure factors of the distinct modes (per-block partials)
//   k_rho_reduce, k_estimators      - FP64 combine, estimator coefficients, pressure and energy
//   k_force                         - long-range force scatter, total force in the caller's order
// Each workgroup reads its (system, block) from a launch plan and touches only
// that system's buffers.  Every reduction runs over one system's partials in
// a fixed order, so results are bitwise reproducible and do not depend on the
// other systems of the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <type_traits>

#include "rbsog_impl.hpp"

namespace rbsog {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// ----------------------------------------------------------------------------
// Precision forms
// ----------------------------------------------------------------------------

// FP32C: 32-bit fixed-point fractional coordinates (exact minimum image and
// exact integer phases), FP32 arithmetic, FP64 partial sums.
struct F32 {
    using real = float;
    using fix = uint32_t;
    using sfix = int32_t;
    struct alignas(16) Rec {
        uint32_t x, y, z;
        float q;
    };
};

// FP64: 64-bit fixed point, double arithmetic throughout.
struct F64 {
    using real = double;
    using fix = uint64_t;
    using sfix = int64_t;
    struct alignas(16) Rec {
        uint64_t x, y, z;
        double q;
    };
};

// per-mode data for the force scatter: integer mode, wave vector, A = a Im rho,
// B = a Re rho with a = (S/(P V)) c^r / |k|^2
template <class real>
struct alignas(16) Coef {
    int32_t mx, my, mz, pad;
    real kx, ky, kz, A, B;
};

// Buffer pointers read from a descriptor are generic pointers; accesses made
// through gp() and gload() are issued as global-memory instructions, and a
// load whose address is the same for the whole wavefront becomes a scalar load.
#define RB_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ RB_GLOBAL T *gp(T *p)
{
    return (RB_GLOBAL T *)(p);
}
template <class T>
__device__ __forceinline__ const RB_GLOBAL T *gp(const T *p)
{
    return (const RB_GLOBAL T *)(p);
}
// load of a struct (HIP vector types, records) as whole dwords
template <class T>
__device__ __forceinline__ T gload(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "dword multiple");
    T out;
    const RB_GLOBAL uint32_t *src = (const RB_GLOBAL uint32_t *)(p);
    uint32_t *dst = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (int k = 0; k < static_cast<int>(sizeof(T) / 4); ++k) dst[k] = src[k];
    return out;
}
template <class T>
__device__ __forceinline__ void gstore(T *p, const T &v)
{
    static_assert(sizeof(T) % 4 == 0, "dword multiple");
    RB_GLOBAL uint32_t *dst = (RB_GLOBAL uint32_t *)(p);
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&v);
#pragma unroll
    for (int k = 0; k < static_cast<int>(sizeof(T) / 4); ++k) dst[k] = src[k];
}

__device__ inline float fix_to_real(int32_t v, float scale) { return static_cast<float>(v) * scale; }
__device__ inline double fix_to_real(int64_t v, double scale) { return static_cast<double>(v) * scale; }

template <class T>
__device__ inline T wave_sum(T v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// wave-wide minimum and maximum, returned as wave-uniform (scalar) values
__device__ inline float wave_min_uniform(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ inline float wave_max_uniform(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the sampler's draws
// ----------------------------------------------------------------------------

__device__ inline uint4 philox4x32_10(uint4 c, uint2 k)
{
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// (0,1) uniform from the top 52 bits of a 64-bit word
__device__ inline double unit_open(uint32_t hi, uint32_t lo)
{
    const uint64_t w = (static_cast<uint64_t>(hi) << 32) | lo;
    return (static_cast<double>(w >> 12) + 0.5) * 0x1.0p-52;
}

struct SampArgs {
    double L[3];
    int tri;              // general cell: h, h^-1 and the quadrature table below
    double h[9], hi[9], V;
    const double *gltab;  // [2][kGl^3]: w_i w_j w_k exp(-pi^2 s^2 d^T C d) for s = s_0 and s_0/sqrt2
    double B[2];       // bounds of g_2/q' and g_4/q' (exact start draws)
    int P, M, variant, mcap;
    uint32_t key0, key1, step, sys;
    const SogTables *tab;
    int32_t *mraw;     // m_r (P x 3) then m_nr (P x 3)
    int4 *modes;       // distinct modes
    int32_t *cnt;      // [mcap] r multiplicities, then [mcap] nr
    StepResults *res;  // nd, status, acceptance counts
};

__device__ void draw_normals(const SampArgs &a, uint32_t t, uint32_t sxy, uint32_t sz, double z[3])
{
#pragma clang fp contract(off)
    const uint2 key = make_uint2(a.key0, a.key1);
    const uint4 o1 = philox4x32_10(make_uint4(t, sxy, a.step, a.sys), key);
    const uint4 o2 = philox4x32_10(make_uint4(t, sz, a.step, a.sys), key);
    const double u1 = unit_open(o1.x, o1.y), u2 = unit_open(o1.z, o1.w);
    const double u3 = unit_open(o2.x, o2.y), u4 = unit_open(o2.z, o2.w);
    const double r1 = sqrt(-2.0 * log(u1));
    const double r2 = sqrt(-2.0 * log(u3));
    z[0] = r1 * cos(2.0 * kPi * u2);
    z[1] = r1 * sin(2.0 * kPi * u2);
    z[2] = r2 * cos(2.0 * kPi * u4);
}

// The independent non-radial chain's proposal is the radial one with s0
// scaled by this factor (sqrt(2) wider): its weight P^nr/q then stays bounded
// where P^nr decays like |k|^4 exp(-s0^2 |k|^2/4).
constexpr double kNrWiden = 0.70710678118654752440;

// App. D: m*_xi = round(h^T u) with u_xi ~ N(0, 1/(2 pi^2 s0^2)), i.e. round(sig_xi z_xi)
__device__ void round_proposal(const SampArgs &a, const double z[3], int m[3], double widen = 1.0)
{
#pragma clang fp contract(off)
    const double s0 = a.tab->s[0] * widen;
    if (a.tri) {
        // (h^T u)_i = sum_j h_ji u_j, u = z / (sqrt2 pi s0)
        const double c = 1.0 / (sqrt(2.0) * kPi * s0);
        for (int i = 0; i < 3; ++i) {
            double v = round(c * (a.h[i] * z[0] + a.h[3 + i] * z[1] + a.h[6 + i] * z[2]));
            v = fmin(fmax(v, -1073741824.0), 1073741824.0);
            m[i] = static_cast<int>(v);
        }
        return;
    }
    for (int d = 0; d < 3; ++d) {
        const double sig = a.L[d] / (sqrt(2.0) * kPi * s0);
        double v = round(sig * z[d]);
        v = fmin(fmax(v, -1073741824.0), 1073741824.0);
        m[d] = static_cast<int>(v);
    }
}

// importance weight w = P^r(m)/q(m) (unnormalised, 0 at m = 0) and the
// recalibration ratio R = P^nr(m)/P^r(m) (unnormalised); with wnr, also the
// non-radial weight P^nr(m)/q'(m), q' the widened proposal, and with wrw the
// radial one P^r(m)/q'(m)
__device__ void mode_weights(const SampArgs &a, const int m[3], double *w, double *R, double *wnr = nullptr,
                             double *wrw = nullptr)
{
#pragma clang fp contract(off)
    if (m[0] == 0 && m[1] == 0 && m[2] == 0) {
        *w = 0.0;
        *R = 0.0;
        if (wnr) *wnr = 0.0;
        if (wrw) *wrw = 0.0;
        return;
    }
    double k2 = 0.0;
    if (a.tri) {
        // k = 2 pi h^-T m
        for (int i = 0; i < 3; ++i) {
            const double k = 2.0 * kPi * (a.hi[i] * m[0] + a.hi[3 + i] * m[1] + a.hi[6 + i] * m[2]);
            k2 += k * k;
        }
    } else {
        for (int d = 0; d < 3; ++d) {
            const double k = 2.0 * kPi * m[d] / a.L[d];
            k2 += k * k;
        }
    }
    const SogTables *t = a.tab;
    double a5 = 0.0, a7 = 0.0;
    for (int l = 0; l < a.M; ++l) {
        const double e = exp(-t->s[l] * t->s[l] * k2 / 4.0);
        a5 += t->wt[l] * t->s5[l] * e;
        a7 += t->wt[l] * t->s7[l] * e;
    }
    const double target = k2 * a5;
    // general cell: eq. proposal's integral over the unit cube around m by the
    // tensor Gauss-Legendre rule, exp(-a (2 (Cm).d + d^T C d)) split into the
    // tabulated exp(-a d^T C d) (times the weights) and one factor per axis,
    // with exp(-a m^T C m) outside; C = h^-1 h^-T, a = pi^2 s^2
    auto pmf_cell = [&](double s0, int tabi) {
        const double aa = kPi * kPi * s0 * s0;
        double C[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                C[3 * i + j] = a.hi[3 * i] * a.hi[3 * j] + a.hi[3 * i + 1] * a.hi[3 * j + 1] +
                               a.hi[3 * i + 2] * a.hi[3 * j + 2];
        double cm[3], mm = 0.0;
        for (int i = 0; i < 3; ++i) {
            cm[i] = C[3 * i] * m[0] + C[3 * i + 1] * m[1] + C[3 * i + 2] * m[2];
            mm += m[i] * cm[i];
        }
        double e[3][kGl];
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < kGl; ++i) e[d][i] = exp(-2.0 * aa * cm[d] * t->glx[i]);
        // every lane reads the same table entries: a row's kGl loads are
        // issued together (the sum keeps its order)
        const RB_GLOBAL double *T = gp(a.gltab) + tabi * (kGl * kGl * kGl);
        double acc = 0.0;
        for (int i = 0; i < kGl; ++i)
            for (int j = 0; j < kGl; ++j) {
                const RB_GLOBAL double *Tr = T + (i * kGl + j) * kGl;
                double t[kGl];
#pragma unroll
                for (int k = 0; k < kGl; ++k) t[k] = Tr[k];
                double row = 0.0;
#pragma unroll
                for (int k = 0; k < kGl; ++k) row += t[k] * e[2][k];
                acc += e[0][i] * e[1][j] * row;
            }
        const double rs = sqrt(kPi) * s0;
        return rs * rs * rs / a.V * exp(-aa * mm) * acc;
    };
    auto pmf = [&](double s0) {
        if (a.tri) return pmf_cell(s0, s0 == t->s[0] ? 0 : 1);
        double q = 1.0;
        for (int d = 0; d < 3; ++d) {
            const double sig = a.L[d] / (sqrt(2.0) * kPi * s0);
            const double c = 1.0 / (sqrt(2.0) * sig);
            double qd;
            if (m[d] == 0) {
                qd = erf(0.5 * c);
            } else {
                const double am = fabs(static_cast<double>(m[d]));
                qd = 0.5 * (erfc((am - 0.5) * c) - erfc((am + 0.5) * c));
            }
            q *= qd;
        }
        return q;
    };
    *w = target / pmf(t->s[0]);
    *R = k2 * a7 / a5;
    if (wnr || wrw) {
        const double qw = pmf(t->s[0] * kNrWiden);
        if (wnr) *wnr = target * *R / qw;
        if (wrw) *wrw = target / qw;
    }
}

// Tries of the rejection draw that starts a chain (each accepted with
// probability above 0.08 for the boxes tested: failing all has probability
// below 1e-37).
constexpr int kStartTries = 1024;

// Algorithm 1 steps 2-3 for one system per workgroup of 256 threads.
// Slot 0 holds the r-chain's start state, slot t+1 the t-th proposal.  The
// exchange form's non-radial start state is slot P+1; the independent
// non-radial chain's start state is slot P+1 and its t-th proposal slot
// P+2+t (their weights P^nr/q' in s_w).
//
// Start states: every chain starts each step from an exact draw of its own
// target, by rejection from the rounded Gaussian with width parameter
// s_0/sqrt2: try t draws m (normals of streams 3, 4 for the r-chain, 8, 9 for
// the non-radial one, at counter t) and passes iff u B < g(m)/q'(m), u the
// first (r) or second (non-radial) uniform of stream 7 at counter t and B the
// host's bound of g/q'.  The first passing try is the start state.
__global__ __launch_bounds__(256) void k_sampler(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp)
{
#pragma clang fp contract(off)
    __shared__ int3 s_mode[kMaxModes];
    __shared__ double s_w[kMaxModes], s_R[kMaxModes];
    __shared__ double s_ur[kMaxP], s_unr[kMaxP];
    __shared__ int16_t s_sr[kMaxP], s_snr[kMaxP];
    __shared__ int16_t s_rep[kMaxModes], s_didx[kMaxModes];
    __shared__ uint8_t s_used[kMaxModes];
    __shared__ int s_cnt_r[kMaxModes], s_cnt_nr[kMaxModes];
    __shared__ int s_first[2], s_nd;
    __shared__ long long s_acc[2];

    const SysDesc &D = desc[blockIdx.x];
    const SysStep &St = stp[blockIdx.x];
    SampArgs a;
    for (int d = 0; d < 3; ++d) a.L[d] = St.L[d];
    a.tri = St.tri;
    for (int i = 0; i < 9; ++i) {
        a.h[i] = St.h[i];
        a.hi[i] = St.hi[i];
    }
    a.V = St.V;
    a.gltab = D.gltab;
    a.B[0] = St.Bstart[0];
    a.B[1] = St.Bstart[1];
    a.P = D.P;
    a.M = D.M;
    a.variant = D.variant;
    a.mcap = D.mcap;
    a.key0 = D.key0;
    a.key1 = D.key1;
    a.step = St.step;
    a.sys = D.sys;
    a.tab = &D.tab;
    a.mraw = D.mraw;
    a.modes = D.modes;
    a.cnt = D.cnt;
    a.res = D.res;

    const int tid = threadIdx.x;
    const int P = a.P;
    const bool indep = a.variant == RBSOG_RECAL_INDEPENDENT;
    const bool exch = a.variant == RBSOG_RECAL_EXCHANGE;
    const bool nrstart = indep || exch;
    const int nslots = a.mcap;  // P + 1, P + 2 (exchange) or 2P + 2 (independent)
    const int nr0 = P + 1;      // slot of the non-radial start state
    if (a.tri) {
        // the proposal pmf's quadrature table for this step's cell, both widths
        constexpr int nn = kGl * kGl * kGl;
        double C[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                C[3 * i + j] = a.hi[3 * i] * a.hi[3 * j] + a.hi[3 * i + 1] * a.hi[3 * j + 1] +
                               a.hi[3 * i + 2] * a.hi[3 * j + 2];
        RB_GLOBAL double *gt = gp(D.gltab);
        for (int idx = tid; idx < 2 * nn; idx += blockDim.x) {
            const int wi = idx / nn, r = idx % nn;
            const int i = r / (kGl * kGl), j = (r / kGl) % kGl, k = r % kGl;
            const double s0 = D.tab.s[0] * (wi ? kNrWiden : 1.0);
            const double aa = kPi * kPi * s0 * s0;
            const double d[3] = {D.tab.glx[i], D.tab.glx[j], D.tab.glx[k]};
            double dcd = 0.0;
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) dcd += d[p] * C[3 * p + q] * d[q];
            gt[idx] = D.tab.glw[i] * D.tab.glw[j] * D.tab.glw[k] * exp(-aa * dcd);
        }
        __threadfence_block();
        __syncthreads();
    }
    if (tid == 0) {
        s_first[0] = kStartTries;
        s_first[1] = nrstart ? kStartTries : -1;
    }
    __syncthreads();
    // start states: rounds of 256 tries until each chain has a passing one
    for (int base = 0; base < kStartTries; base += blockDim.x) {
        const bool need_r = s_first[0] == kStartTries, need_nr = s_first[1] == kStartTries;
        __syncthreads();  // every thread has read s_first before this round's atomics
        const uint32_t t = static_cast<uint32_t>(base + tid);
        const uint4 o = philox4x32_10(make_uint4(t, 7u, a.step, a.sys), make_uint2(a.key0, a.key1));
        int mr[3] = {0, 0, 0}, mn[3] = {0, 0, 0};
        bool pass_r = false, pass_nr = false;
        if (need_r) {
            double z[3], w, R, wrw;
            draw_normals(a, t, 3u, 4u, z);
            round_proposal(a, z, mr, kNrWiden);
            mode_weights(a, mr, &w, &R, nullptr, &wrw);
            pass_r = unit_open(o.x, o.y) * a.B[0] < wrw;
            if (pass_r) atomicMin(&s_first[0], static_cast<int>(t));
        }
        if (need_nr) {
            double z[3], w, R, wnr;
            draw_normals(a, t, 8u, 9u, z);
            round_proposal(a, z, mn, kNrWiden);
            mode_weights(a, mn, &w, &R, &wnr);
            pass_nr = unit_open(o.z, o.w) * a.B[1] < wnr;
            if (pass_nr) atomicMin(&s_first[1], static_cast<int>(t));
        }
        __syncthreads();
        if (pass_r && s_first[0] == static_cast<int>(t)) {
            s_mode[0] = make_int3(mr[0], mr[1], mr[2]);
            mode_weights(a, mr, &s_w[0], &s_R[0]);
        }
        if (pass_nr && s_first[1] == static_cast<int>(t)) {
            s_mode[nr0] = make_int3(mn[0], mn[1], mn[2]);
            double w, R, wnr;
            mode_weights(a, mn, &w, &R, &wnr);
            // the exchange form's state can move into the r-chain (radial weight);
            // the independent chain weighs its states by P^nr/q'
            s_w[nr0] = indep ? wnr : w;
            s_R[nr0] = R;
        }
        const bool done = s_first[0] < kStartTries && s_first[1] < kStartTries;
        __syncthreads();
        if (done) break;
    }
    for (int t = tid; t < P; t += blockDim.x) {
        double z[3];
        int m[3];
        draw_normals(a, static_cast<uint32_t>(t), 0u, 1u, z);
        round_proposal(a, z, m);
        s_mode[t + 1] = make_int3(m[0], m[1], m[2]);
        mode_weights(a, m, &s_w[t + 1], &s_R[t + 1]);
        const uint4 o = philox4x32_10(make_uint4(static_cast<uint32_t>(t), 2u, a.step, a.sys),
                                      make_uint2(a.key0, a.key1));
        s_ur[t] = unit_open(o.x, o.y);
        s_unr[t] = unit_open(o.z, o.w);
        if (indep) {
            draw_normals(a, static_cast<uint32_t>(t), 5u, 6u, z);
            round_proposal(a, z, m, kNrWiden);
            double w, R;
            s_mode[P + 2 + t] = make_int3(m[0], m[1], m[2]);
            mode_weights(a, m, &w, &R, &s_w[P + 2 + t]);
            s_R[P + 2 + t] = R;
        }
    }
    for (int s = tid; s < nslots; s += blockDim.x) {
        s_used[s] = 0;
        s_cnt_r[s] = 0;
        s_cnt_nr[s] = 0;
    }
    __syncthreads();
    if (s_first[0] >= kStartTries || s_first[1] >= kStartTries) {
        if (tid == 0) {
            a.res->status = -1;
            a.res->nd = 0;
        }
        return;
    }
    // the chains are sequential: one lane walks them
    if (tid == 0) {
        long long acc_r = 0, acc_nr = 0;
        int cur = 0;
        double wcur = s_w[0];
        if (exch) {
            // the second state starts from its exact non-radial draw
            int zs = nr0;
            double rz = s_R[nr0];
            for (int t = 0; t < P; ++t) {
                if (s_ur[t] < s_w[t + 1] / wcur) {
                    cur = t + 1;
                    wcur = s_w[t + 1];
                    ++acc_r;
                }
                const double rx = s_R[cur];
                if (s_unr[t] < rx / rz) {
                    const int tmp = cur;
                    cur = zs;
                    zs = tmp;
                    wcur = s_w[cur];
                    rz = rx;
                    ++acc_nr;
                }
                s_sr[t] = static_cast<int16_t>(cur);
                s_snr[t] = static_cast<int16_t>(zs);
            }
        } else if (a.variant == RBSOG_RECAL_SHARED || indep) {
            for (int t = 0; t < P; ++t) {
                if (s_ur[t] < s_w[t + 1] / wcur) {
                    cur = t + 1;
                    wcur = s_w[t + 1];
                    ++acc_r;
                }
                s_sr[t] = static_cast<int16_t>(cur);
            }
            if (indep) {
                // its own chain from its exact start, target P^nr
                int zs = nr0;
                double wz = s_w[nr0];
                for (int t = 0; t < P; ++t) {
                    const int prop = P + 2 + t;
                    if (s_unr[t] < s_w[prop] / wz) {
                        zs = prop;
                        wz = s_w[prop];
                        ++acc_nr;
                    }
                    s_snr[t] = static_cast<int16_t>(zs);
                }
            } else {
                for (int t = 0; t < P; ++t) s_snr[t] = s_sr[t];
            }
        } else {
            for (int t = 0; t < P; ++t) {
                if (s_ur[t] < s_w[t + 1] / wcur) {
                    cur = t + 1;
                    wcur = s_w[t + 1];
                    ++acc_r;
                }
                s_sr[t] = static_cast<int16_t>(cur);
            }
            int zs = s_sr[0];
            double rz = s_R[zs];
            for (int t = 0; t < P; ++t) {
                const int prop = s_sr[t];
                if (s_unr[t] < s_R[prop] / rz) {
                    zs = prop;
                    rz = s_R[prop];
                    ++acc_nr;
                }
                s_snr[t] = static_cast<int16_t>(zs);
            }
        }
        s_acc[0] = acc_r;
        s_acc[1] = acc_nr;
    }
    __syncthreads();
    for (int t = tid; t < P; t += blockDim.x) {
        s_used[s_sr[t]] = 1;
        s_used[s_snr[t]] = 1;
    }
    __syncthreads();
    // representative of each used slot: the first used slot with the same mode
    for (int s = tid; s < nslots; s += blockDim.x) {
        int rep = s;
        if (s_used[s]) {
            const int3 ms = s_mode[s];
            for (int u = 0; u < s; ++u) {
                if (s_used[u] && s_mode[u].x == ms.x && s_mode[u].y == ms.y && s_mode[u].z == ms.z) {
                    rep = u;
                    break;
                }
            }
        }
        s_rep[s] = static_cast<int16_t>(rep);
    }
    __syncthreads();
    if (tid == 0) {
        int nd = 0;
        for (int s = 0; s < nslots; ++s) {
            if (s_used[s] && s_rep[s] == s) {
                s_didx[s] = static_cast<int16_t>(nd);
                a.modes[nd] = make_int4(s_mode[s].x, s_mode[s].y, s_mode[s].z, 0);
                ++nd;
            }
        }
        s_nd = nd;
    }
    __syncthreads();
    for (int t = tid; t < P; t += blockDim.x) {
        atomicAdd(&s_cnt_r[s_didx[s_rep[s_sr[t]]]], 1);
        atomicAdd(&s_cnt_nr[s_didx[s_rep[s_snr[t]]]], 1);
        const int3 mr = s_mode[s_sr[t]], mn = s_mode[s_snr[t]];
        a.mraw[3 * t] = mr.x;
        a.mraw[3 * t + 1] = mr.y;
        a.mraw[3 * t + 2] = mr.z;
        a.mraw[3 * (P + t)] = mn.x;
        a.mraw[3 * (P + t) + 1] = mn.y;
        a.mraw[3 * (P + t) + 2] = mn.z;
    }
    __syncthreads();
    for (int d = tid; d < a.mcap; d += blockDim.x) {
        const bool in = d < s_nd;
        a.cnt[d] = in ? s_cnt_r[d] : 0;
        a.cnt[a.mcap + d] = in ? s_cnt_nr[d] : 0;
    }
    if (tid == 0) {
        a.res->nd = s_nd;
        a.res->status = 0;
        a.res->acc_r = s_acc[0];
        a.res->acc_nr = s_acc[1];
    }
}

// ----------------------------------------------------------------------------
// Fixed point, binning and the stable cell sort
// ----------------------------------------------------------------------------

// Wave-aggregated counter increment: every active lane adds 1 to
// counter[key]; lanes with equal keys are served by one atomic of their
// leader (the group's first lane), and each lane receives the counter's old
// value plus its rank among those lanes (by lane order).  The groups are
// found with ballots first; then every leader issues its atomic in the same
// instruction, so a wavefront waits for one round trip, not one per key.
template <bool kReturn>
__device__ inline int aggregated_increment(int32_t *counter, int key, bool active)
{
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(active);
    int leader = lane, rank = 0, size = 0;
    while (todo) {
        const int first = __ffsll(static_cast<unsigned long long>(todo)) - 1;
        const int lkey = __shfl(key, first, 64);
        const uint64_t peers = __ballot(active && key == lkey) & todo;
        if ((peers >> lane) & 1ull) {
            leader = first;
            rank = __popcll(peers & ((1ull << lane) - 1ull));
            size = __popcll(peers);
        }
        todo &= ~peers;
    }
    int base = 0;
    if (active && lane == leader) {
        if constexpr (kReturn) base = atomicAdd(&counter[key], size);
        else atomicAdd(&counter[key], size);
    }
    if constexpr (kReturn) return __shfl(base, leader, 64) + rank;
    return 0;
}

// per-cell counters to zero; block 0 also resets the pair work-queue counters
__global__ __launch_bounds__(kCellBlock) void k_zero(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                     const int2 *__restrict__ plan, int32_t *__restrict__ ctrl)
{
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const int64_t c = e.y * static_cast<int64_t>(kCellBlock) + threadIdx.x;
    if (c <= stp[e.x].ncells) {
        D.count[c] = 0;
    }
    if (e.y == 0 && threadIdx.x == 0) {
        D.res->bad_input = 0;
        if (stp[e.x].half) *D.hflag = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < kNumPairGroups) ctrl[threadIdx.x] = 0;
}

// s = x (1/L) wrapped into [0,1) by subtracting floor(s); u = s 2^bits; the
// 32-bit cell coordinate is (u32 n) >> 32 with u32 the top 32 bits of u.
template <class T>
__global__ __launch_bounds__(kAtomBlock) void k_fix(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                    const int2 *__restrict__ plan)
{
#pragma clang fp contract(off)
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const SysStep &St = stp[e.x];
    const int64_t n = D.n;
    const int64_t i = e.y * static_cast<int64_t>(kAtomBlock) + threadIdx.x;
    const bool active = i < n;
    if (!__any(active)) return;
    const int64_t ii = active ? i : 0;
    const double p[3] = {gp(St.x)[ii], gp(St.y)[ii], gp(St.z)[ii]};
    // a NaN or infinite coordinate still gives a cell inside the grid (u < 2^32);
    // the step is flagged and the host reports RBSOG_EINVAL
    const bool bad = active && !(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]));
    if (__any(bad) && threadIdx.x % 64 == 0) atomicOr(&D.res->bad_input, 1);
    const int nc[3] = {St.nc[0], St.nc[1], St.nc[2]};
    RB_GLOBAL typename T::fix *u = gp(static_cast<typename T::fix *>(D.u));
    uint32_t c[3];
    // fractional coordinates s = h^-1 r (a general cell) or r / L
    double sv[3];
    if (St.tri) {
        for (int d = 0; d < 3; ++d) sv[d] = St.hi[3 * d] * p[0] + St.hi[3 * d + 1] * p[1] + St.hi[3 * d + 2] * p[2];
    } else {
        for (int d = 0; d < 3; ++d) sv[d] = p[d] * St.iL[d];
    }
    for (int d = 0; d < 3; ++d) {
        double s = sv[d];
        s -= floor(s);
        uint32_t top;
        if constexpr (sizeof(typename T::fix) == 4) {
            top = static_cast<uint32_t>(static_cast<uint64_t>(s * 4294967296.0) & 0xFFFFFFFFull);
            if (active) u[d * n + i] = top;
        } else {
            if (s >= 1.0) s -= 1.0;
            const uint64_t v = static_cast<uint64_t>(s * 18446744073709551616.0);
            if (active) u[d * n + i] = v;
            top = static_cast<uint32_t>(v >> 32);
        }
        c[d] = static_cast<uint32_t>((static_cast<uint64_t>(top) * static_cast<uint32_t>(nc[d])) >> 32);
    }
    // z fastest: the cells of one column (cx, cy) are consecutive, so a column's
    // atoms are one range of the sorted arrays, ordered by z
    const int32_t id = static_cast<int32_t>(c[2] + static_cast<uint32_t>(nc[2]) * (c[1] + static_cast<uint32_t>(nc[1]) * c[0]));
    if (active) gp(D.cell)[i] = id;
    // the atom's place among its cell's atoms, in the order the counts were
    // taken (the ordering kernel makes the final order independent of it)
    const int slot = aggregated_increment<true>(D.count, id, active);
    if (active) gp(D.slot)[i] = slot;
}

// Two-level exclusive scan of the per-cell counts (and of the per-cell number
// of 64-atom pair blocks) of each system: kScanBlock cells per workgroup, at
// most 1024 workgroups per system.  Pair blocks tile segments of g cells of a
// column (the cells cz = 0, g, 2g, ... own the blocks of their segment), so a
// segment's last block is the only one with idle lanes.
__device__ inline void block_scan_256(int *s_a, int tid)
{
    // Hillis-Steele inclusive scan over 256 ints in shared memory
    for (int o = 1; o < 256; o <<= 1) {
        const int v = tid >= o ? s_a[tid - o] : 0;
        __syncthreads();
        s_a[tid] += v;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_scan_local(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                    const int2 *__restrict__ plan)
{
    __shared__ int s_a[256], s_b[256];
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const SysStep &St = stp[e.x];
    const int64_t m = St.ncells;
    const int nz = St.nc[2], g = St.g;
    const int tid = threadIdx.x;
    const int64_t base = e.y * static_cast<int64_t>(kScanBlock) + 4 * tid;
    int va[4], vb[4], ta = 0, tb = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + k;
        const int c = i < m ? D.count[i] : 0;
        va[k] = c;
        vb[k] = 0;
        if (i < m) {
            const int cz = static_cast<int>(i % nz);
            if (cz % g == 0) {
                int seg = c;
                for (int t = 1; t < g && cz + t < nz; ++t) seg += D.count[i + t];
                vb[k] = (seg + kPairWave - 1) / kPairWave;
            }
            D.nblk[i] = vb[k];
        }
        ta += va[k];
        tb += vb[k];
    }
    s_a[tid] = ta;
    s_b[tid] = tb;
    __syncthreads();
    block_scan_256(s_a, tid);
    block_scan_256(s_b, tid);
    int ea = s_a[tid] - ta, eb = s_b[tid] - tb;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + k;
        if (i < m) {
            D.start[i] = ea;
            D.bstart[i] = eb;
        }
        ea += va[k];
        eb += vb[k];
    }
    if (tid == 255) {
        D.scan_tmp[2 * e.y] = s_a[255];
        D.scan_tmp[2 * e.y + 1] = s_b[255];
    }
}

// Final starts, and the pair-block table (cell, sub-block) of each cell.  A
// workgroup's cells lie in one scan block b (kScanBlock is a multiple of
// kCellBlock); it adds the sums of the scan blocks before b itself, and the
// workgroup holding cell m = ncells also all of them for the totals.
static_assert(kScanBlock % kCellBlock == 0, "a cell workgroup lies in one scan block");
__global__ __launch_bounds__(kCellBlock) void k_scan_add(const SysDesc *__restrict__ desc,
                                                         const SysStep *__restrict__ stp,
                                                         const int2 *__restrict__ plan)
{
    __shared__ int s_a[256], s_b[256];
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const int64_t m = stp[e.x].ncells;
    const int tid = threadIdx.x;
    const int64_t c0 = e.y * static_cast<int64_t>(kCellBlock);
    const int64_t i = c0 + tid;
    const int32_t *sums = D.scan_tmp;
    const int nb = static_cast<int>((m + kScanBlock - 1) / kScanBlock);
    const int b = static_cast<int>(c0 / kScanBlock);
    const bool holds_m = c0 <= m && m < c0 + kCellBlock;
    // offsets of scan block b: the block sums before it
    int pa = 0, pb = 0;
    for (int k = tid; k < b; k += 256) {
        pa += sums[2 * k];
        pb += sums[2 * k + 1];
    }
    s_a[tid] = pa;
    s_b[tid] = pb;
    __syncthreads();
    block_scan_256(s_a, tid);
    block_scan_256(s_b, tid);
    const int oa = s_a[255], ob = s_b[255];
    int ta = 0, tb = 0;
    if (holds_m) {  // uniform over the workgroup
        pa = pb = 0;
        for (int k = tid; k < nb; k += 256) {
            pa += sums[2 * k];
            pb += sums[2 * k + 1];
        }
        __syncthreads();
        s_a[tid] = pa;
        s_b[tid] = pb;
        __syncthreads();
        block_scan_256(s_a, tid);
        block_scan_256(s_b, tid);
        ta = s_a[255];
        tb = s_b[255];
    }
    if (i < m) {
        D.start[i] += oa;
        const int b0 = D.bstart[i] + ob;
        D.bstart[i] = b0;
        const int nbk = D.nblk[i];
        for (int k = 0; k < nbk; ++k) D.blocks[b0 + k] = make_int2(static_cast<int>(i), k);
    } else if (i == m) {
        D.start[m] = ta;
        D.bstart[m] = tb;
    }
}

// The sort key of an atom inside its cell: its z fixed-point coordinate (top
// 32 bits), then its index.  Sorting each cell by z makes every 64-atom pair
// block a thin z-slab, which the pair kernel uses to skip neighbours out of
// reach in z.
template <class T>
__device__ inline uint64_t cell_key(const SysDesc &D, int64_t i)
{
    const typename T::fix uz = gp(static_cast<const typename T::fix *>(D.u))[2 * D.n + i];
    uint32_t top;
    if constexpr (sizeof(typename T::fix) == 4) top = uz;
    else top = static_cast<uint32_t>(uz >> 32);
    return (static_cast<uint64_t>(top) << 32) | static_cast<uint64_t>(i);
}

template <class T>
__global__ __launch_bounds__(kAtomBlock) void k_scatter(const SysDesc *__restrict__ desc, const int2 *__restrict__ plan)
{
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const int64_t i = e.y * static_cast<int64_t>(kAtomBlock) + threadIdx.x;
    const bool active = i < D.n;
    if (!__any(active)) return;
    if (active) {
        const int c = gp(D.cell)[i];
        const int slot = gp(D.slot)[i];
        // the key and the whole record go to the binned slot, so that the
        // ordering kernel reads each cell's records as one contiguous range
        const int64_t pos = gp(D.start)[c] + slot;
        const int64_t n = D.n;
        const RB_GLOBAL typename T::fix *u = gp(static_cast<const typename T::fix *>(D.u));
        typename T::Rec r;
        r.x = u[i];
        r.y = u[n + i];
        r.z = u[2 * n + i];
        r.q = gp(static_cast<const typename T::real *>(D.q))[i];
        gp(D.keys)[pos] = cell_key<T>(D, i);
        gstore(static_cast<typename T::Rec *>(D.urec) + pos, r);
    }
}

// Within each cell, atoms are ordered by their key (z, then index); keys are
// unique, so the order does not depend on the scatter's.  One workgroup of
// kOrderThreads per cell ranks each of the cell's keys against all of them
// (the keys pass through LDS kOrderThreads at a time, every thread holding
// kRankKeys of the keys it ranks in registers; a cell of up to kOrderThreads
// atoms is one tile and one key a thread).  A single-cell system has one
// workgroup per kOrderPart of its keys instead.  The record in binned slot j
// goes to sorted slot rank j, with the atom's index: both reads and writes
// stay inside the cell's range.
constexpr int kOrderThreads = 256;
constexpr int kRankKeys = kOrderPart / kOrderThreads;
static_assert(kOrderThreads * kRankKeys == kOrderPart, "one rank pass per part of a single cell");
template <class T>
__device__ inline void move_sorted(const SysDesc &D, int from, int to, uint64_t key)
{
    gp(D.perm)[to] = static_cast<int>(key & 0xFFFFFFFFull);
    const typename T::Rec r = gload(static_cast<const typename T::Rec *>(D.urec) + from);
    gstore(static_cast<typename T::Rec *>(D.rec) + to, r);
}

template <class T>
__global__ __launch_bounds__(kOrderThreads) void k_order(const SysDesc *__restrict__ desc,
                                                         const SysStep *__restrict__ stp, const int2 *__restrict__ plan)
{
    constexpr int NT = kOrderThreads;
    __shared__ uint64_t s_key[NT];
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const bool single = stp[e.x].ncells == 1;
    const int c = single ? 0 : e.y;
    const int tid = threadIdx.x;
    const int s0 = gp(D.start)[c], s1 = gp(D.start)[c + 1];
    const int cnt = s1 - s0;
    if (cnt == 0) return;
    const RB_GLOBAL uint64_t *keys = gp(D.keys);
    if (cnt <= NT) {  // a single cell this small has one part
        const uint64_t mine = tid < cnt ? keys[s0 + tid] : ~0ull;
        s_key[tid] = mine;
        __syncthreads();
        int rank = 0;
        for (int j = 0; j < cnt; ++j) rank += s_key[j] < mine;
        if (tid < cnt) move_sorted<T>(D, s0 + tid, s0 + rank, mine);
    } else {
        const int lo = single ? e.y * kOrderPart : 0;
        const int hi = single ? min(cnt, lo + kOrderPart) : cnt;
        for (int base = lo; base < hi; base += kOrderPart) {
            uint64_t mine[kRankKeys];
            int rank[kRankKeys];
#pragma unroll
            for (int r = 0; r < kRankKeys; ++r) {
                const int t = base + NT * r + tid;
                mine[r] = t < hi ? keys[s0 + t] : 0ull;
                rank[r] = 0;
            }
            for (int j0 = 0; j0 < cnt; j0 += NT) {
                __syncthreads();  // the previous tile is no longer read
                s_key[tid] = j0 + tid < cnt ? keys[s0 + j0 + tid] : 0ull;
                __syncthreads();
                const int m = min(NT, cnt - j0);
                for (int j = 0; j < m; ++j) {
                    const uint64_t k = s_key[j];
#pragma unroll
                    for (int r = 0; r < kRankKeys; ++r) rank[r] += k < mine[r];
                }
            }
#pragma unroll
            for (int r = 0; r < kRankKeys; ++r) {
                const int t = base + NT * r + tid;
                if (t < hi) move_sorted<T>(D, s0 + t, s0 + rank[r], mine[r]);
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Short-range pair kernel
// ----------------------------------------------------------------------------
//
// One wavefront owns up to 64 atoms of one pair block: a z-slab of a segment
// of g cells of one column (cells are numbered z fastest and sorted by z, so
// a segment is a z-sorted range of the sorted arrays and only its last block
// has idle lanes).  It walks the atoms of the neighbouring cells (full shell:
// every pair is evaluated from both sides, so no atomics and a fixed
// summation order).  The neighbours are contiguous ranges of the sorted
// arrays: with at least four cells per edge (FP32), each of the 9 neighbour
// columns cut to the block's z-window; otherwise a run of cells per
// neighbour column.  They are staged kChunk at a time in LDS; every lane
// tests every staged candidate against r_c and keeps one hit bit per
// candidate; then every lane walks its hit bits, reading partner records
// from LDS, so the expensive SOG kernel runs on wavefronts whose lanes all
// hold a real pair until the lane with the fewest partners in the chunk is
// done.

#ifndef RBSOG_PAIR_CHUNK
#define RBSOG_PAIR_CHUNK 128
#endif
#ifndef RBSOG_PAIR_OCC
#define RBSOG_PAIR_OCC 5
#endif
#ifndef RBSOG_FAST_FILTER
#define RBSOG_FAST_FILTER 1
#endif
#ifndef RBSOG_REL_EVAL
#define RBSOG_REL_EVAL 1
#endif
constexpr int kChunk = RBSOG_PAIR_CHUNK;     // candidates staged per round
constexpr int kMaxRanges = 27;  // at most two per neighbour column (a run split at the periodic seam)
static_assert(kChunk % 32 == 0 && kChunk % 4 == 0, "pair tiling");

template <class T>
struct PairAcc {
    using real = typename T::real;
    // sums over partners j of q_j-weighted terms (the common q_i is applied once per chunk)
    real fx = 0, fy = 0, fz = 0, vxx = 0, vyy = 0, vzz = 0, vxy = 0, vxz = 0, vyz = 0, u = 0;
    int n = 0;  // pairs inside rc
};

// Splitting weights held in registers for the whole kernel.  M > 0: M
// exponentials with compile-time M; M = 0: runtime M read from the table;
// M = -1: the FP32C polynomial form (coefficients of both sums in t).
template <class T, int M>
struct Weights {
    using real = typename T::real;
    real c[M], wt[M], w[M];  // exponent factor, 1/r^3-split weight, 1/r-split weight
    int m = M;
};
template <class T>
struct Weights<T, 0> {  // runtime M: read from the table
    const SogTables *tab;
    int m;
};
template <class T>
struct Weights<T, -1> {
    float pa;
    float pg[kPolyDeg + 1], pf[kPolyDeg + 1];
};

template <class T, int M>
__device__ inline void load_weights(Weights<T, M> &W, const SogTables *__restrict__ tab)
{
    if constexpr (M == -1) {
        W.pa = tab->pa;
#pragma unroll
        for (int k = 0; k <= kPolyDeg; ++k) {
            W.pg[k] = tab->pg[k];
            W.pf[k] = tab->pf[k];
        }

    } else if constexpr (M == 0) {
        W.tab = tab;
        W.m = tab->Me;  // the force weights are zero past M
    } else {
#pragma unroll
        for (int l = 0; l < M; ++l) {
            if constexpr (sizeof(typename T::real) == 4) {
                W.c[l] = tab->c32[l];
                W.wt[l] = tab->wt32[l];
                W.w[l] = tab->w32[l];
            } else {
                W.c[l] = -tab->inv_s2[l];
                W.wt[l] = tab->wt[l];
                W.w[l] = tab->w[l];
            }
        }
    }
}

template <class T, int M, bool E>
__device__ inline typename T::real gauss(const Weights<T, M> &W, int l, typename T::real r2, typename T::real &wl)
{
    using real = typename T::real;
    real c, wtl;
    if constexpr (M == 0) {
        if constexpr (sizeof(real) == 4) {
            c = W.tab->c32[l];
            wtl = W.tab->wt32[l];
            wl = W.tab->w32[l];
        } else {
            c = -W.tab->inv_s2[l];
            wtl = W.tab->wt[l];
            wl = W.tab->w[l];
        }
    } else {
        c = W.c[l];
        wtl = W.wt[l];
        wl = W.w[l];
    }
    real e;
    if constexpr (sizeof(real) == 4) e = __builtin_amdgcn_exp2f(r2 * c);
    else e = exp(r2 * c);
    if constexpr (E) wl *= e;
    return wtl * e;
}

// Horner evaluation of sum_k p[k] t^k
__device__ __forceinline__ float horner(const float *p, float t)
{
    float v = p[kPolyDeg];
#pragma unroll
    for (int k = kPolyDeg - 1; k >= 0; --k) v = v * t + p[k];
    return v;
}

template <class T>
__device__ inline void displacement(const typename T::Rec &ri, const typename T::Rec &rj, typename T::real sx,
                                    typename T::real sy, typename T::real sz, typename T::real &dx,
                                    typename T::real &dy, typename T::real &dz)
{
    using sfix = typename T::sfix;
    dx = fix_to_real(static_cast<sfix>(ri.x - rj.x), sx);
    dy = fix_to_real(static_cast<sfix>(ri.y - rj.y), sy);
    dz = fix_to_real(static_cast<sfix>(ri.z - rj.z), sz);
}

// The SOG short-range kernels of one pair with displacement (dx, dy, dz) and
// partner charge qj: N~(r) = 1/r^3 - sum wt_l e_l for the force and the virial
// (eqs. force_SOG, P_short; 2 w_l/s_l^2 = wt_l) and N(r) = 1/r - sum w_l e_l
// for the energy (eq. U_short), e_l = exp(-r^2/s_l^2), the energy only when E.
// Every lane of the wavefront runs it; a lane with no pair this round (active
// false) and a listed pair farther than rc (possible only through the padded
// fast filter) contribute nothing.  The terms carry q_j only; the caller
// multiplies the sums by q_i.
template <class T, int M, bool E, bool kLaneCount = true>
__device__ __forceinline__ void pair_eval_d(typename T::real dx, typename T::real dy, typename T::real dz,
                                            typename T::real qj, bool active, typename T::real rc2,
                                            const Weights<T, M> &W, PairAcc<T> &acc, uint64_t *wave_inside = nullptr)
{
    using real = typename T::real;
    const real r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if constexpr (!kLaneCount) {
        // the wavefront's lanes with the pair inside, as a lane mask (the
        // same two compares as below, taken as a scalar value)
        static_assert(sizeof(real) == 4, "wave-mask count on the FP32 path only");
        *wave_inside = __builtin_amdgcn_fcmpf(r2, rc2, 4 /* ordered less */) &
                       __builtin_amdgcn_fcmpf(r2, 0.0f, 2 /* ordered greater */);
    }
    const bool inside = active & (r2 < rc2) & (r2 > static_cast<real>(0));  // the atom itself is listed too
    real swt = 0, sw = 0, rinv;
    if constexpr (sizeof(real) == 4) rinv = __builtin_amdgcn_rsqf(r2);
    else rinv = 1.0 / sqrt(r2);
    if constexpr (M == -1) {
        const float t = r2 * W.pa - 1.0f;
        swt = horner(W.pg, t);
        if constexpr (E) sw = horner(W.pf, t);
    } else if constexpr (M == 0) {
        for (int l = 0; l < W.m; ++l) {
            real wl;
            swt += gauss<T, M, E>(W, l, r2, wl);
            if constexpr (E) sw += wl;
        }
    } else {
#pragma unroll
        for (int l = 0; l < M; ++l) {
            real wl;
            swt += gauss<T, M, E>(W, l, r2, wl);
            if constexpr (E) sw += wl;
        }
    }
    // the mask selects the products (r = 0 gives rinv = inf for the atom itself)
    if constexpr (kLaneCount) acc.n += inside;
    const real f = inside ? qj * (rinv * rinv * rinv - swt) : static_cast<real>(0);
    const real fdx = f * dx, fdy = f * dy, fdz = f * dz;
    acc.fx += fdx;
    acc.fy += fdy;
    acc.fz += fdz;
    acc.vxx += fdx * dx;
    acc.vyy += fdy * dy;
    acc.vzz += fdz * dz;
    acc.vxy += fdx * dy;
    acc.vxz += fdx * dz;
    acc.vyz += fdy * dz;
    if constexpr (E) acc.u += inside ? qj * (rinv - sw) : static_cast<real>(0);
}

// rinv^3 - sum_l wt_l e_l (eq. force_SOG) at r^2 = r2 in FP32: the
// charge-free factor of a pair's force and virial, unmasked.
template <class T, int M>
__device__ __forceinline__ float sog_force_factor(float r2, const Weights<T, M> &W)
{
    float swt = 0.0f;
    const float rinv = __builtin_amdgcn_rsqf(r2);
    if constexpr (M == -1) {
        swt = horner(W.pg, r2 * W.pa - 1.0f);
    } else if constexpr (M == 0) {
        for (int l = 0; l < W.m; ++l) {
            float wl;
            swt += gauss<T, M, false>(W, l, r2, wl);
        }
    } else {
#pragma unroll
        for (int l = 0; l < M; ++l) {
            float wl;
            swt += gauss<T, M, false>(W, l, r2, wl);
        }
    }
    return rinv * rinv * rinv - swt;
}

// A pair from fixed-point records: exact minimum-image displacement (integer
// difference, then scaled), r^2 in one fixed evaluation order, so a pair is
// inside from both of its atoms.
template <class T, int M, bool E>
__device__ __forceinline__ void pair_eval(const typename T::Rec &ri, const typename T::Rec &rj, bool active,
                                          typename T::real sx, typename T::real sy, typename T::real sz,
                                          typename T::real rc2, const Weights<T, M> &W, PairAcc<T> &acc)
{
    typename T::real dx, dy, dz;
    displacement<T>(ri, rj, sx, sy, sz, dx, dy, dz);
    pair_eval_d<T, M, E>(dx, dy, dz, rj.q, active, rc2, W, acc);
}

// General cell: the fractional difference of two fixed-point records (a
// minimum image component by component, exact while r_c is at most half the
// cell's smallest perpendicular width), times h.  d_ji = -d_ij exactly, so a
// pair is inside r_c from both of its atoms.
template <class T>
__device__ __forceinline__ void displacement_cell(const typename T::Rec &ri, const typename T::Rec &rj,
                                                  const typename T::real hm[9], typename T::real unit,
                                                  typename T::real &dx, typename T::real &dy, typename T::real &dz)
{
    using sfix = typename T::sfix;
    const typename T::real s0 = fix_to_real(static_cast<sfix>(ri.x - rj.x), unit);
    const typename T::real s1 = fix_to_real(static_cast<sfix>(ri.y - rj.y), unit);
    const typename T::real s2 = fix_to_real(static_cast<sfix>(ri.z - rj.z), unit);
    dx = hm[0] * s0 + hm[1] * s1 + hm[2] * s2;
    dy = hm[3] * s0 + hm[4] * s1 + hm[5] * s2;
    dz = hm[6] * s0 + hm[7] * s1 + hm[8] * s2;
}

template <class T, int M, bool E>
__device__ __forceinline__ void pair_eval_cell(const typename T::Rec &ri, const typename T::Rec &rj, bool active,
                                               const typename T::real hm[9], typename T::real unit,
                                               typename T::real rc2, const Weights<T, M> &W, PairAcc<T> &acc)
{
    typename T::real dx, dy, dz;
    displacement_cell<T>(ri, rj, hm, unit, dx, dy, dz);
    pair_eval_d<T, M, E>(dx, dy, dz, rj.q, active, rc2, W, acc);
}

// m <- 16 m + the four bits (t_k < thr), t0 first: per candidate one compare
// into VCC and one add with carry (the compiler's own form of this step takes
// three instructions).  The t_k come from FMAs, whose results a following VALU
// instruction may read at once.
__device__ __forceinline__ uint32_t push_hits4(uint32_t m, float t0, float t1, float t2, float t3, float thr)
{
    asm("v_cmp_lt_f32_e32 vcc, %1, %5\n\t"
        "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc\n\t"
        "v_cmp_lt_f32_e32 vcc, %2, %5\n\t"
        "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc\n\t"
        "v_cmp_lt_f32_e32 vcc, %3, %5\n\t"
        "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc\n\t"
        "v_cmp_lt_f32_e32 vcc, %4, %5\n\t"
        "v_addc_co_u32_e32 %0, vcc, %0, %0, vcc"
        : "+v"(m)
        : "v"(t0), "v"(t1), "v"(t2), "v"(t3), "v"(thr)
        : "vcc");
    return m;
}

typedef short short2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ short2v as_short2(uint32_t v) { return __builtin_bit_cast(short2v, v); }

// top 16 bits of x and y (y in the high half), and of z
template <class Rec>
__device__ __forceinline__ uint2 pack16(const Rec &r)
{
    return make_uint2((static_cast<uint32_t>(r.x) >> 16) | (static_cast<uint32_t>(r.y) & 0xFFFF0000u),
                      static_cast<uint32_t>(r.z) >> 16);
}

// Candidate k of a chunk in the block-relative tile: each 32-candidate word
// is preceded by a sentinel slot, read by a lane whose hit word is spent.
constexpr int kRelTile = kChunk + kChunk / 32;
__device__ __forceinline__ int rel_slot(int k) { return k + (k >> 5) + 1; }

template <class T>
struct PairShared {
    union {
        typename T::Rec tile[kChunk];  // exact path: fixed-point records
        float4 rtile[kRelTile];        // fast path: (x, y, z) relative to the block origin, q; sentinels
    };
    union {
        float4 rel[kChunk];  // fast filter: coordinates relative to the block origin and their squared norm
        uint2 pk[kChunk];    // FP32 exact filter: top 16 bits of the fixed-point x | y << 16, and of z
    };
    uint32_t mask[kChunk / 32][64];  // hit bits of each lane, one word per 32 candidates
    int pre[kMaxRanges + 1];  // flattened-neighbourhood offset of each range
    int beg[kMaxRanges];
    int split;  // fast path: the block's own atoms are cut out of its ranges
};

// One pair block b of system D (one wavefront).
template <class T, int M, bool E, bool FAST, bool TRI = false>
__device__ __forceinline__ void pair_block(PairShared<T> &sh, const SysDesc &D, const SysStep &St, int b)
{
    using real = typename T::real;
    using Rec = typename T::Rec;
    using fix = typename T::fix;
    using sfix = typename T::sfix;
    const int lane = threadIdx.x;
    const int ncells = St.ncells;
    const int nb_total = gp(D.bstart)[ncells];
    double *part = D.pair_part + 8 * static_cast<int64_t>(b);
    if (b >= nb_total) return;  // slot beyond this step's blocks: the reduction never reads it
    const Rec *__restrict__ rec = static_cast<const Rec *>(D.rec);
    Weights<T, M> W;
    load_weights<T, M>(W, &D.tab);

    const int nx = St.nc[0], ny = St.nc[1], nz = St.nc[2];
    real sx, sy, sz, rc2;
    if constexpr (sizeof(real) == 4) {
        sx = static_cast<float>(St.L[0] * 0x1.0p-32);
        sy = static_cast<float>(St.L[1] * 0x1.0p-32);
        sz = static_cast<float>(St.L[2] * 0x1.0p-32);
        rc2 = D.tab.rc2_32;
    } else {
        sx = St.L[0] * 0x1.0p-64;
        sy = St.L[1] * 0x1.0p-64;
        sz = St.L[2] * 0x1.0p-64;
        rc2 = D.tab.rc2;
    }
    // general cell (TRI): displacements h ds with ds in units of the fixed point
    real hm[9];
    real unit = sizeof(real) == 4 ? static_cast<real>(0x1.0p-32) : static_cast<real>(0x1.0p-64);
    if constexpr (TRI)
        for (int k = 0; k < 9; ++k) hm[k] = static_cast<real>(St.h[k]);
    const RB_GLOBAL int32_t *start = gp(D.start);
    const int2 cb = gload(D.blocks + b);
    // the block's segment: cells c .. c + gs - 1 of one column
    const int c = cb.x;
    const int cz = c % nz, cy = (c / nz) % ny, cx = c / (nz * ny);
    const int gs = min(St.g, nz - cz);
    const int cs = start[c], ce = start[c + gs];
    const int i0 = cs + cb.y * kPairWave;            // the block's first record
    const int nblock = min(kPairWave, ce - i0);      // its atoms
    const int i = i0 + lane;
    const bool valid = i < ce;
    Rec ri{};
    if (valid) ri = gload(rec + i);
    const real rc2_lane = valid ? rc2 : static_cast<real>(-1);  // padding lanes find no partner
    // Fast filter (FP32, at least 4 cells per edge): candidates are tested in
    // float coordinates relative to the first atom of the block, o.  The
    // block lies in one column and spans at most g cells in z; a partner
    // within rc of a block atom lies less than two cells from o along x and
    // y and less than g + 1 along z, under half the box (nx, ny >= 4,
    // nz >= 2 g + 2), so relative coordinates of every pair inside rc are
    // minimum-image offsets and their difference is the displacement.  (A
    // candidate beyond rc that wraps lands half a box away and fails.)
    // The test is |r_j|^2 - 2 r_i.r_j < rcf^2 - |r_i|^2 (three FMAs); with
    // |r| below 45 A its rounding error stays under 1e-3 A^2, far inside the
    // 2 rc 1e-3 A^2 that padding the radius by 1e-3 A adds, so it never drops
    // a pair inside rc.  The atom itself passes it; the pair evaluation
    // applies the exact test 0 < r^2 < rc^2.
    constexpr bool kIsF32 = sizeof(real) == 4;
    const bool fast = RBSOG_FAST_FILTER && kIsF32 && St.fast;
    // Fast-path pairs without the energy sum take their displacement from
    // FP32 block-relative coordinates (two roundings of exact fixed-point
    // offsets, about 1e-6 A); with the energy, whose close pairs (1/r) need
    // it, from exact fixed-point differences.
    constexpr bool kRelEval = kIsF32 && RBSOG_REL_EVAL && !E;
    const fix ox = static_cast<fix>(__shfl(static_cast<long long>(ri.x), 0, 64));
    const fix oy_ = static_cast<fix>(__shfl(static_cast<long long>(ri.y), 0, 64));
    const fix oz_ = static_cast<fix>(__shfl(static_cast<long long>(ri.z), 0, 64));
    const float rcf = static_cast<float>(sqrt(static_cast<double>(rc2))) + 1e-3f;
    // coordinates of a record relative to o: the wrapped fixed-point offset
    // scaled by L (a box) or, as a fractional offset, times h (a general cell)
    float hf[9];
    if constexpr (TRI)
        for (int k = 0; k < 9; ++k) hf[k] = static_cast<float>(St.h[k]);
    auto relpos = [&](const Rec &r, float &px, float &py, float &pz) {
        if constexpr (TRI) {
            const float a = static_cast<float>(static_cast<sfix>(r.x - ox)) * 0x1.0p-32f;
            const float b = static_cast<float>(static_cast<sfix>(r.y - oy_)) * 0x1.0p-32f;
            const float c = static_cast<float>(static_cast<sfix>(r.z - oz_)) * 0x1.0p-32f;
            px = fmaf(hf[0], a, fmaf(hf[1], b, hf[2] * c));
            py = fmaf(hf[3], a, fmaf(hf[4], b, hf[5] * c));
            pz = fmaf(hf[6], a, fmaf(hf[7], b, hf[8] * c));
        } else {
            px = static_cast<float>(static_cast<sfix>(r.x - ox)) * static_cast<float>(sx);
            py = static_cast<float>(static_cast<sfix>(r.y - oy_)) * static_cast<float>(sy);
            pz = static_cast<float>(static_cast<sfix>(r.z - oz_)) * static_cast<float>(sz);
        }
    };
    float xi, yi, zi;
    relpos(ri, xi, yi, zi);
    const float ax = -2.0f * xi, ay = -2.0f * yi, az = -2.0f * zi;
    const float thr = valid ? rcf * rcf - (xi * xi + yi * yi + zi * zi) : -INFINITY;
    // the block's bounding box in relative coordinates (fast path)
    float bx0 = 0.f, bx1 = 0.f, by0 = 0.f, by1 = 0.f, bz0 = 0.f, bz1 = 0.f;
    if (kIsF32 && fast) {
        bx0 = wave_min_uniform(valid ? xi : INFINITY);
        bx1 = wave_max_uniform(valid ? xi : -INFINITY);
        by0 = wave_min_uniform(valid ? yi : INFINITY);
        by1 = wave_max_uniform(valid ? yi : -INFINITY);
        bz0 = wave_min_uniform(valid ? zi : INFINITY);
        bz1 = wave_max_uniform(valid ? zi : -INFINITY);
    }

    if (kIsF32 && fast) {
        // The block's atoms are sorted by z and span [0, zext] in fixed point
        // relative to o.  Each of the 9 neighbour columns (distinct: at least
        // 4 cells per edge) is a z-sorted range of the sorted arrays; it is
        // cut by binary search to the atoms whose z lies in the padded
        // cutoff window [oz - reach, oz + zext + reach], one range, or two
        // where the window wraps around the periodic seam.
        const int nvalid = min(kPairWave, ce - cs - cb.y * kPairWave);
        const sfix rzi = static_cast<sfix>(ri.z - oz_);
        const sfix zext = __shfl(rzi, nvalid - 1, 64);
        // a partner within rc differs by at most rc / w_z in s_z (w_z the
        // distance between the cell's z faces; L_z for a box)
        double zspan;
        if constexpr (TRI)
            zspan = static_cast<double>(rcf) * sqrt(St.hi[6] * St.hi[6] + St.hi[7] * St.hi[7] + St.hi[8] * St.hi[8]);
        else
            zspan = static_cast<double>(rcf) / St.L[2];
        const uint32_t reach = static_cast<uint32_t>(ceil(zspan * 4294967296.0)) + 2u;
        const uint32_t za = static_cast<uint32_t>(oz_) - reach;
        const uint32_t zb = static_cast<uint32_t>(oz_) + static_cast<uint32_t>(zext) + reach;
        if (lane < 9) {
            const int dx = lane % 3 - 1, dy = lane / 3 - 1;
            const int jx = (cx + dx + nx) % nx, jy = (cy + dy + ny) % ny;
            const int col = nz * (jy + ny * jx);
            const int lo = start[col], hi = start[col + nz];
            const RB_GLOBAL uint32_t *zw = reinterpret_cast<const RB_GLOBAL uint32_t *>(gp(rec));
            // first atom of [l, h) with z >= v (above) or z > v (!above)
            auto search = [&](int l, int h, uint32_t v, bool above) {
                while (l < h) {
                    const int m = (l + h) >> 1;
                    const uint32_t zm = zw[4 * m + 2];
                    if (above ? zm < v : zm <= v) l = m + 1;
                    else h = m;
                }
                return l;
            };
            int b0, e0, b1, e1;
            if (za <= zb) {
                b0 = search(lo, hi, za, true);
                e0 = search(b0, hi, zb, false);
                b1 = e1 = lo;
            } else {
                b0 = search(lo, hi, za, true);
                e0 = hi;
                b1 = lo;
                e1 = search(lo, b0, zb, false);
            }
            // The block's own column (lane 4): on the relative-coordinate
            // path the block's atoms, a run inside one of its two pieces,
            // are cut out (their pairs are taken inside the block), and the
            // piece's part above them becomes range 18.
            int b2 = 0, e2 = 0, split = 0;
            if (kRelEval && lane == 4) {
                const int i1 = i0 + nblock;
                if (b0 <= i0 && i1 <= e0) {
                    b2 = i1;
                    e2 = e0;
                    e0 = i0;
                    split = 1;
                } else if (b1 <= i0 && i1 <= e1) {
                    b2 = i1;
                    e2 = e1;
                    e1 = i0;
                    split = 1;
                }
            }
            sh.beg[2 * lane] = b0;
            sh.pre[2 * lane + 1] = e0 - b0;  // lengths for now
            sh.beg[2 * lane + 1] = b1;
            sh.pre[2 * lane + 2] = e1 - b1;
            if (lane == 4) {
                sh.beg[18] = b2;
                sh.pre[19] = e2 - b2;
                sh.split = split;
            }
        } else if (lane >= 19 && lane < kMaxRanges) {
            sh.beg[lane] = 0;
            sh.pre[lane + 1] = 0;
        }
        __syncthreads();
        if (lane == 0) {
            sh.pre[0] = 0;
            for (int k = 0; k < kMaxRanges; ++k) sh.pre[k + 1] += sh.pre[k];
        }
    } else {
        // exact path: lanes 0 .. ncol - 1 each take one neighbour column and
        // its run of cells cz - 1 .. cz + gs (split where it wraps); a
        // dimension with fewer than three cells is taken whole.  A column
        // taken whole in z is cut (FP32) to the block's padded z-window as on
        // the fast path, unless the window covers it: the column is z-sorted
        // (cells in z order, each sorted by z), and displacements here are
        // exact minimum images whatever the window.
        const int ox = nx >= 3 ? 1 : 0, oy = ny >= 3 ? 1 : 0;
        const int wy = 2 * oy + 1, ncol = (2 * ox + 1) * wy;
        bool cut = false;
        uint32_t za = 0, zb = 0;
        if constexpr (kIsF32) {
            const int nvalid = min(kPairWave, ce - cs - cb.y * kPairWave);
            const uint32_t zext = __shfl(static_cast<uint32_t>(ri.z - oz_), nvalid - 1, 64);
            // a partner within rc differs by at most rc / w_z in s_z (w_z the
            // distance between the cell's z faces; L_z for a box)
            double zspan;
            if constexpr (TRI)
                zspan = static_cast<double>(rcf) *
                        sqrt(St.hi[6] * St.hi[6] + St.hi[7] * St.hi[7] + St.hi[8] * St.hi[8]);
            else
                zspan = static_cast<double>(rcf) / St.L[2];
            const uint32_t reach = static_cast<uint32_t>(ceil(zspan * 4294967296.0)) + 2u;
            cut = static_cast<uint64_t>(zext) + 2ull * reach < (1ull << 32);
            za = static_cast<uint32_t>(oz_) - reach;
            zb = static_cast<uint32_t>(oz_) + zext + reach;
        }
        if (lane < ncol) {
            const int dx = lane / wy - ox, dy = lane % wy - oy;
            const int jx = (cx + dx + nx) % nx, jy = (cy + dy + ny) % ny;
            const int col = nz * (jy + ny * jx);
            const int z0 = cz - 1, z1 = cz + gs;  // inclusive
            int b0, e0, b1 = 0, e1 = 0;
            if (nz < 3 || z1 - z0 + 1 >= nz) {
                b0 = start[col];
                e0 = start[col + nz];
                if (cut) {
                    const int lo = b0, hi = e0;
                    const RB_GLOBAL uint32_t *zw = reinterpret_cast<const RB_GLOBAL uint32_t *>(gp(rec));
                    auto search = [&](int l, int h, uint32_t v, bool above) {
                        while (l < h) {
                            const int m = (l + h) >> 1;
                            const uint32_t zm = zw[4 * m + 2];
                            if (above ? zm < v : zm <= v) l = m + 1;
                            else h = m;
                        }
                        return l;
                    };
                    if (za <= zb) {
                        b0 = search(lo, hi, za, true);
                        e0 = search(b0, hi, zb, false);
                    } else {
                        b0 = search(lo, hi, za, true);
                        e0 = hi;
                        b1 = lo;
                        e1 = search(lo, b0, zb, false);
                    }
                }
            } else if (z0 < 0) {
                b0 = start[col + nz - 1];
                e0 = start[col + nz];
                b1 = start[col];
                e1 = start[col + z1 + 1];
            } else if (z1 >= nz) {
                b0 = start[col + z0];
                e0 = start[col + nz];
                b1 = start[col];
                e1 = start[col + z1 - nz + 1];
            } else {
                b0 = start[col + z0];
                e0 = start[col + z1 + 1];
            }
            sh.beg[2 * lane] = b0;
            sh.pre[2 * lane + 1] = e0 - b0;  // lengths for now
            sh.beg[2 * lane + 1] = b1;
            sh.pre[2 * lane + 2] = e1 - b1;
        } else if (lane >= 2 * ncol && lane < kMaxRanges) {
            sh.beg[lane] = 0;
            sh.pre[lane + 1] = 0;
        }
        __syncthreads();
        if (lane == 0) {
            sh.pre[0] = 0;
            for (int k = 0; k < kMaxRanges; ++k) sh.pre[k + 1] += sh.pre[k];
        }
    }
    __syncthreads();
    const int total = sh.pre[kMaxRanges];
    // Candidates go to the chunks in groups of 4 consecutive records, group g to
    // chunk g mod nch: every chunk samples the whole neighbourhood, so each
    // lane's share of partners is about the same in every chunk and the lanes
    // of a wavefront run out of partners together.
    const int ngroups = (total + 3) / 4;
    const int gpc = kChunk / 4;
    const int nch = (ngroups + gpc - 1) / gpc;

    // chunk ch's groups: ch, ch + nch, ...; slots k of the chunk map to
    // flattened indices 4 (ch + nch (k/4)) + k%4, a prefix of them valid
    auto chunk_filled = [&](int ch) {
        const int ng = ch < ngroups ? (ngroups - ch + nch - 1) / nch : 0;
        const int glast = ch + nch * (ng - 1);
        return ng > 0 ? 4 * (ng - 1) + min(4, total - 4 * glast) : 0;
    };
    // the range holding flattened index f: the last r with pre[r] <= f
    auto range_of = [&](int f) {
        int r = 0;
#pragma unroll
        for (int step = 16; step >= 1; step >>= 1)
            if (r + step < kMaxRanges && sh.pre[r + step] <= f) r += step;
        return r;
    };

    double fx = 0, fy = 0, fz = 0, v[6] = {0, 0, 0, 0, 0, 0}, uu = 0;
    int hits = 0;    // in-cutoff partners of this lane's atom
    int hits_w = 0;  // in-cutoff pairs counted for the whole wavefront (relative-coordinate walk)
    // Sentinels of the relative-coordinate walk: far enough that no pair with
    // them is inside rc, near enough that every product stays finite, charge 0.
    if (kRelEval && fast && lane < kChunk / 32) sh.rtile[33 * lane] = make_float4(1e15f, 1e15f, 1e15f, 0.0f);

    // Pairs inside the block (relative-coordinate path): each unordered pair
    // once, by Newton's third law within the wavefront.  In round t lane l
    // meets lane l + t (mod 64), t = 1 .. 32 (t = 32 for l < 32 only), and
    // lane l + t takes the reaction from it by a shuffle, so every sum keeps
    // a fixed order.  The virial and the count of such a pair go in twice,
    // as the full shell's other side would have.  The block's atoms are then
    // cut out of its neighbour ranges (without that cut, which needs them to
    // be one run inside one piece of their column, the phase is skipped).
    const bool intra = kRelEval && kIsF32 && fast && sh.split;
    if constexpr (kRelEval) {
        if (intra) {
            const float qf = valid ? static_cast<float>(ri.q) : 0.0f;
            PairAcc<T> ia;
            for (int t = 1; t <= 32; ++t) {
                const int j = (lane + t) & 63;
                const float xj = __shfl(xi, j, 64), yj = __shfl(yi, j, 64), zj = __shfl(zi, j, 64);
                const float qj = __shfl(qf, j, 64);
                const float dx = xi - xj, dy = yi - yj, dz = zi - zj;
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const bool act = valid & (j < nblock) & ((t < 32) | (lane < 32)) & (r2 < rc2) & (r2 > 0.0f);
                const float k = act ? sog_force_factor<T, M>(r2, W) : 0.0f;
                const float fq = k * qj;
                const float fdx = fq * dx, fdy = fq * dy, fdz = fq * dz;
                const float dx2 = dx + dx, dy2 = dy + dy, dz2 = dz + dz;
                ia.fx += fdx;
                ia.fy += fdy;
                ia.fz += fdz;
                ia.vxx += fdx * dx2;
                ia.vyy += fdy * dy2;
                ia.vzz += fdz * dz2;
                ia.vxy += fdx * dy2;
                ia.vxz += fdx * dz2;
                ia.vyz += fdy * dz2;
                ia.n += act ? 2 : 0;
                // the reaction carries this lane's charge; lane l takes it from lane l - t
                const float kq = k * qf;
                const int src = (lane - t) & 63;
                ia.fx -= __shfl(kq * dx, src, 64);
                ia.fy -= __shfl(kq * dy, src, 64);
                ia.fz -= __shfl(kq * dz, src, 64);
            }
            const double qi = ri.q;
            hits += ia.n;
            fx += qi * ia.fx;
            fy += qi * ia.fy;
            fz += qi * ia.fz;
            v[0] += qi * ia.vxx;
            v[1] += qi * ia.vyy;
            v[2] += qi * ia.vzz;
            v[3] += qi * ia.vxy;
            v[4] += qi * ia.vxz;
            v[5] += qi * ia.vyz;
        }
    }

    for (int ch = 0; ch < nch; ++ch) {
        int filled = chunk_filled(ch);
        if (fast) {
            // Candidates farther than the padded cutoff from the block's
            // bounding box cannot pass the filter for any lane: they are
            // dropped here, and the survivors are packed in their order (the
            // walk then meets every pair in the same order as without the cut).
            int kept = 0;
            for (int k0 = 0; k0 < filled; k0 += 64) {
                const int k = k0 + lane;
                bool keep = false;
                Rec rj{};
                float xj = 0.f, yj = 0.f, zj = 0.f;
                if (k < filled) {
                    const int f = 4 * (ch + nch * (k >> 2)) + (k & 3);
                    const int r = range_of(f);
                    rj = gload(rec + sh.beg[r] + (f - sh.pre[r]));
                    relpos(rj, xj, yj, zj);
                    const float ex = fmaxf(fmaxf(bx0 - xj, xj - bx1), 0.f);
                    const float ey = fmaxf(fmaxf(by0 - yj, yj - by1), 0.f);
                    const float ez = fmaxf(fmaxf(bz0 - zj, zj - bz1), 0.f);
                    keep = fmaf(ez, ez, fmaf(ey, ey, ex * ex)) < rcf * rcf;
                }
                const uint64_t bal = __ballot(keep);
                if (keep) {
                    const int pos = kept + __popcll(bal & ((1ull << lane) - 1ull));
                    sh.rel[pos] = make_float4(xj, yj, zj, xj * xj + yj * yj + zj * zj);
                    if constexpr (kRelEval) sh.rtile[rel_slot(pos)] = make_float4(xj, yj, zj, static_cast<float>(rj.q));
                    else sh.tile[pos] = rj;
                }
                kept += __popcll(bal);
            }
            filled = kept;
        } else {
            for (int k = lane; k < filled; k += 64) {
                const int f = 4 * (ch + nch * (k >> 2)) + (k & 3);
                const int r = range_of(f);
                const Rec rj = gload(rec + sh.beg[r] + (f - sh.pre[r]));
                sh.tile[k] = rj;
                if constexpr (kIsF32 && !FAST && !TRI) sh.pk[k] = pack16(rj);
            }
        }
        // the filter reads whole 32-candidate words: padding candidates never pass
        const int words = (filled + 31) >> 5;
        if (fast)
            for (int k = filled + lane; k < 32 * words; k += 64) {
                sh.rel[k] = make_float4(0.f, 0.f, 0.f, INFINITY);
                if constexpr (!kRelEval) sh.rtile[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        __syncthreads();

        // Filter: one hit bit per candidate, shifted in so that the first
        // candidate of a word ends up in its top bit.  Nothing is written
        // per candidate; each lane stores its words, then walks their set bits.
        for (int w = 0; w < words; ++w) {
            uint32_t m = 0;
            if (fast) {
                // groups of four, the next group's loads issued before this
                // group's tests so that the LDS latency overlaps the arithmetic
                float4 nb[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) nb[k] = sh.rel[32 * w + k];
#pragma unroll
                for (int g = 0; g < 8; ++g) {
                    float4 c[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) c[k] = nb[k];
                    if (g < 7) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) nb[k] = sh.rel[32 * w + 4 * (g + 1) + k];
                    }
                    float t[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        t[k] = fmaf(c[k].x, ax, fmaf(c[k].y, ay, fmaf(c[k].z, az, c[k].w)));
                    }
                    m = push_hits4(m, t[0], t[1], t[2], t[3], thr);
                }
            } else if constexpr (kIsF32 && !FAST && !TRI) {
                // The top 16 bits of the fixed-point coordinates wrap like the
                // box, so their 16-bit differences are minimum images in units
                // u_d = L_d / 2^16; a pair inside rc has sum (d_d/u_d)^2 below
                // St.thr16 (at most 2^30).  The two-term integer dot products
                // add the squares exactly: their wrapped int32 sum is the true
                // sum, below 2^32, read as unsigned.
                const uint2 pi = pack16(ri);
                const uint32_t thr16 = valid ? St.thr16 : 0u;
#pragma unroll
                for (int g = 0; g < 8; ++g) {
                    uint2 c[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) c[k] = sh.pk[32 * w + 4 * g + k];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const short2v dxy = as_short2(pi.x) - as_short2(c[k].x);
                        const short2v dz = as_short2(pi.y) - as_short2(c[k].y);
                        const int r = __builtin_amdgcn_sdot2(dz, dz, __builtin_amdgcn_sdot2(dxy, dxy, 0, false), false);
                        m = m + m + static_cast<uint32_t>(static_cast<uint32_t>(r) < thr16);
                    }
                }
                const int nv = filled - 32 * w;  // candidates of this word; the rest are stale slots
                if (nv < 32) m &= ~0u << (32 - nv);
            } else {
                const int s_end = min(filled, 32 * w + 32);
                for (int s = 32 * w; s < 32 * w + 32; ++s) {
                    bool hit = false;
                    if (s < s_end) {
                        real dx, dy, dz;
                        if constexpr (TRI) displacement_cell<T>(ri, sh.tile[s], hm, unit, dx, dy, dz);
                        else displacement<T>(ri, sh.tile[s], sx, sy, sz, dx, dy, dz);
                        const real d2 = dx * dx + dy * dy + dz * dz;
                        hit = (d2 < rc2_lane) & (d2 > 0);
                    }
                    m = m + m + static_cast<uint32_t>(hit);
                }
            }
            sh.mask[w][lane] = m;
        }

        // Evaluation: every lane takes its hits from its current word in
        // candidate order (the first candidate sits in the top bit), two per round; lanes whose word is spent move to their
        // next word (their own LDS entries, no barrier needed).  Every lane
        // runs both evaluations of a round (a wavefront issues them anyway),
        // a lane without a hit masked off, so no branch splits the round.
        PairAcc<T> acc;
        auto walk = [&](auto rel_tag) {
            constexpr bool kRel = decltype(rel_tag)::value;
            int w = 0;
            // byte offset in the relative tile of candidate 32 w (slot 33 w + 1)
            int wb = static_cast<int>(sizeof(float4));
            uint32_t cur = words > 0 ? sh.mask[0][lane] : 0u;
            for (;;) {
                bool adv = (cur == 0u) & (w + 1 < words);
                if (__any(adv)) {  // a lane's word is spent and it has more: the rarer case
                    do {
                        if (adv) {
                            ++w;
                            wb += 33 * static_cast<int>(sizeof(float4));
                            cur = sh.mask[w][lane];
                        }
                        adv = (cur == 0u) & (w + 1 < words);
                    } while (__any(adv));
                }
                if (!__any(cur != 0u)) break;
                if constexpr (kRel) {
                    // The leading set bit; a spent word gives -1 (the hardware's
                    // result for zero), the word's sentinel slot, whose pair
                    // fails the cutoff test.  Clearing bit (k & 31) leaves a
                    // spent word at zero.
                    int k0, k1;
                    asm("v_ffbh_u32 %0, %1" : "=v"(k0) : "v"(cur));
                    cur &= ~(0x80000000u >> (k0 & 31));
                    asm("v_ffbh_u32 %0, %1" : "=v"(k1) : "v"(cur));
                    cur &= ~(0x80000000u >> (k1 & 31));
                    // FP32 block-relative coordinates: the difference of two exact
                    // minimum-image offsets from o, each rounded once to FP32
                    const char *tb = reinterpret_cast<const char *>(sh.rtile) + wb;
                    const float4 t0 = *reinterpret_cast<const float4 *>(tb + k0 * static_cast<int>(sizeof(float4)));
                    const float4 t1 = *reinterpret_cast<const float4 *>(tb + k1 * static_cast<int>(sizeof(float4)));
                    uint64_t in0, in1;
                    pair_eval_d<T, M, E, false>(xi - t0.x, yi - t0.y, zi - t0.z, t0.w, true, rc2, W, acc, &in0);
                    pair_eval_d<T, M, E, false>(xi - t1.x, yi - t1.y, zi - t1.z, t1.w, true, rc2, W, acc, &in1);
                    hits_w += __popcll(in0) + __popcll(in1);
                } else {
                    // a spent word gives slot 31, a valid record, masked off by active
                    const bool a0 = cur != 0u;
                    const int k0 = __builtin_clz(cur | 1u);
                    cur &= ~(0x80000000u >> k0);
                    const bool a1 = cur != 0u;
                    const int k1 = __builtin_clz(cur | 1u);
                    cur &= ~(0x80000000u >> k1);
                    const Rec r0 = sh.tile[32 * w + k0], r1 = sh.tile[32 * w + k1];
                    if constexpr (TRI) {
                        pair_eval_cell<T, M, E>(ri, r0, a0, hm, unit, rc2, W, acc);
                        pair_eval_cell<T, M, E>(ri, r1, a1, hm, unit, rc2, W, acc);
                    } else {
                        pair_eval<T, M, E>(ri, r0, a0, sx, sy, sz, rc2, W, acc);
                        pair_eval<T, M, E>(ri, r1, a1, sx, sy, sz, rc2, W, acc);
                    }
                }
            }
        };
        if (kIsF32 && fast) walk(std::integral_constant<bool, kRelEval>{});
        else walk(std::false_type{});
        const double qi = ri.q;
        hits += acc.n;
        fx += qi * acc.fx;
        fy += qi * acc.fy;
        fz += qi * acc.fz;
        v[0] += qi * acc.vxx;
        v[1] += qi * acc.vyy;
        v[2] += qi * acc.vzz;
        v[3] += qi * acc.vxy;
        v[4] += qi * acc.vxz;
        v[5] += qi * acc.vyz;
        uu += qi * acc.u;
        __syncthreads();
    }
    if (valid) {
        RB_GLOBAL real *fsr = gp(static_cast<real *>(D.fsr));
        fsr[i] = static_cast<real>(fx);
        fsr[D.n + i] = static_cast<real>(fy);
        fsr[2 * D.n + i] = static_cast<real>(fz);
    }
    // full shell: each pair was seen from both sides
    hits += lane == 0 ? hits_w : 0;
    double out[8] = {0.5 * v[0], 0.5 * v[1], 0.5 * v[2], 0.5 * v[3], 0.5 * v[4], 0.5 * v[5], 0.5 * uu, 0.5 * hits};
    for (int k = 0; k < 8; ++k) out[k] = wave_sum(out[k]);
    if (lane == 0)
        for (int k = 0; k < 8; ++k) gp(part)[k] = out[k];
}

// ----------------------------------------------------------------------------
// Half-shell pair kernel (FP32 fast path): every unordered pair evaluated once
// ----------------------------------------------------------------------------
//
// Newton's third law halves the SOG evaluations and the filter tests.  A block
// takes its own column from its first atom up to the top of its padded
// z-window (a candidate in the block itself only when it follows the lane's
// atom in the sorted order) and the four neighbour columns (+1,-1), (+1,0),
// (+1,+1), (0,+1), each cut to the window; with at least four cells per edge
// every unordered pair inside rc is then visited by exactly one block.  The
// lane's own force accumulates in registers as in the full shell.  The
// reaction on the candidate accumulates per chunk in FP64 in the wavefront's
// own LDS (ds_add_f64; the lanes of one instruction that add to one slot are
// applied in a fixed order and no other wavefront touches the region, so the
// sums are the same bits on every run), and goes out as FP32 to the block's
// slot of a partial buffer, indexed by the candidate's position in the
// block's neighbourhood.  k_pair_gather then adds, for every atom, the
// partials of every block that listed it to its own block's sum, in a fixed
// order.  Blocks whose neighbourhood exceeds the buffer's hcap candidates mark
// their system in k_pair_prep; such a system runs the full shell that step.
//
// Candidates are dealt to chunks in groups of kHalfGroup consecutive records
// (group g to chunk g mod nch): every chunk still samples the whole
// neighbourhood, and the partials are written and read in 64-byte runs.

constexpr int kHalfRanges = 10;  // own column (above the block, wrapped part), 4 columns x 2 pieces
constexpr int kHalfGroup = 16;
static_assert(kHalfGroup == 16 && kChunk % 32 == 0, "a hit word holds two candidate groups");
static_assert(kHrngStride >= 2 * kHalfRanges + 2, "neighbourhood table entry");

// forward neighbour column r = 0..3: (dx, dy) = (1,-1), (1,0), (1,1), (0,1)
__device__ __forceinline__ int fwd_dx(int r) { return r < 3 ? 1 : 0; }
__device__ __forceinline__ int fwd_dy(int r) { return r < 3 ? r - 1 : 1; }

// Padded cutoff of the FP32 fast filter and the z reach of a block's window
// in fixed-point units (the same in every kernel that cuts windows).
__device__ __forceinline__ float fast_rcf(const SysDesc &D)
{
    return static_cast<float>(sqrt(static_cast<double>(D.tab.rc2_32))) + 1e-3f;
}
__device__ __forceinline__ uint32_t window_reach(const SysDesc &D, const SysStep &St)
{
    return static_cast<uint32_t>(ceil(static_cast<double>(fast_rcf(D)) / St.L[2] * 4294967296.0)) + 2u;
}

// first index of [l, h) whose z (fixed point) is >= v (above) or > v (!above)
__device__ __forceinline__ int z_search(const RB_GLOBAL uint32_t *zw, int l, int h, uint32_t v, bool above)
{
    while (l < h) {
        const int m = (l + h) >> 1;
        const uint32_t zm = zw[4 * m + 2];
        if (above ? zm < v : zm <= v) l = m + 1;
        else h = m;
    }
    return l;
}

// The half-shell neighbourhood of every pair block: range starts beg[10],
// flattened prefixes pre[11] (pre[10] = total), chunk count.
__global__ __launch_bounds__(64) void k_pair_prep(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                  const int2 *__restrict__ plan)
{
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const SysStep &St = stp[e.x];
    const int b = e.y;
    const int lane = threadIdx.x;
    const RB_GLOBAL int32_t *start = gp(D.start);
    if (b >= gp(D.bstart)[St.ncells]) return;
    const int nx = St.nc[0], ny = St.nc[1], nz = St.nc[2];
    const int2 cb = gload(D.blocks + b);
    const int c = cb.x;
    const int cz = c % nz, cy = (c / nz) % ny, cx = c / (nz * ny);
    const int gs = min(St.g, nz - cz);
    const int cs = start[c], ce = start[c + gs];
    const int i0 = cs + cb.y * kPairWave;
    const int nvalid = min(kPairWave, ce - i0);
    const RB_GLOBAL uint32_t *zw = reinterpret_cast<const RB_GLOBAL uint32_t *>(gp(D.rec));
    const uint32_t oz = zw[4 * i0 + 2];
    const uint32_t zext = zw[4 * (i0 + nvalid - 1) + 2] - oz;  // a segment is sorted by z
    const uint32_t reach = window_reach(D, St);
    const uint32_t za = oz - reach, zb = oz + zext + reach;
    int b0 = 0, e0 = 0, b1 = 0, e1 = 0;
    if (lane == 0) {
        // own column: from the block's first atom to the window's top, and the
        // part past the periodic seam
        const int col = nz * (cy + ny * cx);
        const int lo = start[col], hi = start[col + nz];
        b0 = i0;
        if (static_cast<uint64_t>(oz) + zext + reach < (1ull << 32)) {
            e0 = z_search(zw, i0, hi, zb, false);
        } else {
            e0 = hi;
            b1 = lo;
            e1 = z_search(zw, lo, i0, zb, false);
        }
    } else if (lane <= 4) {
        const int r = lane - 1;
        const int jx = (cx + fwd_dx(r) + nx) % nx, jy = (cy + fwd_dy(r) + ny) % ny;
        const int col = nz * (jy + ny * jx);
        const int lo = start[col], hi = start[col + nz];
        b0 = z_search(zw, lo, hi, za, true);
        if (za <= zb) {
            e0 = z_search(zw, b0, hi, zb, false);
        } else {
            e0 = hi;
            b1 = lo;
            e1 = z_search(zw, lo, b0, zb, false);
        }
    }
    int beg[kHalfRanges], len[kHalfRanges];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        beg[2 * r] = __shfl(b0, r, 64);
        len[2 * r] = __shfl(e0 - b0, r, 64);
        beg[2 * r + 1] = __shfl(b1, r, 64);
        len[2 * r + 1] = __shfl(e1 - b1, r, 64);
    }
    if (lane == 0) {
        RB_GLOBAL int32_t *h = gp(D.hrng) + static_cast<int64_t>(b) * kHrngStride;
        int pre = 0;
        for (int r = 0; r < kHalfRanges; ++r) {
            h[r] = beg[r];
            h[kHalfRanges + r] = pre;
            pre += len[r];
        }
        h[2 * kHalfRanges] = pre;
        const int ngroups = (pre + kHalfGroup - 1) / kHalfGroup;
        constexpr int gpc = kChunk / kHalfGroup;
        h[2 * kHalfRanges + 1] = (ngroups + gpc - 1) / gpc;
        if (pre > D.hcap) atomicOr(D.hflag, 1);
    }
}

template <class T, bool E>
struct PairSharedHalf {
    float4 rt[kChunk];                        // (x, y, z) relative to the block origin, q
    float r2[kChunk];                         // |r_j|^2 for the filter
    typename T::Rec tile[E ? kChunk : 1];     // fixed-point records (the energy sum's displacements)
    double jac[3][kChunk];                    // reactions on the chunk's candidates
    uint32_t mask[kChunk / 32][64];           // hit bits of each lane
    int beg[kHalfRanges];
    int pre[kHalfRanges + 1];
};

// One pair's SOG terms with the charge product qij = q_i q_j applied: adds the
// force on i, the virial and the energy to acc and returns the force on i in
// (fx, fy, fz) (the reaction on j is its negative).
template <class T, int M, bool E>
__device__ __forceinline__ void pair_eval_r(float dx, float dy, float dz, float qij, bool active, float rc2,
                                            const Weights<T, M> &W, PairAcc<T> &acc, float &fx, float &fy,
                                            float &fz)
{
    const float r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const bool inside = active & (r2 < rc2) & (r2 > 0.0f);
    float swt = 0.0f, sw = 0.0f;
    const float rinv = __builtin_amdgcn_rsqf(r2);
    if constexpr (M == -1) {
        const float t = r2 * W.pa - 1.0f;
        swt = horner(W.pg, t);
        if constexpr (E) sw = horner(W.pf, t);
    } else if constexpr (M == 0) {
        for (int l = 0; l < W.m; ++l) {
            float wl;
            swt += gauss<T, M, E>(W, l, r2, wl);
            if constexpr (E) sw += wl;
        }
    } else {
#pragma unroll
        for (int l = 0; l < M; ++l) {
            float wl;
            swt += gauss<T, M, E>(W, l, r2, wl);
            if constexpr (E) sw += wl;
        }
    }
    acc.n += inside;
    const float f = inside ? qij * (rinv * rinv * rinv - swt) : 0.0f;
    fx = f * dx;
    fy = f * dy;
    fz = f * dz;
    acc.fx += fx;
    acc.fy += fy;
    acc.fz += fz;
    acc.vxx += fx * dx;
    acc.vyy += fy * dy;
    acc.vzz += fz * dz;
    acc.vxy += fx * dy;
    acc.vxz += fx * dz;
    acc.vyz += fy * dz;
    if constexpr (E) acc.u += inside ? qij * (rinv - sw) : 0.0f;
}

// One half-shell pair block b of system D (one wavefront), FP32 fast path.
template <class T, int M, bool E>
__device__ __forceinline__ void pair_block_half(PairSharedHalf<T, E> &sh, const SysDesc &D, const SysStep &St, int b)
{
    using Rec = typename T::Rec;
    const int lane = threadIdx.x;
    const int ncells = St.ncells;
    const int nb_total = gp(D.bstart)[ncells];
    double *part = D.pair_part + 8 * static_cast<int64_t>(b);
    if (b >= nb_total) return;
    const Rec *__restrict__ rec = static_cast<const Rec *>(D.rec);
    Weights<T, M> W;
    load_weights<T, M>(W, &D.tab);
    const int nz = St.nc[2];
    const float sx = static_cast<float>(St.L[0] * 0x1.0p-32);
    const float sy = static_cast<float>(St.L[1] * 0x1.0p-32);
    const float sz = static_cast<float>(St.L[2] * 0x1.0p-32);
    const float rc2 = D.tab.rc2_32;
    const RB_GLOBAL int32_t *start = gp(D.start);
    const int2 cb = gload(D.blocks + b);
    const int c = cb.x;
    const int cz = c % nz;
    const int gs = min(St.g, nz - cz);
    const int cs = start[c], ce = start[c + gs];
    const int i = cs + cb.y * kPairWave + lane;
    const bool valid = i < ce;
    Rec ri{};
    if (valid) ri = gload(rec + i);
    const uint32_t ox = static_cast<uint32_t>(__shfl(static_cast<int>(ri.x), 0, 64));
    const uint32_t oy = static_cast<uint32_t>(__shfl(static_cast<int>(ri.y), 0, 64));
    const uint32_t oz = static_cast<uint32_t>(__shfl(static_cast<int>(ri.z), 0, 64));
    const float rcf = fast_rcf(D);
    const float xi = static_cast<float>(static_cast<int32_t>(ri.x - ox)) * sx;
    const float yi = static_cast<float>(static_cast<int32_t>(ri.y - oy)) * sy;
    const float zi = static_cast<float>(static_cast<int32_t>(ri.z - oz)) * sz;
    const float ax = -2.0f * xi, ay = -2.0f * yi, az = -2.0f * zi;
    const float thr = valid ? rcf * rcf - (xi * xi + yi * yi + zi * zi) : -INFINITY;
    const float qi = valid ? ri.q : 0.0f;

    // the neighbourhood from k_pair_prep
    const RB_GLOBAL int32_t *h = gp(D.hrng) + static_cast<int64_t>(b) * kHrngStride;
    if (lane < kHalfRanges) sh.beg[lane] = h[lane];
    if (lane <= kHalfRanges) sh.pre[lane] = h[kHalfRanges + lane];
    for (int k = lane; k < kChunk; k += 64) {
        sh.jac[0][k] = 0.0;
        sh.jac[1][k] = 0.0;
        sh.jac[2][k] = 0.0;
    }
    __syncthreads();
    const int total = sh.pre[kHalfRanges];
    const int len0 = sh.pre[1];
    constexpr int gpc = kChunk / kHalfGroup;
    const int ngroups = (total + kHalfGroup - 1) / kHalfGroup;
    const int nch = (ngroups + gpc - 1) / gpc;
    const int hcap = D.hcap;
    RB_GLOBAL float *hp = gp(D.hpart) + static_cast<int64_t>(b) * 3 * hcap;

    double fx = 0, fy = 0, fz = 0, v[6] = {0, 0, 0, 0, 0, 0}, uu = 0;
    int hits = 0;
    // chunk ch holds the groups ch, ch + nch, ...: slot k is flattened index
    // kHalfGroup (ch + nch (k / kHalfGroup)) + k % kHalfGroup, a prefix of them valid
    auto flat = [&](int ch, int k) { return kHalfGroup * (ch + nch * (k / kHalfGroup)) + k % kHalfGroup; };
    auto chunk_filled = [&](int ch) {
        const int ng = ch < ngroups ? (ngroups - ch + nch - 1) / nch : 0;
        const int glast = ch + nch * (ng - 1);
        return ng > 0 ? kHalfGroup * (ng - 1) + min(kHalfGroup, total - kHalfGroup * glast) : 0;
    };
    for (int ch = 0; ch < nch; ++ch) {
        const int filled = chunk_filled(ch);
        for (int k = lane; k < filled; k += 64) {
            const int f = flat(ch, k);
            int r = 0;
#pragma unroll
            for (int step = 8; step >= 1; step >>= 1)
                if (r + step < kHalfRanges && sh.pre[r + step] <= f) r += step;
            const Rec rj = gload(rec + sh.beg[r] + (f - sh.pre[r]));
            const float xj = static_cast<float>(static_cast<int32_t>(rj.x - ox)) * sx;
            const float yj = static_cast<float>(static_cast<int32_t>(rj.y - oy)) * sy;
            const float zj = static_cast<float>(static_cast<int32_t>(rj.z - oz)) * sz;
            sh.rt[k] = make_float4(xj, yj, zj, rj.q);
            sh.r2[k] = xj * xj + yj * yj + zj * zj;
            if constexpr (E) sh.tile[k] = rj;
        }
        const int words = (filled + 31) >> 5;
        for (int k = filled + lane; k < 32 * words; k += 64) {
            sh.rt[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            sh.r2[k] = INFINITY;
            if constexpr (E) sh.tile[k] = Rec{};
        }
        __syncthreads();

        for (int w = 0; w < words; ++w) {
            uint32_t m = 0;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                float t[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float4 cj = sh.rt[32 * w + 4 * g + k];
                    t[k] = fmaf(cj.x, ax, fmaf(cj.y, ay, fmaf(cj.z, az, sh.r2[32 * w + 4 * g + k])));
                }
                m = push_hits4(m, t[0], t[1], t[2], t[3], thr);
            }
            // own-column candidates at or below the lane's atom are not its
            // forward partners: the first min(lane + 1, len0) - lo slots of a
            // group starting at flattened index lo < 64
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int lo = kHalfGroup * (ch + nch * (2 * w + hh));
                if (lo < min(len0, kPairWave)) {
                    const int cnt = min(max(min(lane + 1, len0) - lo, 0), kHalfGroup);
                    const uint32_t ex = cnt > 0 ? (0xFFFFu << (16 - cnt)) & 0xFFFFu : 0u;
                    m &= ~(ex << (16 * (1 - hh)));
                }
            }
            sh.mask[w][lane] = m;
        }

        // walk the hit bits, two per round; lanes start at different words
        // so that fewer of them add to one candidate at once
        PairAcc<T> acc;
        {
            int w = words > 0 ? lane % words : 0;
            int seen = 1;
            uint32_t cur = words > 0 ? sh.mask[w][lane] : 0u;
            for (;;) {
                bool adv = (cur == 0u) & (seen < words);
                while (__any(adv)) {
                    if (adv) {
                        w = w + 1 == words ? 0 : w + 1;
                        ++seen;
                        cur = sh.mask[w][lane];
                    }
                    adv = (cur == 0u) & (seen < words);
                }
                if (!__any(cur != 0u)) break;
                const bool a0 = cur != 0u;
                const int k0 = 32 * w + __builtin_clz(cur | 1u);
                cur &= ~(0x80000000u >> (k0 - 32 * w));
                const bool a1 = cur != 0u;
                const int k1 = 32 * w + __builtin_clz(cur | 1u);
                cur &= ~(0x80000000u >> (k1 - 32 * w));
                float f0x, f0y, f0z, f1x, f1y, f1z;
                if constexpr (E) {
                    float dx, dy, dz;
                    const Rec r0 = sh.tile[k0], r1 = sh.tile[k1];
                    displacement<T>(ri, r0, sx, sy, sz, dx, dy, dz);
                    pair_eval_r<T, M, E>(dx, dy, dz, qi * r0.q, a0, rc2, W, acc, f0x, f0y, f0z);
                    displacement<T>(ri, r1, sx, sy, sz, dx, dy, dz);
                    pair_eval_r<T, M, E>(dx, dy, dz, qi * r1.q, a1, rc2, W, acc, f1x, f1y, f1z);
                } else {
                    const float4 t0 = sh.rt[k0], t1 = sh.rt[k1];
                    pair_eval_r<T, M, E>(xi - t0.x, yi - t0.y, zi - t0.z, qi * t0.w, a0, rc2, W, acc, f0x, f0y, f0z);
                    pair_eval_r<T, M, E>(xi - t1.x, yi - t1.y, zi - t1.z, qi * t1.w, a1, rc2, W, acc, f1x, f1y, f1z);
                }
                if (a0) {
                    atomicAdd(&sh.jac[0][k0], -static_cast<double>(f0x));
                    atomicAdd(&sh.jac[1][k0], -static_cast<double>(f0y));
                    atomicAdd(&sh.jac[2][k0], -static_cast<double>(f0z));
                }
                if (a1) {
                    atomicAdd(&sh.jac[0][k1], -static_cast<double>(f1x));
                    atomicAdd(&sh.jac[1][k1], -static_cast<double>(f1y));
                    atomicAdd(&sh.jac[2][k1], -static_cast<double>(f1z));
                }
            }
        }
        hits += acc.n;
        fx += acc.fx;
        fy += acc.fy;
        fz += acc.fz;
        v[0] += acc.vxx;
        v[1] += acc.vyy;
        v[2] += acc.vzz;
        v[3] += acc.vxy;
        v[4] += acc.vxz;
        v[5] += acc.vyz;
        uu += acc.u;
        __syncthreads();
        // the chunk's reactions to the block's partial slots, then cleared
        for (int k = lane; k < 32 * words; k += 64) {
            if (k < filled) {
                const int f = flat(ch, k);
                hp[f] = static_cast<float>(sh.jac[0][k]);
                hp[hcap + f] = static_cast<float>(sh.jac[1][k]);
                hp[2 * hcap + f] = static_cast<float>(sh.jac[2][k]);
            }
            sh.jac[0][k] = 0.0;
            sh.jac[1][k] = 0.0;
            sh.jac[2][k] = 0.0;
        }
        __syncthreads();
    }
    if (valid) {
        RB_GLOBAL float *fsr = gp(static_cast<float *>(D.fsr));
        fsr[i] = static_cast<float>(fx);
        fsr[D.n + i] = static_cast<float>(fy);
        fsr[2 * D.n + i] = static_cast<float>(fz);
    }
    // each unordered pair was evaluated once
    double out[8] = {v[0], v[1], v[2], v[3], v[4], v[5], uu, static_cast<double>(hits)};
    for (int k = 0; k < 8; ++k) out[k] = wave_sum(out[k]);
    if (lane == 0)
        for (int k = 0; k < 8; ++k) gp(part)[k] = out[k];
}

// Per atom of every half-shell block: its own block's sum plus the reactions
// that the blocks listing it left in their partial slots, in a fixed order
// (its own column's blocks, then the columns (-1,+1), (-1,0), (-1,-1), (0,-1),
// each by block index).
__global__ __launch_bounds__(64) void k_pair_gather(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                    const int2 *__restrict__ plan)
{
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const SysStep &St = stp[e.x];
    if (*gp(D.hflag)) return;  // the system ran the full shell this step
    const int b = e.y;
    const int lane = threadIdx.x;
    const RB_GLOBAL int32_t *start = gp(D.start);
    const RB_GLOBAL int32_t *bstart = gp(D.bstart);
    if (b >= bstart[St.ncells]) return;
    const int nx = St.nc[0], ny = St.nc[1], nz = St.nc[2];
    const int2 cb = gload(D.blocks + b);
    const int c = cb.x;
    const int cz = c % nz, cy = (c / nz) % ny, cx = c / (nz * ny);
    const int gs = min(St.g, nz - cz);
    const int cs = start[c], ce = start[c + gs];
    const int t0 = cs + cb.y * kPairWave, t1 = min(ce, t0 + kPairWave);
    const int i = t0 + lane;
    const bool valid = i < t1;
    RB_GLOBAL float *fsr = gp(static_cast<float *>(D.fsr));
    double f[3] = {0.0, 0.0, 0.0};
    if (valid) {
        f[0] = fsr[i];
        f[1] = fsr[D.n + i];
        f[2] = fsr[2 * D.n + i];
    }
    const int hcap = D.hcap;
    const RB_GLOBAL int32_t *hr = gp(D.hrng);
    const RB_GLOBAL float *hp = gp(D.hpart);
    for (int src = 0; src < 5; ++src) {
        int col;
        if (src == 0) {
            col = nz * (cy + ny * cx);
        } else {
            const int r = src - 1;
            const int jx = (cx - fwd_dx(r) + nx) % nx, jy = (cy - fwd_dy(r) + ny) % ny;
            col = nz * (jy + ny * jx);
        }
        const int p0 = 2 * src;  // the source blocks' pieces that lie in this block's column
        const int bs = bstart[col], be = bstart[col + nz];
        for (int sb0 = bs; sb0 < be; sb0 += 64) {
            bool hit = false;
            if (sb0 + lane < be) {
                const RB_GLOBAL int32_t *h = hr + static_cast<int64_t>(sb0 + lane) * kHrngStride;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int beg = h[p0 + q], n = h[kHalfRanges + p0 + q + 1] - h[kHalfRanges + p0 + q];
                    hit |= (n > 0) & (beg < t1) & (beg + n > t0);
                }
            }
            uint64_t mset = __ballot(hit);
            while (mset) {
                const int k = __ffsll(static_cast<unsigned long long>(mset)) - 1;
                mset &= mset - 1;
                const int64_t s = sb0 + k;
                const RB_GLOBAL int32_t *h = hr + s * kHrngStride;
                const RB_GLOBAL float *ps = hp + s * 3 * hcap;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int beg = h[p0 + q], pre = h[kHalfRanges + p0 + q];
                    const int n = h[kHalfRanges + p0 + q + 1] - pre;
                    if (valid && i >= beg && i < beg + n) {
                        const int fi = pre + (i - beg);
                        f[0] += ps[fi];
                        f[1] += ps[hcap + fi];
                        f[2] += ps[2 * hcap + fi];
                    }
                }
            }
        }
    }
    if (valid) {
        fsr[i] = static_cast<float>(f[0]);
        fsr[D.n + i] = static_cast<float>(f[1]);
        fsr[2 * D.n + i] = static_cast<float>(f[2]);
    }
}

// Static schedule: workgroup g runs plan entry g.
// Register budget of the FP32 pair kernel: RBSOG_PAIR_OCC waves per SIMD,
// with or without the energy sum.  At 5 waves the relative-coordinate kernel
// holds its state in 96 registers (100 with the energy sum) with no scratch;
// at 6 it spilled 40 bytes per lane (about 4e7 bytes of scratch traffic a
// launch on 1e6 atoms) and measured even with 5; 7 waves were slower.  FP64
// keeps the default.
template <class T, bool E>
constexpr int pair_min_waves() { return sizeof(typename T::real) == 4 ? RBSOG_PAIR_OCC : 1; }

// Workgroups go to the eight XCDs in turn (workgroup w to XCD w mod 8), each
// XCD with its own L2.  Consecutive plan entries are neighbouring blocks of one
// column, which stage the same neighbour records; this permutation cuts the
// plan into windows of 8 runs of kXcdRun entries and gives each XCD one run per
// window, so those re-reads meet one L2 (HBM fetches per launch fall about
// tenfold) while the idle entries at the end of an over-provisioned plan stay
// spread over all XCDs.  A permutation of the workgroups: no result changes.
constexpr int kXcd = 8, kXcdRun = 128;
__device__ inline int xcd_grouped(int w, int G)
{
    const int base = w / (kXcd * kXcdRun) * (kXcd * kXcdRun);
    const int n = min(kXcd * kXcdRun, G - base);  // entries in this window
    const int q = n / kXcd, r = n % kXcd;         // XCDs below r take q + 1 of them, the others q
    const int o = w - base, x = o % kXcd;
    return base + x * q + min(x, r) + o / kXcd;
}

template <class T, int M, bool E, bool FAST, bool TRI = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(pair_min_waves<T, E>()))) void k_pair(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                             const int2 *__restrict__ plan)
{
    __shared__ PairShared<T> sh;
    const int2 e = plan[xcd_grouped(blockIdx.x, gridDim.x)];
    pair_block<T, M, E, FAST, TRI>(sh, desc[e.x], stp[e.x], e.y);
}

// Half-shell launches: a system whose neighbourhoods outgrew the partial
// buffer this step (flag set by k_pair_prep) runs the full-shell fast path.
template <class T, bool E>
struct PairSmem {
    static constexpr size_t bytes =
        sizeof(PairShared<T>) > sizeof(PairSharedHalf<T, E>) ? sizeof(PairShared<T>) : sizeof(PairSharedHalf<T, E>);
};
template <class T, int M, bool E>
__device__ __forceinline__ void pair_block_hs(char *smem, const SysDesc &D, const SysStep &St, int b)
{
    if (*gp(D.hflag)) pair_block<T, M, E, true>(*reinterpret_cast<PairShared<T> *>(smem), D, St, b);
    else pair_block_half<T, M, E>(*reinterpret_cast<PairSharedHalf<T, E> *>(smem), D, St, b);
}

template <class T, int M, bool E>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(pair_min_waves<T, E>()))) void k_pair_half(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                  const int2 *__restrict__ plan)
{
    __shared__ __attribute__((aligned(16))) char smem[PairSmem<T, E>::bytes];
    const int2 e = plan[xcd_grouped(blockIdx.x, gridDim.x)];
    pair_block_hs<T, M, E>(smem, desc[e.x], stp[e.x], e.y);
}

template <class T, int M, bool E>
__global__ __launch_bounds__(64) void k_pair_half_queue(const SysDesc *__restrict__ desc,
                                                        const SysStep *__restrict__ stp,
                                                        const int2 *__restrict__ plan, int nitems, int32_t *ctrl)
{
    __shared__ __attribute__((aligned(16))) char smem[PairSmem<T, E>::bytes];
    for (;;) {
        int idx = 0;
        if (threadIdx.x == 0) idx = atomicAdd(&ctrl[0], 1);
        idx = __shfl(idx, 0, 64);
        if (idx >= nitems) break;
        const int2 e = plan[idx];
        pair_block_hs<T, M, E>(smem, desc[e.x], stp[e.x], e.y);
        __syncthreads();
    }
}

// Persistent schedule: a fixed number of workgroups take plan entries from a
// global counter (zeroed by k_zero) until all nitems are taken; every
// workgroup leaves once the counter has passed nitems.
template <class T, int M, bool E, bool FAST, bool TRI = false>
__global__ __launch_bounds__(64) void k_pair_queue(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                   const int2 *__restrict__ plan, int nitems, int32_t *ctrl)
{
    __shared__ PairShared<T> sh;
    for (;;) {
        int idx = 0;
        if (threadIdx.x == 0) idx = atomicAdd(&ctrl[0], 1);
        idx = __shfl(idx, 0, 64);
        if (idx >= nitems) break;
        const int2 e = plan[idx];
        pair_block<T, M, E, FAST, TRI>(sh, desc[e.x], stp[e.x], e.y);
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// Structure factors rho_d = sum_j q_j exp(2 pi i m_d . s_j)   (eq. rho_k)
// ----------------------------------------------------------------------------
//
// The phase m.u mod 2^32 of the 32-bit fixed-point fractional coordinate u is
// exact: with u = 2^16 h + l (h, l < 2^16) it is ((m.h) << 16) + m.l, six
// 24-bit multiply-adds.  The hardware sine and cosine take the phase in
// revolutions.  Each workgroup owns kSkChunk atoms of one system; its 256
// threads are (mode, slice) pairs, and the per-mode partial of the workgroup
// goes to global memory in FP64.

struct alignas(16) SkAtom32 {
    int hx, hy, hz;
    float q;
    int lx, ly, lz, pad;
};

__device__ inline void phase_sincos32(const int4 &m, const SkAtom32 &at, float &s, float &c)
{
    // 24-bit multiplies (full rate; |m| < 2^23, halves < 2^16).  The empty asm
    // keeps the compiler from moving the shift into the products, which would
    // turn them into 32-bit (quarter-rate) multiplies by (u & 0xffff0000).
    uint32_t hi = static_cast<uint32_t>(__mul24(m.x, at.hx) + __mul24(m.y, at.hy) + __mul24(m.z, at.hz));
    asm("" : "+v"(hi));
    const uint32_t lo = static_cast<uint32_t>(__mul24(m.x, at.lx) + __mul24(m.y, at.ly) + __mul24(m.z, at.lz));
    const uint32_t ph = (hi << 16) + lo;
    const float rev = static_cast<float>(static_cast<int32_t>(ph)) * 0x1.0p-32f;
    s = __builtin_amdgcn_sinf(rev);
    c = __builtin_amdgcn_cosf(rev);
}

__device__ inline void phase_sincos64(const int4 &m, const F64::Rec &r, double &s, double &c)
{
    const uint64_t ph = static_cast<uint64_t>(static_cast<int64_t>(m.x)) * r.x +
                        static_cast<uint64_t>(static_cast<int64_t>(m.y)) * r.y +
                        static_cast<uint64_t>(static_cast<int64_t>(m.z)) * r.z;
    const double rev = static_cast<double>(static_cast<int64_t>(ph)) * 0x1.0p-64;
    sincospi(2.0 * rev, &s, &c);
}

__device__ inline SkAtom32 split_atom(const F32::Rec &r)
{
    SkAtom32 at;
    at.hx = static_cast<int>(r.x >> 16);
    at.hy = static_cast<int>(r.y >> 16);
    at.hz = static_cast<int>(r.z >> 16);
    at.lx = static_cast<int>(r.x & 0xFFFFu);
    at.ly = static_cast<int>(r.y & 0xFFFFu);
    at.lz = static_cast<int>(r.z & 0xFFFFu);
    at.q = r.q;
    at.pad = 0;
    return at;
}

template <class T>
__global__ __launch_bounds__(256) void k_sk(const SysDesc *__restrict__ desc, const int2 *__restrict__ plan)
{
    using Atom = typename std::conditional<sizeof(typename T::real) == 4, SkAtom32, typename T::Rec>::type;
    __shared__ Atom s_at[256];
    __shared__ double s_red[2][256];
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const int tid = threadIdx.x;
    const int nd = gp(D.res)->nd;
    const int64_t a0 = e.y * static_cast<int64_t>(kSkChunk);
    const int64_t a1 = min(D.n, a0 + kSkChunk);
    const typename T::Rec *__restrict__ rec = static_cast<const typename T::Rec *>(D.rec);
    const int nsl = nd <= 128 ? max(1, 256 / max(nd, 1)) : 1;
    const int items = nd <= 128 ? nsl * nd : 256;
    const int passes = nd <= 128 ? 1 : (nd + 255) / 256;
    for (int pass = 0; pass < passes; ++pass) {
        const int d = nd <= 128 ? tid % max(nd, 1) : pass * 256 + tid;
        const int sl = nd <= 128 ? tid / max(nd, 1) : 0;
        const bool active = tid < items && d < nd;
        const int4 m = active ? gload(D.modes + d) : make_int4(0, 0, 0, 0);
        double accr = 0.0, acci = 0.0;
        for (int64_t c0 = a0; c0 < a1; c0 += 256) {
            const int cnt = static_cast<int>(min(static_cast<int64_t>(256), a1 - c0));
            if (tid < cnt) {
                const typename T::Rec r = gload(rec + c0 + tid);
                if constexpr (sizeof(typename T::real) == 4) s_at[tid] = split_atom(r);
                else s_at[tid] = r;
            }
            __syncthreads();
            if (active) {
                // FP64 accumulation of each term: atoms sorted by cell have
                // nearly equal phases at small |m|, so an FP32 running sum
                // grows well above the result and loses bits at every add
                // (FP64 adds run at the FP32 rate on this chip)
                for (int k = sl; k < cnt; k += nsl) {
                    const Atom at = s_at[k];
                    const double q = static_cast<double>(at.q);
                    if constexpr (sizeof(typename T::real) == 4) {
                        float sn, cs;
                        phase_sincos32(m, at, sn, cs);
                        accr = fma(q, static_cast<double>(cs), accr);
                        acci = fma(q, static_cast<double>(sn), acci);
                    } else {
                        double sn, cs;
                        phase_sincos64(m, at, sn, cs);
                        accr = fma(q, cs, accr);
                        acci = fma(q, sn, acci);
                    }
                }
            }
            __syncthreads();
        }
        s_red[0][tid] = accr;
        s_red[1][tid] = acci;
        __syncthreads();
        if (sl == 0 && active) {
            double r = 0.0, im = 0.0;
            const int stride = nd <= 128 ? nd : 0;
            for (int k = 0; k < nsl; ++k) {
                r += s_red[0][tid + k * stride];
                im += s_red[1][tid + k * stride];
            }
            RB_GLOBAL double *p = gp(D.rho_part) + 2 * (e.y * static_cast<int64_t>(D.mcap) + d);
            p[0] = r;
            p[1] = im;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// FP64 combine: rho per mode, pair-kernel partials
// ----------------------------------------------------------------------------

__device__ inline double block_sum_256(double v, double *s_tmp)
{
    const int tid = threadIdx.x;
    s_tmp[tid] = v;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (tid < o) s_tmp[tid] += s_tmp[tid + o];
        __syncthreads();
    }
    const double r = s_tmp[0];
    __syncthreads();
    return r;
}

// plan entry (s, k): k < mcap sums mode k over the structure-factor blocks,
// k == mcap sums the pair-kernel partials
__global__ __launch_bounds__(256) void k_rho_reduce(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                    const int2 *__restrict__ plan)
{
    __shared__ double s_tmp[256];
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const int tid = threadIdx.x;
    const int d = e.y;
    StepResults *res = D.res;
    if (d < D.mcap) {
        if (d >= gp(res)->nd) return;
        double r = 0.0, im = 0.0;
        const RB_GLOBAL double *rp = gp(D.rho_part);
        for (int64_t b = tid; b < D.sk_blocks; b += 256) {
            const RB_GLOBAL double *p = rp + 2 * (b * D.mcap + d);
            r += p[0];
            im += p[1];
        }
        r = block_sum_256(r, s_tmp);
        im = block_sum_256(im, s_tmp);
        if (tid == 0) {
            D.rho[2 * d] = r;
            D.rho[2 * d + 1] = im;
        }
    } else {
        // slice of the pair-block partials: blocks [k c, (k + 1) c), c = ceil(npair / kPairRed)
        const int k = d - D.mcap;
        const int64_t npair = gp(D.bstart)[stp[e.x].ncells];
        const int64_t c = (npair + kPairRed - 1) / kPairRed;
        const int64_t b0 = k * c, b1 = min(npair, b0 + c);
        const RB_GLOBAL double *pp = gp(D.pair_part);
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t b = b0 + tid; b < b1; b += 256)
            for (int j = 0; j < 8; ++j) acc[j] += pp[8 * b + j];
        for (int j = 0; j < 8; ++j) {
            const double s = block_sum_256(acc[j], s_tmp);
            if (tid == 0) D.pair_red[8 * k + j] = s;
        }
    }
}

// Estimators of Sec. 3.2 and App. B over the distinct modes d with
// multiplicities c^r_d, c^nr_d (one workgroup per system):
//   P^{F,r*}  =  S^r/(4 V^2 P) sum_d c^r_d |rho_d|^2/|k_d|^2 I            (eq. P_approx_r)
//   P^{F,nr*} = -S^nr/(8 V^2 P) sum_d c^nr_d |rho_d|^2 k_d k_d^T/|k_d|^4  (eq. P_approx_nr)
//     (shared sampler: the r-chain's modes, -S^r/(8 V^2 P) sum_d c^r_d R_d |rho_d|^2 k_d k_d^T/|k_d|^4
//      with R_d = |k_d|^2 sum_l wt_l s_l^7 e_l / sum_l wt_l s_l^5 e_l the ratio P^nr S^nr/(P^r S^r))
//   U^{F*}    =  S/(2 V P) sum_d c^r_d |rho_d|^2/|k_d|^2, S = S^r/2
//   force coefficients a_d = (S/(P V)) c^r_d/|k_d|^2                      (eq. f_approx)
template <class T>
__global__ __launch_bounds__(256) void k_estimators(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp)
{
    __shared__ double s_tmp[256];
    const SysDesc &D = desc[blockIdx.x];
    const SysStep &St = stp[blockIdx.x];
    const int tid = threadIdx.x;
    const int nd = gp(D.res)->nd;
    const double L[3] = {St.L[0], St.L[1], St.L[2]};
    const double V = St.V;
    const double S = 0.5 * St.Sr;
    const int P = D.P;
    const bool shared = D.variant == RBSOG_RECAL_SHARED;
    // short-range virial, energy and pair count: the slices in order
    if (tid < 8) {
        double s = 0.0;
        for (int k = 0; k < kPairRed; ++k) s += D.pair_red[8 * k + tid];
        StepResults *r = D.res;
        if (tid < 6) r->vir[tid] = s;
        else if (tid == 6) r->UN = s;
        else r->npairs = s;
    }
    __syncthreads();
    double sr = 0.0, su = 0.0, snr[6] = {0, 0, 0, 0, 0, 0};
    const bool wide = D.tab.Me > D.tab.M;
    for (int d = tid; d < nd; d += 256) {
        const int4 m = D.modes[d];
        double k[3];
        if (St.tri) {
            // k = 2 pi h^-T m
            for (int i = 0; i < 3; ++i) k[i] = 2.0 * kPi * (St.hi[i] * m.x + St.hi[3 + i] * m.y + St.hi[6 + i] * m.z);
        } else {
            k[0] = 2.0 * kPi * m.x / L[0];
            k[1] = 2.0 * kPi * m.y / L[1];
            k[2] = 2.0 * kPi * m.z / L[2];
        }
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double re = D.rho[2 * d], im = D.rho[2 * d + 1];
        const double r2 = re * re + im * im;
        const int cr = D.cnt[d], cnr = D.cnt[D.mcap + d];
        sr += cr * r2 / k2;
        if (wide) {
            // energy kernel of Me terms over the M-term one that the modes were drawn from:
            // sum_{l<Me} w_l s_l^3 e_l / sum_{l<M} w_l s_l^3 e_l (w_l s_l^3 = wt_l s_l^5 / 2)
            double num = 0.0, den = 0.0;
            for (int l = 0; l < D.tab.Me; ++l) {
                const double t = D.tab.w[l] * D.tab.s[l] * D.tab.s[l] * D.tab.s[l] *
                                 exp(-D.tab.s[l] * D.tab.s[l] * k2 / 4.0);
                num += t;
                if (l < D.tab.M) den += t;
            }
            su += cr * r2 / k2 * (num / den);
        }
        double g = cnr * r2 / (k2 * k2);
        if (shared) {
            double a5 = 0.0, a7 = 0.0;
            for (int l = 0; l < D.tab.M; ++l) {
                const double e = exp(-D.tab.s[l] * D.tab.s[l] * k2 / 4.0);
                a5 += D.tab.wt[l] * D.tab.s5[l] * e;
                a7 += D.tab.wt[l] * D.tab.s7[l] * e;
            }
            g *= k2 * a7 / a5;
        }
        snr[0] += g * k[0] * k[0];
        snr[1] += g * k[1] * k[1];
        snr[2] += g * k[2] * k[2];
        snr[3] += g * k[0] * k[1];
        snr[4] += g * k[0] * k[2];
        snr[5] += g * k[1] * k[2];
        const double ad = S / (P * V) * cr / k2;
        using real = typename T::real;
        Coef<real> cf;
        cf.mx = m.x;
        cf.my = m.y;
        cf.mz = m.z;
        cf.pad = 0;
        cf.kx = static_cast<real>(k[0]);
        cf.ky = static_cast<real>(k[1]);
        cf.kz = static_cast<real>(k[2]);
        cf.A = static_cast<real>(ad * im);
        cf.B = static_cast<real>(ad * re);
        static_cast<Coef<real> *>(D.coef)[d] = cf;
    }
    sr = block_sum_256(sr, s_tmp);
    if (wide) su = block_sum_256(su, s_tmp);
    for (int k = 0; k < 6; ++k) snr[k] = block_sum_256(snr[k], s_tmp);
    if (tid == 0) {
        StepResults *r = D.res;
        const double ck = D.ck;
        const double pr = ck * St.Sr / (4.0 * V * V * P) * sr;
        const double cnr = -ck * (shared ? St.Sr : St.Snr) / (8.0 * V * V * P);
        const int ix[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) {
                const int q = 3 * al + be;
                r->Pr[q] = al == be ? pr : 0.0;
                r->Pnr[q] = cnr * snr[ix[al][be]];
                r->PN[q] = ck * r->vir[ix[al][be]] / V;
                r->Ptot[q] = r->PN[q] + r->Pr[q] + r->Pnr[q];
            }
        r->UF = ck * S / (2.0 * V * P) * (wide ? su : sr);
        r->UN = ck * r->UN;
        for (int k = 0; k < 6; ++k) r->vir[k] *= ck;
        r->Uself = D.Uself;
        r->Sr = St.Sr;
        r->Snr = St.Snr;
    }
}

// ----------------------------------------------------------------------------
// Long-range force scatter (eq. f_approx) and the total force in caller order
// ----------------------------------------------------------------------------

// sr: add the short-range force (the step's output); without it the kernel
// writes the long-range part alone to (ox, oy, oz) (inspection)
template <class T>
__global__ __launch_bounds__(kAtomBlock) void k_force(const SysDesc *__restrict__ desc, const SysStep *__restrict__ stp,
                                                      const int2 *__restrict__ plan, int sr, double *ox, double *oy,
                                                      double *oz)
{
    using real = typename T::real;
    const int2 e = plan[blockIdx.x];
    const SysDesc &D = desc[e.x];
    const SysStep &St = stp[e.x];
    const int64_t n = D.n;
    const int nd = gp(D.res)->nd;
    const Coef<real> *cf = static_cast<const Coef<real> *>(D.coef);
    const int64_t t = e.y * static_cast<int64_t>(kAtomBlock) + threadIdx.x;
    if (t >= n) return;
    const typename T::Rec r = gload(static_cast<const typename T::Rec *>(D.rec) + t);
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if constexpr (sizeof(real) == 4) {
        const SkAtom32 at = split_atom(r);
        for (int d0 = 0; d0 < nd; d0 += 32) {
            float hx = 0.f, hy = 0.f, hz = 0.f;
            const int d1 = min(nd, d0 + 32);
            auto term = [&](const Coef<float> &c) {
                float sn, cs;
                phase_sincos32(make_int4(c.mx, c.my, c.mz, 0), at, sn, cs);
                const float g = c.A * cs - c.B * sn;
                hx += g * c.kx;
                hy += g * c.ky;
                hz += g * c.kz;
            };
            // four modes' coefficients loaded together (scalar loads, one wait),
            // terms added in mode order
            int d = d0;
            for (; d + 4 <= d1; d += 4) {
                Coef<float> c[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) c[k] = gload(cf + d + k);
#pragma unroll
                for (int k = 0; k < 4; ++k) term(c[k]);
            }
            for (; d < d1; ++d) term(gload(cf + d));
            gx += hx;
            gy += hy;
            gz += hz;
        }
    } else {
        for (int d = 0; d < nd; ++d) {
            const Coef<double> c = gload(cf + d);
            double sn, cs;
            phase_sincos64(make_int4(c.mx, c.my, c.mz, 0), r, sn, cs);
            const double g = c.A * cs - c.B * sn;
            gx += g * c.kx;
            gy += g * c.ky;
            gz += g * c.kz;
        }
    }
    const RB_GLOBAL real *fsr = gp(static_cast<const real *>(D.fsr));
    const double q = static_cast<double>(r.q);
    const int i = gp(D.perm)[t];
    const double ck = D.ck;
    if (sr) {
        gp(St.fx)[i] = ck * (static_cast<double>(fsr[t]) - q * gx);
        gp(St.fy)[i] = ck * (static_cast<double>(fsr[n + t]) - q * gy);
        gp(St.fz)[i] = ck * (static_cast<double>(fsr[2 * n + t]) - q * gz);
    } else {
        gp(ox)[i] = ck * (-q * gx);
        gp(oy)[i] = ck * (-q * gy);
        gp(oz)[i] = ck * (-q * gz);
    }
}

// r <- mu r (FP64) for the positions of each system
__global__ __launch_bounds__(kAtomBlock) void k_rescale(const SysDesc *__restrict__ desc,
                                                        const SysStep *__restrict__ stp,
                                                        const int2 *__restrict__ plan)
{
    const int2 e = plan[blockIdx.x];
    const SysStep &St = stp[e.x];
    const int64_t i = e.y * static_cast<int64_t>(kAtomBlock) + threadIdx.x;
    if (i >= desc[e.x].n) return;
    RB_GLOBAL double *x = gp(const_cast<double *>(St.x)), *y = gp(const_cast<double *>(St.y)),
                     *z = gp(const_cast<double *>(St.z));
    x[i] *= St.mu[0];
    y[i] *= St.mu[1];
    z[i] *= St.mu[2];
}

// ----------------------------------------------------------------------------
// NPT integration (the splitting of eq. Langevin_NPT; host side in npt.cpp).
// One system, caller order, FP64.
// ----------------------------------------------------------------------------

// B: p += c F
__global__ __launch_bounds__(kNptBlock) void k_npt_kick(int64_t n, double c, const double *__restrict__ F,
                                                        double *__restrict__ px, double *__restrict__ py,
                                                        double *__restrict__ pz)
{
    const int64_t i = blockIdx.x * static_cast<int64_t>(kNptBlock) + threadIdx.x;
    if (i >= n) return;
    px[i] += c * F[i];
    py[i] += c * F[n + i];
    pz[i] += c * F[2 * n + i];
}

// A: exact flow over one substep with the box moving linearly, per axis
// r <- a r + b p/m, p <- p/a (a = L_new/L_old, b = the substep)
__global__ __launch_bounds__(kNptBlock) void k_npt_drift(int64_t n, double ax, double ay, double az, double bx,
                                                         double by, double bz, const double *__restrict__ mass,
                                                         double *__restrict__ x, double *__restrict__ y,
                                                         double *__restrict__ z, double *__restrict__ px,
                                                         double *__restrict__ py, double *__restrict__ pz)
{
    const int64_t i = blockIdx.x * static_cast<int64_t>(kNptBlock) + threadIdx.x;
    if (i >= n) return;
    const double m = mass[i];
    x[i] = ax * x[i] + bx * px[i] / m;
    y[i] = ay * y[i] + by * py[i] / m;
    z[i] = az * z[i] + bz * pz[i] / m;
    px[i] = px[i] / ax;
    py[i] = py[i] / ay;
    pz[i] = pz[i] / az;
}

// O: Ornstein-Uhlenbeck update p <- c p + sc sqrt(m) xi with three standard
// normals per atom, Box-Muller of the Philox draws (atom, 16, step, sys) and
// (atom, 17, step, sys)
__global__ __launch_bounds__(kNptBlock) void k_npt_ou(int64_t n, double c, double sc,
                                                      const double *__restrict__ mass, double *__restrict__ px,
                                                      double *__restrict__ py, double *__restrict__ pz,
                                                      uint32_t key0, uint32_t key1, uint32_t step, uint32_t sys)
{
#pragma clang fp contract(off)
    const int64_t i = blockIdx.x * static_cast<int64_t>(kNptBlock) + threadIdx.x;
    if (i >= n) return;
    const uint2 key = make_uint2(key0, key1);
    const uint4 o1 = philox4x32_10(make_uint4(static_cast<uint32_t>(i), 16u, step, sys), key);
    const uint4 o2 = philox4x32_10(make_uint4(static_cast<uint32_t>(i), 17u, step, sys), key);
    const double u1 = unit_open(o1.x, o1.y), u2 = unit_open(o1.z, o1.w);
    const double u3 = unit_open(o2.x, o2.y), u4 = unit_open(o2.z, o2.w);
    const double r1 = sqrt(-2.0 * log(u1));
    const double r2 = sqrt(-2.0 * log(u3));
    const double s = sc * sqrt(mass[i]);
    px[i] = c * px[i] + s * (r1 * cos(2.0 * kPi * u2));
    py[i] = c * py[i] + s * (r1 * sin(2.0 * kPi * u2));
    pz[i] = c * pz[i] + s * (r2 * cos(2.0 * kPi * u4));
}

// sum_i p_i p_i^T / m_i: per-block partials (xx, yy, zz, xy, xz, yz)
__global__ __launch_bounds__(kNptBlock) void k_npt_kinetic_part(int64_t n, const double *__restrict__ mass,
                                                                const double *__restrict__ px,
                                                                const double *__restrict__ py,
                                                                const double *__restrict__ pz,
                                                                double *__restrict__ part)
{
    __shared__ double s_w[kNptBlock / 64][6];
    const int64_t i = blockIdx.x * static_cast<int64_t>(kNptBlock) + threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        const double im = 1.0 / mass[i], a = px[i], b = py[i], c = pz[i];
        v[0] = a * a * im;
        v[1] = b * b * im;
        v[2] = c * c * im;
        v[3] = a * b * im;
        v[4] = a * c * im;
        v[5] = b * c * im;
    }
    for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
    const int wv = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 6; ++k) s_w[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        double t = 0;
        for (int w = 0; w < kNptBlock / 64; ++w) t += s_w[w][threadIdx.x];
        part[6 * static_cast<int64_t>(blockIdx.x) + threadIdx.x] = t;
    }
}

// one workgroup: the partials in a fixed order
__global__ __launch_bounds__(256) void k_npt_kinetic_sum(int64_t nblocks, const double *__restrict__ part,
                                                         double *__restrict__ kin)
{
    __shared__ double s_v[256][6];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nblocks; b += 256)
        for (int k = 0; k < 6; ++k) v[k] += part[6 * b + k];
    for (int k = 0; k < 6; ++k) s_v[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o)
            for (int k = 0; k < 6; ++k) s_v[threadIdx.x][k] += s_v[threadIdx.x + o][k];
        __syncthreads();
    }
    if (threadIdx.x < 6) kin[threadIdx.x] = s_v[0][threadIdx.x];
}

inline const int2 *plan_ptr(const Batch &b, PlanKind k) { return b.d_plan + b.plan_off[k]; }
inline unsigned plan_grid(const Batch &b, PlanKind k) { return static_cast<unsigned>(b.plan_len[k]); }
inline unsigned nsys(const Batch &b) { return static_cast<unsigned>(b.sys.size()); }

}  // namespace

// ----------------------------------------------------------------------------
// Launchers (every launch covers all systems of the batch)
// ----------------------------------------------------------------------------

hipError_t record_sample_fence(Batch &b)
{
    if (b.sys.empty()) return hipSuccess;
    return hipEventRecord(b.ev_up, b.stream);
}

hipError_t launch_sample_fenced(Batch &b)
{
    if (b.sys.empty()) return hipSuccess;
    // on the second stream, after what the first held at the fence
    hipError_t e = hipStreamWaitEvent(b.aux, b.ev_up, 0);
    if (e != hipSuccess) return e;
    timer_begin(b, "sampler", b.aux);
    hipLaunchKernelGGL(k_sampler, dim3(nsys(b)), dim3(256), 0, b.aux, b.d_desc, b.d_step);
    timer_end(b, "sampler", b.aux);
    return hipGetLastError();
}

hipError_t launch_sample(Batch &b)
{
    // on the second stream, after everything queued so far on the first
    const hipError_t e = record_sample_fence(b);
    return e == hipSuccess ? launch_sample_fenced(b) : e;
}

template <class T>
static hipError_t bin_and_sort_t(Batch &b)
{
    timer_begin(b, "bin", b.stream);
    hipLaunchKernelGGL(k_zero, dim3(plan_grid(b, kPlanCells)), dim3(kCellBlock), 0, b.stream, b.d_desc, b.d_step,
                       plan_ptr(b, kPlanCells), b.d_ctrl);
    hipLaunchKernelGGL(k_fix<T>, dim3(plan_grid(b, kPlanAtoms)), dim3(kAtomBlock), 0, b.stream, b.d_desc, b.d_step,
                       plan_ptr(b, kPlanAtoms));
    hipLaunchKernelGGL(k_scan_local, dim3(plan_grid(b, kPlanScan)), dim3(256), 0, b.stream, b.d_desc, b.d_step,
                       plan_ptr(b, kPlanScan));
    hipLaunchKernelGGL(k_scan_add, dim3(plan_grid(b, kPlanCells)), dim3(kCellBlock), 0, b.stream, b.d_desc, b.d_step,
                       plan_ptr(b, kPlanCells));
    hipLaunchKernelGGL(k_scatter<T>, dim3(plan_grid(b, kPlanAtoms)), dim3(kAtomBlock), 0, b.stream, b.d_desc,
                       plan_ptr(b, kPlanAtoms));
    hipLaunchKernelGGL(k_order<T>, dim3(plan_grid(b, kPlanCell1)), dim3(kOrderThreads), 0, b.stream, b.d_desc, b.d_step,
                       plan_ptr(b, kPlanCell1));
    timer_end(b, "bin", b.stream);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? hipEventRecord(b.ev_bin, b.stream) : e;
}

hipError_t launch_bin_and_sort(Batch &b)
{
    if (b.sys.empty()) return hipSuccess;
    return b.precision == RBSOG_PREC_FP64 ? bin_and_sort_t<F64>(b) : bin_and_sort_t<F32>(b);
}

template <class T, int M, bool E, bool FAST, bool TRI = false>
static void pair_launch_group(Batch &b, int group)
{
    const int64_t first = b.pair_split[group], items = b.pair_split[group + 1] - first;
    if (items <= 0) return;
    const int2 *plan = plan_ptr(b, kPlanPair) + first;
    if (b.pair_schedule == kPairPersistent) {
        const int64_t wgs = std::min<int64_t>(items, static_cast<int64_t>(b.num_cu) * b.pair_wg_per_cu);
        hipLaunchKernelGGL((k_pair_queue<T, M, E, FAST, TRI>), dim3(static_cast<unsigned>(wgs)), dim3(64), 0,
                           b.stream, b.d_desc, b.d_step, plan, static_cast<int>(items), b.d_ctrl + group);
    } else {
        hipLaunchKernelGGL((k_pair<T, M, E, FAST, TRI>), dim3(static_cast<unsigned>(items)), dim3(64), 0, b.stream,
                           b.d_desc, b.d_step, plan);
    }
}

// Half shell: neighbourhoods, pair kernel, gather of the reactions.
template <class T, int M, bool E>
static void pair_launch_half(Batch &b, int group)
{
    const int64_t first = b.pair_split[group], items = b.pair_split[group + 1] - first;
    if (items <= 0) return;
    const int2 *plan = plan_ptr(b, kPlanPair) + first;
    const unsigned grid = static_cast<unsigned>(items);
    hipLaunchKernelGGL(k_pair_prep, dim3(grid), dim3(64), 0, b.stream, b.d_desc, b.d_step, plan);
    if (b.pair_schedule == kPairPersistent) {
        const int64_t wgs = std::min<int64_t>(items, static_cast<int64_t>(b.num_cu) * b.pair_wg_per_cu);
        hipLaunchKernelGGL((k_pair_half_queue<T, M, E>), dim3(static_cast<unsigned>(wgs)), dim3(64), 0, b.stream,
                           b.d_desc, b.d_step, plan, static_cast<int>(items), b.d_ctrl + group);
    } else {
        hipLaunchKernelGGL((k_pair_half<T, M, E>), dim3(grid), dim3(64), 0, b.stream, b.d_desc, b.d_step, plan);
    }
    hipLaunchKernelGGL(k_pair_gather, dim3(grid), dim3(64), 0, b.stream, b.d_desc, b.d_step, plan);
}

// one launch per path: the FP32 relative-coordinate filter (full and half
// shell) exists only in FP32
template <class T, int M, bool E>
static void pair_launch(Batch &b, int form)
{
    pair_launch_group<T, M, E, false>(b, kNumPaths * form);
    pair_launch_group<T, M, E, true, true>(b, kNumPaths * form + 3);
    if constexpr (sizeof(typename T::real) == 4) {
        pair_launch_group<T, M, E, true>(b, kNumPaths * form + 1);
        pair_launch_half<T, M, E>(b, kNumPaths * form + 2);
    }
}

template <class T, bool E>
static void pair_forms(Batch &b)
{
    // one launch per form of the SOG kernels: the FP32C polynomial form, the
    // M = 10 exponentials with the weights in registers, runtime M
    if constexpr (sizeof(typename T::real) == 4) pair_launch<T, -1, E>(b, kFormPoly);
    pair_launch<T, 10, E>(b, kFormExp10);
    pair_launch<T, 0, E>(b, kFormExpM);
}

template <class T>
static hipError_t pair_t(Batch &b)
{
    timer_begin(b, "pair", b.stream);
    if (b.want_energy) pair_forms<T, true>(b);
    else pair_forms<T, false>(b);
    timer_end(b, "pair", b.stream);
    return hipGetLastError();
}

hipError_t launch_pair(Batch &b)
{
    if (b.sys.empty() || b.plan_len[kPlanPair] == 0) return hipSuccess;
    return b.precision == RBSOG_PREC_FP64 ? pair_t<F64>(b) : pair_t<F32>(b);
}

template <class T>
static hipError_t kspace_t(Batch &b)
{
    // structure factors on the second stream once the records are sorted,
    // beside the pair kernel; the first stream joins before the reductions
    hipError_t e = hipStreamWaitEvent(b.aux, b.ev_bin, 0);
    if (e != hipSuccess) return e;
    timer_begin(b, "sk", b.aux);
    hipLaunchKernelGGL(k_sk<T>, dim3(plan_grid(b, kPlanSk)), dim3(256), 0, b.aux, b.d_desc, plan_ptr(b, kPlanSk));
    timer_end(b, "sk", b.aux);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(b.ev_sk, b.aux);
    if (e == hipSuccess) e = hipStreamWaitEvent(b.stream, b.ev_sk, 0);
    if (e != hipSuccess) return e;
    timer_begin(b, "reduce", b.stream);
    hipLaunchKernelGGL(k_rho_reduce, dim3(plan_grid(b, kPlanReduce)), dim3(256), 0, b.stream, b.d_desc, b.d_step,
                       plan_ptr(b, kPlanReduce));
    hipLaunchKernelGGL(k_estimators<T>, dim3(nsys(b)), dim3(256), 0, b.stream, b.d_desc, b.d_step);
    timer_end(b, "reduce", b.stream);
    timer_begin(b, "force", b.stream);
    hipLaunchKernelGGL(k_force<T>, dim3(plan_grid(b, kPlanAtoms)), dim3(kAtomBlock), 0, b.stream, b.d_desc, b.d_step,
                       plan_ptr(b, kPlanAtoms), 1, nullptr, nullptr, nullptr);
    timer_end(b, "force", b.stream);
    return hipGetLastError();
}

hipError_t launch_kspace(Batch &b)
{
    if (b.sys.empty()) return hipSuccess;
    return b.precision == RBSOG_PREC_FP64 ? kspace_t<F64>(b) : kspace_t<F32>(b);
}

// the long-range force of the last step alone, into caller-order device
// arrays (a batch of one system)
hipError_t launch_long_range_force(Batch &b, double *fx, double *fy, double *fz)
{
    if (b.sys.size() != 1) return hipErrorInvalidValue;
    if (b.precision == RBSOG_PREC_FP64)
        hipLaunchKernelGGL(k_force<F64>, dim3(plan_grid(b, kPlanAtoms)), dim3(kAtomBlock), 0, b.stream, b.d_desc,
                           b.d_step, plan_ptr(b, kPlanAtoms), 0, fx, fy, fz);
    else
        hipLaunchKernelGGL(k_force<F32>, dim3(plan_grid(b, kPlanAtoms)), dim3(kAtomBlock), 0, b.stream, b.d_desc,
                           b.d_step, plan_ptr(b, kPlanAtoms), 0, fx, fy, fz);
    return hipGetLastError();
}

hipError_t launch_rescale(Batch &b)
{
    if (b.sys.empty()) return hipSuccess;
    hipLaunchKernelGGL(k_rescale, dim3(plan_grid(b, kPlanAtoms)), dim3(kAtomBlock), 0, b.stream, b.d_desc, b.d_step,
                       plan_ptr(b, kPlanAtoms));
    return hipGetLastError();
}

static unsigned npt_grid(int64_t n) { return static_cast<unsigned>((n + kNptBlock - 1) / kNptBlock); }

hipError_t launch_npt_kick(hipStream_t s, int64_t n, double c, const double *F, double *px, double *py, double *pz)
{
    hipLaunchKernelGGL(k_npt_kick, dim3(npt_grid(n)), dim3(kNptBlock), 0, s, n, c, F, px, py, pz);
    return hipGetLastError();
}

hipError_t launch_npt_drift(hipStream_t s, int64_t n, const double a[3], const double b[3], const double *mass,
                            double *x, double *y, double *z, double *px, double *py, double *pz)
{
    hipLaunchKernelGGL(k_npt_drift, dim3(npt_grid(n)), dim3(kNptBlock), 0, s, n, a[0], a[1], a[2], b[0], b[1], b[2],
                       mass, x, y, z, px, py, pz);
    return hipGetLastError();
}

hipError_t launch_npt_ou(hipStream_t s, int64_t n, double c, double sc, const double *mass, double *px, double *py,
                         double *pz, uint64_t seed, uint32_t step, uint32_t sys)
{
    hipLaunchKernelGGL(k_npt_ou, dim3(npt_grid(n)), dim3(kNptBlock), 0, s, n, c, sc, mass, px, py, pz,
                       static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), step, sys);
    return hipGetLastError();
}

hipError_t launch_npt_kinetic(hipStream_t s, int64_t n, const double *mass, const double *px, const double *py,
                              const double *pz, double *part, int64_t nblocks, double *kin)
{
    if (nblocks != static_cast<int64_t>(npt_grid(n))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_npt_kinetic_part, dim3(npt_grid(n)), dim3(kNptBlock), 0, s, n, mass, px, py, pz, part);
    hipLaunchKernelGGL(k_npt_kinetic_sum, dim3(1), dim3(256), 0, s, nblocks, part, kin);
    return hipGetLastError();
}

}  // namespace rbsog
