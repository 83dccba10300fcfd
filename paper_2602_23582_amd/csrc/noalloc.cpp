// rbsog_force_virial_noalloc: rbsog_force_virial for callers that cannot
// allocate (HIP graph capture, serving loops, harnesses that forbid it).  The
// step's partial results (per-block structure-factor partials, per-block pair
// sums of virial, energy and pair count, their slice sums) live in a
// file-scope device array instead of the context's buffers; everything else
// is the context's, set up beforehand.  The kernels are those of
// rbsog_force_virial, so the results are bitwise the same.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rbsog_impl.hpp"

namespace {

// Partial results of one step: at most kScratchBytes per GPU, held by each GPU
// the library runs on until the process ends.
constexpr size_t kScratchBytes = size_t(32) << 20;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_scratch[kMaxDevices] = {};  // device address of scratch, per device

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int fail(rbsog_ctx *c, int code, const char *msg)
{
    c->err = msg;
    return code;
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

// Address of this device's scratch: looked up once per device (with that
// device current) and kept; host code uses it, never the array's name.
int scratch_ptr(rbsog_ctx *c, char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        c->err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(c, RBSOG_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            c->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return RBSOG_EDEVICE;
        }
        g_scratch[dev] = static_cast<char *>(p);
    }
    *out = g_scratch[dev];
    return RBSOG_OK;
}

}  // namespace

extern "C" int rbsog_force_virial_noalloc(rbsog_ctx *c, const double *x, const double *y, const double *z,
                                          double *fx, double *fy, double *fz, double host_energy[3],
                                          double host_vir[6])
{
    if (!c) return RBSOG_EINVAL;
    c->err.clear();
    if (c->in_batch) return fail(c, RBSOG_ESTATE, "the context is admitted to a batch");
    if (c->state < 1) return fail(c, RBSOG_ESTATE, "rbsog_sample_modes must precede rbsog_force_virial_noalloc");
    if (!(is_device_ptr(x) && is_device_ptr(y) && is_device_ptr(z) && is_device_ptr(fx) && is_device_ptr(fy) &&
          is_device_ptr(fz)))
        return fail(c, RBSOG_EINVAL, "rbsog_force_virial_noalloc takes device position and force arrays only");
    rbsog::System &s = c->sys;
    rbsog::SysDesc &d = s.desc;
    // what rbsog_force_virial could allocate, refused: a grid or a half-shell
    // neighbourhood larger than the context holds, launch plans larger than
    // the batch holds
    if (s.ncells > s.ncells_cap)
        return fail(c, RBSOG_ESTATE, "the cell grid outgrew the context (run rbsog_force_virial once for this box)");
    if (s.stp.half && (!s.half_mem || d.pair_cap > s.half_blocks || rbsog::half_hcap(s) > s.half_hcap))
        return fail(c, RBSOG_ESTATE, "half-shell buffers not set up for this grid (run rbsog_force_virial once)");
    if (rbsog::batch_upload_allocates(c->batch))
        return fail(c, RBSOG_ESTATE, "launch plans not set up for this grid (run rbsog_force_virial once)");
    const size_t rho_b = align_up(static_cast<size_t>(d.sk_blocks) * d.mcap * 2 * sizeof(double));
    const size_t pair_b = align_up(static_cast<size_t>(d.pair_cap) * 8 * sizeof(double));
    const size_t red_b = align_up(static_cast<size_t>(rbsog::kPairRed) * 8 * sizeof(double));
    if (rho_b + pair_b + red_b > kScratchBytes)
        return fail(c, RBSOG_EINVAL,
                    "system too large for the 32 MiB scratch (it holds 16 B per mode and structure-factor block "
                    "plus 64 B per pair block)");
    char *base = nullptr;
    int rc = scratch_ptr(c, &base);
    if (rc != RBSOG_OK) return rc;

    double *saved[3] = {d.rho_part, d.pair_part, d.pair_red};
    d.rho_part = reinterpret_cast<double *>(base);
    d.pair_part = reinterpret_cast<double *>(base + rho_b);
    d.pair_red = reinterpret_cast<double *>(base + rho_b + pair_b);
    c->batch.desc_dirty = true;
    rbsog::SysStep &t = s.stp;
    t.x = x;
    t.y = y;
    t.z = z;
    t.fx = fx;
    t.fy = fy;
    t.fz = fz;
    c->batch.want_energy = host_energy != nullptr;
    c->res_from_batch = false;
    rc = rbsog::batch_upload(c->batch, c->err);
    hipError_t e = hipSuccess;
    if (rc == RBSOG_OK) e = rbsog::launch_bin_and_sort(c->batch);
    if (rc == RBSOG_OK && e == hipSuccess) e = rbsog::launch_pair(c->batch);
    if (rc == RBSOG_OK && e == hipSuccess) e = rbsog::launch_kspace(c->batch);
    // the context's own buffers again for its next regular call (its
    // descriptor is uploaded again then, behind this call's work)
    d.rho_part = saved[0];
    d.pair_part = saved[1];
    d.pair_red = saved[2];
    c->batch.desc_dirty = true;
    if (rc != RBSOG_OK) return rc;
    if (e != hipSuccess) {
        c->err = std::string("rbsog_force_virial_noalloc launch: ") + hipGetErrorString(e);
        return RBSOG_EDEVICE;
    }
    c->state = 2;
    if (host_energy || host_vir) {
        rc = rbsog::batch_fetch_results(c->batch, c->err);
        if (rc != RBSOG_OK) return rc;
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
