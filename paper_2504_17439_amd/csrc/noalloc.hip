// Allocation-free self-energy moments: the FP64 TDA path of gw_sigma_moments
// (Secs. 2.3 and eqs. convolution_occ / convolution_vir) with every scratch
// buffer carved from one file-scope device array instead of the handle's
// workspace, for callers that cannot allocate device memory.
//
// The array lives in the code object: each device the library runs on holds
// its own copy at its own address, resolved once per device (with the device
// current) by hipGetSymbolAddress when a handle is created on it.  Host code
// never passes the array's name to a kernel or a copy: in host code that name
// is a host-side stand-in, not a device address.  Calls on one device share
// the array, so calls that overlap on one device race.
#include "internal.h"

#include <mutex>

namespace gwm {

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[GW_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

inline size_t up256(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

}  // namespace

// Resolves the device address of the scratch array on `device`, which must be
// the current device.  Called by gw_create once per device; later calls reuse
// the first result.
gw_status noalloc_resolve(int device, std::string* err) {
    if (device < 0 || device >= kMaxDevices) {
        if (err) *err = "no-alloc scratch: device index out of range";
        return GW_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_tried[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_tried[device] = true;
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
        if (e != hipSuccess) (void)hipGetLastError();
    }
    if (!g_scratch_ptr[device]) {
        if (err) *err = std::string("no-alloc scratch: hipGetSymbolAddress failed: ") +
                        hipGetErrorString(g_scratch_err[device]);
        return GW_EHIP;
    }
    return GW_OK;
}

static void* noalloc_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Layout of the scratch for one call (bytes, each region 256-aligned):
// V, D, X (recursion), R (moments), the split-K partials of R_n, the folded
// intermediate of the contraction (all nmo^2 columns) and its split
// partials.  The minimum of a split region is one split; what is left goes
// to more splits, capped at what the default path would use.
struct NoallocPlan {
    size_t off_V, off_D, off_X, off_R, off_part, off_zt, off_acc, total;
    size_t part_cap, zt_cap, acc_cap;  // doubles
};

static bool noalloc_plan(int nocc, int nvir, int naux, int nmom_max, NoallocPlan& p) {
    const size_t ov = (size_t)nocc * nvir, nmo = (size_t)nocc + nvir, A = (size_t)naux;
    const size_t nt = (size_t)nmom_max + 1;
    const size_t d = sizeof(double);
    size_t off = 0;
    p.off_V = off; off += up256(A * ov * d);
    p.off_D = off; off += up256(ov * d);
    p.off_X = off; off += up256(A * ov * d);
    p.off_R = off; off += up256(nt * A * A * d);
    const size_t part_min = A * A, zt_min = nt * A * nmo * nmo, acc_min = 2 * nt * nmo * nmo;
    const size_t fixed = off + up256(part_min * d) + up256(zt_min * d) + up256(acc_min * d);
    if (fixed > GW_NOALLOC_SCRATCH_BYTES) return false;
    size_t spare = (GW_NOALLOC_SCRATCH_BYTES - fixed) / d;
    // extra splits of R_n = X V^T (up to 16), then contraction splits (up to 64)
    size_t part_extra = std::min(spare, 15 * part_min);
    spare -= part_extra;
    size_t acc_extra = std::min(spare, 63 * acc_min);
    size_t zt_extra = 0;
    p.part_cap = part_min + part_extra;
    p.acc_cap = acc_min + acc_extra;
    p.zt_cap = zt_min + zt_extra;
    p.off_part = off; off += up256(p.part_cap * d);
    p.off_zt = off; off += up256(p.zt_cap * d);
    p.off_acc = off; off += up256(p.acc_cap * d);
    p.total = off;
    return p.total <= GW_NOALLOC_SCRATCH_BYTES;
}

gw_status sigma_moments_noalloc(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                                const double* L, double* sigma_occ, double* sigma_vir) {
    NoallocPlan p;
    if (!noalloc_plan(nocc, nvir, naux, nmom_max, p))
        return set_err(h, GW_EINVAL, "gw_sigma_moments_noalloc: the system needs more than the " +
                                         std::to_string((size_t)GW_NOALLOC_SCRATCH_BYTES) +
                                         "-byte static scratch");
    char* base = (char*)noalloc_ptr(h->device);
    if (!base) {
        std::string msg;
        gw_status st = noalloc_resolve(h->device, &msg);
        if (st != GW_OK) return set_err(h, st, msg);
        base = (char*)noalloc_ptr(h->device);
    }
    double* V = (double*)(base + p.off_V);
    double* D = (double*)(base + p.off_D);
    double* X = (double*)(base + p.off_X);
    double* R = (double*)(base + p.off_R);
    Scratch part{-1, (double*)(base + p.off_part), p.part_cap};
    Scratch zt{-1, (double*)(base + p.off_zt), p.zt_cap};
    Scratch acc{-1, (double*)(base + p.off_acc), p.acc_cap};
    GW_TRY(tda_moments_half_f64(h, nocc, nvir, naux, nmom_max, eps, L, R, V, D, X, part));
    return sigma_from_R_f64_bufs(h, nocc, nvir, naux, nmom_max, eps, L, R, (size_t)-1, zt, acc, sigma_occ,
                                 sigma_vir);
}

}  // namespace gwm
