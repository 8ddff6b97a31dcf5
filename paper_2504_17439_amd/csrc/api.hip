// C ABI entry points: handle management, argument validation, dispatch.
#include "internal.h"

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace gwm {

gw_status set_err(Handle* h, gw_status st, const std::string& msg) {
    if (h) h->last_error = msg;
    return st;
}

void* ws_get(Handle* h, int slot, size_t bytes) {
    if (slot < 0 || slot >= WS_COUNT) return nullptr;
    DevBuf& b = h->ws[slot];
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return b.ptr;
    if (b.ptr) {
        // the stream may still use the old buffer
        if (hipStreamSynchronize(h->stream) != hipSuccess) {
            set_err(h, GW_EHIP, "ws_get: stream synchronize failed");
            return nullptr;
        }
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = (bytes + 255) & ~(size_t)255;
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        b.ptr = nullptr;
        (void)hipGetLastError();
        set_err(h, GW_ENOMEM, "device workspace allocation failed (" + std::to_string(want) + " bytes)");
        return nullptr;
    }
    b.bytes = want;
    return b.ptr;
}

double* scratch_get(Handle* h, const Scratch& s, size_t n) {
    if (s.slot >= 0) return (double*)ws_get(h, s.slot, sizeof(double) * std::max<size_t>(n, 1));
    if (n > s.cap || !s.ptr) {
        set_err(h, GW_ENOMEM, "fixed scratch region too small (" + std::to_string(n) + " doubles needed, " +
                                  std::to_string(s.cap) + " available)");
        return nullptr;
    }
    return s.ptr;
}

size_t scratch_max(const Scratch& s) { return s.slot >= 0 ? SIZE_MAX : s.cap; }

KTimer::KTimer(Handle* hh, const char* family) : h(hh) {
    if (!h->timing || !family) return;
    TimedLaunch t;
    t.family = family;
    if (hipEventCreate(&t.start) != hipSuccess || hipEventCreate(&t.stop) != hipSuccess) return;
    if (hipEventRecord(t.start, h->stream) != hipSuccess) return;
    h->timed.push_back(t);
    idx = (int)h->timed.size() - 1;
}

void KTimer::stop() {
    if (idx >= 0) (void)hipEventRecord(h->timed[idx].stop, h->stream);
    idx = -1;
}

static void clear_timed(Handle* h) {
    for (auto& t : h->timed) {
        if (t.start) (void)hipEventDestroy(t.start);
        if (t.stop) (void)hipEventDestroy(t.stop);
    }
    h->timed.clear();
}

}  // namespace gwm

using gwm::Handle;

struct gw_handle_s : public Handle {};

namespace {

thread_local std::string g_static_err;

gw_status validate_common(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                          const double* L) {
    if (nocc < 1 || nvir < 1 || naux < 1)
        return gwm::set_err(h, GW_EINVAL, "nocc, nvir and naux must be >= 1");
    if (nmom_max < 1 || nmom_max % 2 == 0 || nmom_max > 15)
        return gwm::set_err(h, GW_EINVAL, "nmom_max must be odd and in [1, 15]");
    if (!eps || !L) return gwm::set_err(h, GW_EINVAL, "eps and L must be non-null");
    long long ov = (long long)nocc * nvir;
    if (ov > 0x7fffffffLL || (long long)naux * (nocc + nvir) > 0x7fffffffLL)
        return gwm::set_err(h, GW_EINVAL, "problem too large for 32-bit K dimensions");
    // energies: finite, occupied strictly below virtual
    std::vector<double> e(nocc + nvir);
    if (hipMemcpyAsync(e.data(), eps, sizeof(double) * e.size(), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return gwm::set_err(h, GW_EINVAL, "eps is not a readable device pointer");
    double omax = -INFINITY, vmin = INFINITY;
    for (int p = 0; p < nocc + nvir; ++p) {
        if (!std::isfinite(e[p])) return gwm::set_err(h, GW_EINVAL, "eps contains a non-finite value");
        if (p < nocc) omax = std::fmax(omax, e[p]);
        else vmin = std::fmin(vmin, e[p]);
    }
    if (!(omax < vmin)) return gwm::set_err(h, GW_EINVAL, "every occupied energy must lie below every virtual one");
    return GW_OK;
}

gw_status check_opts(Handle* h, gw_precision prec, const gw_opts* o) {
    if (prec != GW_FP64 && prec != GW_MIXED) return gwm::set_err(h, GW_EINVAL, "unknown precision");
    if (o) {
        if (o->nquad < 0 || o->nquad == 1 || o->nquad > 512)
            return gwm::set_err(h, GW_EINVAL, "nquad must be 0 (default) or in [2, 512]");
        if (!(o->quad_scale >= 0.0) || !std::isfinite(o->quad_scale))
            return gwm::set_err(h, GW_EINVAL, "quad_scale must be finite and >= 0");
    }
    return GW_OK;
}

}  // namespace

extern "C" {

gw_status gw_create(gw_handle* out, int device) {
    if (!out) return GW_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        g_static_err = "gw_create: no such HIP device";
        return GW_EINVAL;
    }
    gw_handle h = new (std::nothrow) gw_handle_s();
    if (!h) return GW_ENOMEM;
    h->device = device;
    h->ws.resize(gwm::WS_COUNT);
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess) {
        g_static_err = "gw_create: stream creation failed";
        delete h;
        return GW_EHIP;
    }
    h->stream = h->own_stream;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
            h->cus = cus;
    }
    if (rocblas_create_handle(&h->blas) != rocblas_status_success) {
        g_static_err = "gw_create: rocblas_create_handle failed";
        (void)hipStreamDestroy(h->own_stream);
        delete h;
        return GW_ELIB;
    }
    rocblas_set_stream(h->blas, h->stream);
    // device address of the allocation-free entry point's static scratch, once
    // per device (a failure is reported by that entry point, not here)
    {
        std::string ignored;
        (void)gwm::noalloc_resolve(device, &ignored);
    }
    *out = h;
    return GW_OK;
}

gw_status gw_set_stream(gw_handle h, void* s) {
    if (!h) return GW_EINVAL;
    h->stream = (hipStream_t)s;  // NULL is the device's default (null) stream
    rocblas_set_stream(h->blas, h->stream);
    return GW_OK;
}

gw_status gw_synchronize(gw_handle h) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipStreamSynchronize(h->stream));
    return GW_OK;
}

gw_status gw_timing_enable(gw_handle h, int enable) {
    if (!h) return GW_EINVAL;
    h->timing = enable != 0;
    return GW_OK;
}

gw_status gw_timing_reset(gw_handle h) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipStreamSynchronize(h->stream));
    gwm::clear_timed(h);
    return GW_OK;
}

gw_status gw_timing_read(gw_handle h, const char* family, double* total_ms, long* launches) {
    if (!h || !family || !total_ms || !launches) return GW_EINVAL;
    GW_HIP(h, hipStreamSynchronize(h->stream));
    double tot = 0.0;
    long n = 0;
    for (auto& t : h->timed) {
        if (t.family != family) continue;
        float ms = 0.0f;
        GW_HIP(h, hipEventElapsedTime(&ms, t.start, t.stop));
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    return GW_OK;
}

gw_status gw_destroy(gw_handle h) {
    if (!h) return GW_OK;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    (void)hipStreamSynchronize(h->own_stream);
    gwm::aux_destroy(h);
    gwm::clear_timed(h);
    for (auto& b : h->ws)
        if (b.ptr) (void)hipFree(b.ptr);
    if (h->blas) rocblas_destroy_handle(h->blas);
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
    delete h;
    return GW_OK;
}

const char* gw_last_error(gw_handle h) {
    if (!h) return g_static_err.c_str();
    return h->last_error.c_str();
}

gw_status gw_moments_tda(gw_handle h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                         const double* L, gw_precision prec, const gw_opts* opts, double* R, double* eta) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    GW_TRY(validate_common(h, nocc, nvir, naux, nmom_max, eps, L));
    GW_TRY(check_opts(h, prec, opts));
    if (!R) return gwm::set_err(h, GW_EINVAL, "R must be non-null");
    if (prec == GW_MIXED && !eta) return gwm::tda_moments_mixed(h, nocc, nvir, naux, nmom_max, eps, L, R);
    return gwm::tda_moments_f64(h, nocc, nvir, naux, nmom_max, eps, L, R, eta);
}

gw_status gw_moments_rpa(gw_handle h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                         const double* L, gw_precision prec, const gw_opts* opts, double* R, double* eta) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    GW_TRY(validate_common(h, nocc, nvir, naux, nmom_max, eps, L));
    GW_TRY(check_opts(h, prec, opts));
    if (!R) return gwm::set_err(h, GW_EINVAL, "R must be non-null");
    if (prec == GW_MIXED && !eta) return gwm::rpa_moments_mixed(h, nocc, nvir, naux, nmom_max, eps, L, opts, R);
    return gwm::rpa_moments_f64(h, nocc, nvir, naux, nmom_max, eps, L, opts, R, eta);
}

gw_status gw_sigma_from_R(gw_handle h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                          const double* L, const double* R, gw_precision prec, const gw_opts* opts,
                          double* sigma_occ, double* sigma_vir) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    GW_TRY(validate_common(h, nocc, nvir, naux, nmom_max, eps, L));
    GW_TRY(check_opts(h, prec, opts));
    if (!R || !sigma_occ || !sigma_vir) return gwm::set_err(h, GW_EINVAL, "R and sigma outputs must be non-null");
    if (prec == GW_MIXED)
        return gwm::sigma_from_R_mixed(h, nocc, nvir, naux, nmom_max, eps, L, R, opts, sigma_occ, sigma_vir);
    return gwm::sigma_from_R_f64(h, nocc, nvir, naux, nmom_max, eps, L, R, opts, sigma_occ, sigma_vir);
}

gw_status gw_sigma_moments(gw_handle h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max,
                           const double* eps, const double* L, gw_precision prec, const gw_opts* opts,
                           double* sigma_occ, double* sigma_vir) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    GW_TRY(validate_common(h, nocc, nvir, naux, nmom_max, eps, L));
    GW_TRY(check_opts(h, prec, opts));
    if (screening != GW_TDA && screening != GW_RPA) return gwm::set_err(h, GW_EINVAL, "unknown screening");
    if (!sigma_occ || !sigma_vir) return gwm::set_err(h, GW_EINVAL, "sigma outputs must be non-null");
    if (prec == GW_MIXED && nmom_max > 11)
        return gwm::set_err(h, GW_EINVAL, "mixed precision: nmom_max must be <= 11");
    const long n2 = (long)naux * naux;
    double* R = (double*)gwm::ws_get(h, gwm::WS_R, sizeof(double) * (nmom_max + 1) * n2);
    if (!R) return GW_ENOMEM;
    if (screening == GW_TDA && prec == GW_MIXED)
        GW_TRY(gwm::tda_moments_mixed(h, nocc, nvir, naux, nmom_max, eps, L, R));
    else if (screening == GW_TDA)
        GW_TRY(gwm::tda_moments_f64(h, nocc, nvir, naux, nmom_max, eps, L, R, nullptr));
    else if (prec == GW_MIXED)
        GW_TRY(gwm::rpa_moments_mixed(h, nocc, nvir, naux, nmom_max, eps, L, opts, R));
    else
        GW_TRY(gwm::rpa_moments_f64(h, nocc, nvir, naux, nmom_max, eps, L, opts, R, nullptr));
    if (prec == GW_MIXED)
        return gwm::sigma_from_R_mixed(h, nocc, nvir, naux, nmom_max, eps, L, R, opts, sigma_occ, sigma_vir);
    return gwm::sigma_from_R_f64(h, nocc, nvir, naux, nmom_max, eps, L, R, opts, sigma_occ, sigma_vir);
}

gw_status gw_sigma_moments_noalloc(gw_handle h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                                   const double* L, double* sigma_occ, double* sigma_vir) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    GW_TRY(validate_common(h, nocc, nvir, naux, nmom_max, eps, L));
    if (!sigma_occ || !sigma_vir) return gwm::set_err(h, GW_EINVAL, "sigma outputs must be non-null");
    return gwm::sigma_moments_noalloc(h, nocc, nvir, naux, nmom_max, eps, L, sigma_occ, sigma_vir);
}

gw_status gw_poles(gw_handle h, int nmo, int nmom_max, const double* sigma_occ, const double* sigma_vir,
                   const double* fock, const gw_opts* opts, int* npole_occ, int* npole_vir, double* pole_e,
                   double* pole_v, double* E, double* chi, double* qp_e, double* qp_w) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (nmo < 1) return gwm::set_err(h, GW_EINVAL, "nmo must be >= 1");
    if (nmom_max < 1 || nmom_max % 2 == 0 || nmom_max > 15)
        return gwm::set_err(h, GW_EINVAL, "nmom_max must be odd and in [1, 15]");
    if (!sigma_occ || !sigma_vir || !fock || !npole_occ || !npole_vir || !pole_e || !pole_v || !E || !qp_e || !qp_w)
        return gwm::set_err(h, GW_EINVAL, "gw_poles: a required pointer is null");
    return gwm::poles_f64(h, nmo, nmom_max, sigma_occ, sigma_vir, fock, opts, npole_occ, npole_vir, pole_e,
                          pole_v, E, chi, qp_e, qp_w);
}

gw_status gw_eigh(gw_handle h, int n, double* A, double* w) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (n < 1) return gwm::set_err(h, GW_EINVAL, "gw_eigh: n must be >= 1");
    if (!A || !w) return gwm::set_err(h, GW_EINVAL, "gw_eigh: A and w must be non-null");
    double* work = (double*)gwm::ws_get(h, gwm::WS_MISC, sizeof(double) * ((size_t)n + 16));
    if (!work) return GW_ENOMEM;
    int* info = (int*)(work + n + 8);
    GW_TRY(gwm::eigh_rows(h, n, A, w, work, info));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    return GW_OK;
}

gw_status gw_fsgw(gw_handle h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max,
                  const double* eps, const double* L, const double* F0, gw_precision prec, const gw_opts* opts,
                  const gw_fsgw_opts* fopts, double* F, double* qp_e, double* qp_w, gw_fsgw_info* info) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    GW_TRY(validate_common(h, nocc, nvir, naux, nmom_max, eps, L));
    GW_TRY(check_opts(h, prec, opts));
    if (screening != GW_TDA && screening != GW_RPA) return gwm::set_err(h, GW_EINVAL, "unknown screening");
    if (nmom_max % 2 == 0 || nmom_max > 15)
        return gwm::set_err(h, GW_EINVAL, "fsGW: nmom_max must be odd and <= 15");
    if (prec == GW_MIXED && nmom_max > 11)
        return gwm::set_err(h, GW_EINVAL, "mixed precision: nmom_max must be <= 11");
    if (!F || !qp_e || !qp_w) return gwm::set_err(h, GW_EINVAL, "gw_fsgw: F, qp_e and qp_w must be non-null");
    if (fopts && (fopts->tol < 0 || fopts->fock_tol < 0 || fopts->zeta_tol < 0 || fopts->max_outer < 0 ||
                  fopts->max_fock < 0 || fopts->diis_space < 0))
        return gwm::set_err(h, GW_EINVAL, "gw_fsgw: negative option");
    return gwm::fsgw_run(h, screening, nocc, nvir, naux, nmom_max, eps, L, F0, prec, opts, fopts, F, qp_e, qp_w,
                         info);
}

gw_status gw_naf(gw_handle h, int nocc, int nvir, int naux, const double* L, double eps_naf, int full_space,
                 double* L_naf, int* nnaf, double* eigenvalues) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (nocc < 1 || nvir < 1 || naux < 1) return gwm::set_err(h, GW_EINVAL, "nocc, nvir and naux must be >= 1");
    if (!L || !L_naf || !nnaf) return gwm::set_err(h, GW_EINVAL, "gw_naf: L, L_naf and nnaf must be non-null");
    if (!(eps_naf >= 0.0) || !std::isfinite(eps_naf)) return gwm::set_err(h, GW_EINVAL, "gw_naf: eps_naf must be >= 0");
    if (full_space != 0 && full_space != 1) return gwm::set_err(h, GW_EINVAL, "gw_naf: full_space must be 0 or 1");
    const long long nmo = nocc + nvir;
    if (nmo * nmo > 0x7fffffffLL || (long long)naux * nmo * nmo > (1LL << 40))
        return gwm::set_err(h, GW_EINVAL, "gw_naf: problem too large");
    *nnaf = 0;
    return gwm::naf_run(h, nocc, nvir, naux, L, eps_naf, full_space, L_naf, nnaf, eigenvalues);
}

gw_status gw_qsgw(gw_handle h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                  const double* L, gw_precision prec, const gw_opts* opts, const gw_qsgw_opts* qopts, double* qp_e,
                  double* C, double* F, gw_qsgw_info* info) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    GW_TRY(validate_common(h, nocc, nvir, naux, nmom_max, eps, L));
    GW_TRY(check_opts(h, prec, opts));
    if (screening != GW_TDA && screening != GW_RPA) return gwm::set_err(h, GW_EINVAL, "unknown screening");
    if (nmom_max % 2 == 0 || nmom_max > 15)
        return gwm::set_err(h, GW_EINVAL, "qsGW: nmom_max must be odd and <= 15");
    if (prec == GW_MIXED && nmom_max > 11)
        return gwm::set_err(h, GW_EINVAL, "mixed precision: nmom_max must be <= 11");
    if (!qp_e) return gwm::set_err(h, GW_EINVAL, "gw_qsgw: qp_e must be non-null");
    if (qopts && (qopts->scheme < 0 || qopts->scheme > 1 || qopts->srg_s < 0 || qopts->delta < 0 ||
                  qopts->tol < 0 || qopts->max_iter < 0 || qopts->max_scf < 0 || qopts->scf_tol < 0 ||
                  qopts->diis_space < 0 || !std::isfinite(qopts->srg_s) || !std::isfinite(qopts->delta)))
        return gwm::set_err(h, GW_EINVAL, "gw_qsgw: invalid option");
    return gwm::qsgw_run(h, screening, nocc, nvir, naux, nmom_max, eps, L, prec, opts, qopts, qp_e, C, F, info);
}

gw_status gw_spectral(gw_handle h, int nmo, int dim, int ld_chi, const double* E, const double* chi, int nomega,
                      const double* omega, double delta, double* A, double* A_orb) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (nmo < 1 || dim < 1 || ld_chi < dim || nomega < 1)
        return gwm::set_err(h, GW_EINVAL, "gw_spectral: need nmo, dim, nomega >= 1 and ld_chi >= dim");
    if ((long long)nmo * ld_chi > (1LL << 40) || (long long)nmo * nomega > (1LL << 40))
        return gwm::set_err(h, GW_EINVAL, "gw_spectral: problem too large");
    if (!(delta > 0.0) || !std::isfinite(delta)) return gwm::set_err(h, GW_EINVAL, "gw_spectral: delta must be > 0");
    if (!E || !chi || !omega) return gwm::set_err(h, GW_EINVAL, "gw_spectral: E, chi and omega must be non-null");
    if (!A && !A_orb) return gwm::set_err(h, GW_EINVAL, "gw_spectral: A and A_orb are both null");
    return gwm::spectral_run(h, nmo, dim, ld_chi, E, chi, nomega, omega, delta, A, A_orb);
}

gw_status gw_aufbau(gw_handle h, int nmo, int dim, int ld_chi, const double* E, const double* chi, double nelec,
                    double* rho, gw_aufbau_info* info) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (nmo < 1 || dim < 1 || ld_chi < dim)
        return gwm::set_err(h, GW_EINVAL, "gw_aufbau: need nmo, dim >= 1 and ld_chi >= dim");
    if ((long long)nmo * ld_chi > (1LL << 40)) return gwm::set_err(h, GW_EINVAL, "gw_aufbau: problem too large");
    if (!(nelec >= 0.0) || !std::isfinite(nelec)) return gwm::set_err(h, GW_EINVAL, "gw_aufbau: nelec must be >= 0");
    if (!E || !chi) return gwm::set_err(h, GW_EINVAL, "gw_aufbau: E and chi must be non-null");
    return gwm::aufbau_run(h, nmo, dim, ld_chi, E, chi, nelec, rho, info);
}

gw_status gw_zeta_shift(gw_handle h, int nmo, int nmom_max, int npole_occ, int npole_vir, const double* fock,
                        const double* pole_e, const double* pole_v, double nelec, const gw_zeta_opts* zopts,
                        double* E, double* chi, double* qp_e, double* qp_w, gw_zeta_info* info) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (nmo < 1) return gwm::set_err(h, GW_EINVAL, "nmo must be >= 1");
    if (nmom_max < 1 || nmom_max % 2 == 0 || nmom_max > 15)
        return gwm::set_err(h, GW_EINVAL, "nmom_max must be odd and in [1, 15]");
    const long long cap = (long long)nmo * (nmom_max + 1) / 2;
    if (npole_occ < 0 || npole_vir < 0 || npole_occ > cap || npole_vir > cap)
        return gwm::set_err(h, GW_EINVAL, "gw_zeta_shift: pole counts out of range");
    if (!(nelec >= 0.0) || !std::isfinite(nelec)) return gwm::set_err(h, GW_EINVAL, "gw_zeta_shift: nelec must be >= 0");
    if (zopts && (zopts->zeta_tol < 0 || !std::isfinite(zopts->zeta_lo) || !std::isfinite(zopts->zeta_hi)))
        return gwm::set_err(h, GW_EINVAL, "gw_zeta_shift: invalid options");
    if (!fock || !pole_e || !pole_v || !E || !qp_e || !qp_w)
        return gwm::set_err(h, GW_EINVAL, "gw_zeta_shift: a required pointer is null");
    return gwm::zeta_shift_run(h, nmo, nmom_max, npole_occ, npole_vir, fock, pole_e, pole_v, nelec, zopts, E, chi,
                               qp_e, qp_w, info);
}

gw_status gw_evgw(gw_handle h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                  const double* L, gw_precision prec, const gw_opts* opts, const gw_evgw_opts* eopts, double* qp_e,
                  double* qp_w, gw_evgw_info* info) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    GW_TRY(validate_common(h, nocc, nvir, naux, nmom_max, eps, L));
    GW_TRY(check_opts(h, prec, opts));
    if (screening != GW_TDA && screening != GW_RPA) return gwm::set_err(h, GW_EINVAL, "unknown screening");
    if (nmom_max % 2 == 0 || nmom_max > 15)
        return gwm::set_err(h, GW_EINVAL, "evGW: nmom_max must be odd and <= 15");
    if (prec == GW_MIXED && nmom_max > 11)
        return gwm::set_err(h, GW_EINVAL, "mixed precision: nmom_max must be <= 11");
    if (!qp_e || !qp_w) return gwm::set_err(h, GW_EINVAL, "gw_evgw: qp_e and qp_w must be non-null");
    if (eopts && (eopts->tol < 0 || eopts->max_iter < 0 || eopts->g0 < 0 || eopts->g0 > 1 || eopts->w0 < 0 ||
                  eopts->w0 > 1))
        return gwm::set_err(h, GW_EINVAL, "gw_evgw: bad option (g0, w0 in {0, 1}; tol, max_iter >= 0)");
    return gwm::evgw_run(h, screening, nocc, nvir, naux, nmom_max, eps, L, prec, opts, eopts, qp_e, qp_w, info);
}

gw_status gw_batch_create(gw_handle h, int nsys, const gw_system* sys, gw_screening screening, int nmom_max,
                          gw_precision prec, const gw_opts* opts, const gw_batch_opts* bopts, gw_batch* batch) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (!batch) return gwm::set_err(h, GW_EINVAL, "gw_batch_create: batch must be non-null");
    *batch = nullptr;
    if (nsys < 1 || !sys) return gwm::set_err(h, GW_EINVAL, "gw_batch_create: need at least one system");
    if (screening != GW_TDA && screening != GW_RPA) return gwm::set_err(h, GW_EINVAL, "unknown screening");
    GW_TRY(check_opts(h, prec, opts));
    if (prec == GW_MIXED && nmom_max > 11)
        return gwm::set_err(h, GW_EINVAL, "mixed precision: nmom_max must be <= 11");
    if (prec == GW_MIXED && nmom_max % 2 == 0)
        return gwm::set_err(h, GW_EINVAL, "mixed precision: nmom_max must be odd");
    if (bopts && (bopts->split_target < 0 || bopts->small_tile_nmo < 0))
        return gwm::set_err(h, GW_EINVAL, "gw_batch_create: negative option");
    for (int i = 0; i < nsys; ++i) {
        GW_TRY(validate_common(h, sys[i].nocc, sys[i].nvir, sys[i].naux, nmom_max, sys[i].eps, sys[i].L));
        if (!sys[i].sigma_occ || !sys[i].sigma_vir)
            return gwm::set_err(h, GW_EINVAL, "gw_batch_create: sigma outputs must be non-null");
    }
    return gwm::batch_create(h, nsys, sys, screening, nmom_max, prec, opts, bopts, batch);
}

gw_status gw_batch_run(gw_batch batch) {
    if (!batch) return GW_EINVAL;
    return gwm::batch_run(batch);
}

gw_status gw_batch_info(gw_batch batch, int* njobs, int* nwaves, int* graph, int* split_target,
                        int* small_tile_nmo) {
    if (!batch) return GW_EINVAL;
    return gwm::batch_info(batch, njobs, nwaves, graph, split_target, small_tile_nmo);
}

gw_status gw_batch_destroy(gw_batch batch) {
    gwm::batch_destroy(batch);
    return GW_OK;
}

long gw_mlp_param_count(void) { return gwm::mlp_param_count(); }

gw_status gw_mlp_features(gw_handle h, int nocc, int nvir, int naux, const double* eps, const double* L,
                          float* feat) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (nocc < 1 || nvir < 1 || naux < 1 || !eps || !L || !feat)
        return gwm::set_err(h, GW_EINVAL, "gw_mlp_features: bad sizes or null pointer");
    return gwm::mlp_features(h, nocc, nvir, naux, eps, L, feat);
}

gw_status gw_mlp_forward(gw_handle h, int rows, const float* params, const float* norm, const float* x, float* act,
                         float* y) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (rows < 1 || !params || !norm || !x || !y) return gwm::set_err(h, GW_EINVAL, "gw_mlp_forward: bad arguments");
    return gwm::mlp_forward(h, rows, params, norm, x, act, y);
}

gw_status gw_mlp_backward(gw_handle h, int rows, const float* params, const float* norm, const float* x,
                          const float* act, const float* y, const float* target, float* grad, float* loss) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (rows < 1 || !params || !norm || !x || !act || !y || !target || !grad)
        return gwm::set_err(h, GW_EINVAL, "gw_mlp_backward: bad arguments");
    return gwm::mlp_backward(h, rows, params, norm, x, act, y, target, grad, loss);
}

gw_status gw_mlp_norm(gw_handle h, int rows, const float* x, const float* target, float* norm) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (rows < 1 || !x || !target || !norm) return gwm::set_err(h, GW_EINVAL, "gw_mlp_norm: bad arguments");
    return gwm::mlp_norm(h, rows, x, target, norm);
}

gw_status gw_mlp_target(gw_handle h, int nmo, const double* F, const double* eps, float* target) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (nmo < 1 || !F || !eps || !target) return gwm::set_err(h, GW_EINVAL, "gw_mlp_target: bad arguments");
    return gwm::mlp_target(h, nmo, F, eps, target);
}

gw_status gw_mlp_warm_start(gw_handle h, int nocc, int nvir, int naux, const double* eps, const double* L,
                            const float* params, const float* norm, double* F0) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (nocc < 1 || nvir < 1 || naux < 1 || !eps || !L || !params || !norm || !F0)
        return gwm::set_err(h, GW_EINVAL, "gw_mlp_warm_start: bad sizes or null pointer");
    return gwm::mlp_warm_start(h, nocc, nvir, naux, eps, L, params, norm, F0);
}

gw_status gw_mlp_adam(gw_handle h, int step, float lr, float beta1, float beta2, float eps, float* params,
                      const float* grad, float* m, float* v) {
    if (!h) return GW_EINVAL;
    GW_HIP(h, hipSetDevice(h->device));
    if (step < 1 || !params || !grad || !m || !v || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return gwm::set_err(h, GW_EINVAL, "gw_mlp_adam: bad arguments");
    return gwm::mlp_adam(h, step, lr, beta1, beta2, eps, params, grad, m, v);
}

}  // extern "C"
