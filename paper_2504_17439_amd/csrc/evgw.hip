// Eigenvalue self-consistent moment GW (App. A, Alg. A1): evGW, evGW0 (W kept
// at the reference), G with W updated, and G0W0 as the case with nothing
// updated.  Two sets of orbital energies live on the device: eps_G enters the
// eps-power factors of the convolution (eqs. convolution_occ / convolution_vir),
// eps_W the energy differences of the density-response recursion
// (eq. energy_differences).  Every iteration runs the hot path (moments,
// self-energy moments, block Lanczos, upfolded Hamiltonian with f =
// diag(eps_ref), QP assignment by eq. quasiparticle_energy_update) and replaces
// eps_G and / or eps_W by the QP energies (or their DIIS extrapolation over
// the last iterations, error vector = QP energies - input energies, on the
// host: nmo-vectors); the loop stops when, for every quasiparticle-like
// orbital (QP weight >= 0.9 in both iterations; all orbitals if none is), the
// QP energy differs by at most tol from the energy that went into the
// iteration (the fixed-point residual; for the plain loop the change since
// the previous iteration): an orbital embedded in a satellite band has no
// stable QP assignment.  Unless the caller sets opts->moment_eps, the
// Lanczos inside the loop deflates at the moments' accuracy (FP64 1e-12,
// mixed 1e-9), not the unit roundoff: directions resolved from rounding
// noise give satellite poles whose assignment moves by ~1e-5 Ha between
// iterations and keep the loop from converging.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gwm {

namespace {

__global__ void diag_kernel(int M, const double* __restrict__ d, double* __restrict__ A) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)M * M) return;
    const int r = (int)(i / M), c = (int)(i % M);
    A[i] = r == c ? d[r] : 0.0;
}

}  // namespace

gw_status evgw_run(Handle* h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                   const double* L, gw_precision prec, const gw_opts* opts, const gw_evgw_opts* eo, double* qp_e,
                   double* qp_w, gw_evgw_info* info) {
    const bool g0 = eo && eo->g0, w0 = eo && eo->w0;
    const double tol = (eo && eo->tol > 0) ? eo->tol : 1e-6;
    const int max_iter = (eo && eo->max_iter > 0) ? eo->max_iter : 30;
    const int diis_space = (eo && eo->diis_space != 0) ? eo->diis_space : 12;
    gw_opts lo = opts ? *opts : gw_opts{};
    if (!(lo.moment_eps > 0)) lo.moment_eps = prec == GW_MIXED ? 1e-9 : 1e-12;
    opts = &lo;
    const int M = nocc + nvir, nt = nmom_max + 1;
    const long M2 = (long)M * M;
    const int cap = M * nt / 2;
    const long ldv = 2L * cap;
    const long dim_max = (long)M * (nmom_max + 2);

    double* sig = (double*)ws_get(h, WS_FS2, sizeof(double) * 2 * nt * M2);
    double* pol = (double*)ws_get(h, WS_FS3, sizeof(double) * (2 * cap + (long)M * ldv));
    double* vec = (double*)ws_get(h, WS_FS4, sizeof(double) * (dim_max + 3 * M + M2));
    double* R = (double*)ws_get(h, WS_R, sizeof(double) * nt * (long)naux * naux);
    if (!sig || !pol || !vec || !R) return GW_ENOMEM;
    double* so = sig;
    double* sv = sig + nt * M2;
    double* pole_e = pol;
    double* pole_v = pol + 2 * cap;
    double* E = vec;
    double* eG = vec + dim_max;
    double* eW = eG + M;
    double* fock = eW + M;

    hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((M2 + 255) / 256)), dim3(256), 0, h->stream, M, eps, fock);
    GW_CHECK_LAUNCH(h);
    GW_TRY(copy_f64(h, eG, eps, M));
    GW_TRY(copy_f64(h, eW, eps, M));
    std::vector<double> prev(M), cur(M), wcur(M), wprev(M, 1.0), xin(M), err(M), next(M);
    GW_HIP(h, hipMemcpyAsync(prev.data(), eps, sizeof(double) * M, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    xin = prev;                      // the energies the updated set(s) hold
    Diis diis{std::max(diis_space, 1), (size_t)M, {}, {}, {}};

    int it = 0;
    bool converged = false;
    double change = -1.0;
    for (it = 1; it <= max_iter; ++it) {
        // screening on eps_W, convolution on eps_G
        if (screening == GW_TDA && prec == GW_MIXED) GW_TRY(tda_moments_mixed(h, nocc, nvir, naux, nmom_max, eW, L, R));
        else if (screening == GW_TDA) GW_TRY(tda_moments_f64(h, nocc, nvir, naux, nmom_max, eW, L, R, nullptr));
        else if (prec == GW_MIXED) GW_TRY(rpa_moments_mixed(h, nocc, nvir, naux, nmom_max, eW, L, opts, R));
        else GW_TRY(rpa_moments_f64(h, nocc, nvir, naux, nmom_max, eW, L, opts, R, nullptr));
        if (prec == GW_MIXED) GW_TRY(sigma_from_R_mixed(h, nocc, nvir, naux, nmom_max, eG, L, R, opts, so, sv));
        else GW_TRY(sigma_from_R_f64(h, nocc, nvir, naux, nmom_max, eG, L, R, opts, so, sv));
        int no = 0, nv = 0;
        GW_TRY(poles_f64(h, M, nmom_max, so, sv, fock, opts, &no, &nv, pole_e, pole_v, E, nullptr, qp_e, qp_w));
        GW_HIP(h, hipMemcpyAsync(cur.data(), qp_e, sizeof(double) * M, hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipMemcpyAsync(wcur.data(), qp_w, sizeof(double) * M, hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        bool any = false;
        for (int p = 0; p < M; ++p) any = any || (wcur[p] >= 0.9 && wprev[p] >= 0.9);
        change = 0.0;
        for (int p = 0; p < M; ++p)
            if (!any || (wcur[p] >= 0.9 && wprev[p] >= 0.9)) change = std::max(change, std::fabs(cur[p] - xin[p]));
        if (g0 && w0) {
            converged = true;
            break;
        }
        if (diis_space > 0) {
            for (int p = 0; p < M; ++p) err[p] = cur[p] - xin[p];
            diis.push(cur.data(), err.data());
            const double* x = diis.extrapolate();
            next.assign(x, x + M);
        } else {
            next = cur;
        }
        if (!w0) {
            // the next screening needs D_ia = eps_a - eps_i > 0
            const double ho = *std::max_element(next.begin(), next.begin() + nocc);
            const double lv = *std::min_element(next.begin() + nocc, next.end());
            if (!(ho < lv)) {
                if (info) *info = gw_evgw_info{it, 0, change};
                return set_err(h, GW_ENUMERIC, "evGW: occupied and virtual QP energies cross");
            }
        }
        GW_HIP(h, hipMemcpyAsync(vec + dim_max + 2 * M + M2, next.data(), sizeof(double) * M, hipMemcpyHostToDevice,
                                 h->stream));
        if (!g0) GW_TRY(copy_f64(h, eG, vec + dim_max + 2 * M + M2, M));
        if (!w0) GW_TRY(copy_f64(h, eW, vec + dim_max + 2 * M + M2, M));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        xin = next;
        if (change < tol) {
            converged = true;
            break;
        }
        wprev = wcur;
    }
    if (info) *info = gw_evgw_info{std::min(it, max_iter), converged ? 1 : 0, change};
    if (!converged) return set_err(h, GW_ENOCONV, "evGW: no convergence within max_iter iterations");
    return GW_OK;
}

}  // namespace gwm
