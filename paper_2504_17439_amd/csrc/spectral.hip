// Green's-function post-processing of the upfolded Hamiltonian:
//   spectral function (eqs. ret_GF, spectrum),
//   Aufbau filling and correlated density matrix (eq. density),
//   electron-number conserving one-shot GW through a shift of the auxiliary
//   energies (Sec. 3.5).
//
// The spectral function is a Lorentzian-weighted sum over the eigenstates of
// H~, for every (orbital p, frequency w)
//   A_p(w) = sum_a chi_{pa}^2 K_a(w),  K_a(w) = (delta/pi) / ((w - E_a)^2 + delta^2),
// i.e. the matrix product of the squared amplitudes [nmo][dim] with the
// Lorentzian matrix [dim][nomega]: one kernel writes K (one division per
// state and frequency, frequencies in chunks of at most 2^27 entries), one
// squares the amplitudes, and the product runs as an FP64 GEMM on the matrix
// cores (rocBLAS).  The total A(w) is the column sum of the A_p when they
// are computed, else the product of the state weights w_a = sum_p chi_{pa}^2
// with K.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gwm {

namespace {

unsigned nbk(long n) { return (unsigned)((n + 255) / 256); }

// K[a][k] = (delta/pi) / ((omega_k - E_a)^2 + delta^2), [dim][nw]
__global__ void lorentz_matrix_kernel(int dim, int nw, const double* __restrict__ E, const double* __restrict__ omega,
                                      double delta, double* __restrict__ K) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)dim * nw) return;
    const int a = (int)(i / nw), k = (int)(i % nw);
    const double x = omega[k] - E[a];
    K[i] = (delta / M_PI) / (x * x + delta * delta);
}

// C2[p][a] = chi[p][a]^2, [nmo][dim] packed
__global__ void square_kernel(int nmo, int dim, long ld, const double* __restrict__ chi, double* __restrict__ C2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)nmo * dim) return;
    const int p = (int)(i / dim), a = (int)(i % dim);
    const double x = chi[(long)p * ld + a];
    C2[i] = x * x;
}

// out[c] = sum_r f(X[r][c]), f(x) = x^2 (SQ) or x: column sums of a row-major
// [rows][ld] array (the physical weight of state c when X = chi).  Block: 64
// columns x 16 row groups (row r in group r % 16), partial sums combined in
// LDS in a fixed order.  Grid: ceil(cols / 64).
template <bool SQ>
__global__ __launch_bounds__(1024) void colsum_kernel(int rows, int cols, long ld, const double* __restrict__ X,
                                                      double* __restrict__ out) {
    __shared__ double part[16][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int a = blockIdx.x * 64 + c;
    double s = 0.0;
    if (a < cols) {
#pragma unroll 4
        for (int r = g; r < rows; r += 16) {
            const double x = X[(long)r * ld + a];
            s += SQ ? x * x : x;
        }
    }
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && a < cols) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += part[k][c];
        out[a] = t;
    }
}

template <bool SQ>
gw_status colsum(Handle* h, int rows, int cols, long ld, const double* X, double* out) {
    hipLaunchKernelGGL(colsum_kernel<SQ>, dim3((unsigned)((cols + 63) / 64)), dim3(1024), 0, h->stream, rows, cols,
                       ld, X, out);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status state_weights(Handle* h, int nmo, int dim, long ld, const double* chi, double* wt) {
    return colsum<true>(h, nmo, dim, ld, chi, wt);
}

__global__ void fill_kernel(long n, double v, double* __restrict__ x) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// chi[p][a] = H[a][p] (H: eigenvectors as rows, dim x dim)
__global__ void rows_to_chi_kernel(int M, int dim, long ldchi, const double* __restrict__ H,
                                   double* __restrict__ chi) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)M * dim) return;
    const int p = (int)(i / dim), a = (int)(i % dim);
    chi[(long)p * ldchi + a] = H[(long)a * dim + p];
}

}  // namespace

gw_status spectral_run(Handle* h, int nmo, int dim, int ld_chi, const double* E, const double* chi, int nomega,
                       const double* omega, double delta, double* A, double* A_orb) {
    const long kc = std::max(1L, std::min((long)nomega, (1L << 27) / dim));
    double* K = (double*)ws_get(h, WS_FS1, sizeof(double) * (size_t)dim * kc);
    double* wt = (double*)ws_get(h, WS_MISC, sizeof(double) * ((size_t)dim + 16));
    double* C2 = A_orb ? (double*)ws_get(h, WS_FS0, sizeof(double) * (size_t)nmo * dim) : nullptr;
    if (!K || !wt || (A_orb && !C2)) return GW_ENOMEM;
    if (A_orb) {
        hipLaunchKernelGGL(square_kernel, dim3(nbk((long)nmo * dim)), dim3(256), 0, h->stream, nmo, dim,
                           (long)ld_chi, chi, C2);
        GW_CHECK_LAUNCH(h);
    }
    // the total: column sums of A_orb when it is computed, else the state
    // weights times K
    if (A && !A_orb) GW_TRY(state_weights(h, nmo, dim, ld_chi, chi, wt));
    if (rocblas_set_stream(h->blas, h->stream) != rocblas_status_success)
        return set_err(h, GW_ELIB, "rocblas_set_stream");
    for (long k0 = 0; k0 < nomega; k0 += kc) {
        const int nw = (int)std::min(kc, (long)nomega - k0);
        hipLaunchKernelGGL(lorentz_matrix_kernel, dim3(nbk((long)dim * nw)), dim3(256), 0, h->stream, dim, nw, E,
                           omega + k0, delta, K);
        GW_CHECK_LAUNCH(h);
        if (A_orb) GW_TRY(gemm_rowmajor(h, false, false, nmo, nw, dim, 1.0, C2, dim, K, nw, 0.0, A_orb + k0, nomega));
        else GW_TRY(gemm_rowmajor(h, false, false, 1, nw, dim, 1.0, wt, dim, K, nw, 0.0, A + k0, nomega));
    }
    if (A && A_orb) GW_TRY(colsum<false>(h, nmo, nomega, nomega, A_orb, A));
    return GW_OK;
}

gw_status aufbau_run(Handle* h, int nmo, int dim, int ld_chi, const double* E, const double* chi, double nelec,
                     double* rho, gw_aufbau_info* info) {
    double* wt = (double*)ws_get(h, WS_MISC, sizeof(double) * ((size_t)dim + 16));
    if (!wt) return GW_ENOMEM;
    GW_TRY(state_weights(h, nmo, dim, ld_chi, chi, wt));
    std::vector<double> hw(dim), he(dim);
    GW_HIP(h, hipMemcpyAsync(hw.data(), wt, sizeof(double) * dim, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipMemcpyAsync(he.data(), E, sizeof(double) * dim, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    for (int a = 1; a < dim; ++a)
        if (!(he[a] >= he[a - 1])) return set_err(h, GW_EINVAL, "gw_aufbau: E must be ascending");
    double cum = 0.0, best = std::fabs(nelec);
    int n = 0;
    for (int a = 0; a < dim; ++a) {
        cum += 2.0 * hw[a];
        if (std::fabs(cum - nelec) < best) {
            best = std::fabs(cum - nelec);
            n = a + 1;
        }
    }
    double tr = 0.0;
    for (int a = 0; a < n; ++a) tr += 2.0 * hw[a];
    if (rho) {
        const long M2 = (long)nmo * nmo;
        if (rocblas_set_stream(h->blas, h->stream) != rocblas_status_success)
            return set_err(h, GW_ELIB, "rocblas_set_stream");
        if (n > 0) GW_TRY(gemm_rowmajor(h, false, true, nmo, nmo, n, 2.0, chi, ld_chi, chi, ld_chi, 0.0, rho, nmo));
        else {
            hipLaunchKernelGGL(fill_kernel, dim3(nbk(M2)), dim3(256), 0, h->stream, M2, 0.0, rho);
            GW_CHECK_LAUNCH(h);
        }
        GW_HIP(h, hipStreamSynchronize(h->stream));
    }
    if (info) {
        info->nfill = n;
        info->nelec = tr;
        info->homo = n > 0 ? n - 1 : -1;
        info->lumo = n < dim ? n : -1;
        if (n > 0 && n < dim) info->mu = 0.5 * (he[n - 1] + he[n]);
        else info->mu = n > 0 ? he[n - 1] : he[0];
    }
    return GW_OK;
}

gw_status zeta_shift_run(Handle* h, int nmo, int nmom_max, int npole_occ, int npole_vir, const double* fock,
                         const double* pole_e, const double* pole_v, double nelec, const gw_zeta_opts* zo, double* E,
                         double* chi, double* qp_e, double* qp_w, gw_zeta_info* info) {
    double zlo = -1.0, zhi = 1.0;
    if (zo && zo->zeta_hi > zo->zeta_lo) {
        zlo = zo->zeta_lo;
        zhi = zo->zeta_hi;
    }
    const double ztol = (zo && zo->zeta_tol > 0) ? zo->zeta_tol : 1e-13;
    const int M = nmo, np = npole_occ + npole_vir;
    const long ldv = (long)nmo * (nmom_max + 1);
    const long dim_max = (long)nmo * (nmom_max + 2);
    const long dim = (long)M + np;
    double* H = (double*)ws_get(h, WS_FS4, sizeof(double) * (dim * dim + 3 * dim + 16));
    int* dinfo = (int*)ws_get(h, WS_FS6, sizeof(int) * 64);
    if (!H || !dinfo) return GW_ENOMEM;
    ZetaSearch zs;
    zs.M = M;
    zs.np = np;
    zs.F = fock;
    zs.pole_e = pole_e;
    zs.pole_v = pole_v;
    zs.ldv = ldv;
    zs.H = H;
    zs.w = H + dim * dim;
    zs.work = zs.w + dim;
    zs.wt = zs.work + dim;
    zs.info = dinfo;
    double zeta = 0.0, tr = 0.0;
    int nf = 0;
    GW_TRY(zeta_solve(h, zs, nelec, 0.0, zlo, zhi, ztol, &zeta, &tr, &nf));
    GW_TRY(copy_f64(h, E, zs.w, (size_t)dim));
    if (chi) {
        hipLaunchKernelGGL(rows_to_chi_kernel, dim3(nbk((long)M * dim)), dim3(256), 0, h->stream, M, (int)dim,
                           dim_max, zs.H, chi);
        GW_CHECK_LAUNCH(h);
    }
    GW_TRY(qp_assign_dev(h, M, (int)dim, zs.H, zs.w, qp_e, qp_w));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    if (info) {
        info->zeta = zeta;
        info->nfill = nf;
        info->nelec = tr;
        info->eig_calls = zs.eig_calls;
    }
    return GW_OK;
}

}  // namespace gwm
