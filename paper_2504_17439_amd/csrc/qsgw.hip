// Quasiparticle self-consistent moment GW (Sec. 3.3, App. A Alg. A2).
//
// State: mean-field orbitals (rows of Ut, in the reference MO basis) and
// energies e.  One iteration:
//   L_P <- C^T L_P C (C = Ut^T); moments and self-energy moments with e
//   (screening and Green's function), block Lanczos -> auxiliary poles
//   (e_l, v_pl), already diagonal in the external space;
//   static potential at eps_p = e_p (static_potential_kernel):
//     SRG        V_pq = sum_l v_pl v_ql (D_pl + D_ql) / (D_pl^2 + D_ql^2) (1 - exp(-(D_pl^2 + D_ql^2) s)),
//     Lorentzian V_pq = 1/2 sum_l v_pl v_ql [D_pl / (D_pl^2 + delta^2) + D_ql / (D_ql^2 + delta^2)],
//   D_pl = e_p - e_l; V moved to the reference basis, Vr = C V C^T, and
//   replaced by the DIIS extrapolation over the potentials built so far
//   (error vector Vr - the potential of the previous SCF, zero at the start);
//   SCF of (f[rho] + Vr) C = C e with f[rho] = h + J[rho] - K[rho]/2 (the core
//   Hamiltonian of the Fock loop, f[rho0] = diag(eps)), rho from the nocc
//   lowest orbitals (exchange built from those orbitals, K = 2 sum_P
//   (Co L_P)^T (Co L_P)), DIIS over the Fock matrices with the commutator
//   F rho - rho F as error vector, until max |rho_k - rho_{k-1}| < scf_tol;
//   converged when the sorted e change by less than tol.
// The QP energies are the final mean-field e (unit weights).
//
// Device work: GEMMs and eigensolves through rocBLAS / rocSOLVER, the static
// potential as a tiled kernel (O(nmo^2 npole), one exp per element and pole);
// the host keeps the two DIIS extrapolations (at most diis_space and
// outer_diis pairs of nmo^2 vectors) and the convergence tests.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gwm {

namespace {

unsigned nbq(long n) { return (unsigned)((n + 255) / 256); }

constexpr int QT = 32;   // (p, q) tile edge
constexpr int QL = 64;   // poles per LDS chunk

// V[p][q] for a 32 x 32 tile per block, 256 threads, 4 rows per thread.
// SRG: SCHEME 0, Lorentzian: SCHEME 1.  Poles: e [np], v [M][ldv] (columns).
template <int SCHEME>
__global__ __launch_bounds__(256) void static_potential_kernel(int M, int np, const double* __restrict__ eps,
                                                               const double* __restrict__ pe,
                                                               const double* __restrict__ pv, long ldv, double s,
                                                               double delta, double* __restrict__ V) {
    __shared__ double vp[QT][QL + 1];
    __shared__ double vq[QT][QL + 1];
    __shared__ double el[QL];
    const int tid = threadIdx.x;
    const int tq = tid % QT, tp = tid / QT;   // tp in [0, 8): rows 4 tp .. 4 tp + 3
    const int p0 = blockIdx.y * QT, q0 = blockIdx.x * QT;
    const int q = q0 + tq;
    const double eq = q < M ? eps[q] : 0.0;
    double ep[4], acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int p = p0 + 4 * tp + j;
        ep[j] = p < M ? eps[p] : 0.0;
        acc[j] = 0.0;
    }
    const double d2 = delta * delta;
    for (int l0 = 0; l0 < np; l0 += QL) {
#pragma unroll
        for (int i = 0; i < (QT * QL) / 256; ++i) {
            const int e = tid + 256 * i;
            const int r = e / QL, c = e % QL;
            const bool ok = l0 + c < np;
            vp[r][c] = (ok && p0 + r < M) ? pv[(long)(p0 + r) * ldv + l0 + c] : 0.0;
            vq[r][c] = (ok && q0 + r < M) ? pv[(long)(q0 + r) * ldv + l0 + c] : 0.0;
        }
        if (tid < QL) el[tid] = l0 + tid < np ? pe[l0 + tid] : 0.0;
        __syncthreads();
        for (int c = 0; c < QL; ++c) {
            const double e = el[c];
            const double dq = eq - e;
            const double wq = vq[tq][c];
            if (SCHEME == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double dp = ep[j] - e;
                    const double x = dp * dp + dq * dq;
                    const double g = x > 0.0 ? (dp + dq) * (-expm1(-x * s)) / x : 0.0;
                    acc[j] += vp[4 * tp + j][c] * wq * g;
                }
            } else {
                const double aq = dq / (dq * dq + d2);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double dp = ep[j] - e;
                    const double g = 0.5 * (dp / (dp * dp + d2) + aq);
                    acc[j] += vp[4 * tp + j][c] * wq * g;
                }
            }
        }
        __syncthreads();
    }
    if (q >= M) return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int p = p0 + 4 * tp + j;
        if (p < M) V[(long)p * M + q] = acc[j];
    }
}

__global__ void qs_diag_kernel(int M, const double* __restrict__ d, double s, int nlead, double* __restrict__ X) {
    // X = diag(d) (d non-null) or diag(s * 1_{p < nlead})
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)M * M) return;
    const int r = (int)(i / M), c = (int)(i % M);
    double v = 0.0;
    if (r == c) v = d ? d[r] : (r < nlead ? s : 0.0);
    X[i] = v;
}

// out = a + cb*b + cc*c + d (elementwise; d nullable)
__global__ void qs_comb_kernel(long n, const double* __restrict__ a, const double* __restrict__ b, double cb,
                               const double* __restrict__ c, double cc, const double* __restrict__ d,
                               double* __restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = a[i] + cb * b[i] + cc * c[i] + (d ? d[i] : 0.0);
}

__global__ void qs_transpose_kernel(int M, const double* __restrict__ X, double* __restrict__ Y) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)M * M) return;
    const int r = (int)(i / M), c = (int)(i % M);
    Y[(long)c * M + r] = X[i];
}

}  // namespace

gw_status qsgw_run(Handle* h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                   const double* L, gw_precision prec, const gw_opts* opts, const gw_qsgw_opts* qo, double* qp_e,
                   double* Cout, double* Fout, gw_qsgw_info* info) {
    const int scheme = qo ? qo->scheme : 0;
    const double srg_s = (qo && qo->srg_s > 0) ? qo->srg_s : 500.0;
    const double delta = (qo && qo->delta > 0) ? qo->delta : 1e-3;
    const double tol = (qo && qo->tol > 0) ? qo->tol : 1e-6;
    const int max_iter = (qo && qo->max_iter > 0) ? qo->max_iter : 30;
    const int max_scf = (qo && qo->max_scf > 0) ? qo->max_scf : 200;
    const double scf_tol = (qo && qo->scf_tol > 0) ? qo->scf_tol : 1e-10;
    const int diis_space = (qo && qo->diis_space > 0) ? qo->diis_space : 12;
    const int outer_space = (qo && qo->outer_diis != 0) ? qo->outer_diis : 12;
    const int M = nocc + nvir, A = naux, nt = nmom_max + 1;
    const long M2 = (long)M * M;
    const int cap = M * nt / 2;
    const long ldv = 2L * cap;

    double* Lc = (double*)ws_get(h, WS_FS0, sizeof(double) * A * M2);
    double* T = (double*)ws_get(h, WS_FS1, sizeof(double) * A * M2);
    double* sig = (double*)ws_get(h, WS_FS2, sizeof(double) * 2 * nt * M2);
    double* pol = (double*)ws_get(h, WS_FS3, sizeof(double) * (2 * cap + (long)M * ldv));
    double* mat = (double*)ws_get(h, WS_FS5, sizeof(double) * (13 * M2 + 4 * M + A + 64));
    double* R = (double*)ws_get(h, WS_R, sizeof(double) * nt * (long)A * A);
    int* dinfo = (int*)ws_get(h, WS_FS6, sizeof(int) * 64);
    if (!Lc || !T || !sig || !pol || !mat || !R || !dinfo) return GW_ENOMEM;
    double* so = sig;
    double* sv = sig + nt * M2;
    double* pole_e = pol;
    double* pole_v = pol + 2 * cap;
    double* hcore = mat;              // reference basis throughout
    double* Ut = mat + M2;            // orbitals as rows
    double* Vc = mat + 2 * M2;        // static potential, orbital basis
    double* Vr = mat + 3 * M2;        // static potential, reference basis
    double* F = mat + 4 * M2;         // f[rho] + Vr
    double* Fx = mat + 5 * M2;        // DIIS extrapolation -> eigenvectors
    double* rho = mat + 6 * M2;
    double* J = mat + 7 * M2;
    double* K = mat + 8 * M2;
    double* tmp = mat + 9 * M2;
    double* err = mat + 10 * M2;      // F rho - rho F
    double* rhon = mat + 11 * M2;
    double* ecur = mat + 12 * M2;     // [M] mean-field energies
    double* enew = ecur + M;          // [M]
    double* wtmp = enew + M;          // [M] eig work
    double* jv = wtmp + M;            // [A]
    double* Co = jv + A;              // [nocc][M] occupied orbitals (rows), rho = 2 Co^T Co

    if (rocblas_set_stream(h->blas, h->stream) != rocblas_status_success)
        return set_err(h, GW_ELIB, "rocblas_set_stream");

    // core Hamiltonian from the reference density; start: C = 1, e = eps, rho = rho0
    hipLaunchKernelGGL(qs_diag_kernel, dim3(nbq(M2)), dim3(256), 0, h->stream, M, (const double*)nullptr, 2.0, nocc,
                       rho);
    GW_CHECK_LAUNCH(h);
    GW_TRY(fock_jk(h, A, M, L, rho, J, K, T, jv));
    hipLaunchKernelGGL(qs_diag_kernel, dim3(nbq(M2)), dim3(256), 0, h->stream, M, eps, 0.0, 0, tmp);
    GW_CHECK_LAUNCH(h);
    hipLaunchKernelGGL(qs_comb_kernel, dim3(nbq(M2)), dim3(256), 0, h->stream, M2, tmp, J, -1.0, K, 0.5,
                       (const double*)nullptr, hcore);
    GW_CHECK_LAUNCH(h);
    hipLaunchKernelGGL(qs_diag_kernel, dim3(nbq(M2)), dim3(256), 0, h->stream, M, (const double*)nullptr, 1.0, M, Ut);
    GW_CHECK_LAUNCH(h);
    // the first nocc rows of diag(1_{p < nocc}) are the reference occupied orbitals
    hipLaunchKernelGGL(qs_diag_kernel, dim3(nbq(M2)), dim3(256), 0, h->stream, M, (const double*)nullptr, 1.0, nocc,
                       Co);
    GW_CHECK_LAUNCH(h);
    GW_TRY(copy_f64(h, ecur, eps, (size_t)M));

    std::vector<double> hF((size_t)M2), hE((size_t)M2), hr((size_t)M2), hrn((size_t)M2), he(M), hen(M);
    std::vector<double> hVo, hVi, hVe;   // outer DIIS: built potential, potential in use, their difference
    Diis outer{std::max(outer_space, 1), (size_t)M2, {}, {}, {}};
    if (outer_space > 0) {
        hVo.resize((size_t)M2);
        hVi.assign((size_t)M2, 0.0);
        hVe.resize((size_t)M2);
    }
    GW_HIP(h, hipMemcpyAsync(hr.data(), rho, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipMemcpyAsync(he.data(), eps, sizeof(double) * M, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));

    int it = 0, scf_steps = 0;
    bool converged = false;
    double last = -1.0;
    // Fock matrix of the current rho (= 2 Co^T Co) plus Vr into F
    auto build_fock = [&]() -> gw_status {
        GW_TRY(fock_jk_occ(h, A, M, L, rho, Co, nocc, J, K, T, (size_t)A * M2, jv));
        hipLaunchKernelGGL(qs_comb_kernel, dim3(nbq(M2)), dim3(256), 0, h->stream, M2, hcore, J, 1.0, K, -0.5,
                           (const double*)Vr, F);
        GW_CHECK_LAUNCH(h);
        return GW_OK;
    };
    for (it = 1; it <= max_iter; ++it) {
        // one-shot GW in the current orbital basis: L_P <- Ut L_P Ut^T
        GW_TRY(gemm_rm_batched(h, false, true, M, M, M, L, M, M2, Ut, M, 0, T, M, M2, A));
        GW_TRY(gemm_rm_batched(h, false, false, M, M, M, Ut, M, 0, T, M, M2, Lc, M, M2, A));
        if (screening == GW_TDA && prec == GW_MIXED) GW_TRY(tda_moments_mixed(h, nocc, nvir, A, nmom_max, ecur, Lc, R));
        else if (screening == GW_TDA) GW_TRY(tda_moments_f64(h, nocc, nvir, A, nmom_max, ecur, Lc, R, nullptr));
        else if (prec == GW_MIXED) GW_TRY(rpa_moments_mixed(h, nocc, nvir, A, nmom_max, ecur, Lc, opts, R));
        else GW_TRY(rpa_moments_f64(h, nocc, nvir, A, nmom_max, ecur, Lc, opts, R, nullptr));
        if (prec == GW_MIXED) GW_TRY(sigma_from_R_mixed(h, nocc, nvir, A, nmom_max, ecur, Lc, R, opts, so, sv));
        else GW_TRY(sigma_from_R_f64(h, nocc, nvir, A, nmom_max, ecur, Lc, R, opts, so, sv));
        int no = 0, nv = 0;
        GW_TRY(poles_lanczos(h, M, nmom_max, so, sv, opts, pole_e, pole_v, ldv, &no, &nv));
        if (rocblas_set_stream(h->blas, h->stream) != rocblas_status_success)
            return set_err(h, GW_ELIB, "rocblas_set_stream");
        // static potential in the orbital basis, then Vr = Ut^T Vc Ut
        {
            dim3 grid((unsigned)((M + QT - 1) / QT), (unsigned)((M + QT - 1) / QT));
            if (scheme == 1)
                hipLaunchKernelGGL(static_potential_kernel<1>, grid, dim3(256), 0, h->stream, M, no + nv, ecur,
                                   pole_e, pole_v, ldv, srg_s, delta, Vc);
            else
                hipLaunchKernelGGL(static_potential_kernel<0>, grid, dim3(256), 0, h->stream, M, no + nv, ecur,
                                   pole_e, pole_v, ldv, srg_s, delta, Vc);
            GW_CHECK_LAUNCH(h);
        }
        GW_TRY(gemm_rowmajor(h, false, false, M, M, M, 1.0, Vc, M, Ut, M, 0.0, tmp, M));
        GW_TRY(gemm_rowmajor(h, true, false, M, M, M, 1.0, Ut, M, tmp, M, 0.0, Vr, M));
        if (outer_space > 0) {
            GW_HIP(h, hipMemcpyAsync(hVo.data(), Vr, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
            GW_HIP(h, hipStreamSynchronize(h->stream));
            for (long i = 0; i < M2; ++i) hVe[i] = hVo[i] - hVi[i];
            outer.push(hVo.data(), hVe.data());
            const double* x = outer.extrapolate();
            hVi.assign(x, x + M2);
            GW_HIP(h, hipMemcpyAsync(Vr, hVi.data(), sizeof(double) * M2, hipMemcpyHostToDevice, h->stream));
        }

        // SCF of eq. qp_scf from the current density
        Diis diis{diis_space, (size_t)M2, {}, {}, {}};
        for (int step = 0; step < max_scf; ++step) {
            GW_TRY(build_fock());
            GW_TRY(gemm_rowmajor(h, false, false, M, M, M, 1.0, F, M, rho, M, 0.0, err, M));
            GW_TRY(gemm_rowmajor(h, false, false, M, M, M, -1.0, rho, M, F, M, 1.0, err, M));
            GW_HIP(h, hipMemcpyAsync(hF.data(), F, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
            GW_HIP(h, hipMemcpyAsync(hE.data(), err, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
            GW_HIP(h, hipStreamSynchronize(h->stream));
            diis.push(hF.data(), hE.data());
            const double* next = diis.extrapolate();
            GW_HIP(h, hipMemcpyAsync(Fx, next, sizeof(double) * M2, hipMemcpyHostToDevice, h->stream));
            GW_TRY(eigh_rows(h, M, Fx, enew, wtmp, dinfo));
            // rho = 2 sum_{i<nocc} u_i u_i^T (rows of Fx)
            GW_TRY(gemm_rowmajor(h, true, false, M, M, nocc, 2.0, Fx, M, Fx, M, 0.0, rhon, M));
            GW_HIP(h, hipMemcpyAsync(hrn.data(), rhon, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
            GW_HIP(h, hipStreamSynchronize(h->stream));
            ++scf_steps;
            double change = 0.0;
            for (long i = 0; i < M2; ++i) change = std::max(change, std::fabs(hrn[i] - hr[i]));
            GW_TRY(copy_f64(h, rho, rhon, (size_t)M2));
            GW_TRY(copy_f64(h, Co, Fx, (size_t)nocc * M));
            hr.swap(hrn);
            if (change < scf_tol) break;
        }
        // orbitals and energies of f[rho] + Vr
        GW_TRY(build_fock());
        GW_TRY(copy_f64(h, Ut, F, (size_t)M2));
        GW_TRY(eigh_rows(h, M, Ut, enew, wtmp, dinfo));
        GW_HIP(h, hipMemcpyAsync(hen.data(), enew, sizeof(double) * M, hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        std::vector<double> a(hen), b(he);
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        last = 0.0;
        for (int p = 0; p < M; ++p) last = std::max(last, std::fabs(a[p] - b[p]));
        GW_TRY(copy_f64(h, ecur, enew, (size_t)M));
        he.swap(hen);
        if (last < tol) {
            converged = true;
            break;
        }
    }
    if (it > max_iter) it = max_iter;
    GW_TRY(copy_f64(h, qp_e, ecur, (size_t)M));
    if (Cout) {
        // C[p][k] = Ut[k][p]: columns are the orbitals
        hipLaunchKernelGGL(qs_transpose_kernel, dim3(nbq(M2)), dim3(256), 0, h->stream, M, (const double*)Ut, Cout);
        GW_CHECK_LAUNCH(h);
    }
    if (Fout) GW_TRY(copy_f64(h, Fout, F, (size_t)M2));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    if (info) {
        info->iterations = it;
        info->scf_steps = scf_steps;
        info->converged = converged ? 1 : 0;
        info->last_change = last;
    }
    return converged ? GW_OK : set_err(h, GW_ENOCONV, "qsGW: reached max_iter without converging");
}

}  // namespace gwm
