// Fock / chemical-potential self-consistent moment GW (Sec. 3.6, Alg. 2).
//
// State: the Fock matrix F in the reference MO basis.  One outer iteration:
//   eig F -> orbital energies e, rotation C (rows of Ut are the orbitals);
//   L_P <- C^T L_P C, h <- C^T h C  (strided-batched GEMMs);
//   self-energy moments in that basis (TDA or RPA screening, FP64 or mixed);
//   block Lanczos -> auxiliary poles (e_aux, W);
//   Fock loop in the rotated basis, starting from diag(e):
//     zeta such that Tr rho = N_e, where rho = 2 sum_{a < n} chi_a chi_a^T over
//     the n lowest states of H~ = [[F, W], [W^T, diag(e_aux + zeta)]] and n
//     minimises |2 sum_{a<n} |chi_a|^2 - N_e| (Aufbau);
//     F' = h + J[rho] - K[rho]/2 (density-fitted J and K);
//     DIIS(12) over the F' with error vectors rho_k - rho_{k-1}, until the
//     density changes by less than fock_tol;
//   QP energies of H~(F, zeta); F back to the reference basis.
// The outer loop stops when the Fock matrix it returns (reference basis)
// differs from the one it started from by less than tol in every element (the
// first iteration against F0): a fixed point of the rebuild.  The QP change
// between iterations is reported, not tested: orbitals embedded in satellite
// bands change their assignment at the 1e-6 Ha level near the fixed point.
// The core Hamiltonian h = diag(eps) - (J[rho0] - K[rho0]/2), rho0 =
// 2 diag(1_occ), makes F[rho0] = diag(eps) for the reference.
//
// Eigensolves: rocSOLVER dsyevd.  Products: rocBLAS (row-major wrappers).
// The small host-side work (Aufbau counts, the zeta root search, the DIIS
// extrapolation over at most 12 nmo^2 vectors) runs on the CPU between
// device calls; every O(nmo^3) or larger step runs on the device.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gwm {

namespace {

unsigned nbk(long n) { return (unsigned)((n + 255) / 256); }

gw_status blas_st(Handle* h, rocblas_status st, const char* what) {
    if (st != rocblas_status_success)
        return set_err(h, GW_ELIB, std::string(what) + ": " + rocblas_status_to_string(st));
    return GW_OK;
}

__global__ void set_diag_kernel(int M, const double* __restrict__ d, double s, int nlead, double* __restrict__ X) {
    // X = diag(d) (d non-null) or diag(s * 1_{p < nlead})
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)M * M) return;
    int r = (int)(i / M), c = (int)(i % M);
    double v = 0.0;
    if (r == c) v = d ? d[r] : (r < nlead ? s : 0.0);
    X[i] = v;
}

// out = a + ca * b + cb * c
__global__ void comb3_kernel(long n, const double* __restrict__ a, double ca, const double* __restrict__ b,
                             double cb, const double* __restrict__ c, double* __restrict__ out) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + ca * b[i] + cb * c[i];
}

// wt[a] = sum_{p < M} H[a][p]^2 (physical weight of eigenvector a; one wave per row)
__global__ void phys_weight_kernel(int dim, int M, const double* __restrict__ H, double* __restrict__ wt) {
    long a = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (a >= dim) return;
    const double* row = H + a * dim;
    double s = 0.0;
    for (int p = lane; p < M; p += 64) s += row[p] * row[p];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) wt[a] = s;
}

// J = sum_P L_P tr(L_P rho),  K = sum_P L_P rho L_P  for L [A][M][M] (each L_P symmetric).
// B[P][i][p] = G[P][p][i] for blocks of M x n (one z-slice per P), 32 x 32
// tiles through LDS so that both the reads and the writes are coalesced.
__global__ __launch_bounds__(256) void blk_transpose_kernel(int M, int n, const double* __restrict__ G,
                                                            double* __restrict__ B) {
    __shared__ double t[32][33];
    const long off = (long)blockIdx.z * M * n;
    const int i0 = blockIdx.x * 32, p0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int p = p0 + r, i = i0 + tx;
        t[r][tx] = (p < M && i < n) ? G[off + (long)p * n + i] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, p = p0 + tx;
        if (i < n && p < M) B[off + (long)i * M + p] = t[tx][r];
    }
}

// K = alpha sum_s part[s] (fixed order over the S split-k partial products)
__global__ void sum_parts_kernel(long n, int S, double alpha, const double* __restrict__ part,
                                 double* __restrict__ K) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int s = 0; s < S; ++s) acc += part[(long)s * n + i];
    K[i] = alpha * acc;
}

// Number of groups of P for a split-k exchange product: the largest divisor
// of A up to 16 (1 if there is none).
int split_groups(int A) {
    for (int c = std::min(16, A); c >= 2; --c)
        if (A % c == 0) return c;
    return 1;
}

}  // namespace

// Row-major batched C_b = op(A_b) op(B_b) (strides in elements, 0 = shared operand).
gw_status gemm_rm_batched(Handle* h, bool ta, bool tb, int m, int n, int k, const double* A, int lda, long sA,
                          const double* B, int ldb, long sB, double* C, int ldc, long sC, int batch) {
    const double one = 1.0, zero = 0.0;
    rocblas_operation oa = ta ? rocblas_operation_transpose : rocblas_operation_none;
    rocblas_operation ob = tb ? rocblas_operation_transpose : rocblas_operation_none;
    return blas_st(h,
                   rocblas_dgemm_strided_batched(h->blas, ob, oa, n, m, k, &one, B, ldb, sB, A, lda, sA, &zero, C,
                                                 ldc, sC, batch),
                   "rocblas_dgemm_strided_batched");
}

gw_status fock_jk(Handle* h, int A, int M, const double* L, const double* rho, double* J, double* K, double* T,
             double* v) {
    const long M2 = (long)M * M;
    const double one = 1.0, zero = 0.0;
    // row-major L as [A][M2] is column-major [M2][A]
    GW_TRY(blas_st(h, rocblas_dgemv(h->blas, rocblas_operation_transpose, (int)M2, A, &one, L, (int)M2, rho, 1, &zero,
                                    v, 1),
                   "rocblas_dgemv"));
    GW_TRY(blas_st(h, rocblas_dgemv(h->blas, rocblas_operation_none, (int)M2, A, &one, L, (int)M2, v, 1, &zero, J, 1),
                   "rocblas_dgemv"));
    // T_P = rho L_P, then K = sum_{(P,r)} T[(P,r)][p] L[(P,r)][q]; that sum
    // runs over A M terms into only (M/128)(M/64) output tiles, so it is split
    // over groups of P into partial products added in a fixed order.
    GW_TRY(gemm_rm_batched(h, false, false, M, M, M, rho, M, 0, L, M, M2, T, M, M2, A));
    const int S = split_groups(A);
    double* part = S > 1 ? (double*)ws_get(h, WS_KPART, sizeof(double) * S * M2) : nullptr;
    if (!part) {
        // no room for the partial products: the unsplit product (same result)
        if (S > 1) h->last_error.clear();
        return gemm_rowmajor(h, true, false, M, M, A * M, 1.0, T, M, L, M, 0.0, K, M);
    }
    const int kc = (A / S) * M;
    GW_TRY(gemm_rm_batched(h, true, false, M, M, kc, T, M, (long)kc * M, L, M, (long)kc * M, part, M, M2, S));
    hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((M2 + 255) / 256)), dim3(256), 0, h->stream, M2, S, 1.0,
                       (const double*)part, K);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status fock_jk_occ(Handle* h, int A, int M, const double* L, const double* rho, const double* Co, int nocc,
                      double* J, double* K, double* B, size_t bcap, double* v) {
    const long M2 = (long)M * M;
    const double one = 1.0, zero = 0.0;
    GW_TRY(blas_st(h, rocblas_dgemv(h->blas, rocblas_operation_transpose, (int)M2, A, &one, L, (int)M2, rho, 1, &zero,
                                    v, 1),
                   "rocblas_dgemv"));
    GW_TRY(blas_st(h, rocblas_dgemv(h->blas, rocblas_operation_none, (int)M2, A, &one, L, (int)M2, v, 1, &zero, J, 1),
                   "rocblas_dgemv"));
    // B_P = Co L_P (nocc x M), then K = 2 sum_{(P,i)} B[(P,i)][p] B[(P,i)][q].
    // L_P is symmetric, so B_P^T = L_P Co^T: all P at once as one tall GEMM
    // G = [L_0; L_1; ...] Co^T ((A M) x nocc), then a per-P transpose; the
    // batched form is the fallback when B cannot hold both copies.
    const long bsz = (long)A * M * nocc;
    if (2 * bsz <= (long)bcap && A <= 65535) {
        double* G = B + bsz;
        GW_TRY(gemm_rowmajor(h, false, true, A * M, nocc, M, 1.0, L, M, Co, M, 0.0, G, nocc));
        hipLaunchKernelGGL(blk_transpose_kernel, dim3((unsigned)((nocc + 31) / 32), (unsigned)((M + 31) / 32), (unsigned)A),
                           dim3(256), 0, h->stream, M, nocc, (const double*)G, B);
        GW_CHECK_LAUNCH(h);
        // K has only (M/128)(M/64) output tiles for a contraction over A nocc
        // rows: split that sum over S groups of P (S | A) into partial
        // products in the freed G region, then add them in a fixed order.
        const int S = split_groups(A);
        if (S > 1 && (long)S * M2 <= bsz) {
            const int kc = (A / S) * nocc;
            GW_TRY(gemm_rm_batched(h, true, false, M, M, kc, B, M, (long)kc * M, B, M, (long)kc * M, G, M, M2, S));
            hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((M2 + 255) / 256)), dim3(256), 0, h->stream, M2, S,
                               2.0, (const double*)G, K);
            GW_CHECK_LAUNCH(h);
            return GW_OK;
        }
    } else {
        GW_TRY(gemm_rm_batched(h, false, false, nocc, M, M, Co, M, 0, L, M, M2, B, M, (long)nocc * M, A));
    }
    return gemm_rowmajor(h, true, false, M, M, A * nocc, 2.0, B, M, B, M, 0.0, K, M);
}

gw_status zeta_trace(Handle* h, ZetaSearch& s, double z, double nelec, double* tr, int* nfill) {
    GW_TRY(upfold_eigh(h, s.M, s.np, s.F, s.pole_e, z, s.pole_v, s.ldv, s.H, s.w, s.work, s.info));
    ++s.eig_calls;
    const int dim = s.M + s.np;
    hipLaunchKernelGGL(phys_weight_kernel, dim3((unsigned)((dim + 3) / 4)), dim3(256), 0, h->stream, dim, s.M, s.H,
                       s.wt);
    GW_CHECK_LAUNCH(h);
    s.hw.resize(dim);
    GW_HIP(h, hipMemcpyAsync(s.hw.data(), s.wt, sizeof(double) * dim, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    double cum = 0.0, best = std::fabs(nelec);
    int nb = 0;
    for (int a = 0; a < dim; ++a) {
        cum += 2.0 * s.hw[a];
        if (std::fabs(cum - nelec) < best) {
            best = std::fabs(cum - nelec);
            nb = a + 1;
        }
    }
    double t = 0.0;
    for (int a = 0; a < nb; ++a) t += 2.0 * s.hw[a];
    *tr = t;
    *nfill = nb;
    return GW_OK;
}

gw_status zeta_solve(Handle* h, ZetaSearch& s, double nelec, double z0in, double zlo, double zhi, double ztol,
                     double* zeta, double* tr, int* nfill) {
    double lo, hi, flo, fhi;
    double half = 1e-3;
    const double z0 = std::min(std::max(z0in, zlo), zhi);
    for (;;) {
        lo = std::max(zlo, z0 - half);
        hi = std::min(zhi, z0 + half);
        GW_TRY(zeta_trace(h, s, lo, nelec, tr, nfill));
        flo = *tr - nelec;
        GW_TRY(zeta_trace(h, s, hi, nelec, tr, nfill));
        fhi = *tr - nelec;
        if (flo * fhi <= 0.0 || (lo == zlo && hi == zhi)) break;
        half *= 10.0;
    }
    double best = std::fabs(flo) < std::fabs(fhi) ? lo : hi;
    double fbest = std::fabs(flo) < std::fabs(fhi) ? flo : fhi;
    double last = hi;
    if (flo * fhi < 0.0) {
        int side = 0;
        double width = hi - lo;
        for (int it = 0; it < 100; ++it) {
            double z = (lo * fhi - hi * flo) / (fhi - flo);
            // bisect when false position leaves the bracket or the bracket stops halving
            if (!(z > lo && z < hi) || (it % 3 == 2 && hi - lo > 0.5 * width)) z = 0.5 * (lo + hi);
            if (it % 3 == 2) width = hi - lo;
            GW_TRY(zeta_trace(h, s, z, nelec, tr, nfill));
            last = z;
            const double f = *tr - nelec;
            if (std::fabs(f) < std::fabs(fbest)) {
                best = z;
                fbest = f;
            }
            if (std::fabs(f) < ztol || hi - lo < 1e-13) break;
            if ((f < 0) == (flo < 0)) {
                lo = z;
                flo = f;
                if (side == -1) fhi *= 0.5;
                side = -1;
            } else {
                hi = z;
                fhi = f;
                if (side == 1) flo *= 0.5;
                side = 1;
            }
        }
    }
    *zeta = best;
    if (last != best) GW_TRY(zeta_trace(h, s, best, nelec, tr, nfill));
    return GW_OK;
}

gw_status fsgw_run(Handle* h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                   const double* L, const double* F0, gw_precision prec, const gw_opts* opts,
                   const gw_fsgw_opts* fo, double* F, double* qp_e, double* qp_w, gw_fsgw_info* info) {
    const double tol = (fo && fo->tol > 0) ? fo->tol : 1e-6;
    const int max_outer = (fo && fo->max_outer > 0) ? fo->max_outer : 30;
    const int max_fock = (fo && fo->max_fock > 0) ? fo->max_fock : 50;
    const double fock_tol = (fo && fo->fock_tol > 0) ? fo->fock_tol : 1e-8;
    const int diis_space = (fo && fo->diis_space > 0) ? fo->diis_space : 12;
    const double zeta_tol = (fo && fo->zeta_tol > 0) ? fo->zeta_tol : 1e-13;
    double zlo = -1.0, zhi = 1.0;
    if (fo && fo->zeta_hi > fo->zeta_lo) {
        zlo = fo->zeta_lo;
        zhi = fo->zeta_hi;
    }
    const int M = nocc + nvir, A = naux, nt = nmom_max + 1;
    const long M2 = (long)M * M;
    const double nelec = 2.0 * nocc;
    const int cap = M * nt / 2;
    const long ldv = 2L * cap;
    const long dim_max = (long)M * (nmom_max + 2);

    // workspace (slots private to this loop)
    double* Lc = (double*)ws_get(h, WS_FS0, sizeof(double) * A * M2);        // rotated L
    double* T = (double*)ws_get(h, WS_FS1, sizeof(double) * A * M2);         // batched-product scratch
    double* sig = (double*)ws_get(h, WS_FS2, sizeof(double) * 2 * nt * M2);  // moments, both sectors
    double* pol = (double*)ws_get(h, WS_FS3, sizeof(double) * (2 * cap + (long)M * ldv));
    double* Hh = (double*)ws_get(h, WS_FS4, sizeof(double) * (dim_max * dim_max + 3 * dim_max));
    double* mat = (double*)ws_get(h, WS_FS5, sizeof(double) * (12 * M2 + 4 * M + A + 64));
    double* R = (double*)ws_get(h, WS_R, sizeof(double) * nt * (long)A * A);
    int* dinfo = (int*)ws_get(h, WS_FS6, sizeof(int) * 64);
    if (!Lc || !T || !sig || !pol || !Hh || !mat || !R || !dinfo) return GW_ENOMEM;
    double* so = sig;
    double* sv = sig + nt * M2;
    double* pole_e = pol;
    double* pole_v = pol + 2 * cap;
    double* Hw = Hh + dim_max * dim_max;  // eigenvalues
    double* Hwork = Hw + dim_max;
    double* Hwt = Hwork + dim_max;        // physical weights
    double* hcore = mat;                  // reference basis
    double* Fr = mat + M2;                // current F (reference basis)
    double* Ut = mat + 2 * M2;            // eigenvectors of Fr as rows
    double* hc = mat + 3 * M2;            // rotated core Hamiltonian
    double* Fc = mat + 4 * M2;            // Fock matrix in the rotated basis
    double* Fn = mat + 5 * M2;            // F[rho]
    double* rho = mat + 6 * M2;
    double* J = mat + 7 * M2;
    double* K = mat + 8 * M2;
    double* tmp = mat + 9 * M2;
    double* ecur = mat + 12 * M2;         // [M]
    double* wtmp = ecur + M;              // [M] eig work
    double* jv = wtmp + M;                // [A]

    // core Hamiltonian from the reference density
    hipLaunchKernelGGL(set_diag_kernel, dim3(nbk(M2)), dim3(256), 0, h->stream, M, (const double*)nullptr, 2.0, nocc,
                       rho);
    GW_CHECK_LAUNCH(h);
    GW_TRY(fock_jk(h, A, M, L, rho, J, K, T, jv));
    hipLaunchKernelGGL(set_diag_kernel, dim3(nbk(M2)), dim3(256), 0, h->stream, M, eps, 0.0, 0, tmp);
    GW_CHECK_LAUNCH(h);
    hipLaunchKernelGGL(comb3_kernel, dim3(nbk(M2)), dim3(256), 0, h->stream, M2, tmp, -1.0, J, 0.5, K, hcore);
    GW_CHECK_LAUNCH(h);
    if (F0) GW_TRY(copy_f64(h, Fr, F0, M2));
    else {
        hipLaunchKernelGGL(set_diag_kernel, dim3(nbk(M2)), dim3(256), 0, h->stream, M, eps, 0.0, 0, Fr);
        GW_CHECK_LAUNCH(h);
    }

    std::vector<double> hrho((size_t)M2), hrho_old((size_t)M2), hFn((size_t)M2), herr((size_t)M2),
        hqp(M), hqp_prev(M), hF((size_t)M2), hF_prev((size_t)M2);
    int outer = 0, fock_steps = 0;
    bool converged = false;
    double zeta = 0.0, last_dqp = -1.0, last_dF = -1.0;
    // the Fock matrix the first iteration starts from
    GW_HIP(h, hipMemcpyAsync(hF_prev.data(), Fr, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    int np = 0;

    ZetaSearch zs;
    zs.M = M;
    zs.F = Fc;
    zs.pole_e = pole_e;
    zs.pole_v = pole_v;
    zs.ldv = ldv;
    zs.H = Hh;
    zs.w = Hw;
    zs.work = Hwork;
    zs.wt = Hwt;
    zs.info = dinfo;

    for (outer = 0; outer < max_outer; ++outer) {
        // orbitals of the current F
        GW_TRY(copy_f64(h, Ut, Fr, M2));
        GW_TRY(eigh_rows(h, M, Ut, ecur, wtmp, dinfo));
        // L_P <- C^T L_P C with C = Ut^T;  h <- C^T h C
        GW_TRY(gemm_rm_batched(h, false, true, M, M, M, L, M, M2, Ut, M, 0, T, M, M2, A));
        GW_TRY(gemm_rm_batched(h, false, false, M, M, M, Ut, M, 0, T, M, M2, Lc, M, M2, A));
        GW_TRY(gemm_rowmajor(h, false, true, M, M, M, 1.0, hcore, M, Ut, M, 0.0, tmp, M));
        GW_TRY(gemm_rowmajor(h, false, false, M, M, M, 1.0, Ut, M, tmp, M, 0.0, hc, M));
        // self-energy moments and auxiliary poles in this basis
        if (screening == GW_TDA && prec == GW_MIXED) GW_TRY(tda_moments_mixed(h, nocc, nvir, A, nmom_max, ecur, Lc, R));
        else if (screening == GW_TDA) GW_TRY(tda_moments_f64(h, nocc, nvir, A, nmom_max, ecur, Lc, R, nullptr));
        else if (prec == GW_MIXED) GW_TRY(rpa_moments_mixed(h, nocc, nvir, A, nmom_max, ecur, Lc, opts, R));
        else GW_TRY(rpa_moments_f64(h, nocc, nvir, A, nmom_max, ecur, Lc, opts, R, nullptr));
        if (prec == GW_MIXED) GW_TRY(sigma_from_R_mixed(h, nocc, nvir, A, nmom_max, ecur, Lc, R, opts, so, sv));
        else GW_TRY(sigma_from_R_f64(h, nocc, nvir, A, nmom_max, ecur, Lc, R, opts, so, sv));
        int no = 0, nv = 0;
        GW_TRY(poles_lanczos(h, M, nmom_max, so, sv, opts, pole_e, pole_v, ldv, &no, &nv));
        np = no + nv;

        // Fock loop in the rotated basis
        hipLaunchKernelGGL(set_diag_kernel, dim3(nbk(M2)), dim3(256), 0, h->stream, M, ecur, 0.0, 0, Fc);
        GW_CHECK_LAUNCH(h);
        std::fill(hrho_old.begin(), hrho_old.end(), 0.0);
        for (int p = 0; p < nocc; ++p) hrho_old[(size_t)p * M + p] = 2.0;
        Diis diis{diis_space, (size_t)M2, {}, {}, {}};
        for (int step = 0; step < max_fock; ++step) {
            // zeta: root of Tr rho(zeta) - N_e, from the previous zeta
            double tr = 0.0;
            int nf = 0;
            zs.np = np;
            GW_TRY(zeta_solve(h, zs, nelec, zeta, zlo, zhi, zeta_tol, &zeta, &tr, &nf));
            // rho = 2 sum_{a < nf} chi_a chi_a^T (physical rows of the lowest nf eigenvectors)
            GW_TRY(gemm_rowmajor(h, true, false, M, M, nf, 2.0, Hh, M + np, Hh, M + np, 0.0, rho, M));
            GW_TRY(fock_jk(h, A, M, Lc, rho, J, K, T, jv));
            hipLaunchKernelGGL(comb3_kernel, dim3(nbk(M2)), dim3(256), 0, h->stream, M2, hc, 1.0, J, -0.5, K, Fn);
            GW_CHECK_LAUNCH(h);
            ++fock_steps;
            GW_HIP(h, hipMemcpyAsync(hrho.data(), rho, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
            GW_HIP(h, hipMemcpyAsync(hFn.data(), Fn, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
            GW_HIP(h, hipStreamSynchronize(h->stream));
            double emax = 0.0;
            for (long i = 0; i < M2; ++i) {
                herr[i] = hrho[i] - hrho_old[i];
                emax = std::max(emax, std::fabs(herr[i]));
            }
            hrho_old.swap(hrho);
            if (emax < fock_tol) {
                GW_TRY(copy_f64(h, Fc, Fn, M2));
                break;
            }
            diis.push(hFn.data(), herr.data());
            const double* next = diis.extrapolate();
            GW_HIP(h, hipMemcpyAsync(Fc, next, sizeof(double) * M2, hipMemcpyHostToDevice, h->stream));
            GW_HIP(h, hipStreamSynchronize(h->stream));
        }
        // QP energies of this iteration, F back to the reference basis
        GW_TRY(upfold_eigh(h, M, np, Fc, pole_e, zeta, pole_v, ldv, Hh, Hw, Hwork, dinfo));
        ++zs.eig_calls;
        GW_TRY(qp_assign_dev(h, M, M + np, Hh, Hw, qp_e, qp_w));
        GW_TRY(gemm_rowmajor(h, false, false, M, M, M, 1.0, Fc, M, Ut, M, 0.0, tmp, M));
        GW_TRY(gemm_rowmajor(h, true, false, M, M, M, 1.0, Ut, M, tmp, M, 0.0, Fr, M));
        GW_HIP(h, hipMemcpyAsync(hqp.data(), qp_e, sizeof(double) * M, hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipMemcpyAsync(hF.data(), Fr, sizeof(double) * M2, hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        std::sort(hqp.begin(), hqp.end());
        if (outer > 0) {
            last_dqp = 0.0;
            for (int p = 0; p < M; ++p) last_dqp = std::max(last_dqp, std::fabs(hqp[p] - hqp_prev[p]));
        }
        hqp_prev.swap(hqp);
        last_dF = 0.0;
        for (long i = 0; i < M2; ++i) last_dF = std::max(last_dF, std::fabs(hF[i] - hF_prev[i]));
        hF_prev.swap(hF);
        if (last_dF < tol) {
            converged = true;
            ++outer;
            break;
        }
    }
    GW_TRY(copy_f64(h, F, Fr, M2));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    if (info) {
        info->iterations = outer;
        info->fock_steps = fock_steps;
        info->eig_calls = zs.eig_calls;
        info->converged = converged ? 1 : 0;
        info->zeta = zeta;
        info->last_dqp = last_dqp;
        info->last_dF = last_dF;
    }
    return converged ? GW_OK : set_err(h, GW_ENOCONV, "fsGW: outer loop reached max_outer without converging");
}

}  // namespace gwm
