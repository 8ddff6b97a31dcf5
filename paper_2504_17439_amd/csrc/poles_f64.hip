// Auxiliary poles from self-energy moments and the upfolded Hamiltonian
// (eq. effH and its block-Lanczos construction; eqs. ret_GF and
// quasiparticle_energy_update), FP64 on the device.
//
// Per sector, with moments T[0..N] (N = 2m+1), first mapped to the moments of
// e' = (e - c)/s (c = tr T1 / tr T0, s = weighted spread) so powers stay O(1):
//   B0 = T[0]^{1/2} (pseudo-inverse B0^+ drops eigenvalues below pinv_tol*max),
//   S[n] = B0^+ T[n] B0^+,  the block Hankel matrices H0 = [S[k+l]], H1 = [S[k+l+1]].
//   Lanczos block j is kept as coefficients C_j = [C_j0 .. C_j,j-1] on Q1 e^k:
//     A_j  = C_j H1 C_j^T
//     Rhat = shift(C_j) - A_j C_j - B_{j-1} C_{j-1}
//     B_j^2 = Rhat H0 Rhat^T,  B_j = (B_j^2)^{1/2},  C_{j+1} = B_j^+ Rhat
//   B_j^2 is known only to noise_j = kappa eps (sum_k |Rhat_k|_F)^2 max_{n<=2j} |S[n]|_F
//   (cancellation once the coefficients grow): eigenvalues below
//   max(pinv_tol |S[2]|_F, noise_j) are deflated, below -max(neg_tol |S[2]|_F, 10 noise_j)
//   the input is rejected as not a moment sequence.
//   The block tridiagonal H_s (diagonal A_1..A_{m+1}, off-diagonal B_1..B_m)
//   is diagonalised, H_s = U diag(e') U^T, e = c + s e', and the poles couple
//   as v = B0 U[first block].
// Dense products: rocBLAS dgemm; eigensolves: rocSOLVER dsyevd (both column-
// major; row-major data is passed as its transpose where that matters).
#include "internal.h"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

namespace gwm {

namespace {

gw_status blas_ok(Handle* h, rocblas_status st, const char* what) {
    if (st != rocblas_status_success)
        return set_err(h, GW_ELIB, std::string(what) + ": " + rocblas_status_to_string(st));
    return GW_OK;
}

// Row-major C[m x n] = alpha op(A) op(B) + beta C.
gw_status gemm_rm(Handle* h, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
                  const double* B, int ldb, double beta, double* C, int ldc) {
    if (m == 0 || n == 0) return GW_OK;
    rocblas_operation oa = ta ? rocblas_operation_transpose : rocblas_operation_none;
    rocblas_operation ob = tb ? rocblas_operation_transpose : rocblas_operation_none;
    return blas_ok(h, rocblas_dgemm(h->blas, ob, oa, n, m, k, &alpha, B, ldb, A, lda, &beta, C, ldc),
                   "rocblas_dgemm");
}

__global__ void scale_rows_kernel(int n, int cols, const double* __restrict__ X, const double* __restrict__ s,
                                  double* __restrict__ Y) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n * cols) return;
    Y[i] = X[i] * s[i / cols];
}

// In place X <- (X + X^T)/2 (one thread per unordered pair).
__global__ void symmetrize_kernel(int n, double* X) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n * n) return;
    int r = (int)(i / n), c = (int)(i % n);
    if (r >= c) return;
    double a = 0.5 * (X[(long)r * n + c] + X[(long)c * n + r]);
    X[(long)r * n + c] = a;
    X[(long)c * n + r] = a;
}

// dst[(bi*M + i) * ld + bj*M + j] = src[i*M + j]
__global__ void put_block_kernel(int M, const double* __restrict__ src, double* __restrict__ dst, long ld, int bi,
                                 int bj) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)M * M) return;
    int r = (int)(i / M), c = (int)(i % M);
    dst[((long)bi * M + r) * ld + (long)bj * M + c] = src[i];
}

// Hankel: H[(k*M+i)][(l*M+j)] = S[k+l+off][i][j], k,l in [0, nb)
__global__ void hankel_kernel(int M, int nb, int off, const double* __restrict__ S, double* __restrict__ H) {
    long dim = (long)nb * M;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dim * dim) return;
    long r = i / dim, c = i % dim;
    int k = (int)(r / M), l = (int)(c / M);
    int ii = (int)(r % M), jj = (int)(c % M);
    H[i] = S[((long)(k + l + off) * M + ii) * M + jj];
}

// column sums of squares: wt[c] = sum_r X[r][c]^2
__global__ void colnorm2_kernel(int rows, int cols, const double* __restrict__ X, double* __restrict__ wt) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) {
        double x = X[(long)r * cols + c];
        s += x * x;
    }
    wt[c] = s;
}

// pack kept poles: e_out[col0+t] = e[idx[t]], v_out[p][col0+t] = v[p][idx[t]]
__global__ void pack_poles_kernel(int M, int nd, int nk, const int* __restrict__ idx, const double* __restrict__ e,
                                  const double* __restrict__ v, double* __restrict__ e_out,
                                  double* __restrict__ v_out, long ldv, int col0) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)(M + 1) * nk) return;
    int t = (int)(i % nk);
    int p = (int)(i / nk);
    int s = idx[t];
    if (p == M) e_out[col0 + t] = e[s];
    else v_out[(long)p * ldv + col0 + t] = v[(long)p * nd + s];
}

// H~ = [[fock, W], [W^T, diag(e + zeta)]], W = v[:, :np] (row stride ldv)
__global__ void upfold_kernel(int M, int np, const double* __restrict__ fock, const double* __restrict__ e,
                              double zeta, const double* __restrict__ v, long ldv, double* __restrict__ H) {
    long dim = M + np;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dim * dim) return;
    long r = i / dim, c = i % dim;
    double x = 0.0;
    if (r < M && c < M) x = fock[r * M + c];
    else if (r < M) x = v[r * ldv + (c - M)];
    else if (c < M) x = v[c * ldv + (r - M)];
    else if (r == c) x = e[r - M] + zeta;
    H[i] = x;
}

// chi[p][a] = Ut[a][p] for p < M (physical rows of the eigenvectors)
__global__ void chi_kernel(int M, int dim, long ldchi, const double* __restrict__ Ut, double* __restrict__ chi) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)M * dim) return;
    int p = (int)(i / dim), a = (int)(i % dim);
    chi[(long)p * ldchi + a] = Ut[(long)a * dim + p];
}

// QP assignment: alpha_p = argmax_a Ut[a][p]^2 (lowest a on ties).
__global__ void qp_kernel(int M, int dim, const double* __restrict__ Ut, const double* __restrict__ E,
                          double* __restrict__ qe, double* __restrict__ qw) {
    int p = blockIdx.x;
    __shared__ double bw[256];
    __shared__ int ba[256];
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int a = threadIdx.x; a < dim; a += blockDim.x) {
        double x = Ut[(long)a * dim + p];
        double w = x * x;
        if (w > best) { best = w; bi = a; }
    }
    bw[threadIdx.x] = best;
    ba[threadIdx.x] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            double w2 = bw[threadIdx.x + s];
            int a2 = ba[threadIdx.x + s];
            if (w2 > bw[threadIdx.x] || (w2 == bw[threadIdx.x] && a2 < ba[threadIdx.x])) {
                bw[threadIdx.x] = w2;
                ba[threadIdx.x] = a2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        qe[p] = E[ba[0]];
        qw[p] = bw[0];
    }
}

// Ts[n][e] = sum_k coef[n][k] T[k][e]   (binomial shift / scale of moments)
__global__ void shift_moments_kernel(int nt, long m2, const double* __restrict__ coef, const double* __restrict__ T,
                                     double* __restrict__ Ts) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m2) return;
    double t[16];
    for (int k = 0; k < nt; ++k) t[k] = T[(long)k * m2 + i];
    for (int n = 0; n < nt; ++n) {
        double acc = 0.0;
        for (int k = 0; k <= n; ++k) acc += coef[n * 16 + k] * t[k];
        Ts[(long)n * m2 + i] = acc;
    }
}

// out[k*rows + p] = sum_{c < w} X[p*ld + k*w + c]^2   (row sums of squares per column block)
__global__ void block_rowsq_kernel(int rows, int w, int nb, long ld, const double* __restrict__ X,
                                   double* __restrict__ out) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)rows * nb) return;
    int k = (int)(i / rows), p = (int)(i % rows);
    const double* x = X + (long)p * ld + (long)k * w;
    double s = 0.0;
    for (int c = 0; c < w; ++c) s += x[c] * x[c];
    out[i] = s;
}

__global__ void diag_kernel(int n, int nm, const double* __restrict__ T, double* __restrict__ d) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)nm * n) return;
    long b = i / n, p = i % n;
    d[i] = T[b * (long)n * n + p * n + p];
}

__global__ void affine_kernel(long n, double c, double s, double* __restrict__ e) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) e[i] = c + s * e[i];
}

unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

struct Eig {
    double* A;     // in: symmetric n x n; out: row i = eigenvector i
    double* w;     // eigenvalues ascending
    double* work;  // n
    int* info;
};

gw_status syevd(Handle* h, int n, Eig& e, bool vectors) {
    if (vectors) {
        void* ws = ws_get(h, WS_EIG, syev_tridiag_bytes(n));
        if (!ws) return GW_ENOMEM;
        return syev_tridiag(h, n, e.A, e.w, e.work, e.info, ws);
    }
    GW_TRY(blas_ok(h,
                   rocsolver_dsyevd(h->blas, vectors ? rocblas_evect_original : rocblas_evect_none,
                                    rocblas_fill_upper, n, e.A, n, e.w, e.work, e.info),
                   "rocsolver_dsyevd"));
    int info = 0;
    GW_HIP(h, hipMemcpyAsync(&info, e.info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    if (info != 0) return set_err(h, GW_ENUMERIC, "eigensolver did not converge");
    return GW_OK;
}

// X (M x M, PSD) -> symmetric sqrt and pseudo-inverse sqrt.  With rel, the
// cut and the negativity bound are tol * max|w| and neg * max|w|; otherwise
// they are the absolute values tol and neg.
gw_status sqrt_pinv(Handle* h, int M, const double* X, bool rel, double tol, double neg, double* Xs,
                    double* Xi, double* scratch /* 3 M^2 + 3M */, int* info) {
    double* A = scratch;
    double* Y = scratch + (long)M * M;
    double* w = scratch + 2L * M * M;
    double* work = w + M;
    double* sv = work + M;
    GW_TRY(copy_f64(h, A, X, (size_t)M * M));
    Eig e{A, w, work, info};
    GW_TRY(syevd(h, M, e, true));
    std::vector<double> hw(M);
    GW_HIP(h, hipMemcpyAsync(hw.data(), w, sizeof(double) * M, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    double wmax = 1e-300;
    for (double x : hw) wmax = std::max(wmax, std::fabs(x));
    const double cut = rel ? tol * wmax : tol;
    const double negb = rel ? neg * wmax : neg;
    if (hw[0] < -negb) return set_err(h, GW_ENUMERIC, "moment matrix is not positive semi-definite");
    std::vector<double> s1(M), s2(M);
    for (int i = 0; i < M; ++i) {
        bool keep = hw[i] > cut;
        s1[i] = keep ? std::sqrt(hw[i]) : 0.0;
        s2[i] = keep ? 1.0 / std::sqrt(hw[i]) : 0.0;
    }
    for (int pass = 0; pass < 2; ++pass) {
        double* out = pass == 0 ? Xs : Xi;
        if (!out) continue;
        GW_HIP(h, hipMemcpyAsync(sv, pass == 0 ? s1.data() : s2.data(), sizeof(double) * M, hipMemcpyHostToDevice,
                                 h->stream));
        hipLaunchKernelGGL(scale_rows_kernel, dim3(nblk((long)M * M)), dim3(256), 0, h->stream, M, M, A, sv, Y);
        GW_CHECK_LAUNCH(h);
        // out = Ut^T diag(s) Ut
        GW_TRY(gemm_rm(h, true, false, M, M, M, 1.0, A, M, Y, M, 0.0, out, M));
        // the host vectors must outlive the async copy
        GW_HIP(h, hipStreamSynchronize(h->stream));
    }
    return GW_OK;
}

gw_status symmetrize(Handle* h, int n, double* X) {
    hipLaunchKernelGGL(symmetrize_kernel, dim3(nblk((long)n * n)), dim3(256), 0, h->stream, n, X);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

// One sector: packs kept poles at columns [col0, col0 + npole) of e_out / v_out.
gw_status lanczos_sector(Handle* h, int M, int N, const double* T_in, double pinv_tol, double neg_tol, double kappa,
                         double* e_out, double* v_out, long ldv, int col0, int* npole) {
    const int m = (N - 1) / 2;
    const int nb = m + 1;
    const long M2 = (long)M * M;
    const long dimH = (long)nb * M;
    const int NT = N + 1;
    double* sc = (double*)ws_get(h, WS_LZ0, sizeof(double) * (3 * M2 + 4L * M + 16));
    double* S = (double*)ws_get(h, WS_LZ1, sizeof(double) * NT * M2);
    double* Hk = (double*)ws_get(h, WS_LZ2, sizeof(double) * 2 * dimH * dimH);
    double* Cb = (double*)ws_get(h, WS_LZ3, sizeof(double) * 4 * M * dimH);
    double* sm = (double*)ws_get(h, WS_LZ4, sizeof(double) * 8 * M2);
    double* Hs = (double*)ws_get(h, WS_LZ5, sizeof(double) * (dimH * dimH + 3 * dimH + (long)M * dimH + 16));
    int* info = (int*)ws_get(h, WS_RPA_INFO, sizeof(int) * 64);
    double* T = (double*)ws_get(h, WS_LZ7, sizeof(double) * (NT * M2 + 16L * 16 + (long)M * (NT + 2)));
    if (!sc || !S || !Hk || !Cb || !sm || !Hs || !info || !T) return GW_ENOMEM;
    double* dcoef = T + NT * M2;
    double* rowsq = dcoef + 16 * 16;
    // host helpers: Frobenius norms through row sums of squares
    auto frob_blocks = [&](const double* X, int rows, int w, int nb, long ld, std::vector<double>& out) -> gw_status {
        hipLaunchKernelGGL(block_rowsq_kernel, dim3(nblk((long)rows * nb)), dim3(256), 0, h->stream, rows, w, nb, ld, X,
                           rowsq);
        GW_CHECK_LAUNCH(h);
        std::vector<double> hv((size_t)rows * nb);
        GW_HIP(h, hipMemcpyAsync(hv.data(), rowsq, sizeof(double) * hv.size(), hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        out.assign(nb, 0.0);
        for (int k = 0; k < nb; ++k) {
            double acc = 0.0;
            for (int p = 0; p < rows; ++p) acc += hv[(size_t)k * rows + p];
            out[k] = std::sqrt(acc);
        }
        return GW_OK;
    };
    // shift / scale: c = tr T1 / tr T0, s = sqrt(tr T2 / tr T0 - c^2)
    double c = 0.0, sc_ = 1.0;
    {
        hipLaunchKernelGGL(diag_kernel, dim3(nblk((long)M * std::min(NT, 3))), dim3(256), 0, h->stream, M,
                           std::min(NT, 3), T_in, rowsq);
        GW_CHECK_LAUNCH(h);
        std::vector<double> hd((size_t)M * std::min(NT, 3));
        GW_HIP(h, hipMemcpyAsync(hd.data(), rowsq, sizeof(double) * hd.size(), hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        double tr[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < std::min(NT, 3); ++b)
            for (int p = 0; p < M; ++p) tr[b] += hd[(size_t)b * M + p];
        c = tr[1] / tr[0];
        double var = NT > 2 ? tr[2] / tr[0] - c * c : 0.0;
        sc_ = var > 0.0 ? std::sqrt(var) : std::max(std::fabs(c), 1.0);
        if (!std::isfinite(c) || !std::isfinite(sc_))
            return set_err(h, GW_ENUMERIC, "moments: trace of the zeroth moment is not positive");
        std::vector<double> coef(16 * 16, 0.0);
        for (int n = 0; n < NT; ++n) {
            double binom = 1.0;
            for (int k = 0; k <= n; ++k) {
                // C(n,k) (-c)^{n-k} / s^n
                coef[n * 16 + k] = binom * std::pow(-c, n - k) / std::pow(sc_, n);
                binom = binom * (n - k) / (k + 1);
            }
        }
        GW_HIP(h, hipMemcpyAsync(dcoef, coef.data(), sizeof(double) * 256, hipMemcpyHostToDevice, h->stream));
        hipLaunchKernelGGL(shift_moments_kernel, dim3(nblk(M2)), dim3(256), 0, h->stream, NT, M2, dcoef, T_in, T);
        GW_CHECK_LAUNCH(h);
        GW_HIP(h, hipStreamSynchronize(h->stream));
    }
    double* H0 = Hk;
    double* H1 = Hk + dimH * dimH;
    double* Cx[2] = {Cb, Cb + M * dimH};
    double* Rh = Cb + 2 * M * dimH;
    double* tmp = Cb + 3 * M * dimH;
    double* B0 = sm;
    double* B0i = sm + M2;
    double* Aj = sm + 2 * M2;
    double* Bj = sm + 3 * M2;
    double* Bji = sm + 4 * M2;
    double* Bprev = sm + 5 * M2;
    double* B2 = sm + 6 * M2;

    // B0 and its pseudo-inverse
    GW_TRY(sqrt_pinv(h, M, T, true, pinv_tol, neg_tol, B0, B0i, sc, info));
    // S[n] = B0^+ T[n] B0^+
    for (int n = 0; n < NT; ++n) {
        GW_TRY(gemm_rm(h, false, false, M, M, M, 1.0, T + n * M2, M, B0i, M, 0.0, B2, M));
        GW_TRY(gemm_rm(h, false, false, M, M, M, 1.0, B0i, M, B2, M, 0.0, S + n * M2, M));
        GW_TRY(symmetrize(h, M, S + n * M2));
    }
    // Frobenius norms of S[n]: the scale of the deflation thresholds
    std::vector<double> snorm(NT, 0.0);
    for (int n = 0; n < NT; ++n) {
        std::vector<double> one;
        GW_TRY(frob_blocks(S + n * M2, M, M, 1, M, one));
        snorm[n] = one[0];
    }
    const double ref = NT > 2 ? snorm[2] : snorm[0];
    const double eps_m = 2.220446049250313e-16;
    hipLaunchKernelGGL(hankel_kernel, dim3(nblk(dimH * dimH)), dim3(256), 0, h->stream, M, nb, 0, S, H0);
    GW_CHECK_LAUNCH(h);
    hipLaunchKernelGGL(hankel_kernel, dim3(nblk(dimH * dimH)), dim3(256), 0, h->stream, M, nb, 1, S, H1);
    GW_CHECK_LAUNCH(h);
    GW_TRY(fill_f64(h, Hs, (size_t)(dimH * dimH), 0.0));
    // C_1 = [I, 0, ...]
    GW_TRY(fill_f64(h, Cx[0], (size_t)(2 * M * dimH), 0.0));
    {
        std::vector<double> I((size_t)M2, 0.0);
        for (int i = 0; i < M; ++i) I[(size_t)i * M + i] = 1.0;
        GW_HIP(h, hipMemcpyAsync(sc, I.data(), sizeof(double) * M2, hipMemcpyHostToDevice, h->stream));
        hipLaunchKernelGGL(put_block_kernel, dim3(nblk(M2)), dim3(256), 0, h->stream, M, sc, Cx[0], dimH, 0, 0);
        GW_CHECK_LAUNCH(h);
        GW_HIP(h, hipStreamSynchronize(h->stream));
    }
    int cur = 0;
    for (int j = 1; j <= nb; ++j) {
        double* C = Cx[cur];
        double* Cp = Cx[cur ^ 1];
        const int K = j * M;
        // A_j = C_j H1 C_j^T
        GW_TRY(gemm_rm(h, false, false, M, K, K, 1.0, C, (int)dimH, H1, (int)dimH, 0.0, tmp, (int)dimH));
        GW_TRY(gemm_rm(h, false, true, M, M, K, 1.0, tmp, (int)dimH, C, (int)dimH, 0.0, Aj, M));
        GW_TRY(symmetrize(h, M, Aj));
        hipLaunchKernelGGL(put_block_kernel, dim3(nblk(M2)), dim3(256), 0, h->stream, M, Aj, Hs, dimH, j - 1, j - 1);
        GW_CHECK_LAUNCH(h);
        if (j == nb) break;
        // Rhat = shift(C_j) - A_j C_j - B_{j-1} C_{j-1}   (width (j+1) M)
        GW_TRY(fill_f64(h, Rh, (size_t)(M * dimH), 0.0));
        GW_HIP(h, hipMemcpy2DAsync(Rh + M, sizeof(double) * dimH, C, sizeof(double) * dimH, sizeof(double) * K, M,
                                   hipMemcpyDeviceToDevice, h->stream));
        GW_TRY(gemm_rm(h, false, false, M, K, M, -1.0, Aj, M, C, (int)dimH, 1.0, Rh, (int)dimH));
        if (j > 1)
            GW_TRY(gemm_rm(h, false, false, M, (j - 1) * M, M, -1.0, Bprev, M, Cp, (int)dimH, 1.0, Rh, (int)dimH));
        // B_j^2 = Rhat H0 Rhat^T
        const int K1 = (j + 1) * M;
        GW_TRY(gemm_rm(h, false, false, M, K1, K1, 1.0, Rh, (int)dimH, H0, (int)dimH, 0.0, tmp, (int)dimH));
        GW_TRY(gemm_rm(h, false, true, M, M, K1, 1.0, tmp, (int)dimH, Rh, (int)dimH, 0.0, B2, M));
        GW_TRY(symmetrize(h, M, B2));
        std::vector<double> rnorm;
        GW_TRY(frob_blocks(Rh, M, M, j + 1, dimH, rnorm));
        double rn = 0.0;
        for (double x : rnorm) rn += x;
        double smax = 0.0;
        for (int n = 0; n <= std::min(2 * j, NT - 1); ++n) smax = std::max(smax, snorm[n]);
        const double noise = kappa * eps_m * rn * rn * smax;
        GW_TRY(sqrt_pinv(h, M, B2, false, std::max(pinv_tol * ref, noise), std::max(neg_tol * ref, 10.0 * noise), Bj,
                         Bji, sc, info));
        hipLaunchKernelGGL(put_block_kernel, dim3(nblk(M2)), dim3(256), 0, h->stream, M, Bj, Hs, dimH, j - 1, j);
        GW_CHECK_LAUNCH(h);
        hipLaunchKernelGGL(put_block_kernel, dim3(nblk(M2)), dim3(256), 0, h->stream, M, Bj, Hs, dimH, j, j - 1);
        GW_CHECK_LAUNCH(h);
        // C_{j+1} = B_j^+ Rhat  (into the buffer of C_{j-1}, no longer needed)
        GW_TRY(fill_f64(h, Cp, (size_t)(M * dimH), 0.0));
        GW_TRY(gemm_rm(h, false, false, M, K1, M, 1.0, Bji, M, Rh, (int)dimH, 0.0, Cp, (int)dimH));
        GW_TRY(copy_f64(h, Bprev, Bj, (size_t)M2));
        cur ^= 1;
    }
    // eig(H_s); v = B0 U[first block] = B0 (Ut[:, :M])^T
    double* e = Hs + dimH * dimH;
    double* work = e + dimH;
    double* wt = work + dimH;
    double* vfull = wt + dimH;
    {
        Eig E{Hs, e, work, info};
        GW_TRY(syevd(h, (int)dimH, E, true));
    }
    {
        // e = c + s e'
        hipLaunchKernelGGL(affine_kernel, dim3(nblk(dimH)), dim3(256), 0, h->stream, dimH, c, sc_, e);
        GW_CHECK_LAUNCH(h);
    }
    GW_TRY(gemm_rm(h, false, true, M, (int)dimH, M, 1.0, B0, M, Hs, (int)dimH, 0.0, vfull, (int)dimH));
    hipLaunchKernelGGL(colnorm2_kernel, dim3(nblk(dimH)), dim3(256), 0, h->stream, M, (int)dimH, vfull, wt);
    GW_CHECK_LAUNCH(h);
    std::vector<double> hwt(dimH);
    GW_HIP(h, hipMemcpyAsync(hwt.data(), wt, sizeof(double) * dimH, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    double wmax = 1e-300;
    for (double x : hwt) wmax = std::max(wmax, x);
    std::vector<int> idx;
    for (long i = 0; i < dimH; ++i)
        if (hwt[i] > 1e-14 * wmax) idx.push_back((int)i);
    int nk = (int)idx.size();
    int* didx = (int*)ws_get(h, WS_MISC, sizeof(int) * (dimH + 16));
    if (!didx) return GW_ENOMEM;
    if (nk > 0) {
        GW_HIP(h, hipMemcpyAsync(didx, idx.data(), sizeof(int) * nk, hipMemcpyHostToDevice, h->stream));
        hipLaunchKernelGGL(pack_poles_kernel, dim3(nblk((long)(M + 1) * nk)), dim3(256), 0, h->stream, M,
                           (int)dimH, nk, didx, e, vfull, e_out, v_out, ldv, col0);
        GW_CHECK_LAUNCH(h);
        GW_HIP(h, hipStreamSynchronize(h->stream));
    }
    *npole = nk;
    return GW_OK;
}

Handle* aux_handle(Handle* h) {
    if (h->aux) return h->aux;
    Handle* a = new (std::nothrow) Handle();
    if (!a) {
        set_err(h, GW_ENOMEM, "companion handle: out of host memory");
        return nullptr;
    }
    a->device = h->device;
    a->cus = h->cus;
    a->ws.resize(WS_COUNT);
    if (hipStreamCreateWithFlags(&a->own_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete a;
        set_err(h, GW_EHIP, "companion handle: stream creation failed");
        return nullptr;
    }
    a->stream = a->own_stream;
    if (rocblas_create_handle(&a->blas) != rocblas_status_success) {
        (void)hipStreamDestroy(a->own_stream);
        delete a;
        set_err(h, GW_ELIB, "companion handle: rocblas_create_handle failed");
        return nullptr;
    }
    rocblas_set_stream(a->blas, a->stream);
    h->aux = a;
    return a;
}

// Both sectors' block Lanczos at once: the occupied one on the companion
// handle in a second host thread (its own stream, rocBLAS handle and
// workspaces), the virtual one on h; each is a long chain of small
// launch-latency-bound steps and host decisions, so the two overlap on the
// device.  The occupied poles land at columns [0, no) of pole_e / pole_v, the
// virtual ones are computed into a scratch and moved to [no, no + nv).  The
// companion stream starts after the work queued on h's stream and h's stream
// continues after it.
gw_status lanczos_two_sectors(Handle* h, int M, int N, const double* so, const double* sv, double pinv_tol,
                              double neg_tol, double kappa, double* pole_e, double* pole_v, long ldv, int* no,
                              int* nv) {
    Handle* a = aux_handle(h);
    if (!a) return GW_EHIP;
    const long cap = (long)M * (N + 1) / 2;
    double* tmp = (double*)ws_get(h, WS_POLE_TMP, sizeof(double) * (size_t)(cap + (long)M * cap));
    if (!tmp) return GW_ENOMEM;
    hipEvent_t fork = nullptr, join = nullptr;
    GW_HIP(h, hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(fork);
        return set_err(h, GW_EHIP, "lanczos: event creation failed");
    }
    struct Events {
        hipEvent_t a, b;
        ~Events() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{fork, join};
    GW_HIP(h, hipEventRecord(fork, h->stream));
    GW_HIP(h, hipStreamWaitEvent(a->stream, fork, 0));
    gw_status st_occ = GW_OK;
    int n_occ = 0, n_vir = 0;
    std::thread worker([&] {
        if (hipSetDevice(a->device) != hipSuccess) {
            (void)hipGetLastError();
            st_occ = set_err(a, GW_EHIP, "lanczos: hipSetDevice failed in the worker thread");
            return;
        }
        st_occ = lanczos_sector(a, M, N, so, pinv_tol, neg_tol, kappa, pole_e, pole_v, ldv, 0, &n_occ);
    });
    const gw_status st_vir = lanczos_sector(h, M, N, sv, pinv_tol, neg_tol, kappa, tmp, tmp + cap, cap, 0, &n_vir);
    worker.join();
    // h's stream waits for the occupied sector whatever happened
    GW_HIP(h, hipEventRecord(join, a->stream));
    GW_HIP(h, hipStreamWaitEvent(h->stream, join, 0));
    if (st_occ != GW_OK) return set_err(h, st_occ, a->last_error);
    if (st_vir != GW_OK) return st_vir;
    if (n_vir > 0) {
        GW_HIP(h, hipMemcpyAsync(pole_e + n_occ, tmp, sizeof(double) * n_vir, hipMemcpyDeviceToDevice, h->stream));
        GW_HIP(h, hipMemcpy2DAsync(pole_v + n_occ, sizeof(double) * ldv, tmp + cap, sizeof(double) * cap,
                                   sizeof(double) * n_vir, M, hipMemcpyDeviceToDevice, h->stream));
    }
    *no = n_occ;
    *nv = n_vir;
    return GW_OK;
}

}  // namespace

void aux_destroy(Handle* h) {
    Handle* a = h->aux;
    if (!a) return;
    (void)hipStreamSynchronize(a->stream);
    for (auto& b : a->ws)
        if (b.ptr) (void)hipFree(b.ptr);
    if (a->blas) rocblas_destroy_handle(a->blas);
    if (a->own_stream) (void)hipStreamDestroy(a->own_stream);
    delete a;
    h->aux = nullptr;
}

gw_status poles_f64(Handle* h, int nmo, int nmom_max, const double* sigma_occ, const double* sigma_vir,
                    const double* fock, const gw_opts* opts, int* npole_occ, int* npole_vir, double* pole_e,
                    double* pole_v, double* E, double* chi, double* qp_e, double* qp_w) {
    const double pinv_tol = (opts && opts->pinv_tol > 0) ? opts->pinv_tol : 1e-12;
    const double neg_tol = (opts && opts->neg_tol > 0) ? opts->neg_tol : 1e-8;
    // deflation level: kappa * (relative accuracy of the input moments)
    const double kappa = (opts && opts->moment_eps > 0) ? opts->moment_eps / 2.220446049250313e-16 : 1.0;
    const int M = nmo;
    const int cap = nmo * (nmom_max + 1) / 2;
    const long ldv = 2L * cap;
    GW_TRY(blas_ok(h, rocblas_set_stream(h->blas, h->stream), "rocblas_set_stream"));
    int no = 0, nv = 0;
    GW_TRY(lanczos_two_sectors(h, M, nmom_max, sigma_occ, sigma_vir, pinv_tol, neg_tol, kappa, pole_e, pole_v, ldv,
                               &no, &nv));
    *npole_occ = no;
    *npole_vir = nv;
    const int np = no + nv;
    const long dim = (long)M + np;
    const long dim_max = (long)nmo * (nmom_max + 2);
    double* H = (double*)ws_get(h, WS_LZ6, sizeof(double) * (dim * dim + 2 * dim + 16));
    int* info = (int*)ws_get(h, WS_RPA_INFO, sizeof(int) * 64);
    if (!H || !info) return GW_ENOMEM;
    hipLaunchKernelGGL(upfold_kernel, dim3(nblk(dim * dim)), dim3(256), 0, h->stream, M, np, fock, pole_e, 0.0,
                       pole_v, ldv, H);
    GW_CHECK_LAUNCH(h);
    double* w = H + dim * dim;
    {
        Eig e{H, w, w + dim, info};
        GW_TRY(syevd(h, (int)dim, e, true));
    }
    GW_TRY(copy_f64(h, E, w, (size_t)dim));
    if (chi) {
        hipLaunchKernelGGL(chi_kernel, dim3(nblk((long)M * dim)), dim3(256), 0, h->stream, M, (int)dim, dim_max, H,
                           chi);
        GW_CHECK_LAUNCH(h);
    }
    hipLaunchKernelGGL(qp_kernel, dim3(M), dim3(256), 0, h->stream, M, (int)dim, H, w, qp_e, qp_w);
    GW_CHECK_LAUNCH(h);
    GW_HIP(h, hipStreamSynchronize(h->stream));
    return GW_OK;
}

// ---------------------------------------------------------------------------
// Helpers shared with the self-consistent loop
// ---------------------------------------------------------------------------

gw_status gemm_rowmajor(Handle* h, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
                        const double* B, int ldb, double beta, double* C, int ldc) {
    return gemm_rm(h, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

gw_status eigh_rows(Handle* h, int n, double* A, double* w, double* work, int* info) {
    Eig e{A, w, work, info};
    return syevd(h, n, e, true);
}

gw_status poles_lanczos(Handle* h, int nmo, int nmom_max, const double* sigma_occ, const double* sigma_vir,
                        const gw_opts* opts, double* pole_e, double* pole_v, long ldv, int* npole_occ,
                        int* npole_vir) {
    const double pinv_tol = (opts && opts->pinv_tol > 0) ? opts->pinv_tol : 1e-12;
    const double neg_tol = (opts && opts->neg_tol > 0) ? opts->neg_tol : 1e-8;
    const double kappa = (opts && opts->moment_eps > 0) ? opts->moment_eps / 2.220446049250313e-16 : 1.0;
    GW_TRY(blas_ok(h, rocblas_set_stream(h->blas, h->stream), "rocblas_set_stream"));
    int no = 0, nv = 0;
    GW_TRY(lanczos_two_sectors(h, nmo, nmom_max, sigma_occ, sigma_vir, pinv_tol, neg_tol, kappa, pole_e, pole_v,
                               ldv, &no, &nv));
    *npole_occ = no;
    *npole_vir = nv;
    return GW_OK;
}

gw_status upfold_eigh(Handle* h, int M, int np, const double* fock, const double* pole_e, double zeta,
                      const double* pole_v, long ldv, double* H, double* w, double* work, int* info) {
    const long dim = (long)M + np;
    hipLaunchKernelGGL(upfold_kernel, dim3(nblk(dim * dim)), dim3(256), 0, h->stream, M, np, fock, pole_e, zeta,
                       pole_v, ldv, H);
    GW_CHECK_LAUNCH(h);
    return eigh_rows(h, (int)dim, H, w, work, info);
}

gw_status qp_assign_dev(Handle* h, int M, int dim, const double* Ut, const double* E, double* qp_e, double* qp_w) {
    hipLaunchKernelGGL(qp_kernel, dim3(M), dim3(256), 0, h->stream, M, dim, Ut, E, qp_e, qp_w);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

}  // namespace gwm
