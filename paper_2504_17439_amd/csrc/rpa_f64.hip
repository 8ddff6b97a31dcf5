// RPA density-response moments, FP64 (Sec. 2.2).
//
// Zeroth moment:  eta~^{(0)} = G D^-1 (I - 4 V^T (I + 4 V D^-1 V^T)^-1 V D^-1)
//   G = G_main + G_offset
//   G_main   = (2/pi) int_0^inf z^2 Q(z) ((I + Q(z))^-1 - I) V F(z) dz,  Q = 4 V F D V^T, F = (D^2+z^2)^-1
//   G_offset = V D + 4 int_0^inf V D E(z) V^T V E(z) dz,                  E = exp(-z D)
// Quadrature: n-point Gauss-Legendre on (-1,1) mapped by z = s(1+x)/(1-x).
//
// All 2n aux-space matrices (Q_j and T_j = V D E_j V^T) come from ONE batched
// symmetric product; (I+Q_j)^-1 from one batched Cholesky; and the 2n
// contributions to G from ONE launch whose K index runs over (Q block, node),
// node innermost, with the per-node column factors F_j / E_j applied to the
// V fragments in registers (node_sum_f64).
// Recursion: eta~^{(1)} = V D, eta~^{(n)} = D o (4 R_{n-2} V + D o eta~^{(n-2)}).
#include "internal.h"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace gwm {

namespace {

// Gauss-Legendre rule on (-1, 1) by Newton iteration on P_n (three-term
// recurrence), mapped to (0, inf) with z = s (1+x)/(1-x).
void mapped_gauss_legendre(int n, double s, std::vector<double>& z, std::vector<double>& w) {
    z.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double x = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(x), p0 = P_{n-1}(x)
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double wx = 2.0 / ((1.0 - x * x) * dp * dp);
        z[i] = s * (1.0 + x) / (1.0 - x);
        w[i] = wx * 2.0 * s / ((1.0 - x) * (1.0 - x));
    }
}

// ascale[b][ia]: b < nq: 4 F_j D;  b >= nq: D E_j
// bscale[b][ia]: b < nq: F_j;      b >= nq: E_j
__global__ void rpa_scales_kernel(int nq, long ov, const double* __restrict__ D,
                                  const double* __restrict__ z, double* __restrict__ as,
                                  double* __restrict__ bs) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2L * nq * ov) return;
    int b = (int)(idx / ov);
    long ia = idx - (long)b * ov;
    double d = D[ia];
    if (b < nq) {
        double zj = z[b];
        double f = 1.0 / (d * d + zj * zj);
        as[idx] = 4.0 * f * d;
        bs[idx] = f;
    } else {
        double e = exp(-z[b - nq] * d);
        as[idx] = d * e;
        bs[idx] = e;
    }
}

// In place on QT [2nq][A][A]:  b < nq: c_b (I - (I+Q_b)^-1 - Q_b);  b >= nq: 4 w_j T_b.
// Minv holds (I+Q_b)^-1 in its row-major upper triangle (rocSOLVER potri, column-major lower).
__global__ void rpa_form_s_kernel(int nq, int naux, const double* __restrict__ coef,
                                  const double* __restrict__ Minv, double* __restrict__ QT) {
    long n2 = (long)naux * naux;
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2L * nq * n2) return;
    int b = (int)(idx / n2);
    long e = idx - (long)b * n2;
    int m = (int)(e / naux), n = (int)(e - (long)m * naux);
    double c = coef[b];
    if (b < nq) {
        const double* Mi = Minv + (long)b * n2;
        double mi = (m <= n) ? Mi[(long)m * naux + n] : Mi[(long)n * naux + m];
        QT[idx] = c * ((m == n ? 1.0 : 0.0) - mi - QT[idx]);
    } else {
        QT[idx] = c * QT[idx];
    }
}

__global__ void add_identity_kernel(int nb, int naux, double* __restrict__ M) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)nb * naux) return;
    long b = i / naux, d = i - b * naux;
    M[b * (long)naux * naux + d * naux + d] += 1.0;
}

__global__ void scale_cols_kernel(long rows, long cols, const double* __restrict__ X,
                                  const double* __restrict__ d, double* __restrict__ Y) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    Y[idx] = X[idx] * d[idx % cols];
}

__global__ void recip_kernel(long n, const double* __restrict__ d, double* __restrict__ r) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = 1.0 / d[i];
}

gw_status blas_status(Handle* h, rocblas_status st, const char* what) {
    if (st != rocblas_status_success)
        return set_err(h, GW_ELIB, std::string(what) + ": " + rocblas_status_to_string(st));
    return GW_OK;
}

// C = V diag(as_b) V^T for each batch b (symmetric), mirrored reduction into out.
gw_status batched_sym(Handle* h, int naux, long ov, int batch, const double* V, const double* as,
                      double alpha, double diag, double* out) {
    GemmF64 g;
    g.M = naux; g.N = naux; g.K = (int)ov; g.batch = batch;
    g.a_kc = true; g.A = V; g.lda = ov; g.ascale = as; g.ascale_bs = ov;
    g.b_kc = true; g.B = V; g.ldb = ov;
    g.sym_upper = true;
    g.epi = EPI_PARTIAL;
    g.tag = "rpa_quad";
    plan_split(g, 2 * h->cus);
    g.ldc = naux; g.c_ps = (long)naux * naux;
    double* part = (double*)ws_get(h, WS_SPLIT, sizeof(double) * (size_t)g.nsplit * batch * g.c_ps);
    if (!part) return GW_ENOMEM;
    g.C = part;
    GW_TRY(gemm_f64(h, g));
    return reduce_splits(h, part, g.nsplit, g.c_ps, batch, naux, naux, naux, true, alpha, diag, out,
                         (long)naux * naux, naux);
}

}  // namespace

static gw_status rpa_eta0_f64(Handle* h, int nocc, int nvir, int naux, const double* eps,
                              const double* V, const double* D, const gw_opts* opts, double* eta0,
                              bool digit_nodes) {
    const long ov = (long)nocc * nvir;
    const int nmo = nocc + nvir;
    const long n2 = (long)naux * naux;
    const int nq = (opts && opts->nquad > 0) ? opts->nquad : 48;
    // grid scale: median of D, from the energies on the host
    double s = (opts && opts->quad_scale > 0.0) ? opts->quad_scale : 0.0;
    if (s <= 0.0) {
        std::vector<double> e(nmo);
        GW_HIP(h, hipMemcpyAsync(e.data(), eps, sizeof(double) * nmo, hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        std::vector<double> d(ov);
        for (int i = 0; i < nocc; ++i)
            for (int a = 0; a < nvir; ++a) d[(long)i * nvir + a] = e[nocc + a] - e[i];
        // numpy's median: mean of the two middle values for even counts
        size_t mid = d.size() / 2;
        std::nth_element(d.begin(), d.begin() + mid, d.end());
        double hi = d[mid];
        if (d.size() % 2 == 0) {
            double lo = *std::max_element(d.begin(), d.begin() + mid);
            s = 0.5 * (lo + hi);
        } else {
            s = hi;
        }
    }
    std::vector<double> z, w;
    mapped_gauss_legendre(nq, s, z, w);
    std::vector<double> coef(2 * nq);
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < nq; ++j) {
        coef[j] = (2.0 / pi) * w[j] * z[j] * z[j];
        coef[nq + j] = 4.0 * w[j];
    }

    double* misc = (double*)ws_get(h, WS_MISC, sizeof(double) * (3 * nq + 8));
    double* tables = (double*)ws_get(h, WS_RPA_SCALE, sizeof(double) * 4 * nq * ov);
    double* QT = (double*)ws_get(h, WS_RPA_QT, sizeof(double) * 2 * nq * n2);
    double* Minv = (double*)ws_get(h, WS_RPA_S, sizeof(double) * nq * n2);
    int* info = (int*)ws_get(h, WS_RPA_INFO, sizeof(int) * (2 * nq + 8));
    double* G = (double*)ws_get(h, WS_RPA_G, sizeof(double) * naux * ov);
    if (!misc || !tables || !QT || !Minv || !info || !G) return GW_ENOMEM;
    double* dz = misc;
    double* dcoef = misc + nq;
    GW_HIP(h, hipMemcpyAsync(dz, z.data(), sizeof(double) * nq, hipMemcpyHostToDevice, h->stream));
    GW_HIP(h, hipMemcpyAsync(dcoef, coef.data(), sizeof(double) * 2 * nq, hipMemcpyHostToDevice, h->stream));
    double* as = tables;
    double* bs = tables + 2L * nq * ov;
    {
        long tot = 2L * nq * ov;
        hipLaunchKernelGGL(rpa_scales_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h->stream,
                           nq, ov, D, dz, as, bs);
        GW_CHECK_LAUNCH(h);
    }
    // Q_j (b < nq) and T_j (b >= nq) in one batched symmetric product
    if (digit_nodes) GW_TRY(node_products_mixed(h, naux, ov, 2 * nq, V, as, QT));
    else GW_TRY(batched_sym(h, naux, ov, 2 * nq, V, as, 1.0, 0.0, QT));
    // (I + Q_j)^-1 by batched Cholesky
    GW_TRY(copy_f64(h, Minv, QT, (size_t)nq * n2));
    {
        long tot = (long)nq * naux;
        hipLaunchKernelGGL(add_identity_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h->stream,
                           nq, naux, Minv);
        GW_CHECK_LAUNCH(h);
    }
    GW_TRY(blas_status(h, rocblas_set_stream(h->blas, h->stream), "rocblas_set_stream"));
    GW_TRY(blas_status(h, rocsolver_dpotrf_strided_batched(h->blas, rocblas_fill_lower, naux, Minv, naux, n2,
                                                           info, nq),
                       "rocsolver_dpotrf_strided_batched"));
    GW_TRY(blas_status(h, rocsolver_dpotri_strided_batched(h->blas, rocblas_fill_lower, naux, Minv, naux, n2,
                                                           info + nq, nq),
                       "rocsolver_dpotri_strided_batched"));
    {
        std::vector<int> hinfo(2 * nq);
        GW_HIP(h, hipMemcpyAsync(hinfo.data(), info, sizeof(int) * 2 * nq, hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        for (int j = 0; j < 2 * nq; ++j)
            if (hinfo[j] != 0) return set_err(h, GW_ENUMERIC, "RPA quadrature: I + Q(z) not positive definite");
    }
    {
        long tot = 2L * nq * n2;
        hipLaunchKernelGGL(rpa_form_s_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h->stream,
                           nq, naux, dcoef, Minv, QT);
        GW_CHECK_LAUNCH(h);
    }
    // G = V o D + sum_b S_b (V o g_b): one launch over all nodes, the node
    // index innermost in K so that each V slab is loaded once for all nodes
    if (digit_nodes) GW_TRY(node_sum_mixed(h, naux, ov, 2 * nq, QT, V, bs, D, G));
    else GW_TRY(node_sum_f64(h, naux, ov, 2 * nq, QT, V, bs, V, D, G, Scratch{WS_RPA_PART}));
    // Woodbury: Hm = (G o D^-1) V^T, Pm = I + 4 (V o D^-1) V^T, Y = Hm Pm^-1,
    // eta~0 = D^-1 o (G - 4 Y V)
    double* Dinv = as;  // the quadrature scale tables are no longer needed
    {
        hipLaunchKernelGGL(recip_kernel, dim3((unsigned)((ov + 255) / 256)), dim3(256), 0, h->stream, ov, D,
                           Dinv);
        GW_CHECK_LAUNCH(h);
    }
    double* Hm = Minv;          // [A][A]
    double* Pm = Minv + n2;     // [A][A] (nq >= 2 guaranteed by validation)
    {
        GemmF64 g;
        g.M = naux; g.N = naux; g.K = (int)ov;
        g.a_kc = true; g.A = G; g.lda = ov; g.ascale = Dinv;
        g.b_kc = true; g.B = V; g.ldb = ov;
        g.epi = EPI_PARTIAL;
        plan_split(g, 2 * h->cus);
        g.ldc = naux; g.c_ps = n2;
        double* part = (double*)ws_get(h, WS_SPLIT, sizeof(double) * (size_t)g.nsplit * n2);
        if (!part) return GW_ENOMEM;
        g.C = part;
        GW_TRY(gemm_f64(h, g));
        GW_TRY(reduce_splits(h, part, g.nsplit, n2, 1, naux, naux, naux, false, 1.0, 0.0, Hm, 0, naux));
    }
    GW_TRY(batched_sym(h, naux, ov, 1, V, Dinv, 4.0, 1.0, Pm));
    GW_TRY(blas_status(h, rocsolver_dpotrf(h->blas, rocblas_fill_lower, naux, Pm, naux, info),
                       "rocsolver_dpotrf"));
    // row-major Hm seen column-major is Hm^T: solving Pm Z = Hm^T gives Z^T = Hm Pm^-1 in place
    GW_TRY(blas_status(h, rocsolver_dpotrs(h->blas, rocblas_fill_lower, naux, naux, Pm, naux, Hm, naux),
                       "rocsolver_dpotrs"));
    {
        int hinfo = 0;
        GW_HIP(h, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        GW_HIP(h, hipStreamSynchronize(h->stream));
        if (hinfo != 0) return set_err(h, GW_ENUMERIC, "RPA: I + 4 V D^-1 V^T not positive definite");
    }
    {
        GemmF64 g;
        g.M = naux; g.N = (int)ov; g.K = naux;
        g.a_kc = true; g.A = Hm; g.lda = naux;
        g.b_kc = false; g.B = V; g.b_klo = ov;
        g.epi = EPI_AXPBY; g.alpha = -4.0; g.X = G; g.ldx = ov; g.dg = nullptr; g.cs = Dinv;
        g.C = eta0; g.ldc = ov;
        GW_TRY(gemm_f64(h, g));
    }
    return GW_OK;
}

gw_status rpa_eta0(Handle* h, int nocc, int nvir, int naux, const double* eps, const double* V, const double* D,
                   const gw_opts* opts, double* eta0, bool digit_nodes) {
    return rpa_eta0_f64(h, nocc, nvir, naux, eps, V, D, opts, eta0, digit_nodes);
}

gw_status rpa_moments_f64(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                          const double* L, const gw_opts* opts, double* R, double* eta) {
    const long ov = (long)nocc * nvir;
    const long xsz = (long)naux * ov;
    const long n2 = (long)naux * naux;
    double* V = (double*)ws_get(h, WS_V, sizeof(double) * xsz);
    double* D = (double*)ws_get(h, WS_D, sizeof(double) * ov);
    if (!V || !D) return GW_ENOMEM;
    GW_TRY(gather_ov(h, nocc, nvir, naux, eps, L, V, D));
    // even and odd chains, updated in place unless every eta~^{(n)} is requested
    double* chain[2];
    if (eta) {
        chain[0] = eta;
        chain[1] = eta + xsz;
    } else {
        chain[0] = (double*)ws_get(h, WS_X0, sizeof(double) * xsz);
        chain[1] = (double*)ws_get(h, WS_X1, sizeof(double) * xsz);
        if (!chain[0] || !chain[1]) return GW_ENOMEM;
    }
    GW_TRY(rpa_eta0_f64(h, nocc, nvir, naux, eps, V, D, opts, chain[0], false));
    hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)((xsz + 255) / 256)), dim3(256), 0, h->stream,
                       (long)naux, ov, V, D, chain[1]);
    GW_CHECK_LAUNCH(h);
    for (int n = 0; n <= nmom_max; ++n) {
        double* Xn;
        if (n >= 2) {
            const double* Xp = eta ? eta + (n - 2) * xsz : chain[n & 1];
            Xn = eta ? eta + n * xsz : chain[n & 1];
            GemmF64 g;
            g.M = naux; g.N = (int)ov; g.K = naux;
            g.a_kc = true; g.A = R + (n - 2) * n2; g.lda = naux;
            g.b_kc = false; g.B = V; g.b_klo = ov;
            g.epi = EPI_AXPBY; g.alpha = 4.0; g.X = Xp; g.ldx = ov; g.dg = D; g.cs = D;
            g.C = Xn; g.ldc = ov;
            g.tag = "recur_rv";
            GW_TRY(gemm_f64(h, g));
        } else {
            Xn = chain[n];
        }
        // R_n = eta~^{(n)} V^T (symmetric)
        GemmF64 g;
        g.M = naux; g.N = naux; g.K = (int)ov;
        g.a_kc = true; g.A = Xn; g.lda = ov;
        g.b_kc = true; g.B = V; g.ldb = ov;
        g.sym_upper = true;
        g.epi = EPI_PARTIAL;
        g.tag = "recur_xvt";
        plan_split(g, 2 * h->cus);
        g.ldc = naux; g.c_ps = n2;
        double* part = (double*)ws_get(h, WS_SPLIT, sizeof(double) * (size_t)g.nsplit * n2);
        if (!part) return GW_ENOMEM;
        g.C = part;
        GW_TRY(gemm_f64(h, g));
        GW_TRY(reduce_splits(h, part, g.nsplit, n2, 1, naux, naux, naux, true, 1.0, 0.0, R + n * n2, 0, naux));
    }
    return GW_OK;
}

}  // namespace gwm
