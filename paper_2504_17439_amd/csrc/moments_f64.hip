// Density-response moments, FP64 path (Sec. 2.3 TDA; RPA in rpa_f64.hip).
//
// TDA:  X_0 = V,  X_{n+1} = D o X_n + 2 (X_n V^T) V,  R_n = X_n V^T
// (all eta~^{(n)} requested), or the half-order form below (R only).
// R_n is symmetric (V A^n V^T with A symmetric), so only its upper 128x128
// tiles are computed, split over K = ov, and mirrored in the reduction.
#include "internal.h"

#include <algorithm>

namespace gwm {

namespace {

__global__ void gather_ov_kernel(int nocc, int nvir, int naux, const double* __restrict__ eps,
                                 const double* __restrict__ L, double* __restrict__ V,
                                 double* __restrict__ D) {
    const int nmo = nocc + nvir;
    const long ov = (long)nocc * nvir;
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long total = (long)naux * ov;
    if (idx >= total) return;
    long P = idx / ov;
    long ia = idx - P * ov;
    int i = (int)(ia / nvir), a = (int)(ia - (long)i * nvir);
    V[idx] = L[(P * nmo + i) * nmo + nocc + a];
    if (P == 0) D[ia] = eps[nocc + a] - eps[i];
}

__global__ void fill_kernel(double* p, size_t n, double v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

}  // namespace

gw_status fill_f64(Handle* h, double* p, size_t n, double v) {
    if (n == 0) return GW_OK;
    size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, h->stream, p, n, v);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status copy_f64(Handle* h, double* dst, const double* src, size_t n) {
    if (n == 0 || dst == src) return GW_OK;
    GW_HIP(h, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    return GW_OK;
}

gw_status gather_ov(Handle* h, int nocc, int nvir, int naux, const double* eps, const double* L,
                    double* V, double* D) {
    long total = (long)naux * nocc * nvir;
    hipLaunchKernelGGL(gather_ov_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, h->stream,
                       nocc, nvir, naux, eps, L, V, D);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

// R = X diag(s) V^T (symmetric when X = V or s = 1 with X V^T symmetric):
// upper tiles, split-K partials in `part`, mirrored reduction.  s is nullable.
static gw_status syrk_xvt(Handle* h, int naux, long ov, const double* X, const double* V, double* R,
                          const Scratch& part, const double* s = nullptr) {
    GemmF64 g;
    g.M = naux; g.N = naux; g.K = (int)ov;
    g.a_kc = true; g.A = X; g.lda = ov; g.ascale = s;
    g.b_kc = true; g.B = V; g.ldb = ov;
    g.sym_upper = true;
    g.epi = EPI_PARTIAL;
    g.tag = "recur_xvt";
    g.ldc = naux; g.c_ps = (long)naux * naux;
    plan_split(g, 2 * h->cus);
    limit_split(g, scratch_max(part));
    double* buf = scratch_get(h, part, (size_t)g.nsplit * g.c_ps);
    if (!buf) return set_err(h, GW_ENOMEM, "syrk_xvt: split-K scratch too small");
    g.C = buf;
    GW_TRY(gemm_f64(h, g));
    return reduce_splits(h, buf, g.nsplit, g.c_ps, 1, naux, naux, naux, true, 1.0, 0.0, R, 0, naux);
}

// Xn = cs o (alpha * R V + dg o X)   (row-wise: every column ia scaled)
static gw_status update_rv(Handle* h, int naux, long ov, const double* R, const double* V, double alpha,
                           const double* X, const double* dg, const double* cs, double* Xn) {
    GemmF64 g;
    g.M = naux; g.N = (int)ov; g.K = naux;
    g.a_kc = true; g.A = R; g.lda = naux;
    g.b_kc = false; g.B = V; g.b_klo = ov;
    g.epi = EPI_AXPBY;
    g.alpha = alpha; g.X = X; g.ldx = ov; g.dg = dg; g.cs = cs;
    g.C = Xn; g.ldc = ov;
    g.tag = "recur_rv";
    return gemm_f64(h, g);
}

// Half-order form of the TDA moments (used when the eta~ are not requested):
// with A = D + 2 V^T V symmetric and X_k = V A^k,
//   R_{2k}   = V A^{2k}   V^T = X_k X_k^T
//   R_{2k+1} = V A^{2k+1} V^T = X_k D X_k^T + 2 R_k R_k
// so only X_0 .. X_{N/2} are formed (22 instead of 34 naux^2 ov flop units at N = 11).
static gw_status tda_moments_half(Handle* h, int naux, long ov, int nmom_max, const double* V, const double* D,
                                  double* X, double* R, const Scratch& part) {
    const long asz = (long)naux * naux;
    const long xsz = (long)naux * ov;
    GW_TRY(copy_f64(h, X, V, xsz));
    const int K = nmom_max / 2;
    for (int k = 0; k <= K; ++k) {
        if (2 * k <= nmom_max) GW_TRY(syrk_xvt(h, naux, ov, X, X, R + 2 * k * asz, part));
        if (2 * k + 1 <= nmom_max) {
            double* Ro = R + (2 * k + 1) * asz;
            GW_TRY(syrk_xvt(h, naux, ov, X, X, Ro, part, D));
            // Ro += 2 R_k R_k   (R_k is complete: k <= 2k)
            GemmF64 g;
            g.M = naux; g.N = naux; g.K = naux;
            g.a_kc = true; g.A = R + k * asz; g.lda = naux;
            g.b_kc = false; g.B = R + k * asz; g.b_klo = naux;
            g.epi = EPI_AXPBY; g.alpha = 2.0; g.X = Ro; g.ldx = naux;
            g.C = Ro; g.ldc = naux;
            g.tag = "recur_rr";
            GW_TRY(gemm_f64(h, g));
        }
        if (k < K) GW_TRY(update_rv(h, naux, ov, R + k * asz, V, 2.0, X, D, nullptr, X));
    }
    return GW_OK;
}

gw_status tda_moments_half_f64(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                               const double* L, double* R, double* V, double* D, double* X, const Scratch& part) {
    const long ov = (long)nocc * nvir;
    GW_TRY(gather_ov(h, nocc, nvir, naux, eps, L, V, D));
    return tda_moments_half(h, naux, ov, nmom_max, V, D, X, R, part);
}

gw_status tda_moments_f64(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                          const double* L, double* R, double* eta) {
    const long ov = (long)nocc * nvir;
    const long xsz = (long)naux * ov;
    double* V = (double*)ws_get(h, WS_V, sizeof(double) * xsz);
    double* D = (double*)ws_get(h, WS_D, sizeof(double) * ov);
    if (!V || !D) return GW_ENOMEM;
    GW_TRY(gather_ov(h, nocc, nvir, naux, eps, L, V, D));
    if (!eta) {
        double* X = (double*)ws_get(h, WS_X0, sizeof(double) * xsz);
        if (!X) return GW_ENOMEM;
        return tda_moments_half(h, naux, ov, nmom_max, V, D, X, R, Scratch{WS_SPLIT});
    }
    double* xb[2] = {nullptr, nullptr};
    if (!eta) {
        xb[0] = (double*)ws_get(h, WS_X0, sizeof(double) * xsz);
        xb[1] = (double*)ws_get(h, WS_X1, sizeof(double) * xsz);
        if (!xb[0] || !xb[1]) return GW_ENOMEM;
    } else {
        GW_TRY(copy_f64(h, eta, V, xsz));
    }
    const double* Xc = eta ? eta : V;
    const long asz = (long)naux * naux;
    for (int n = 0; n <= nmom_max; ++n) {
        GW_TRY(syrk_xvt(h, naux, ov, Xc, V, R + n * asz, Scratch{WS_SPLIT}));
        if (n == nmom_max) break;
        double* Xn = eta ? eta + (n + 1) * xsz : xb[n & 1];
        GW_TRY(update_rv(h, naux, ov, R + n * asz, V, 2.0, Xc, D, nullptr, Xn));
        Xc = Xn;
    }
    return GW_OK;
}

}  // namespace gwm
