// Natural auxiliary functions (Sec. 2.1, eq. NAF): M_PQ = sum_{vw} V_{P,vw}
// V_{Q,vw} over the particle-hole pairs (i, a) (or over all nmo^2 pairs),
// its eigenvectors with eigenvalue above eps_naf, and the projection of the
// interaction tensor onto them.  FP64 throughout (rocBLAS GEMMs, rocSOLVER
// eigensolve); this runs once per system, before the hot path.
#include "internal.h"

#include <vector>

namespace gwm {

namespace {

// V[P][i * nvir + a] = L[P][i][nocc + a]
__global__ void naf_gather_kernel(int naux, int nocc, int nvir, const double* __restrict__ L, double* __restrict__ V) {
    const long ov = (long)nocc * nvir;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)naux * ov) return;
    const long P = i / ov, r = i % ov;
    const int o = (int)(r / nvir), a = (int)(r % nvir);
    const int nmo = nocc + nvir;
    V[i] = L[(P * nmo + o) * nmo + nocc + a];
}

}  // namespace

gw_status naf_run(Handle* h, int nocc, int nvir, int naux, const double* L, double eps_naf, int full_space,
                  double* L_naf, int* nnaf, double* eigenvalues) {
    const int nmo = nocc + nvir;
    const long M2 = (long)nmo * nmo;
    const long ov = (long)nocc * nvir;
    const long K = full_space ? M2 : ov;
    double* Mpq = (double*)ws_get(h, WS_FS0, sizeof(double) * ((long)naux * naux + 2L * naux));
    double* V = full_space ? nullptr : (double*)ws_get(h, WS_FS1, sizeof(double) * naux * ov);
    int* info = (int*)ws_get(h, WS_FS6, sizeof(int) * 64);
    if (!Mpq || (!full_space && !V) || !info) return GW_ENOMEM;
    double* w = Mpq + (long)naux * naux;
    double* work = w + naux;
    const double* X = L;
    if (!full_space) {
        const long n = (long)naux * ov;
        hipLaunchKernelGGL(naf_gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, naux, nocc,
                           nvir, L, V);
        GW_CHECK_LAUNCH(h);
        X = V;
    }
    // M = X X^T (naux x naux), then its eigenvectors as rows, eigenvalues ascending
    GW_TRY(gemm_rowmajor(h, false, true, naux, naux, (int)K, 1.0, X, (int)K, X, (int)K, 0.0, Mpq, naux));
    GW_TRY(eigh_rows(h, naux, Mpq, w, work, info));
    std::vector<double> hw(naux);
    GW_HIP(h, hipMemcpyAsync(hw.data(), w, sizeof(double) * naux, hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    int keep = 0;
    for (int k = 0; k < naux; ++k) keep += hw[k] > eps_naf;
    *nnaf = keep;
    if (eigenvalues) GW_TRY(copy_f64(h, eigenvalues, w, naux));
    if (keep == 0) return set_err(h, GW_ENUMERIC, "NAF: no eigenvalue of M above eps_naf");
    // kept vectors: the last `keep` rows (ascending eigenvalues), L_naf = U_kept L
    GW_TRY(gemm_rowmajor(h, false, false, keep, (int)M2, naux, 1.0, Mpq + (long)(naux - keep) * naux, naux, L,
                         (int)M2, 0.0, L_naf, (int)M2));
    return GW_OK;
}

}  // namespace gwm
