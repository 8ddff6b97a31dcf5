// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gwmom.h"

namespace gwm {

// ---------------------------------------------------------------------------
// Handle and workspace
// ---------------------------------------------------------------------------

// A grow-only device buffer owned by the handle.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct TimedLaunch {
    std::string family;
    hipEvent_t start = nullptr, stop = nullptr;
};

struct Handle {
    bool timing = false;
    std::vector<TimedLaunch> timed;
    int device = 0;
    int cus = 256;           // compute units of the device (split planning)
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    rocblas_handle blas = nullptr;
    std::string last_error;
    // named workspaces (see WS_* below)
    std::vector<DevBuf> ws;
    hipEvent_t ev = nullptr;
    // companion handle for work that runs beside this handle's own (its own
    // stream, rocBLAS handle and workspaces; the occupied-sector Lanczos),
    // created on first use and destroyed with this handle
    Handle* aux = nullptr;
};

enum WsSlot {
    WS_V = 0, WS_D, WS_X0, WS_X1, WS_X2, WS_X3, WS_R, WS_SPLIT, WS_Z, WS_SIGACC,
    WS_RPA_SCALE, WS_RPA_QT, WS_RPA_S, WS_RPA_G, WS_RPA_INFO, WS_MISC,
    WS_LZ0, WS_LZ1, WS_LZ2, WS_LZ3, WS_LZ4, WS_LZ5, WS_LZ6, WS_LZ7,
    WS_MIX0, WS_MIX1, WS_MIX2, WS_MIX3, WS_MIX4, WS_MIX5, WS_MIX6,
    WS_FS0, WS_FS1, WS_FS2, WS_FS3, WS_FS4, WS_FS5, WS_FS6, WS_FS7,
    WS_RC0, WS_RC1, WS_RC2, WS_RC3, WS_RC4, WS_RC5,
    WS_KPART, WS_RPA_PART, WS_POLE_TMP, WS_EIG, WS_RPA_VLT, WS_RPA_SD, WS_RPA_EX, WS_RPA_AD, WS_RPA_QP,
    WS_COUNT
};

// Returns nullptr on failure (and records the message).
void* ws_get(Handle* h, int slot, size_t bytes);
// Frees the companion handle of h (if any); gw_destroy calls it.
void aux_destroy(Handle* h);

// Symmetric eigensolver (own Householder tridiagonalisation, rocSOLVER
// dstedc + dormtr): A [n][n] symmetric (the lower triangle of the row-major
// view defines it) is overwritten with the eigenvectors (row i = eigenvector i of
// the row-major view), w receives the eigenvalues ascending; work holds n
// doubles, info one int, ws syev_tridiag_bytes(n) bytes.
size_t syev_tridiag_bytes(int n);
gw_status syev_tridiag(Handle* h, int n, double* A, double* w, double* work, int* info, void* ws);

// Device scratch of doubles: a handle workspace slot (grown on demand), or a
// fixed region supplied by the caller (slot < 0), which never grows.
struct Scratch {
    int slot = -1;
    double* ptr = nullptr;
    size_t cap = 0;  // doubles, fixed region only
};
// Pointer to at least n doubles, or nullptr (a fixed region that is too small,
// or a failed allocation; the message is recorded).
double* scratch_get(Handle* h, const Scratch& s, size_t n);
// Largest request scratch_get can serve (SIZE_MAX for a workspace slot).
size_t scratch_max(const Scratch& s);

// Error plumbing: every internal routine returns gw_status.
gw_status set_err(Handle* h, gw_status st, const std::string& msg);

#define GW_HIP(h, call)                                                         \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess)                                                   \
            return ::gwm::set_err((h), GW_EHIP,                                 \
                                  std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

#define GW_CHECK_LAUNCH(h) GW_HIP(h, hipGetLastError())

#define GW_TRY(expr)                     \
    do {                                 \
        gw_status s_ = (expr);           \
        if (s_ != GW_OK) return s_;      \
    } while (0)

// Brackets one launch with events when timing is enabled on the handle.
struct KTimer {
    Handle* h;
    int idx = -1;
    KTimer(Handle* hh, const char* family);
    void stop();
};

// ---------------------------------------------------------------------------
// FP64 MFMA GEMM (gemm_f64.hip)
// ---------------------------------------------------------------------------
//
// C(m, n) = sum_k A(m, k) B(k, n) over a batch, with optional split-K.
//
// Operand A:
//   a_kc = true :  A(m,k) = A[m*lda + k]                           (k contiguous)
//   a_kc = false:  A(m,k) = A[a_off + (k/a_kdiv)*a_khi + (k%a_kdiv)*a_klo + m]
//   ascale (a_kc only, nullable): A(m,k) *= ascale[batch*ascale_bs + k]
// Operand B:
//   b_kc = true :  B(k,n) = B[n*ldb + k]
//   b_kc = false:  B(k,n) = B[b_off + (k/b_kdiv)*b_khi + (k%b_kdiv)*b_klo + n]
// Batch b adds a_bs*b, b_bs*b, c_bs*b to the A, B, C base pointers.
// Split s of nsplit covers k in [s*kchunk, min(K, (s+1)*kchunk)).
// sym_upper: only 128x128 tiles with tile_row <= tile_col are computed (M == N).
// Epilogues:
//   EPI_PARTIAL: C[(b*nsplit + s)*c_ps + m*ldc + n]  = acc      (or += when accumulate)
//   EPI_AXPBY  : C[b*c_bs + m*ldc + n] = cs[n] * (alpha*acc + X[b*x_bs + m*ldx + n] * dg[n])
//                (cs, X, dg nullable: 1, 0, 1)
enum GemmEpi { EPI_PARTIAL = 0, EPI_AXPBY = 1 };

struct GemmF64 {
    int M = 0, N = 0, K = 0;
    int batch = 1;
    bool a_kc = true, b_kc = true;
    const double* A = nullptr; long lda = 0; long a_off = 0, a_kdiv = 1L << 62, a_khi = 0, a_klo = 0;
    const double* ascale = nullptr; long ascale_bs = 0;
    const double* B = nullptr; long ldb = 0; long b_off = 0, b_kdiv = 1L << 62, b_khi = 0, b_klo = 0;
    long a_bs = 0, b_bs = 0, c_bs = 0;
    int nsplit = 1; int kchunk = 0;
    bool sym_upper = false;
    int epi = EPI_PARTIAL;
    bool accumulate = false;
    double* C = nullptr; long ldc = 0; long c_ps = 0;
    double alpha = 1.0;
    const double* X = nullptr; long ldx = 0; long x_bs = 0;
    const double* dg = nullptr;
    const double* cs = nullptr;
    const char* tag = nullptr;  // timing family (nullable)
};

gw_status gemm_f64(Handle* h, const GemmF64& g);

// Choose nsplit / kchunk for a launch on `slots` concurrent work groups (two
// per CU): the split count minimising (rounds of work groups) x (K per work
// group), the smaller count on near ties (fewer partials to reduce).
void plan_split(GemmF64& g, int slots);
// The same choice for `items` independent work items of K each.
int best_splits(long items, int K, int slots, int max_ns);
// Lower nsplit (re-chunking K) so that the partials, nsplit * batch * c_ps
// doubles, fit in max_doubles; nsplit stays >= 1.
void limit_split(GemmF64& g, size_t max_doubles);

// Node sum of the RPA quadrature on the FP64 MFMA:
//   G[P][ia] = X0[P][ia] d0[ia] + sum_{b < nb} sum_Q S[b][P][Q] V[Q][ia] gtab[b][ia]
// S [nb][naux][naux], V and X0 [naux][ov], gtab [nb][ov], d0 [ov]; node groups
// accumulate into partials in `part` (up to 8 x naux x ov doubles), reduced
// in a fixed order.
gw_status node_sum_f64(Handle* h, int naux, long ov, int nb, const double* S, const double* V, const double* gtab,
                       const double* X0, const double* d0, double* G, const Scratch& part);

// out[b][m][n] = alpha * sum_s part[(b*nsplit+s)*ps + m*ld + n] (+ diag on m == n),
// read from the upper triangle (m <= n) when `mirror`, which makes out exactly symmetric.
gw_status reduce_splits(Handle* h, const double* part, int nsplit, long ps, int batch,
                        int M, int N, long ld, bool mirror, double alpha, double diag,
                        double* out, long out_bs, long ldo);

// ---------------------------------------------------------------------------
// Moment / sigma building blocks (moments.hip, sigma.hip)
// ---------------------------------------------------------------------------

// V[P][i*nvir+a] = L[P][i][nocc+a];  D[i*nvir+a] = eps[nocc+a] - eps[i].
gw_status gather_ov(Handle* h, int nocc, int nvir, int naux, const double* eps,
                    const double* L, double* V, double* D);

// Stage 1 of the self-energy contraction over every column j = x*nmo + q of L
// viewed as [naux][nmo*nmo]:  Zt[n][P][j] = sum_{t<=n} s_{n,t}(x) sum_Q R_t[P][Q] L[Q][j],
// s_{n,t}(x) = 2 C(n,t) sigma_x^t eps_x^{n-t}, sigma_x = -1 (x < nocc) or +1;
// each symmetric pair (x, q), x <= q, is formed once (Zt: nt naux nmo^2 doubles).
gw_status sigma_fold_f64(Handle* h, int nt, int naux, int nmo, int nocc, const double* eps,
                         const double* R, const double* L, double* Zt);

gw_status sigma_from_R_f64(Handle* h, int nocc, int nvir, int naux, int nmom_max,
                           const double* eps, const double* L, const double* R,
                           const gw_opts* opts, double* sigma_occ, double* sigma_vir);

gw_status sigma_from_R_mixed(Handle* h, int nocc, int nvir, int naux, int nmom_max,
                             const double* eps, const double* L, const double* R,
                             const gw_opts* opts, double* sigma_occ, double* sigma_vir);

gw_status tda_moments_f64(Handle* h, int nocc, int nvir, int naux, int nmom_max,
                          const double* eps, const double* L, double* R, double* eta);

// The half-order FP64 TDA moments on caller buffers: V [naux][ov], D [ov],
// X [naux][ov], split-K partials in `part` (at least naux^2 doubles).
gw_status tda_moments_half_f64(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                               const double* L, double* R, double* V, double* D, double* X, const Scratch& part);

// FP64 self-energy moments from R_t on caller buffers: the folded
// intermediate in `zt` ((nmom_max+1) naux nmo^2 doubles, refused with
// GW_ENOMEM above zcap_bytes) and the contraction's split partials in `acc`
// (at least 2 (nmom_max+1) nmo^2 doubles).
gw_status sigma_from_R_f64_bufs(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                                const double* L, const double* R, size_t zcap_bytes, const Scratch& zt,
                                const Scratch& acc, double* sigma_occ, double* sigma_vir);

// TDA moments R[nmom_max+1][naux][naux] with int8 digit products (mixed precision).
gw_status tda_moments_mixed(Handle* h, int nocc, int nvir, int naux, int nmom_max,
                            const double* eps, const double* L, double* R);

gw_status rpa_moments_f64(Handle* h, int nocc, int nvir, int naux, int nmom_max,
                          const double* eps, const double* L, const gw_opts* opts,
                          double* R, double* eta);

// eta~^{(0)} [naux][nocc*nvir] of RPA screening by the quadrature (Sec. 2.2),
// from the gathered V [naux][ov] and D [ov].  With digit_nodes the node
// products and the node sum run as int8 digit products
// (node_products_mixed, node_sum_mixed); everything else is FP64.
gw_status rpa_eta0(Handle* h, int nocc, int nvir, int naux, const double* eps, const double* V, const double* D,
                   const gw_opts* opts, double* eta0, bool digit_nodes = false);

// Q[b] = V diag(as[b]) V^T for b < nb (V [naux][ov], as [nb][ov], Q [nb][naux][naux],
// both triangles) as symmetric int8 digit products: V's row digits once,
// V o as[b] digitised per node, split-k partials reduced in a fixed order.
gw_status node_products_mixed(Handle* h, int naux, long ov, int nb, const double* V, const double* as,
                              double* Q);

// As node_sum_f64 with X0 = V, in int8 digit products: V digitised once
// (per-column scales), each S[b] by rows, one digit GEMM per node whose
// epilogue adds gtab[b] o (S[b] V) to G (the first node starts from V o d0).
gw_status node_sum_mixed(Handle* h, int naux, long ov, int nb, const double* S, const double* V,
                         const double* gtab, const double* d0, double* G);

// RPA density-response moments with the recursion as int8 digit products
// (eta~^{(0)} from the FP64 quadrature): R [nmom_max+1][naux][naux].
gw_status rpa_moments_mixed(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                            const double* L, const gw_opts* opts, double* R);

gw_status poles_f64(Handle* h, int nmo, int nmom_max, const double* sigma_occ,
                    const double* sigma_vir, const double* fock, const gw_opts* opts,
                    int* npole_occ, int* npole_vir, double* pole_e, double* pole_v,
                    double* E, double* chi, double* qp_e, double* qp_w);

// Row-major C[m x n] = alpha op(A) op(B) + beta C (rocBLAS).
gw_status gemm_rowmajor(Handle* h, bool ta, bool tb, int m, int n, int k, double alpha, const double* A, int lda,
                        const double* B, int ldb, double beta, double* C, int ldc);

// Symmetric eigensolve in place: A (n x n) -> rows are eigenvectors, w ascending
// (work: n doubles, info: device int).
gw_status eigh_rows(Handle* h, int n, double* A, double* w, double* work, int* info);

// Auxiliary poles of both sectors (block Lanczos), packed as in gw_poles.
gw_status poles_lanczos(Handle* h, int nmo, int nmom_max, const double* sigma_occ, const double* sigma_vir,
                        const gw_opts* opts, double* pole_e, double* pole_v, long ldv, int* npole_occ,
                        int* npole_vir);

// Eigensystem of H~ = [[fock, W], [W^T, diag(pole_e + zeta)]], W = pole_v[:, :np]:
// H (dim^2, dim = M + np) receives the eigenvectors as rows, w the eigenvalues.
gw_status upfold_eigh(Handle* h, int M, int np, const double* fock, const double* pole_e, double zeta,
                      const double* pole_v, long ldv, double* H, double* w, double* work, int* info);

// Row-major batched C_b = op(A_b) op(B_b) (strides in elements, 0 = shared operand).
gw_status gemm_rm_batched(Handle* h, bool ta, bool tb, int m, int n, int k, const double* A, int lda, long sA,
                          const double* B, int ldb, long sB, double* C, int ldc, long sC, int batch);

// Density-fitted Coulomb and exchange matrices of a density rho (M x M):
// J_pq = sum_P L[P][p][q] sum_rs L[P][r][s] rho_rs, K_pq = sum_P (L_P rho L_P)_pq.
// Scratch: T [A][M][M], v [A].
gw_status fock_jk(Handle* h, int A, int M, const double* L, const double* rho, double* J, double* K, double* T,
                  double* v);
// The same with rho = 2 Co^T Co given by its nocc occupied orbitals (rows of
// Co, length M): K = 2 sum_P (Co L_P)^T (Co L_P), a factor M / nocc fewer
// flops.  B: bcap doubles, at least nocc * M * A (twice that for the
// one-GEMM form).
gw_status fock_jk_occ(Handle* h, int A, int M, const double* L, const double* rho, const double* Co, int nocc,
                      double* J, double* K, double* B, size_t bcap, double* v);

// Pulay extrapolation over the last `space` pairs (x_i, e_i): sum_i c_i x_i with
// sum_i c_i = 1 minimising |sum_i c_i e_i|^2.  Host vectors of length n.
struct Diis {
    int space;
    size_t n;
    std::vector<std::vector<double>> xs, es;
    std::vector<double> out;

    void push(const double* x, const double* e) {
        xs.emplace_back(x, x + n);
        es.emplace_back(e, e + n);
        if ((int)xs.size() > space) {
            xs.erase(xs.begin());
            es.erase(es.begin());
        }
    }
    // Solve the bordered system by Gaussian elimination with partial pivoting;
    // a vanishing pivot falls back to the newest vector.
    const double* extrapolate() {
        const int m = (int)xs.size();
        const int d = m + 1;
        std::vector<double> B((size_t)d * d, 0.0), rhs(d, 0.0);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j <= i; ++j) {
                double s = 0.0;
                for (size_t t = 0; t < n; ++t) s += es[i][t] * es[j][t];
                B[(size_t)i * d + j] = B[(size_t)j * d + i] = s;
            }
        for (int i = 0; i < m; ++i) B[(size_t)m * d + i] = B[(size_t)i * d + m] = -1.0;
        rhs[m] = -1.0;
        out.assign(xs.back().begin(), xs.back().end());
        for (int c = 0; c < d; ++c) {
            int piv = c;
            for (int r = c + 1; r < d; ++r)
                if (std::fabs(B[(size_t)r * d + c]) > std::fabs(B[(size_t)piv * d + c])) piv = r;
            if (std::fabs(B[(size_t)piv * d + c]) < 1e-300) return out.data();
            if (piv != c) {
                for (int k = 0; k < d; ++k) std::swap(B[(size_t)c * d + k], B[(size_t)piv * d + k]);
                std::swap(rhs[c], rhs[piv]);
            }
            for (int r = c + 1; r < d; ++r) {
                double f = B[(size_t)r * d + c] / B[(size_t)c * d + c];
                if (f == 0.0) continue;
                for (int k = c; k < d; ++k) B[(size_t)r * d + k] -= f * B[(size_t)c * d + k];
                rhs[r] -= f * rhs[c];
            }
        }
        std::vector<double> coef(d);
        for (int r = d - 1; r >= 0; --r) {
            double s = rhs[r];
            for (int k = r + 1; k < d; ++k) s -= B[(size_t)r * d + k] * coef[k];
            coef[r] = s / B[(size_t)r * d + r];
        }
        std::fill(out.begin(), out.end(), 0.0);
        for (int i = 0; i < m; ++i)
            for (size_t t = 0; t < n; ++t) out[t] += coef[i] * xs[i][t];
        return out.data();
    }
};


// Electron-number search over the shift zeta of the auxiliary energies
// (eq. density, Sec. 3.5).  The system is H~(zeta) as in upfold_eigh; H, w,
// work, wt (each sized for dim = M + np) and info are device scratch, and
// after every evaluation H / w hold the eigensystem at the last zeta asked.
struct ZetaSearch {
    int M = 0, np = 0;
    const double* F = nullptr;
    const double* pole_e = nullptr;
    const double* pole_v = nullptr;
    long ldv = 0;
    double* H = nullptr;
    double* w = nullptr;
    double* work = nullptr;
    double* wt = nullptr;
    int* info = nullptr;
    int eig_calls = 0;
    std::vector<double> hw;
};

// Aufbau filling of H~(z): nfill minimises |2 sum_{a<n} |chi_a|^2 - nelec|
// (lowest n on ties), tr = 2 sum_{a<nfill} |chi_a|^2.
gw_status zeta_trace(Handle* h, ZetaSearch& s, double z, double nelec, double* tr, int* nfill);

// Root of Tr rho(zeta) - nelec: bracket +-1e-3 Ha around z0 (clamped to
// [zlo, zhi]), widened tenfold until the sign changes or the bracket is
// [zlo, zhi]; then Illinois false position with bisection safeguards, to
// ztol electrons or a 1e-13 Ha bracket.  Without a sign change, the end with
// the smaller residual.  On return s.H / s.w hold the eigensystem at *zeta.
gw_status zeta_solve(Handle* h, ZetaSearch& s, double nelec, double z0, double zlo, double zhi, double ztol,
                     double* zeta, double* tr, int* nfill);

// QP energies / weights from an H~ eigensystem (device outputs).
gw_status qp_assign_dev(Handle* h, int M, int dim, const double* Ut, const double* E, double* qp_e, double* qp_w);

gw_status naf_run(Handle* h, int nocc, int nvir, int naux, const double* L, double eps_naf, int full_space,
                  double* L_naf, int* nnaf, double* eigenvalues);

gw_status spectral_run(Handle* h, int nmo, int dim, int ld_chi, const double* E, const double* chi, int nomega,
                       const double* omega, double delta, double* A, double* A_orb);
gw_status aufbau_run(Handle* h, int nmo, int dim, int ld_chi, const double* E, const double* chi, double nelec,
                     double* rho, gw_aufbau_info* info);
gw_status zeta_shift_run(Handle* h, int nmo, int nmom_max, int npole_occ, int npole_vir, const double* fock,
                         const double* pole_e, const double* pole_v, double nelec, const gw_zeta_opts* zo, double* E,
                         double* chi, double* qp_e, double* qp_w, gw_zeta_info* info);

gw_status qsgw_run(Handle* h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                   const double* L, gw_precision prec, const gw_opts* opts, const gw_qsgw_opts* qo, double* qp_e,
                   double* C, double* F, gw_qsgw_info* info);

gw_status evgw_run(Handle* h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                   const double* L, gw_precision prec, const gw_opts* opts, const gw_evgw_opts* eo, double* qp_e,
                   double* qp_w, gw_evgw_info* info);

gw_status fsgw_run(Handle* h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                   const double* L, const double* F0, gw_precision prec, const gw_opts* opts,
                   const gw_fsgw_opts* fo, double* F, double* qp_e, double* qp_w, gw_fsgw_info* info);

// Allocation-free FP64 TDA self-energy moments on the library's static
// scratch (noalloc.hip); noalloc_resolve finds the scratch on the current device.
gw_status noalloc_resolve(int device, std::string* err);
gw_status sigma_moments_noalloc(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                                const double* L, double* sigma_occ, double* sigma_vir);

gw_status batch_create(Handle* h, int nsys, const gw_system* sys, gw_screening screening, int nmom_max,
                       gw_precision prec, const gw_opts* opts, const gw_batch_opts* bo, gw_batch* out);
gw_status batch_run(gw_batch b);
gw_status batch_info(gw_batch b, int* njobs, int* nwaves, int* graph, int* split_target, int* small_tile_nmo);
void batch_destroy(gw_batch b);

long mlp_param_count();
gw_status mlp_norm(Handle* h, int rows, const float* x, const float* t, float* norm);
gw_status mlp_target(Handle* h, int nmo, const double* F, const double* eps, float* t);
gw_status mlp_warm_start(Handle* h, int nocc, int nvir, int naux, const double* eps, const double* L,
                         const float* prm, const float* norm, double* F0);
gw_status mlp_features(Handle* h, int nocc, int nvir, int naux, const double* eps, const double* L, float* feat);
gw_status mlp_forward(Handle* h, int rows, const float* prm, const float* norm, const float* x, float* act, float* y);
gw_status mlp_backward(Handle* h, int rows, const float* prm, const float* norm, const float* x, const float* act,
                       const float* y, const float* t, float* grad, float* loss);
gw_status mlp_adam(Handle* h, int step, float lr, float b1, float b2, float eps, float* prm, const float* grad,
                   float* m, float* v);

// Elementwise helpers (moments.hip)
gw_status fill_f64(Handle* h, double* p, size_t n, double v);
gw_status copy_f64(Handle* h, double* dst, const double* src, size_t n);

}  // namespace gwm
