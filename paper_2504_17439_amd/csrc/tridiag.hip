// Symmetric eigensolver of the pole stage: the eigenpairs of the block
// tridiagonal Lanczos matrices (Sec. 2.3), of the Gram matrices of the
// Lanczos blocks (their square roots and pseudo-inverses) and of the upfolded
// Hamiltonian H~ (Sec. 2.4) all come from here.
//
// The input is defined by the lower triangle of its row-major view, and the
// reduction works on B = J A J (J the index reversal; reverse_kernel), i.e.
// from the far end of the orbital order.  B = Q T Q^T is reached by
// Householder reflectors, one column at a time, in the classical unblocked
// order (reflector k annihilates column k below the subdiagonal; the
// trailing matrix takes the symmetric rank-2 update A <- A - v w^T - w v^T
// with w = tau A v + alpha2 v, alpha2 = -tau^2 v^T A v / 2).  T's eigenpairs
// then come from rocSOLVER's divide and conquer (dstedc), B's eigenvectors
// from applying Q to T's, blocked in compact WY form (apply_q: two rocBLAS
// dgemm and one dtrsm per block of 64 reflectors), and A's from reversing
// their components.  The reflectors are kept in LAPACK's layout (lower
// triangle, column-major, v_k below the subdiagonal of column k with its
// leading 1 implicit, e_k on the subdiagonal).
//
// The reduction is bound by launches and memory, not by arithmetic: a
// library tridiagonalisation issues several kernels per column (norm,
// symmetric matrix-vector product, dot products, rank-2 update, ...).  Here
// column k takes two launches:
//   * trd_step: every work group owns one 64 x 64 tile of the trailing lower
//     triangle and applies the still-pending rank-2 update of reflector k-1
//     to it (written back), so the update of one step and the matrix-vector
//     product of the next share one pass over the matrix; column k after
//     that update is x, and the tile writes its share of y = A22 x (both
//     halves of the symmetric product) as a partial vector, and its shares of
//     x^T y and |x|^2 as partial scalars;
//   * trd_reduce: one work group per row block sums that block's partial
//     vectors into y (a fixed order, 16 interleaved partial sums per row
//     meeting in a fixed tree), and one more sums the partial scalars and
//     forms beta, tau and alpha2.
// The reflector is never formed before the product: with v = (x - beta e0) s,
// s = 1/(alpha - beta), one has A22 v = (y - beta a0) s (a0 the first column
// of A22) and v^T A22 v = (x^T y - 2 beta y_0 + beta^2 a_00) s^2, so the next
// trd_step rebuilds v and w row by row from x, y and a0 (column k+1, which
// trd_step k leaves untouched).  No work group waits for or signals another
// inside a launch: the launch boundaries are the only synchronisation.
// Column k itself is rewritten into reflector form by trd_step k+1, which
// never reads it.
#include "internal.h"

#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace gwm {

namespace {

constexpr int TB = 64;  // tile edge
constexpr int NT = 256;  // threads per work group: 64 rows x 4 column quarters

struct TrdWork {
    double* X;       // [2][n]          column k after its pending update (rows > k), by parity of k
    double* Y;       // [n]             y = A22 x of the last reduced step (rows > k)
    double* part;    // [nbt][nbt][64]  per-tile partial vectors of y
    double* tsc;     // [nbt][nbt]      per-tile partial x^T y
    double* s2p;     // [nbt]           per-row-block partial |x|^2 (rows > k+1)
    double* scal;    // [2][8]          beta, tau, s, alpha2, w_k[k+1] of step k, by parity
};

constexpr int RT = 1024;  // threads of a reduce work group: 64 rows x 16 groups of partner blocks
constexpr int RG = RT / TB;

// the partial vectors of row block B summed into y in one fixed order:
// thread (lane, g) sums partner blocks kb + g, kb + g + 16, ..., then the 16
// group sums meet in a fixed binary tree.  The row blocks and the scalar
// work group both use it, so y_0 agrees bit for bit.  Every thread gets y of
// row B*64 + (its lane); red holds RT doubles of LDS.
__device__ inline double row_block_y(const double* part, int nbt, int kb, int B, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, g = tid >> 6;
    const double* pp = part + (long)B * nbt * TB + lane;
    double y = 0.0;
    for (int J = kb + g; J < nbt; J += RG) y += pp[(long)J * TB];
    red[tid] = y;
    __syncthreads();
    for (int s = RG / 2; s > 0; s >>= 1) {
        if (g < s) red[tid] += red[tid + s * TB];
        __syncthreads();
    }
    return red[lane];
}

// sum over the work group of one value per thread, fixed tree order
__device__ inline double block_sum(double v, double* red) {
    const int tid = threadIdx.x;
    __syncthreads();
    red[tid] = v;
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    return red[0];
}

// One Householder step (column k) on the lower triangle of the column-major
// n x n matrix A (leading dimension lda): applies reflector k-1 (from the
// scalars trd_reduce left) and writes the partials of y = A22 x.  Grid: one
// work group per lower tile (R >= C) of block rows/columns kb = k/64 .. nbt-1.
__global__ __launch_bounds__(NT) void trd_step_kernel(int n, long lda, int k, int nbt, double* A, double* d,
                                                      TrdWork wk) {
    __shared__ double sv[2][TB], sw[2][TB], sx[2][TB];
    __shared__ double syc[TB][TB + 1];
    __shared__ double sred[4][TB];
    __shared__ double syr[TB], sycol[TB];
    __shared__ double sdot[NT];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int p = k & 1, q = p ^ 1;
    const int kb = k / TB;
    // tile (R, C), R >= C, from the linear index over the trailing lower triangle
    const int t = blockIdx.x;
    int rr = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((rr + 1) * (rr + 2) / 2 <= t) ++rr;
    while (rr * (rr + 1) / 2 > t) --rr;
    const int cc = t - rr * (rr + 1) / 2;
    const int R = kb + rr, C = kb + cc;
    const bool diag = R == C;
    const int r0 = R * TB, c0 = C * TB;

    // the tile's elements: rows r0 + lane, columns c0 + 16 wv + j
    const int i = r0 + lane;
    double a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int col = c0 + wv * 16 + j;
        a[j] = (i < n && col < n && i >= col && col >= k) ? A[(long)col * lda + i] : 0.0;
    }

    // reflector k-1, still to be applied to rows/columns >= k
    const bool pend = k > 0;
    double bq = 0.0, tq = 0.0, sq = 0.0, aq = 0.0, wkk = 0.0;
    if (pend) {
        const double* sc = wk.scal + q * 8;
        bq = sc[0];
        tq = sc[1];
        sq = sc[2];
        aq = sc[3];
        wkk = sc[4];
    }
    if (tid < 2 * TB) {
        const int which = tid >> 6;
        const int ii = (which ? c0 : r0) + lane;
        double v = 0.0, w = 0.0, x = 0.0;
        if (ii < n && ii >= k) {
            const double aik = A[(long)k * lda + ii];  // column k (lower: ii >= k)
            if (pend) {
                v = (ii == k) ? 1.0 : wk.X[q * n + ii] * sq;
                w = tq * sq * (wk.Y[ii] - bq * aik) + aq * v;
            }
            if (ii > k) x = aik - v * wkk - w;
        }
        sv[which][lane] = v;
        sw[which][lane] = w;
        sx[which][lane] = x;
    }
    __syncthreads();

    // the tile: pending update (written back), then its share of y = A22 x
    const double vi = sv[0][lane], wi = sw[0][lane], xi = sx[0][lane];
    double yr = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int cl = wv * 16 + j;
        const int col = c0 + cl;
        double yc = 0.0;
        if (i < n && col < n && i >= col && col >= k) {
            double x = a[j];
            if (pend) x -= vi * sw[1][cl] + wi * sv[1][cl];
            if (col > k) {
                A[(long)col * lda + i] = x;
                yr += x * sx[1][cl];
                if (i != col) yc = x * xi;
            } else if (i == k) {
                d[k] = x;
            }
        }
        syc[cl][lane] = yc;
    }
    sred[wv][lane] = yr;
    __syncthreads();
    {
        // column sums of the transposed half: thread (cl, quarter) sums 16 rows
        const int cl = tid & 63, qq = tid >> 6;
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += syc[cl][qq * 16 + u];
        sdot[tid] = acc;
    }
    __syncthreads();
    if (tid < TB) {
        syr[tid] = sred[0][tid] + sred[1][tid] + sred[2][tid] + sred[3][tid];
        sycol[tid] = sdot[tid] + sdot[TB + tid] + sdot[2 * TB + tid] + sdot[3 * TB + tid];
    }
    __syncthreads();
    // partial vectors, the tile's x^T y share and (diagonal tiles) x, |x|^2
    double dot = 0.0, sq2 = 0.0;
    if (tid < TB) {
        const double y = diag ? syr[tid] + sycol[tid] : syr[tid];
        wk.part[((long)R * nbt + C) * TB + tid] = y;
        dot = sx[0][tid] * y;
        if (!diag) dot += sx[1][tid] * sycol[tid];
        if (diag) {
            const int ii = r0 + tid;
            if (ii < n) {
                const double xv = sx[0][tid];
                wk.X[p * n + ii] = xv;
                if (ii > k + 1) sq2 = xv * xv;
                // column k-1 in reflector form: e_{k-1} on the subdiagonal, v below
                if (pend && ii >= k) A[(long)(k - 1) * lda + ii] = (ii == k) ? bq : wk.X[q * n + ii] * sq;
            }
        }
    } else if (tid < 2 * TB && !diag) {
        wk.part[((long)C * nbt + R) * TB + lane] = sycol[lane];
    }
    // wave 0 holds every nonzero term: reduce it in registers
    if (wv == 0) {
        for (int o = 32; o > 0; o >>= 1) {
            dot += __shfl_xor(dot, o);
            sq2 += __shfl_xor(sq2, o);
        }
        if (lane == 0) {
            wk.tsc[(long)R * nbt + C] = dot;
            if (diag) wk.s2p[R] = sq2;
        }
    }
}

// Finishes step k: work group 0 forms the reflector's scalars, work group
// 1 + b sums the partial vectors of row block kb + b into y.
__global__ __launch_bounds__(RT) void trd_reduce_kernel(int n, long lda, int k, int nbt, const double* A,
                                                        double* e, double* tau, TrdWork wk) {
    __shared__ double red[RT];
    const int tid = threadIdx.x;
    const int kb = k / TB, m = nbt - kb;
    if (blockIdx.x > 0) {
        const int B = kb + (int)blockIdx.x - 1;
        const double y = row_block_y(wk.part, nbt, kb, B, red);
        const int i = B * TB + tid;
        if (tid < TB && i < n) wk.Y[i] = (i > k) ? y : 0.0;
        return;
    }
    // y_0 = y[k+1], summed exactly as its row block sums it
    const int B1 = (k + 1) / TB;
    const double y0 = __shfl(row_block_y(wk.part, nbt, kb, B1, red), (k + 1) - B1 * TB);
    double xy = 0.0, s2 = 0.0;
    for (int idx = tid; idx < m * m; idx += RT) {
        const int r1 = idx / m, c1 = idx - r1 * m;
        if (c1 <= r1) xy += wk.tsc[(long)(kb + r1) * nbt + kb + c1];
    }
    for (int B = kb + tid; B < nbt; B += RT) s2 += wk.s2p[B];
    xy = block_sum(xy, red);
    s2 = block_sum(s2, red);
    if (tid != 0) return;
    const double alpha = wk.X[(k & 1) * n + k + 1];
    const double a00 = A[(long)(k + 1) * lda + k + 1];
    double beta = alpha, tk = 0.0, sk = 0.0, a2 = 0.0;
    if (s2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + s2), alpha);
        tk = (beta - alpha) / beta;
        sk = 1.0 / (alpha - beta);
        const double vav = (xy - 2.0 * beta * y0 + beta * beta * a00) * sk * sk;
        a2 = -0.5 * tk * tk * vav;
    }
    double* sc = wk.scal + (k & 1) * 8;
    sc[0] = beta;
    sc[1] = tk;
    sc[2] = sk;
    sc[3] = a2;
    sc[4] = tk * sk * (y0 - beta * a00) + a2;  // w_k[k+1]  (v_k[k+1] = 1)
    e[k] = beta;
    tau[k] = tk;
}

// B = J A J (J the index reversal), lower triangle of the column-major view,
// from the lower triangle of the row-major view of A (the one the Lanczos
// matrices and LAPACK's convention define):  B(i, j) = A(n-1-i, n-1-j),
// i >= j.  Reducing B from its first column is reducing A from its last, as
// LAPACK's and rocSOLVER's upper-triangle reduction does; the moment matrices
// are strongly graded (eigenvalues spread over many decades, the small ones
// at the far end of the orbital order), and the small eigenpairs that the
// pseudo-inverse square roots keep are reproduced far better in that
// direction.
__global__ void reverse_kernel(int n, const double* __restrict__ A, double* __restrict__ B) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const long j = idx / n, i = idx - j * n;
    if (i >= j) B[idx] = A[(long)(n - 1 - j) * n + (n - 1 - i)];
}

// column a of V (an eigenvector of B) -> the eigenvector of A: components reversed
__global__ void unreverse_kernel(int n, double* __restrict__ V) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long half = n / 2;
    if (idx >= (long)n * half) return;
    const long a = idx / half, p = idx - a * half;
    double* col = V + a * n;
    const double t = col[p];
    col[p] = col[n - 1 - p];
    col[n - 1 - p] = t;
}

// Back-transformation C <- Q C, Q = H_0 H_1 ... H_{n-2} (the reflectors of
// the reduction), in blocks of QB reflectors applied last block first: the
// block H_k0 ... H_k1-1 is I - V T V^T with V the block's reflectors (unit
// entry explicit, rows k0+1 .. n-1), and T's inverse is the upper triangular
// S = diag(1/tau) + strictly_upper(V^T V) (the UT transform of Joffrain,
// Low, Quintana-Orti, van de Geijn and Van Zee), so
// C[k0+1:, :] -= V (S \ (V^T C[k0+1:, :])) is two GEMMs and one triangular
// solve.  A reflector with tau = 0 is the identity: its column of V is zero
// and its diagonal entry of S is 1.
constexpr int QB = 64;

// V [nr][bj] column-major (ld nr), rows k0+1 .. n-1: column c is reflector
// k = k0 + c, zero above row k+1, one at row k+1, the stored v below.
__global__ void build_v_kernel(int n, int k0, int bj, const double* __restrict__ Zr, const double* __restrict__ tau,
                               double* __restrict__ V) {
    const int nr = n - k0 - 1;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nr * bj) return;
    const int c = (int)(idx / nr), r = (int)(idx - (long)c * nr);
    const int i = k0 + 1 + r, k = k0 + c;
    double x = 0.0;
    if (tau[k] != 0.0) {
        if (i == k + 1) x = 1.0;
        else if (i > k + 1) x = Zr[(long)k * n + i];
    }
    V[idx] = x;
}

// S [bj][bj] column-major from G = V^T V and tau
__global__ void ut_factor_kernel(int bj, const double* __restrict__ G, const double* __restrict__ tau,
                                 double* __restrict__ S) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= bj * bj) return;
    const int c = idx / bj, r = idx - c * bj;
    double x = 0.0;
    if (r < c) x = G[idx];
    else if (r == c) x = tau[c] != 0.0 ? 1.0 / tau[c] : 1.0;
    S[idx] = x;
}

gw_status check_solver(Handle* h, rocblas_status st, const char* what) {
    if (st == rocblas_status_success) return GW_OK;
    return set_err(h, GW_ELIB, std::string(what) + " failed: " + rocblas_status_to_string(st));
}


}  // namespace

size_t syev_tridiag_bytes(int n) {
    const long nbt = (n + TB - 1) / TB;
    const long doubles = 3L * n + nbt * nbt * TB + nbt * nbt + nbt + 16 + (long)n + (long)n * n +
                         (long)n * QB + 2L * QB * QB + (long)QB * n;
    return sizeof(double) * (size_t)doubles;
}

namespace {

gw_status apply_q(Handle* h, int n, const double* Zr, const double* tau, double* C, double* V) {
    double* G = V + (long)n * QB;
    double* S = G + QB * QB;
    double* W1 = S + QB * QB;
    const double one = 1.0, zero = 0.0, mone = -1.0;
    const int nref = n - 1;
    for (int k0 = ((nref - 1) / QB) * QB; k0 >= 0; k0 -= QB) {
        const int bj = std::min(QB, nref - k0), nr = n - k0 - 1;
        hipLaunchKernelGGL(build_v_kernel, dim3((unsigned)(((long)nr * bj + 255) / 256)), dim3(256), 0, h->stream, n,
                           k0, bj, Zr, tau, V);
        GW_CHECK_LAUNCH(h);
        GW_TRY(check_solver(h,
                            rocblas_dgemm(h->blas, rocblas_operation_transpose, rocblas_operation_none, bj, bj, nr,
                                          &one, V, nr, V, nr, &zero, G, bj),
                            "rocblas_dgemm"));
        hipLaunchKernelGGL(ut_factor_kernel, dim3((unsigned)((bj * bj + 255) / 256)), dim3(256), 0, h->stream, bj, G,
                           tau + k0, S);
        GW_CHECK_LAUNCH(h);
        double* Cs = C + k0 + 1;  // rows k0+1 .. n-1, ld n
        GW_TRY(check_solver(h,
                            rocblas_dgemm(h->blas, rocblas_operation_transpose, rocblas_operation_none, bj, n, nr,
                                          &one, V, nr, Cs, n, &zero, W1, bj),
                            "rocblas_dgemm"));
        GW_TRY(check_solver(h,
                            rocblas_dtrsm(h->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                                          rocblas_diagonal_non_unit, bj, n, &one, S, bj, W1, bj),
                            "rocblas_dtrsm"));
        GW_TRY(check_solver(h,
                            rocblas_dgemm(h->blas, rocblas_operation_none, rocblas_operation_none, nr, n, bj, &mone, V,
                                          nr, W1, bj, &one, Cs, n),
                            "rocblas_dgemm"));
    }
    return GW_OK;
}

}  // namespace

gw_status syev_tridiag(Handle* h, int n, double* A, double* w, double* work, int* info, void* ws) {
    const int nbt = (n + TB - 1) / TB;
    TrdWork wk;
    wk.X = (double*)ws;
    wk.Y = wk.X + 2L * n;
    wk.part = wk.Y + n;
    wk.tsc = wk.part + (long)nbt * nbt * TB;
    wk.s2p = wk.tsc + (long)nbt * nbt;
    wk.scal = wk.s2p + nbt;
    double* tau = wk.scal + 16;
    double* Z = tau + n;
    double* Vq = Z + (long)n * n;
    // B = J A J into Z; B = Q T Q^T: d -> w, e -> work, reflectors -> lower triangle of Z
    hipLaunchKernelGGL(reverse_kernel, dim3((unsigned)(((long)n * n + 255) / 256)), dim3(256), 0, h->stream, n, A,
                       Z);
    GW_CHECK_LAUNCH(h);
    for (int k = 0; k < n; ++k) {
        const int kb = k / TB, m = nbt - kb;
        hipLaunchKernelGGL(trd_step_kernel, dim3(m * (m + 1) / 2), dim3(NT), 0, h->stream, n, (long)n, k, nbt, Z,
                           w, wk);
        GW_CHECK_LAUNCH(h);
        if (k + 1 < n) {
            hipLaunchKernelGGL(trd_reduce_kernel, dim3(m + 1), dim3(RT), 0, h->stream, n, (long)n, k, nbt, Z, work,
                               tau, wk);
            GW_CHECK_LAUNCH(h);
        }
    }
    // T's eigenvectors into A, then Q applied to them (the eigenvectors of B),
    // then their components reversed (the eigenvectors of A)
    GW_TRY(check_solver(h, rocsolver_dstedc(h->blas, rocblas_evect_tridiagonal, n, w, work, A, n, info),
                        "rocsolver_dstedc"));
    int hinfo = 0;
    GW_HIP(h, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    GW_HIP(h, hipStreamSynchronize(h->stream));
    if (hinfo != 0) return set_err(h, GW_ENUMERIC, "tridiagonal eigensolver did not converge");
    if (n > 1) {
        GW_TRY(apply_q(h, n, Z, tau, A, Vq));
        hipLaunchKernelGGL(unreverse_kernel, dim3((unsigned)(((long)n * (n / 2) + 255) / 256)), dim3(256), 0,
                           h->stream, n, A);
        GW_CHECK_LAUNCH(h);
    }
    return GW_OK;
}

}  // namespace gwm
