// Self-energy moments from R_t in mixed precision: int8 fixed-point digits on
// the integer MFMA with exact int32 accumulation, combined in FP64.
//
// Same contraction as the FP64 path (eqs. convolution_occ / convolution_vir
// with eq. w_moments):
//   stage 1  Zt^{(n)}[x,q,P] = sum_t s_{n,t}(x) sum_Q R_t[P,Q] L[Q,x,q]
//   stage 2  Sigma^{(n)}[p,q] = sum_{x in sector} sum_P L[P,x,p] Zt^{(n)}[x,q,P]
//
// Number format.  Every operand row (A) or column (B) of a contraction is
// scaled by a power of two 2^e so that |a| 2^-e < 1/2, then written in base
// 255 as
//   a = 2^e (d0/255 + d1/255^2 + d2/255^3 + d3/255^4),  d_i integers in [-127, 127],
// four int8 values (ND = 4; the remainder after d3 is below 2^-33 of 2^e).
// Base 255 rather than 256: balanced base-256 digits need the value 128,
// which int8 does not hold.  The product of two such numbers keeps the ten
// terms of digit weight w = i + j <= 3 (the dropped terms are ~2^-32 of the
// leading one).  Each weight has its own int32 MFMA accumulator; |d_i d_j| <=
// 127^2 and at most four pairs share a weight, so the sums are exact for up to
// 32768 k.  The weights are combined in FP64 (sum_w acc_w 255^-(w+2)) and
// scaled by 2^(e_row + e_col): the only error left is the truncation of the
// operands, not any accumulation error.
// The folded stage-1 result is stored as an FP32 value plus a BF16 residual
// (~32 significant bits); stage 2 re-digitises it per (x, q) column.
#include "mixed_jobs.h"

#include <algorithm>
#include <climits>
#include <cmath>

namespace gwm {

typedef int i32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int MK = MIX_MK;    // k per MFMA (v_mfma_i32_16x16x64_i8): 64 one-byte digits
constexpr int ND = MIX_ND;    // digits per operand
constexpr int MAXW = 3;       // largest digit weight i + j kept in a product
constexpr int KEXACT = 32768; // k over which the int32 digit sums stay exact

// FP64 weight of an int32 accumulator of digit weight w: 255^-(w + 2), the
// correctly rounded reciprocal of an integer that FP64 holds exactly
__device__ __forceinline__ constexpr double wscale(int w) {
    return w == 0 ? 1.0 / 65025.0
         : w == 1 ? 1.0 / 16581375.0
         : w == 2 ? 1.0 / 4228250625.0
         : w == 3 ? 1.0 / 1078203909375.0
                  : 1.0 / 274941996890625.0;
}

__device__ __forceinline__ void digitsN(double a, int e, i8* dg) {
    double x = ldexp(a, -e);          // |x| < 1/2 (<= 1/2 after the clamp below)
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const double y = x * 255.0;
        const double q = fmin(127.0, fmax(-127.0, rint(y)));
        x = y - q;                    // |x| <= 1/2
        dg[d] = (i8)(int)q;
    }
}

__device__ __forceinline__ int scale_exp(double amax) {
    // 2^e with amax * 2^-e in [1/4, 1/2) (e = ilogb + 2); zero rows get e = 0
    return amax > 0.0 ? ilogb(amax) + 2 : 0;
}

__device__ __forceinline__ unsigned pack4(const i8* d) {
    return (unsigned)(unsigned char)d[0] | ((unsigned)(unsigned char)d[1] << 8) |
           ((unsigned)(unsigned char)d[2] << 16) | ((unsigned)(unsigned char)d[3] << 24);
}

// ---------------------------------------------------------------------------
// Operand preparation
// ---------------------------------------------------------------------------

// Column exponents of L viewed as [naux][ncol]: e[j] over Q (one thread per column).
__global__ void col_exp_kernel(int naux, long ncol, const double* __restrict__ L, int* __restrict__ e) {
    long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ncol) return;
    double m = 0.0;
    for (int Q = 0; Q < naux; ++Q) m = fmax(m, fabs(L[(long)Q * ncol + j]));
    e[j] = scale_exp(m);
}

// Digit planes are k-blocked: digit (row, k) of a plane with `rows` rows sits at
// byte ((k / 64) * rows + row) * 64 + k % 64, so the 64 k of one MFMA step of 16
// consecutive rows are 1 KB of contiguous memory (whole cache lines).

// Row scales and k-blocked digit planes of X[rows][cols] (times cs[c] when cs is
// set), zero-padded to kpad (a multiple of 64): one block per row, the row
// maximum by a block reduction, then 8 consecutive k per thread so that each
// digit plane gets one 8-byte store per thread and step.  With Yd set, the
// same pass also writes the planes of X o D (D = d2[c]) with their own row
// scales e2, so X is read twice instead of four times.
__global__ __launch_bounds__(256) void digitise_rows_kernel(long rows, int cols, int kpad,
                                                            const double* __restrict__ X,
                                                            const double* __restrict__ cs, int* __restrict__ e,
                                                            i8* __restrict__ Xd, const double* __restrict__ d2,
                                                            int* __restrict__ e2, i8* __restrict__ Yd) {
    const long row = blockIdx.x;
    const double* __restrict__ x = X + row * cols;
    __shared__ double red[2][256];
    double m = 0.0, m2 = 0.0;
    for (int c = threadIdx.x; c < cols; c += 256) {
        const double v = x[c];
        m = fmax(m, fabs(v * (cs ? cs[c] : 1.0)));
        if (Yd) m2 = fmax(m2, fabs(v * d2[c]));
    }
    red[0][threadIdx.x] = m;
    red[1][threadIdx.x] = m2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    const int ex = scale_exp(red[0][0]);
    const int ex2 = scale_exp(red[1][0]);
    if (threadIdx.x == 0) {
        e[row] = ex;
        if (Yd) e2[row] = ex2;
    }
    const long plane = rows * (long)kpad;
    for (int c0 = threadIdx.x * 8; c0 < kpad; c0 += 256 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = c0 + u < cols ? x[c0 + u] : 0.0;
        const long o = ((long)(c0 >> 6) * rows + row) * 64 + (c0 & 63);
        i8 dg[ND][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            i8 t[ND];
            digitsN(v[u] * (cs && c0 + u < cols ? cs[c0 + u] : 1.0), ex, t);
#pragma unroll
            for (int d = 0; d < ND; ++d) dg[d][u] = t[d];
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) *(uint2*)(Xd + d * plane + o) = make_uint2(pack4(dg[d]), pack4(dg[d] + 4));
        if (Yd) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                i8 t[ND];
                digitsN(c0 + u < cols ? v[u] * d2[c0 + u] : 0.0, ex2, t);
#pragma unroll
                for (int d = 0; d < ND; ++d) dg[d][u] = t[d];
            }
#pragma unroll
            for (int d = 0; d < ND; ++d) *(uint2*)(Yd + d * plane + o) = make_uint2(pack4(dg[d]), pack4(dg[d] + 4));
        }
    }
}

// L digits, transposed: Ld[d] k-blocked over rows j (k = Q) = digits of L[Q][j] (Q < naux, else 0),
// 32x32 LDS tiles.
__global__ void digits_lt_kernel(int naux, long ncol, int Ap, const double* __restrict__ L,
                                 const int* __restrict__ e, i8* __restrict__ Ld) {
    __shared__ double tile[32][33];
    const long j0 = (long)blockIdx.x * 32;
    const int q0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
    for (int r = ty; r < 32; r += 8) {
        int Q = q0 + r;
        long j = j0 + tx;
        tile[r][tx] = (Q < naux && j < ncol) ? L[(long)Q * ncol + j] : 0.0;
    }
    __syncthreads();
    const long plane = ncol * (long)Ap;
    for (int r = ty; r < 32; r += 8) {
        long j = j0 + r;
        int Q = q0 + tx;
        if (j >= ncol || Q >= Ap) continue;
        i8 dg[ND] = {};
        if (Q < naux) digitsN(tile[tx][r], e[j], dg);
        long o = ((long)(Q >> 6) * ncol + j) * 64 + (Q & 63);
#pragma unroll
        for (int d = 0; d < ND; ++d) Ld[d * plane + o] = dg[d];
    }
}

// Long rows in two passes that keep the whole chip busy.  Pass one: the row
// exponents, scale_exp of max_c |X cs| by integer atomicMax over the row's
// 8192-column chunks into e, preset to INT_MIN (a row with no non-zero
// element keeps it), and with d2 set the same for X o D into e2 (cs is then
// unset).  Pass two: the digits of 16 rows x 128 columns per work group (a
// thread: one row, 8 consecutive columns), so that the 16 rows' 64-byte k
// rows of one k block, adjacent in the k-blocked planes, are written together
// (1 KB per plane); one block per row would leave isolated 64-byte pieces,
// rows x 64 bytes apart.  INT_MIN reads as 0 and is written back as 0 by the
// first column's thread (the others may read either value: the same digits).
constexpr int RCH = 8192;
__global__ __launch_bounds__(256) void fill_i32_kernel(int* __restrict__ p, long n, int v) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void row_exp_kernel(int cols, const double* __restrict__ X,
                                                      const double* __restrict__ cs, int* __restrict__ e,
                                                      const double* __restrict__ d2, int* __restrict__ e2) {
    const long row = blockIdx.y;
    const int c0 = blockIdx.x * RCH;
    const double* __restrict__ x = X + row * cols;
    double m = 0.0, m2 = 0.0;
    if (c0 + RCH <= cols) {
        // a whole chunk: no guards, so that the loads of an unrolled group issue together
#pragma unroll 8
        for (int i = 0; i < RCH / 256; ++i) {
            const int c = c0 + i * 256 + (int)threadIdx.x;
            const double v = x[c] * (cs ? cs[c] : 1.0);
            m = fmax(m, fabs(v));
            if (d2) m2 = fmax(m2, fabs(v * d2[c]));
        }
    } else {
        for (int i = 0; i < RCH / 256; ++i) {
            const int c = c0 + i * 256 + (int)threadIdx.x;
            if (c < cols) {
                const double v = x[c] * (cs ? cs[c] : 1.0);
                m = fmax(m, fabs(v));
                if (d2) m2 = fmax(m2, fabs(v * d2[c]));
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        m = fmax(m, __shfl_xor(m, o));
        m2 = fmax(m2, __shfl_xor(m2, o));
    }
    __shared__ double red[2][4];
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = m;
        red[1][threadIdx.x >> 6] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        m2 = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        if (m > 0.0) atomicMax(e + row, scale_exp(m));
        if (d2 && m2 > 0.0) atomicMax(e2 + row, scale_exp(m2));
    }
}

__global__ __launch_bounds__(256) void row_digits_kernel(long rows, int cols, int kpad, const double* __restrict__ X,
                                                         const double* __restrict__ cs, int* __restrict__ e,
                                                         i8* __restrict__ Xd, const double* __restrict__ d2,
                                                         int* __restrict__ e2, i8* __restrict__ Yd) {
    const long row = (long)blockIdx.y * 16 + (threadIdx.x >> 4);
    const int c0 = blockIdx.x * 128 + (int)(threadIdx.x & 15) * 8;
    if (row >= rows || c0 >= kpad) return;
    int ex = e[row];
    if (ex == INT_MIN) ex = 0;
    int ex2 = 0;
    if (Yd) {
        ex2 = e2[row];
        if (ex2 == INT_MIN) ex2 = 0;
    }
    if (c0 == 0) {
        e[row] = ex;
        if (Yd) e2[row] = ex2;
    }
    const double* __restrict__ x = X + row * cols;
    double v[8];
    if (c0 + 8 <= cols) {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = x[c0 + u] * (cs ? cs[c0 + u] : 1.0);
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = c0 + u < cols ? x[c0 + u] * (cs ? cs[c0 + u] : 1.0) : 0.0;
    }
    const long plane = rows * (long)kpad;
    const long o = ((long)(c0 >> 6) * rows + row) * 64 + (c0 & 63);
    i8 dg[ND][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        i8 q[ND];
        digitsN(v[u], ex, q);
#pragma unroll
        for (int d = 0; d < ND; ++d) dg[d][u] = q[d];
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) *(uint2*)(Xd + d * plane + o) = make_uint2(pack4(dg[d]), pack4(dg[d] + 4));
    if (Yd) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            i8 q[ND];
            digitsN(c0 + u < cols ? v[u] * d2[c0 + u] : 0.0, ex2, q);
#pragma unroll
            for (int d = 0; d < ND; ++d) dg[d][u] = q[d];
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) *(uint2*)(Yd + d * plane + o) = make_uint2(pack4(dg[d]), pack4(dg[d] + 4));
    }
}

// Row exponents of X o as_b for all nb column scales as_b (the RPA quadrature
// nodes) in one read of X: e[b][row] = scale_exp(max_c |X[row][c] as_b[c]|),
// by integer atomicMax into e preset to INT_MIN, as row_exp_kernel does for
// one scale.  A work group takes 16 rows x 512 columns (a thread: one row, the
// columns cg + 16 u), so that each as_b chunk is read once per 16 rows; the
// 16 threads of a row reduce each node's maximum by shuffles.
__global__ __launch_bounds__(256) void node_row_exp_kernel(int rows, int cols, const double* __restrict__ X,
                                                           const double* __restrict__ as, int nb,
                                                           int* __restrict__ e) {
    const int r = threadIdx.x >> 4, cg = threadIdx.x & 15;
    const int row = blockIdx.y * 16 + r;
    const int c0 = blockIdx.x * 512 + cg;
    double x[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) {
        const int c = c0 + u * 16;
        x[u] = (row < rows && c < cols) ? X[(long)row * cols + c] : 0.0;
    }
    for (int b = 0; b < nb; ++b) {
        const double* __restrict__ a = as + (long)b * cols;
        double m = 0.0;
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int c = c0 + u * 16;
            if (c < cols) m = fmax(m, fabs(x[u] * a[c]));
        }
        m = fmax(m, __shfl_xor(m, 1));
        m = fmax(m, __shfl_xor(m, 2));
        m = fmax(m, __shfl_xor(m, 4));
        m = fmax(m, __shfl_xor(m, 8));
        if (cg == 0 && row < rows && m > 0.0) atomicMax(e + (long)b * rows + row, scale_exp(m));
    }
}

// col_exp_kernel and digits_lt_kernel in one read of X[naux][ncol]: 16 columns
// per work group of 512 threads, kept in registers (4 consecutive rows per
// thread and 128-row pass, NP passes: naux <= Ap <= 128 NP), the column maxima
// by shuffles and LDS; the digits then go through LDS so that every plane is
// written in 16-byte stores of whole 64-byte k rows (1 KB of contiguous
// memory per wave).
template <int NP>
__global__ __launch_bounds__(512) void digits_cols_kernel(int naux, long ncol, int Ap,
                                                             const double* __restrict__ X, int* __restrict__ e,
                                                             i8* __restrict__ Xd) {
    constexpr int JS = 128 * NP + 16;  // LDS bytes per column of one plane (the 16 spread the banks)
    __shared__ double red[8][16];
    __shared__ __attribute__((aligned(16))) unsigned char dl[ND * 16 * JS];
    const int t = threadIdx.x;
    const int jj = t & 15, qr = t >> 4;
    const long j0 = (long)blockIdx.x * 16;
    const long j = j0 + jj;
    const bool jok = j < ncol;
    double v[NP][4];
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int Q = 128 * i + 4 * qr + r;
            v[i][r] = (jok && Q < naux) ? X[(long)Q * ncol + j] : 0.0;
            m = fmax(m, fabs(v[i][r]));
        }
    // the four lanes of a wave on one column, then the eight waves
    m = fmax(m, __shfl_xor(m, 16));
    m = fmax(m, __shfl_xor(m, 32));
    if ((t & 63) < 16) red[t >> 6][jj] = m;
    __syncthreads();
    m = red[0][jj];
#pragma unroll
    for (int w = 1; w < 8; ++w) m = fmax(m, red[w][jj]);
    const int ex = scale_exp(m);
    if (qr == 0 && jok) e[j] = ex;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        i8 dg[ND][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            i8 q[ND];
            digitsN(v[i][r], ex, q);
#pragma unroll
            for (int d = 0; d < ND; ++d) dg[d][r] = q[d];
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) *(unsigned*)(dl + (d * 16 + jj) * JS + 128 * i + 4 * qr) = pack4(dg[d]);
    }
    __syncthreads();
    const int nkb = Ap / 64;
    const long plane = ncol * (long)Ap;
    // 16-byte chunk c of k block kb of column cj, plane d
    for (int idx = t; idx < ND * nkb * 64; idx += 512) {
        const int c = idx & 3, cj = (idx >> 2) & 15, rest = idx >> 6;
        const int kb = rest % nkb, d = rest / nkb;
        if (j0 + cj >= ncol) continue;
        const uint4 val = *(const uint4*)(dl + (d * 16 + cj) * JS + kb * 64 + c * 16);
        *(uint4*)(Xd + d * plane + ((long)kb * ncol + j0 + cj) * 64 + c * 16) = val;
    }
}

// ---------------------------------------------------------------------------
// Stage 1: R_t . L for all t of a 16(P) x 128(j) tile, fold, FP32 + BF16-residual output
// ---------------------------------------------------------------------------

constexpr double binom2(int n, int k) {
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (n - k + i) / i;
    return 2.0 * c;
}

// LDS slab rows hold 64 k (64 B); the 16-byte chunk c of row r is stored at
// chunk c ^ f(r), f(r) = ((r >> 1) & 3) ^ ((r >> 3) & 1).  A b128 read of one
// chunk column by 16 rows then touches 16 distinct 16-byte slots modulo 256 B,
// and each group of 8 rows 8 distinct slots modulo 128 B, so it is free of bank
// conflicts whether the LDS serves 8 or 16 lanes of a b128 read per cycle.
__device__ __forceinline__ int swz(int row, int chunk) { return chunk ^ ((row >> 1) & 3) ^ ((row >> 3) & 1); }

typedef unsigned char lds_t;

// Tile: 16 P rows x FC = fold_cols(NT) columns j, all NT moments t.  Wave w
// owns TPW moments (t group w % TG) for the 64 columns of column group w / TG
// (four 16-column blocks): 4 weights x TPW x 4 int32 accumulator blocks, at
// most 192 registers, which stay in AGPRs.  The R digits (A operand, private
// to a wave's moments) go from memory straight to registers, double
// buffered; the L digits (B operand, shared by the waves) go through an
// NS-stage LDS pipeline.  After the k loop the waves exchange their FP64
// values through LDS so that each wave folds all NT moments of its columns.
template <int NT>
struct FoldSlab {
    static constexpr int TPW = fold_tpw(NT);
    static constexpr int TG = fold_tg(NT);
    static constexpr int CG = fold_cg(NT);
    static constexpr int FC = fold_cols(NT);
    static constexpr int NS = 4;                               // B stages
    static constexpr int B_ROWS = ND * FC;                     // (d, c) rows of a B stage
    static constexpr int BST = B_ROWS * 64;                    // bytes per B stage
    static constexpr int XCH = NT * 4 * CG * 64 * 4 * 8;       // bytes of the epilogue exchange
    static constexpr int LDS = NS * BST > XCH ? NS * BST : XCH;
    static_assert(TG * CG == 4 && TPW * TG >= NT && TPW <= 3 && CG <= 2, "fold wave layout");
};

// Pair block t of nb x nb upper blocks (X <= Y), row by row.
__device__ __forceinline__ void pair_block_of(int t, int nb, int& X, int& Y) {
    int r = 0;
    while (t >= nb - r) { t -= nb - r; ++r; }
    X = r;
    Y = r + t;
}

// Binary search of the job whose first work item is the largest <= item.
template <typename Job>
__device__ __forceinline__ int find_job(const Job* __restrict__ jobs, int njobs, long item) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].item0 <= item) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

__device__ __forceinline__ i32x4 lds_b128(const lds_t* p) { return *(const i32x4*)p; }

// s_waitcnt immediate that waits for vmcnt <= n (n < 64) and for nothing else:
// vmcnt bits [3:0] and [15:14], expcnt [6:4] = 7, lgkmcnt [11:8] = 15.
constexpr int vmcnt_only(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

__device__ __forceinline__ i32x4 mfma8(i32x4 a, i32x4 b, i32x4 c) {
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

template <int NT>
__device__ __forceinline__ void fold_tile(const FoldJob& g, int pb, int ct, lds_t* lds) {
    using FS = FoldSlab<NT>;
    constexpr int TPW = FS::TPW, TG = FS::TG, CG = FS::CG, FC = FS::FC;
    constexpr int B_ROWS = FS::B_ROWS, BST = FS::BST, NS = FS::NS;
    const i8* __restrict__ Rd = g.Rd;
    const int* __restrict__ eR = g.eR;
    const i8* __restrict__ Ld = g.Ld;
    const int* __restrict__ eL = g.eL;
    const double* __restrict__ eps = g.eps;
    const int naux = g.naux, Ap = g.Ap, nmo = g.nmo, nocc = g.nocc;
    const long ncol = g.ncol, rplane = g.rplane, lplane = g.lplane;
    float* __restrict__ Zt = g.Zt;
    u16* __restrict__ Zl = g.Zl;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lr = lane & 15;
    const int lk = lane >> 4;
    const long c0 = (long)ct * FC;
    const int P0 = pb * 16;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int tg = wv % TG, cg = wv / TG;       // this wave's moment group and column group
    const int t0 = tg * TPW;

    // A operand: lane (lr, lk) holds row P0 + lr and k chunk lk of the 16 x 64
    // block of moment t, i.e. byte ((kt * NT * naux) + t * naux + P) * 64 + 16 lk
    // of each digit plane; rows past naux read a clamped (valid) row.  Moments
    // past NT (when TPW does not divide NT) repeat the last one; their results
    // are never used.
    const int rrows64 = NT * naux * 64;               // bytes per k block of an R plane
    unsigned voffA[3];
#pragma unroll
    for (int tt = 0; tt < 3; ++tt)
        voffA[tt] = (unsigned)((min(t0 + tt, NT - 1) * naux + min(P0 + lr, naux - 1)) * 64 + lk * 16);
    auto ldA = [&](int kt, int tt, int d) -> i32x4 {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)(Rd + d * rplane), (short)0, (int)rplane, 0x00020000);
        return __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voffA[tt], kt * rrows64, 0));
    };

    // B operand by LDS-DMA buffer loads (16 bytes per lane; one wave
    // instruction fills 1 KB of LDS at M0 + 16 * lane).  Vector s of wave w
    // fills stage rows s * 64 + 16 w + (lane >> 2), slot lane & 3: d = s / CG,
    // c = 64 (s % CG) + 16 w + (lane >> 2).  The lane fetches the global chunk
    // that the swizzle puts in its slot; columns past ncol read a clamped row.
    static_assert((B_ROWS * 4) % 256 == 0, "slab vectors per thread");
    constexpr int BVT = B_ROWS * 4 / 256;
    const long M2 = lplane / Ap;                      // rows of an L digit plane
    const int lrow = lane >> 2;
    const int gch = swz(lrow, lane & 3);              // swz is an involution in the chunk
    // column group h of the tile is pair block ct * CG + h; its column c_in =
    // 16 w + (lane >> 2) is the pair (8 X + (c_in >> 3), 8 Y + (c_in & 7)).
    // Past the last block or the orbital range a lane reads a clamped (valid,
    // unused) row.
    unsigned offB[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        int X, Y;
        pair_block_of(min(ct * CG + h, g.nblk - 1), g.nb, X, Y);
        const int cin = wv * 16 + lrow;
        const int x = min(8 * X + (cin >> 3), nmo - 1), y = min(8 * Y + (cin & 7), nmo - 1);
        offB[h] = (unsigned)(((long)x * nmo + y) * 64 + gch * 16);
    }
    auto ldB = [&](int kt) {
        lds_t* B = lds + (kt % NS) * BST + wv * 16 * 64;
        const int kc = min(kt, Ap / MK - 1);          // past the end: refetch a valid block (unused)
#pragma unroll
        for (int s = 0; s < BVT; ++s) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(Ld + (s / CG) * lplane + (long)kc * M2 * 64), (short)0, (int)(M2 * 64), 0x00020000);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(B + s * 64 * 64),
                                                     16, offB[s % CG], 0, 0, 0);
        }
    };

    // one exact int32 accumulator per digit weight, own moment and column
    // block (sized for TPW <= 3; entries past TPW are never touched)
    i32x4 acc[MAXW + 1][3][4];
#pragma unroll
    for (int w = 0; w <= MAXW; ++w)
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) acc[w][tt][cb] = (i32x4){0, 0, 0, 0};

    // Every step issues the same loads in the same order: the A blocks two
    // steps ahead (three register buffers: an A block has two steps' MFMAs to
    // arrive), then the B stage NS - 1 ahead (past the end: valid refetches
    // whose data is never read).  The prologue issues B(0), A(0), B(1), A(1),
    // B(2) as if steps -2 and -1 had run.  So when step kt starts, only the
    // loads of step kt - 1 (A(kt + 1), B(kt + NS - 2)) and the B loads of step
    // kt - 2 are younger than A(kt), and B(kt) is older still: both have
    // landed once vmcnt <= 2 BVT + 4 TPW.
    static_assert(NS >= 3, "B(kt) must be issued before A(kt)");
    const int nkt = Ap / MK;

    // The scales of this lane's results (the exponents of its rows (t, P)
    // and of its columns, eps of the orbitals of its folded pairs) are
    // fetched ahead of the k loop, so that the epilogues wait on no memory.
    int eRv[3][4], eLv[4];
    bool cokv[4];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            eRv[tt][r] = eR[(long)min(t0 + tt, NT - 1) * naux + min(P0 + 4 * lk + r, naux - 1)];
    {
        const int pbk = ct * CG + cg;
        int BX, BY;
        pair_block_of(min(pbk, g.nblk - 1), g.nb, BX, BY);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int cin = cb * 16 + lr;
            const int x = 8 * BX + (cin >> 3), y = 8 * BY + (cin & 7);
            cokv[cb] = pbk < g.nblk && x < nmo && y < nmo;
            eLv[cb] = eL[cokv[cb] ? (long)x * nmo + y : 0];
        }
    }
    double epx[CG], epy[CG];
#pragma unroll
    for (int i = 0; i < CG; ++i) {
        int BX, BY;
        pair_block_of(min(ct * CG + i, g.nblk - 1), g.nb, BX, BY);
        const int cin = wv * 16 + lr;
        epx[i] = eps[min(8 * BX + (cin >> 3), nmo - 1)];
        epy[i] = eps[min(8 * BY + (cin & 7), nmo - 1)];
    }

    i32x4 a0[3][ND], a1[3][ND], a2[3][ND];
    ldB(0);
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
        for (int d = 0; d < ND; ++d) a0[tt][d] = ldA(0, tt, d);
    ldB(1);
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
        for (int d = 0; d < ND; ++d) a1[tt][d] = ldA(min(1, nkt - 1), tt, d);
    ldB(2);
    const int boff = cg * 64 * 64 + lr * 64 + swz(lr, lk) * 16;
    auto step = [&](int kt, i32x4 (&acur)[3][ND], i32x4 (&anext)[3][ND]) {
        // own loads up to stage kt done; the plain s_barrier (no fence, which
        // would wait for every outstanding LDS-DMA load) then makes all waves'
        // stage kt visible and frees stage kt - 1 for the refill below
        // (the builtin, unlike an asm statement, is seen by the compiler's
        // own wait placement, which then adds no stricter waits for A(kt))
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(vmcnt_only(2 * BVT + 4 * TPW));
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        const int kn = min(kt + 2, nkt - 1);
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
            for (int d = 0; d < ND; ++d) anext[tt][d] = ldA(kn, tt, d);
        ldB(kt + NS - 1);
        const lds_t* B = lds + (kt % NS) * BST + boff;
        // B digits in order: the products of weight w need digits <= w
        i32x4 b[4][ND];
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) b[cb][d] = lds_b128(B + (d * FC + cb * 16) * 64);
#pragma unroll
        for (int w = 0; w <= MAXW; ++w)
#pragma unroll
            for (int ii = 0; ii <= w; ++ii)
#pragma unroll
                for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        if (ii < ND && w - ii < ND) acc[w][tt][cb] = mfma8(acur[tt][ii], b[cb][w - ii], acc[w][tt][cb]);
        // schedule: loads, reads of digits 0 and 1, then per weight w its
        // products with the reads of digit w + 2 among them
        __builtin_amdgcn_sched_group_barrier(0x020, 4 * TPW + BVT, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);          // digits 0, 1
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * TPW, 0);    // weight 0
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);          // digit 2
        __builtin_amdgcn_sched_group_barrier(0x008, 8 * TPW, 0);    // weight 1
        __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);          // digit 3
        __builtin_amdgcn_sched_group_barrier(0x008, 12 * TPW, 0);   // weight 2
        __builtin_amdgcn_sched_group_barrier(0x008, 16 * TPW, 0);   // weight 3
    };
    // whole triples without conditions (so that the compiler's own waits on
    // the A registers see one path), then the remainder
    int kt = 0;
    for (; kt + 3 <= nkt; kt += 3) {
        step(kt, a0, a2);
        step(kt + 1, a1, a0);
        step(kt + 2, a2, a1);
    }
    if (kt < nkt) step(kt, a0, a2);
    if (kt + 1 < nkt) step(kt + 1, a1, a0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    // epilogue 1: FP64 combination and scaling of this wave's moments into the
    // exchange X[t][q][lane][r] (q = 4 cg + cb: the column block); the slab
    // buffers are free (barrier above)
    double* X = (double*)lds;
    constexpr int NQ = 4 * CG;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
        for (int tt = 0; tt < TPW; ++tt) {
            const int t = t0 + tt;
            if (t >= NT) continue;
            double v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double z = 0.0;
#pragma unroll
                for (int w = MAXW; w >= 0; --w) z += (double)acc[w][tt][cb][r] * wscale(w);
                z = ldexp(z, eRv[tt][r] + eLv[cb]);
                v[r] = (cokv[cb] && P0 + 4 * lk + r < naux) ? z : 0.0;
            }
            double* dst = X + (((long)t * NQ + cg * 4 + cb) * 64 + lane) * 4;
            *(double4*)dst = make_double4(v[0], v[1], v[2], v[3]);
        }
    }
    __syncthreads();

    // epilogue 2: wave w folds all moments of column blocks q = w + 4 i (pair
    // block ct * CG + i, pairs 16 w .. 16 w + 15): binomial / eps-power fold
    // with the sign (-1)^t of an occupied orbital, FP32 + BF16 residual store
    // of the four consecutive rows P0 + 4 lk + r, at (x, y) with eps_x and,
    // off the diagonal blocks, at (y, x) with eps_y
#pragma unroll
    for (int i = 0; i < CG; ++i) {
        const int q = wv + 4 * i;
        const int pbk = ct * CG + i;
        if (pbk >= g.nblk) continue;
        int BX, BY;
        pair_block_of(pbk, g.nb, BX, BY);
        const int cin = wv * 16 + lr;
        const int x = 8 * BX + (cin >> 3), y = 8 * BY + (cin & 7);
        if (x >= nmo || y >= nmo) continue;
        double a[NT][4];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double4 v = *(const double4*)(X + (((long)t * NQ + q) * 64 + lane) * 4);
            a[t][0] = v.x; a[t][1] = v.y; a[t][2] = v.z; a[t][3] = v.w;
        }
#pragma unroll
        for (int o = 0; o < 2; ++o) {
            if (o == 1 && BX == BY) break;
            const int xo = o ? y : x;
            const long row = o ? (long)y * nmo + x : (long)x * nmo + y;
            const double ex = o ? epy[i] : epx[i];
            const bool occ = xo < nocc;
            double pw[NT];
            pw[0] = 1.0;
#pragma unroll
            for (int k = 1; k < NT; ++k) pw[k] = pw[k - 1] * ex;
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                float hv[4];
                unsigned lv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double z = 0.0;
#pragma unroll
                    for (int t = 0; t <= n; ++t) z += binom2(n, t) * pw[n - t] * ((occ && (t & 1)) ? -a[t][r] : a[t][r]);
                    const float hi = (float)z;
                    const unsigned lb = __float_as_uint((float)(z - (double)hi));
                    hv[r] = hi;
                    lv[r] = (lb + 0x7fffu + ((lb >> 16) & 1u)) >> 16;
                }
                const long off = ((long)n * ncol + row) * Ap + P0 + 4 * lk;
                *(float4*)(Zt + off) = make_float4(hv[0], hv[1], hv[2], hv[3]);
                *(uint2*)(Zl + off) = make_uint2(lv[0] | (lv[1] << 16), lv[2] | (lv[3] << 16));
            }
        }
    }
    // the next tile of a persistent work group reuses the LDS
    __syncthreads();
}

// Single job: XCD-aware grouped raster over (P-block, column tile).  Work
// group b runs on XCD b % 8; each XCD walks groups of 4 P-blocks x 8 column
// tiles, which share their R-digit (A) and L-digit (B) slabs through its L2
// (per k step 4 A slabs + 8 B slabs of distinct data for 32 tiles).
template <int NT>
__global__ __launch_bounds__(256, 1) void fold_mixed_kernel(FoldJob g) {
    __shared__ __attribute__((aligned(16))) lds_t lds[FoldSlab<NT>::LDS];
    const int nPg = (g.nP + 3) / 4;
    const int b = blockIdx.x;
    const int xcd = b & 7, local = b >> 3;
    const int grp = (local >> 5) * 8 + xcd;
    const int w = local & 31;
    const int pb = (grp % nPg) * 4 + (w & 3);
    const int ct = (grp / nPg) * 8 + (w >> 2);
    if (pb >= g.nP || ct >= g.nC) return;
    fold_tile<NT>(g, pb, ct, lds);
}

// Grouped, persistent, XCD-aware: the tiles of every job are cut into groups
// of 4 P-blocks x 8 column tiles (which share their R- and L-digit slabs),
// numbered job after job (item0 = a job's first group).  Work group b runs on
// XCD x = b % 8 and is work group b / 8 of that XCD's W = gridDim / 8; XCD x
// takes the groups x, x + 8, x + 16, ... and its work groups walk that
// sequence's tiles (32 per group) with stride W, so the tiles of one group
// run together on one XCD and meet in its L2.  LDS is free again at the start
// of each tile: fold_tile ends with a barrier.
template <int NT>
__global__ __launch_bounds__(256, 1) void fold_grouped_kernel(const FoldJob* __restrict__ jobs, int njobs,
                                                              long groups) {
    __shared__ __attribute__((aligned(16))) lds_t lds[FoldSlab<NT>::LDS];
    const int x = blockIdx.x & 7;
    const long W = gridDim.x >> 3;
    for (long k = blockIdx.x >> 3;; k += W) {
        const long grp = (k >> 5) * 8 + x;
        if (grp >= groups) break;
        const FoldJob g = jobs[find_job(jobs, njobs, grp)];
        const long gl = grp - g.item0;
        const int nPg = (g.nP + 3) / 4;
        const int w = (int)(k & 31);
        const int pb = (int)(gl % nPg) * 4 + (w & 3);
        const int ct = (int)(gl / nPg) * 8 + (w >> 2);
        if (pb < g.nP && ct < g.nC) fold_tile<NT>(g, pb, ct, lds);
    }
}

// Stage-1 result to digits: per row r = n * ncol + c (one wave) the exponent
// of max_P |Zt| and the digits of Zt + Zl (FP32 + BF16 residual) into the
// k-blocked planes Zd[d] (rows = nt * ncol, k = P).  Each lane holds 8
// consecutive P per 512-wide pass (Ap <= 64 * 8 * ZPASS), so reads are 32 + 16
// bytes and every digit plane gets one 8-byte store per lane and pass.
constexpr int ZPASS = 8;
__device__ __forceinline__ void zdig_row(const ZdigJob& g, long row, int lane) {
    const long rows = g.rows;
    const int Ap = g.Ap;
    const float* __restrict__ Zt = g.Zt;
    const u16* __restrict__ Zl = g.Zl;
    int* __restrict__ eZ = g.eZ;
    i8* __restrict__ Zd = g.Zd;
    const float* z = Zt + row * Ap;
    const u16* zl = Zl + row * Ap;
    float4 v[ZPASS][2];
    uint4 w[ZPASS];
    float m = 0.f;
#pragma unroll
    for (int ps = 0; ps < ZPASS; ++ps) {
        const int c = ps * 512 + lane * 8;
        v[ps][0] = v[ps][1] = make_float4(0.f, 0.f, 0.f, 0.f);
        w[ps] = make_uint4(0, 0, 0, 0);
        if (c < Ap) {
            v[ps][0] = *(const float4*)(z + c);
            v[ps][1] = *(const float4*)(z + c + 4);
            w[ps] = *(const uint4*)(zl + c);
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v[ps][0].x), fabsf(v[ps][0].y)), fmaxf(fabsf(v[ps][0].z), fabsf(v[ps][0].w))));
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v[ps][1].x), fabsf(v[ps][1].y)), fmaxf(fabsf(v[ps][1].z), fabsf(v[ps][1].w))));
        }
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    const int e = scale_exp((double)m);
    if (lane == 0) eZ[row] = e;
    const long plane = rows * (long)Ap;
#pragma unroll
    for (int ps = 0; ps < ZPASS; ++ps) {
        const int c = ps * 512 + lane * 8;
        if (c >= Ap) continue;
        i8 dg[ND][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float4 vv = v[ps][u >> 2];
            const float hv = (u & 3) == 0 ? vv.x : (u & 3) == 1 ? vv.y : (u & 3) == 2 ? vv.z : vv.w;
            const unsigned lw = (u >> 1) == 0 ? w[ps].x : (u >> 1) == 1 ? w[ps].y : (u >> 1) == 2 ? w[ps].z : w[ps].w;
            const unsigned lb = (u & 1) ? (lw & 0xffff0000u) : (lw << 16);
            i8 t[ND];
            digitsN((double)hv + (double)__uint_as_float(lb), e, t);
#pragma unroll
            for (int d = 0; d < ND; ++d) dg[d][u] = t[d];
        }
        const long o = ((long)(c >> 6) * rows + row) * 64 + (c & 63);
#pragma unroll
        for (int d = 0; d < ND; ++d) *(uint2*)(Zd + d * plane + o) = make_uint2(pack4(dg[d]), pack4(dg[d] + 4));
    }
}

__global__ __launch_bounds__(256) void zdig_kernel(ZdigJob g) {
    const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row < g.rows) zdig_row(g, row, threadIdx.x & 63);
}

// Grouped: one wave per row over the rows of all jobs.
__global__ __launch_bounds__(256) void zdig_grouped_kernel(const ZdigJob* __restrict__ jobs, int njobs, long total) {
    const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= total) return;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].item0 <= row) lo = mid;
        else hi = mid - 1;
    }
    const ZdigJob g = jobs[lo];
    zdig_row(g, row - g.item0, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// Stage 2: Sigma^{(n)}[p,q] += sum_{x,P} L[P,x,p] Zt^{(n)}[x,q,P]
// TM x 64 upper tiles (TM = 64 or 128), 4 waves of TM/2 x 32, promotion to
// FP64 once per x.
// ---------------------------------------------------------------------------

// Upper tiles of a symmetric M x M result in (64 R)-row x 64-column tiles:
// row block bi keeps the column blocks bj >= R bi (those that reach the
// diagonal or lie right of it); TN = ceil(M / 64) column blocks.
__device__ inline void upper_tile_rect(int t, int TN, int& bi, int& bj, int R = 2) {
    int r = 0;
    while (t >= TN - R * r) { t -= TN - R * r; ++r; }
    bi = r;
    bj = R * r + t;
}

// One work group: a TM x 64 upper tile of Sigma^{(n)} (TM = 64: half the
// accumulators, two work groups per CU; 128 in grouped launches for large
// molecules) for one sector and one split of that sector's x range; 4 waves
// of TM/2 x 32; the pipeline stages are OPA + C_OPB bytes apart.  The (x, k-block)
// steps form one double-buffered LDS-DMA pipeline; the int32 digit-weight
// accumulators are promoted to FP64 with the row and column scales at the
// end of every x.
constexpr int C_OPA = ND * 128 * 64;  // bytes of the A (128-row) slab (32 KB)
constexpr int C_OPB = ND * 64 * 64;   // bytes of the B (64-row) slab (16 KB)
constexpr int C_BUF = C_OPA + C_OPB;

template <int TM>
__device__ __forceinline__ void contract_tile(const ContractArgs& g, int tile, int split, int zi, lds_t* lds) {
    static_assert(TM == 128 || TM == 64, "contraction tile height");
    constexpr int NI = TM / 32;          // 16-row blocks per wave
    constexpr int HA = TM / 64;          // 64-row halves of the A slab
    constexpr int OPA = ND * TM * 64;    // bytes of the A slab
    constexpr int BUF = OPA + C_OPB;     // bytes of one pipeline stage
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lr = lane & 15;
    const int lk = lane >> 4;
    const int n = zi % g.nt;
    const int sector = zi / g.nt;
    const int nxs = sector ? g.nxs[1] : g.nxs[0];
    const int xs0 = sector ? g.xs0[1] : g.xs0[0];
    if (nxs <= 0) return;
    int bi, bj;
    upper_tile_rect(tile, g.tilesN, bi, bj, HA);
    const int m0 = bi * TM, n0 = bj * 64;
    const int per = (nxs + g.nsplit - 1) / g.nsplit;
    const int xa = xs0 + split * per;
    const int xb = min(xs0 + nxs, xa + per);
    if (xa >= xb) return;
    const int M = g.nmo;
    const long M2 = (long)M * M;
    const long zrows = (long)g.nt * g.ncol;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * 32;

    // LDS-DMA staging as in stage 1: vector s of wave w fills slab rows
    // s * 64 + 16 w + (lane >> 2).  A slab (d, i): d = s / HA, i = 64 (s % HA)
    // + 16 w + (lane >> 2); B slab (d, i): d = s, i = 16 w + (lane >> 2).
    // Rows past nmo read clamped rows.
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int lrow = lane >> 2;
    const int gch = swz(lrow, lane & 3);
    unsigned offA[HA];
#pragma unroll
    for (int h = 0; h < HA; ++h) offA[h] = (unsigned)(min(m0 + h * 64 + wv * 16 + lrow, M - 1) * 64 + gch * 16);
    const unsigned offB = (unsigned)(min(n0 + wv * 16 + lrow, M - 1) * 64 + gch * 16);
    auto load = [&](int x, int kt, int buf) {
        lds_t* A = lds + buf * BUF + wv * 16 * 64;
        lds_t* B = A + OPA;
        const unsigned soA = (unsigned)x * M * 64u;
        const unsigned soB = (unsigned)((long)n * g.ncol + (long)(x - g.x0) * M) * 64u;
#pragma unroll
        for (int s = 0; s < ND * HA; ++s) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(g.Ld + (s / HA) * g.lplane + (long)kt * M2 * 64), (short)0, (int)(M2 * 64), 0x00020000);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(A + s * 64 * 64),
                                                     16, offA[s % HA], soA, 0, 0);
        }
#pragma unroll
        for (int s = 0; s < ND; ++s) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(g.Zd + s * g.zplane + (long)kt * zrows * 64), (short)0, (int)(zrows * 64), 0x00020000);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(B + s * 64 * 64),
                                                     16, offB, soB, 0, 0);
        }
    };

    double acc64[NI][2][4];
    i32x4 acc[MAXW + 1][NI][2];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int w = 0; w <= MAXW; ++w) acc[w][i][j] = (i32x4){0, 0, 0, 0};
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
        }
    const int* eZn = g.eZ + (long)n * g.ncol;
    const int nkt = g.Ap / MK;
    const int so = swz(lr, lk) * 16;

    load(xa, 0, 0);
    // x outer, k-blocks inner: the int32 accumulators are carried by the inner
    // loop only (they stay in accumulation registers) and promoted after it.
    // Each step first waits for its own slabs and the barrier, then refills
    // the other buffer, so that the refill overlaps the whole step.
    int it = 0;                    // global step: buffer parity
    for (int x = xa; x < xb; ++x) {
        // this x's row (p) and column (q) exponents, fetched before its k
        // loop so that the promotion after it waits on no memory
        int ep[NI][4], eq[2];
        {
            const long xl = x - g.x0;
#pragma unroll
            for (int j = 0; j < 2; ++j) eq[j] = eZn[xl * M + min(n0 + wn + j * 16 + lr, M - 1)];
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) ep[i][r] = g.eL[(long)x * M + min(m0 + wm + i * 16 + 4 * lk + r, M - 1)];
        }
        for (int kt = 0; kt < nkt; ++kt, ++it) {
            const int cur = it & 1;
            const bool wrap = kt + 1 == nkt;
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (!wrap || x + 1 < xb) load(wrap ? x + 1 : x, wrap ? 0 : kt + 1, cur ^ 1);
            const lds_t* A = lds + cur * BUF;
            const lds_t* B = A + OPA;
            i32x4 b[2][ND];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int d = 0; d < ND; ++d) b[j][d] = lds_b128(B + (d * 64 + wn + j * 16 + lr) * 64 + so);
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                i32x4 a[ND];
#pragma unroll
                for (int d = 0; d < ND; ++d) a[d] = lds_b128(A + (d * TM + wm + i * 16 + lr) * 64 + so);
#pragma unroll
                for (int w = 0; w <= MAXW; ++w)
#pragma unroll
                    for (int ii = 0; ii <= w; ++ii)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            if (ii < ND && w - ii < ND) acc[w][i][j] = mfma8(a[ii], b[j][w - ii], acc[w][i][j]);
            }
        }
        // end of this x: promote with the row (p) and column (q) scales
        // (rows and columns past nmo read a clamped exponent; their results
        // are never stored)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int i = 0; i < NI; ++i) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double z = 0.0;
#pragma unroll
                    for (int w = MAXW; w >= 0; --w) z += (double)acc[w][i][j][r] * wscale(w);
                    acc64[i][j][r] += ldexp(z, ep[i][r] + eq[j]);
                }
#pragma unroll
                for (int w = 0; w <= MAXW; ++w) acc[w][i][j] = (i32x4){0, 0, 0, 0};
            }
        }
    }
    double* dst = g.part + (((long)sector * g.nt + n) * g.nsplit_total + g.split_off + split) * M2;
    // read every old value before the first store (the stores could alias
    // the later loads as far as the compiler knows)
    double old[NI][2][4];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int col = min(n0 + wn + j * 16 + lr, M - 1);
                const int row = min(m0 + wm + i * 16 + 4 * lk + r, M - 1);
                old[i][j][r] = dst[(long)row * M + col];
            }
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            int col = n0 + wn + j * 16 + lr;
            if (col >= M) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = m0 + wm + i * 16 + 4 * lk + r;
                if (row >= M) continue;
                dst[(long)row * M + col] = old[i][j][r] + acc64[i][j][r];
            }
        }
    // the next item of a persistent work group refills buffer 0: every wave
    // has finished reading the slabs of this one
    __syncthreads();
}

// XCD-aware mapping of a 1D grid onto (tile, group): work group b runs on XCD
// b % 8, and all tiles of one group are placed on the same XCD, so the tiles
// that share a row block (A slabs) or a column block (B slabs) meet in that
// XCD's L2.  Returns false for the padding work groups of the last round.
__device__ __forceinline__ bool xcd_group_item(int tiles, int groups, int& tile, int& group) {
    const int b = blockIdx.x;
    const int xcd = b & 7, local = b >> 3;
    group = (local / tiles) * 8 + xcd;
    tile = local - (local / tiles) * tiles;
    return group < groups;
}

// One work group per (upper 64 x 64 tile, split, sector * nt + n); groups
// are (split, z).  64-row tiles keep half the accumulators of 128-row ones
// and need 64 KB of LDS, so that two work groups share a CU (one wave per
// SIMD left every stall of a 128-row tile exposed: 17.2 against 16.1 ms at
// nocc 100, nvir 400, naux 1500, N 11).
__global__ __launch_bounds__(256, 2) void contract_mixed_kernel(ContractArgs g, int tiles) {
    __shared__ __attribute__((aligned(16))) lds_t lds[2 * (ND * 64 * 64 + C_OPB)];
    int tile, grp;
    if (!xcd_group_item(tiles, g.nsplit * 2 * g.nt, tile, grp)) return;
    contract_tile<64>(g, tile, grp % g.nsplit, grp / g.nsplit, lds);
}

// Grouped, persistent, XCD-aware: the work items of a job, ordered (tile,
// n, split, sector) with the tile fastest, are cut into groups of 32
// consecutive items (consecutive n share the L-digit slabs of their x range),
// numbered job after job (item0 = a job's first group).  As in stage 1, XCD
// x takes the groups x, x + 8, ... and its work groups walk their items with
// stride W = gridDim / 8; contract_tile ends with a barrier, so no wave
// starts loading the next item while another still reads the slabs of the
// last one.
__global__ __launch_bounds__(256, 1) void contract_grouped_kernel(const ContractArgs* __restrict__ jobs, int njobs,
                                                                  long groups) {
    __shared__ __attribute__((aligned(16))) lds_t lds[2 * C_BUF];
    const int x = blockIdx.x & 7;
    const long W = gridDim.x >> 3;
    for (long k = blockIdx.x >> 3;; k += W) {
        const long grp = (k >> 5) * 8 + x;
        if (grp >= groups) break;
        const ContractArgs g = jobs[find_job(jobs, njobs, grp)];
        const long i = (grp - g.item0) * 32 + (k & 31);
        const int T = g.tiles;
        if (i >= (long)T * g.nt * g.nsplit * 2) continue;
        long r = i / T;
        const int n = (int)(r % g.nt);
        r /= g.nt;
        const int split = (int)(r % g.nsplit);
        const int sector = (int)(r / g.nsplit);
        if (g.tm == 64) contract_tile<64>(g, (int)(i % T), split, sector * g.nt + n, lds);
        else contract_tile<128>(g, (int)(i % T), split, sector * g.nt + n, lds);
    }
}

// The same when every job of the launch has 64-row tiles: 64 KB of LDS and
// two work groups per CU.
__global__ __launch_bounds__(256, 2) void contract_grouped64_kernel(const ContractArgs* __restrict__ jobs, int njobs,
                                                                  long groups) {
    __shared__ __attribute__((aligned(16))) lds_t lds[2 * (ND * 64 * 64 + C_OPB)];
    const int x = blockIdx.x & 7;
    const long W = gridDim.x >> 3;
    for (long k = blockIdx.x >> 3;; k += W) {
        const long grp = (k >> 5) * 8 + x;
        if (grp >= groups) break;
        const ContractArgs g = jobs[find_job(jobs, njobs, grp)];
        const long i = (grp - g.item0) * 32 + (k & 31);
        const int T = g.tiles;
        if (i >= (long)T * g.nt * g.nsplit * 2) continue;
        long r = i / T;
        const int n = (int)(r % g.nt);
        r /= g.nt;
        const int split = (int)(r % g.nsplit);
        const int sector = (int)(r / g.nsplit);
        contract_tile<64>(g, (int)(i % T), split, sector * g.nt + n, lds);
    }
}

// ---------------------------------------------------------------------------
// Digit GEMM: C[m][n] = sum_k A[m][k] B[n][k] with A, B given as k-blocked digit
// planes with one exponent per row (the digit format above).  Every split
// covers at most KEXACT k, so its int32 digit-weight sums are exact and are
// combined in FP64 once, in the epilogue.  128 x 64 tiles, 4 waves of 64 x 32,
// the same LDS-DMA pipeline as stage 2.  Epilogues: FP64 split partials (upper
// tiles only when sym) or Xout = Dv[n] * Xin + alpha * C (in place allowed).
// ---------------------------------------------------------------------------
struct DgemmArgs {
    const i8* A;
    long aplane;
    int arows;
    const int* eA;
    const i8* B;
    long bplane;
    int brows;
    const int* eB;
    int M, N, nkb;    // output rows / cols; k-blocks of 64
    int nsplit;       // splits of the k-block range (at most KEXACT / 64 k-blocks each)
    int sym, tilesN;  // upper tiles only (M == N); column tiles
    int eshift;       // extra power of two of the product
    double* part;     // [nsplit][M][N] (Xout == nullptr)
    double* Xout;
    const double* Xin;
    const double* Dv;
    double alpha;
    const double* Cs;  // per-column scale of the product in the Xout epilogue (nullptr: 1)
};

// W4: also keep the weight-4 products d2 x d2, d1 x d3 and d3 x d1 (a fifth
// accumulator).  In a Gram-type product (B = A or A o D) the diagonal d2 x d2
// terms are squares and accumulate coherently over k, and for rows with a wide
// dynamic range (most entries far below the row maximum, whose leading digit
// is then d1) d1 x d3 is the leading-times-last product of those entries:
// without them the moments carry ~1e-8 relative error, with them ~5e-10.
template <bool W4, int TM = 128>
__device__ __forceinline__ void dgemm_tile(const DgemmArgs& g, int tile, int split, lds_t* lds) {
    static_assert(TM == 128 || TM == 64, "digit GEMM tile height");
    constexpr int NW = W4 ? MAXW + 2 : MAXW + 1;
    constexpr int NI = TM / 32;          // 16-row blocks per wave
    constexpr int HA = TM / 64;          // 64-row halves of the A slab
    constexpr int OPA = ND * TM * 64;    // bytes of the A slab
    constexpr int BUF = OPA + C_OPB;     // bytes of one pipeline stage
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lr = lane & 15;
    const int lk = lane >> 4;
    int bi, bj;
    if (g.sym) upper_tile_rect(tile, g.tilesN, bi, bj, HA);
    else {
        bi = tile / g.tilesN;
        bj = tile - bi * g.tilesN;
    }
    const int m0 = bi * TM, n0 = bj * 64;
    const int per = (g.nkb + g.nsplit - 1) / g.nsplit;
    const int ka = split * per;
    const int kb_end = min(g.nkb, ka + per);
    const int total = kb_end - ka;
    const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * 32;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int lrow = lane >> 2;
    const int gch = swz(lrow, lane & 3);
    unsigned offA[HA];
#pragma unroll
    for (int h = 0; h < HA; ++h) offA[h] = (unsigned)(min(m0 + h * 64 + wv * 16 + lrow, g.M - 1) * 64 + gch * 16);
    const unsigned offB = (unsigned)(min(n0 + wv * 16 + lrow, g.N - 1) * 64 + gch * 16);
    auto load = [&](int kb, int buf) {
        lds_t* A = lds + buf * BUF + wv * 16 * 64;
        lds_t* B = A + OPA;
#pragma unroll
        for (int s = 0; s < ND * HA; ++s) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(g.A + (s / HA) * g.aplane + (long)kb * g.arows * 64), (short)0, g.arows * 64, 0x00020000);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(A + s * 64 * 64),
                                                     16, offA[s % HA], 0, 0, 0);
        }
#pragma unroll
        for (int s = 0; s < ND; ++s) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(g.B + s * g.bplane + (long)kb * g.brows * 64), (short)0, g.brows * 64, 0x00020000);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(B + s * 64 * 64),
                                                     16, offB, 0, 0, 0);
        }
    };
    i32x4 acc[NW][NI][2];
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[w][i][j] = (i32x4){0, 0, 0, 0};
    const int so = swz(lr, lk) * 16;
    if (total > 0) load(ka, 0);
    for (int it = 0; it < total; ++it) {
        const int cur = it & 1;
        // wait for this step's slabs; the refill of the other buffer then
        // overlaps the whole step
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (it + 1 < total) load(ka + it + 1, cur ^ 1);
        const lds_t* A = lds + cur * BUF;
        const lds_t* B = A + OPA;
        i32x4 b[2][ND];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int d = 0; d < ND; ++d) b[j][d] = lds_b128(B + (d * 64 + wn + j * 16 + lr) * 64 + so);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            i32x4 a[ND];
#pragma unroll
            for (int d = 0; d < ND; ++d) a[d] = lds_b128(A + (d * TM + wm + i * 16 + lr) * 64 + so);
#pragma unroll
            for (int w = 0; w <= MAXW; ++w)
#pragma unroll
                for (int ii = 0; ii <= w; ++ii)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        if (ii < ND && w - ii < ND) acc[w][i][j] = mfma8(a[ii], b[j][w - ii], acc[w][i][j]);
            if (W4)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[NW - 1][i][j] = mfma8(a[2], b[j][2], acc[NW - 1][i][j]);
                    acc[NW - 1][i][j] = mfma8(a[1], b[j][3], acc[NW - 1][i][j]);
                    acc[NW - 1][i][j] = mfma8(a[3], b[j][1], acc[NW - 1][i][j]);
                }
        }
    }
    // combine the weights and scale by 2^(e_row + e_col) once, then the
    // epilogue.  Every input of the epilogue is loaded before the first
    // store: the stores could alias those arrays as far as the compiler
    // knows, so interleaved loads would each wait for a memory round trip.
    int ec[2], er[NI][4];
    double dv[2], cs[2], xin[2][NI][4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = min(n0 + wn + j * 16 + lr, g.N - 1);
        ec[j] = g.eB[col];
        dv[j] = g.Xout ? g.Dv[col] : 0.0;
        cs[j] = g.Cs ? g.Cs[col] : 1.0;
    }
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) er[i][r] = g.eA[min(m0 + wm + i * 16 + 4 * lk + r, g.M - 1)];
    if (g.Xout) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = min(n0 + wn + j * 16 + lr, g.N - 1);
                    const int row = min(m0 + wm + i * 16 + 4 * lk + r, g.M - 1);
                    xin[j][i][r] = g.Xin[(long)row * g.N + col];
                }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = n0 + wn + j * 16 + lr;
        if (col >= g.N) continue;
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + 4 * lk + r;
                if (row >= g.M) continue;
                double z = 0.0;
#pragma unroll
                for (int w = NW - 1; w >= 0; --w) z += (double)acc[w][i][j][r] * wscale(w);
                const double c = ldexp(z, er[i][r] + ec[j] + g.eshift);
                const long o = (long)row * g.N + col;
                if (g.Xout) g.Xout[o] = dv[j] * xin[j][i][r] + g.alpha * (cs[j] * c);
                else g.part[(long)split * g.M * g.N + o] = c;
            }
    }
}

// Split products: a 2D grid (tile, split), spread over the XCDs.  The unsplit
// update: XCD groups of 8 column tiles x all row tiles, so the row tiles that
// share a column block of B meet in one L2.  64 x 64 tiles: 144-160 registers
// and 64 KB of LDS, so that two work groups share a CU (128 x 64 tiles held
// one wave per SIMD: 13.4 against 11.4 ms of digit GEMMs per TDA set at
// nocc 100, nvir 400, naux 1500, N 11).
template <bool W4>
__global__ __launch_bounds__(256, 2) void dgemm_mixed_kernel(DgemmArgs g, int gtiles, int groups) {
    __shared__ __attribute__((aligned(16))) lds_t lds[2 * (ND * 64 * 64 + C_OPB)];
    if (g.nsplit > 1 || g.sym) {
        dgemm_tile<W4, 64>(g, blockIdx.x, blockIdx.y, lds);
    } else {
        int t, grp;
        if (!xcd_group_item(gtiles, groups, t, grp)) return;
        const int rows = (g.M + 63) / 64;
        const int bi = t % rows, bj = grp * 8 + t / rows;
        if (bj >= g.tilesN) return;
        dgemm_tile<W4, 64>(g, bi * g.tilesN + bj, 0, lds);
    }
}

template <int NT>
void launch_fold_mixed(Handle* h, const FoldJob& g) {
    // every padded row P < Ap is written (zeros for P >= naux): stage 2 reads all Ap rows
    // groups of 4 P-blocks x 8 column tiles, 8 groups per round of the XCDs
    const long groups = (long)((g.nP + 3) / 4) * ((g.nC + 7) / 8);
    const long rounds = (groups + 7) / 8;
    hipLaunchKernelGGL((fold_mixed_kernel<NT>), dim3((unsigned)(rounds * 8 * 32)), dim3(256), 0, h->stream, g);
}

unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }

// Row exponents and k-blocked digit planes of X[rows][cols] (times cs), and
// with Yd set also those of X o D (D = d2[c], exponents e2; cs then unset):
// rows of 4096 or more columns by the exponent pass and the tiled digit pass,
// shorter rows by the one-block-per-row kernel.
void launch_digitise_rows(Handle* h, long rows, int cols, int kpad, const double* X, const double* cs, int* e,
                          i8* Xd, const double* d2 = nullptr, int* e2 = nullptr, i8* Yd = nullptr) {
    if (cols < 4096 || rows > 65535) {
        hipLaunchKernelGGL(digitise_rows_kernel, dim3((unsigned)rows), dim3(256), 0, h->stream, rows, cols, kpad, X,
                           cs, e, Xd, d2, e2, Yd);
        return;
    }
    hipLaunchKernelGGL(fill_i32_kernel, dim3(nb256(rows)), dim3(256), 0, h->stream, e, rows, INT_MIN);
    if (Yd) hipLaunchKernelGGL(fill_i32_kernel, dim3(nb256(rows)), dim3(256), 0, h->stream, e2, rows, INT_MIN);
    hipLaunchKernelGGL(row_exp_kernel, dim3((unsigned)((cols + RCH - 1) / RCH), (unsigned)rows), dim3(256), 0,
                       h->stream, cols, X, cs, e, Yd ? d2 : nullptr, Yd ? e2 : nullptr);
    hipLaunchKernelGGL(row_digits_kernel, dim3((unsigned)((kpad + 127) / 128), (unsigned)((rows + 15) / 16)),
                       dim3(256), 0, h->stream, rows, cols, kpad, X, cs, e, Xd, Yd ? d2 : nullptr, Yd ? e2 : nullptr,
                       Yd);
}

// The digit pass of launch_digitise_rows alone, for rows of 4096 or more
// columns whose exponents (times cs) are already in e (preset INT_MIN, set by
// atomicMax).
void launch_row_digits(Handle* h, long rows, int cols, int kpad, const double* X, const double* cs, int* e, i8* Xd) {
    hipLaunchKernelGGL(row_digits_kernel, dim3((unsigned)((kpad + 127) / 128), (unsigned)((rows + 15) / 16)),
                       dim3(256), 0, h->stream, rows, cols, kpad, X, cs, e, Xd, (const double*)nullptr, (int*)nullptr,
                       (i8*)nullptr);
}

// Column exponents and transposed k-blocked digit planes of X[naux][ncol]
// (k = the row index, zero-padded to Ap): one read for Ap <= 2048, else the
// exponent pass followed by the LDS-transposing digit pass.
void launch_digitise_cols(Handle* h, int naux, long ncol, int Ap, const double* X, int* e, i8* Xd) {
    const dim3 g((unsigned)((ncol + 15) / 16)), b(512);
    if (Ap <= 512) hipLaunchKernelGGL(digits_cols_kernel<4>, g, b, 0, h->stream, naux, ncol, Ap, X, e, Xd);
    else if (Ap <= 1024) hipLaunchKernelGGL(digits_cols_kernel<8>, g, b, 0, h->stream, naux, ncol, Ap, X, e, Xd);
    else if (Ap <= 1536) hipLaunchKernelGGL(digits_cols_kernel<12>, g, b, 0, h->stream, naux, ncol, Ap, X, e, Xd);
    else if (Ap <= 2048) hipLaunchKernelGGL(digits_cols_kernel<16>, g, b, 0, h->stream, naux, ncol, Ap, X, e, Xd);
    else {
        hipLaunchKernelGGL(col_exp_kernel, dim3(nb256(ncol)), dim3(256), 0, h->stream, naux, ncol, X, e);
        hipLaunchKernelGGL(digits_lt_kernel, dim3((unsigned)((ncol + 31) / 32), (unsigned)((Ap + 31) / 32)), dim3(256),
                           0, h->stream, naux, ncol, Ap, X, e, Xd);
    }
}

}  // namespace

gw_status sigma_from_R_mixed(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                             const double* L, const double* R, const gw_opts* opts, double* sigma_occ,
                             double* sigma_vir) {
    const int nmo = nocc + nvir;
    const int nt = nmom_max + 1;
    const long M2 = (long)nmo * nmo;
    const int Ap = (naux + MK - 1) / MK * MK;
    if (nt > 12) return set_err(h, GW_EINVAL, "mixed precision: nmom_max must be <= 11");
    if (Ap > 512 * ZPASS) return set_err(h, GW_EINVAL, "mixed precision: naux must be <= 4096");
    static_assert(512 * ZPASS <= KEXACT, "exact int32 digit sums over the aux index");
    if ((long)nt * naux * 64 >= (1L << 31) || M2 * 64 >= (1L << 31))
        return set_err(h, GW_EINVAL, "mixed precision: digit plane rows exceed 31-bit byte offsets");
    // --- operand digits
    const long lplane = M2 * Ap;
    const long rrows = (long)nt * naux;
    const long rplane = rrows * Ap;
    i8* Ld = (i8*)ws_get(h, WS_MIX0, sizeof(i8) * ND * lplane);
    int* eL = (int*)ws_get(h, WS_MIX1, sizeof(int) * (M2 + rrows));
    i8* Rd = (i8*)ws_get(h, WS_MIX2, sizeof(i8) * ND * rplane);
    if (!Ld || !eL || !Rd) return GW_ENOMEM;
    int* eR = eL + M2;
    GW_TRY(mixed_prep(h, naux, nmo, nt, L, R, Ld, eL, Rd, eR));
    // --- stage-1 intermediates for every (x, q) column (each symmetric pair is
    // formed once and written to both of its columns): FP32 + BF16 residual,
    // the ND int8 digit planes and one exponent per (n, x, q) row
    const long zrows = (long)nt * M2;
    const size_t zbytes = (size_t)zrows * Ap * (sizeof(float) + sizeof(u16) + ND * sizeof(i8)) + sizeof(int) * zrows;
    if (opts && opts->zchunk_bytes && zbytes > opts->zchunk_bytes)
        return set_err(h, GW_ENOMEM, "sigma (mixed): the folded intermediate needs " + std::to_string(zbytes) +
                                         " bytes, above the cap of " + std::to_string(opts->zchunk_bytes));
    // the stage-2 kernel addresses the digit plane rows with 31-bit byte offsets
    if (zrows * 64 >= (1L << 31)) return set_err(h, GW_EINVAL, "mixed precision: nt * nmo^2 rows exceed 31-bit offsets");
    float* Zt = (float*)ws_get(h, WS_MIX3, sizeof(float) * zrows * Ap);
    u16* Zl = (u16*)ws_get(h, WS_MIX5, sizeof(u16) * zrows * Ap);
    i8* Zd = (i8*)ws_get(h, WS_MIX6, sizeof(i8) * ND * zrows * Ap);
    int* eZ = (int*)ws_get(h, WS_MIX4, sizeof(int) * zrows);
    if (!Zt || !Zl || !Zd || !eZ) return GW_ENOMEM;
    // 64 x 64 upper tiles, two work groups per CU
    const int tiles = mixed_upper_tiles(nmo, 64);
    const int S = best_splits((long)tiles * nt * 2, naux * std::max(nocc, nvir), 2 * h->cus, 64);
    const long part_per_sector = (long)nt * S * M2;
    double* acc = (double*)ws_get(h, WS_SIGACC, sizeof(double) * 2 * part_per_sector);
    if (!acc) return GW_ENOMEM;
    GW_TRY(fill_f64(h, acc, (size_t)2 * part_per_sector, 0.0));
    {
        KTimer tm(h, "sigma_fold");
        const FoldJob fj = make_fold_job(nt, Rd, eR, Ld, eL, eps, naux, Ap, nmo, nocc, rplane, lplane, Zt, Zl);
        switch (nt) {
            case 2: launch_fold_mixed<2>(h, fj); break;
            case 4: launch_fold_mixed<4>(h, fj); break;
            case 6: launch_fold_mixed<6>(h, fj); break;
            case 8: launch_fold_mixed<8>(h, fj); break;
            case 10: launch_fold_mixed<10>(h, fj); break;
            case 12: launch_fold_mixed<12>(h, fj); break;
            default: return set_err(h, GW_EINVAL, "mixed precision: nmom_max+1 must be even and <= 12");
        }
        tm.stop();
        GW_CHECK_LAUNCH(h);
    }
    {
        KTimer tm(h, "mixed_zdig");
        const ZdigJob zj{zrows, Ap, Zt, Zl, eZ, Zd, 0};
        hipLaunchKernelGGL(zdig_kernel, dim3((unsigned)((zrows + 3) / 4)), dim3(256), 0, h->stream, zj);
        tm.stop();
        GW_CHECK_LAUNCH(h);
    }
    {
        ContractArgs a;
        a.Ld = Ld; a.lplane = lplane; a.eL = eL;
        a.Zd = Zd; a.zplane = zrows * Ap; a.eZ = eZ;
        a.nmo = nmo; a.Ap = Ap; a.naux = naux;
        a.x0 = 0;
        a.xs0[0] = 0; a.nxs[0] = nocc;
        a.xs0[1] = nocc; a.nxs[1] = nvir;
        a.nt = nt; a.nsplit = S; a.tilesN = (nmo + 63) / 64; a.tiles = tiles; a.ncol = M2; a.tm = 64;
        a.part = acc;
        a.nsplit_total = S; a.split_off = 0; a.item0 = 0;
        KTimer tm(h, "sigma_contract");
        const long rounds = ((long)S * 2 * nt + 7) / 8;
        hipLaunchKernelGGL(contract_mixed_kernel, dim3((unsigned)(rounds * 8 * tiles)), dim3(256), 0, h->stream, a,
                           tiles);
        tm.stop();
        GW_CHECK_LAUNCH(h);
    }
    GW_TRY(reduce_splits(h, acc, S, M2, nt, nmo, nmo, nmo, true, 1.0, 0.0, sigma_occ, M2, nmo));
    GW_TRY(reduce_splits(h, acc + part_per_sector, S, M2, nt, nmo, nmo, nmo, true, 1.0, 0.0, sigma_vir, M2, nmo));
    return GW_OK;
}

FoldJob make_fold_job(int nt, const i8* Rd, const int* eR, const i8* Ld, const int* eL, const double* eps, int naux,
                      int Ap, int nmo, int nocc, long rplane, long lplane, float* Zt, u16* Zl) {
    FoldJob g;
    g.Rd = Rd; g.eR = eR; g.Ld = Ld; g.eL = eL; g.eps = eps;
    g.naux = naux; g.Ap = Ap; g.nmo = nmo; g.nocc = nocc;
    g.ncol = (long)nmo * nmo; g.rplane = rplane; g.lplane = lplane;
    g.nb = (nmo + 7) / 8;
    g.nblk = g.nb * (g.nb + 1) / 2;
    g.Zt = Zt; g.Zl = Zl;
    g.item0 = 0;
    g.nP = Ap / 16;
    const int cg = fold_cols(nt) / 64;
    g.nC = (g.nblk + cg - 1) / cg;
    return g;
}

gw_status mixed_prep(Handle* h, int naux, int nmo, int nt, const double* L, const double* R, i8* Ld, int* eL,
                     i8* Rd, int* eR) {
    const long M2 = (long)nmo * nmo;
    const int Ap = mixed_Ap(naux);
    const long rrows = (long)nt * naux;
    KTimer tm(h, "mixed_prep");
    launch_digitise_cols(h, naux, M2, Ap, L, eL, Ld);
    launch_digitise_rows(h, rrows, naux, Ap, R, nullptr, eR, Rd);
    tm.stop();
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status launch_fold_grouped(Handle* h, int nt, const FoldJob* jobs, int njobs, long total, int grid) {
    if (total <= 0) return GW_OK;
    // a whole number of work groups per XCD
    const dim3 g((unsigned)std::max(8, grid / 8 * 8));
    switch (nt) {
        case 2: hipLaunchKernelGGL((fold_grouped_kernel<2>), g, dim3(256), 0, h->stream, jobs, njobs, total); break;
        case 4: hipLaunchKernelGGL((fold_grouped_kernel<4>), g, dim3(256), 0, h->stream, jobs, njobs, total); break;
        case 6: hipLaunchKernelGGL((fold_grouped_kernel<6>), g, dim3(256), 0, h->stream, jobs, njobs, total); break;
        case 8: hipLaunchKernelGGL((fold_grouped_kernel<8>), g, dim3(256), 0, h->stream, jobs, njobs, total); break;
        case 10: hipLaunchKernelGGL((fold_grouped_kernel<10>), g, dim3(256), 0, h->stream, jobs, njobs, total); break;
        case 12: hipLaunchKernelGGL((fold_grouped_kernel<12>), g, dim3(256), 0, h->stream, jobs, njobs, total); break;
        default: return set_err(h, GW_EINVAL, "mixed precision: nmom_max+1 must be even and <= 12");
    }
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status launch_zdig_grouped(Handle* h, const ZdigJob* jobs, int njobs, long total_rows) {
    if (total_rows <= 0) return GW_OK;
    hipLaunchKernelGGL(zdig_grouped_kernel, dim3((unsigned)((total_rows + 3) / 4)), dim3(256), 0, h->stream, jobs,
                       njobs, total_rows);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status launch_contract_grouped(Handle* h, const ContractArgs* jobs, int njobs, long total, int grid, bool all64) {
    if (total <= 0) return GW_OK;
    // a whole number of work groups per XCD (two per CU with 64-row tiles only)
    if (all64) {
        const dim3 g((unsigned)std::max(8, 2 * grid / 8 * 8));
        hipLaunchKernelGGL(contract_grouped64_kernel, g, dim3(256), 0, h->stream, jobs, njobs, total);
        GW_CHECK_LAUNCH(h);
        return GW_OK;
    }
    const dim3 g((unsigned)std::max(8, grid / 8 * 8));
    hipLaunchKernelGGL(contract_grouped_kernel, g, dim3(256), 0, h->stream, jobs, njobs, total);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

// ---------------------------------------------------------------------------
// TDA moments with digit GEMMs (half-order form, as in the FP64 path):
//   R_2k = X_k X_k^T,  R_2k+1 = X_k D X_k^T + 2 R_k R_k,  X_k+1 = D o X_k + 2 R_k V.
// X stays FP64; each product digitises its operands (X rows, (X o D) rows,
// R_k rows, V^T rows once) and combines its exact int32 digit sums in FP64.
// The symmetric products (X X^T, X D X^T, R_k R_k) keep the three weight-4
// digit products as well (thirteen).
// ---------------------------------------------------------------------------
namespace {

gw_status launch_dgemm(Handle* h, const DgemmArgs& g0, const char* tag) {
    // 64 x 64 tiles, two work groups per CU
    constexpr int TM = 64;
    DgemmArgs g = g0;
    const int T = (g.M + TM - 1) / TM;
    g.tilesN = (g.N + 63) / 64;
    const long tiles = g.sym ? (long)mixed_upper_tiles(g.M, TM) : (long)T * g.tilesN;
    int gtiles = 0, groups = 0;
    dim3 grid((unsigned)tiles, (unsigned)g.nsplit);
    if (!(g.sym || g.nsplit > 1)) {
        gtiles = T * 8;
        groups = (g.tilesN + 7) / 8;
        grid = dim3((unsigned)((groups + 7) / 8 * 8 * gtiles));
    }
    KTimer tm(h, tag);
    if (g.sym) hipLaunchKernelGGL(dgemm_mixed_kernel<true>, grid, dim3(256), 0, h->stream, g, gtiles, groups);
    else hipLaunchKernelGGL(dgemm_mixed_kernel<false>, grid, dim3(256), 0, h->stream, g, gtiles, groups);
    tm.stop();
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

// digit planes (rows x kpad, k-blocked) of X[rows][cols], and with Yd set also
// those of X o D (D = d2[c])
gw_status digitise_rows(Handle* h, long rows, long cols, int kpad, const double* X, int* e, i8* Xd,
                        const double* d2 = nullptr, int* e2 = nullptr, i8* Yd = nullptr) {
    launch_digitise_rows(h, rows, (int)cols, kpad, X, nullptr, e, Xd, d2, e2, Yd);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

// RPA recursion operands: X1 = V o D (the odd chain's start) and D2 = D o D.
__global__ void rpa_prep_kernel(long rows, long ov, const double* __restrict__ V, const double* __restrict__ D,
                                double* __restrict__ X1, double* __restrict__ D2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * ov) return;
    const double d = D[i % ov];
    X1[i] = V[i] * d;
    if (i < ov) D2[i] = d * d;
}

}  // namespace

gw_status tda_moments_mixed(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps, const double* L,
                            double* R) {
    const long ov = (long)nocc * nvir;
    const int Kp = (int)((ov + MK - 1) / MK * MK);
    const int Ap = mixed_Ap(naux);
    if (ov * 64 >= (1L << 31) || (long)naux * 64 >= (1L << 31))
        return set_err(h, GW_EINVAL, "mixed precision: nocc*nvir too large for the digit recursion");
    if (Ap > KEXACT) return set_err(h, GW_EINVAL, "mixed precision: naux must be <= 32768 for the digit recursion");
    const long asz = (long)naux * naux;
    double* V = (double*)ws_get(h, WS_V, sizeof(double) * naux * ov);
    double* D = (double*)ws_get(h, WS_D, sizeof(double) * ov);
    double* X = (double*)ws_get(h, WS_X0, sizeof(double) * naux * ov);
    i8* Vt = (i8*)ws_get(h, WS_RC0, sizeof(i8) * ND * ov * Ap);
    i8* Xd = (i8*)ws_get(h, WS_RC1, sizeof(i8) * ND * (long)naux * Kp);
    i8* Yd = (i8*)ws_get(h, WS_RC2, sizeof(i8) * ND * (long)naux * Kp);
    i8* Rk = (i8*)ws_get(h, WS_RC3, sizeof(i8) * ND * (long)naux * Ap);
    int* ex = (int*)ws_get(h, WS_RC4, sizeof(int) * (ov + 3L * naux));
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device);
    const int tiles = mixed_upper_tiles(naux);
    const int nkbX = Kp / MK;
    // enough splits to fill the chip, and at most KEXACT k per split (exact int32 sums)
    const int S = std::max((nkbX + KEXACT / MK - 1) / (KEXACT / MK),
                           std::max(1, std::min(nkbX, (3 * ncu + tiles - 1) / tiles)));
    const int nkbR = Ap / MK;                         // k blocks of the R_k R_k product (Ap <= KEXACT)
    const int S2 = std::max(1, std::min(nkbR, (3 * ncu + tiles - 1) / tiles));
    double* part = (double*)ws_get(h, WS_RC5, sizeof(double) * (S + S2) * asz);
    if (!V || !D || !X || !Vt || !Xd || !Yd || !Rk || !ex || !part) return GW_ENOMEM;
    int *eVt = ex, *eX = ex + ov, *eY = eX + naux, *eR = eY + naux;
    GW_TRY(gather_ov(h, nocc, nvir, naux, eps, L, V, D));
    {
        KTimer tm(h, "recur_digits");
        launch_digitise_cols(h, naux, ov, Ap, V, eVt, Vt);
        tm.stop();
        GW_CHECK_LAUNCH(h);
    }
    GW_TRY(copy_f64(h, X, V, (size_t)naux * ov));
    DgemmArgs sy{};
    sy.M = sy.N = naux;
    sy.nkb = nkbX;
    sy.nsplit = S;
    sy.sym = 1;
    sy.part = part;
    sy.A = Xd; sy.aplane = (long)naux * Kp; sy.arows = naux; sy.eA = eX;
    const int K = nmom_max / 2;
    for (int k = 0; k <= K; ++k) {
        const bool odd = 2 * k + 1 <= nmom_max;
        {
            KTimer tm(h, "recur_digits");
            // X and, for the odd moment, X o D in one pass
            if (odd) GW_TRY(digitise_rows(h, naux, ov, Kp, X, eX, Xd, D, eY, Yd));
            else GW_TRY(digitise_rows(h, naux, ov, Kp, X, eX, Xd));
            tm.stop();
        }
        {
            DgemmArgs g = sy;
            g.B = Xd; g.bplane = (long)naux * Kp; g.brows = naux; g.eB = eX;
            GW_TRY(launch_dgemm(h, g, "recur_xvt"));
            GW_TRY(reduce_splits(h, part, S, asz, 1, naux, naux, naux, true, 1.0, 0.0, R + 2 * k * asz, asz, naux));
        }
        if (odd || k < K) {
            // digits of R_k (complete: k <= 2k), for R_k R_k and the X update
            KTimer tm(h, "recur_digits");
            GW_TRY(digitise_rows(h, naux, naux, Ap, R + k * asz, eR, Rk));
            tm.stop();
        }
        if (odd) {
            // R_2k+1 = X_k D X_k^T + 2 R_k R_k: both symmetric digit products
            // into one set of split partials (the factor 2 as a power of two)
            DgemmArgs g = sy;
            g.B = Yd; g.bplane = (long)naux * Kp; g.brows = naux; g.eB = eY;
            GW_TRY(launch_dgemm(h, g, "recur_xvt"));
            DgemmArgs r = sy;
            r.A = Rk; r.aplane = (long)naux * Ap; r.arows = naux; r.eA = eR;
            r.B = Rk; r.bplane = (long)naux * Ap; r.brows = naux; r.eB = eR;
            r.nkb = nkbR; r.nsplit = S2; r.eshift = 1;
            r.part = part + (long)S * asz;
            GW_TRY(launch_dgemm(h, r, "recur_rr"));
            GW_TRY(reduce_splits(h, part, S + S2, asz, 1, naux, naux, naux, true, 1.0, 0.0, R + (2 * k + 1) * asz,
                                 asz, naux));
        }
        if (k < K) {
            DgemmArgs g{};
            g.A = Rk; g.aplane = (long)naux * Ap; g.arows = naux; g.eA = eR;
            g.B = Vt; g.bplane = ov * Ap; g.brows = (int)ov; g.eB = eVt;
            g.M = naux; g.N = (int)ov; g.nkb = Ap / MK; g.nsplit = 1; g.sym = 0;
            g.Xout = X; g.Xin = X; g.Dv = D; g.alpha = 2.0;
            GW_TRY(launch_dgemm(h, g, "recur_rv"));
        }
    }
    return GW_OK;
}

// RPA (Sec. 2.2): eta~^{(0)} by the FP64 quadrature, eta~^{(1)} = V o D, then on
// the even and odd chains R_n = eta~^{(n)} V^T and
//   eta~^{(n+2)} = D^2 o eta~^{(n)} + 4 R_n (V o D),
// both products as int8 digit GEMMs: R_n on the upper tiles (thirteen digit
// products, mirrored, as the FP64 form), the update with the row digits of R_n
// against the digits of V o D transposed (k = P) and the D^2 / 4 epilogue.
gw_status node_products_mixed(Handle* h, int naux, long ov, int nb, const double* V, const double* as,
                              double* Q) {
    if (naux <= 0 || nb <= 0) return GW_OK;
    const int Kp = (int)((ov + MK - 1) / MK * MK);
    if (ov * 64 >= (1L << 31) || (long)naux * 64 >= (1L << 31))
        return set_err(h, GW_EINVAL, "mixed precision: RPA quadrature too large for the digit node products");
    const long n2 = (long)naux * naux;
    i8* Vd = (i8*)ws_get(h, WS_RPA_AD, sizeof(i8) * 2 * ND * (long)naux * Kp);
    int* ex = (int*)ws_get(h, WS_RPA_EX, sizeof(int) * (ov + 2L * naux + (long)nb * naux));
    if (!Vd || !ex) return GW_ENOMEM;
    i8* Ad = Vd + ND * (long)naux * Kp;
    int* eV = ex;
    int* eA = ex + naux;
    int* eN = ex + 2L * naux;  // [nb][naux] exponents of V o as_b
    // long rows: every node's row exponents in one pass over V, then only the
    // digit pass per node
    const bool all_exps = ov >= 4096 && naux <= 65535 * 16;
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device);
    const int tiles = mixed_upper_tiles(naux);
    const int nkb = Kp / MK;
    const int S = std::max((nkb + KEXACT / MK - 1) / (KEXACT / MK),
                           std::max(1, std::min(nkb, (3 * ncu + tiles - 1) / tiles)));
    double* part = (double*)ws_get(h, WS_RPA_QP, sizeof(double) * S * n2);
    if (!part) return GW_ENOMEM;
    KTimer tm(h, "rpa_quad");
    GW_TRY(digitise_rows(h, naux, ov, Kp, V, eV, Vd));
    if (all_exps) {
        hipLaunchKernelGGL(fill_i32_kernel, dim3(nb256((long)nb * naux)), dim3(256), 0, h->stream, eN,
                           (long)nb * naux, INT_MIN);
        hipLaunchKernelGGL(node_row_exp_kernel, dim3((unsigned)((ov + 511) / 512), (unsigned)((naux + 15) / 16)),
                           dim3(256), 0, h->stream, naux, (int)ov, V, as, nb, eN);
        GW_CHECK_LAUNCH(h);
    }
    for (int b = 0; b < nb; ++b) {
        // digits of V o as[b] by rows (k = ia)
        if (all_exps) {
            eA = eN + (long)b * naux;
            launch_row_digits(h, naux, (int)ov, Kp, V, as + (long)b * ov, eA, Ad);
        } else {
            launch_digitise_rows(h, naux, (int)ov, Kp, V, as + (long)b * ov, eA, Ad);
        }
        GW_CHECK_LAUNCH(h);
        DgemmArgs g{};
        g.M = g.N = naux;
        g.nkb = nkb;
        g.nsplit = S;
        g.sym = 1;
        g.part = part;
        g.A = Ad; g.aplane = (long)naux * Kp; g.arows = naux; g.eA = eA;
        g.B = Vd; g.bplane = (long)naux * Kp; g.brows = naux; g.eB = eV;
        GW_TRY(launch_dgemm(h, g, nullptr));
        GW_TRY(reduce_splits(h, part, S, n2, 1, naux, naux, naux, true, 1.0, 0.0, Q + b * n2, n2, naux));
    }
    tm.stop();
    return GW_OK;
}

gw_status node_sum_mixed(Handle* h, int naux, long ov, int nb, const double* S, const double* V,
                         const double* gtab, const double* d0, double* G) {
    if (naux <= 0 || ov <= 0 || nb <= 0) return GW_OK;
    const int Ap = mixed_Ap(naux);
    if (ov * 64 >= (1L << 31) || Ap > KEXACT)
        return set_err(h, GW_EINVAL, "mixed precision: RPA quadrature too large for the digit node sum");
    const long n2 = (long)naux * naux;
    i8* Vlt = (i8*)ws_get(h, WS_RPA_VLT, sizeof(i8) * ND * ov * Ap);
    i8* Sd = (i8*)ws_get(h, WS_RPA_SD, sizeof(i8) * ND * (long)naux * Ap + sizeof(double) * (ov + 1));
    int* ex = (int*)ws_get(h, WS_RPA_EX, sizeof(int) * (ov + naux));
    if (!Vlt || !Sd || !ex) return GW_ENOMEM;
    double* ones = (double*)(Sd + ND * (long)naux * Ap);
    int* eV = ex;
    int* eS = ex + ov;
    KTimer tm(h, "rpa_quad");
    // B operand: V's digit planes transposed (k = Q, one scale per column ia)
    launch_digitise_cols(h, naux, ov, Ap, V, eV, Vlt);
    GW_CHECK_LAUNCH(h);
    GW_TRY(fill_f64(h, ones, (size_t)ov, 1.0));
    for (int b = 0; b < nb; ++b) {
        GW_TRY(digitise_rows(h, naux, naux, Ap, S + b * n2, eS, Sd));
        DgemmArgs u{};
        u.A = Sd; u.aplane = (long)naux * Ap; u.arows = naux; u.eA = eS;
        u.B = Vlt; u.bplane = ov * Ap; u.brows = (int)ov; u.eB = eV;
        u.M = naux; u.N = (int)ov; u.nkb = Ap / MK; u.nsplit = 1; u.sym = 0;
        // G = V o d0 + g_0 o (S_0 V), then G += g_b o (S_b V)
        u.Xout = G; u.Xin = b == 0 ? V : G; u.Dv = b == 0 ? d0 : ones;
        u.alpha = 1.0; u.Cs = gtab + (long)b * ov;
        GW_TRY(launch_dgemm(h, u, nullptr));
    }
    tm.stop();
    return GW_OK;
}

gw_status rpa_moments_mixed(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                            const double* L, const gw_opts* opts, double* R) {
    const long ov = (long)nocc * nvir;
    const int Kp = (int)((ov + MK - 1) / MK * MK);
    const int Ap = mixed_Ap(naux);
    if (ov * 64 >= (1L << 31) || (long)naux * 64 >= (1L << 31))
        return set_err(h, GW_EINVAL, "mixed precision: nocc*nvir too large for the digit recursion");
    if (Ap > KEXACT) return set_err(h, GW_EINVAL, "mixed precision: naux must be <= 32768 for the digit recursion");
    const long asz = (long)naux * naux;
    const long xsz = (long)naux * ov;
    double* V = (double*)ws_get(h, WS_V, sizeof(double) * xsz);
    double* D = (double*)ws_get(h, WS_D, sizeof(double) * ov);
    double* X[2] = {(double*)ws_get(h, WS_X0, sizeof(double) * xsz), (double*)ws_get(h, WS_X1, sizeof(double) * xsz)};
    i8* VDt = (i8*)ws_get(h, WS_RC0, sizeof(i8) * ND * ov * Ap);
    i8* Xd = (i8*)ws_get(h, WS_RC1, sizeof(i8) * ND * (long)naux * Kp);
    i8* Vd = (i8*)ws_get(h, WS_RC2, sizeof(i8) * ND * (long)naux * Kp);
    i8* Rk = (i8*)ws_get(h, WS_RC3, sizeof(i8) * ND * (long)naux * Ap);
    int* ex = (int*)ws_get(h, WS_RC4, sizeof(int) * (ov + 3L * naux));
    double* D2 = (double*)ws_get(h, WS_MISC, sizeof(double) * (ov + 16));
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device);
    const int tiles = mixed_upper_tiles(naux);
    const int nkbX = Kp / MK;
    const int S = std::max((nkbX + KEXACT / MK - 1) / (KEXACT / MK),
                           std::max(1, std::min(nkbX, (3 * ncu + tiles - 1) / tiles)));
    double* part = (double*)ws_get(h, WS_RC5, sizeof(double) * S * asz);
    if (!V || !D || !X[0] || !X[1] || !VDt || !Xd || !Vd || !Rk || !ex || !D2 || !part) return GW_ENOMEM;
    int *eVDt = ex, *eX = ex + ov, *eV = eX + naux, *eR = eV + naux;
    GW_TRY(gather_ov(h, nocc, nvir, naux, eps, L, V, D));
    GW_TRY(rpa_eta0(h, nocc, nvir, naux, eps, V, D, opts, X[0], true));
    hipLaunchKernelGGL(rpa_prep_kernel, dim3(nb256(xsz)), dim3(256), 0, h->stream, (long)naux, ov, V, D, X[1], D2);
    GW_CHECK_LAUNCH(h);
    {
        KTimer tm(h, "recur_digits");
        // the update's B operand: V o D, transposed digit planes (k = P, per-column scales)
        launch_digitise_cols(h, naux, ov, Ap, X[1], eVDt, VDt);
        GW_CHECK_LAUNCH(h);
        // the B operand of R_n = eta~^{(n)} V^T: row digit planes of V (k = ia)
        GW_TRY(digitise_rows(h, naux, ov, Kp, V, eV, Vd));
        tm.stop();
    }
    for (int n = 0; n <= nmom_max; ++n) {
        double* Xn = X[n & 1];
        {
            KTimer tm(h, "recur_digits");
            GW_TRY(digitise_rows(h, naux, ov, Kp, Xn, eX, Xd));
            tm.stop();
        }
        DgemmArgs g{};
        g.M = g.N = naux;
        g.nkb = nkbX;
        g.nsplit = S;
        g.sym = 1;
        g.part = part;
        g.A = Xd; g.aplane = (long)naux * Kp; g.arows = naux; g.eA = eX;
        g.B = Vd; g.bplane = (long)naux * Kp; g.brows = naux; g.eB = eV;
        GW_TRY(launch_dgemm(h, g, "recur_xvt"));
        GW_TRY(reduce_splits(h, part, S, asz, 1, naux, naux, naux, true, 1.0, 0.0, R + n * asz, asz, naux));
        if (n + 2 <= nmom_max) {
            {
                KTimer tm(h, "recur_digits");
                GW_TRY(digitise_rows(h, naux, naux, Ap, R + n * asz, eR, Rk));
                tm.stop();
            }
            DgemmArgs u{};
            u.A = Rk; u.aplane = (long)naux * Ap; u.arows = naux; u.eA = eR;
            u.B = VDt; u.bplane = ov * Ap; u.brows = (int)ov; u.eB = eVDt;
            u.M = naux; u.N = (int)ov; u.nkb = Ap / MK; u.nsplit = 1; u.sym = 0;
            u.Xout = Xn; u.Xin = Xn; u.Dv = D2; u.alpha = 4.0;
            GW_TRY(launch_dgemm(h, u, "recur_rv"));
        }
    }
    return GW_OK;
}

}  // namespace gwm
