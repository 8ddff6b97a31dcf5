// FP64 MFMA GEMM for gfx950 (v_mfma_f64_16x16x4_f64), used by every dense
// contraction of the FP64 path: R_n = eta~ V^T, the recursion updates
// D o X + c R V (Secs. 2.2-2.3), the RPA quadrature products and the
// self-energy contraction over (P, x) (eq. w_moments, eqs. convolution_*).
//
// Tile: 128 x 128 output per 256-thread workgroup (4 wave64s, 64 x 64 each,
// 4 x 4 MFMA blocks of 16 x 16), K staged 16 at a time through a double-
// buffered LDS tile with register prefetch of the next K slab.
#include "internal.h"

#include <algorithm>

namespace gwm {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int TBM = 128;
constexpr int TBN = 128;
constexpr int TBK = 16;
constexpr int TPAD = 2;
constexpr int NTHR = 256;
constexpr int GROUP_M = 8;  // grouped raster: 8 tile rows share one B column slab

__device__ inline void upper_tile(int t, int T, int& bi, int& bj) {
    int r = 0;
    while (t >= T - r) { t -= T - r; ++r; }
    bi = r;
    bj = r + t;
}

template <bool AKC, bool BKC>
__global__ __launch_bounds__(NTHR, 2) void gemm_f64_kernel(GemmF64 g, int tiles_m, int tiles_n) {
    __shared__ double As[2][TBK][TBM + TPAD];
    __shared__ double Bs[2][TBK][TBN + TPAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int split = blockIdx.y;
    const int batch = blockIdx.z;

    // --- tile coordinates (XCD-aware: consecutive logical tiles stay on one XCD)
    int bi, bj;
    {
        int nwg = gridDim.x;
        int bid = blockIdx.x;
        int logical = bid;
        if ((nwg & 7) == 0) logical = (bid & 7) * (nwg >> 3) + (bid >> 3);
        if (g.sym_upper) {
            upper_tile(logical, tiles_m, bi, bj);
        } else {
            int per_group = GROUP_M * tiles_n;
            int group = logical / per_group;
            int first_m = group * GROUP_M;
            int gsize = min(tiles_m - first_m, GROUP_M);
            int in = logical - group * per_group;
            bi = first_m + in % gsize;
            bj = in / gsize;
        }
    }
    const int m0 = bi * TBM;
    const int n0 = bj * TBN;
    const int kbeg = split * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);

    const double* Ab = g.A + (long)batch * g.a_bs;
    const double* Bb = g.B + (long)batch * g.b_bs;
    const double* asc = g.ascale ? g.ascale + (long)batch * g.ascale_bs : nullptr;

    double ra[8], rb[8];

    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int idx = e * NTHR + tid;
            if (AKC) {
                int kk = idx & (TBK - 1), mm = idx >> 4;
                int m = m0 + mm, k = k0 + kk;
                double v = 0.0;
                if (m < g.M && k < kend) {
                    v = Ab[(long)m * g.lda + k];
                    if (asc) v *= asc[k];
                }
                ra[e] = v;
            } else {
                int mm = idx & (TBM - 1), kk = idx >> 7;
                int m = m0 + mm, k = k0 + kk;
                double v = 0.0;
                if (m < g.M && k < kend) {
                    long base = g.a_off + (long)(k / g.a_kdiv) * g.a_khi + (long)(k % g.a_kdiv) * g.a_klo;
                    v = Ab[base + m];
                }
                ra[e] = v;
            }
            if (BKC) {
                int kk = idx & (TBK - 1), nn = idx >> 4;
                int n = n0 + nn, k = k0 + kk;
                double v = 0.0;
                if (n < g.N && k < kend) v = Bb[(long)n * g.ldb + k];
                rb[e] = v;
            } else {
                int nn = idx & (TBN - 1), kk = idx >> 7;
                int n = n0 + nn, k = k0 + kk;
                double v = 0.0;
                if (n < g.N && k < kend) {
                    long q = k / g.b_kdiv;
                    long base = g.b_off + q * g.b_khi + (long)(k % g.b_kdiv) * g.b_klo;
                    v = Bb[base + n];
                    if (g.bscale) v *= g.bscale[q * g.bscale_ld + n];
                }
                rb[e] = v;
            }
        }
    };
    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            int idx = e * NTHR + tid;
            if (AKC) As[buf][idx & (TBK - 1)][idx >> 4] = ra[e];
            else As[buf][idx >> 7][idx & (TBM - 1)] = ra[e];
            if (BKC) Bs[buf][idx & (TBK - 1)][idx >> 4] = rb[e];
            else Bs[buf][idx >> 7][idx & (TBN - 1)] = rb[e];
        }
    };

    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

    const int wm = (wave >> 1) * 64;
    const int wn = (wave & 1) * 64;
    const int lrow = lane & 15;
    const int lk = lane >> 4;

    int nkt = (kend > kbeg) ? (kend - kbeg + TBK - 1) / TBK : 0;
    if (nkt > 0) {
        load_tiles(kbeg);
        store_tiles(0);
        __syncthreads();
    }
    int cur = 0;
    for (int kt = 0; kt < nkt; ++kt) {
        bool more = (kt + 1) < nkt;
        if (more) load_tiles(kbeg + (kt + 1) * TBK);
#pragma unroll
        for (int k4 = 0; k4 < TBK / 4; ++k4) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[cur][k4 * 4 + lk][wm + i * 16 + lrow];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[cur][k4 * 4 + lk][wn + j * 16 + lrow];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) store_tiles(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }

    // --- epilogue: lane holds rows (lane>>4) + 4r, column lane&15 of each 16x16 block.
    // Per row block i, every value the epilogue reads is loaded before its
    // first store: the stores could alias those arrays as far as the
    // compiler knows, so interleaved loads would each wait for a round trip.
    const bool partial = g.epi == EPI_PARTIAL;
    const bool rd = partial ? g.accumulate : (g.X != nullptr);
    double dgc[4], csc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = min(n0 + wn + j * 16 + lrow, g.N - 1);
        dgc[j] = (!partial && g.X && g.dg) ? g.dg[col] : 1.0;
        csc[j] = (!partial && g.cs) ? g.cs[col] : 1.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double in[4][4];
        if (rd) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = min(n0 + wn + j * 16 + lrow, g.N - 1);
                    const int row = min(m0 + wm + i * 16 + lk + 4 * r, g.M - 1);
                    in[j][r] = partial ? g.C[((long)batch * g.nsplit + split) * g.c_ps + (long)row * g.ldc + col]
                                       : g.X[(long)batch * g.x_bs + (long)row * g.ldx + col];
                }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int col = n0 + wn + j * 16 + lrow;
            if (col >= g.N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = m0 + wm + i * 16 + lk + 4 * r;
                if (row >= g.M) continue;
                double v = acc[i][j][r];
                if (partial) {
                    double* dst = g.C + ((long)batch * g.nsplit + split) * g.c_ps + (long)row * g.ldc + col;
                    *dst = rd ? in[j][r] + v : v;
                } else {
                    v *= g.alpha;
                    if (rd) v += in[j][r] * dgc[j];
                    g.C[(long)batch * g.c_bs + (long)row * g.ldc + col] = v * csc[j];
                }
            }
        }
    }
}

__global__ void reduce_splits_kernel(const double* part, int nsplit, long ps, int M, int N, long ld,
                                     int mirror, double alpha, double diag, double* out,
                                     long out_bs, long ldo) {
    const int b = blockIdx.z;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)M * N) return;
    int m = (int)(i / N), n = (int)(i % N);
    int mm = m, nn = n;
    if (mirror && m > n) { mm = n; nn = m; }
    const double* p = part + (long)b * nsplit * ps + (long)mm * ld + nn;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += p[(long)k * ps];
    s *= alpha;
    if (m == n) s += diag;
    out[(long)b * out_bs + (long)m * ldo + n] = s;
}

}  // namespace

void plan_split(GemmF64& g, int target_wg) {
    int tm = (g.M + TBM - 1) / TBM, tn = (g.N + TBN - 1) / TBN;
    long tiles = g.sym_upper ? (long)tm * (tm + 1) / 2 : (long)tm * tn;
    tiles *= g.batch;
    int ns = (int)std::max<long>(1, (target_wg + tiles - 1) / tiles);
    int max_ns = std::max(1, g.K / (4 * TBK));
    ns = std::min(ns, max_ns);
    int chunk = (g.K + ns - 1) / ns;
    chunk = (chunk + TBK - 1) / TBK * TBK;
    ns = (g.K + chunk - 1) / chunk;
    g.nsplit = std::max(ns, 1);
    g.kchunk = std::max(chunk, TBK);
}

void limit_split(GemmF64& g, size_t max_doubles) {
    const size_t per = (size_t)std::max(g.batch, 1) * (size_t)std::max<long>(g.c_ps, 1);
    if ((size_t)g.nsplit * per <= max_doubles) return;
    int ns = (int)std::max<size_t>(1, max_doubles / per);
    int chunk = (g.K + ns - 1) / ns;
    chunk = (chunk + TBK - 1) / TBK * TBK;
    g.kchunk = std::max(chunk, TBK);
    g.nsplit = std::max(1, (g.K + g.kchunk - 1) / g.kchunk);
}

gw_status gemm_f64(Handle* h, const GemmF64& g0) {
    GemmF64 g = g0;
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return GW_OK;
    if (g.kchunk <= 0) { g.nsplit = 1; g.kchunk = std::max(g.K, 1); }
    if (g.sym_upper && g.M != g.N) return set_err(h, GW_EINVAL, "gemm_f64: sym_upper needs M == N");
    if (g.nsplit > 1 && g.epi != EPI_PARTIAL)
        return set_err(h, GW_EINVAL, "gemm_f64: split-K needs the partial epilogue");
    int tm = (g.M + TBM - 1) / TBM, tn = (g.N + TBN - 1) / TBN;
    long tiles = g.sym_upper ? (long)tm * (tm + 1) / 2 : (long)tm * tn;
    if (tiles > 0x7fffffffL || g.nsplit > 65535 || g.batch > 65535)
        return set_err(h, GW_EINVAL, "gemm_f64: grid too large");
    dim3 grid((unsigned)tiles, (unsigned)g.nsplit, (unsigned)g.batch);
    KTimer timer(h, g.tag);
    if (g.a_kc && g.b_kc)
        hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, dim3(NTHR), 0, h->stream, g, tm, tn);
    else if (g.a_kc && !g.b_kc)
        hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, dim3(NTHR), 0, h->stream, g, tm, tn);
    else if (!g.a_kc && g.b_kc)
        hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, dim3(NTHR), 0, h->stream, g, tm, tn);
    else
        hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, dim3(NTHR), 0, h->stream, g, tm, tn);
    timer.stop();
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status reduce_splits(Handle* h, const double* part, int nsplit, long ps, int batch, int M, int N,
                        long ld, bool mirror, double alpha, double diag, double* out, long out_bs,
                        long ldo) {
    long n = (long)M * N;
    if (n == 0 || batch == 0) return GW_OK;
    dim3 grid((unsigned)((n + 255) / 256), 1, (unsigned)batch);
    hipLaunchKernelGGL(reduce_splits_kernel, grid, dim3(256), 0, h->stream, part, nsplit, ps, M, N, ld,
                       mirror ? 1 : 0, alpha, diag, out, out_bs, ldo);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

}  // namespace gwm
