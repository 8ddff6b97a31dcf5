// Self-energy moments from the aux-space cores R_t (FP64 path).
//
// eqs. convolution_occ / convolution_vir with eq. w_moments:
//   Sigma^{(n)}_pq = sum_x sum_{t<=n} s_{n,t}(x) sum_PQ L[P,p,x] R_t[P,Q] L[Q,q,x]
//   s_{n,t}(x) = 2 C(n,t) (-1)^t eps_x^{n-t}  (x occupied: hole moments)
//              = 2 C(n,t)        eps_x^{n-t}  (x virtual:  particle moments)
//
// Stage 1 (sigma_fold_kernel): Zt^{(n)}[P,x,q] = sum_t s_{n,t}(x) (R_t L)[P,x,q]
//   -- all t for one (P-block, pair-block) tile stay in registers, and the
//   binomial / eps-power fold happens in the epilogue, so the per-t products
//   never reach HBM.  L symmetric in (p,q) means L[Q,q,x] = L[Q,x,q], so the
//   column index j = x*nmo + q walks L's rows contiguously, and (R_t L) is
//   symmetric in (x, q): each pair x <= q is formed once and folded into
//   both of its columns (half the products of the full column range).
// Stage 2 (gemm_f64): Sigma^{(n)}[p,q] = sum_{P, x in sector} L[P,x,p] Zt^{(n)}[P,x,q],
//   upper 128x128 tiles only, split-K partials, then one reduction that
//   mirrors the upper triangle (exactly symmetric).
#include "internal.h"

#include <algorithm>

namespace gwm {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int FBP = 16;   // P rows per tile
constexpr int FBN = 64;   // columns per tile (4 waves x 16)
constexpr int FBK = 16;   // Q slab
constexpr int FTHR = 256;

constexpr double binom2(int n, int k) {
    // 2 * C(n, k), exact in double for n < 64
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (n - k + i) / i;
    return 2.0 * c;
}

// Pair blocks of stage 1: Z_t[P, x, q] = sum_Q R_t[P,Q] L[Q,x,q] is symmetric
// in (x, q) because L[Q] is, so only the pairs x <= q are formed, in 8 x 8
// blocks (X, Y) with X <= Y over nb = ceil(nmo / 8) blocks per side; column
// c of a block is x = 8X + (c >> 3), q = 8Y + (c & 7).  Diagonal blocks form
// all 64 pairs (and each writes only its own output), the others write the
// fold of each pair twice: with eps_x at (x, q) and with eps_q at (q, x).
__device__ __forceinline__ void pair_block(int t, int nb, int& X, int& Y) {
    int r = 0;
    while (t >= nb - r) { t -= nb - r; ++r; }
    X = r;
    Y = r + t;
}

template <int NT>
__global__ __launch_bounds__(FTHR, 2) void sigma_fold_kernel(const double* __restrict__ R,
                                                              const double* __restrict__ L,
                                                              const double* __restrict__ eps, int naux,
                                                              int nmo, int nocc, int nb,
                                                              double* __restrict__ Zt) {
    __shared__ double Ra[2][NT][FBK][FBP];
    __shared__ double Lb[2][FBK][FBN + 2];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int lrow = lane & 15;
    const int lk = lane >> 4;
    int BX, BY;
    pair_block(blockIdx.x, nb, BX, BY);
    const int P0 = blockIdx.y * FBP;
    const long nmo2 = (long)nmo * nmo;

    // the L column this thread loads: pair c = tid & 63 of the block
    const int cl = tid & 63;
    const int xl = 8 * BX + (cl >> 3), ql = 8 * BY + (cl & 7);
    const long jl = (xl < nmo && ql < nmo) ? (long)xl * nmo + ql : 0;

    double rr[NT];
    double rl[4];

    auto load = [&](int q0) {
        {
            int k = tid & 15, p = tid >> 4;
            int P = P0 + p, Q = q0 + k;
            bool ok = (P < naux) && (Q < naux);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                rr[t] = ok ? R[((long)t * naux + P) * naux + Q] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int k = e * 4 + (tid >> 6);
            int Q = q0 + k;
            rl[e] = Q < naux ? L[(long)Q * nmo2 + jl] : 0.0;
        }
    };
    auto store = [&](int buf) {
        int k = tid & 15, p = tid >> 4;
#pragma unroll
        for (int t = 0; t < NT; ++t) Ra[buf][t][k][p] = rr[t];
#pragma unroll
        for (int e = 0; e < 4; ++e) Lb[buf][e * 4 + (tid >> 6)][cl] = rl[e];
    };

    v4d acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};

    const int nkt = (naux + FBK - 1) / FBK;
    load(0);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int kt = 0; kt < nkt; ++kt) {
        bool more = kt + 1 < nkt;
        if (more) load((kt + 1) * FBK);
#pragma unroll
        for (int k4 = 0; k4 < FBK / 4; ++k4) {
            double b = Lb[cur][k4 * 4 + lk][wave * 16 + lrow];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                double a = Ra[cur][t][k4 * 4 + lk][lrow];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
        }
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }

    // epilogue: lane owns pair c and rows lk + 4r; binomial / eps-power fold
    // for each output of the pair
    const int c = wave * 16 + lrow;
    const int x = 8 * BX + (c >> 3), q = 8 * BY + (c & 7);
    if (x >= nmo || q >= nmo) return;
    const bool twin = BX < BY;   // also the transposed output (q, x)
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        if (o == 1 && !twin) break;
        const int xo = o ? q : x;            // the orbital whose energy folds this output
        const long col = o ? (long)q * nmo + x : (long)x * nmo + q;
        const double ex = eps[xo];
        const bool occ = xo < nocc;
        double pw[NT];
        pw[0] = 1.0;
#pragma unroll
        for (int k = 1; k < NT; ++k) pw[k] = pw[k - 1] * ex;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int P = P0 + lk + 4 * r;
            if (P >= naux) continue;
            double a[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) a[t] = (occ && (t & 1)) ? -acc[t][r] : acc[t][r];
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                double z = 0.0;
#pragma unroll
                for (int t = 0; t <= n; ++t) z += binom2(n, t) * pw[n - t] * a[t];
                Zt[((long)n * naux + P) * nmo2 + col] = z;
            }
        }
    }
}

template <int NT>
void launch_fold(Handle* h, int naux, int nmo, int nocc, const double* eps, const double* R,
                 const double* L, double* Zt) {
    const int nb = (nmo + 7) / 8;
    dim3 grid((unsigned)(nb * (nb + 1) / 2), (unsigned)((naux + FBP - 1) / FBP));
    hipLaunchKernelGGL((sigma_fold_kernel<NT>), grid, dim3(FTHR), 0, h->stream, R, L, eps, naux, nmo,
                       nocc, nb, Zt);
}

}  // namespace

gw_status sigma_fold_f64(Handle* h, int nt, int naux, int nmo, int nocc, const double* eps,
                         const double* R, const double* L, double* Zt) {
    const long nb = (nmo + 7) / 8;
    if (nb * (nb + 1) / 2 > 0x7fffffffL || (naux + FBP - 1) / FBP > 65535)
        return set_err(h, GW_EINVAL, "sigma_fold: grid too large");
    KTimer timer(h, "sigma_fold");
    switch (nt) {
        case 2: launch_fold<2>(h, naux, nmo, nocc, eps, R, L, Zt); break;
        case 4: launch_fold<4>(h, naux, nmo, nocc, eps, R, L, Zt); break;
        case 6: launch_fold<6>(h, naux, nmo, nocc, eps, R, L, Zt); break;
        case 8: launch_fold<8>(h, naux, nmo, nocc, eps, R, L, Zt); break;
        case 10: launch_fold<10>(h, naux, nmo, nocc, eps, R, L, Zt); break;
        case 12: launch_fold<12>(h, naux, nmo, nocc, eps, R, L, Zt); break;
        case 14: launch_fold<14>(h, naux, nmo, nocc, eps, R, L, Zt); break;
        case 16: launch_fold<16>(h, naux, nmo, nocc, eps, R, L, Zt); break;
        default: return set_err(h, GW_EINVAL, "sigma_fold: nmom_max+1 must be even and <= 16");
    }
    timer.stop();
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

gw_status sigma_from_R_f64_bufs(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                                const double* L, const double* R, size_t zcap_bytes, const Scratch& zt,
                                const Scratch& accs, double* sigma_occ, double* sigma_vir) {
    const int nmo = nocc + nvir;
    const int nt = nmom_max + 1;
    const long nmo2 = (long)nmo * nmo;
    // the folded intermediate of every (x, q) is formed at once (stage 1 writes
    // each symmetric pair to both of its columns)
    const size_t zn = (size_t)nt * naux * nmo2;
    if (zn * sizeof(double) > zcap_bytes)
        return set_err(h, GW_ENOMEM, "sigma (FP64): the folded intermediate needs " +
                                         std::to_string(zn * sizeof(double)) + " bytes, above the cap of " +
                                         std::to_string(zcap_bytes));
    double* Zt = scratch_get(h, zt, zn);
    if (!Zt) return GW_ENOMEM;

    const int T = (nmo + 127) / 128;
    const int tiles = T * (T + 1) / 2;
    int S = best_splits((long)tiles * nt, naux * std::max(nocc, nvir), 2 * h->cus, 64);
    S = (int)std::min<size_t>((size_t)S, std::max<size_t>(1, scratch_max(accs) / (2 * (size_t)nt * nmo2)));
    const long part_per_sector = (long)nt * S * nmo2;
    double* acc = scratch_get(h, accs, (size_t)2 * part_per_sector);
    if (!acc) return GW_ENOMEM;

    GW_TRY(sigma_fold_f64(h, nt, naux, nmo, nocc, eps, R, L, Zt));
    for (int sector = 0; sector < 2; ++sector) {
        const int xs0 = sector == 0 ? 0 : nocc, nxs = sector == 0 ? nocc : nvir;
        GemmF64 g;
        g.M = nmo; g.N = nmo; g.K = naux * nxs; g.batch = nt;
        g.a_kc = false; g.A = L; g.a_off = (long)xs0 * nmo; g.a_kdiv = nxs; g.a_khi = nmo2; g.a_klo = nmo;
        g.b_kc = false; g.B = Zt; g.b_off = (long)xs0 * nmo; g.b_kdiv = nxs; g.b_khi = nmo2;
        g.b_klo = nmo; g.b_bs = (long)naux * nmo2;
        g.sym_upper = true;
        g.epi = EPI_PARTIAL;
        g.nsplit = S;
        g.kchunk = ((g.K + S - 1) / S + 15) / 16 * 16;
        g.nsplit = (g.K + g.kchunk - 1) / g.kchunk;
        g.C = acc + sector * part_per_sector; g.ldc = nmo; g.c_ps = nmo2;
        g.tag = "sigma_contract";
        GW_TRY(gemm_f64(h, g));
        GW_TRY(reduce_splits(h, g.C, g.nsplit, nmo2, nt, nmo, nmo, nmo, true, 1.0, 0.0,
                             sector == 0 ? sigma_occ : sigma_vir, nmo2, nmo));
    }
    return GW_OK;
}

gw_status sigma_from_R_f64(Handle* h, int nocc, int nvir, int naux, int nmom_max, const double* eps,
                           const double* L, const double* R, const gw_opts* opts, double* sigma_occ,
                           double* sigma_vir) {
    const size_t cap = (opts && opts->zchunk_bytes) ? opts->zchunk_bytes : SIZE_MAX;
    return sigma_from_R_f64_bufs(h, nocc, nvir, naux, nmom_max, eps, L, R, cap, Scratch{WS_Z}, Scratch{WS_SIGACC},
                                 sigma_occ, sigma_vir);
}

}  // namespace gwm
