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
//   both of its columns (half the products of the full column range).  Both
//   operands reach LDS by direct-to-LDS loads: the rows (t, P) of R_t as
//   k-contiguous rows, the 64 pair columns of L as k rows.
// Stage 2 (gemm_f64): Sigma^{(n)}[p,q] = sum_{P, x in sector} L[P,x,p] Zt^{(n)}[P,x,q],
//   upper 128x128 tiles only, split-K partials, then one reduction that
//   mirrors the upper triangle (exactly symmetric).
#include "internal.h"
#include "lds_f64.h"

#include <algorithm>

namespace gwm {

namespace {

constexpr int FBP = 16;   // P rows per tile
constexpr int FBC = 64;   // pair columns per tile (one 8 x 8 pair block; 16 per wave)
constexpr int FBK = 16;   // Q per slab
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

// LDS of one stage: the A slab (rows (t, p), t < NT, p < 16, as k-contiguous
// rows of 16 Q) then the B slab (16 Q rows of the 64 pair columns).
template <int NT>
struct FoldStage {
    static constexpr int AROWS = NT * FBP;
    static constexpr int ASLAB = AROWS * FBK;       // doubles
    static constexpr int BSLAB = FBK * FBC;         // doubles
    static constexpr int SIZE = ASLAB + BSLAB;
    static constexpr int AINS = AROWS / 8 / 4;      // A instructions per wave and slab (8 rows each)
    static constexpr int BINS = BSLAB / 128 / 4;    // B instructions per wave and slab (2 Q rows each)
    static_assert(AROWS % 32 == 0 && BSLAB % 512 == 0, "fold slab split over four waves");
};

// Tile: 16 P rows x one pair block, all NT moments; wave w owns pair columns
// 16 w .. 16 w + 15 (acc[t] = its 16 x 16 block of R_t L).  Work group b runs
// on XCD b % 8; each XCD walks groups of 4 P-blocks x 8 pair blocks, which
// share their R rows and L columns through its L2.
template <int NT>
__global__ __launch_bounds__(FTHR, 2) void sigma_fold_kernel(const double* __restrict__ R,
                                                              const double* __restrict__ L,
                                                              const double* __restrict__ eps, int naux,
                                                              int nmo, int nocc, int nb, int nblk,
                                                              double* __restrict__ Zt) {
    using FS = FoldStage<NT>;
    __shared__ __attribute__((aligned(16))) double lds[2 * FS::SIZE];

    const int nP = (naux + FBP - 1) / FBP;
    int pb, ct;
    {
        const int nPg = (nP + 3) / 4;
        const int b = blockIdx.x;
        const int xcd = b & 7, local = b >> 3;
        const int grp = (local >> 5) * 8 + xcd;
        const int w = local & 31;
        pb = (grp % nPg) * 4 + (w & 3);
        ct = (grp / nPg) * 8 + (w >> 2);
        if (pb >= nP || ct >= nblk) return;
    }
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    int BX, BY;
    pair_block(ct, nb, BX, BY);
    const int P0 = pb * FBP;
    const long nmo2 = (long)nmo * nmo;
    const int nkt = (naux + FBK - 1) / FBK;

    // A instruction i = wv AINS + ii covers rows 8i .. 8i + 7 = moment i / 2,
    // rows p = 8 (i & 1) + (lane >> 3); lane slot lane & 7 holds the k pair
    // c = (lane & 7) ^ (lane >> 3) (the row's swizzle).  Rows past naux and
    // pairs past the Q end are masked.
    const int ca = (lane & 7) ^ (lane >> 3);
    unsigned voffA[FS::AINS];
#pragma unroll
    for (int ii = 0; ii < FS::AINS; ++ii) {
        const int i = wv * FS::AINS + ii;
        const int p = 8 * (i & 1) + (lane >> 3);
        voffA[ii] = P0 + p < naux ? (unsigned)(((long)p * naux + 2 * ca) * 8) : LDS_MASKED;
    }
    // B instruction j = wv BINS + jj covers Q rows 2j, 2j + 1 (lane >> 5) of
    // the slab; the lane's slot 2 (lane & 31) holds pair column c = slot ^
    // sw(2j).  Columns past the orbital range are masked; a pair (q, q + 1)
    // with only q = nmo - 1 inside is masked and its first element written
    // after the load (odd nmo).
    long colB[FS::BINS];
    unsigned voffB[FS::BINS];
    bool fixB[FS::BINS];
#pragma unroll
    for (int jj = 0; jj < FS::BINS; ++jj) {
        const int j = wv * FS::BINS + jj;
        const int c = (2 * (lane & 31)) ^ ksw(2 * j);
        const int x = 8 * BX + (c >> 3), q = 8 * BY + (c & 7);
        colB[jj] = (long)x * nmo + q;
        const bool ok = x < nmo && q + 1 < nmo;
        fixB[jj] = x < nmo && q + 1 == nmo;
        voffB[jj] = ok ? (unsigned)(((long)(lane >> 5) * nmo2 + colB[jj]) * 8) : LDS_MASKED;
    }

    auto issue = [&](int kt, double* S) {
        const int k0 = kt * FBK;
        const bool tail = k0 + FBK > naux;
#pragma unroll
        for (int ii = 0; ii < FS::AINS; ++ii) {
            const int i = wv * FS::AINS + ii;
            const int t = i >> 1;
            const double* base = R + ((long)t * naux + P0) * naux + k0;
            const unsigned v = (tail && k0 + 2 * ca + 1 >= naux) ? LDS_MASKED : voffA[ii];
            dma16(f64_rsrc(base), S + i * 128, v);
        }
        double* SB = S + FS::ASLAB;
#pragma unroll
        for (int jj = 0; jj < FS::BINS; ++jj) {
            const int j = wv * FS::BINS + jj;
            const int kr = 2 * j + (lane >> 5);
            const double* base = L + (long)min(k0 + 2 * j, naux - 1) * nmo2;
            dma16(f64_rsrc(base), SB + j * 128, k0 + kr < naux ? voffB[jj] : LDS_MASKED);
        }
    };
    // after the loads of slab kt have landed: the lone first elements of
    // pairs that straddle the Q end (odd naux) or the orbital end (odd nmo)
    auto fix = [&](int kt, double* S) {
        const int k0 = kt * FBK;
        if ((naux & 1) && k0 + FBK > naux) {
#pragma unroll
            for (int ii = 0; ii < FS::AINS; ++ii) {
                const int i = wv * FS::AINS + ii;
                const int p = 8 * (i & 1) + (lane >> 3);
                if (k0 + 2 * ca == naux - 1 && P0 + p < naux)
                    S[i * 128 + 2 * lane] = R[((long)(i >> 1) * naux + P0 + p) * naux + naux - 1];
            }
        }
        if (nmo & 1) {
            double* SB = S + FS::ASLAB;
#pragma unroll
            for (int jj = 0; jj < FS::BINS; ++jj) {
                const int j = wv * FS::BINS + jj;
                const int kr = 2 * j + (lane >> 5);
                if (fixB[jj] && k0 + kr < naux) SB[j * 128 + 2 * lane] = L[(long)(k0 + kr) * nmo2 + colB[jj]];
            }
        }
    };

    v4d acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};

    issue(0, lds);
    for (int kt = 0; kt < nkt; ++kt) {
        double* S = lds + (kt & 1) * FS::SIZE;
        // own loads of slab kt done (and its fix-ups written); the barrier
        // makes the slab visible to every wave and frees the other stage,
        // whose reads all ended before it, for the refill below
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        fix(kt, S);
        __syncthreads();
        if (kt + 1 < nkt) issue(kt + 1, lds + ((kt + 1) & 1) * FS::SIZE);
        const double* SB = S + FS::ASLAB;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const v2d fb = frag_kr<FBC>(SB, wv * 16, h, lane);
            v2d fa[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) fa[t] = frag_kc(S, t * 16, h, lane);
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(e ? fa[t].y : fa[t].x, e ? fb.y : fb.x, acc[t],
                                                                 0, 0, 0);
        }
    }

    // epilogue: lane owns pair c and rows lk + 4r; binomial / eps-power fold
    // for each output of the pair
    const int lrow = lane & 15;
    const int lk = lane >> 4;
    const int c = wv * 16 + lrow;
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
    const int nb = (nmo + 7) / 8, nblk = nb * (nb + 1) / 2;
    const long nP = (naux + FBP - 1) / FBP;
    // groups of 4 P-blocks x 8 pair blocks, 8 groups (one per XCD) per round
    const long groups = (nP + 3) / 4 * ((nblk + 7) / 8);
    const long rounds = (groups + 7) / 8;
    hipLaunchKernelGGL((sigma_fold_kernel<NT>), dim3((unsigned)(rounds * 8 * 32)), dim3(FTHR), 0, h->stream, R, L,
                       eps, naux, nmo, nocc, nb, nblk, Zt);
}

}  // namespace

gw_status sigma_fold_f64(Handle* h, int nt, int naux, int nmo, int nocc, const double* eps,
                         const double* R, const double* L, double* Zt) {
    const long nb = (nmo + 7) / 8;
    const long groups = ((naux + FBP - 1) / FBP + 3) / 4 * ((nb * (nb + 1) / 2 + 7) / 8);
    if ((groups + 7) / 8 * 256 > 0x7fffffffL) return set_err(h, GW_EINVAL, "sigma_fold: grid too large");
    // slabs are addressed by 32-bit byte offsets: 16 rows of R, two rows of L
    if ((long)FBP * naux * 8 >= (1L << 31) || 2L * nmo * nmo * 8 >= (1L << 31))
        return set_err(h, GW_EINVAL, "sigma_fold: naux or nmo too large");
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
