// FP64 MFMA GEMM for gfx950 (v_mfma_f64_16x16x4_f64), used by every dense
// contraction of the FP64 path: R_n = eta~ V^T, the recursion updates
// D o X + c R V (Secs. 2.2-2.3), the RPA quadrature products and the
// self-energy contraction over (P, x) (eq. w_moments, eqs. convolution_*).
//
// Tile: 128 x 128 output per 256-thread workgroup (4 wave64s, 64 x 64 each,
// 4 x 4 MFMA blocks of 16 x 16; two workgroups per CU), K staged 16 at a time
// through two LDS stages filled by direct-to-LDS buffer loads (16 bytes per
// lane; no register staging, so no load result is waited for inside a K
// step).  Lanes outside the operand get a buffer offset past the resource's
// range and deposit zeros, which masks ragged rows and the K tail; the one
// element of a pair that straddles an odd edge is written from a register.
//
// The LDS layouts of the two operands are those of lds_f64.h (k-contiguous
// rows for a k-contiguous operand, k rows of 128 elements for a strided one).
#include "internal.h"
#include "lds_f64.h"

#include <algorithm>

namespace gwm {

namespace {

constexpr int TBM = 128;
constexpr int TBN = 128;
constexpr int TBK = 16;
constexpr int NTHR = 256;
constexpr int SLAB = TBM * TBK;            // doubles per operand slab
constexpr int STAGE = 2 * SLAB;            // doubles per stage (two stages per workgroup)
constexpr int GROUP_M = 8;                 // grouped raster: 8 tile rows share one B column slab
constexpr unsigned MASKED = LDS_MASKED;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base) { return f64_rsrc(base); }

__device__ inline void upper_tile(int t, int T, int& bi, int& bj) {
    int r = 0;
    while (t >= T - r) { t -= T - r; ++r; }
    bi = r;
    bj = r + t;
}

struct Operand {
    const double* X;   // batch-adjusted base
    long ld;           // k-contiguous: row stride
    long off, khi, klo;
    int d;             // strided: k = q d + r (d = 0: k not divided)
    int R, r0;
};

// Per-operand slab loader: wave w issues four 1 KB DMA instructions per slab.
//  k-contiguous: instruction i covers rows 8(4w + i) .. +7 (128 B each); lane
//    l takes row 8(4w + i) + (l >> 3), pair slot l & 7, i.e. the k pair
//    c = (l & 7) ^ (row & 7).
//  strided: instruction i covers k row 4w + i (128 doubles); lane l takes the
//    pair of elements r = (2l) ^ sw, r + 1, sw = 16 ((krow >> 1) & 3).
// A pair with only its first element inside the operand (odd K at the K end,
// or an odd row count at the edge) is masked in the DMA; once the DMA has
// landed, loader_fix writes that element (a slow path taken only by slabs
// that have such a pair).
template <bool KC>
struct Loader {
    unsigned voff[4];     // rows (k-contiguous) or elements (strided) outside the operand masked
    int kp2[4];           // k-contiguous: 2c, the pair's first k relative to the slab
    int q[4], rem[4];     // strided: (k / d, k % d) of the wave's four k rows
    long o[4];            // strided: element offset of the k row of the last issued slab
};

template <bool KC>
__device__ __forceinline__ void loader_init(Loader<KC>& L, const Operand& op, int wv, int lane, int kbeg) {
    if (KC) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 8 * (4 * wv + i) + (lane >> 3);
            const int c = (lane & 7) ^ (r & 7);
            L.kp2[i] = 2 * c;
            L.voff[i] = (op.r0 + r < op.R) ? (unsigned)(((long)r * op.ld + 2 * c) * 8) : MASKED;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kr = 4 * wv + i;
            const int r = (2 * lane) ^ (16 * ((kr >> 1) & 3));
            const int left = op.R - op.r0 - r;   // elements of the pair inside the operand
            L.voff[i] = left >= 2 ? (unsigned)(r * 8) : MASKED;
            const int k = kbeg + kr;
            if (op.d > 0) {
                L.q[i] = k / op.d;
                L.rem[i] = k - L.q[i] * op.d;
            } else {
                L.q[i] = 0;
                L.rem[i] = k;
            }
        }
    }
}

// DMA of the slab at k0 into S (SLAB doubles); k >= kend reads zero.
template <bool KC>
__device__ __forceinline__ void loader_issue(Loader<KC>& L, const Operand& op, int wv, int lane, int k0, int kend,
                                             double* S) {
    if (KC) {
        const __amdgpu_buffer_rsrc_t rs = rsrc(op.X + (long)op.r0 * op.ld + k0);
        const bool tail = k0 + TBK > kend;   // uniform: this slab reaches the K end
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            // pairs not wholly before the K end are masked (loader_fix writes a
            // lone first element)
            const unsigned v = (tail && k0 + L.kp2[i] + 1 >= kend) ? MASKED : L.voff[i];
            dma16(rs, S + (4 * wv + i) * 128, v);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kr = 4 * wv + i;
            const bool kok = k0 + kr < kend;
            const long o = op.off + (long)L.q[i] * op.khi + (long)L.rem[i] * op.klo + op.r0;
            L.o[i] = o;
            const __amdgpu_buffer_rsrc_t rs = rsrc(op.X + (kok ? o : 0));
            dma16(rs, S + kr * 128, kok ? L.voff[i] : MASKED);
            // advance this k row by one slab (16 k)
            if (op.d > 0) {
                int rr = L.rem[i] + TBK;
                int qv = L.q[i];
                while (rr >= op.d) { rr -= op.d; ++qv; }
                L.rem[i] = rr;
                L.q[i] = qv;
            } else {
                L.rem[i] += TBK;
            }
        }
    }
}

// After the DMA of the slab at k0 has landed: write the first element of each
// pair that straddles the K end (k-contiguous, odd K) or the row edge
// (strided, odd row count).  Slow path, taken only by slabs with such pairs.
template <bool KC>
__device__ __forceinline__ void loader_fix(const Loader<KC>& L, const Operand& op, int wv, int lane, int k0,
                                           int kend, double* S) {
    if (KC) {
        if (k0 + TBK <= kend || !(kend & 1)) return;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = k0 + L.kp2[i];
            const int r = 8 * (4 * wv + i) + (lane >> 3);
            if (kk == kend - 1 && L.voff[i] != MASKED) S[r * 16 + 2 * (lane & 7)] = op.X[(long)(op.r0 + r) * op.ld + kk];
        }
    } else {
        if (op.r0 + TBM <= op.R || !(op.R & 1)) return;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kr = 4 * wv + i;
            const int r = (2 * lane) ^ (16 * ((kr >> 1) & 3));
            if (op.R - op.r0 - r == 1 && k0 + kr < kend) S[kr * 128 + 2 * lane] = op.X[L.o[i] + r];
        }
    }
}

// Fragment of a 16-row block (rows rb .. rb+15) for k8-step h.
template <bool KC>
__device__ __forceinline__ v2d frag(const double* S, int rb, int h, int lane) {
    return KC ? frag_kc(S, rb, h, lane) : frag_kr<TBM>(S, rb, h, lane);
}

template <bool AKC, bool BKC>
__global__ __launch_bounds__(NTHR, 2) void gemm_f64_kernel(GemmF64 g, int tiles_m, int tiles_n) {
    __shared__ __attribute__((aligned(16))) double lds[2 * STAGE];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
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
    const int nkt = (kend > kbeg) ? (kend - kbeg + TBK - 1) / TBK : 0;

    Operand oa, ob;
    oa.X = g.A + (long)batch * g.a_bs; oa.ld = g.lda; oa.off = g.a_off; oa.khi = g.a_khi; oa.klo = g.a_klo;
    oa.d = g.a_kdiv >= (1L << 31) ? 0 : (int)g.a_kdiv; oa.R = g.M; oa.r0 = m0;
    ob.X = g.B + (long)batch * g.b_bs; ob.ld = g.ldb; ob.off = g.b_off; ob.khi = g.b_khi; ob.klo = g.b_klo;
    ob.d = g.b_kdiv >= (1L << 31) ? 0 : (int)g.b_kdiv; ob.R = g.N; ob.r0 = n0;
    const double* asc = (AKC && g.ascale) ? g.ascale + (long)batch * g.ascale_bs : nullptr;
    const bool scaled = asc != nullptr;

    Loader<AKC> la;
    Loader<BKC> lb;
    loader_init<AKC>(la, oa, wv, lane, kbeg);
    loader_init<BKC>(lb, ob, wv, lane, kbeg);

    // k scale of the next slab, per lane the pairs (2(4h + g), +1) of k8-steps
    // h = 0, 1 (loaded one slab ahead; k past the end reads a clamped index:
    // the A values there are zero)
    v2d scn[2] = {(v2d){1.0, 1.0}, (v2d){1.0, 1.0}};
    auto load_scale = [&](int k0) {
        if (scaled) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = k0 + 2 * (4 * h + (lane >> 4));
                const int k1 = min(k + 1, kend - 1), kc = min(k, kend - 1);
                scn[h] = (v2d){asc[kc], asc[k1]};
            }
        }
    };

    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

    const int wm = (wv >> 1) * 64;
    const int wn = (wv & 1) * 64;

    if (nkt > 0) {
        loader_issue<AKC>(la, oa, wv, lane, kbeg, kend, lds);
        loader_issue<BKC>(lb, ob, wv, lane, kbeg, kend, lds + SLAB);
        load_scale(kbeg);
        for (int kt = 0; kt < nkt; ++kt) {
            double* S = lds + (kt & 1) * STAGE;
            // own DMAs of stage kt (and the fix-up loads) done; write the
            // fix-ups, then the barrier makes stage kt visible to every wave
            // and frees the other stage for the refill below
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            loader_fix<AKC>(la, oa, wv, lane, kbeg + kt * TBK, kend, S);
            loader_fix<BKC>(lb, ob, wv, lane, kbeg + kt * TBK, kend, S + SLAB);
            __syncthreads();
            const v2d sc0 = scn[0], sc1 = scn[1];
            if (kt + 1 < nkt) {
                const int k1 = kbeg + (kt + 1) * TBK;
                double* Sn = lds + ((kt + 1) & 1) * STAGE;
                loader_issue<AKC>(la, oa, wv, lane, k1, kend, Sn);
                loader_issue<BKC>(lb, ob, wv, lane, k1, kend, Sn + SLAB);
                load_scale(k1);
            }
            const double* SA = S;
            const double* SB = S + SLAB;
            v2d fa[2][4], fb[2][4];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int i = 0; i < 4; ++i) fa[h][i] = frag<AKC>(SA, wm + i * 16, h, lane);
#pragma unroll
                for (int j = 0; j < 4; ++j) fb[h][j] = frag<BKC>(SB, wn + j * 16, h, lane);
            }
            if (scaled) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    fa[0][i] *= sc0;
                    fa[1][i] *= sc1;
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 2; ++e)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(e ? fa[h][i].y : fa[h][i].x,
                                                                            e ? fb[h][j].y : fb[h][j].x,
                                                                            acc[i][j], 0, 0, 0);
            // the other stage is refilled at the next step only after every
            // wave has passed this step's reads (the barrier at its top)
        }
    }

    const int lrow = lane & 15;
    const int lk = lane >> 4;
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

// Node sum of the RPA quadrature (Sec. 2.2, eq. Gmain and the offset
// integral): P_grp[P][ia] = sum_{b in group} sum_Q S_b[P][Q] V[Q][ia] g_b[ia].
// The K index runs over (Q block, node) with the node innermost, so a 16 x 128
// slab of V is loaded once per Q block and its fragments stay in registers
// for every node of the group; only the 128 x 16 slabs of S_b stream through
// LDS.  The node's column factor g_b (a function of D_ia) scales the V
// fragments in registers before its MFMAs.
__global__ __launch_bounds__(NTHR, 2) void node_sum_kernel(const double* __restrict__ S, const double* __restrict__ V,
                                                           const double* __restrict__ gtab, int naux, int ov, int nb,
                                                           int ngrp, int tiles_m, int tiles_n,
                                                           double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) double lds[4 * SLAB];   // A stages 0, 1; B stages 0, 1
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int grp = blockIdx.y;

    int bi, bj;
    {
        int nwg = gridDim.x;
        int bid = blockIdx.x;
        int logical = bid;
        if ((nwg & 7) == 0) logical = (bid & 7) * (nwg >> 3) + (bid >> 3);
        int per_group = GROUP_M * tiles_n;
        int group = logical / per_group;
        int first_m = group * GROUP_M;
        int gsize = min(tiles_m - first_m, GROUP_M);
        int in = logical - group * per_group;
        bi = first_m + in % gsize;
        bj = in / gsize;
    }
    const int m0 = bi * TBM;
    const int n0 = bj * TBN;
    const int b0 = (int)((long)nb * grp / ngrp), b1 = (int)((long)nb * (grp + 1) / ngrp);
    const int nbg = b1 - b0;
    const int nq = (naux + TBK - 1) / TBK;
    const int nsteps = nq * nbg;
    const long n2 = (long)naux * naux;

    Operand oa, ob;
    oa.X = S; oa.ld = naux; oa.off = 0; oa.khi = 0; oa.klo = 0; oa.d = 0; oa.R = naux; oa.r0 = m0;
    ob.X = V; ob.ld = 0; ob.off = 0; ob.khi = 0; ob.klo = ov; ob.d = 0; ob.R = ov; ob.r0 = n0;
    Loader<true> la;
    Loader<false> lb;
    loader_init<true>(la, oa, wv, lane, 0);
    loader_init<false>(lb, ob, wv, lane, 0);

    const int wm = (wv >> 1) * 64;
    const int wn = (wv & 1) * 64;
    const int gcol0 = n0 + wn + (lane & 15);   // the lane's column in block j is gcol0 + 16 j

    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

    auto issue_a = [&](int step) {
        const int qb = step / nbg, b = b0 + step - qb * nbg;
        Operand o = oa;
        o.X = S + (long)b * n2;
        loader_issue<true>(la, o, wv, lane, qb * TBK, naux, lds + (step & 1) * SLAB);
    };
    double gn[4];
    auto load_g = [&](int step) {
        const int b = b0 + step % nbg;
#pragma unroll
        for (int j = 0; j < 4; ++j) gn[j] = gtab[(long)b * ov + min(gcol0 + 16 * j, ov - 1)];
    };

    if (nsteps > 0) {
        issue_a(0);
        loader_issue<false>(lb, ob, wv, lane, 0, naux, lds + 2 * SLAB);
        load_g(0);
        v2d fb[2][4];
        for (int st = 0; st < nsteps; ++st) {
            const int qb = st / nbg;
            const bool first = st == qb * nbg;
            double* SA = lds + (st & 1) * SLAB;
            double* SB = lds + (2 + (qb & 1)) * SLAB;
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            {
                Operand o = oa;
                o.X = S + (long)(b0 + st - qb * nbg) * n2;
                loader_fix<true>(la, o, wv, lane, qb * TBK, naux, SA);
            }
            if (first) loader_fix<false>(lb, ob, wv, lane, qb * TBK, naux, SB);
            __syncthreads();
            double g[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) g[j] = gn[j];
            if (st + 1 < nsteps) {
                issue_a(st + 1);
                load_g(st + 1);
            }
            if (first) {
                if (qb + 1 < nq) loader_issue<false>(lb, ob, wv, lane, (qb + 1) * TBK, naux, lds + (2 + ((qb + 1) & 1)) * SLAB);
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int j = 0; j < 4; ++j) fb[h][j] = frag<false>(SB, wn + j * 16, h, lane);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                v2d fa[4], fs[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) fa[i] = frag<true>(SA, wm + i * 16, h, lane);
#pragma unroll
                for (int j = 0; j < 4; ++j) fs[j] = fb[h][j] * g[j];
#pragma unroll
                for (int e = 0; e < 2; ++e)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(e ? fa[i].y : fa[i].x,
                                                                            e ? fs[j].y : fs[j].x, acc[i][j], 0, 0, 0);
            }
        }
    }

    const int lrow = lane & 15;
    const int lk = lane >> 4;
    double* out = part + (long)grp * naux * ov;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn + j * 16 + lrow;
            if (col >= ov) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + i * 16 + lk + 4 * r;
                if (row < naux) out[(long)row * ov + col] = acc[i][j][r];
            }
        }
}

// G = X0 o d0 + sum_grp part[grp], groups added in order
__global__ void node_sum_reduce_kernel(long n, long ov, int ngrp, const double* __restrict__ part,
                                       const double* __restrict__ X0, const double* __restrict__ d0,
                                       double* __restrict__ G) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = X0[i] * d0[i % ov];
    for (int g = 0; g < ngrp; ++g) s += part[(long)g * n + i];
    G[i] = s;
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

// Symmetric results (mirror set, M == N): one work group per upper 32 x 32
// tile sums that tile's partials row by row (coalesced reads), writes it and
// writes its mirror image through an LDS transpose; a diagonal tile reads the
// upper triangle of itself.  The same sums in the same order as
// reduce_splits_kernel, whose mirrored reads go down columns of the partials.
__global__ __launch_bounds__(256) void reduce_splits_sym_kernel(const double* __restrict__ part, int nsplit, long ps,
                                                                int M, long ld, double alpha, double diag,
                                                                double* __restrict__ out, long out_bs, long ldo) {
    const int T = (M + 31) / 32;
    int t = blockIdx.x, bi = 0;
    while (t >= T - bi) {
        t -= T - bi;
        ++bi;
    }
    const int bj = bi + t;
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const double* __restrict__ pb = part + (long)blockIdx.z * nsplit * ps;
    double* __restrict__ ob = out + (long)blockIdx.z * out_bs;
    for (int r = ty; r < 32; r += 8) {
        const int m = bi * 32 + r, n = bj * 32 + tx;
        if (m >= M || n >= M) continue;
        const double* p = pb + (long)min(m, n) * ld + max(m, n);
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += p[(long)k * ps];
        s *= alpha;
        if (m == n) s += diag;
        ob[(long)m * ldo + n] = s;
        tile[r][tx] = s;
    }
    if (bi == bj) return;  // the same for the whole work group
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int m = bj * 32 + r, n = bi * 32 + tx;  // out[m][n] = s(n, m)
        if (m >= M || n >= M) continue;
        ob[(long)m * ldo + n] = tile[tx][r];
    }
}

}  // namespace

int best_splits(long items, int K, int slots, int max_ns) {
    max_ns = std::max(1, std::min(max_ns, std::max(1, K / (4 * TBK))));
    slots = std::max(slots, 1);
    double best = 1e300;
    int best_ns = 1;
    for (int ns = 1; ns <= max_ns; ++ns) {
        const long chunk = ((K + ns - 1) / ns + TBK - 1) / TBK * TBK;
        const long wgs = items * ns;
        const long rounds = (wgs + slots - 1) / slots;
        // a 1% penalty per doubling of the split count keeps the partials few on near ties
        const double cost = (double)rounds * (double)chunk * (1.0 + 0.01 * std::log2((double)ns));
        if (cost < best) {
            best = cost;
            best_ns = ns;
        }
    }
    return best_ns;
}

void plan_split(GemmF64& g, int slots) {
    int tm = (g.M + TBM - 1) / TBM, tn = (g.N + TBN - 1) / TBN;
    long tiles = g.sym_upper ? (long)tm * (tm + 1) / 2 : (long)tm * tn;
    tiles *= g.batch;
    int ns = best_splits(tiles, g.K, slots, 65535);
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
    // a k-contiguous slab is addressed by 32-bit byte offsets from its first row
    if ((g.a_kc && (long)TBM * g.lda * 8 >= (1L << 30)) || (g.b_kc && (long)TBN * g.ldb * 8 >= (1L << 30)))
        return set_err(h, GW_EINVAL, "gemm_f64: leading dimension too large");
    if ((!g.a_kc && g.a_kdiv < (1L << 31) && g.a_kdiv <= 0) || (!g.b_kc && g.b_kdiv < (1L << 31) && g.b_kdiv <= 0))
        return set_err(h, GW_EINVAL, "gemm_f64: bad k divisor");
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

gw_status node_sum_f64(Handle* h, int naux, long ov, int nb, const double* S, const double* V, const double* gtab,
                       const double* X0, const double* d0, double* G, const Scratch& part_scr) {
    if (naux <= 0 || ov <= 0) return GW_OK;
    if (ov > 0x7fffffffL / 8) return set_err(h, GW_EINVAL, "node_sum: ov too large");
    const int tm = (naux + TBM - 1) / TBM, tn = (int)((ov + TBN - 1) / TBN);
    const long tiles = (long)tm * tn;
    // node groups: fewest rounds of work groups x nodes per group (a few
    // groups even out the last round; each adds a partial to reduce)
    const int slots = 2 * h->cus;
    int ngrp = 1;
    double best = 1e300;
    for (int ng = 1; ng <= std::min(nb, 8); ++ng) {
        const long rounds = (tiles * ng + slots - 1) / slots;
        const double cost = (double)rounds * ((nb + ng - 1) / ng) * (1.0 + 0.02 * (ng - 1));
        if (cost < best) { best = cost; ngrp = ng; }
    }
    if ((size_t)ngrp * naux * ov > scratch_max(part_scr)) {
        ngrp = (int)std::max<size_t>(1, scratch_max(part_scr) / ((size_t)naux * ov));
        if ((size_t)ngrp * naux * ov > scratch_max(part_scr))
            return set_err(h, GW_ENOMEM, "node_sum: partial buffer too small");
    }
    double* part = scratch_get(h, part_scr, (size_t)ngrp * naux * ov);
    if (!part) return GW_ENOMEM;
    if (tiles > 0x7fffffffL) return set_err(h, GW_EINVAL, "node_sum: grid too large");
    {
        KTimer timer(h, "rpa_quad");
        hipLaunchKernelGGL(node_sum_kernel, dim3((unsigned)tiles, (unsigned)ngrp), dim3(NTHR), 0, h->stream, S, V, gtab,
                           naux, (int)ov, nb, ngrp, tm, tn, part);
        GW_CHECK_LAUNCH(h);
        const long n = (long)naux * ov;
        hipLaunchKernelGGL(node_sum_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, n, ov,
                           ngrp, part, X0, d0, G);
        GW_CHECK_LAUNCH(h);
        timer.stop();
    }
    return GW_OK;
}

gw_status reduce_splits(Handle* h, const double* part, int nsplit, long ps, int batch, int M, int N,
                        long ld, bool mirror, double alpha, double diag, double* out, long out_bs,
                        long ldo) {
    long n = (long)M * N;
    if (n == 0 || batch == 0) return GW_OK;
    if (mirror && M == N) {
        const long T = (M + 31) / 32;
        hipLaunchKernelGGL(reduce_splits_sym_kernel, dim3((unsigned)(T * (T + 1) / 2), 1, (unsigned)batch), dim3(256),
                           0, h->stream, part, nsplit, ps, M, ld, alpha, diag, out, out_bs, ldo);
        GW_CHECK_LAUNCH(h);
        return GW_OK;
    }
    dim3 grid((unsigned)((n + 255) / 256), 1, (unsigned)batch);
    hipLaunchKernelGGL(reduce_splits_kernel, grid, dim3(256), 0, h->stream, part, nsplit, ps, M, N, ld,
                       mirror ? 1 : 0, alpha, diag, out, out_bs, ldo);
    GW_CHECK_LAUNCH(h);
    return GW_OK;
}

}  // namespace gwm
