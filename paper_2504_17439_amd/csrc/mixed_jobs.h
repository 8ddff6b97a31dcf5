// Job descriptors of the mixed-precision self-energy stages, shared by the
// single-molecule path and the batched planner.
#pragma once

#include "internal.h"

#include <algorithm>

namespace gwm {

typedef unsigned short u16;  // BF16 bit patterns
typedef signed char i8;      // one base-255 digit

constexpr int MIX_ND = 4;   // int8 digits per operand
constexpr int MIX_MK = 64;  // k per MFMA step (64 B per row); digit planes are padded to a multiple of it

// One stage-1 job: a molecule's R_t digits and all its L digit columns, taken
// as 8 x 8 blocks of orbital pairs (x, y), x <= y (nblk upper blocks of nb
// per side); every pair is written to both of its rows (x, y) and (y, x) of
// Zt / Zl [nt][ncol = nmo^2][Ap].  item0 / nP / nC index its tiles in grouped
// launches (item0 in tile groups).
struct FoldJob {
    const i8* Rd;
    const int* eR;
    const i8* Ld;
    const int* eL;
    const double* eps;
    int naux, Ap, nmo, nocc;
    long ncol, rplane, lplane;
    int nb, nblk;
    float* Zt;
    u16* Zl;
    long item0;  // grouped launches: first tile group (fold_groups) of this job
    int nP, nC;  // P-blocks (Ap / 16) and column tiles (fold_cols / 64 pair blocks each)
};

struct ZdigJob {
    long rows;  // nt * ncol of the job
    int Ap;
    const float* Zt;
    const u16* Zl;
    int* eZ;
    i8* Zd;
    long item0;  // first global row in grouped launches
};

struct ContractArgs {
    const i8* Ld; long lplane; const int* eL;   // L digit planes, k-blocked, rows (x, p) = nmo^2; exps per row
    const i8* Zd; long zplane; const int* eZ;   // Z digit planes, k-blocked, rows (n, c) = nt * ncol; exps per row
    int nmo, Ap, naux;
    int x0;                                      // first x of the chunk
    int xs0[2], nxs[2];                          // per sector: first x, count (within the chunk)
    int nt, nsplit, tilesN, tiles;               // column blocks of 64, upper tm x 64 tiles
    int tm;                                      // tile height: 128, or 64 (grouped launches only)
    long ncol;
    double* part;                                // [2][nt][nsplit_total][nmo][nmo] FP64, accumulated
    int nsplit_total, split_off;                 // this job's splits are slots split_off .. + nsplit
    long item0;                                  // grouped launches: first item group (contract_groups)
};

inline int mixed_Ap(int naux) { return (naux + MIX_MK - 1) / MIX_MK * MIX_MK; }

// Tile groups of a stage-1 job in grouped launches: 4 P-blocks x 8 column tiles.
inline long fold_groups(const FoldJob& f) { return (long)((f.nP + 3) / 4) * ((f.nC + 7) / 8); }

// Item groups of a stage-2 job in grouped launches: 32 consecutive work items
// (tile, n, split, sector).
inline long contract_groups(const ContractArgs& a) { return ((long)a.tiles * a.nt * a.nsplit * 2 + 31) / 32; }

// Stage-1 tile shape for nt moments: each of the 4 waves owns fold_tpw(nt)
// moments (int32 accumulators for 4 digit weights x 4 column blocks each),
// fold_tg(nt) groups of waves split the moments, the rest split the columns;
// the tile is 16 P rows x fold_cols(nt) columns.
__host__ __device__ constexpr int fold_tpw(int nt) { return nt <= 2 ? 1 : (nt == 4 || nt == 8) ? 2 : 3; }
__host__ __device__ constexpr int fold_tg(int nt) { return (nt + fold_tpw(nt) - 1) / fold_tpw(nt); }
__host__ __device__ constexpr int fold_cg(int nt) { return 4 / fold_tg(nt); }
__host__ __device__ constexpr int fold_cols(int nt) { return 64 * fold_cg(nt); }

// Upper tm-row x 64-column tiles (tm = 128 or 64) of a symmetric M x M
// result: row block bi keeps column blocks bj >= (tm / 64) bi.
inline int mixed_upper_tiles(int M, int tm = 128) {
    const int R = tm / 64, TM = (M + tm - 1) / tm, TN = (M + 63) / 64;
    int n = 0;
    for (int bi = 0; bi < TM; ++bi) n += std::max(0, TN - R * bi);
    return n;
}

// Scales and k-blocked digit planes of L (rows (x, q)) and of R_t (rows (t, P)).
gw_status mixed_prep(Handle* h, int naux, int nmo, int nt, const double* L, const double* R, i8* Ld, int* eL,
                     i8* Rd, int* eR);

FoldJob make_fold_job(int nt, const i8* Rd, const int* eR, const i8* Ld, const int* eL, const double* eps, int naux,
                      int Ap, int nmo, int nocc, long rplane, long lplane, float* Zt, u16* Zl);

// Grouped launches over device job tables; total = the groups of all jobs
// (item0 prefix sums of fold_groups / contract_groups, set by the caller;
// zdig: rows).
gw_status launch_fold_grouped(Handle* h, int nt, const FoldJob* jobs, int njobs, long total, int grid);
gw_status launch_zdig_grouped(Handle* h, const ZdigJob* jobs, int njobs, long total_rows);
gw_status launch_contract_grouped(Handle* h, const ContractArgs* jobs, int njobs, long total, int grid,
                                  bool all64);

}  // namespace gwm
