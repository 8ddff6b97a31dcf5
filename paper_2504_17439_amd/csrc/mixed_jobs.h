// Job descriptors of the mixed-precision self-energy stages, shared by the
// single-molecule path and the batched planner.
#pragma once

#include "internal.h"

namespace gwm {

typedef unsigned short u16;

constexpr int MIX_ND = 4;   // BF16 digits per operand
constexpr int MIX_MK = 32;  // k per MFMA step; digit planes are padded to a multiple of it

// One stage-1 job: a molecule's R_t digits and the x range [j0, j0 + ncol) of
// its L digit columns.  item0 / nP / nC index its tiles in grouped launches.
struct FoldJob {
    const u16* Rd;
    const int* eR;
    const u16* Ld;
    const int* eL;
    const double* eps;
    int naux, Ap, nmo, nocc;
    long j0, ncol, rplane, lplane;
    float* Zt;
    u16* Zl;
    long item0;
    int nP, nC;  // P-blocks (Ap / 16) and 128-column tiles
};

struct ZdigJob {
    long rows;  // nt * ncol of the job
    int Ap;
    const float* Zt;
    const u16* Zl;
    int* eZ;
    u16* Zd;
    long item0;  // first global row in grouped launches
};

struct ContractArgs {
    const u16* Ld; long lplane; const int* eL;  // L digit planes, k-blocked, rows (x, p) = nmo^2; exps per row
    const u16* Zd; long zplane; const int* eZ;  // Z digit planes, k-blocked, rows (n, c) = nt * ncol; exps per row
    int nmo, Ap, naux;
    int x0;                                      // first x of the chunk
    int xs0[2], nxs[2];                          // per sector: first x, count (within the chunk)
    int nt, nsplit, tiles_T;
    long ncol;
    double* part;                                // [2][nt][nsplit_total][nmo][nmo] FP64, accumulated
    int nsplit_total, split_off;                 // this job's splits are slots split_off .. + nsplit
    long item0;                                  // grouped launches: first work item of this job
};

inline int mixed_Ap(int naux) { return (naux + MIX_MK - 1) / MIX_MK * MIX_MK; }

// Scales and k-blocked digit planes of L (rows (x, q)) and of R_t (rows (t, P)).
gw_status mixed_prep(Handle* h, int naux, int nmo, int nt, const double* L, const double* R, u16* Ld, int* eL,
                     u16* Rd, int* eR);

FoldJob make_fold_job(const u16* Rd, const int* eR, const u16* Ld, const int* eL, const double* eps, int naux,
                      int Ap, int nmo, int nocc, long j0, long ncol, long rplane, long lplane, float* Zt, u16* Zl);

// Grouped launches over device job tables (item0 prefix sums set by the caller).
gw_status launch_fold_grouped(Handle* h, int nt, const FoldJob* jobs, int njobs, long total, int grid);
gw_status launch_zdig_grouped(Handle* h, const ZdigJob* jobs, int njobs, long total_rows);
gw_status launch_contract_grouped(Handle* h, const ContractArgs* jobs, int njobs, long total, int grid);

}  // namespace gwm
