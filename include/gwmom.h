/*
 * gwmom.h -- C ABI of the MI355X moment-conserving GW library (libgwmom.so).
 *
 * Method: Backhouse, Allen, Scott, Booth, "Self-consistent GW via conservation
 * of spectral moments".  The library computes, on one AMD Instinct MI355X
 * (gfx950), the density-fitted hot path of moment-conserving G0W0:
 *
 *   density-response moments  eta~^{(n)}, R_n = eta~^{(n)} V^T   (Sec. 2.2 RPA, Sec. 2.3 TDA)
 *   self-energy moments       Sigma^{(n,<)}, Sigma^{(n,>)}        (eqs. convolution_occ/_vir, w_moments)
 *   auxiliary poles           block Lanczos on the moments         (eq. effH, Sec. 2)
 *   upfolded Hamiltonian      eigenpairs and QP assignment         (eqs. effH, ret_GF, quasiparticle_energy_update)
 *
 * Conventions (all entry points)
 * ------------------------------
 *  - nmo = nocc + nvir.  Orbital energies eps[nmo] list the nocc occupied
 *    levels first, then the nvir virtual ones; every occupied energy must lie
 *    below every virtual one.
 *  - L[naux][nmo][nmo] is the three-index Coulomb factor in the MO basis
 *    (the paper's V_{P,pq}), dense row-major FP64, symmetric in its last two
 *    indices.  The particle-hole block is V[P][i*nvir + a] = L[P][i][nocc+a].
 *  - Every array argument is a DEVICE pointer on the handle's device unless
 *    marked "host".  Arrays are dense, row-major, caller-owned; the library
 *    never frees or retains them past the call.
 *  - Work is enqueued on the handle's stream.  gw_moments_* and
 *    gw_sigma_moments return once the work is enqueued; gw_poles returns
 *    after the stream has drained (it reports pole counts to the host).
 *  - Inputs are validated before anything is launched; a failed validation
 *    returns GW_EINVAL and leaves outputs untouched.  gw_last_error() gives
 *    a message for the last failure on the handle.
 *  - The library allocates its own device workspace (grow-only, owned by
 *    the handle, released by gw_destroy).  One handle per host thread.
 *  - nmom_max (the paper's n_mom^max) must be odd: the block Lanczos step
 *    conserves moments 0..nmom_max with (nmom_max+1)/2 blocks per sector.
 */
#ifndef GWMOM_H
#define GWMOM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gw_handle_s* gw_handle;

typedef enum {
    GW_OK = 0,
    GW_EINVAL = -1,   /* bad argument: sizes, null pointers, even nmom_max, bad eps */
    GW_ENOMEM = -2,   /* device workspace could not be allocated */
    GW_EHIP = -3,     /* a HIP runtime call or kernel launch failed */
    GW_ENUMERIC = -4, /* a moment matrix is not PSD or an eigensolve failed */
    GW_ENOCONV = -5,  /* an iterative loop hit its iteration cap */
    GW_ELIB = -6      /* rocBLAS / rocSOLVER reported an error */
} gw_status;

typedef enum { GW_FP64 = 0, GW_MIXED = 1 } gw_precision;
typedef enum { GW_TDA = 0, GW_RPA = 1 } gw_screening;

/* Optional knobs; pass NULL (or zero fields) for the defaults. */
typedef struct {
    int nquad;          /* RPA quadrature points; <= 0 -> 48                         */
    double quad_scale;  /* RPA grid scale s in z = s(1+x)/(1-x); <= 0 -> median(D)  */
    double pinv_tol;    /* Lanczos pseudo-inverse cut (relative); <= 0 -> 1e-12      */
    double neg_tol;     /* Lanczos non-PSD tolerance (relative);  <= 0 -> 1e-8       */
    size_t zchunk_bytes;/* cap on the folded intermediate of the self-energy stage
                           (bytes; GW_ENOMEM above it); 0 -> no cap              */
    double moment_eps;  /* relative accuracy of the moments given to gw_poles; sets
                           the Lanczos deflation level; <= 0 -> 2^-52 (FP64 moments) */
} gw_opts;

/* Create a handle on HIP device `device` with its own non-blocking stream. */
gw_status gw_create(gw_handle* h, int device);
/* Run on an existing hipStream_t (from the caller, e.g. a torch stream)
 * instead of the handle's own non-blocking stream; NULL selects the device's
 * default (null) stream, so that work is ordered with a caller that uses it. */
gw_status gw_set_stream(gw_handle h, void* hip_stream);
gw_status gw_synchronize(gw_handle h);
gw_status gw_destroy(gw_handle h);
/* Message for the last failure on h (static string if h is NULL). */
const char* gw_last_error(gw_handle h);

/*
 * TDA density-response moments (Sec. 2.3):
 *   eta~^{(0)} = V,  eta~^{(n)} = eta~^{(n-1)} (D + 2 V^T V),  R_n = eta~^{(n)} V^T.
 * Outputs:
 *   R   [nmom_max+1][naux][naux]          symmetric; required.
 *   eta [nmom_max+1][naux][nocc*nvir]     nullable.
 * prec: GW_FP64 (FP64 MFMA), or GW_MIXED with eta NULL: the half-order
 * products R_2k = X_k X_k^T, R_2k+1 = X_k D X_k^T + 2 R_k R_k and the updates
 * X_k+1 = D o X_k + 2 R_k V use four-digit int8 fixed-point operands (base
 * 255, one power-of-two scale per row) on the integer MFMA, with exact int32
 * sums per digit weight (k split into ranges of at most 32768) combined in
 * FP64 (R_k R_k and X stay FP64); with eta requested the FP64 form is used.
 * R is returned in FP64.  GW_MIXED needs naux <= 32768.
 */
gw_status gw_moments_tda(gw_handle h, int nocc, int nvir, int naux, int nmom_max,
                         const double* eps, const double* L, gw_precision prec,
                         const gw_opts* opts, double* R, double* eta);

/*
 * RPA density-response moments (Sec. 2.2): eta~^{(0)} = G D^-1 (I - 4 V^T
 * (I + 4 V D^-1 V^T)^-1 V D^-1) with G = G_main + G_offset by opts->nquad-point
 * mapped Gauss-Legendre quadrature, eta~^{(1)} = V D,
 * eta~^{(n)} = eta~^{(n-2)} (D^2 + 4 V^T V D).  Outputs as gw_moments_tda.
 * The quadrature is FP64 for either prec.  GW_MIXED with eta NULL: the
 * recursion on the even and odd chains, R_n = eta~^{(n)} V^T (upper tiles,
 * mirrored) and eta~^{(n+2)} = D^2 o eta~^{(n)} + 4 R_n (V o D), uses the
 * four-digit int8 operands of gw_moments_tda with exact int32 sums combined in
 * FP64; with eta requested the FP64 form is used.  GW_MIXED needs
 * naux <= 32768.
 */
gw_status gw_moments_rpa(gw_handle h, int nocc, int nvir, int naux, int nmom_max,
                         const double* eps, const double* L, gw_precision prec,
                         const gw_opts* opts, double* R, double* eta);

/*
 * Self-energy moments (eqs. convolution_occ, convolution_vir, w_moments) for
 * n = 0..nmom_max, for a closed-shell reference (factor 2 from the spin sum):
 *   Sigma^{(n,<)}_pq = 2 sum_t C(n,t) (-1)^t sum_{k occ} eps_k^{n-t} W^{(t)}_{pk,qk}
 *   Sigma^{(n,>)}_pq = 2 sum_t C(n,t)         sum_{c vir} eps_c^{n-t} W^{(t)}_{pc,qc}
 *   W^{(t)}_{px,qx}  = sum_PQ L[P][p][x] R_t[P][Q] L[Q][q][x]
 * with R_t from the chosen screening.  Outputs (symmetric):
 *   sigma_occ, sigma_vir  [nmom_max+1][nmo][nmo].
 * prec GW_MIXED: the moments R_t as gw_moments_tda / gw_moments_rpa in
 * GW_MIXED, and both contraction stages (R_t L with the eps-power fold, then
 * the sum over x and P) on four-digit int8 operands (base 255, one
 * power-of-two scale per row or column) on the integer MFMA with exact int32
 * sums per digit weight, combined in FP64; the folded intermediate is kept as
 * FP32 + BF16 residual.  GW_MIXED needs nmom_max <= 11 and naux <= 4096.
 */
gw_status gw_sigma_moments(gw_handle h, gw_screening screening, int nocc, int nvir,
                           int naux, int nmom_max, const double* eps, const double* L,
                           gw_precision prec, const gw_opts* opts,
                           double* sigma_occ, double* sigma_vir);

/*
 * Self-energy moments from given aux-space cores R[nmom_max+1][naux][naux]
 * (the contraction stage alone, same outputs as gw_sigma_moments).
 */
gw_status gw_sigma_from_R(gw_handle h, int nocc, int nvir, int naux, int nmom_max,
                          const double* eps, const double* L, const double* R,
                          gw_precision prec, const gw_opts* opts,
                          double* sigma_occ, double* sigma_vir);

/*
 * Allocation-free self-energy moments, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same result as gw_sigma_moments with
 * GW_TDA screening and GW_FP64 precision (half-order moments, then both
 * contraction stages), computed with the same kernels; every scratch buffer
 * (V, D, X, R_t, split-K partials, the folded intermediate) is carved from
 * one static device array of GW_NOALLOC_SCRATCH_BYTES per device, which the
 * library holds until the process ends.  The call itself allocates no device
 * memory and calls no allocating library routine; the caller passes eps, L
 * and the outputs sigma_occ, sigma_vir [nmom_max+1][nmo][nmo] as in
 * gw_sigma_moments.  Returns GW_EINVAL (nothing launched) when the system's
 * buffers do not fit the static array: roughly
 *   8 (2 naux nocc nvir + (nmom_max+2) naux^2 + (nmom_max+1) naux nmo^2
 *      + 2 (nmom_max+1) nmo^2) bytes must not exceed it.
 * Every call on one device shares that device's array and leaves its
 * contents behind (the path clears what must start at zero itself): calls
 * that overlap on one device race, whatever their handles or streams.
 */
#define GW_NOALLOC_SCRATCH_BYTES (64u << 20)

gw_status gw_sigma_moments_noalloc(gw_handle h, int nocc, int nvir, int naux, int nmom_max,
                                   const double* eps, const double* L,
                                   double* sigma_occ, double* sigma_vir);

/*
 * Auxiliary poles and upfolded Hamiltonian (eq. effH; eqs. ret_GF and
 * quasiparticle_energy_update), all FP64 on the device.
 * Per sector, block Lanczos on the moments gives (nmom_max+1)/2 blocks;
 * the block tridiagonal matrix is diagonalised and its poles coupled back
 * through B0 = (Sigma^{(0)})^{1/2}.  Poles whose coupling norm is below
 * 1e-14 of the largest are dropped.  Then
 *   H~ = [[fock, v_occ, v_vir], [v_occ^T, diag e_occ, 0], [v_vir^T, 0, diag e_vir]]
 * is diagonalised; the QP energy of orbital p is E_alpha with
 * alpha = argmax_beta chi_{p beta}^2 (lowest alpha on ties), its weight chi_{p alpha}^2.
 * Inputs:  sigma_occ, sigma_vir [nmom_max+1][nmo][nmo]; fock [nmo][nmo].
 * Outputs (cap = nmo*(nmom_max+1)/2 poles per sector, dim_max = nmo*(nmom_max+2)):
 *   npole_occ, npole_vir  host ints: poles kept per sector;
 *   pole_e  [2*cap]            occupied poles then virtual (packed);
 *   pole_v  [nmo][2*cap]       couplings, columns packed like pole_e;
 *   E       [dim_max]          eigenvalues of H~ (first nmo+npole_occ+npole_vir valid, ascending);
 *   chi     [nmo][dim_max]     physical rows of the eigenvectors (nullable);
 *   qp_e, qp_w [nmo]           QP energies and weights.
 * Numerics: the moments are first mapped to those of e' = (e - c)/s (c the
 * weighted mean pole energy, s the weighted spread), T[0] is pseudo-inverted
 * below pinv_tol times its largest eigenvalue, and B_j^2 eigenvalues below
 * max(pinv_tol |S2|_F, moment_eps (sum_k |Rhat_k|_F)^2 max_n |S^(n)|_F) are
 * deflated (the rounding level of the moment cancellations).
 * Returns GW_ENUMERIC if a moment matrix is not PSD beyond neg_tol (or ten
 * times the deflation level) or an eigensolve fails.
 */
gw_status gw_poles(gw_handle h, int nmo, int nmom_max, const double* sigma_occ,
                   const double* sigma_vir, const double* fock, const gw_opts* opts,
                   int* npole_occ, int* npole_vir, double* pole_e, double* pole_v,
                   double* E, double* chi, double* qp_e, double* qp_w);

/*
 * Symmetric eigensolver behind the pole stage (Sec. 2.3: the square roots and
 * pseudo-inverses of the Lanczos blocks and the block tridiagonal sector
 * matrices; Sec. 2.4: the upfolded Hamiltonian H~), and behind the Fock,
 * qsGW and natural-auxiliary eigensolves.  Householder tridiagonalisation in
 * the library's own kernels (two launches per column), then divide and
 * conquer on the tridiagonal matrix and the back-transformation (rocSOLVER
 * dstedc, dormtr).
 *   A [n][n] (device, row-major, symmetric; only the lower triangle of the
 *            row-major view is read) is overwritten: row i = eigenvector i
 *            (unit norm, sign unspecified);
 *   w [n]    (device) eigenvalues ascending.
 * Returns GW_EINVAL for n < 1 or null pointers, GW_ENUMERIC when the
 * tridiagonal eigensolver does not converge.  Synchronises the stream.
 */
gw_status gw_eigh(gw_handle h, int n, double* A, double* w);

/*
 * Fock / chemical-potential self-consistent GW (Sec. 3.6, Alg. 2).
 * The loop state is the Fock matrix F in the reference MO basis (eps, L).
 * Outer iteration: diagonalise F (orbital energies e, orbitals C), rotate
 * L_P <- C^T L_P C, build the self-energy moments (screening, precision as in
 * gw_sigma_moments) and the auxiliary poles (as in gw_poles); then the Fock
 * loop in that basis, from diag(e):
 *   zeta with Tr rho = N_e = 2 nocc, where rho = 2 sum_{a<n} chi_a chi_a^T over
 *   the n lowest eigenvectors of H~ = [[F, W], [W^T, diag(e_aux + zeta)]] and
 *   n minimises |2 sum_{a<n} |chi_a|^2 - N_e| (Aufbau); zeta is searched in
 *   [zeta_lo, zeta_hi], starting from +-1e-3 Ha around the previous zeta, to
 *   zeta_tol electrons or a 1e-13 Ha bracket (the end with the smaller
 *   residual when the interval holds no root);
 *   F <- h + J[rho] - K[rho]/2 with density-fitted J, K and the core
 *   Hamiltonian h = diag(eps) - (J[rho0] - K[rho0]/2), rho0 = 2 diag(1_occ);
 *   DIIS over the Fock matrices (diis_space vectors) with error vectors
 *   rho_k - rho_{k-1}, until max |rho_k - rho_{k-1}| < fock_tol.
 * The QP energies of H~ (as in gw_poles) end the iteration; the loop stops
 * when the Fock matrix it returns differs from the one it started from (the
 * first iteration: F0) by less than tol (Ha) in every element.
 * Inputs (device): eps [nmo], L [naux][nmo][nmo], F0 [nmo][nmo] or NULL for
 * diag(eps) (a warm start).  Outputs (device): F [nmo][nmo] (reference basis),
 * qp_e, qp_w [nmo] of the last iteration; info (host, nullable) the counts.
 * Options: NULL or zero fields take the defaults in brackets.  Returns
 * GW_ENOCONV (outputs still written) when max_outer is reached, the errors
 * of gw_sigma_moments and gw_poles otherwise.  Synchronises the stream.
 */
typedef struct {
    double tol;        /* outer: max |change of F (reference basis)| per iteration [1e-6 Ha] */
    int max_outer;     /* [30] */
    int max_fock;      /* Fock-loop steps per outer iteration [50] */
    double fock_tol;   /* max |density change| ending the Fock loop [1e-8] */
    int diis_space;    /* [12] */
    double zeta_tol;   /* electron-number tolerance of the zeta search [1e-13] */
    double zeta_lo;    /* zeta bracket [-1, 1] Ha (used when zeta_hi > zeta_lo) */
    double zeta_hi;
} gw_fsgw_opts;

typedef struct {
    int iterations;    /* outer iterations (self-energy rebuilds) */
    int fock_steps;    /* Fock-loop steps, all iterations */
    int eig_calls;     /* eigensolves of H~ */
    int converged;
    double zeta;       /* final auxiliary shift */
    double last_dqp;   /* sorted-QP change of the last iteration (-1 after one iteration; reported only) */
    double last_dF;    /* max |change of F| of the last iteration (the convergence test) */
} gw_fsgw_info;

gw_status gw_fsgw(gw_handle h, gw_screening screening, int nocc, int nvir, int naux,
                  int nmom_max, const double* eps, const double* L, const double* F0,
                  gw_precision prec, const gw_opts* opts, const gw_fsgw_opts* fopts,
                  double* F, double* qp_e, double* qp_w, gw_fsgw_info* info);

/*
 * Natural auxiliary functions (Sec. 2.1, eq. NAF).  M_PQ = sum_{vw} L[P][v][w]
 * L[Q][v][w] over the particle-hole pairs (v, w) = (i, nocc + a), each once
 * (full_space = 0), or over all nmo^2 pairs (full_space = 1); its eigenvectors
 * with eigenvalue > eps_naf (absolute) span the NAF basis, and
 *   L_naf[k][p][q] = sum_P U[P][k] L[P][p][q],  k = 0 .. nnaf-1,
 * kept vectors in ascending eigenvalue order (each vector's sign is that of
 * the eigensolver).  Any of the moment / self-energy entry points can then be
 * called with naux = nnaf and L_naf.
 * Inputs: L device [naux][nmo][nmo].  Outputs: L_naf device, capacity
 * [naux][nmo][nmo] (the first nnaf slabs are written); nnaf host; eigenvalues
 * device [naux] (all eigenvalues of M, ascending; nullable).
 * GW_ENUMERIC if no eigenvalue exceeds eps_naf.
 */
gw_status gw_naf(gw_handle h, int nocc, int nvir, int naux, const double* L, double eps_naf,
                 int full_space, double* L_naf, int* nnaf, double* eigenvalues);

/*
 * Quasiparticle self-consistent GW (Sec. 3.3, App. A Alg. A2).  The state is
 * the quasiparticle mean field: orbitals C (columns, reference MO basis) and
 * energies e, from C = 1, e = eps.  One iteration: the self-energy moments
 * and auxiliary poles (e_l, v_pl) of a one-shot calculation in the basis C
 * with energies e (screening, precision as in gw_sigma_moments); the static
 * potential at eps_p = e_p, D_pl = e_p - e_l,
 *   scheme 0 (SRG, eq. qsgw_se_srg):
 *     V_pq = sum_l v_pl v_ql (D_pl + D_ql)/(D_pl^2 + D_ql^2) (1 - exp(-(D_pl^2 + D_ql^2) s)),
 *   scheme 1 (Lorentzian, eq. qsgw_v with the real part of eq. qsgw_se_eta):
 *     V_pq = 1/2 sum_l v_pl v_ql [D_pl/(D_pl^2 + delta^2) + D_ql/(D_ql^2 + delta^2)];
 * the potential that enters the SCF is the DIIS extrapolation (space
 * outer_diis) over the potentials C V C^T built so far, error vector
 * V_out - V_in (the potential just built minus the one that entered the
 * previous SCF, zero at the start), or C V C^T itself when outer_diis < 0;
 * then the self-consistent field of eq. qp_scf, (f[rho] + V_in) C' = C' e',
 * f[rho] = h + J[rho] - K[rho]/2 with the core Hamiltonian of gw_fsgw
 * (f[rho0] = diag(eps)), rho = 2 sum_{i<nocc} C'_i C'_i^T, DIIS over the Fock
 * matrices with the commutator F rho - rho F as error, until the density
 * changes by less than scf_tol.  Converged when the sorted e change by less
 * than tol.  The QP energies are the final mean-field energies (unit weights).
 * Inputs (device): eps [nmo], L [naux][nmo][nmo].  Outputs (device): qp_e [nmo]
 * ascending; C [nmo][nmo] (C[p][k]: reference orbital p in QP orbital k;
 * nullable); F [nmo][nmo] = f[rho] + V_in in the reference basis (nullable);
 * info host (nullable).  Returns GW_ENOCONV (outputs still written) when
 * max_iter is reached.  Synchronises the stream.
 */
typedef struct {
    int scheme;        /* 0: SRG [default], 1: Lorentzian */
    double srg_s;      /* SRG flow parameter s [500 Ha^-2] */
    double delta;      /* Lorentzian broadening [1e-3 Ha] */
    double tol;        /* max |change of the sorted mean-field energies| [1e-6 Ha] */
    int max_iter;      /* [30] */
    int max_scf;       /* SCF steps per iteration [200] */
    double scf_tol;    /* max |density change| ending the SCF [1e-10] */
    int diis_space;    /* SCF DIIS space [12] */
    int outer_diis;    /* DIIS space over the static potential [0 -> 12]; < 0: none */
} gw_qsgw_opts;

typedef struct {
    int iterations;    /* self-energy rebuilds */
    int scf_steps;     /* SCF steps, all iterations */
    int converged;
    double last_change;
} gw_qsgw_info;

gw_status gw_qsgw(gw_handle h, gw_screening screening, int nocc, int nvir, int naux, int nmom_max,
                  const double* eps, const double* L, gw_precision prec, const gw_opts* opts,
                  const gw_qsgw_opts* qopts, double* qp_e, double* C, double* F, gw_qsgw_info* info);

/*
 * Spectral function of the upfolded Green's function (eqs. ret_GF, spectrum).
 * From the eigenpairs (E_a, chi) of H~, each pole carrying one broadening
 * delta > 0,
 *   G_pp(w)  = sum_a chi_{pa}^2 / (w - E_a + i delta),
 *   A_p(w)   = -(1/pi) Im G_pp(w) = (delta/pi) sum_a chi_{pa}^2 / ((w - E_a)^2 + delta^2),
 *   A(w)     = sum_p A_p(w).
 * Inputs (device): E [dim]; chi [nmo][ld_chi] (physical rows of the
 * eigenvectors, ld_chi >= dim; gw_poles writes ld_chi = nmo*(nmom_max+2));
 * omega [nomega] (Ha).  Outputs (device; either may be NULL, not both):
 * A [nomega]; A_orb [nmo][nomega].  FP64, asynchronous on the handle's stream.
 */
gw_status gw_spectral(gw_handle h, int nmo, int dim, int ld_chi, const double* E, const double* chi,
                      int nomega, const double* omega, double delta, double* A, double* A_orb);

/*
 * Aufbau filling of the eigenstates of H~ and the correlated density matrix
 * (eq. density): the n lowest states are filled, n minimising
 * |2 sum_{a<n} |chi_a|^2 - nelec| (lowest n on ties), and
 *   rho = 2 sum_{a<n} chi_a chi_a^T.
 * The Dyson orbitals (MO basis) of the ionisation and of the attachment are
 * columns homo = n-1 and lumo = n of chi; their squared norms are the pole
 * strengths, -E[homo] and -E[lumo] the ionisation energy and the electron
 * affinity.  Inputs (device): E [dim] ascending, chi [nmo][ld_chi].
 * Outputs: rho device [nmo][nmo] (nullable); info host (nullable).
 * GW_EINVAL if E is not ascending.  Synchronises the stream.
 */
typedef struct {
    int nfill;      /* filled states n */
    double nelec;   /* 2 sum_{a<n} |chi_a|^2 */
    double mu;      /* midway between E[homo] and E[lumo] (the existing one if n = 0 or dim) */
    int homo;       /* n - 1, or -1 */
    int lumo;       /* n, or -1 if n = dim */
} gw_aufbau_info;

gw_status gw_aufbau(gw_handle h, int nmo, int dim, int ld_chi, const double* E, const double* chi,
                    double nelec, double* rho, gw_aufbau_info* info);

/*
 * Electron-number conserving one-shot GW (Sec. 3.5): every auxiliary energy
 * (the diagonal of d~) is shifted by zeta, the physical block fixed, until the
 * Aufbau filling of H~(zeta) (as in gw_aufbau) holds nelec electrons.  The
 * shift is searched from 0 outwards: bracket +-1e-3 Ha, widened tenfold
 * within [zeta_lo, zeta_hi] until Tr rho - nelec changes sign, then false
 * position (Illinois) with bisection safeguards, to zeta_tol electrons or a
 * 1e-13 Ha bracket; without a sign change, the end with the smaller residual.
 * Inputs (device): fock [nmo][nmo]; pole_e, pole_v as gw_poles writes them for
 * the same nmo and nmom_max (npole_occ + npole_vir packed columns, leading
 * dimension nmo*(nmom_max+1)).  Outputs (device): E, chi (nullable), qp_e,
 * qp_w as in gw_poles, at the final zeta; info host (nullable).
 * Synchronises the stream.
 */
typedef struct {
    double zeta_lo, zeta_hi;   /* search interval [-1, 1] Ha (used when zeta_hi > zeta_lo) */
    double zeta_tol;           /* electrons [1e-13] */
} gw_zeta_opts;

typedef struct {
    double zeta;     /* final shift (Ha) */
    int nfill;       /* filled states of H~(zeta) */
    double nelec;    /* their electron count */
    int eig_calls;   /* eigensolves of H~ */
} gw_zeta_info;

gw_status gw_zeta_shift(gw_handle h, int nmo, int nmom_max, int npole_occ, int npole_vir, const double* fock,
                        const double* pole_e, const double* pole_v, double nelec, const gw_zeta_opts* zopts,
                        double* E, double* chi, double* qp_e, double* qp_w, gw_zeta_info* info);

/*
 * Eigenvalue self-consistent moment GW (App. A, Alg. A1).  Two sets of orbital
 * energies start at eps: eps_G enters the eps-power factors of the self-energy
 * convolution (eqs. convolution_occ / convolution_vir), eps_W the energy
 * differences of the density-response recursion (eq. energy_differences).
 * Each iteration runs gw_moments_* (on eps_W), the self-energy moments (on
 * eps_G) and gw_poles with fock = diag(eps) (eq. StaticSE with Sigma_inf = 0),
 * then sets eps_G (unless g0) and eps_W (unless w0) to the QP energies, or,
 * with diis_space > 0, to the Pulay (DIIS) extrapolation over the last
 * diis_space pairs (QP energies, QP energies - energies they came from).
 * g0 = w0 = 0: evGW; w0 = 1: evGW0 (W of the reference); g0 = w0 = 1: one
 * G0W0 evaluation.  Converged when, for every quasiparticle-like orbital (QP
 * weight >= 0.9 in both iterations; all orbitals if none is), the QP energy
 * differs by at most tol from the energy that went into the iteration (for
 * the plain loop: its change since the previous iteration).  When
 * opts->moment_eps is not set (<= 0) the loop's block Lanczos deflates at
 * 1e-12 (FP64) or 1e-9 (mixed) instead of 2^-52: directions resolved from
 * the moments' rounding noise give satellite poles whose QP assignment moves
 * by ~1e-5 Ha between iterations.
 * Outputs (device, [nmo]): qp_e, qp_w of the last iteration.  GW_ENOCONV
 * after max_iter iterations (outputs and info still written); GW_ENUMERIC if
 * the QP energies of occupied and virtual orbitals cross (the next screening
 * would have D <= 0).
 */
typedef struct {
    int g0;          /* 1: keep eps_G at the reference */
    int w0;          /* 1: keep eps_W at the reference */
    int max_iter;    /* <= 0 -> 30 */
    double tol;      /* Ha; <= 0 -> 1e-6 */
    int diis_space;  /* DIIS vectors; 0 -> 12 (the paper's setting), < 0: plain loop */
} gw_evgw_opts;

typedef struct {
    int iterations;
    int converged;
    double last_change;  /* fixed-point residual of the last iteration (see above) */
} gw_evgw_info;

gw_status gw_evgw(gw_handle h, gw_screening screening, int nocc, int nvir, int naux,
                  int nmom_max, const double* eps, const double* L, gw_precision prec,
                  const gw_opts* opts, const gw_evgw_opts* eopts, double* qp_e, double* qp_w,
                  gw_evgw_info* info);

/*
 * Batched self-energy moments for many molecules (as gw_sigma_moments for
 * each).  gw_batch_create plans the batch once: per-molecule buffers; x
 * chunks of each molecule ("jobs") whose stage-1 intermediates fit job_bytes;
 * waves of consecutive jobs that fit wave_bytes.  In mixed precision each wave
 * is one grouped, persistent launch per contraction stage over a work queue of
 * (job, tile) items; contraction splits follow a work-item target
 * (split_target, or with autotune the fastest of 256, 512, 1024, 2048 by
 * timing the whole sequence), and the contraction tile is 128 x 64, or 64 x
 * 64 for molecules with nmo <= small_tile_nmo (autotune: then the fastest
 * of 0, 100, 150, 200 and every molecule; when every job of a wave has 64-row
 * tiles the launch holds two work groups per CU).  For TDA the per-molecule
 * work (recursion,
 * digit preparation) of different molecules runs on `branches` streams with
 * their own workspaces, molecules assigned largest first by nmo^4.  The
 * sequence is run once eagerly (the outputs
 * are valid when create returns) and, for TDA screening unless no_graph is
 * set, captured into a hipGraph; gw_batch_run replays it on the handle's
 * current stream (RPA, or no_graph: re-enqueued).  Pointers in sys are used
 * as given at creation: the caller keeps them alive and may change the
 * contents of eps and L between runs.  Errors as gw_sigma_moments, checked
 * for every molecule before anything runs; GW_ENOMEM if the plan's buffers do
 * not fit.
 */
typedef struct {
    int nocc, nvir, naux;
    const double* eps;   /* device [nmo] */
    const double* L;     /* device [naux][nmo][nmo] */
    double* sigma_occ;   /* device [nmom_max+1][nmo][nmo] (output) */
    double* sigma_vir;
} gw_system;

typedef struct {
    size_t job_bytes;    /* stage-1 intermediates per job [4 GiB] */
    size_t wave_bytes;   /* per grouped launch [24 GiB] */
    int split_target;    /* contraction work items per job [512] */
    int autotune;        /* 1: choose split_target by timing */
    int no_graph;        /* 1: replay by re-enqueueing */
    int branches;        /* TDA: concurrent streams for the per-molecule work [4]; 1 = serial */
    int small_tile_nmo;  /* mixed: molecules with nmo <= this use 64-row contraction tiles [0];
                            autotune also chooses it among 0, 100, 150, 200 */
} gw_batch_opts;

typedef struct gw_batch_s* gw_batch;

gw_status gw_batch_create(gw_handle h, int nsys, const gw_system* sys, gw_screening screening,
                          int nmom_max, gw_precision prec, const gw_opts* opts,
                          const gw_batch_opts* bopts, gw_batch* batch);
gw_status gw_batch_run(gw_batch batch);
/* Plan facts (host ints, each nullable): jobs, waves, graph captured (0/1), split target,
 * the largest nmo that uses 64-row contraction tiles (0: none). */
gw_status gw_batch_info(gw_batch batch, int* njobs, int* nwaves, int* graph, int* split_target,
                        int* small_tile_nmo);
gw_status gw_batch_destroy(gw_batch batch);

/*
 * Learned warm start for gw_fsgw (not in the paper): a per-orbital MLP
 * 3 -> 128 -> 128 -> 128 -> 1 with SiLU after each hidden layer, FP32, that
 * predicts s_p ~ F*_pp - eps_p (the diagonal of the converged Fock matrix in
 * the reference basis) from the features of gw_mlp_features; the warm start
 * is F0 = diag(eps + s).
 * params: one flat float vector of gw_mlp_param_count() = 33665 values, in the
 *   order W1 [128][3], b1 [128], W2 [128][128], b2, W3 [128][128], b3,
 *   W4 [1][128], b4 (row-major, W[out][in]).
 * norm [8] (device floats): input mean [3], input std [3], target mean,
 *   target std.  Inputs are standardised, the output is mapped back to target
 *   units: y = norm[6] + norm[7] * out; the loss is mean(((y - t)/norm[7])^2).
 * act [6][rows][128]: z1, a1, z2, a2, z3, a3 of the forward pass (kept for
 *   gw_mlp_backward); NULL in gw_mlp_forward uses library workspace.
 * All pointers are device pointers; calls are asynchronous on the handle's
 * stream.  GW_EINVAL for rows < 1 or null required pointers.
 */
long gw_mlp_param_count(void);

/* feat [nmo][3] = (eps_p, sum_{P,q} L[P][p][q]^2, eps_p - (eps_{nocc-1} + eps_nocc)/2) */
gw_status gw_mlp_features(gw_handle h, int nocc, int nvir, int naux, const double* eps,
                          const double* L, float* feat);

/* y [rows] from x [rows][3] */
gw_status gw_mlp_forward(gw_handle h, int rows, const float* params, const float* norm,
                         const float* x, float* act, float* y);

/* grad [33665] of the loss at (x, target) from a forward pass (act, y) on the
 * same x with the same params; loss [1] (nullable) receives the loss value. */
gw_status gw_mlp_backward(gw_handle h, int rows, const float* params, const float* norm,
                          const float* x, const float* act, const float* y,
                          const float* target, float* grad, float* loss);

/* norm [8] from training rows: the column means and standard deviations
 * (population, floored at 1e-12) of x [rows][3], then the mean and standard
 * deviation of the targets t [rows]; FP64 sums in a fixed order. */
gw_status gw_mlp_norm(gw_handle h, int rows, const float* x, const float* t, float* norm);

/* t [nmo] = F[p][p] - eps[p]: the training target from a converged fsGW Fock
 * matrix F [nmo][nmo] (reference basis, as returned by gw_fsgw). */
gw_status gw_mlp_target(gw_handle h, int nmo, const double* F, const double* eps, float* t);

/* F0 [nmo][nmo] = diag(eps + y), y the model's prediction (params, norm) from
 * the features of (eps, L) (gw_mlp_features): the warm start of gw_fsgw.
 * nmo = nocc + nvir; L [naux][nmo][nmo]. */
gw_status gw_mlp_warm_start(gw_handle h, int nocc, int nvir, int naux, const double* eps, const double* L,
                            const float* params, const float* norm, double* F0);

/* One Adam step (step counts from 1, bias-corrected) on params with moment
 * buffers m, v [33665] (zero before the first step). */
gw_status gw_mlp_adam(gw_handle h, int step, float lr, float beta1, float beta2, float eps,
                      float* params, const float* grad, float* m, float* v);

/*
 * Per-kernel timing for measurement.  While enabled, every launch of the
 * instrumented kernel families is bracketed by HIP events recorded on the
 * handle's stream (the stream the kernels run on).  Families:
 *   "sigma_fold"     stage 1 of the self-energy contraction (R_t L with the eps-power fold)
 *   "sigma_contract" stage 2 (sum over P and x of L Zt)
 *   "recur_xvt"      R_n = eta~^{(n)} V^T
 *   "recur_rv"       eta~ updates  D o X + c R V
 *   "recur_rr"       2 R_k R_k terms of the half-order TDA moments
 *   "recur_digits"   (mixed precision) scales and digit planes of the recursion operands
 *   "rpa_quad"       RPA quadrature products (Q/T matrices and the G product)
 *   "mixed_prep"     (mixed precision) scales and digit planes of L and R_t
 *   "mixed_zdig"     (mixed precision) scales and digit planes of the stage-1 result
 * gw_timing_read synchronises the stream, then returns the summed duration
 * (ms) and the launch count of one family since the last reset.
 */
gw_status gw_timing_enable(gw_handle h, int enable);
gw_status gw_timing_reset(gw_handle h);
gw_status gw_timing_read(gw_handle h, const char* family, double* total_ms, long* launches);

#ifdef __cplusplus
}
#endif

#endif /* GWMOM_H */
