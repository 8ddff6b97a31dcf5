"""Fock / chemical-potential self-consistent moment GW (paper Sec. 3.6, Alg. 2),
oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Readings of the algorithm box taken here (it gives the loop structure, not
its numerics):
  * the reference is Hartree-Fock-like: with rho0 = 2 diag(1_occ) the core
    Hamiltonian is h = diag(eps) - (J[rho0] - K[rho0]/2), so F[rho0] = diag(eps);
    J and K are the density-fitted Coulomb and exchange matrices of L;
  * electron number (eq. density): the lowest n eigenstates of H~ are filled,
    n chosen to minimise |2 sum_{alpha<n} |chi_alpha|^2 - N_e| (Aufbau);
  * zeta (the shift of the auxiliary poles) is found by bisection of
    Tr rho(zeta) - N_e on [-1, 1] Ha, to 1e-13 electrons or a 1e-13 Ha
    bracket: Tr rho is flat in zeta, and a looser electron count leaves zeta,
    and with it rho, uncertain above the density tolerance of the Fock loop;
  * the Fock loop is a DIIS (12 vectors) extrapolation of the Fock matrices
    F[rho_k] with error vectors rho_k - rho_{k-1}; zeta is re-optimised at
    every Fock step (order="interleaved", the default and the device's
    order), and the loop ends when the density stops changing (max element
    below fock_tol), so at convergence F = F[rho] and Tr rho = N_e.  The
    algorithm box nests the two instead: a Fock loop at fixed zeta inside a
    loop over the electron number (order="nested": zeta from the current F,
    the Fock loop to convergence at that zeta, zeta again from the converged
    F, until zeta stops moving).  Both end at the same fixed point
    (F = F[rho], Tr rho(zeta) = N_e); the interleaved order reaches it in
    fewer Fock steps;
  * an outer iteration diagonalises the converged F, rotates L into its
    eigenbasis and rebuilds the self-energy moments there; the outer loop
    stops when the Fock matrix it returns (reference basis) differs from the
    one it started from by less than `tol` Ha in every element (the first
    iteration against F0): a fixed point of the rebuild.  The sorted QP
    energies are not the test: orbitals embedded in satellite bands (QP
    weight < 0.9) change their assignment between iterations at the 1e-6 Ha
    level near the fixed point, and a loop judged on them can wander.
"""
from __future__ import annotations

import numpy as np

from . import gw


def jk(L: np.ndarray, rho: np.ndarray):
    """J_pq = sum_P L[P,p,q] sum_rs L[P,r,s] rho_rs,  K_pq = sum_P (L_P rho L_P)_pq."""
    v = np.einsum("Prs,rs->P", L, rho)
    J = np.einsum("P,Ppq->pq", v, L)
    K = np.einsum("Ppr,rs,Psq->pq", L, rho, L, optimize=True)
    return J, K


def core_hamiltonian(eps: np.ndarray, L: np.ndarray, nocc: int):
    rho0 = np.diag(np.r_[np.full(nocc, 2.0), np.zeros(eps.shape[0] - nocc)])
    J, K = jk(L, rho0)
    return np.diag(eps) - (J - 0.5 * K)


def fock(h, L, rho):
    J, K = jk(L, rho)
    return h + J - 0.5 * K


def upfolded(F, e_aux, W, zeta):
    nmo = F.shape[0]
    n = nmo + e_aux.shape[0]
    H = np.zeros((n, n))
    H[:nmo, :nmo] = F
    H[:nmo, nmo:] = W
    H[nmo:, :nmo] = W.T
    H[nmo:, nmo:] = np.diag(e_aux + zeta)
    return H


def aufbau(E, chi, nelec):
    """Fill the lowest n states; n minimises |2 sum_{a<n} |chi_a|^2 - nelec|."""
    w = (chi * chi).sum(axis=0)
    cum = np.r_[0.0, 2.0 * np.cumsum(w)]
    n = int(np.argmin(np.abs(cum - nelec)))
    rho = 2.0 * chi[:, :n] @ chi[:, :n].T
    return rho, n


def density(F, e_aux, W, zeta, nelec):
    E, U = np.linalg.eigh(upfolded(F, e_aux, W, zeta))
    chi = U[: F.shape[0]]
    rho, n = aufbau(E, chi, nelec)
    return rho, E, chi


def trace_density(F, e_aux, W, zeta, nelec):
    return float(np.trace(density(F, e_aux, W, zeta, nelec)[0]))


def solve_zeta(F, e_aux, W, nelec, lo=-1.0, hi=1.0, tol=1e-13, maxit=100):
    """Root of Tr rho(zeta) - nelec on [lo, hi] by bisection, to tol electrons
    (or a bracket narrower than 1e-13 Ha).  Raising zeta lifts the auxiliary
    poles, which moves weight onto the physical states, so the count is
    non-decreasing in zeta; without a sign change the end with the smaller
    residual is returned."""
    flo = trace_density(F, e_aux, W, lo, nelec) - nelec
    fhi = trace_density(F, e_aux, W, hi, nelec) - nelec
    if flo * fhi > 0:
        return lo if abs(flo) < abs(fhi) else hi
    if flo == 0.0:
        return lo
    if fhi == 0.0:
        return hi
    best, fbest = (lo, flo) if abs(flo) < abs(fhi) else (hi, fhi)
    for _ in range(maxit):
        mid = 0.5 * (lo + hi)
        fm = trace_density(F, e_aux, W, mid, nelec) - nelec
        if abs(fm) < abs(fbest):
            best, fbest = mid, fm
        if abs(fm) < tol or hi - lo < 1e-13:
            break
        if (flo < 0) == (fm < 0):
            lo, flo = mid, fm
        else:
            hi, fhi = mid, fm
    return best


class DIIS:
    """Pulay extrapolation: keep the last `space` pairs (x_i, e_i) and return
    sum_i c_i x_i with sum_i c_i = 1 minimising |sum_i c_i e_i|^2."""

    def __init__(self, space=12):
        self.space = space
        self.vecs, self.errs = [], []

    def update(self, x, e):
        self.vecs.append(np.array(x, dtype=float))
        self.errs.append(np.array(e, dtype=float))
        if len(self.vecs) > self.space:
            self.vecs.pop(0)
            self.errs.pop(0)
        n = len(self.vecs)
        B = np.zeros((n + 1, n + 1))
        for i in range(n):
            for j in range(n):
                B[i, j] = np.vdot(self.errs[i], self.errs[j])
        B[n, :n] = B[:n, n] = -1.0
        rhs = np.zeros(n + 1)
        rhs[n] = -1.0
        try:
            c = np.linalg.solve(B, rhs)[:n]
        except np.linalg.LinAlgError:
            return self.vecs[-1].copy()
        return sum(ci * v for ci, v in zip(c, self.vecs))


def qp_energies(F, e_aux, W, zeta):
    E, U = np.linalg.eigh(upfolded(F, e_aux, W, zeta))
    qp, wt, _ = gw.qp_assign(E, U[: F.shape[0]])
    return qp, wt


def fock_loop_nested(hc, Lc, Fc, e_aux, W, nelec, rho_old, max_fock, fock_tol, diis_space, max_zeta=30,
                     zeta_tol=1e-10):
    """The inner loops of the algorithm box in its own nesting: zeta for the
    current Fock matrix, then the Fock loop (DIIS over F[rho_k], error
    rho_k - rho_{k-1}) at that fixed zeta until the density settles, then
    zeta again from the converged F; repeated until zeta moves by less than
    zeta_tol.  Returns (Fc, rho, zeta, fock_steps)."""
    steps = 0
    zeta = None
    rho = rho_old
    for _ in range(max_zeta):
        z_new = solve_zeta(Fc, e_aux, W, nelec)
        if zeta is not None and abs(z_new - zeta) < zeta_tol:
            zeta = z_new
            break
        zeta = z_new
        diis = DIIS(diis_space)
        for _ in range(max_fock):
            rho, _, _ = density(Fc, e_aux, W, zeta, nelec)
            Fn = fock(hc, Lc, rho)
            steps += 1
            err = rho - rho_old
            rho_old = rho
            if np.abs(err).max() < fock_tol:
                Fc = Fn
                break
            Fc = diis.update(Fn, err)
    return Fc, rho_old, zeta, steps


def fsgw(eps, L, nocc, nmom_max, screening="tda", F0=None, tol=1e-6, max_outer=30,
         max_fock=50, fock_tol=1e-8, diis_space=12, pinv_tol=1e-12, order="interleaved"):
    """Run fsGW from the reference (eps, L).  F0 (in the reference MO basis)
    warm-starts the loop; None means F0 = diag(eps).  order selects how zeta
    and the Fock loop are combined ("interleaved": zeta at every Fock step;
    "nested": the algorithm box's nesting, see fock_loop_nested).  Returns a
    dict with the converged Fock matrix F (reference basis), the sorted QP
    energies per outer iteration, the QP energies and weights per orbital of
    the last iteration (orbitals of the final F, ascending), the outer
    iteration count, the inner (Fock) step count and the last change of F."""
    if order not in ("interleaved", "nested"):
        raise ValueError(order)
    nmo = eps.shape[0]
    nelec = 2.0 * nocc
    h = core_hamiltonian(eps, L, nocc)
    F = np.diag(eps).copy() if F0 is None else np.array(F0, dtype=float)
    history = []
    fock_steps = 0
    converged = False
    for it in range(max_outer):
        # orbitals and energies of the current Fock matrix
        e_cur, C = np.linalg.eigh(F)
        Lc = np.einsum("ap,Pab,bq->Ppq", C, L, C, optimize=True)
        hc = C.T @ h @ C
        so, sv, _ = gw.gw_moments(e_cur, Lc, nocc, nmom_max, screening)
        eo, vo = gw.poles_from_moments(list(so), pinv_tol)
        ev, vv = gw.poles_from_moments(list(sv), pinv_tol)
        e_aux = np.concatenate([eo, ev])
        W = np.concatenate([vo, vv], axis=1)
        Fc = np.diag(e_cur)
        diis = DIIS(diis_space)
        # mean-field density of Fc = diag(e_cur) (ascending): the first error's reference
        rho_old = np.diag(np.r_[np.full(nocc, 2.0), np.zeros(nmo - nocc)])
        zeta = 0.0
        if order == "nested":
            Fc, rho_old, zeta, steps = fock_loop_nested(hc, Lc, Fc, e_aux, W, nelec, rho_old, max_fock, fock_tol,
                                                        diis_space)
            fock_steps += steps
        for _ in range(max_fock if order == "interleaved" else 0):
            zeta = solve_zeta(Fc, e_aux, W, nelec)
            rho, _, _ = density(Fc, e_aux, W, zeta, nelec)
            Fn = fock(hc, Lc, rho)
            fock_steps += 1
            err = rho - rho_old
            rho_old = rho
            if np.abs(err).max() < fock_tol:
                Fc = Fn
                break
            Fc = diis.update(Fn, err)
        qp, wt = qp_energies(Fc, e_aux, W, zeta)
        history.append(np.sort(qp))
        F_new = C @ Fc @ C.T
        last_dF = float(np.abs(F_new - F).max())
        F = F_new
        rho_ref = C @ rho_old @ C.T
        if last_dF < tol:
            converged = True
            break
    return dict(F=F, rho=rho_ref, qp=history[-1], qp_orb=qp, qp_weight=wt, history=history,
                iterations=len(history), fock_steps=fock_steps, converged=converged, zeta=zeta,
                last_dF=last_dF)
