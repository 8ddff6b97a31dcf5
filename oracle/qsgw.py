"""Quasiparticle self-consistent moment GW (paper Sec. 3.3, App. A Alg. A2),
oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The loop state is the quasiparticle mean field: orbitals C (columns, in the
reference MO basis) and energies eps_mf, starting from C = 1, eps_mf = eps.
One iteration:
  1. a one-shot GW in the basis C with the energies eps_mf (both in the
     screening and in the Green's function): L_P -> C^T L_P C, moments,
     auxiliary poles per sector (the block Lanczos output is already the
     diagonal representation of the external space: energies e_l, couplings
     v_{p l});
  2. the static potential V^Sigma from those poles at eps_p = eps_mf:
       Lorentzian (eq. qsgw_v with the real part of eq. qsgw_se_eta):
         V_pq = 1/2 sum_l v_pl v_ql [D_pl/(D_pl^2 + delta^2) + D_ql/(D_ql^2 + delta^2)],
       SRG (eq. qsgw_se_srg, the sum over l implicit in the printed form):
         V_pq = sum_l v_pl v_ql (D_pl + D_ql)/(D_pl^2 + D_ql^2) (1 - exp(-(D_pl^2 + D_ql^2) s)),
       with D_pl = eps_p - e_l (eq. qsgw_se_srg_delta); V^Sigma is moved to the
       reference basis as C V C^T;
  3. the self-consistent field of eq. qp_scf, (f[rho] + V^Sigma) C = C eps,
     with f[rho] = h + J[rho] - K[rho]/2 from the density-fitted integrals and
     the core Hamiltonian of the Fock-loop oracle (f[rho0] = diag(eps)),
     rho = 2 sum_{i<nocc} C_i C_i^T over the nocc lowest orbitals, DIIS over
     the Fock matrices with the commutator F rho - rho F as error, until the
     density changes by less than scf_tol (max element);
  4. converged when the sorted eps_mf change by less than tol.
The potential that enters step 3 is, as in the paper's other self-consistent
loops, a DIIS extrapolation (space outer_diis, default 12) over the potentials
built so far, with error vector V_out - V_in (the potential just built minus
the one that went into the previous SCF, V_in = 0 at the start); outer_diis <= 0
takes V_out as it is.

Readings taken here (the paper gives no values): SRG is the default with
s = 500 Ha^-2; the Lorentzian broadening defaults to delta = 1e-3 Ha; the QP
energies reported are the mean-field eps_mf (unit weights, the Green's
function the paper chooses for qsGW).
"""
from __future__ import annotations

import numpy as np

from . import fsgw, gw


def static_potential(eps_mf, e_aux, W, scheme="srg", s=500.0, delta=1e-3):
    """V^Sigma_pq from auxiliary poles (e_aux [n], W [nmo][n]) at the energies
    eps_mf, by eq. qsgw_se_srg (scheme 'srg') or by eq. qsgw_v with the real
    part of eq. qsgw_se_eta (scheme 'lorentzian')."""
    nmo = eps_mf.shape[0]
    V = np.zeros((nmo, nmo))
    for l in range(e_aux.shape[0]):
        d = eps_mf - e_aux[l]                          # D_pl for every p
        vv = np.outer(W[:, l], W[:, l])
        if scheme == "srg":
            x = d[:, None] ** 2 + d[None, :] ** 2
            with np.errstate(invalid="ignore", divide="ignore"):
                g = (d[:, None] + d[None, :]) / x * (1.0 - np.exp(-x * s))
            g[x == 0.0] = 0.0
        elif scheme == "lorentzian":
            a = d / (d * d + delta * delta)
            g = 0.5 * (a[:, None] + a[None, :])
        else:
            raise ValueError(scheme)
        V += vv * g
    return V


def scf(hcore, L, V, nocc, rho_start, scf_tol=1e-10, max_scf=200, diis_space=12):
    """Self-consistent field of eq. qp_scf: returns (eps, C, rho, F, steps)."""
    rho = rho_start.copy()
    diis = fsgw.DIIS(diis_space)
    for step in range(1, max_scf + 1):
        F = fsgw.fock(hcore, L, rho) + V
        Fx = diis.update(F, F @ rho - rho @ F)
        e, C = np.linalg.eigh(Fx)
        rho_new = 2.0 * C[:, :nocc] @ C[:, :nocc].T
        change = np.abs(rho_new - rho).max()
        rho = rho_new
        if change < scf_tol:
            break
    F = fsgw.fock(hcore, L, rho) + V
    e, C = np.linalg.eigh(F)
    return e, C, rho, F, step


def one_shot_poles(eps_mf, C, L, nocc, nmom_max, screening="tda"):
    """Step 1: auxiliary poles of the one-shot GW self-energy in the basis C."""
    Lc = np.einsum("pi,Ppq,qj->Pij", C, L, C, optimize=True)
    so, sv, _ = gw.gw_moments(eps_mf, Lc, nocc, nmom_max, screening)
    eo, vo = gw.poles_from_moments(list(so))
    ev, vv = gw.poles_from_moments(list(sv))
    return np.r_[eo, ev], np.concatenate([vo, vv], axis=1)


def qsgw(eps, L, nocc, nmom_max, screening="tda", scheme="srg", s=500.0, delta=1e-3, tol=1e-6,
         max_iter=30, scf_tol=1e-10, max_scf=200, diis_space=12, pole_fn=None, outer_diis=12):
    """Alg. A2.  pole_fn(eps_mf, C) may replace step 1 (the brute-force pins
    pass the exact self-energy poles).  Returns dict(qp, C, F, V, iterations,
    scf_steps, converged, last_change); V is the potential of the last SCF."""
    nmo = eps.shape[0]
    hcore = fsgw.core_hamiltonian(eps, L, nocc)
    C = np.eye(nmo)
    e_mf = np.array(eps, dtype=float)
    rho = np.diag(np.r_[np.full(nocc, 2.0), np.zeros(nmo - nocc)])
    converged, last, steps, it = False, -1.0, 0, 0
    F = np.diag(e_mf)
    V = np.zeros((nmo, nmo))
    outer = fsgw.DIIS(outer_diis) if outer_diis > 0 else None
    for it in range(1, max_iter + 1):
        if pole_fn is None:
            e_aux, W = one_shot_poles(e_mf, C, L, nocc, nmom_max, screening)
        else:
            e_aux, W = pole_fn(e_mf, C)
        Vc = static_potential(e_mf, e_aux, W, scheme, s, delta)
        V_out = C @ Vc @ C.T
        V = V_out if outer is None else outer.update(V_out, V_out - V)
        e_new, C_new, rho, F, n = scf(hcore, L, V, nocc, rho, scf_tol, max_scf, diis_space)
        steps += n
        last = float(np.abs(np.sort(e_new) - np.sort(e_mf)).max())
        e_mf, C = e_new, C_new
        if last < tol:
            converged = True
            break
    return dict(qp=e_mf, C=C, F=F, V=V, iterations=it, scf_steps=steps, converged=converged, last_change=last)
