"""Brute-force references for small systems (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Everything here diagonalises the full particle-hole problem, so it is
independent of the moment recursions it is used to pin:

* TDA (Sec. 2.3): A = D + 2 V^T V = X diag(Omega) X^T, eta^{(n)} = A^n.
* RPA (Sec. 2.2): Mcal = D^1/2 (D + 4 V^T V) D^1/2 = U diag(Omega^2) U^T,
  (X+Y) = D^1/2 U Omega^-1/2, eta^{(n)} = (X+Y) Omega^n (X+Y)^T.
* Exact G0W0 self-energy poles: with rho^nu_pq = sum_P L[P,p,q] (V (X+Y))[P,nu],
  hole poles at eps_k - Omega_nu with couplings sqrt(2) rho^nu_{p k} and particle
  poles at eps_c + Omega_nu with couplings sqrt(2) rho^nu_{p c}; the sqrt(2) is
  the closed-shell spin factor.
"""
from __future__ import annotations

import numpy as np


def tda_modes(V: np.ndarray, D: np.ndarray):
    A = np.diag(D) + 2.0 * V.T @ V
    Omega, X = np.linalg.eigh(A)
    return Omega, X


def rpa_modes(V: np.ndarray, D: np.ndarray):
    sD = np.sqrt(D)
    Mcal = sD[:, None] * (np.diag(D) + 4.0 * V.T @ V) * sD[None, :]
    w2, U = np.linalg.eigh(Mcal)
    Omega = np.sqrt(w2)
    XpY = sD[:, None] * U / np.sqrt(Omega)[None, :]
    return Omega, XpY


def eta_from_modes(Omega, XpY, nmom_max):
    """eta^{(n)} = (X+Y) Omega^n (X+Y)^T, n = 0..nmom_max (ov x ov)."""
    return [(XpY * Omega[None, :] ** n) @ XpY.T for n in range(nmom_max + 1)]


def exact_poles(eps, L, nocc, Omega, XpY):
    """Hole and particle poles of the exact (screened) G0W0 self-energy."""
    nmo = eps.shape[0]
    nvir = nmo - nocc
    V = np.ascontiguousarray(L[:, :nocc, nocc:]).reshape(L.shape[0], nocc * nvir)
    Z = V @ XpY                                        # [P, nu]
    rho = np.tensordot(Z, L, axes=(0, 0))              # rho[nu, p, q]
    nex = Omega.shape[0]
    e_occ = (eps[None, :nocc] - Omega[:, None]).reshape(-1)          # (nu, k)
    v_occ = np.sqrt(2.0) * rho[:, :, :nocc].transpose(1, 0, 2).reshape(nmo, nex * nocc)
    e_vir = (eps[None, nocc:] + Omega[:, None]).reshape(-1)          # (nu, c)
    v_vir = np.sqrt(2.0) * rho[:, :, nocc:].transpose(1, 0, 2).reshape(nmo, nex * nvir)
    return e_occ, v_occ, e_vir, v_vir


def moments_of_poles(e, v, nmom_max):
    """T^{(n)} = sum_lambda v_{p lambda} v_{q lambda} e_lambda^n."""
    return [(v * e[None, :] ** n) @ v.T for n in range(nmom_max + 1)]


def exact_upfolded(eps, e_occ, v_occ, e_vir, v_vir):
    """Exact upfolded Hamiltonian of full-frequency G0W0 with the given poles."""
    nmo = eps.shape[0]
    e_aux = np.concatenate([e_occ, e_vir])
    W = np.concatenate([v_occ, v_vir], axis=1)
    dim = nmo + e_aux.shape[0]
    H = np.zeros((dim, dim))
    H[:nmo, :nmo] = np.diag(eps)
    H[:nmo, nmo:] = W
    H[nmo:, :nmo] = W.T
    H[nmo:, nmo:] = np.diag(e_aux)
    return H


def exact_g0w0(eps, L, nocc, screening="tda"):
    """Exact QP spectrum of full-frequency G0W0 by diagonalising the exact
    upfolded Hamiltonian (tiny systems only)."""
    nmo = eps.shape[0]
    nvir = nmo - nocc
    V = np.ascontiguousarray(L[:, :nocc, nocc:]).reshape(L.shape[0], nocc * nvir)
    D = (eps[None, nocc:] - eps[:nocc, None]).reshape(-1)
    Omega, XpY = tda_modes(V, D) if screening == "tda" else rpa_modes(V, D)
    eo, vo, ev, vv = exact_poles(eps, L, nocc, Omega, XpY)
    H = exact_upfolded(eps, eo, vo, ev, vv)
    E, U = np.linalg.eigh(H)
    return dict(E=E, chi=U[:nmo, :], e_occ=eo, v_occ=vo, e_vir=ev, v_vir=vv,
                Omega=Omega, XpY=XpY)


def exact_ev_step(eps_ref, eps_g, eps_w, L, nocc, screening="tda"):
    """The loop body of eigenvalue self-consistent GW with the exact
    full-frequency self-energy: excitations from the screening built on
    eps_W, Green's-function poles at eps_G -+ Omega, f = diag(eps_ref)."""
    nmo = eps_ref.shape[0]
    nvir = nmo - nocc
    V = np.ascontiguousarray(L[:, :nocc, nocc:]).reshape(L.shape[0], nocc * nvir)
    D = (eps_w[None, nocc:] - eps_w[:nocc, None]).reshape(-1)
    Omega, XpY = tda_modes(V, D) if screening == "tda" else rpa_modes(V, D)
    eo, vo, ev, vv = exact_poles(eps_g, L, nocc, Omega, XpY)
    H = exact_upfolded(eps_ref, eo, vo, ev, vv)
    E, U = np.linalg.eigh(H)
    chi = U[:nmo, :]
    w = chi ** 2
    alpha = np.argmax(w, axis=1)
    return E[alpha], w[np.arange(nmo), alpha]
