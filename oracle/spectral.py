"""Green's function post-processing of the upfolded Hamiltonian, oracle side:
spectral function (eqs. ret_GF, spectrum), Aufbau filling and electron number
(eq. density), frontier Dyson orbitals, and the electron-number shift of the
auxiliary energies for a one-shot calculation (Sec. 3.5, electron number
conservation).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Inputs are the eigenpairs of H~ as the rest of the oracle returns them:
E [dim] ascending and chi [nmo][dim], the physical rows of the eigenvectors.

Readings taken here:
  * the retarded Green's function carries one broadening delta > 0 for every
    pole, G_pq(w) = sum_a chi_pa chi_qa / (w - E_a + i delta), and the
    spectral function is the trace A(w) = -(1/pi) sum_p Im G_pp(w); the
    per-orbital terms A_p(w) = -(1/pi) Im G_pp(w) are returned beside it;
  * Aufbau: the n lowest eigenstates are occupied, n minimising
    |2 sum_{a<n} |chi_a|^2 - N_e| (lowest n on ties), rho = 2 sum_{a<n}
    chi_a chi_a^T; the chemical potential is placed midway between the
    highest occupied and the lowest empty state, whose physical parts are
    the Dyson orbitals of the ionisation and the attachment (in the MO basis;
    their squared norms are the pole strengths);
  * the electron-number shift zeta is added to every auxiliary energy (the
    diagonal of d~) with the physical block fixed.  The shift is meant to be
    small, so the root of Tr rho(zeta) - N_e is bracketed outwards from
    zeta = 0 (half-width 1e-3 Ha, widened tenfold within [lo, hi] until the
    sign changes) and then bisected: a fixed wide bracket can hold jumps of
    the Aufbau count at both ends and no sign change.
"""
from __future__ import annotations

import numpy as np

from . import fsgw, gw


def greens_function(E, chi, omega, delta):
    """G_pp(w) for every orbital p and frequency w (eq. ret_GF), complex
    [nmo][nomega], as the plain Lehmann sum over poles."""
    E = np.asarray(E, dtype=float)
    chi = np.asarray(chi, dtype=float)
    omega = np.asarray(omega, dtype=float)
    G = np.zeros((chi.shape[0], omega.shape[0]), dtype=complex)
    for a in range(E.shape[0]):
        G += np.outer(chi[:, a] ** 2, 1.0 / (omega - E[a] + 1j * delta))
    return G


def spectral_function(E, chi, omega, delta):
    """A(w) = -(1/pi) sum_p Im G_pp(w) (eq. spectrum) and the per-orbital
    A_p(w) = -(1/pi) Im G_pp(w): returns (A [nomega], A_p [nmo][nomega])."""
    Ap = -np.imag(greens_function(E, chi, omega, delta)) / np.pi
    return Ap.sum(axis=0), Ap


def aufbau_state(E, chi, nelec):
    """Aufbau filling of the eigenstates of H~ (eq. density).  Returns a dict
    with the density matrix, the number of filled states, the electron count
    of that filling, the chemical potential (midway between the frontier
    states), the frontier state indices and their Dyson orbitals."""
    E = np.asarray(E, dtype=float)
    rho, n = fsgw.aufbau(E, chi, nelec)
    dim = E.shape[0]
    homo = n - 1 if n > 0 else -1
    lumo = n if n < dim else -1
    if homo >= 0 and lumo >= 0:
        mu = 0.5 * (E[homo] + E[lumo])
    else:
        mu = E[homo] if homo >= 0 else E[lumo]
    return dict(rho=rho, nfill=n, nelec=float(np.trace(rho)), mu=float(mu), homo=homo, lumo=lumo,
                dyson_homo=chi[:, homo].copy() if homo >= 0 else None,
                dyson_lumo=chi[:, lumo].copy() if lumo >= 0 else None)


def solve_zeta_from_zero(fock, e_aux, W, nelec, lo=-1.0, hi=1.0, tol=1e-13):
    """Root of Tr rho(zeta) - N_e nearest zeta = 0: outward bracketing, then
    bisection (the end with the smaller residual when [lo, hi] holds no
    sign change)."""
    half = 1e-3
    while True:
        a, b = max(lo, -half), min(hi, half)
        fa = fsgw.trace_density(fock, e_aux, W, a, nelec) - nelec
        fb = fsgw.trace_density(fock, e_aux, W, b, nelec) - nelec
        if fa * fb <= 0.0 or (a == lo and b == hi):
            break
        half *= 10.0
    return fsgw.solve_zeta(fock, e_aux, W, nelec, a, b, tol)


def g0w0_number_conserving(fock, e_aux, W, nelec, lo=-1.0, hi=1.0, tol=1e-13):
    """One-shot GW with the auxiliary energies shifted by zeta so that the
    Aufbau filling of H~ holds N_e electrons; returns zeta, the eigenpairs
    of H~(zeta), the QP energies and weights, and the Aufbau state."""
    zeta = solve_zeta_from_zero(fock, e_aux, W, nelec, lo, hi, tol)
    E, U = np.linalg.eigh(fsgw.upfolded(fock, e_aux, W, zeta))
    chi = U[: fock.shape[0]]
    qp, wt, _ = gw.qp_assign(E, chi)
    return dict(zeta=zeta, E=E, chi=chi, qp=qp, qp_weight=wt, state=aufbau_state(E, chi, nelec))
