"""Pins of the fsGW oracle (Sec. 3.6, Alg. 2) against facts fixed outside it:
explicit four-index integrals, decoupled limits, the Krylov property of DIIS,
the fixed-point conditions of the converged loop, and the weak-coupling order.
"""
import numpy as np
import pytest

import gwsynth
from oracle import fsgw as fs
from oracle import gw as ogw


def _eri(L):
    """(pq|rs) = sum_P L[P,p,q] L[P,r,s], written out as a four-index tensor."""
    A, M, _ = L.shape
    eri = np.zeros((M, M, M, M))
    for P in range(A):
        eri += L[P][:, :, None, None] * L[P][None, None, :, :]
    return eri


def test_jk_match_four_index_integrals():
    eps, L = gwsynth.system(2, 5, 9, 3)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((7, 7))
    rho = X @ X.T
    J, K = fs.jk(L, rho)
    eri = _eri(L)
    M = L.shape[1]
    Jr = np.zeros((M, M))
    Kr = np.zeros((M, M))
    for p in range(M):
        for q in range(M):
            Jr[p, q] = sum(eri[p, q, r, s] * rho[r, s] for r in range(M) for s in range(M))
            Kr[p, q] = sum(eri[p, r, q, s] * rho[r, s] for r in range(M) for s in range(M))
    assert np.abs(J - Jr).max() < 1e-12 * np.abs(Jr).max()
    assert np.abs(K - Kr).max() < 1e-12 * np.abs(Kr).max()


def test_reference_density_reproduces_reference_fock():
    """Reading of Alg. 2's h: F[rho0] = diag(eps) for the closed-shell reference density."""
    o, v = 3, 6
    eps, L = gwsynth.system(o, v, 15, 2)
    h = fs.core_hamiltonian(eps, L, o)
    rho0 = np.diag(np.r_[np.full(o, 2.0), np.zeros(v)])
    assert np.abs(fs.fock(h, L, rho0) - np.diag(eps)).max() < 1e-13


def test_aufbau_without_coupling_is_the_mean_field_density():
    """W = 0: H~ is block diagonal, so filling to N_e electrons gives the
    ground-state density of F itself, whatever the auxiliary energies."""
    rng = np.random.default_rng(4)
    M, o, na = 8, 3, 11
    X = rng.standard_normal((M, M))
    F = (X + X.T) / 2
    e_aux = rng.uniform(-3, 3, na)
    W = np.zeros((M, na))
    rho, _, _ = fs.density(F, e_aux, W, 0.0, 2.0 * o)
    w, U = np.linalg.eigh(F)
    assert np.abs(rho - 2.0 * U[:, :o] @ U[:, :o].T).max() < 1e-12
    assert abs(np.trace(rho) - 2 * o) < 1e-12


def test_diis_solves_a_linear_fixed_point_in_n_plus_one_steps():
    """Pulay extrapolation on x = A x + b with errors g(x) - x is a Krylov
    method: in exact arithmetic it reaches the fixed point in <= n + 1 steps."""
    rng = np.random.default_rng(7)
    n = 5
    A = 0.5 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x_star = np.linalg.solve(np.eye(n) - A, b)
    d = fs.DIIS(space=12)
    x = np.zeros(n)
    for _ in range(n + 1):
        gx = A @ x + b
        x = d.update(gx, gx - x)
    assert np.abs(x - x_star).max() < 1e-9


def _poles(eps, L, o, N):
    so, sv, _ = ogw.gw_moments(eps, L, o, N, "tda")
    eo, vo = ogw.poles_from_moments(list(so))
    ev, vv = ogw.poles_from_moments(list(sv))
    return np.concatenate([eo, ev]), np.concatenate([vo, vv], axis=1)


def test_zeta_restores_the_electron_number():
    o, v, A, N = 3, 9, 20, 3
    eps, L = gwsynth.system(o, v, A, 1)
    e_aux, W = _poles(eps, L, o, N)
    F = np.diag(eps)
    z = fs.solve_zeta(F, e_aux, W, 2.0 * o)
    assert -1.0 <= z <= 1.0
    assert abs(fs.trace_density(F, e_aux, W, z, 2.0 * o) - 2 * o) < 1e-8


@pytest.fixture(scope="module")
def converged():
    o, v, A, N = 3, 9, 20, 3
    eps, L = gwsynth.system(o, v, A, 1)
    r = fs.fsgw(eps, L, o, N)
    return o, N, eps, L, r


def test_fsgw_converges_to_a_self_consistent_fock_matrix(converged):
    o, N, eps, L, r = converged
    assert r["converged"]
    h = fs.core_hamiltonian(eps, L, o)
    assert abs(np.trace(r["rho"]) - 2 * o) < 1e-8
    # F = F[rho] at convergence (density converged to 1e-8)
    assert np.abs(r["F"] - fs.fock(h, L, r["rho"])).max() < 1e-8
    assert np.abs(r["F"] - r["F"].T).max() < 1e-12


def test_warm_starts_reach_the_same_quasiparticles(converged):
    o, N, eps, L, r = converged
    exact = fs.fsgw(eps, L, o, N, F0=r["F"])
    assert exact["iterations"] == 1        # one rebuild reproduces its own fixed point
    assert np.abs(exact["qp"] - r["qp"]).max() < 1e-6
    diag = fs.fsgw(eps, L, o, N, F0=np.diag(np.diag(r["F"])))
    assert diag["converged"]
    assert np.abs(diag["qp"] - r["qp"]).max() < 1e-6


def test_fsgw_shift_is_fourth_order_in_the_coupling():
    """Scaling L by lam scales the integrals (pq|rs) by lam^2.  The reference
    is self-consistent at mean-field level (F[rho0] = diag(eps)), so the QP
    shift is the correlation part, second order in the integrals: O(lam^4);
    the density change it induces enters F only at O(lam^6)."""
    o, v, A, N = 2, 6, 12, 3
    eps, L = gwsynth.system(o, v, A, 5)
    shifts = []
    for lam in (0.2, 0.1):
        r = fs.fsgw(eps, lam * L, o, N)
        assert r["converged"]
        shifts.append(np.abs(r["qp"][o - 1:o + 1] - np.sort(eps)[o - 1:o + 1]))
    ratio = shifts[1] / shifts[0]
    assert np.all(np.abs(ratio - 1.0 / 16.0) < 0.005), ratio


@pytest.mark.parametrize("seed", [1, 2])
def test_nested_and_interleaved_orders_reach_one_fixed_point(seed):
    """The algorithm box nests a fixed-zeta Fock loop inside the
    electron-number loop; the oracle (and the device) re-solve zeta at every
    Fock step.  Both orders stop at F = F[rho], Tr rho(zeta) = N_e, so the
    converged Fock matrix, density and QP energies agree (to the loop
    tolerances), whatever the number of Fock steps it takes."""
    o, v, A, N = 3, 9, 30, 3
    eps, L = gwsynth.system(o, v, A, seed)
    a = fs.fsgw(eps, L, o, N, tol=1e-9, fock_tol=1e-10, order="interleaved")
    b = fs.fsgw(eps, L, o, N, tol=1e-9, fock_tol=1e-10, order="nested")
    assert a["converged"] and b["converged"]
    assert np.abs(a["F"] - b["F"]).max() < 1e-7
    assert np.abs(a["rho"] - b["rho"]).max() < 1e-7
    assert np.abs(a["qp"] - b["qp"]).max() < 1e-7
    assert abs(a["zeta"] - b["zeta"]) < 1e-9
    assert abs(np.trace(b["rho"]) - 2 * o) < 1e-8
    # the nested order's converged F is a fixed point of the Fock map
    h = fs.core_hamiltonian(eps, L, o)
    assert np.abs(fs.fock(h, L, b["rho"]) - b["F"]).max() < 1e-6
