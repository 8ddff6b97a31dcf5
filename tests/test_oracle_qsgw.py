"""Pins of the quasiparticle self-consistent loop (Sec. 3.3, App. A Alg. A2):
the two regularised static potentials against the downfolded self-energy
(eq. downfoldedSE) and against each other in their limits, the SCF fixed point
of eq. qp_scf, the exact-self-energy loop where the moments resolve every
pole, the converged fixed point, the fixed-point equation with the potential
written basis-free in the reference orbitals, and the coupling order of the
qsGW shift."""
import numpy as np
import pytest

import gwsynth
from oracle import brute, fsgw, gw, qsgw


def random_poles(nmo=5, npole=9, seed=0):
    rng = np.random.default_rng(seed)
    eps = np.sort(rng.uniform(-1.5, 2.0, nmo))
    e_aux = rng.uniform(-4.0, 5.0, npole)
    W = 0.3 * rng.standard_normal((nmo, npole))
    return eps, e_aux, W


def sigma_downfolded(omega, e_aux, W):
    """Sigma(omega) = W (omega - d~)^-1 W^T as a matrix product (eq. downfoldedSE)."""
    return W @ np.linalg.inv(omega * np.eye(e_aux.shape[0]) - np.diag(e_aux)) @ W.T


def test_lorentzian_potential_small_broadening_is_the_symmetrised_self_energy():
    eps, e_aux, W = random_poles()
    V = qsgw.static_potential(eps, e_aux, W, "lorentzian", delta=1e-9)
    n = eps.shape[0]
    ref = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            ref[p, q] = 0.5 * (sigma_downfolded(eps[p], e_aux, W)[p, q] + sigma_downfolded(eps[q], e_aux, W)[p, q])
    assert np.abs(V - ref).max() < 1e-9 * np.abs(ref).max()
    assert np.array_equal(V, V.T)


def test_srg_large_s_diagonal_is_the_self_energy_at_eps():
    """(D + D)/(2 D^2) = 1/D: for s -> inf the SRG diagonal is Sigma_pp(eps_p)."""
    eps, e_aux, W = random_poles(seed=1)
    V = qsgw.static_potential(eps, e_aux, W, "srg", s=1e8)
    for p in range(eps.shape[0]):
        assert abs(V[p, p] - sigma_downfolded(eps[p], e_aux, W)[p, p]) < 1e-12 * max(1.0, abs(V[p, p]))
    assert np.abs(V - V.T).max() == 0.0


def test_srg_small_s_series():
    """1 - exp(-x s) = x s + O(s^2): V / s -> sum_l v_pl v_ql (D_pl + D_ql)."""
    eps, e_aux, W = random_poles(seed=2)
    s = 1e-7
    V = qsgw.static_potential(eps, e_aux, W, "srg", s=s)
    Dm = eps[:, None] - e_aux[None, :]
    ref = (W * Dm) @ W.T + W @ (W * Dm).T
    assert np.abs(V / s - ref).max() < 1e-5 * np.abs(ref).max()


def test_lorentzian_large_broadening_series():
    """D/(D^2 + delta^2) -> D/delta^2: V delta^2 -> 1/2 sum_l v v (D_pl + D_ql)."""
    eps, e_aux, W = random_poles(seed=3)
    delta = 1e5
    V = qsgw.static_potential(eps, e_aux, W, "lorentzian", delta=delta)
    Dm = eps[:, None] - e_aux[None, :]
    ref = 0.5 * ((W * Dm) @ W.T + W @ (W * Dm).T)
    assert np.abs(V * delta ** 2 - ref).max() < 1e-8 * np.abs(ref).max()


def test_scf_reference_is_a_fixed_point_and_solutions_satisfy_the_equation():
    o = 3
    eps, L = gwsynth.system(o, 7, 20, 3)
    h = fsgw.core_hamiltonian(eps, L, o)
    rho0 = np.diag(np.r_[np.full(o, 2.0), np.zeros(7)])
    e, C, rho, F, steps = qsgw.scf(h, L, np.zeros((10, 10)), o, rho0)
    assert np.abs(e - eps).max() < 1e-13 and steps == 1
    # with a static potential: (f[rho] + V) C = C eps, rho/2 a rank-nocc projector
    rng = np.random.default_rng(0)
    V = 0.02 * rng.standard_normal((10, 10))
    V = V + V.T
    e, C, rho, F, steps = qsgw.scf(h, L, V, o, rho0, scf_tol=1e-12)
    Fx = fsgw.fock(h, L, rho) + V
    assert np.abs(Fx @ C - C * e[None, :]).max() < 1e-10
    assert np.abs(Fx @ rho - rho @ Fx).max() < 1e-10
    P = rho / 2
    assert np.abs(P @ P - P).max() < 1e-12 and abs(np.trace(rho) - 2 * o) < 1e-12


@pytest.mark.parametrize("scheme", ["srg", "lorentzian"])
def test_matches_exact_self_energy_loop_when_pole_count_fits(scheme):
    """o=1, v=2, naux=3, N=3: the moments resolve every pole of the exact
    self-energy in any orbital basis, so both loops share every iterate."""
    o = 1
    eps, L = gwsynth.system(o, 2, 3, 5, amp=1.0)

    def exact(e_mf, C):
        Lc = np.einsum("pi,Ppq,qj->Pij", C, L, C)
        V = np.ascontiguousarray(Lc[:, :o, o:]).reshape(3, -1)
        D = (e_mf[None, o:] - e_mf[:o, None]).reshape(-1)
        Om, XpY = brute.tda_modes(V, D)
        eo, vo, ev, vv = brute.exact_poles(e_mf, Lc, o, Om, XpY)
        return np.r_[eo, ev], np.concatenate([vo, vv], axis=1)

    kw = dict(scheme=scheme, delta=0.05, tol=1e-11, max_iter=80)
    r = qsgw.qsgw(eps, L, o, 3, "tda", **kw)
    ex = qsgw.qsgw(eps, L, o, 3, "tda", pole_fn=exact, **kw)
    assert r["converged"] and ex["converged"]
    assert np.abs(r["qp"] - ex["qp"]).max() < 1e-9


def test_converged_state_is_a_fixed_point():
    o = 3
    eps, L = gwsynth.system(o, 9, 20, 3)
    r = qsgw.qsgw(eps, L, o, 5, "tda", tol=1e-10, max_iter=80)
    assert r["converged"]
    e_aux, W = qsgw.one_shot_poles(r["qp"], r["C"], L, o, 5, "tda")
    V = r["C"] @ qsgw.static_potential(r["qp"], e_aux, W) @ r["C"].T
    rho = 2.0 * r["C"][:, :o] @ r["C"][:, :o].T
    e, _, _, _, _ = qsgw.scf(fsgw.core_hamiltonian(eps, L, o), L, V, o, rho)
    assert np.abs(e - r["qp"]).max() < 1e-9


def test_shift_is_fourth_order_in_the_coupling():
    """With L scaled by a, Sigma and V^Sigma scale as a^4 and f[rho] - diag(eps)
    responds at O(a^2) relative: halving a divides the qsGW shift by ~16."""
    o = 2
    shifts = []
    for amp in (0.1, 0.05):
        eps, L = gwsynth.system(o, 6, 20, 7, amp=amp)
        r = qsgw.qsgw(eps, L, o, 5, "tda", tol=1e-14, max_iter=80)
        assert r["converged"]
        shifts.append(np.abs(r["qp"] - eps)[o - 1:o + 1].max())
    assert 14.0 < shifts[0] / shifts[1] < 18.0


def test_fixed_point_equation_in_the_reference_basis():
    """Basis-free form of eq. qsgw_v: V = 1/2 sum_p {|p><p|, Re Sigma(eps_p)}
    with |p> the QP orbitals and Sigma written in the reference basis; the
    converged orbitals must solve (f[rho] + V) C = C eps with this V."""
    o = 1
    eps, L = gwsynth.system(o, 2, 3, 5, amp=1.0)
    delta = 0.05

    def exact(e_mf, C):
        Lc = np.einsum("pi,Ppq,qj->Pij", C, L, C)
        V = np.ascontiguousarray(Lc[:, :o, o:]).reshape(3, -1)
        D = (e_mf[None, o:] - e_mf[:o, None]).reshape(-1)
        Om, XpY = brute.tda_modes(V, D)
        eo, vo, ev, vv = brute.exact_poles(e_mf, Lc, o, Om, XpY)
        return np.r_[eo, ev], np.concatenate([vo, vv], axis=1)

    r = qsgw.qsgw(eps, L, o, 3, "tda", scheme="lorentzian", delta=delta, tol=1e-12, max_iter=100, pole_fn=exact)
    assert r["converged"]
    C, e = r["C"], r["qp"]
    e_aux, Wc = exact(e, C)
    Wr = C @ Wc                                   # couplings in the reference basis
    V = np.zeros((3, 3))
    for p in range(3):
        d = e[p] - e_aux
        S = (Wr * (d / (d * d + delta * delta))[None, :]) @ Wr.T
        P = np.outer(C[:, p], C[:, p])
        V += 0.5 * (P @ S + S @ P)
    rho = 2.0 * C[:, :o] @ C[:, :o].T
    F = fsgw.fock(fsgw.core_hamiltonian(eps, L, o), L, rho) + V
    assert np.abs(F @ C - C * e[None, :]).max() < 1e-9


def test_outer_diis_reaches_the_plain_loop_fixed_point():
    """DIIS over the static potential changes the path, not the fixed point."""
    o = 3
    eps, L = gwsynth.system(o, 9, 20, 1)
    a = qsgw.qsgw(eps, L, o, 5, "tda", tol=1e-11, max_iter=80, outer_diis=12)
    b = qsgw.qsgw(eps, L, o, 5, "tda", tol=1e-11, max_iter=80, outer_diis=0)
    assert a["converged"] and b["converged"] and a["iterations"] < b["iterations"]
    assert np.abs(a["qp"] - b["qp"]).max() < 1e-9


@pytest.mark.parametrize("seed", [0, 4])
def test_outer_diis_converges_where_the_plain_loop_stalls(seed):
    """Lorentzian potential, delta = 1e-3: the plain loop still moves after 40
    rebuilds; with DIIS the loop ends on a state that one more plain rebuild
    (poles, potential, SCF) leaves in place."""
    o, N = 3, 5
    eps, L = gwsynth.system(o, 9, 20, seed)
    plain = qsgw.qsgw(eps, L, o, N, "tda", scheme="lorentzian", tol=1e-8, max_iter=40, outer_diis=0)
    assert not plain["converged"]
    r = qsgw.qsgw(eps, L, o, N, "tda", scheme="lorentzian", tol=1e-10, max_iter=60)
    assert r["converged"]
    e_aux, W = qsgw.one_shot_poles(r["qp"], r["C"], L, o, N, "tda")
    V = r["C"] @ qsgw.static_potential(r["qp"], e_aux, W, "lorentzian") @ r["C"].T
    rho = 2.0 * r["C"][:, :o] @ r["C"][:, :o].T
    e, _, _, _, _ = qsgw.scf(fsgw.core_hamiltonian(eps, L, o), L, V, o, rho)
    assert np.abs(e - r["qp"]).max() < 1e-8
