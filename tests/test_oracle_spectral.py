"""Pins of the Green's-function post-processing (eqs. ret_GF, spectrum,
downfoldedSE, density; Sec. 3.5): the Lehmann sum over the eigenpairs of H~
against the resolvent of the physical block with the downfolded self-energy,
the Lorentzian closed forms of the non-interacting limit, the spectral sum
rule, the Aufbau filling against brute force, and the electron-number shift
against an independently built shifted Hamiltonian."""
import numpy as np
import pytest

import gwsynth
from oracle import fsgw, gw, spectral


def g0w0_poles(o=3, v=8, A=20, nmom=5, seed=0, screening="tda"):
    eps, L = gwsynth.system(o, v, A, seed)
    r = gw.g0w0(eps, L, o, nmom, screening)
    e_aux = np.r_[r["e_occ"], r["e_vir"]]
    W = np.concatenate([r["v_occ"], r["v_vir"]], axis=1)
    return eps, r, e_aux, W


@pytest.mark.parametrize("screening", ["tda", "rpa"])
def test_lehmann_sum_equals_downfolded_resolvent(screening):
    """G(z) = [z - f - W (z - d~)^-1 W^T]^-1 at z = w + i delta (eqs. effH,
    downfoldedSE); its diagonal must equal the pole sum over H~'s eigenpairs."""
    eps, r, e_aux, W = g0w0_poles(screening=screening, seed=1)
    omega = np.linspace(-2.5, 4.0, 57)
    delta = 0.03
    A, Ap = spectral.spectral_function(r["E"], r["chi"], omega, delta)
    f = np.diag(eps)
    nmo = eps.shape[0]
    for k, w in enumerate(omega):
        z = w + 1j * delta
        sig = (W / (z - e_aux)) @ W.T
        G = np.linalg.inv(z * np.eye(nmo) - f - sig)
        ref = -np.imag(np.diag(G)) / np.pi
        assert np.abs(Ap[:, k] - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())
        assert abs(A[k] - ref.sum()) < 1e-10 * max(1.0, abs(ref.sum()))


def test_noninteracting_lorentzians():
    """No auxiliary poles: A_p is a unit Lorentzian at eps_p, peak 1/(pi delta),
    half maximum at eps_p +- delta."""
    eps = np.array([-1.0, -0.4, 0.3, 1.7])
    chi = np.eye(4)
    delta = 1e-3
    for p in range(4):
        _, Ap = spectral.spectral_function(eps, chi, [eps[p], eps[p] + delta, eps[p] - delta], delta)
        assert abs(Ap[p, 0] - 1.0 / (np.pi * delta)) < 1e-12 / delta
        assert abs(Ap[p, 1] - 0.5 / (np.pi * delta)) < 1e-12 / delta
        assert abs(Ap[p, 2] - 0.5 / (np.pi * delta)) < 1e-12 / delta
        others = [q for q in range(4) if q != p]
        assert np.abs(Ap[others, 0]).max() < 1e-3


def test_spectral_sum_rule():
    """Each A_p integrates to sum_a chi_pa^2 = 1 (completeness of H~'s
    eigenvectors): checked as the broad-Lorentzian limit pi Y A_p(0; Y) -> 1
    and by quadrature over a wide window."""
    eps, r, _, _ = g0w0_poles(seed=2)
    Y = 1e9
    _, Ap = spectral.spectral_function(r["E"], r["chi"], [0.0], Y)
    assert np.abs(np.pi * Y * Ap[:, 0] - 1.0).max() < 1e-12
    delta = 0.05
    omega = np.linspace(-400.0, 400.0, 320001)
    A, _ = spectral.spectral_function(r["E"], r["chi"][:2], omega, delta)
    integral = np.trapezoid(A, omega)
    tail = 2 * 2 * delta / (np.pi * 400.0)      # two orbitals, both tails
    assert abs(integral - 2.0) < 2 * tail


def test_aufbau_noninteracting():
    eps = np.array([-1.1, -0.7, -0.2, 0.4, 0.9])
    st = spectral.aufbau_state(eps, np.eye(5), 6.0)
    assert st["nfill"] == 3 and st["homo"] == 2 and st["lumo"] == 3
    assert np.array_equal(st["rho"], np.diag([2.0, 2.0, 2.0, 0.0, 0.0]))
    assert st["mu"] == pytest.approx(0.1, abs=1e-15)
    assert np.array_equal(st["dyson_homo"], np.eye(5)[2])
    assert np.array_equal(st["dyson_lumo"], np.eye(5)[3])


def test_aufbau_against_brute_force():
    eps, r, _, _ = g0w0_poles(o=4, v=9, A=25, seed=3)
    E, chi = r["E"], r["chi"]
    for nelec in (8.0, 7.3, 0.0, 2.0 * eps.shape[0]):
        st = spectral.aufbau_state(E, chi, nelec)
        best, nb = None, None
        for n in range(E.shape[0] + 1):
            c = 2.0 * sum(float(chi[:, a] @ chi[:, a]) for a in range(n))
            if best is None or abs(c - nelec) < best - 1e-15:
                best, nb = abs(c - nelec), n
        assert st["nfill"] == nb
        # rho/2 is a partial sum of projectors: symmetric, eigenvalues in [0, 1]
        w = np.linalg.eigvalsh(st["rho"] / 2.0)
        assert w.min() > -1e-12 and w.max() < 1 + 1e-12
        assert np.abs(st["rho"] - st["rho"].T).max() == 0.0
    st = spectral.aufbau_state(E, chi, 8.0)
    assert st["homo"] == st["nfill"] - 1 and E[st["homo"]] < st["mu"] < E[st["lumo"]]
    # the Dyson orbital of the ionisation: squared norm = its pole strength
    assert abs(st["dyson_homo"] @ st["dyson_homo"] - float(chi[:, st["homo"]] @ chi[:, st["homo"]])) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 3, 7])
def test_zeta_shift_conserves_electron_number(seed):
    """The shifted Hamiltonian, rebuilt through the pole-by-sector upfolding
    with every auxiliary energy moved by zeta, fills to N_e electrons."""
    eps, r, e_aux, W = g0w0_poles(seed=seed)
    out = spectral.g0w0_number_conserving(np.diag(eps), e_aux, W, 6.0)
    z = out["zeta"]
    assert abs(z) < 0.05
    H = gw.upfolded_hamiltonian(np.diag(eps), r["e_occ"] + z, r["v_occ"], r["e_vir"] + z, r["v_vir"])
    E, U = np.linalg.eigh(H)
    w = (U[: eps.shape[0]] ** 2).sum(axis=0)
    cum = np.r_[0.0, 2.0 * np.cumsum(w)]
    assert np.abs(cum - 6.0).min() < 1e-12
    assert np.abs(E - out["E"]).max() < 1e-12
    # without the shift the one-shot filling misses N_e
    assert abs(spectral.aufbau_state(r["E"], r["chi"], 6.0)["nelec"] - 6.0) > 1e-6


def test_electron_count_grows_with_zeta():
    """Raising the auxiliary energies moves weight onto the physical states
    below the Fermi level: Tr rho(zeta) is non-decreasing."""
    eps, r, e_aux, W = g0w0_poles(seed=4)
    zs = np.linspace(-0.02, 0.02, 41)
    tr = [fsgw.trace_density(np.diag(eps), e_aux, W, z, 6.0) for z in zs]
    assert np.all(np.diff(tr) > -1e-12)
    assert tr[-1] - tr[0] > 1e-5


def test_zeta_irrelevant_without_coupling():
    """Vanishing couplings: the count is exactly 2 nocc for any small zeta."""
    eps = np.array([-1.0, -0.5, 0.4, 1.2])
    e_aux = np.array([-2.0, 2.5])
    W = np.zeros((4, 2))
    out = spectral.g0w0_number_conserving(np.diag(eps), e_aux, W, 4.0)
    assert out["state"]["nelec"] == 4.0
    assert np.array_equal(np.sort(out["qp"]), eps)
