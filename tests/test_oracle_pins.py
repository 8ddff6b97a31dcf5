"""Pins for the FP64 oracle: each test fixes part of it against something
other than itself (brute-force diagonalisation, closed forms, textbook
limits, invariants), so that a dropped term, a wrong sign or index or a
transposed operand in the oracle fails at least one of them."""
from math import comb

import numpy as np
import pytest

import gwsynth
from oracle import brute, gw, quadrature


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def small(o=3, v=5, A=7, seed=1, amp=1.0):
    eps, L = gwsynth.system(o, v, A, seed, amp=amp)
    V, D = gw.particle_hole(eps, L, o)
    return eps, L, V, D


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("screening", ["tda", "rpa"])
@pytest.mark.parametrize("seed", [1, 2])
def test_moments_equal_exact_lehmann_moments(screening, seed):
    """Recursion moments equal the moments of the exact G0W0 self-energy poles
    obtained by full diagonalisation of the particle-hole problem."""
    o, N = 3, 7
    eps, L, V, D = small(o=o, v=6, A=9, seed=seed)
    so, sv, _ = gw.gw_moments(eps, L, o, N, screening, nquad=48)
    Om, XpY = brute.tda_modes(V, D) if screening == "tda" else brute.rpa_modes(V, D)
    eo, vo, ev, vv = brute.exact_poles(eps, L, o, Om, XpY)
    To = brute.moments_of_poles(eo, vo, N)
    Tv = brute.moments_of_poles(ev, vv, N)
    for n in range(N + 1):
        assert rel(so[n], To[n]) < 1e-12
        assert rel(sv[n], Tv[n]) < 1e-12


@pytest.mark.parametrize("screening", ["tda", "rpa"])
def test_eta_tilde_equals_V_eta(screening):
    """eta~^{(n)} = V eta^{(n)} with eta^{(n)} = (X+Y) Omega^n (X+Y)^T (eq. alt_dd)."""
    eps, L, V, D = small()
    N = 6
    eta = gw.tda_eta(V, D, N) if screening == "tda" else gw.rpa_eta(V, D, N, nquad=48)
    Om, XpY = brute.tda_modes(V, D) if screening == "tda" else brute.rpa_modes(V, D)
    ex = brute.eta_from_modes(Om, XpY, N)
    for n in range(N + 1):
        assert rel(eta[n], V @ ex[n]) < 1e-12


# ---------------------------------------------------------------- P2
def test_tda_zeroth_hole_moment_closed_form():
    """TDA eta^{(0)} = I, so Sigma^{(0,<)}_pq = 2 sum_{k,ia} (pk|ia)(qk|ia)."""
    o = 3
    eps, L, V, D = small(o=o)
    so, sv, _ = gw.gw_moments(eps, L, o, 1, "tda")
    eri_pkia = np.einsum("Ppk,Pia->pkia", L[:, :, :o], L[:, :o, o:])
    ref = 2.0 * np.einsum("pkia,qkia->pq", eri_pkia, eri_pkia)
    eri_pcia = np.einsum("Ppc,Pia->pcia", L[:, :, o:], L[:, :o, o:])
    refv = 2.0 * np.einsum("pcia,qcia->pq", eri_pcia, eri_pcia)
    assert rel(so[0], ref) < 1e-13
    assert rel(sv[0], refv) < 1e-13


# ---------------------------------------------------------------- P3
def test_rpa_first_moment_and_zeroth_moment_identity():
    """RPA: eta~^{(1)} = V D, and eta^{(0)} (A+B) eta^{(0)} = A - B = D."""
    eps, L, V, D = small()
    eta = gw.rpa_eta(V, D, 1, nquad=48)
    assert rel(eta[1], V * D[None, :]) < 1e-15
    Om, XpY = brute.rpa_modes(V, D)
    e0 = brute.eta_from_modes(Om, XpY, 0)[0]
    ApB = np.diag(D) + 4.0 * V.T @ V
    assert rel(e0 @ ApB @ e0, np.diag(D)) < 1e-12


# ---------------------------------------------------------------- P4
def test_woodbury_equals_direct_inverse():
    """eta~^{(0)} = G (A+B)^-1 with A+B = D + 4 V^T V: the Woodbury form of the
    paper equals the dense inverse, for any G."""
    eps, L, V, D = small()
    rng = np.random.default_rng(5)
    G = rng.standard_normal(V.shape)
    ApB = np.diag(D) + 4.0 * V.T @ V
    assert rel(gw.rpa_eta0_from_G(G, V, D), G @ np.linalg.inv(ApB)) < 1e-12


def test_G_is_eta0_times_A_plus_B():
    """G = eta~^{(0)} (A+B) = V sqrt((A-B)(A+B)) from the exact modes."""
    eps, L, V, D = small()
    Om, XpY = brute.rpa_modes(V, D)
    e0 = brute.eta_from_modes(Om, XpY, 0)[0]
    ApB = np.diag(D) + 4.0 * V.T @ V
    assert rel(gw.rpa_G_quadrature(V, D, 48), V @ e0 @ ApB) < 1e-12


# ---------------------------------------------------------------- P5
@pytest.mark.parametrize("v,d", [(0.3, 0.8), (0.05, 2.5), (1.0, 0.4)])
def test_scalar_pair_closed_form(v, d):
    """o = v = naux = 1: G_offset = v d + 2 v^3 and
    G_main = v (sqrt(d^2 + 4 d v^2) - d - 2 v^2)."""
    V = np.array([[v]])
    D = np.array([d])
    Gm, Go = gw.rpa_G_quadrature(V, D, 48, parts=True)
    # the mapped rule integrates exp(-2 d z) with a sub-exponential error
    # when 2 d s is small, hence the loose bound; the formula is what is pinned
    gm_ref = v * (np.sqrt(d * d + 4 * d * v * v) - d - 2 * v * v)
    go_ref = v * d + 2 * v ** 3
    assert abs(Gm[0, 0] - gm_ref) < 1e-7 * abs(go_ref)
    assert abs(Go[0, 0] - go_ref) < 1e-7 * abs(go_ref)


# ---------------------------------------------------------------- P6
def test_quadrature_converges_geometrically_to_exact_eta0():
    eps, L, V, D = small(o=4, v=12, A=20, seed=3, amp=0.6)
    ex = gw.rpa_eta0_exact(V, D)
    errs = [rel(gw.rpa_eta0_from_G(gw.rpa_G_quadrature(V, D, nq), V, D), ex) for nq in (6, 12, 24, 48)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 1e-5 and errs[3] < 1e-13


def test_quadrature_grid_integrates_known_functions():
    """int_0^inf exp(-a z) dz = 1/a and int_0^inf dz/(z^2+a^2) = pi/(2a)."""
    z, w = quadrature.mapped_gauss_legendre(48, 1.0)
    for a in (0.3, 1.0, 4.0):
        # the exponential maps to an essential singularity at x = 1: slower, still tight
        assert abs((w * np.exp(-a * z)).sum() - 1.0 / a) < 2e-7 / a
        assert abs((w / (z * z + a * a)).sum() - np.pi / (2 * a)) < 1e-12


# ---------------------------------------------------------------- P7
def test_offset_integral_closed_form():
    """int_0^inf exp(-z (D_ia + D_jb)) dz = 1/(D_ia + D_jb), so
    G_offset = V D + 4 sum_ia V_{P,ia} D_ia K_{ia,jb} / (D_ia + D_jb), K = V^T V."""
    eps, L, V, D = small(o=3, v=7, A=10, seed=4)
    _, Go = gw.rpa_G_quadrature(V, D, 48, parts=True)
    K = V.T @ V
    ref = V * D[None, :] + 4.0 * (V * D[None, :]) @ (K / (D[:, None] + D[None, :]))
    assert rel(Go, ref) < 1e-13


# ---------------------------------------------------------------- P8
@pytest.mark.parametrize("screening", ["tda", "rpa"])
def test_second_order_limit(screening):
    """L -> lam L: Sigma^{(n)} / lam^4 tends to the moments of the direct
    (ring) second-order self-energy of a closed-shell reference,
    hole: 2 sum_{k,i,a} (pk|ia)(qk|ia) (eps_k + eps_i - eps_a)^n,
    particle: 2 sum_{c,i,a} (pc|ia)(qc|ia) (eps_c + eps_a - eps_i)^n,
    with a relative gap that shrinks like lam^2."""
    o, v, N = 3, 5, 5
    eps, L, V, D = small(o=o, v=v, A=7, seed=2, amp=1.0)
    eri_k = np.einsum("Ppk,Pia->pkia", L[:, :, :o], L[:, :o, o:])
    eri_c = np.einsum("Ppc,Pia->pcia", L[:, :, o:], L[:, :o, o:])
    ek, ec = eps[:o], eps[o:]
    ei, ea = eps[:o], eps[o:]
    Eh = ek[:, None, None] + ei[None, :, None] - ea[None, None, :]
    Ep = ec[:, None, None] + ea[None, None, :] - ei[None, :, None]
    gaps = []
    for lam in (1e-2, 5e-3):
        so, sv, _ = gw.gw_moments(eps, lam * L, o, N, screening, nquad=48)
        g = 0.0
        for n in range(N + 1):
            rh = 2.0 * np.einsum("pkia,qkia,kia->pq", eri_k, eri_k, Eh ** n)
            rp = 2.0 * np.einsum("pcia,qcia,cia->pq", eri_c, eri_c, Ep ** n)
            g = max(g, rel(so[n] / lam ** 4, rh), rel(sv[n] / lam ** 4, rp))
        gaps.append(g)
    assert gaps[0] < 1e-3
    assert 3.0 < gaps[0] / gaps[1] < 5.0


# ---------------------------------------------------------------- P9
@pytest.mark.parametrize("screening", ["tda", "rpa"])
def test_symmetry_and_positivity(screening):
    o, N = 4, 7
    eps, L = gwsynth.system(o, 12, 30, 7)
    V, D = gw.particle_hole(eps, L, o)
    eta = gw.tda_eta(V, D, N) if screening == "tda" else gw.rpa_eta(V, D, N, nquad=48)
    R = gw.w_core(eta, V)
    for r in R:
        assert rel(r, r.T) < 1e-12
    so, sv, asym = gw.sigma_moments(eps, L, o, R)
    assert asym < 1e-12 * max(np.abs(so).max(), np.abs(sv).max())
    for n in range(0, N + 1, 2):
        for s in (so[n], sv[n]):
            w = np.linalg.eigvalsh(s)
            assert w.min() > -1e-12 * w.max()


# ---------------------------------------------------------------- P10
@pytest.mark.parametrize("N", [1, 3, 5, 7, 11])
def test_poles_reproduce_conserved_moments(N):
    o = 4
    eps, L = gwsynth.system(o, 12, 30, 11)
    so, sv, _ = gw.gw_moments(eps, L, o, N, "tda")
    for T in (so, sv):
        e, vv = gw.poles_from_moments(list(T))
        for n in range(N + 1):
            assert rel((vv * e[None, :] ** n) @ vv.T, T[n]) < 1e-9


def test_even_nmom_rejected():
    eps, L = gwsynth.system(2, 4, 6, 0)
    so, sv, _ = gw.gw_moments(eps, L, 2, 2, "tda")
    with pytest.raises(ValueError):
        gw.poles_from_moments(list(so))


def test_non_psd_zeroth_moment_rejected():
    T = [np.diag([1.0, -0.5]), np.eye(2)]
    with pytest.raises(gw.LanczosError):
        gw.poles_from_moments(T)


# ---------------------------------------------------------------- P11
@pytest.mark.parametrize("screening", ["tda", "rpa"])
def test_exact_when_pole_count_fits(screening):
    """o=1, v=2, naux=3: each sector has at most ov * o = 2 (hole) or
    ov * v = 4 (particle) poles, which N = 3 (two blocks of size 3) resolves
    exactly, so moment GW reproduces full-frequency G0W0 exactly."""
    o = 1
    eps, L = gwsynth.system(o, 2, 3, 5, amp=1.0)
    r = gw.g0w0(eps, L, o, 3, screening)
    ex = brute.exact_g0w0(eps, L, o, screening)
    qp_ex, w_ex, _ = gw.qp_assign(ex["E"], ex["chi"])
    assert np.abs(r["qp"] - qp_ex).max() < 1e-9
    assert np.abs(r["qp_weight"] - w_ex).max() < 1e-9
    # every exact pole is recovered
    for e_ex, e_mom in ((ex["e_occ"], r["e_occ"]), (ex["e_vir"], r["e_vir"])):
        for e in e_ex:
            assert np.abs(e_mom - e).min() < 1e-8


# ---------------------------------------------------------------- P12, P13
def test_frontier_qp_converge_with_moment_order():
    o = 4
    eps, L = gwsynth.system(o, 16, 40, 3)
    ex = brute.exact_g0w0(eps, L, o, "tda")
    qp_ex, w_ex, _ = gw.qp_assign(ex["E"], ex["chi"])
    front = slice(o - 3, o + 3)
    errs = []
    for N in (3, 7, 11):
        r = gw.g0w0(eps, L, o, N, "tda")
        errs.append(np.abs(r["qp"] - qp_ex)[front].max())
        # P13: moment poles stay inside the hull of the exact sector poles
        assert r["e_occ"].min() > ex["e_occ"].min() - 1e-9
        assert r["e_occ"].max() < ex["e_occ"].max() + 1e-9
        assert r["e_vir"].min() > ex["e_vir"].min() - 1e-9
        assert r["e_vir"].max() < ex["e_vir"].max() + 1e-9
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


# ---------------------------------------------------------------- P16
def test_weak_coupling_rpa_tda_agree_and_reduce_to_bare():
    """With V -> lam V both screenings give eta~^{(n)} = V D^n + O(lam^3)."""
    eps, L, V, D = small()
    lam = 1e-4
    Vs = lam * V
    N = 5
    et = gw.tda_eta(Vs, D, N)
    er = gw.rpa_eta(Vs, D, N, nquad=48)
    for n in range(N + 1):
        bare = Vs * D[None, :] ** n
        assert rel(et[n], bare) < 1e-6
        assert rel(er[n], bare) < 1e-6


def test_particle_hole_layout():
    o = 2
    eps, L = gwsynth.system(o, 3, 4, 9)
    V, D = gw.particle_hole(eps, L, o)
    for P in range(4):
        for i in range(o):
            for a in range(3):
                assert V[P, i * 3 + a] == L[P, i, o + a]
                assert D[i * 3 + a] == eps[o + a] - eps[i]


def test_generator_recipe():
    eps, L = gwsynth.system(5, 19, 80, 0)
    assert eps.shape == (24,) and L.shape == (80, 24, 24)
    assert np.all(np.diff(eps[:5]) >= 0) and np.all(np.diff(eps[5:]) >= 0)
    assert eps[:5].min() >= -1.5 and eps[:5].max() <= -0.3
    assert eps[5:].min() >= 0.1 and eps[5:].max() <= 3.0
    assert np.array_equal(L, L.transpose(0, 2, 1))
    # the envelope: |p-q| = 8 is damped by e^-1 relative to the diagonal neighbours
    e1, L1 = gwsynth.system(5, 19, 80, 0)
    assert np.array_equal(L, L1)


def test_poles_stable_for_weakly_coupled_orbitals():
    """A fast-decaying factor (decay length 2) leaves the hole-sector zeroth
    moment with a condition number near 1e28.  The shifted/scaled Lanczos
    with noise-aware deflation still returns poles whose moments match every
    conserved moment; the pseudo-inverse cut of T[0] at 1e-12 relative bounds
    the cross-coupling it drops to ~sqrt(1e-12) of the largest element."""
    o, v, A = 6, 60, 50
    eps, L = gwsynth.system(o, v, A, 2, decay=2.0)
    for N in (3, 11):
        so, sv, _ = gw.gw_moments(eps, L, o, N, "tda")
        for T, bound in ((so, 1e-6), (sv, 1e-11)):
            e, vv = gw.poles_from_moments(list(T))
            for n in range(N + 1):
                assert rel((vv * e[None, :] ** n) @ vv.T, T[n]) < bound


def test_shift_scale_is_exact_affine_map():
    """Moments of e' = (e - c)/s computed by the binomial transform equal the
    moments of explicitly mapped poles."""
    rng = np.random.default_rng(3)
    e = rng.uniform(-3, 5, 17)
    vv = rng.standard_normal((4, 17))
    T = [(vv * e ** n) @ vv.T for n in range(8)]
    Ts, c, s = gw.shift_scale(T)
    for n in range(8):
        assert rel(Ts[n], (vv * ((e - c) / s) ** n) @ vv.T) < 1e-12


def test_sigma_rows_match_full_moments():
    """The row-restricted evaluation used for spot checks of large systems
    agrees with the full contraction."""
    o = 3
    eps, L = gwsynth.system(o, 9, 14, 6)
    V, D = gw.particle_hole(eps, L, o)
    R = gw.w_core(gw.tda_eta(V, D, 5), V)
    so, sv, _ = gw.sigma_moments(eps, L, o, R)
    ro, rv = gw.sigma_moment_rows(eps, L, o, R, [0, 4, 11])
    for n in range(6):
        assert rel(ro[n], so[n][[0, 4, 11]]) < 1e-13
        assert rel(rv[n], sv[n][[0, 4, 11]]) < 1e-13
