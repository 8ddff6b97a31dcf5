"""Pins of the natural-auxiliary-function compression (Sec. 2.1, eq. NAF):
an orthogonal change of auxiliary basis leaves every product of the
interaction, and so every moment and QP energy, unchanged; a tensor of low
auxiliary rank compresses to exactly that rank; truncation removes exactly
the discarded eigenvalues from the particle-hole Gram matrix."""
import numpy as np

import gwsynth
from oracle import gw, naf


def low_rank(o, v, A, rank, seed):
    """L[P] = sum_r B[P,r] C[r] with C symmetric in (p,q): aux rank `rank`."""
    eps, L = gwsynth.system(o, v, rank, seed)
    rng = np.random.default_rng(seed + 100)
    B = np.linalg.qr(rng.standard_normal((A, rank)))[0]     # orthonormal columns
    return eps, np.tensordot(B, L, axes=(1, 0))


def test_full_rank_naf_is_an_orthogonal_rotation():
    o = 3
    eps, L = gwsynth.system(o, 8, 20, 1)
    Ln, kept, w = naf.naf(L, o, eps_naf=0.0, full_space=True)
    assert Ln.shape[0] == 20
    G = L.reshape(20, -1)
    Gn = Ln.reshape(20, -1)
    assert np.abs(Gn.T @ Gn - G.T @ G).max() < 1e-13 * np.abs(G.T @ G).max()


def test_moments_and_qp_unchanged_without_truncation():
    o = 3
    eps, L = gwsynth.system(o, 8, 20, 1)
    Ln, _, _ = naf.naf(L, o, eps_naf=0.0, full_space=True)
    a = gw.g0w0(eps, L, o, 5, "tda")
    b = gw.g0w0(eps, Ln, o, 5, "tda")
    for n in range(6):
        assert np.abs(a["sigma_occ"][n] - b["sigma_occ"][n]).max() < 1e-12 * np.abs(a["sigma_occ"][n]).max()
    assert np.abs(a["qp"] - b["qp"]).max() < 1e-10


def test_low_rank_tensor_compresses_to_its_rank_exactly():
    o, v, A, rank = 3, 8, 30, 12
    eps, L = low_rank(o, v, A, rank, 2)
    for full in (False, True):
        Ln, kept, w = naf.naf(L, o, eps_naf=1e-10, full_space=full)
        assert Ln.shape[0] == rank
        assert np.abs(w[:-rank]).max() < 1e-12 * w.max()
    Ln, _, _ = naf.naf(L, o, eps_naf=1e-10, full_space=True)
    a = gw.g0w0(eps, L, o, 5, "rpa")
    b = gw.g0w0(eps, Ln, o, 5, "rpa")
    assert np.abs(a["qp"] - b["qp"]).max() < 1e-9


def test_truncation_removes_the_discarded_eigenvalues():
    """|| V^T V - V_naf^T V_naf ||_F^2 = sum of the squared discarded
    eigenvalues of M (ov space)."""
    o = 3
    eps, L = gwsynth.system(o, 8, 20, 3)
    M = naf.naf_matrix(L, o)
    w = np.linalg.eigvalsh(M)
    cut = 0.5 * (w[5] + w[6])                     # drop the six smallest
    Ln, kept, _ = naf.naf(L, o, eps_naf=cut)
    assert Ln.shape[0] == 14
    V = np.ascontiguousarray(L[:, :o, o:]).reshape(20, -1)
    Vn = np.ascontiguousarray(Ln[:, :o, o:]).reshape(14, -1)
    err2 = np.sum((V.T @ V - Vn.T @ Vn) ** 2)
    assert abs(err2 - np.sum(w[:6] ** 2)) < 1e-10 * np.sum(w[:6] ** 2)
