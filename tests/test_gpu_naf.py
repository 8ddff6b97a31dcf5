"""Natural auxiliary functions on the device (gw_naf) against the oracle,
and the compressed tensor in the hot path."""
import numpy as np
import pytest

import gwsynth
from oracle import gw, naf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    from paper_2504_17439_amd import gwmom
    h = gwmom.Handle(0)
    yield h
    h.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def low_rank(o, v, A, rank, seed):
    eps, L = gwsynth.system(o, v, rank, seed)
    rng = np.random.default_rng(seed + 100)
    B = np.linalg.qr(rng.standard_normal((A, rank)))[0]
    return eps, np.tensordot(B, L, axes=(1, 0))


@pytest.mark.parametrize("full", [False, True])
def test_naf_matches_oracle(handle, full):
    o, v, A = 5, 19, 80
    eps, L = gwsynth.system(o, v, A, 0)
    w_ref = np.linalg.eigvalsh(naf.naf_matrix(L, o, full))
    cut = 0.5 * (w_ref[20] + w_ref[21])                   # keep 59 of 80
    Ln_ref, kept, _ = naf.naf(L, o, cut, full)
    Ln, w = handle.naf(dev(L), o, cut, full)
    assert Ln.shape[0] == Ln_ref.shape[0] == 59
    assert np.abs(host(w) - w_ref).max() < 1e-12 * w_ref.max()
    # sign-invariant: the projected Gram matrix over all orbital pairs
    G = host(Ln).reshape(59, -1)
    G_ref = Ln_ref.reshape(59, -1)
    gg, gg_ref = G.T @ G, G_ref.T @ G_ref
    assert np.abs(gg - gg_ref).max() < 1e-11 * np.abs(gg_ref).max()


def test_compressed_low_rank_tensor_gives_the_same_moments(handle):
    o, v, A, rank, N = 10, 40, 150, 90, 7
    eps, L = low_rank(o, v, A, rank, 3)
    e, l = dev(eps), dev(L)
    cut = 1e-9 * np.linalg.eigvalsh(naf.naf_matrix(L, o, True)).max()
    Ln, w = handle.naf(l, o, cut, full_space=True)
    assert Ln.shape[0] == rank
    so, sv = handle.sigma_moments(e, l, o, N, "tda")
    so_n, sv_n = handle.sigma_moments(e, Ln.contiguous(), o, N, "tda")
    for a, b in ((so, so_n), (sv, sv_n)):
        a, b = host(a), host(b)
        for n in range(N + 1):
            assert np.abs(a[n] - b[n]).max() < 1e-10 * np.abs(a[n]).max(), n
    # and the oracle's G0W0 on the oracle's compressed tensor
    Ln_ref, _, _ = naf.naf(L, o, cut, full_space=True)
    ref = gw.g0w0(eps, Ln_ref, o, N, "tda")
    fock = dev(np.diag(eps))
    res = handle.poles(so_n, sv_n, fock)
    front = slice(o - 3, o + 3)
    assert np.abs(host(res["qp"])[front] - ref["qp"][front]).max() < 1e-8


def test_naf_rejects_bad_arguments(handle):
    from paper_2504_17439_amd import gwmom
    eps, L = gwsynth.system(3, 9, 30, 1)
    with pytest.raises(gwmom.GWError, match="GW_EINVAL"):
        handle.naf(dev(L), 3, -1.0)
    with pytest.raises(gwmom.GWError, match="GW_ENUMERIC"):
        handle.naf(dev(L), 3, 1e30)
