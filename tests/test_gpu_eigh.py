"""GPU checks of the symmetric eigensolver behind the pole stage (gw_eigh:
own Householder tridiagonalisation, then divide and conquer).

Eigenvalues are compared with LAPACK's (numpy.linalg.eigvalsh) and with
closed forms; eigenvectors through properties that fix them whatever the
sign or the basis inside a degenerate eigenspace: the residual |A V - V W|,
the orthonormality |V V^T - I| and, for well separated eigenvalues, the
agreement of |<v_i, u_i>| with 1 against LAPACK's vectors.  The sizes span
one and several 64-wide tiles, ragged tails, and the 3000 / 4145 orders of
the Lanczos sector and upfolded matrices at nocc 100, nvir 400."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


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


def random_sym(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n)) * scale
    return (B + B.T) / 2.0


def check(handle, A, vec_tol=None, gap_check=True):
    import torch
    n = A.shape[0]
    a = dev(A)
    wd, Vd = handle.eigh(a)
    w, V = host(wd), host(Vd)
    ref = np.linalg.eigvalsh(A)
    norm = max(np.abs(ref).max(), 1e-300)
    assert np.all(np.diff(w) >= 0), "eigenvalues not ascending"
    tol = 50 * n * EPS * norm if vec_tol is None else vec_tol
    assert np.abs(w - ref).max() <= tol, (n, np.abs(w - ref).max(), tol)
    # rows of V are the eigenvectors (products in FP64 on the device)
    res = float((a @ Vd.T - Vd.T * wd).abs().max())
    assert res <= tol, (n, res, tol)
    orth = float((Vd @ Vd.T - torch.eye(n, dtype=torch.float64, device=a.device)).abs().max())
    assert orth <= 50 * n * EPS, (n, orth)
    if gap_check and n <= 1500:
        _, U = np.linalg.eigh(A)
        gap = np.minimum(np.r_[np.inf, np.diff(ref)], np.r_[np.diff(ref), np.inf])
        ok = gap > 1e-6 * norm
        overlap = np.abs(np.einsum("ij,ji->i", V, U))
        assert np.abs(overlap[ok] - 1.0).max() <= 1e-8, (n, np.abs(overlap[ok] - 1.0).max())
    return w, V


@pytest.mark.parametrize("n", [1, 2, 3, 17, 63, 64, 65, 130, 257, 500])
def test_random_symmetric(handle, n):
    check(handle, random_sym(n, 100 + n))


def test_two_by_two_closed_form(handle):
    a, b, c = 0.3, -1.7, 2.2
    A = np.array([[a, b], [b, c]])
    w, _ = check(handle, A)
    m, r = (a + c) / 2, np.hypot((a - c) / 2, b)
    assert np.allclose(w, [m - r, m + r], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [5, 64, 129])
def test_tridiagonal_toeplitz_closed_form(handle, n):
    # tridiag(1, 0, 1): eigenvalues 2 cos(k pi / (n + 1)), k = 1..n
    A = np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)
    w, _ = check(handle, A)
    exact = np.sort(2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    assert np.abs(w - exact).max() <= 50 * n * EPS


@pytest.mark.parametrize("kind", ["zero", "identity", "diagonal", "block"])
def test_degenerate_and_decoupled(handle, kind):
    # zero and already-diagonal columns take the tau = 0 branch of every
    # reflector; repeated eigenvalues leave the basis free (properties only)
    n = 150
    if kind == "zero":
        A = np.zeros((n, n))
    elif kind == "identity":
        A = 3.0 * np.eye(n)
    elif kind == "diagonal":
        A = np.diag(np.repeat([-1.0, 0.5, 2.0], n // 3))
    else:
        A = np.zeros((n, n))
        A[:70, :70] = 2.0 * np.eye(70)
        A[70:, 70:] = random_sym(n - 70, 7)
    check(handle, A, vec_tol=1e-12 * max(1.0, np.abs(A).max()) * n, gap_check=kind == "block")


def test_lower_triangle_only_read(handle):
    # the row-major lower triangle defines the matrix (LAPACK's UPLO='L' on a
    # row-major array): garbage above it must not matter
    n = 97
    A = random_sym(n, 3)
    B = np.tril(A) + np.triu(np.full((n, n), 1e3), 1)
    w, V = handle.eigh(dev(B))
    assert np.abs(host(w) - np.linalg.eigvalsh(A)).max() <= 50 * n * EPS * np.abs(A).max() * 4


def test_input_left_unchanged_and_repeatable(handle):
    n = 200
    A = random_sym(n, 11)
    a = dev(A)
    w1, V1 = handle.eigh(a)
    w2, V2 = handle.eigh(a)
    assert np.array_equal(host(a), A)
    # the reductions sum in a fixed order: two runs agree bit for bit
    assert np.array_equal(host(w1), host(w2)) and np.array_equal(host(V1), host(V2))


@pytest.mark.parametrize("n", [3000, 4145])
def test_pole_stage_orders(handle, n):
    # spread spectrum of the scale of the pole energies (Ha)
    A = random_sym(n, n, scale=0.5) + np.diag(np.linspace(-20.0, 10.0, n))
    check(handle, A, gap_check=False)


@pytest.mark.parametrize("n", [84, 100, 300])
def test_rpa_after_eigensolves_on_the_same_handle(handle, n):
    # the eigensolver must leave the handle's library state intact: RPA
    # moments (batched Cholesky inverses on the same rocBLAS handle) after an
    # eigensolve equal those of a fresh handle
    import gwsynth
    import torch
    from paper_2504_17439_amd import gwmom
    o, v, A, N = 3, 9, 30, 5
    eps, L = gwsynth.system(o, v, A, 4, amp=0.3)
    e, l = dev(eps), dev(L)
    fresh = gwmom.Handle(0)
    try:
        ref = [host(x) for x in fresh.sigma_moments(e, l, o, N, "rpa", "fp64")]
        fresh.eigh(dev(random_sym(n, n)))
        so, sv = fresh.sigma_moments(e, l, o, N, "rpa", "fp64")
        for a, b in zip((host(so), host(sv)), ref):
            assert np.isfinite(a).all()
            assert np.abs(a - b).max() <= 1e-12 * max(1.0, np.abs(b).max())
    finally:
        fresh.close()


def test_rejects_bad_arguments(handle):
    import torch
    from paper_2504_17439_amd import gwmom
    with pytest.raises(gwmom.GWError):
        handle._call("gw_eigh", 0, gwmom._ptr(None), gwmom._ptr(None))
    a = torch.zeros(4, 4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(gwmom.GWError):
        handle._call("gw_eigh", 4, gwmom._ptr(a), gwmom._ptr(None))
