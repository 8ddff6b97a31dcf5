"""GPU parity: the HIP path through the C ABI against the FP64 oracle,
element by element on the same seeded inputs (FP64 bar: 1e-10 relative to
the largest element of each moment)."""
import numpy as np
import pytest

import gwsynth
from oracle import gw as ogw

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def handle():
    import torch
    from paper_2504_17439_amd import gwmom
    assert torch.cuda.is_available()
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


# (nocc, nvir, naux, nmom_max, seed): tiny, the small FP64 TDA case, ragged
# multi-tile cases and a degenerate one-pair case
CASES = [
    (1, 1, 1, 1, 0),
    (5, 19, 80, 3, 0),
    (7, 37, 131, 5, 3),
    (3, 45, 260, 7, 4),
    (12, 30, 150, 11, 5),
    (4, 21, 67, 5, 6),        # odd nmo and odd naux: the lone-element edges of the fold's operands
]


@pytest.mark.parametrize("o,v,A,N,seed", CASES)
def test_tda_moments(handle, o, v, A, N, seed):
    print(f"\n[case] tda moments o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L = gwsynth.system(o, v, A, seed)
    V, D = ogw.particle_hole(eps, L, o)
    eta_ref = ogw.tda_eta(V, D, N)
    R_ref = ogw.w_core(eta_ref, V)
    R, eta = handle.moments(dev(eps), dev(L), o, N, "tda", eta=True)
    R, eta = host(R), host(eta)
    for n in range(N + 1):
        assert rel(R[n], R_ref[n]) < TOL, n
        assert rel(eta[n], eta_ref[n]) < TOL, n
        assert np.array_equal(R[n], R[n].T)
    # without eta the device uses the half-order products (R_2k = X_k X_k^T,
    # R_2k+1 = X_k D X_k^T + 2 R_k R_k): same moments, different rounding
    R2 = host(handle.moments(dev(eps), dev(L), o, N, "tda"))
    for n in range(N + 1):
        assert rel(R2[n], R_ref[n]) < TOL, n
        assert rel(R2[n], R[n]) < TOL, n
        assert np.array_equal(R2[n], R2[n].T)


@pytest.mark.parametrize("o,v,A,N,seed", CASES)
def test_tda_sigma(handle, o, v, A, N, seed):
    print(f"\n[case] tda sigma o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L = gwsynth.system(o, v, A, seed)
    so_ref, sv_ref, _ = ogw.gw_moments(eps, L, o, N, "tda")
    so, sv = handle.sigma_moments(dev(eps), dev(L), o, N, "tda")
    so, sv = host(so), host(sv)
    for n in range(N + 1):
        assert rel(so[n], so_ref[n]) < TOL, n
        assert rel(sv[n], sv_ref[n]) < TOL, n
        assert np.array_equal(so[n], so[n].T) and np.array_equal(sv[n], sv[n].T)


def test_sigma_intermediate_cap(handle):
    """The folded intermediate ((N+1) naux nmo^2 doubles: every (x, q) column,
    each symmetric pair formed once) is refused with GW_ENOMEM, outputs
    untouched, when opts.zchunk_bytes is below it; at exactly its size the
    result equals the uncapped one."""
    import torch
    from paper_2504_17439_amd import gwmom
    o, v, A, N = 4, 21, 70, 5
    print(f"\n[case] intermediate cap o={o} v={v} A={A} N={N}", flush=True)
    eps, L = gwsynth.system(o, v, A, 8)
    e, l = dev(eps), dev(L)
    so1, sv1 = handle.sigma_moments(e, l, o, N, "tda")
    need = (N + 1) * A * (o + v) ** 2 * 8
    out = (torch.full((N + 1, o + v, o + v), 3.0, dtype=torch.float64, device="cuda:0"),
           torch.full((N + 1, o + v, o + v), 3.0, dtype=torch.float64, device="cuda:0"))
    with pytest.raises(gwmom.GWError, match="GW_ENOMEM"):
        handle.sigma_moments(e, l, o, N, "tda", opts={"zchunk_bytes": need - 8}, out=out)
    assert bool((out[0] == 3.0).all()) and bool((out[1] == 3.0).all())
    so2, sv2 = handle.sigma_moments(e, l, o, N, "tda", opts={"zchunk_bytes": need})
    so1, sv1, so2, sv2 = map(host, (so1, sv1, so2, sv2))
    assert rel(so2, so1) < 1e-13 and rel(sv2, sv1) < 1e-13


RPA_CASES = [
    (1, 1, 1, 1, 0),
    (6, 20, 50, 5, 1),
    (7, 37, 131, 7, 3),
    (4, 21, 67, 5, 6),
]


@pytest.mark.parametrize("o,v,A,N,seed", RPA_CASES)
def test_rpa_moments(handle, o, v, A, N, seed):
    print(f"\n[case] rpa moments o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L = gwsynth.system(o, v, A, seed)
    V, D = ogw.particle_hole(eps, L, o)
    eta_ref = ogw.rpa_eta(V, D, N, nquad=48)
    R_ref = ogw.w_core(eta_ref, V)
    R, eta = handle.moments(dev(eps), dev(L), o, N, "rpa", eta=True)
    R, eta = host(R), host(eta)
    for n in range(N + 1):
        assert rel(R[n], R_ref[n]) < TOL, n
        assert rel(eta[n], eta_ref[n]) < TOL, n


@pytest.mark.parametrize("o,v,A,N,seed", RPA_CASES[1:])
def test_rpa_sigma(handle, o, v, A, N, seed):
    print(f"\n[case] rpa sigma o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L = gwsynth.system(o, v, A, seed)
    so_ref, sv_ref, _ = ogw.gw_moments(eps, L, o, N, "rpa", nquad=48)
    so, sv = handle.sigma_moments(dev(eps), dev(L), o, N, "rpa")
    so, sv = host(so), host(sv)
    for n in range(N + 1):
        assert rel(so[n], so_ref[n]) < TOL, n
        assert rel(sv[n], sv_ref[n]) < TOL, n


def test_rpa_quadrature_options(handle):
    """nquad and quad_scale reach the device grid: 24 points at scale 1.7
    match the oracle with the same grid."""
    o, v, A, N = 5, 15, 40, 3
    eps, L = gwsynth.system(o, v, A, 2)
    V, D = ogw.particle_hole(eps, L, o)
    R_ref = ogw.w_core(ogw.rpa_eta(V, D, N, nquad=24, scale=1.7), V)
    R = host(handle.moments(dev(eps), dev(L), o, N, "rpa", opts={"nquad": 24, "quad_scale": 1.7}))
    for n in range(N + 1):
        assert rel(R[n], R_ref[n]) < TOL


def test_invalid_arguments_rejected(handle):
    from paper_2504_17439_amd import gwmom
    eps, L = gwsynth.system(3, 5, 7, 0)
    e, l = dev(eps), dev(L)
    with pytest.raises(gwmom.GWError) as ei:
        handle.moments(e, l, 3, 2, "tda")             # even nmom_max
    assert ei.value.status == gwmom.GW_EINVAL
    bad = eps.copy()
    bad[0] = 5.0                                      # occupied above virtual
    with pytest.raises(gwmom.GWError) as ei:
        handle.moments(dev(bad), l, 3, 3, "tda")
    assert ei.value.status == gwmom.GW_EINVAL
    bad = eps.copy()
    bad[4] = np.nan
    with pytest.raises(gwmom.GWError) as ei:
        handle.sigma_moments(dev(bad), l, 3, 3, "tda")
    assert ei.value.status == gwmom.GW_EINVAL
