"""GPU parity for the auxiliary poles, the upfolded Hamiltonian and the QP
energies.  Several block-Lanczos gauges are equally correct, so only
gauge-invariant quantities are compared: the moments the poles reproduce,
the sorted pole energies, the spectrum of H~ and the QP energies/weights."""
import numpy as np
import pytest

import gwsynth
from oracle import brute
from oracle import gw as ogw

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


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


def run(handle, o, v, A, N, seed, screening="tda"):
    eps, L = gwsynth.system(o, v, A, seed)
    e, l = dev(eps), dev(L)
    so, sv = handle.sigma_moments(e, l, o, N, screening)
    out = handle.poles(so, sv, dev(np.diag(eps)))
    res = {k: (host(x) if x is not None else None) for k, x in out.items() if k != "packed"}
    res["sigma_occ"], res["sigma_vir"] = host(so), host(sv)
    return eps, L, res


@pytest.mark.parametrize("o,v,A,N,seed", [(5, 19, 80, 3, 0), (4, 12, 30, 7, 11), (6, 30, 100, 11, 2)])
def test_poles_reproduce_moments(handle, o, v, A, N, seed):
    print(f"\n[case] poles o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L, r = run(handle, o, v, A, N, seed)
    for key, T in (("occ", r["sigma_occ"]), ("vir", r["sigma_vir"])):
        e, vv = r["e_" + key], r["v_" + key]
        assert e.shape[0] == (o + v) * (N + 1) // 2
        for n in range(N + 1):
            assert rel((vv * e[None, :] ** n) @ vv.T, T[n]) < 1e-9, (key, n)


@pytest.mark.parametrize("o,v,A,N,seed", [(5, 19, 80, 3, 0), (4, 12, 30, 7, 11)])
def test_poles_and_qp_match_oracle(handle, o, v, A, N, seed):
    print(f"\n[case] qp o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L, r = run(handle, o, v, A, N, seed)
    ref = ogw.g0w0(eps, L, o, N, "tda")
    assert np.abs(np.sort(r["e_occ"]) - np.sort(ref["e_occ"])).max() < 1e-9
    assert np.abs(np.sort(r["e_vir"]) - np.sort(ref["e_vir"])).max() < 1e-9
    assert np.abs(r["E"] - ref["E"]).max() < 1e-9
    assert np.abs(r["qp"] - ref["qp"]).max() < 1e-9
    assert np.abs(r["qp_weight"] - ref["qp_weight"]).max() < 1e-8
    # the physical block of the eigenvectors is a partial isometry row-wise:
    # sum_alpha chi_{p alpha} chi_{q alpha} = delta_pq
    chi = r["chi"]
    assert np.abs(chi @ chi.T - np.eye(o + v)).max() < 1e-10


def test_exact_when_pole_count_fits(handle):
    """o=1, v=2, naux=3, N=3: the moment expansion is exact (rank-deficient
    moments exercise the pseudo-inverse path) and matches full-frequency G0W0."""
    o = 1
    eps, L = gwsynth.system(o, 2, 3, 5, amp=1.0)
    so, sv = handle.sigma_moments(dev(eps), dev(L), o, 3, "tda")
    r = {k: (host(x) if x is not None else None) for k, x in handle.poles(so, sv, dev(np.diag(eps))).items()
         if k != "packed"}
    ex = brute.exact_g0w0(eps, L, o, "tda")
    qp_ex, w_ex, _ = ogw.qp_assign(ex["E"], ex["chi"])
    assert np.abs(r["qp"] - qp_ex).max() < 1e-8
    assert np.abs(r["qp_weight"] - w_ex).max() < 1e-8


def test_non_psd_moment_is_rejected(handle):
    from paper_2504_17439_amd import gwmom
    nmo, N = 3, 1
    so = np.zeros((N + 1, nmo, nmo))
    so[0] = np.diag([1.0, -0.5, 0.2])
    so[1] = np.eye(nmo)
    sv = np.zeros((N + 1, nmo, nmo))
    sv[0] = np.eye(nmo)
    sv[1] = np.eye(nmo)
    with pytest.raises(gwmom.GWError) as ei:
        handle.poles(dev(so), dev(sv), dev(np.eye(nmo)))
    assert ei.value.status == gwmom.GW_ENUMERIC
