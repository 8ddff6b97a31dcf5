"""RPA screening at the sizes of its two configurations.

FP64 (nocc=40, nvir=160, naux=600, nmom_max=7, 48-point quadrature): the
density-response and self-energy moments against the oracle computed in full,
and the G0W0 QP energies of the 10 orbitals nearest the Fermi level against
the oracle's block Lanczos and upfolded diagonalisation.

Mixed precision (nocc=100, nvir=400, naux=1500, nmom_max=11): the oracle's
full RPA run at this size takes minutes of CPU, so the mixed moments are
held to the mixed tolerance against the device FP64 form (itself held to the
oracle above and at the small sizes), together with the invariants that hold
at any size and the frontier QP energies within 1e-6 Ha."""
import numpy as np
import pytest

import gwsynth
from oracle import gw as ogw

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def qp_of(so, sv, eps):
    eo, vo = ogw.poles_from_moments(list(so))
    ev, vv = ogw.poles_from_moments(list(sv))
    H = ogw.upfolded_hamiltonian(np.diag(eps), eo, vo, ev, vv)
    E, U = np.linalg.eigh(H)
    qp, _, _ = ogw.qp_assign(E, U[: eps.shape[0]])
    return qp


@pytest.fixture(scope="module")
def handle():
    from paper_2504_17439_amd import gwmom
    h = gwmom.Handle(0)
    yield h
    h.close()


def test_rpa_fp64_config_matches_oracle(handle):
    import torch
    o, v, A, N = 40, 160, 600, 7
    print(f"\n[case] rpa fp64 o={o} v={v} A={A} N={N} seed=0", flush=True)
    eps, L = gwsynth.system(o, v, A, 0)
    so_ref, sv_ref, R_ref = ogw.gw_moments(eps, L, o, N, "rpa", nquad=48)
    e = torch.from_numpy(eps).to("cuda:0")
    l = torch.from_numpy(L).to("cuda:0")
    R = handle.moments(e, l, o, N, "rpa").cpu().numpy()
    so, sv = handle.sigma_moments(e, l, o, N, "rpa")
    p = handle.poles(so, sv, torch.diag(e).contiguous())
    torch.cuda.synchronize()
    so, sv = so.cpu().numpy(), sv.cpu().numpy()
    for n in range(N + 1):
        assert rel(R[n], R_ref[n]) < TOL, ("R", n)
        assert rel(so[n], so_ref[n]) < TOL, ("occ", n)
        assert rel(sv[n], sv_ref[n]) < TOL, ("vir", n)
    qp_ref = qp_of(so_ref, sv_ref, eps)
    front = slice(o - 5, o + 5)
    err = np.abs(p["qp"].cpu().numpy()[front] - qp_ref[front]).max()
    print(f"rpa fp64 frontier QP error {err:.3e} Ha", flush=True)
    assert err < 1e-8


def test_rpa_mixed_config_against_fp64(handle):
    import torch
    o, v, A, N = 100, 400, 1500, 11
    print(f"\n[case] rpa mixed o={o} v={v} A={A} N={N} seed=0", flush=True)
    e, l = gwsynth.system_device(o, v, A, 0)
    R64 = handle.moments(e, l, o, N, "rpa").cpu().numpy()
    Rm = handle.moments(e, l, o, N, "rpa", precision="mixed").cpu().numpy()
    so64, sv64 = handle.sigma_moments(e, l, o, N, "rpa")
    som, svm = handle.sigma_moments(e, l, o, N, "rpa", precision="mixed")
    fock = torch.diag(e).contiguous()
    q64 = handle.poles(so64, sv64, fock)["qp"].cpu().numpy()
    qm = handle.poles(som, svm, fock, opts={"moment_eps": 1e-9})["qp"].cpu().numpy()
    torch.cuda.synchronize()
    errs = [rel(Rm[n], R64[n]) for n in range(N + 1)]
    print("rpa mixed R errors " + " ".join(f"{x:.2e}" for x in errs), flush=True)
    assert max(errs) < 1e-8
    for n in range(N + 1):
        for a, b in ((som[n], so64[n]), (svm[n], sv64[n])):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert rel(a, b) < 1e-8, n
            assert np.array_equal(a, a.T)
        # moments of a PSD response: R_n symmetric, even moments PSD
        assert np.abs(R64[n] - R64[n].T).max() <= 1e-12 * np.abs(R64[n]).max()
        if n % 2 == 0:
            assert np.linalg.eigvalsh(Rm[n]).min() > -1e-8 * np.abs(Rm[n]).max()
    front = slice(o - 5, o + 5)
    err = np.abs(qm[front] - q64[front]).max()
    print(f"rpa mixed frontier QP error vs fp64 {err:.3e} Ha", flush=True)
    assert err < 1e-6
