"""fsGW on the device (gw_fsgw) against the oracle loop (Sec. 3.6, Alg. 2).

Small systems: the converged Fock matrix and the sorted QP energies agree
with the oracle (1e-6 Ha, the QP bar; both loops stop when an iteration
changes F by less than 1e-6 Ha).  At the learned-warm-start test size
(nmo = 300, naux = 1050, nocc = 60, N = 5, H~ of dimension 2100) the oracle
loop is too slow to run, so the test checks what holds at any size: the loop
converges, a warm start from its own converged F is a fixed point (one
iteration, the same QP energies for the orbitals with QP weight >= 0.9 --
satellite-embedded orbitals have no stable assignment, reading R6), and
mixed-precision self-energies give the same frontier QPs.
"""
import numpy as np
import pytest

import gwsynth
from oracle import fsgw as ofs

pytestmark = pytest.mark.gpu

QP_TOL = 1e-6


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


def physical_qp_diff(a, b):
    """Largest QP difference over the orbitals whose QP weight is >= 0.9 in
    both loops (orbitals of each loop's final F, ascending)."""
    qa, wa, qb, wb = host(a["qp"]), host(a["qp_weight"]), host(b["qp"]), host(b["qp_weight"])
    m = (wa >= 0.9) & (wb >= 0.9)
    assert m.sum() >= 0.5 * len(m)
    return float(np.abs(qa[m] - qb[m]).max())


@pytest.mark.parametrize("o,v,A,N,seed,scr", [
    (3, 9, 20, 3, 1, "tda"),
    (4, 16, 42, 5, 2, "tda"),
    (3, 9, 20, 3, 1, "rpa"),
    (5, 14, 37, 3, 6, "tda"),
])
def test_fsgw_matches_oracle(handle, o, v, A, N, seed, scr):
    print(f"\n[case] fsgw {scr} o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L = gwsynth.system(o, v, A, seed)
    ref = ofs.fsgw(eps, L, o, N, screening=scr)
    assert ref["converged"]
    r = handle.fsgw(dev(eps), dev(L), o, N, screening=scr)
    assert r["converged"]
    qp = np.sort(host(r["qp"]))
    assert np.abs(qp - ref["qp"]).max() < QP_TOL
    assert np.abs(host(r["F"]) - ref["F"]).max() < QP_TOL
    # the iteration counts depend on where the two loops' rounding puts the
    # last QP changes relative to the 1e-6 threshold: reported, not compared
    print(f"iterations device {r['iterations']} oracle {ref['iterations']}", flush=True)


def test_fsgw_warm_start_from_its_fixed_point(handle):
    o, v, A, N = 4, 16, 42, 5
    eps, L = gwsynth.system(o, v, A, 2)
    e, l = dev(eps), dev(L)
    r = handle.fsgw(e, l, o, N)
    w = handle.fsgw(e, l, o, N, F0=r["F"])
    assert w["iterations"] == 1
    assert physical_qp_diff(w, r) < QP_TOL


@pytest.fixture(scope="module")
def c5_run(handle):
    o, v, A, N = 60, 240, 1050, 5
    print(f"\n[case] fsgw nmo={o + v} naux={A} N={N}", flush=True)
    eps, L = gwsynth.system(o, v, A, 10001)
    e, l = dev(eps), dev(L)
    r = handle.fsgw(e, l, o, N)
    print(f"iterations {r['iterations']} fock steps {r['fock_steps']} eigensolves {r['eig_calls']}", flush=True)
    return o, N, e, l, r


def test_fsgw_converges_at_warm_start_test_size(c5_run):
    o, N, e, l, r = c5_run
    assert r["converged"] and r["iterations"] <= 30
    assert 0 <= r["last_dF"] < QP_TOL
    print(f"last F change {r['last_dF']:.2e}, last sorted-QP change {r['last_dqp']:.2e}", flush=True)
    qp = host(r["qp"])
    assert np.all(np.isfinite(qp))
    F = host(r["F"])
    assert np.abs(F - F.T).max() < 1e-10


def test_fsgw_fixed_point_at_warm_start_test_size(handle, c5_run):
    o, N, e, l, r = c5_run
    w = handle.fsgw(e, l, o, N, F0=r["F"])
    assert w["iterations"] == 1
    assert physical_qp_diff(w, r) < QP_TOL


def test_fsgw_mixed_self_energy_same_frontier_qps(handle):
    o, v, A, N = 20, 80, 300, 5
    print(f"\n[case] fsgw mixed vs fp64 o={o} v={v} A={A} N={N}", flush=True)
    eps, L = gwsynth.system(o, v, A, 3)
    e, l = dev(eps), dev(L)
    ref = handle.fsgw(e, l, o, N)
    mix = handle.fsgw(e, l, o, N, precision="mixed", opts={"moment_eps": 1e-9})
    assert mix["converged"]
    qr, wr = host(ref["qp"]), host(ref["qp_weight"])
    qm = host(mix["qp"])
    front = [p for p in range(o - 5, o + 5) if wr[p] >= 0.9]
    assert len(front) >= 6
    assert np.abs(qm[front] - qr[front]).max() < QP_TOL


def test_fsgw_rejects_bad_arguments(handle):
    from paper_2504_17439_amd import gwmom
    eps, L = gwsynth.system(3, 9, 20, 1)
    e, l = dev(eps), dev(L)
    with pytest.raises(gwmom.GWError, match="GW_EINVAL"):
        handle.fsgw(e, l, 3, 4)
    with pytest.raises(ValueError):
        handle.fsgw(e, l, 3, 3, F0=dev(np.eye(5)))
    with pytest.raises(gwmom.GWError, match="GW_EINVAL"):
        handle.fsgw(e, l, 3, 3, fopts={"tol": -1.0})
