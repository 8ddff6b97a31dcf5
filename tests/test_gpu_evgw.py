"""Eigenvalue self-consistent moment GW (gw_evgw) against the oracle loop of
App. A, Alg. A1, and against the same loop on the exact self-energy where
the moments resolve every pole."""
import numpy as np
import pytest

import gwsynth
from oracle import brute, evgw

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


@pytest.mark.parametrize("diis", [12, 0])
@pytest.mark.parametrize("screening", ["tda", "rpa"])
@pytest.mark.parametrize("g0,w0", [(False, False), (False, True), (True, True)])
def test_evgw_matches_oracle(handle, screening, g0, w0, diis):
    o, v, A, N = 3, 9, 30, 5
    print(f"\n[case] evgw {screening} g0={g0} w0={w0} diis={diis}", flush=True)
    eps, L = gwsynth.system(o, v, A, 4, amp=0.3)
    ref = evgw.evgw(eps, L, o, N, screening, g0=g0, w0=w0, tol=1e-9, max_iter=40, diis_space=diis)
    r = handle.evgw(dev(eps), dev(L), o, N, screening, g0=g0, w0=w0, tol=1e-9, max_iter=40, diis_space=diis)
    assert ref["converged"] and r["converged"]
    assert abs(r["iterations"] - ref["iterations"]) <= (1 if diis else 0)
    assert np.abs(host(r["qp"]) - ref["qp"]).max() < 1e-8
    assert np.abs(host(r["qp_weight"]) - ref["qp_weight"]).max() < 1e-8


def test_evgw_equals_exact_self_energy_loop(handle):
    o = 1
    eps, L = gwsynth.system(o, 2, 3, 5, amp=1.0)
    ex = evgw.evgw(eps, L, o, 3, "tda", tol=1e-11, max_iter=60,
                   step=lambda er, eg, ew: brute.exact_ev_step(er, eg, ew, L, o, "tda"))
    r = handle.evgw(dev(eps), dev(L), o, 3, "tda", tol=1e-11, max_iter=60)
    assert ex["converged"] and r["converged"]
    assert np.abs(host(r["qp"]) - ex["qp"]).max() < 1e-9


def test_mixed_evgw_frontier_within_1e6(handle):
    """Mixed-precision evGW: the frontier QP energies follow the FP64 loop to
    well within 1e-6 Ha.  The whole-spectrum convergence test is not asked
    of it: the Lanczos deflation of moments known to ~1e-9 can keep or drop a
    direction differently from one iteration to the next, which moves some
    deeper orbitals by ~1e-5 Ha and can keep them cycling."""
    o, v, A, N = 20, 80, 300, 7
    eps, L = gwsynth.system(o, v, A, 3)
    e, l = dev(eps), dev(L)
    r64 = handle.evgw(e, l, o, N, "tda", tol=1e-8)
    assert r64["converged"]
    rmx = handle.evgw(e, l, o, N, "tda", precision="mixed", tol=1e-8, max_iter=r64["iterations"] + 2,
                      opts={"moment_eps": 1e-9}, allow_noconv=True)
    q64, qmx = host(r64["qp"]), host(rmx["qp"])
    front = slice(o - 5, o + 5)
    err = np.abs(qmx[front] - q64[front]).max()
    print(f"mixed evGW frontier error {err:.2e} Ha after {rmx['iterations']} iterations (FP64: "
          f"{r64['iterations']}), last change {rmx['last_change']:.2e}", flush=True)
    assert err < 1e-6


def test_diis_converges_where_the_plain_loop_stalls(handle):
    o = 3
    eps, L = gwsynth.system(o, 9, 20, 6, amp=0.3)
    e, l = dev(eps), dev(L)
    plain = handle.evgw(e, l, o, 5, "tda", max_iter=40, diis_space=0, allow_noconv=True)
    d = handle.evgw(e, l, o, 5, "tda", max_iter=40)
    ref = evgw.evgw(eps, L, o, 5, "tda", max_iter=40)
    assert not plain["converged"] and d["converged"] and ref["converged"]
    w = host(d["qp_weight"])
    qpl = (w >= 0.9) & (ref["qp_weight"] >= 0.9)
    assert np.abs(host(d["qp"]) - ref["qp"])[qpl].max() < 1e-7


def test_evgw_rejects_bad_options_and_reports_no_convergence(handle):
    from paper_2504_17439_amd import gwmom
    o = 3
    eps, L = gwsynth.system(o, 9, 30, 4, amp=0.3)
    e, l = dev(eps), dev(L)
    with pytest.raises(gwmom.GWError, match="GW_EINVAL"):
        handle.evgw(e, l, o, 4, "tda")
    with pytest.raises(gwmom.GWError, match="GW_ENOCONV"):
        handle.evgw(e, l, o, 5, "tda", tol=1e-14, max_iter=2)
    r = handle.evgw(e, l, o, 5, "tda", tol=1e-14, max_iter=2, allow_noconv=True)
    assert r["iterations"] == 2 and not r["converged"] and r["last_change"] > 0


def test_fp64_evgw_converges_at_full_size_with_the_loop_deflation(handle):
    """nocc=100, nvir=400, naux=1500, N=11 (seed 0): deflating at the unit
    roundoff the FP64 loop keeps poles resolved from rounding noise and stays
    above a 1e-6 Ha residual; at the loop's default deflation (1e-12) it
    converges in a few iterations, the frontier QPs where the stalled loop
    has them; the mixed loop's frontier QPs within 1e-6 Ha of the FP64 loop's."""
    o, v, A, N = 100, 400, 1500, 11
    print(f"\n[case] evgw fp64 full size o={o} v={v} A={A} N={N}", flush=True)
    eps, L = gwsynth.system(o, v, A, 0)
    e, l = dev(eps), dev(L)
    del L
    r = handle.evgw(e, l, o, N, "tda", tol=1e-6, max_iter=10)
    assert r["converged"] and r["iterations"] <= 6
    s = handle.evgw(e, l, o, N, "tda", tol=1e-6, max_iter=8, opts={"moment_eps": float(np.finfo(float).eps)},
                    allow_noconv=True)
    assert not s["converged"]
    q, qs = host(r["qp"]), host(s["qp"])
    print(f"frontier difference {np.abs(q[o - 1:o + 1] - qs[o - 1:o + 1]).max():.2e} Ha, stalled residual "
          f"{s['last_change']:.2e}", flush=True)
    assert np.abs(q[o - 1:o + 1] - qs[o - 1:o + 1]).max() < 1e-7
    m = handle.evgw(e, l, o, N, "tda", precision="mixed", tol=1e-6, max_iter=10, opts={"moment_eps": 1e-9})
    assert m["converged"]
    assert np.abs(host(m["qp"])[o - 1:o + 1] - q[o - 1:o + 1]).max() < 1e-6
