"""Mixed-precision self-energy moments (int8 base-255 fixed-point digits on the
integer MFMA, exact int32 accumulation per digit weight, FP64 combination)
against the FP64 oracle, and the quasiparticle energies they give against
the FP64 path.

The stated bar for the mixed form is on quasiparticle energies: 1e-6 Ha on
the frontier orbitals.  The moments themselves are held to a tolerance
derived from the number format: four signed base-255 digits carry each
operand row or column to ~2^-33 of its power-of-two scale, the kept digit
products (weight <= 3; <= 4 in symmetric products) drop ~2^-32 of the
leading term, and every int32 sum is exact, so the moments carry a
normwise relative error of order 1e-9 (measured <= 7e-10 at full size);
1e-8 relative to the largest element of each moment leaves a factor ~10 of
margin."""
import numpy as np
import pytest

import gwsynth
from oracle import gw as ogw

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-8


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


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("o,v,A,N,seed,scr", [
    (1, 1, 1, 1, 0, "tda"),
    (4, 21, 67, 5, 6, "tda"),
    (5, 19, 80, 3, 0, "tda"),
    (7, 37, 131, 5, 3, "tda"),
    (12, 30, 150, 11, 5, "tda"),
    (3, 45, 260, 7, 4, "tda"),
    (6, 20, 50, 5, 1, "rpa"),
    (7, 37, 131, 7, 3, "rpa"),
    (12, 30, 150, 11, 5, "rpa"),
])
def test_mixed_sigma_matches_oracle(handle, o, v, A, N, seed, scr):
    print(f"\n[case] mixed sigma {scr} o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L = gwsynth.system(o, v, A, seed)
    so_ref, sv_ref, _ = ogw.gw_moments(eps, L, o, N, scr, nquad=48)
    so, sv = handle.sigma_moments(dev(eps), dev(L), o, N, scr, precision="mixed")
    so, sv = host(so), host(sv)
    for n in range(N + 1):
        assert rel(so[n], so_ref[n]) < MIXED_TOL, (n, rel(so[n], so_ref[n]))
        assert rel(sv[n], sv_ref[n]) < MIXED_TOL, (n, rel(sv[n], sv_ref[n]))
        assert np.array_equal(so[n], so[n].T)


@pytest.mark.parametrize("o,v,A,N,seed", [
    (1, 1, 1, 1, 0),
    (5, 19, 80, 3, 0),
    (7, 37, 131, 5, 3),
    (12, 30, 150, 11, 5),
    (3, 45, 260, 7, 4),
])
def test_mixed_tda_moments_match_oracle(handle, o, v, A, N, seed):
    """The digit-product recursion (half-order form): every R_n within the
    format's tolerance of the oracle recursion, and exactly symmetric."""
    print(f"\n[case] mixed tda moments o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L = gwsynth.system(o, v, A, seed)
    V, D = ogw.particle_hole(eps, L, o)
    R_ref = ogw.w_core(ogw.tda_eta(V, D, N), V)
    R = host(handle.moments(dev(eps), dev(L), o, N, "tda", precision="mixed"))
    for n in range(N + 1):
        assert rel(R[n], R_ref[n]) < MIXED_TOL, (n, rel(R[n], R_ref[n]))
        assert np.array_equal(R[n], R[n].T)


@pytest.mark.parametrize("o,v,A,N,seed", [
    (1, 1, 1, 1, 0),
    (6, 20, 50, 5, 1),
    (7, 37, 131, 7, 3),
    (12, 30, 150, 11, 5),
    (3, 45, 260, 7, 4),
])
def test_mixed_rpa_moments_match_oracle(handle, o, v, A, N, seed):
    """The RPA recursion as digit products (eta~^{(0)} from the FP64
    quadrature): every R_n within the format's tolerance of the oracle's
    recursion on the same 48-point rule, and exactly symmetric."""
    print(f"\n[case] mixed rpa moments o={o} v={v} A={A} N={N} seed={seed}", flush=True)
    eps, L = gwsynth.system(o, v, A, seed)
    V, D = ogw.particle_hole(eps, L, o)
    R_ref = ogw.w_core(ogw.rpa_eta(V, D, N, nquad=48), V)
    R = host(handle.moments(dev(eps), dev(L), o, N, "rpa", precision="mixed"))
    for n in range(N + 1):
        assert rel(R[n], R_ref[n]) < MIXED_TOL, (n, rel(R[n], R_ref[n]))
        assert np.array_equal(R[n], R[n].T)


@pytest.mark.parametrize("scr", ["tda", "rpa"])
def test_mixed_moments_long_ragged_rows_and_zero_row(handle, scr):
    """Rows of 4096 or more (nocc nvir) columns take the exponent pass and the
    16-row-tile digit pass: here 7 x 587 = 4109 columns (not a multiple of
    8, so the last 8-column group is partly padding), 40 aux rows (the last
    row tile is partial) and one aux row of L set to zero, whose X_k rows stay
    zero (the exponent pass leaves them unset and the digit pass reads them as
    0).  Every R_n within the format's tolerance of the oracle recursion."""
    o, v, A, N = 7, 587, 40, 5
    print(f"\n[case] mixed {scr} moments long rows o={o} v={v} A={A} N={N}", flush=True)
    eps, L = gwsynth.system(o, v, A, 9)
    L[5] = 0.0
    V, D = ogw.particle_hole(eps, L, o)
    eta = ogw.tda_eta(V, D, N) if scr == "tda" else ogw.rpa_eta(V, D, N, nquad=48)
    R_ref = ogw.w_core(eta, V)
    R = host(handle.moments(dev(eps), dev(L), o, N, scr, precision="mixed"))
    for n in range(N + 1):
        assert rel(R[n], R_ref[n]) < MIXED_TOL, (n, rel(R[n], R_ref[n]))
        assert np.array_equal(R[n], R[n].T)
        if scr == "tda":
            # zero digits give exact zeros (RPA: covered by the tolerance above)
            assert not R[n][5].any() and not R[n][:, 5].any()


def test_mixed_intermediate_cap(handle):
    """The mixed stage-1 intermediates (FP32 + BF16 residual, four digit
    planes and one exponent per row, for all nmo^2 columns) are refused with
    GW_ENOMEM above opts.zchunk_bytes; at exactly their size the result is the
    uncapped one."""
    from paper_2504_17439_amd import gwmom
    o, v, A, N = 4, 21, 70, 5
    eps, L = gwsynth.system(o, v, A, 8)
    e, l = dev(eps), dev(L)
    so1, sv1 = handle.sigma_moments(e, l, o, N, precision="mixed")
    Ap = (A + 63) // 64 * 64
    rows = (N + 1) * (o + v) ** 2
    need = rows * Ap * (4 + 2 + 4) + 4 * rows
    with pytest.raises(gwmom.GWError, match="GW_ENOMEM"):
        handle.sigma_moments(e, l, o, N, precision="mixed", opts={"zchunk_bytes": need - 1})
    so2, sv2 = handle.sigma_moments(e, l, o, N, precision="mixed", opts={"zchunk_bytes": need})
    assert rel(host(so2), host(so1)) < 1e-13 and rel(host(sv2), host(sv1)) < 1e-13


def test_mixed_qp_energies_within_1e6_ha(handle):
    """nmom_max = 11 on a 100-orbital system: QP energies from the mixed
    moments (Lanczos told the moments carry ~1e-9 relative error) agree with
    those from the FP64 moments within 1e-6 Ha on the frontier orbitals."""
    import torch
    o, v, A, N = 20, 80, 300, 11
    print(f"\n[case] mixed QP o={o} v={v} A={A} N={N}", flush=True)
    eps, L = gwsynth.system(o, v, A, 0)
    e, l = dev(eps), dev(L)
    f = torch.diag(e).contiguous()
    so, sv = handle.sigma_moments(e, l, o, N, precision="fp64")
    ref = handle.poles(so, sv, f)
    mo, mv = handle.sigma_moments(e, l, o, N, precision="mixed")
    res = handle.poles(mo, mv, f, opts={"moment_eps": 1e-9})
    qp_ref, w_ref = host(ref["qp"]), host(ref["qp_weight"])
    qp = host(res["qp"])
    front = [p for p in range(o - 5, o + 5) if w_ref[p] >= 0.9]
    assert len(front) >= 6
    err = np.abs(qp[front] - qp_ref[front]).max()
    print(f"frontier QP error {err:.2e} Ha", flush=True)
    assert err < 1e-6
