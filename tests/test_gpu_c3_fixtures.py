"""Full-size parity against stored oracle results (nocc=100, nvir=400,
naux=1500, nmom_max=11, seed 0; TDA and RPA screening, FP64 and mixed).

The oracle needs minutes of CPU at this size (the RPA quadrature alone runs
48 nodes of 1500 x 40000 x 1500 products), so tests/golden/make_golden.py
(oracle only) stored sampled rows of every R_n and of both self-energy
sectors, and the oracle's QP energies and weights from its own block Lanczos
and upfolded diagonalisation.  The device runs on the same host-generated
inputs.  Bars: FP64 1e-10 relative to the largest element of each moment;
mixed 1e-8 (the digit format's truncation); QP energies of the orbitals near
the Fermi level with QP weight >= 0.9 (the frontier set): 1e-8 Ha (FP64) and
1e-6 Ha (mixed)."""
import os

import numpy as np
import pytest

import gwsynth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
O, V_, A, N = 100, 400, 1500, 11
FRONT = slice(O - 5, O + 5)   # HOMO-4 .. LUMO+4


def fixture(scr):
    f = np.load(os.path.join(HERE, "golden", f"c3_{scr}_g0w0.npz"))
    assert (int(f["nocc"]), int(f["nvir"]), int(f["naux"]), int(f["nmom_max"])) == (O, V_, A, N)
    return {k: f[k] for k in f.files}


@pytest.fixture(scope="module")
def c3_inputs():
    import torch
    from paper_2504_17439_amd import gwmom
    print("\n[case] full-size fixtures o=100 v=400 A=1500 N=11 seed=0 (host inputs)", flush=True)
    eps, L = gwsynth.system(O, V_, A, 0)
    h = gwmom.Handle(0)
    e = torch.from_numpy(eps).to("cuda:0")
    l = torch.from_numpy(L).to("cuda:0")
    yield dict(h=h, e=e, l=l, eps=eps)
    h.close()


def run(c3, scr, prec):
    import torch
    h, e, l = c3["h"], c3["e"], c3["l"]
    print(f"[case] {scr} {prec}", flush=True)
    R = h.moments(e, l, O, N, scr, precision=prec)
    so, sv = h.sigma_moments(e, l, O, N, scr, precision=prec)
    opts = {"moment_eps": 1e-9} if prec == "mixed" else None
    p = h.poles(so, sv, torch.diag(e).contiguous(), opts=opts)
    torch.cuda.synchronize()
    return dict(R=R.cpu().numpy(), so=so.cpu().numpy(), sv=sv.cpu().numpy(), qp=p["qp"].cpu().numpy(),
                qw=p["qp_weight"].cpu().numpy())


def check(out, ref, tol, qp_tol, label):
    rows_r, rows_s = list(ref["r_rows"]), list(ref["sigma_rows"])
    worst = {"R": 0.0, "so": 0.0, "sv": 0.0}
    for n in range(N + 1):
        er = np.abs(out["R"][n][rows_r] - ref["R_rows"][n]).max() / ref["R_absmax"][n]
        eo = np.abs(out["so"][n][rows_s] - ref["so_rows"][n]).max() / ref["so_absmax"][n]
        ev = np.abs(out["sv"][n][rows_s] - ref["sv_rows"][n]).max() / ref["sv_absmax"][n]
        worst["R"], worst["so"], worst["sv"] = max(worst["R"], er), max(worst["so"], eo), max(worst["sv"], ev)
        assert er < tol, (label, "R", n, er)
        assert eo < tol, (label, "sigma_occ", n, eo)
        assert ev < tol, (label, "sigma_vir", n, ev)
    # frontier: weight >= 0.9 in the oracle and on the device (reading R6)
    idx = [p for p in range(O - 5, O + 5) if ref["qp_weight"][p] >= 0.9 and out["qw"][p] >= 0.9]
    assert len(idx) >= 6, idx
    qerr = np.abs(out["qp"][idx] - ref["qp"][idx]).max()
    print(f"{label}: R {worst['R']:.2e}  sigma_occ {worst['so']:.2e}  sigma_vir {worst['sv']:.2e}  "
          f"frontier QP {qerr:.2e} Ha over {len(idx)} orbitals", flush=True)
    assert qerr < qp_tol, (label, qerr)


@pytest.mark.parametrize("scr", ["rpa", "tda"])
def test_c3_fp64_matches_oracle_fixture(c3_inputs, scr):
    check(run(c3_inputs, scr, "fp64"), fixture(scr), 1e-10, 1e-8, f"{scr} fp64")


@pytest.mark.parametrize("scr", ["rpa", "tda"])
def test_c3_mixed_matches_oracle_fixture(c3_inputs, scr):
    check(run(c3_inputs, scr, "mixed"), fixture(scr), 1e-8, 1e-6, f"{scr} mixed")
