"""Write the oracle regression fixtures of this folder.

The paper prints no worked example that can be reproduced without its
molecules and basis sets, so the fixtures here are values of the oracle
itself, written by this script (which calls only ``oracle/`` and the seeded
input generator): a later change to the oracle's arithmetic shows up as a
mismatch in ``tests/test_oracle_golden.py`` and has to be justified.

    python tests/golden/make_golden.py [small] [c3_tda] [c3_rpa] [c4_tda]

The full-size fixtures (``c3_*.npz``: sampled rows and QP energies at nocc=100,
nvir=400, naux=1500, nmom_max=11) take minutes of CPU; the GPU tests at that
size compare the device against them instead of running the oracle there.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gwsynth  # noqa: E402
from oracle import brute, gw  # noqa: E402


def c1_tda():
    """Plain FP64 TDA one-shot GW: nocc=5, nvir=19, naux=80, nmom_max=3, seed 0."""
    eps, L = gwsynth.system(5, 19, 80, 0)
    r = gw.g0w0(eps, L, 5, 3, "tda")
    lines = ["# oracle one-shot GW, TDA, nocc=5 nvir=19 naux=80 nmom_max=3, gwsynth.system seed 0",
             "# written by tests/golden/make_golden.py (oracle only)",
             "# section moments: n, |Sigma_occ^(n)|_F, |Sigma_vir^(n)|_F, |R_n|_F"]
    for n in range(4):
        lines.append(f"moment {n} {np.linalg.norm(r['sigma_occ'][n]):.17e} {np.linalg.norm(r['sigma_vir'][n]):.17e} "
                     f"{np.linalg.norm(r['R'][n]):.17e}")
    lines.append("# section qp: p, eps_p, QP energy, QP weight")
    for p in range(24):
        lines.append(f"qp {p} {eps[p]:.17e} {r['qp'][p]:.17e} {r['qp_weight'][p]:.17e}")
    return "\n".join(lines) + "\n"


C3 = (100, 400, 1500, 11)                 # nocc, nvir, naux, nmom_max of the full-size configuration
C3_R_ROWS = [0, 733, 1499]                 # sampled rows P of every R_n
C3_SIGMA_ROWS = [0, 57, 99, 100, 101, 250, 499]   # deepest hole, HOMO, LUMO, ..., highest virtual


def c3_fixture(screening):
    """Oracle one-shot GW at nocc=100, nvir=400, naux=1500, nmom_max=11 (seed 0):
    sampled rows of every R_n and of both self-energy moment sectors, and the
    QP energies / weights of every orbital from the oracle's block Lanczos and
    upfolded diagonalisation.  Minutes of CPU (RPA: the 48-node quadrature)."""
    o, v, A, N = C3
    eps, L = gwsynth.system(o, v, A, 0)
    r = gw.g0w0(eps, L, o, N, screening)
    R = np.asarray(r["R"])
    return dict(
        nocc=o, nvir=v, naux=A, nmom_max=N, seed=0,
        r_rows=np.array(C3_R_ROWS), R_rows=R[:, C3_R_ROWS, :],
        sigma_rows=np.array(C3_SIGMA_ROWS),
        so_rows=r["sigma_occ"][:, C3_SIGMA_ROWS, :], sv_rows=r["sigma_vir"][:, C3_SIGMA_ROWS, :],
        so_absmax=np.abs(r["sigma_occ"]).reshape(N + 1, -1).max(axis=1),
        sv_absmax=np.abs(r["sigma_vir"]).reshape(N + 1, -1).max(axis=1),
        R_absmax=np.abs(R).reshape(N + 1, -1).max(axis=1),
        qp=r["qp"], qp_weight=r["qp_weight"])


C4 = (80, 320, 1400, 7, 400)   # the largest molecule shape of the 64-molecule batch, seed 400
C4_R_ROWS = [0, 699, 1399]
C4_SIGMA_ROWS = [0, 79, 80, 81, 250, 399]


def c4_fixture():
    """Oracle TDA self-energy moments at nocc=80, nvir=320, naux=1400,
    nmom_max=7 (gwsynth.system seed 400; the largest molecule shape of the
    batch workload): sampled rows of every R_n and of both sectors."""
    o, v, A, N, seed = C4
    eps, L = gwsynth.system(o, v, A, seed)
    V, D = gw.particle_hole(eps, L, o)
    R = np.asarray(gw.w_core(gw.tda_eta(V, D, N), V))
    so, sv, _ = gw.sigma_moments(eps, L, o, R)
    return dict(
        nocc=o, nvir=v, naux=A, nmom_max=N, seed=seed,
        r_rows=np.array(C4_R_ROWS), R_rows=R[:, C4_R_ROWS, :],
        sigma_rows=np.array(C4_SIGMA_ROWS),
        so_rows=so[:, C4_SIGMA_ROWS, :], sv_rows=sv[:, C4_SIGMA_ROWS, :],
        so_absmax=np.abs(so).reshape(N + 1, -1).max(axis=1),
        sv_absmax=np.abs(sv).reshape(N + 1, -1).max(axis=1),
        R_absmax=np.abs(R).reshape(N + 1, -1).max(axis=1))


def exact_tiny():
    """Exact full-frequency one-shot GW by brute force: nocc=1, nvir=2, naux=3, seed 5, amp 1."""
    out = []
    for scr in ("tda", "rpa"):
        eps, L = gwsynth.system(1, 2, 3, 5, amp=1.0)
        ex = brute.exact_g0w0(eps, L, 1, scr)
        qp, wt, _ = gw.qp_assign(ex["E"], ex["chi"])
        out.append(f"# exact one-shot GW ({scr}), nocc=1 nvir=2 naux=3, gwsynth.system seed 5 amp 1.0")
        out.append("# p, QP energy, QP weight")
        for p in range(3):
            out.append(f"{scr} {p} {qp[p]:.17e} {wt[p]:.17e}")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    which = sys.argv[1:] or ["small", "c3_tda", "c3_rpa"]
    if "small" in which:
        with open(os.path.join(HERE, "c1_tda_g0w0.txt"), "w") as f:
            f.write(c1_tda())
        with open(os.path.join(HERE, "exact_tiny_g0w0.txt"), "w") as f:
            f.write(exact_tiny())
    for scr in ("tda", "rpa"):
        if f"c3_{scr}" in which:
            np.savez_compressed(os.path.join(HERE, f"c3_{scr}_g0w0.npz"), **c3_fixture(scr))
    if "c4_tda" in which:
        np.savez_compressed(os.path.join(HERE, "c4_tda_sigma.npz"), **c4_fixture())
    print("written", " ".join(which))
