"""Write the oracle regression fixtures of this folder.

The paper prints no worked example that can be reproduced without its
molecules and basis sets, so the fixtures here are values of the oracle
itself, written by this script (which calls only ``oracle/`` and the seeded
input generator): a later change to the oracle's arithmetic shows up as a
mismatch in ``tests/test_oracle_golden.py`` and has to be justified.

    python tests/golden/make_golden.py
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
    with open(os.path.join(HERE, "c1_tda_g0w0.txt"), "w") as f:
        f.write(c1_tda())
    with open(os.path.join(HERE, "exact_tiny_g0w0.txt"), "w") as f:
        f.write(exact_tiny())
    print("written")
