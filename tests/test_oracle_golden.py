"""The oracle against its own stored values (tests/golden, written by
tests/golden/make_golden.py from the oracle alone): a change to the oracle's
arithmetic that moves them must come with the reading of the paper that
justifies it.  The paper prints no worked example that can be reproduced
without its molecules and basis sets, so these are regression values, not
paper values; the pins of the method itself are in the other oracle tests."""
import os

import numpy as np

import gwsynth
from oracle import brute, gw

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rows(name, tag):
    out = []
    for line in open(os.path.join(HERE, name)):
        if line.startswith(tag + " "):
            out.append([float(x) for x in line.split()[1:]])
    return np.array(out)


def test_c1_tda_one_shot_regression():
    eps, L = gwsynth.system(5, 19, 80, 0)
    r = gw.g0w0(eps, L, 5, 3, "tda")
    mom = rows("c1_tda_g0w0.txt", "moment")
    for n, so, sv, rn in mom:
        n = int(n)
        assert abs(np.linalg.norm(r["sigma_occ"][n]) - so) <= 1e-12 * so
        assert abs(np.linalg.norm(r["sigma_vir"][n]) - sv) <= 1e-12 * sv
        assert abs(np.linalg.norm(r["R"][n]) - rn) <= 1e-12 * rn
    qp = rows("c1_tda_g0w0.txt", "qp")
    assert qp.shape == (24, 4)
    assert np.array_equal(qp[:, 1], eps)
    assert np.abs(r["qp"] - qp[:, 2]).max() < 1e-10
    assert np.abs(r["qp_weight"] - qp[:, 3]).max() < 1e-10


def test_exact_tiny_one_shot_regression():
    for scr in ("tda", "rpa"):
        eps, L = gwsynth.system(1, 2, 3, 5, amp=1.0)
        ex = brute.exact_g0w0(eps, L, 1, scr)
        qp, wt, _ = gw.qp_assign(ex["E"], ex["chi"])
        ref = rows("exact_tiny_g0w0.txt", scr)
        assert np.abs(qp - ref[:, 1]).max() < 1e-12
        assert np.abs(wt - ref[:, 2]).max() < 1e-12
