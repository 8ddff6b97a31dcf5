"""What a warm start of the fsGW loop must supply to halve its outer
iterations: a study on the oracle (CPU, FP64), not collected by pytest.

    python tests/warmstart_study.py [--sizes 40 60] [--seeds 8] [--jobs 8] [--out FILE]

For each synthetic system (gwsynth recipe: nocc = M/5, naux = 3.5 M,
nmom_max = 5, the shapes of the warm-start training set) the cold loop
(F0 = diag(eps)) gives the converged Fock matrix F* in the reference basis;
the loop is then restarted from starting matrices built from F*:

  diag_exact      diag(F*_pp): the best a per-orbital diagonal shift can do;
  full_exact      F* itself: the floor of any warm start;
  full_noise_d    F* plus a symmetric Gaussian perturbation of rms d Ha;
  offdiag_rank_r  diag(F*_pp) plus the best rank-r approximation of the
                  off-diagonal part of F* - diag(eps);
  occvir_exact    diag(F*_pp) plus the exact occupied-virtual block of F*.

Each row records the outer iterations, the Fock steps, the largest QP
difference from the cold fixed point over the orbitals with QP weight >= 0.9
in both loops, and whether the loop converged (the oracle loop stops when an
iteration changes F by less than 1e-6 Ha; a start at the fixed point takes
one iteration).  The
summary gives per variant the mean iteration ratio cold / warm over the
systems whose cold and warm loops both converged.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

NOISE = (1e-2, 1e-3, 1e-4)
RANKS = (1, 2, 4, 8)


def shape(M):
    return M // 5, M - M // 5, int(round(3.5 * M))


def starts(eps, F, nocc, seed):
    import numpy as np
    d = np.diag(np.diag(F))
    out = {"diag_exact": d, "full_exact": F}
    rng = np.random.default_rng(seed + 99)
    for s in NOISE:
        G = rng.standard_normal(F.shape) * s
        out[f"full_noise_{s:g}"] = F + (G + G.T) / np.sqrt(2.0)
    off = F - np.diag(np.diag(F))
    w, U = np.linalg.eigh(off)
    order = np.argsort(-np.abs(w))
    for r in RANKS:
        k = order[:r]
        out[f"offdiag_rank_{r}"] = d + (U[:, k] * w[k]) @ U[:, k].T
    ov = d.copy()
    ov[:nocc, nocc:] = F[:nocc, nocc:]
    ov[nocc:, :nocc] = F[nocc:, :nocc]
    out["occvir_exact"] = ov
    return out


def run_system(args):
    M, seed, nmom, max_outer = args
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    import gwsynth
    from oracle import fsgw as of
    o, v, A = shape(M)
    eps, L = gwsynth.system(o, v, A, seed)
    t0 = time.time()
    cold = of.fsgw(eps, L, o, nmom, max_outer=max_outer)
    rows = [dict(M=M, seed=seed, variant="cold", iterations=cold["iterations"], fock_steps=cold["fock_steps"],
                 converged=bool(cold["converged"]), qp_diff=0.0, seconds=time.time() - t0)]
    F = cold["F"]
    off = F - np.diag(np.diag(F))
    rows[0]["offdiag_rms"] = float(np.sqrt((off ** 2).mean()))
    rows[0]["diag_shift_rms"] = float(np.sqrt(((np.diag(F) - eps) ** 2).mean()))
    for name, F0 in starts(eps, F, o, seed).items():
        t0 = time.time()
        w = of.fsgw(eps, L, o, nmom, F0=F0, max_outer=max_outer)
        phys = (w["qp_weight"] >= 0.9) & (cold["qp_weight"] >= 0.9)
        rows.append(dict(M=M, seed=seed, variant=name, iterations=w["iterations"], fock_steps=w["fock_steps"],
                         converged=bool(w["converged"]),
                         qp_diff=float(np.abs(w["qp_orb"][phys] - cold["qp_orb"][phys]).max()),
                         seconds=time.time() - t0))
    return rows


def summarise(rows):
    import numpy as np
    cold = {(r["M"], r["seed"]): r for r in rows if r["variant"] == "cold"}
    out = {}
    for name in sorted({r["variant"] for r in rows} - {"cold"}):
        ratios, its, cits, dq = [], [], [], []
        for r in rows:
            if r["variant"] != name:
                continue
            c = cold[(r["M"], r["seed"])]
            if not (c["converged"] and r["converged"]):
                continue
            ratios.append(c["iterations"] / r["iterations"])
            its.append(r["iterations"])
            cits.append(c["iterations"])
            dq.append(r["qp_diff"])
        out[name] = dict(systems=len(ratios), cold_iterations_mean=float(np.mean(cits)) if cits else None,
                         warm_iterations_mean=float(np.mean(its)) if its else None,
                         iteration_ratio=float(np.mean(cits) / np.mean(its)) if its else None,
                         max_qp_difference=float(max(dq)) if dq else None)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", type=int, nargs="+", default=[40, 60])
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--seed0", type=int, default=1)
    ap.add_argument("--nmom", type=int, default=5)
    ap.add_argument("--max-outer", type=int, default=30)
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    tasks = [(M, s, a.nmom, a.max_outer) for M in a.sizes for s in range(a.seed0, a.seed0 + a.seeds)]
    rows = []
    with ProcessPoolExecutor(a.jobs) as ex:
        for rs in ex.map(run_system, tasks):
            rows.extend(rs)
            c = rs[0]
            print(f"M {c['M']} seed {c['seed']}: cold {c['iterations']} it ({c['seconds']:.0f} s); " +
                  " ".join(f"{r['variant']} {r['iterations']}" for r in rs[1:]), flush=True)
    res = dict(command="python tests/warmstart_study.py " + " ".join(argv if argv is not None else sys.argv[1:]),
               sizes=a.sizes, seeds=a.seeds, nmom_max=a.nmom, summary=summarise(rows), rows=rows)
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(json.dumps(res["summary"], indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
