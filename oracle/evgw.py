"""Eigenvalue self-consistent moment GW (paper App. A, Alg. A1: evGW, evGW0,
and G0W0 as its fixed-point-free case), oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The algorithm box keeps two sets of orbital energies: eps_G enters the
Green's function (the eps-power factors of the convolution,
eqs. convolution_occ / convolution_vir) and eps_W the screening (the energy
differences D of eq. energy_differences in the density-response recursion).
Both start at the reference eps; the static part stays f = diag(eps),
Sigma_inf = 0 (eq. StaticSE).  Each iteration builds the moments, the
auxiliary poles and the upfolded Hamiltonian, assigns QP energies by
eq. quasiparticle_energy_update, and then replaces eps_G (unless g0) and
eps_W (unless w0) by them.

Readings taken here (the box gives the loop, not its numerics):
  * convergence: the largest difference between the QP energies of an
    iteration and the energies that went into it (for the plain loop: the
    previous iteration's QP energies), over the orbitals whose QP weight is
    at least 0.9 in both iterations (all orbitals if none is), is below
    `tol` (1e-6 Ha);
  * the updated energies are the Pulay (DIIS, 12 vectors) extrapolation of
    the QP energies with those differences as error vectors (the paper's
    self-consistent runs keep a DIIS space of 12); diis_space = 0 gives the
    plain loop; the QP energy of an orbital embedded in
    a satellite band has no stable assignment and is left out of the test;
    with g0 and w0 both set nothing is updated and the loop is one G0W0
    evaluation;
  * the QP energy of orbital p is the H~ eigenvalue of largest physical
    weight |chi_p alpha|^2 (ties to the lowest alpha), as in G0W0;
  * the block Lanczos inside the loop deflates at a moment accuracy of
    1e-12 (relative), not the unit roundoff: the recursion and the
    convolution leave the FP64 moments a few digits short of it, and
    directions resolved from that rounding noise give satellite poles whose
    QP assignment moves by ~1e-5 Ha from one iteration to the next.
"""
from __future__ import annotations

import numpy as np

from . import fsgw, gw


def ev_step(eps_ref, eps_g, eps_w, L, nocc, nmom_max, screening="tda", nquad=48, scale=None, moment_eps=gw.EPS):
    """One pass of the loop body of Alg. A1: moments with eps_W, convolution
    with eps_G, poles, H~ with f = diag(eps_ref), QP assignment."""
    V, D = gw.particle_hole(eps_w, L, nocc)
    if screening == "tda":
        eta = gw.tda_eta(V, D, nmom_max)
    else:
        eta = gw.rpa_eta(V, D, nmom_max, nquad, scale)
    R = gw.w_core(eta, V)
    so, sv, _ = gw.sigma_moments(eps_g, L, nocc, R)
    eo, vo = gw.poles_from_moments(list(so), moment_eps=moment_eps)
    ev, vv = gw.poles_from_moments(list(sv), moment_eps=moment_eps)
    H = gw.upfolded_hamiltonian(np.diag(eps_ref), eo, vo, ev, vv)
    E, U = np.linalg.eigh(H)
    qp, wt, _ = gw.qp_assign(E, U[: eps_ref.shape[0]])
    return qp, wt


def evgw(eps, L, nocc, nmom_max, screening="tda", g0=False, w0=False, tol=1e-6, max_iter=30,
         nquad=48, scale=None, step=None, diis_space=12, moment_eps=1e-12):
    """Alg. A1.  Returns dict(qp, qp_weight, iterations, converged, history).
    `step` replaces the loop body (same signature as ``ev_step``), e.g. by a
    brute-force one.  With diis_space > 0 the updated energies are the Pulay
    extrapolation (the paper's self-consistent runs keep a DIIS space of 12)
    over the pairs (QP energies, QP energies - the energies they came from);
    diis_space = 0 is the plain loop."""
    step = step or (lambda er, eg, ew: ev_step(er, eg, ew, L, nocc, nmom_max, screening, nquad, scale, moment_eps))
    eps = np.asarray(eps, dtype=np.float64)
    eps_g = eps.copy()
    eps_w = eps.copy()
    prev_wt = np.ones_like(eps)
    history = []
    qp = wt = None
    x = eps.copy()
    diis = fsgw.DIIS(diis_space) if diis_space > 0 else None
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        qp, wt = step(eps, eps_g, eps_w)
        qpl = (wt >= 0.9) & (prev_wt >= 0.9)
        if not qpl.any():
            qpl[:] = True
        change = float(np.abs(qp - x)[qpl].max())
        history.append(change)
        if g0 and w0:
            converged = True
            break
        nxt = qp.copy() if diis is None else diis.update(qp, qp - x)
        if not g0:
            eps_g = nxt.copy()
        if not w0:
            eps_w = nxt.copy()
        x = nxt
        if change < tol:
            converged = True
            break
        prev_wt = wt.copy()
    return dict(qp=qp, qp_weight=wt, iterations=it, converged=converged, history=history)
