"""FP64 CPU oracle for moment-conserving GW (Backhouse, Allen, Scott, Booth,
"Self-consistent GW via conservation of spectral moments").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain NumPy/SciPy: every
function follows one passage of the paper in its order and notation, with no
blocking, fusion or reordering beyond what the formula states.

Conventions
-----------
eps : [nmo] orbital energies, occupied first (nocc of them), then virtual.
L   : [naux][nmo][nmo] three-index factor, symmetric in its last two indices;
      the paper's V_{P,pq} (Sec. 2.1, low-rank factorisation of (pq|rs)).
V   : [naux][nocc*nvir], V[P, i*nvir + a] = L[P, i, nocc + a]  (particle-hole block).
D   : [nocc*nvir],       D[i*nvir + a] = eps[nocc + a] - eps[i]  (eq. energy_differences).

Readings of the paper taken here:
  * the W^{(n)} inside the t-sum of eqs. convolution_occ / convolution_vir
    is read as W^{(t)};
  * the self-energy moments of a closed-shell (spin-restricted) reference
    carry a factor 2 from the spin sum over the screening bubble's electron
    line, on top of the paper's expression, while the factor 2 (TDA) and 4
    (RPA) inside the density-response recursions are the paper's own;
  * the RPA zeroth-moment integrals use the mapped Gauss-Legendre grid of
    ``oracle.quadrature``;
  * the block Lanczos recursion conserves moments 0..nmom_max for odd
    nmom_max with (nmom_max + 1) / 2 blocks per sector; it runs on shifted
    and scaled moments and deflates directions whose residual is below the
    rounding level of the moment cancellations (see ``block_lanczos``).
"""
from __future__ import annotations

from math import comb

import numpy as np
from . import quadrature


# --------------------------------------------------------------------------
# Inputs (Sec. 2.1 and eq. energy_differences)
# --------------------------------------------------------------------------

def particle_hole(eps: np.ndarray, L: np.ndarray, nocc: int):
    """V[P, ia] = L[P, i, nocc+a] and D[ia] = eps_a - eps_i (ia = i*nvir + a)."""
    nmo = eps.shape[0]
    nvir = nmo - nocc
    V = np.ascontiguousarray(L[:, :nocc, nocc:]).reshape(L.shape[0], nocc * nvir)
    D = (eps[None, nocc:] - eps[:nocc, None]).reshape(nocc * nvir)
    return V, D


# --------------------------------------------------------------------------
# Density-response moments eta~^{(n)} (Sec. 2.2 RPA, Sec. 2.3 TDA)
# --------------------------------------------------------------------------

def tda_eta(V: np.ndarray, D: np.ndarray, nmom_max: int):
    """TDA moments (Sec. 2.3): eta~^{(0)} = V and
    eta~^{(n)} = eta~^{(n-1)} (D + 2 V^T V), evaluated as
    eta~^{(n-1)} D + 2 (eta~^{(n-1)} V^T) V without forming the ov x ov matrix."""
    eta = [V.copy()]
    for _ in range(nmom_max):
        prev = eta[-1]
        eta.append(prev * D[None, :] + 2.0 * (prev @ V.T) @ V)
    return eta


def rpa_G_quadrature(V: np.ndarray, D: np.ndarray, nquad: int = 48, scale: float | None = None,
                     parts: bool = False):
    """G = G_main + G_offset of Sec. 2.2 (eq. Gmain and the offset integral),
    with Q(z) = 4 V F(z) D V^T, F(z) = (D^2 + z^2)^-1, E(z) = exp(-z D).

    G_main = (1/pi) int_{-inf}^{inf} z^2 Q (( I + Q )^-1 - I) V F dz
           = (2/pi) int_0^inf (...) dz                 (even integrand)
    G_offset = V D + 4 int_0^inf V D E V^T V E dz
    """
    if scale is None:
        scale = quadrature.default_scale(D)
    z, w = quadrature.mapped_gauss_legendre(nquad, scale)
    naux = V.shape[0]
    eye = np.eye(naux)
    G_main = np.zeros_like(V)
    G_off = V * D[None, :]
    for zj, wj in zip(z, w):
        F = 1.0 / (D * D + zj * zj)
        Q = 4.0 * (V * (F * D)[None, :]) @ V.T
        inv = np.linalg.inv(eye + Q)
        G_main += (2.0 / np.pi) * wj * zj * zj * (Q @ (inv - eye)) @ (V * F[None, :])
        E = np.exp(-zj * D)
        G_off += 4.0 * wj * ((V * (D * E)[None, :]) @ V.T) @ (V * E[None, :])
    if parts:
        return G_main, G_off
    return G_main + G_off


def rpa_eta0_from_G(G: np.ndarray, V: np.ndarray, D: np.ndarray):
    """Zeroth RPA moment from G (Sec. 2.2):
    eta~^{(0)} = G D^-1 ( I - 4 V^T ( I + 4 V D^-1 V^T )^-1 V D^-1 ),
    applied right to left without forming an ov x ov matrix."""
    naux = V.shape[0]
    GDi = G / D[None, :]
    VDi = V / D[None, :]
    P = np.eye(naux) + 4.0 * VDi @ V.T
    return GDi - 4.0 * (GDi @ V.T) @ np.linalg.solve(P, VDi)


def rpa_eta(V: np.ndarray, D: np.ndarray, nmom_max: int, nquad: int = 48,
            scale: float | None = None, eta0: np.ndarray | None = None):
    """RPA moments (Sec. 2.2): eta~^{(0)} from the quadrature, eta~^{(1)} = V D,
    eta~^{(n)} = eta~^{(n-2)} (D^2 + 4 V^T V D), evaluated as
    eta~^{(n-2)} D^2 + 4 (eta~^{(n-2)} V^T) (V D)."""
    if eta0 is None:
        eta0 = rpa_eta0_from_G(rpa_G_quadrature(V, D, nquad, scale), V, D)
    VD = V * D[None, :]
    eta = [eta0, VD.copy()]
    for n in range(2, nmom_max + 1):
        prev = eta[n - 2]
        eta.append(prev * (D * D)[None, :] + 4.0 * (prev @ V.T) @ VD)
    return eta[: nmom_max + 1]


def rpa_eta0_exact(V: np.ndarray, D: np.ndarray):
    """Closed form of the zeroth RPA moment for small ov: with
    Mcal = D^1/2 (D + 4 V^T V) D^1/2 = U Omega^2 U^T, the RPA moments are
    eta^{(n)} = D^1/2 U Omega^{n-1} U^T D^1/2, so eta~^{(0)} = V D^1/2 Mcal^-1/2 D^1/2."""
    sD = np.sqrt(D)
    Mcal = sD[:, None] * (np.diag(D) + 4.0 * V.T @ V) * sD[None, :]
    w2, U = np.linalg.eigh(Mcal)
    if w2.min() <= 0.0:
        raise np.linalg.LinAlgError("RPA instability: non-positive Omega^2")
    eta0 = sD[:, None] * ((U / np.sqrt(w2)[None, :]) @ U.T) * sD[None, :]
    return V @ eta0


def w_core(eta, V: np.ndarray):
    """R_t = eta~^{(t)} V^T, the aux-space core of eq. w_moments:
    W^{(t)}_{px,qx} = sum_PQ L_{P,px} R_t[P,Q] L_{Q,qx}."""
    return [e @ V.T for e in eta]


# --------------------------------------------------------------------------
# Self-energy moments (eqs. convolution_occ / convolution_vir, eq. w_moments)
# --------------------------------------------------------------------------

def sigma_moments(eps: np.ndarray, L: np.ndarray, nocc: int, R):
    """Hole and particle self-energy moments Sigma^{(n,<)}, Sigma^{(n,>)} for
    n = 0..len(R)-1, symmetrised.

    Sigma^{(n,<)}_pq = 2 sum_{t<=n} C(n,t) (-1)^t sum_{k occ} eps_k^{n-t} W^{(t)}_{pk,qk}
    Sigma^{(n,>)}_pq = 2 sum_{t<=n} C(n,t)         sum_{c vir} eps_c^{n-t} W^{(t)}_{pc,qc}
    with W^{(t)}_{px,qx} = sum_PQ L[P,p,x] R_t[P,Q] L[Q,q,x].
    Returns (sig_occ[nmom+1][nmo][nmo], sig_vir[...], max asymmetry)."""
    nmom = len(R) - 1
    nmo = eps.shape[0]
    sig_occ = np.zeros((nmom + 1, nmo, nmo))
    sig_vir = np.zeros((nmom + 1, nmo, nmo))
    for t in range(nmom + 1):
        Y = np.tensordot(R[t], L, axes=(1, 0))        # Y[P,q,x] = sum_Q R_t[P,Q] L[Q,q,x]
        for x in range(nmo):
            Lx = np.ascontiguousarray(L[:, :, x])        # [P, p] at fixed x
            Yx = np.ascontiguousarray(Y[:, :, x])        # [P, q] at fixed x
            W = Lx.T @ Yx                                # W^{(t)}_{px,qx}
            for n in range(t, nmom + 1):
                if x < nocc:
                    sig_occ[n] += 2.0 * comb(n, t) * (-1.0) ** t * eps[x] ** (n - t) * W
                else:
                    sig_vir[n] += 2.0 * comb(n, t) * eps[x] ** (n - t) * W
    asym = max(np.abs(s - s.T).max() for s in list(sig_occ) + list(sig_vir))
    sig_occ = 0.5 * (sig_occ + sig_occ.transpose(0, 2, 1))
    sig_vir = 0.5 * (sig_vir + sig_vir.transpose(0, 2, 1))
    return sig_occ, sig_vir, asym


def sigma_moment_rows(eps: np.ndarray, L: np.ndarray, nocc: int, R, rows):
    """Rows p in `rows` of Sigma^{(n,<)} and Sigma^{(n,>)} (unsymmetrised), by
    the same definition as ``sigma_moments`` restricted to fixed p:
    W^{(t)}_{px,qx} = sum_Q (sum_P L[P,p,x] R_t[P,Q]) L[Q,q,x].
    For spot checks of large systems."""
    nmom = len(R) - 1
    nmo = eps.shape[0]
    rows = list(rows)
    so = np.zeros((nmom + 1, len(rows), nmo))
    sv = np.zeros((nmom + 1, len(rows), nmo))
    for t in range(nmom + 1):
        for r, p in enumerate(rows):
            U = np.ascontiguousarray(L[:, p, :]).T @ R[t]          # U[x, Q] = sum_P L[P,p,x] R_t[P,Q]
            for x in range(nmo):
                w = U[x] @ np.ascontiguousarray(L[:, :, x])       # W^{(t)}_{px,qx} over q
                for n in range(t, nmom + 1):
                    if x < nocc:
                        so[n, r] += 2.0 * comb(n, t) * (-1.0) ** t * eps[x] ** (n - t) * w
                    else:
                        sv[n, r] += 2.0 * comb(n, t) * eps[x] ** (n - t) * w
    return so, sv


def gw_moments(eps, L, nocc, nmom_max, screening="tda", nquad=48, scale=None):
    """One-shot pipeline of Alg. 1 up to the self-energy moments:
    V, D -> eta~^{(n)} -> R_t -> Sigma^{(n,<)}, Sigma^{(n,>)}."""
    V, D = particle_hole(eps, L, nocc)
    if screening == "tda":
        eta = tda_eta(V, D, nmom_max)
    elif screening == "rpa":
        eta = rpa_eta(V, D, nmom_max, nquad, scale)
    else:
        raise ValueError(screening)
    R = w_core(eta, V)
    so, sv, _ = sigma_moments(eps, L, nocc, R)
    return so, sv, R


# --------------------------------------------------------------------------
# Block Lanczos from moments (upfolded self-energy of eq. effH)
# --------------------------------------------------------------------------

class LanczosError(RuntimeError):
    pass


EPS = np.finfo(float).eps


def _sym_sqrt_pinv(X: np.ndarray, tol: float, neg: float):
    """Symmetric square root and pseudo-inverse square root of a PSD matrix:
    eigenvalues <= tol are dropped; any below -neg raises LanczosError."""
    X = 0.5 * (X + X.T)
    w, U = np.linalg.eigh(X)
    if w.min() < -neg:
        raise LanczosError("moment matrix is not positive semi-definite")
    keep = w > tol
    Uk = U[:, keep]
    sw = np.sqrt(w[keep])
    return (Uk * sw) @ Uk.T, (Uk / sw) @ Uk.T


def shift_scale(T):
    """Moments of the affinely mapped pole energies e' = (e - c) / s,
    T'^{(n)} = s^-n sum_k C(n,k) (-c)^{n-k} T^{(k)}, with c the weighted mean
    tr T1 / tr T0 and s the weighted spread sqrt(tr T2 / tr T0 - c^2).
    Conserving T'^{(0..N)} is the same as conserving T^{(0..N)}; the map only
    keeps the powers of the energy near unit size."""
    t0 = np.trace(T[0])
    c = np.trace(T[1]) / t0
    s = np.sqrt(max(np.trace(T[2]) / t0 - c * c, 0.0)) if len(T) > 2 else 0.0
    if not s > 0.0:
        s = max(abs(c), 1.0)
    Ts = [sum(comb(n, k) * (-c) ** (n - k) * T[k] for k in range(n + 1)) / s ** n for n in range(len(T))]
    return Ts, c, s


def block_lanczos(T, pinv_tol: float = 1e-12, neg_tol: float = 1e-8, kappa: float = 1.0,
                  moment_eps: float = EPS):
    """Block tridiagonal representation that conserves the moments T[0..N].

    T[n] = v e^n v^T for some pole set (e, v).  With B0 = T[0]^{1/2} and the
    orthonormal block Q1 = B0^+ v, each Lanczos block is kept as a polynomial
    in e applied to Q1,  Q_j = sum_k C[j][k] Q1 e^k,  so every inner product
    is a combination of S^{(n)} = B0^+ T[n] B0^+ = Q1 e^n Q1^T:

      A_j   = sum_{k,l} C_j,k S^{(k+l+1)} C_j,l^T
      Rhat  = sum_k (C_j,k-1 - A_j C_j,k - B_{j-1} C_{j-1},k) Q1 e^k
      B_j^2 = sum_{k,l} Rhat_k S^{(k+l)} Rhat_l^T,  B_j = (B_j^2)^{1/2}
      C_{j+1},k = B_j^+ Rhat_k

    For odd N = 2m+1 this runs to j = m+1 blocks and conserves moments 0..N.

    Deflation: B_j^2 is a small difference of large terms once the
    coefficients grow, so its eigenvalues are only known to about
    noise_j = kappa * eps_m * (sum_k |Rhat_k|_F)^2 * max_{n<=2j} |S^{(n)}|_F,
    with eps_m the relative accuracy of the input moments (machine epsilon
    for FP64 moments).
    Eigenvalues below max(pinv_tol |S^{(2)}|_F, noise_j) are dropped (those
    directions have converged), and eigenvalues below
    -max(neg_tol |S^{(2)}|_F, 10 noise_j) mean the input is not a moment
    sequence (LanczosError).  T[0] itself is cut at pinv_tol times its largest
    eigenvalue.  Returns (A_blocks, B_blocks, B0)."""
    N = len(T) - 1
    if N < 1 or N % 2 == 0:
        raise ValueError("nmom_max must be odd")
    m = (N - 1) // 2
    nmo = T[0].shape[0]
    w0 = np.linalg.eigvalsh(0.5 * (T[0] + T[0].T))
    wmax = max(float(np.abs(w0).max()), np.finfo(float).tiny)
    B0, B0i = _sym_sqrt_pinv(T[0], pinv_tol * wmax, neg_tol * wmax)
    S = [B0i @ Tn @ B0i for Tn in T]
    S = [0.5 * (s + s.T) for s in S]
    snorm = [float(np.linalg.norm(s)) for s in S]
    ref = snorm[2] if N >= 2 else snorm[0]
    eye = np.eye(nmo)

    A_blocks, B_blocks = [], []
    C_prev, C_cur, B_prev = None, [eye], None
    for j in range(1, m + 2):
        Aj = np.zeros((nmo, nmo))
        for k, Ck in enumerate(C_cur):
            for l, Cl in enumerate(C_cur):
                Aj += Ck @ S[k + l + 1] @ Cl.T
        Aj = 0.5 * (Aj + Aj.T)
        A_blocks.append(Aj)
        if j == m + 1:
            break
        Rh = []
        for k in range(j + 1):
            r = np.zeros((nmo, nmo))
            if k >= 1:
                r += C_cur[k - 1]
            if k < j:
                r -= Aj @ C_cur[k]
            if C_prev is not None and k < j - 1:
                r -= B_prev @ C_prev[k]
            Rh.append(r)
        B2 = np.zeros((nmo, nmo))
        for k, Rk in enumerate(Rh):
            for l, Rl in enumerate(Rh):
                B2 += Rk @ S[k + l] @ Rl.T
        rn = sum(float(np.linalg.norm(r)) for r in Rh)
        noise = kappa * moment_eps * rn * rn * max(snorm[: 2 * j + 1])
        Bj, Bj_inv = _sym_sqrt_pinv(B2, max(pinv_tol * ref, noise), max(neg_tol * ref, 10.0 * noise))
        B_blocks.append(Bj)
        C_prev, C_cur, B_prev = C_cur, [Bj_inv @ r for r in Rh], Bj
    return A_blocks, B_blocks, B0


def block_tridiagonal(A_blocks, B_blocks):
    nb = len(A_blocks)
    n = A_blocks[0].shape[0]
    H = np.zeros((nb * n, nb * n))
    for j, Aj in enumerate(A_blocks):
        H[j * n:(j + 1) * n, j * n:(j + 1) * n] = Aj
    for j, Bj in enumerate(B_blocks):
        H[j * n:(j + 1) * n, (j + 1) * n:(j + 2) * n] = Bj
        H[(j + 1) * n:(j + 2) * n, j * n:(j + 1) * n] = Bj.T
    return H


def poles_from_moments(T, pinv_tol: float = 1e-12, neg_tol: float = 1e-8,
                       weight_tol: float = 1e-14, moment_eps: float = EPS):
    """Auxiliary poles (e[npole], v[nmo][npole]) whose moments v e^n v^T equal
    T[n] for n <= N: shift and scale the moments (``shift_scale``), diagonalise
    the block-tridiagonal Lanczos matrix H_s = U diag(e') U^T, map back
    e = c + s e' and set v = B0 U[first block rows].  Poles whose
    coupling norm is below weight_tol times the largest are dropped (they
    are decoupled directions left by pseudo-inverses)."""
    Ts, c, s = shift_scale([np.asarray(t) for t in T])
    A_blocks, B_blocks, B0 = block_lanczos(Ts, pinv_tol, neg_tol, moment_eps=moment_eps)
    Hs = block_tridiagonal(A_blocks, B_blocks)
    e, U = np.linalg.eigh(Hs)
    e = c + s * e
    nmo = T[0].shape[0]
    v = B0 @ U[:nmo, :]
    wt = (v * v).sum(axis=0)
    keep = wt > weight_tol * max(float(wt.max()), np.finfo(float).tiny)
    return e[keep], v[:, keep]


# --------------------------------------------------------------------------
# Upfolded Hamiltonian, Green's function poles and QP assignment
# (eqs. effH, ret_GF, quasiparticle_energy_update)
# --------------------------------------------------------------------------

def upfolded_hamiltonian(fock: np.ndarray, e_occ, v_occ, e_vir, v_vir):
    """H~ = [[f + Sigma_inf, W~], [W~^T, d~]] with d~ = diag(hole poles, particle
    poles) and W~ = [v_occ, v_vir]; Sigma_inf = 0 for a Hartree-Fock-like
    reference (eq. StaticSE)."""
    nmo = fock.shape[0]
    e_aux = np.concatenate([e_occ, e_vir])
    W = np.concatenate([v_occ, v_vir], axis=1)
    dim = nmo + e_aux.shape[0]
    H = np.zeros((dim, dim))
    H[:nmo, :nmo] = fock
    H[:nmo, nmo:] = W
    H[nmo:, :nmo] = W.T
    H[nmo:, nmo:] = np.diag(e_aux)
    return H


def qp_assign(E: np.ndarray, chi_phys: np.ndarray):
    """eps_p^QP = E_alpha with alpha = argmax_beta |chi_{p beta}|^2 (lowest alpha
    on ties); also returns the QP weight |chi_{p alpha}|^2 and alpha."""
    w = chi_phys * chi_phys
    alpha = np.argmax(w, axis=1)
    rows = np.arange(chi_phys.shape[0])
    return E[alpha], w[rows, alpha], alpha


def g0w0(eps, L, nocc, nmom_max, screening="tda", nquad=48, scale=None,
         pinv_tol=1e-12, neg_tol=1e-8):
    """Alg. 1 end to end: moments -> poles per sector -> H~ -> eigenpairs -> QP."""
    so, sv, R = gw_moments(eps, L, nocc, nmom_max, screening, nquad, scale)
    eo, vo = poles_from_moments(list(so), pinv_tol, neg_tol)
    ev, vv = poles_from_moments(list(sv), pinv_tol, neg_tol)
    H = upfolded_hamiltonian(np.diag(eps), eo, vo, ev, vv)
    E, U = np.linalg.eigh(H)
    nmo = eps.shape[0]
    qp, wt, alpha = qp_assign(E, U[:nmo, :])
    return dict(sigma_occ=so, sigma_vir=sv, R=R, e_occ=eo, v_occ=vo, e_vir=ev, v_vir=vv,
                E=E, chi=U[:nmo, :], qp=qp, qp_weight=wt, qp_alpha=alpha)
