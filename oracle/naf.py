"""Natural auxiliary functions (paper Sec. 2.1, eq. NAF), oracle side.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

M_PQ = sum_{vw} V_{P,vw} V_{Q,vw} is diagonalised; its eigenvectors with
eigenvalue above eps_naf span the NAF basis, and the interaction tensor is
projected into it: L_naf[k] = sum_P U[P,k] L[P].  By default the pair (v,w)
runs over the particle-hole block (i, a), each pair once (the density-
response recursions use exactly V[P, ia]); with full_space it runs over all
nmo^2 pairs (the paper's choice for self-consistent schemes).
Reading taken here: eps_naf is an absolute threshold on the eigenvalues of M.
"""
from __future__ import annotations

import numpy as np


def naf_matrix(L: np.ndarray, nocc: int, full_space: bool = False) -> np.ndarray:
    """M_PQ of eq. NAF."""
    naux = L.shape[0]
    if full_space:
        X = L.reshape(naux, -1)
    else:
        X = np.ascontiguousarray(L[:, :nocc, nocc:]).reshape(naux, -1)
    return X @ X.T


def naf(L: np.ndarray, nocc: int, eps_naf: float = 1e-5, full_space: bool = False):
    """Returns (L_naf [nnaf][nmo][nmo], kept eigenvalues, all eigenvalues)."""
    Mpq = naf_matrix(L, nocc, full_space)
    w, U = np.linalg.eigh(Mpq)
    keep = w > eps_naf
    Uk = U[:, keep]
    L_naf = np.tensordot(Uk.T, L, axes=(1, 0))
    return L_naf, w[keep], w
