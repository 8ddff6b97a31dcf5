"""Seeded synthetic inputs for density-fitted GW: orbital energies and a
three-index Coulomb factor in the MO basis.

This module is shared by the CPU oracle and the GPU path, so it holds none
of the method's arithmetic: it only draws random numbers and shapes them.

Recipe (one system):
  * ``numpy.random.default_rng(seed)``;
  * occupied energies ~ U[occ_lo, occ_hi] Ha, sorted ascending (nocc draws);
  * virtual energies  ~ U[vir_lo, vir_hi] Ha, sorted ascending (nvir draws);
  * G ~ N(0, 1) of shape [naux][nmo][nmo], drawn after the energies;
  * L[P,p,q] = (G[P,p,q] + G[P,q,p]) / sqrt(2) * amp / sqrt(naux)
               * exp(-|p - q| / decay)
    which is symmetric in (p, q), with amp = 0.3 and decay = 8 by default.

The factor L plays the role of the density-fitted interaction V_{P,pq} of
the paper (Sec. 2.1, the low-rank factorisation (pq|rs) = sum_P V_P,pq V_P,rs).
"""
from __future__ import annotations

import numpy as np

OCC_RANGE = (-1.5, -0.3)
VIR_RANGE = (0.1, 3.0)
AMP = 0.3
DECAY = 8.0


def system(nocc: int, nvir: int, naux: int, seed: int = 0,
           amp: float = AMP, decay: float = DECAY,
           occ_range=OCC_RANGE, vir_range=VIR_RANGE,
           dtype=np.float64):
    """Return (eps[nmo], L[naux][nmo][nmo]) as C-contiguous float64 arrays."""
    if nocc < 1 or nvir < 1 or naux < 1:
        raise ValueError("nocc, nvir and naux must be >= 1")
    nmo = nocc + nvir
    rng = np.random.default_rng(seed)
    eo = np.sort(rng.uniform(occ_range[0], occ_range[1], nocc))
    ev = np.sort(rng.uniform(vir_range[0], vir_range[1], nvir))
    eps = np.concatenate([eo, ev]).astype(np.float64)
    idx = np.arange(nmo)
    envelope = (amp / np.sqrt(naux)) * np.exp(-np.abs(idx[:, None] - idx[None, :]) / decay)
    envelope = envelope / np.sqrt(2.0)
    L = np.empty((naux, nmo, nmo), dtype=dtype)
    # Draw aux slabs one at a time so the peak host memory stays near one L.
    for P in range(naux):
        g = rng.standard_normal((nmo, nmo))
        L[P] = (g + g.T) * envelope
    return eps, L


def batch_shapes(nsys: int = 64, seed: int = 0, nmo_lo: int = 60, nmo_hi: int = 400,
                 step: int = 5, occ_frac: float = 0.2, aux_ratio: float = 3.5):
    """Shapes of a batch of molecules: nmo uniform over multiples of `step`
    in [nmo_lo, nmo_hi], nocc = nmo * occ_frac, naux = round(aux_ratio * nmo)."""
    rng = np.random.default_rng(seed)
    choices = np.arange(nmo_lo, nmo_hi + 1, step)
    nmos = rng.choice(choices, size=nsys)
    out = []
    for nmo in nmos:
        nmo = int(nmo)
        nocc = int(round(nmo * occ_frac))
        out.append((nocc, nmo - nocc, int(round(aux_ratio * nmo))))
    return out


def system_device(nocc: int, nvir: int, naux: int, seed: int = 0, device: str = "cuda:0",
                  amp: float = AMP, decay: float = DECAY,
                  occ_range=OCC_RANGE, vir_range=VIR_RANGE):
    """The same recipe drawn on the device with torch's generator (for inputs
    too large to draw on the host quickly).  The values differ from
    ``system`` for the same seed; the distributions and structure do not."""
    import torch
    if nocc < 1 or nvir < 1 or naux < 1:
        raise ValueError("nocc, nvir and naux must be >= 1")
    nmo = nocc + nvir
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    eo = torch.sort(torch.rand(nocc, generator=g, device=device, dtype=f64))[0]
    ev = torch.sort(torch.rand(nvir, generator=g, device=device, dtype=f64))[0]
    eps = torch.cat([occ_range[0] + (occ_range[1] - occ_range[0]) * eo,
                     vir_range[0] + (vir_range[1] - vir_range[0]) * ev]).contiguous()
    idx = torch.arange(nmo, device=device, dtype=f64)
    envelope = (amp / np.sqrt(naux)) * torch.exp(-(idx[:, None] - idx[None, :]).abs() / decay) / np.sqrt(2.0)
    L = torch.empty((naux, nmo, nmo), device=device, dtype=f64)
    for P0 in range(0, naux, 64):
        P1 = min(naux, P0 + 64)
        G = torch.randn((P1 - P0, nmo, nmo), generator=g, device=device, dtype=f64)
        L[P0:P1] = (G + G.transpose(1, 2)) * envelope
    return eps, L


def eigensystem(nmo: int, dim: int, seed: int = 0, orthonormal: bool = True,
                e_lo: float = -3.0, e_hi: float = 4.0):
    """Synthetic eigenpairs of an upfolded Hamiltonian: E [dim] ascending,
    uniform in [e_lo, e_hi] Ha, and chi [nmo][dim], the first nmo rows of a
    random orthogonal matrix (or, for large dim, Gaussian rows scaled to unit
    norm, which keeps the shapes without the O(dim^3) factorisation)."""
    rng = np.random.default_rng(seed)
    E = np.sort(rng.uniform(e_lo, e_hi, dim))
    if orthonormal:
        Q = np.linalg.qr(rng.standard_normal((dim, dim)))[0]
        chi = np.ascontiguousarray(Q[:nmo])
    else:
        chi = rng.standard_normal((nmo, dim))
        chi /= np.linalg.norm(chi, axis=1, keepdims=True)
    return E, chi
