"""Batched self-energy moments (gw_batch_*): grouped persistent launches over
many molecules, captured in a hipGraph, against single-molecule calls and
the oracle.

The grouped kernels run the same per-tile arithmetic as the single-molecule
path; only the contraction splits (and so the FP64 summation order of the
split partials) differ, so batch and single results agree to ~1e-14
relative (1e-12 asserted).  Graph replays are deterministic: bit-identical.
"""
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


def shape(M):
    return M // 5, M - M // 5, int(round(3.5 * M))


def systems(sizes, seed0=0):
    out = []
    for k, M in enumerate(sizes):
        o, v, A = shape(M)
        eps, L = gwsynth.system(o, v, A, seed0 + k)
        out.append((o, eps, L))
    return out


SIZES = [20, 25, 60, 30, 45, 40]


@pytest.mark.parametrize("prec,scr,bopts", [
    ("mixed", "tda", None),
    ("mixed", "tda", {"job_bytes": 1 << 20, "wave_bytes": 3 << 20}),
    ("mixed", "tda", {"small_tile_nmo": 45}),      # 64 x 64 contraction tiles for nmo <= 45
    ("fp64", "tda", None),
    ("mixed", "rpa", None),
])
def test_batch_matches_single_calls(handle, prec, scr, bopts):
    N = 7 if scr == "tda" else 5
    print(f"\n[case] batch {prec} {scr} {bopts}", flush=True)
    sy = systems(SIZES)
    tensors = [(dev(e), dev(L), o) for o, e, L in sy]
    b = handle.batch([(e, l, o) for e, l, o in tensors], N, screening=scr, precision=prec, bopts=bopts)
    info = b.info()
    print(info, flush=True)
    if bopts and "wave_bytes" in bopts:
        assert info["waves"] > 1 and info["jobs"] == len(SIZES)
    if bopts and "small_tile_nmo" in bopts:
        assert info["small_tile_nmo"] == bopts["small_tile_nmo"]
    assert info["graph"] == (scr == "tda")
    for (e, l, o), (so, sv) in zip(tensors, b.sigma):
        ro, rv = handle.sigma_moments(e, l, o, N, screening=scr, precision=prec)
        assert rel(host(so), host(ro)) < 1e-12 and rel(host(sv), host(rv)) < 1e-12
    b.close()


def test_batch_matches_oracle(handle):
    sy = systems([25, 40])
    tensors = [(dev(e), dev(L), o) for o, e, L in sy]
    b = handle.batch([(e, l, o) for e, l, o in tensors], 7)
    for (o, eps, L), (so, sv) in zip(sy, b.sigma):
        ref_o, ref_v, _ = ogw.gw_moments(eps, L, o, 7, "tda")
        so, sv = host(so), host(sv)
        for n in range(8):
            assert rel(so[n], ref_o[n]) < MIXED_TOL and rel(sv[n], ref_v[n]) < MIXED_TOL


def test_graph_replays_are_identical_and_track_inputs(handle):
    import torch
    sy = systems([30, 20, 45], seed0=5)
    tensors = [(dev(e), dev(L), o) for o, e, L in sy]
    b = handle.batch([(e, l, o) for e, l, o in tensors], 7)
    assert b.info()["graph"]
    first = [(host(so).copy(), host(sv).copy()) for so, sv in b.sigma]
    for rep in range(3):
        scratch = torch.randn(1 << 20, device="cuda:0").sum()   # eager work between replays
        for so, sv in b.sigma:
            so.zero_()
            sv.zero_()
        b.run()
        torch.cuda.synchronize()
        for (so, sv), (fo, fv) in zip(b.sigma, first):
            assert np.array_equal(host(so), fo) and np.array_equal(host(sv), fv)
        del scratch
    # new input values through the same pointers
    for e, l, o in tensors:
        l.mul_(0.7)
    b.run()
    for (e, l, o), (so, sv) in zip(tensors, b.sigma):
        ro, rv = handle.sigma_moments(e, l, o, 7, precision="mixed")
        assert rel(host(so), host(ro)) < 1e-12 and rel(host(sv), host(rv)) < 1e-12
    b.close()


def test_autotuned_plan_gives_the_same_moments(handle):
    sy = systems([40, 25, 30], seed0=11)
    tensors = [(dev(e), dev(L), o) for o, e, L in sy]
    b = handle.batch([(e, l, o) for e, l, o in tensors], 7, bopts={"autotune": 1})
    info = b.info()
    # the autotuner's candidates: split targets, and the largest nmo on 64-row
    # contraction tiles (1 << 20: every molecule)
    assert info["split_target"] in (256, 512, 1024, 2048)
    assert info["small_tile_nmo"] in (0, 100, 150, 200, 1 << 20)
    for (e, l, o), (so, sv) in zip(tensors, b.sigma):
        ro, rv = handle.sigma_moments(e, l, o, 7, precision="mixed")
        assert rel(host(so), host(ro)) < 1e-12 and rel(host(sv), host(rv)) < 1e-12
    b.close()


def test_graph_survives_later_workspace_growth(handle):
    """A one-molecule batch with one branch, then a larger call on the same
    handle (its workspace slots grow and are reallocated), then a replay: the
    graph references only batch-owned memory, so the replay still matches."""
    o, eps, L = systems([25], seed0=21)[0]
    e, l = dev(eps), dev(L)
    b = handle.batch([(e, l, o)], 7, bopts={"branches": 1})
    assert b.info()["graph"]
    ob, eb, Lb = systems([90], seed0=22)[0]
    handle.sigma_moments(dev(eb), dev(Lb), ob, 7, precision="mixed")       # grows the handle's workspace
    handle.sigma_moments(dev(eb), dev(Lb), ob, 7, precision="fp64")
    so, sv = b.sigma[0]
    so.zero_()
    sv.zero_()
    b.run()
    ro, rv = handle.sigma_moments(e, l, o, 7, precision="mixed")
    assert rel(host(so), host(ro)) < 1e-12 and rel(host(sv), host(rv)) < 1e-12
    b.close()


def test_batch_rejects_bad_arguments(handle):
    from paper_2504_17439_amd import gwmom
    o, eps, L = systems([20])[0]
    e, l = dev(eps), dev(L)
    with pytest.raises(gwmom.GWError, match="GW_EINVAL"):
        handle.batch([(e, l, o)], 6)
    with pytest.raises(gwmom.GWError, match="GW_EINVAL"):
        handle.batch([(e, l, o)], 13)
    bad = eps.copy()
    bad[o - 1] = bad[o] + 1.0   # occupied above virtual
    with pytest.raises(gwmom.GWError, match="GW_EINVAL"):
        handle.batch([(e, l, o), (dev(bad), l, o)], 7)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_c4_size_batch(handle, prec):
    """The largest molecule shapes of the 64-molecule batch (nmo 355-400,
    nocc = nmo/5, naux = 3.5 nmo, nmom_max 7, TDA): the batch against single
    calls (1e-12), and the nmo = 400 molecule against stored oracle rows
    (tests/golden/c4_tda_sigma.npz, written by make_golden.py from the oracle
    alone): FP64 1e-10, mixed 1e-8 relative to the largest element of each
    moment."""
    import os
    import torch
    f = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_tda_sigma.npz"))
    o0, v0, A0, N, seed = (int(f[k]) for k in ("nocc", "nvir", "naux", "nmom_max", "seed"))
    print(f"\n[case] c4-size batch {prec}: nmo 400 (seed {seed}), 380, 355", flush=True)
    sy = [(o0, *gwsynth.system(o0, v0, A0, seed))]
    for k, M in enumerate((380, 355)):
        o, v, A = shape(M)
        sy.append((o, *gwsynth.system(o, v, A, seed + 1 + k)))
    tensors = [(dev(e), dev(L), o) for o, e, L in sy]
    b = handle.batch([(e, l, o) for e, l, o in tensors], N, precision=prec)
    print(b.info(), flush=True)
    for (e, l, o), (so, sv) in zip(tensors, b.sigma):
        ro, rv = handle.sigma_moments(e, l, o, N, precision=prec)
        assert rel(host(so), host(ro)) < 1e-12 and rel(host(sv), host(rv)) < 1e-12
        del ro, rv
    tol = 1e-10 if prec == "fp64" else MIXED_TOL
    rows = list(f["sigma_rows"])
    so, sv = (host(t) for t in b.sigma[0])
    worst = 0.0
    for n in range(N + 1):
        eo = np.abs(so[n][rows] - f["so_rows"][n]).max() / f["so_absmax"][n]
        ev = np.abs(sv[n][rows] - f["sv_rows"][n]).max() / f["sv_absmax"][n]
        worst = max(worst, eo, ev)
        assert eo < tol and ev < tol, (prec, n, eo, ev)
    print(f"c4-size {prec}: batch vs oracle rows {worst:.2e}", flush=True)
    b.close()
    del tensors
    torch.cuda.empty_cache()
