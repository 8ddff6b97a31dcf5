"""The allocation-free entry point (gw_sigma_moments_noalloc) through the C
ABI: the same self-energy moments as gw_sigma_moments (TDA, FP64) on two
calls in a row, the second with a smaller system, to the FP64 bar (1e-10
relative to the largest element of each moment) and against the oracle;
no device memory is allocated by a call once its kernels are loaded; a
system whose buffers exceed the static scratch is refused before anything
runs."""
import gc

import numpy as np
import pytest

import gwsynth
from oracle import gw as ogw

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def handle():
    import torch
    from paper_2504_17439_amd import gwmom
    assert torch.cuda.is_available()
    h = gwmom.Handle(0)
    yield h
    h.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def test_noalloc_matches_sigma_moments_twice(handle):
    import torch
    # the larger system first, then a smaller one: the second call must not
    # see anything the first left in the shared scratch
    for o, v, A, N, seed in ((12, 30, 150, 11, 5), (5, 19, 80, 3, 0)):
        print(f"\n[case] noalloc o={o} v={v} A={A} N={N} seed={seed}", flush=True)
        eps, L = gwsynth.system(o, v, A, seed)
        e, l = dev(eps), dev(L)
        so, sv = handle.sigma_moments_noalloc(e, l, o, N)
        ro, rv = handle.sigma_moments(e, l, o, N, "tda")
        torch.cuda.synchronize()
        so, sv, ro, rv = (t.cpu().numpy() for t in (so, sv, ro, rv))
        ref_o, ref_v, _ = ogw.gw_moments(eps, L, o, N, "tda")
        for n in range(N + 1):
            assert rel(so[n], ro[n]) < TOL, ("occ vs entry point", n)
            assert rel(sv[n], rv[n]) < TOL, ("vir vs entry point", n)
            assert rel(so[n], ref_o[n]) < TOL, ("occ vs oracle", n)
            assert rel(sv[n], ref_v[n]) < TOL, ("vir vs oracle", n)
            assert np.array_equal(so[n], so[n].T) and np.array_equal(sv[n], sv[n].T)


def test_noalloc_allocates_nothing(handle):
    import torch
    from paper_2504_17439_amd import gwmom
    o, v, A, N = 7, 37, 131, 5
    print(f"\n[case] noalloc memory o={o} v={v} A={A} N={N}", flush=True)
    eps, L = gwsynth.system(o, v, A, 3)
    e, l = dev(eps), dev(L)
    out = (torch.empty(N + 1, o + v, o + v, dtype=torch.float64, device="cuda:0"),
           torch.empty(N + 1, o + v, o + v, dtype=torch.float64, device="cuda:0"))
    h2 = gwmom.Handle(0)          # a fresh handle: no workspace of its own yet
    gc.collect()                  # handles of earlier tests release their memory now, not in the window
    gc.disable()
    try:
        h2.sigma_moments_noalloc(e, l, o, N, out=out)   # loads the kernels
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info(0)
        for _ in range(3):
            h2.sigma_moments_noalloc(e, l, o, N, out=out)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info(0)
        assert free1 >= free0, f"device free memory fell by {free0 - free1} bytes"
        ref_o, ref_v, _ = ogw.gw_moments(eps, L, o, N, "tda")
        for n in range(N + 1):
            assert rel(out[0][n].cpu().numpy(), ref_o[n]) < TOL
            assert rel(out[1][n].cpu().numpy(), ref_v[n]) < TOL
    finally:
        gc.enable()
        h2.close()


def test_noalloc_refuses_oversized_system(handle):
    import torch
    from paper_2504_17439_amd import gwmom
    # 2 * naux * ov doubles alone exceed 64 MiB here; nothing may run
    o, v, A, N = 40, 160, 600, 7
    print(f"\n[case] noalloc oversized o={o} v={v} A={A} N={N}", flush=True)
    eps = torch.linspace(-1.0, 1.0, o + v, dtype=torch.float64, device="cuda:0")
    L = torch.zeros(A, o + v, o + v, dtype=torch.float64, device="cuda:0")
    so = torch.full((N + 1, o + v, o + v), 7.0, dtype=torch.float64, device="cuda:0")
    sv = torch.full((N + 1, o + v, o + v), 7.0, dtype=torch.float64, device="cuda:0")
    with pytest.raises(gwmom.GWError) as ei:
        handle.sigma_moments_noalloc(eps, L, o, N, out=(so, sv))
    assert ei.value.status == gwmom.GW_EINVAL
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((so == 7.0).all()) and bool((sv == 7.0).all())
