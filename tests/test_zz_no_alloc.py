"""ctm_expect_2site_noalloc (for callers that cannot allocate device memory)
against ctm_expect_2site, through the C ABI: the same contraction with its
transients in the library's fixed device array.  Two calls in a row, the
second on a smaller problem; an oversized problem is rejected; the call
changes no device allocation."""
import numpy as np
import pytest

import workloads as wl
from paper_2112_13184_amd import _binding as B

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2112_13184_amd as p
    p.load()
    return p


def test_noalloc_equals_expect_2site(lib):
    H = wl.heisenberg_bond()
    same = True
    for L, D, chi, seed in [(2, 3, 24, 5), (1, 2, 12, 6)]:   # the second call is smaller
        A = wl.random_itps(L, L, D, 2, seed=seed)
        ctx = lib.Ctm(A, L, L, D, chi, rsvd_oversample=8, rsvd_power_iters=1, seed=2)
        ctx.ctm_sweep(4, 0.0)
        for i in range(L * L):
            for dr in (0, 1):
                a = ctx.ctm_expect_2site_noalloc(i, dr, H)   # before the workspace exists
                b = ctx.ctm_expect_2site(i, dr, H)
                assert abs(a - b) <= 1e-13 * max(1.0, abs(b)), (L, D, chi, i, dr, a, b)
                same &= a == b
        ctx.ctm_free()
    print("bitwise equal:", same)


def test_noalloc_allocates_nothing(lib):
    import torch
    H = wl.heisenberg_bond()
    A = wl.random_itps(2, 2, 2, 2, seed=7)
    warm = lib.Ctm(A, 2, 2, 2, 16, rsvd_oversample=8, seed=2)
    warm.ctm_sweep(2, 0.0)
    warm.ctm_expect_2site_noalloc(0, 0, H)
    warm.ctm_expect_2site(0, 0, H)
    ctx = lib.Ctm(A, 2, 2, 2, 16, rsvd_oversample=8, seed=2)
    ctx.ctm_sweep(2, 0.0)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    v = [ctx.ctm_expect_2site_noalloc(i, dr, H) for i in range(4) for dr in (0, 1)]
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert v == [ctx.ctm_expect_2site(i, dr, H) for i in range(4) for dr in (0, 1)]


def test_noalloc_rejects_oversized(lib):
    """D = 4, chi = 64 needs more than the fixed array: CTM_ETOOBIG, and the
    context still works."""
    H = wl.heisenberg_bond()
    A = wl.random_itps(2, 2, 4, 2, seed=1)
    ctx = lib.Ctm(A, 2, 2, 4, 64, rsvd_oversample=32, rsvd_power_iters=1, seed=2)
    ctx.ctm_sweep(1, 0.0)
    with pytest.raises(B.CtmError) as e:
        ctx.ctm_expect_2site_noalloc(0, 0, H)
    assert e.value.status == B.CTM_ETOOBIG
    assert np.isfinite(ctx.ctm_expect_2site(0, 0, H))
