"""soft_match_argmax_noalloc, the argmax entry point that allocates nothing
(its partial results live in the library's static device array), called
through the C-ABI.  Its indices must equal those of soft_match_argmax (the
same kernels on a head's own partial buffer) bit for bit, on two calls in a
row with the second on a smaller input, so nothing left in the shared array
by the first call leaks into the second.  Exact ties go to the first index
and all-NaN grids give -1, as for soft_match_argmax; the indices also equal
the oracle's argmax of the same values.  Inputs are seeded synthetic grids.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_1808_00896_amd import soft

pytestmark = pytest.mark.gpu

CDT = {"fp64": torch.complex128, "fp32": torch.complex64}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def host_grids(n, B, seed, ties=False):
    """n seeded normal complex grids of (2B)^3 elements; with ties, the
    maximum of each grid is copied to an earlier position as well."""
    rng = np.random.default_rng(seed)
    N3 = (2 * B) ** 3
    g = rng.standard_normal((n, N3)) + 1j * rng.standard_normal((n, N3))
    if ties:
        for f in range(n):
            i = int(np.argmax(g[f].real))
            g[f, i // 3] = g[f, i]
    return g


def noalloc(dev, B, n, prec, g):
    idx = torch.full((n,), -7, dtype=torch.int64, device=dev)
    code = soft.PRECISIONS[prec]
    rc = soft.lib().soft_match_argmax_noalloc(B, n, code, ctypes.c_void_p(g.data_ptr()),
                                              ctypes.c_void_p(idx.data_ptr()),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == soft.SOFT_OK, soft.status_string(rc)
    return idx


def with_head(B, n, prec, g):
    with soft.MatchPlan(B, n, precision=prec) as m:
        idx = m.argmax(g.reshape(m.plan.grid_shape()))
        torch.cuda.synchronize()
        return idx.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("first,second", [((32, 5), (8, 3)), ((64, 2), (16, 1)), ((4, 3000), (2, 700))])
def test_noalloc_argmax_matches_head_argmax(dev, prec, first, second):
    for call, (B, n) in enumerate((first, second)):
        print(f"noalloc argmax call {call}: B={B} n={n} {prec}", flush=True)
        gh = host_grids(n, B, seed=1000 * call + B + n, ties=(call == 1))
        g = torch.from_numpy(gh).to(dev).to(CDT[prec]).contiguous()
        got = noalloc(dev, B, n, prec, g)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        want = with_head(B, n, prec, g)
        assert np.array_equal(got, want), (call, got[:8], want[:8])
        # the oracle's argmax of the same values (complex64 widens exactly)
        gv = g.cpu().numpy().astype(np.complex128)
        for f in range(0, n, max(1, n // 7)):
            assert got[f] == int(np.argmax(gv[f].real)), (call, f)


def test_noalloc_argmax_all_nan_and_all_equal(dev):
    B, n = 8, 4
    g = torch.zeros(n, (2 * B) ** 3, dtype=torch.complex128, device=dev)
    g[1:3] = complex(float("nan"), 0.0)
    got = noalloc(dev, B, n, "fp64", g).cpu().numpy()
    assert list(got) == [0, -1, -1, 0]
    assert np.array_equal(got, with_head(B, n, "fp64", g))
