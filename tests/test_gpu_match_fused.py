"""The matching head without grids (soft_match with a NULL grid), through the
C-ABI: the last FFT pass of the inverse reduces its values to argmax partial
results instead of storing them.  The same values are compared with the same
tie rule, so the indices must equal those of soft_match with a grid exactly,
at every FFT length (blocks of fewer and of more than 64 threads) and in
every precision; all-equal grids give index 0, all-NaN grids -1.  The head
with a grid is held to the oracle by test_gpu_match.py.  Inputs are seeded
synthetic data from paper_1808_00896_amd.inputs.
"""
import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs, soft

pytestmark = pytest.mark.gpu

CDT = {"fp64": torch.complex128, "fp32": torch.complex64, "fp32_split": torch.complex64}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(a, dev, prec):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(dev).to(CDT[prec])


def both(m, a, b):
    _, with_grid = m.match(a, b)
    fused = m.match_index(a, b)
    torch.cuda.synchronize()
    return with_grid.cpu().numpy(), fused.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_split"])
@pytest.mark.parametrize("B,n", [(1, 2), (2, 3), (4, 1), (8, 5), (16, 3), (32, 2), (64, 2)])
def test_fused_argmax_equals_grid_argmax(dev, prec, B, n):
    a, b = inputs.sh_pair_batch(n, B, seed=40 + B)
    with soft.MatchPlan(B, n, precision=prec) as m:
        i_grid, i_fused = both(m, to_dev(a, dev, prec), to_dev(b, dev, prec))
    assert np.array_equal(i_grid, i_fused), (i_grid, i_fused)
    assert np.all((i_fused >= 0) & (i_fused < (2 * B) ** 3))


def test_fused_argmax_full_size(dev):
    B, n = 128, 2
    a, b = inputs.sh_pair_batch(n, B, seed=6)
    with soft.MatchPlan(B, n) as m:
        i_grid, i_fused = both(m, to_dev(a, dev, "fp64"), to_dev(b, dev, "fp64"))
    assert np.array_equal(i_grid, i_fused)


@pytest.mark.parametrize("B", [2, 16, 64])
def test_fused_argmax_ties_and_nan(dev, B):
    """Zero inputs: every grid entry is exactly 0, so the first index wins.
    NaN inputs: every entry is NaN, so no index wins (-1)."""
    n = 2
    z = torch.zeros((n, B * B), dtype=torch.complex128, device=dev)
    nan = torch.full((n, B * B), complex(float("nan"), 0.0), dtype=torch.complex128, device=dev)
    with soft.MatchPlan(B, n) as m:
        i_grid, i_fused = both(m, z, z)
        assert np.array_equal(i_grid, [0, 0]) and np.array_equal(i_fused, [0, 0])
        g, i_grid = m.match(nan, z)
        torch.cuda.synchronize()
        assert torch.isnan(g.real).all()
        i_fused = m.match_index(nan, z)
        assert np.array_equal(i_grid.cpu().numpy(), [-1, -1])
        assert np.array_equal(i_fused.cpu().numpy(), [-1, -1])


def test_fused_argmax_needs_own_intermediate(dev):
    B, n = 8, 2
    a, b = inputs.sh_pair_batch(n, B, seed=3)
    with soft.MatchPlan(B, n, inplace_ok=True) as m:
        with pytest.raises(soft.SoftError) as e:
            m.match_index(to_dev(a, dev, "fp64"), to_dev(b, dev, "fp64"))
        assert e.value.status == soft.SOFT_ERR_INVALID
        _, idx = m.match(to_dev(a, dev, "fp64"), to_dev(b, dev, "fp64"))
        torch.cuda.synchronize()
        assert np.all(idx.cpu().numpy() >= 0)
