"""The inverse DWT by Clenshaw's backward summation (inverse "shape" 0x0),
through the C-ABI, against the oracle and against the matrix-core inverse.

Bars as for the other inverse paths: FP64 1e-11 relative to the oracle
(max-norm), FP32 4e-6 and FP32-split 1e-6 against the FP64 oracle on the same
FP32-rounded input; against the matrix-core inverse (same sums in another
order) 1e-13 in FP64.  Inputs are seeded synthetic data from
paper_1808_00896_amd.inputs.
"""
import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs, soft

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32_split": 1e-6, "fp32": 4e-6}
CDT = {"fp64": np.complex128, "fp32_split": np.complex64, "fp32": np.complex64}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(a, dev, prec="fp64"):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=CDT[prec])).to(dev)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def rounded(a, prec):
    return np.asarray(a, dtype=CDT[prec]).astype(np.complex128)


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def clenshaw(plan):
    for i in range(len(plan.describe()["dwt_launches"])):
        plan.set_dwt_shape(i, 1, *soft.CLENSHAW)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_split"])
@pytest.mark.parametrize("B", [1, 2, 4, 8, 16, 32, 64, 128])
def test_clenshaw_inverse_matches_oracle(oracle, dev, prec, B):
    c = rounded(inputs.coeffs_decay(B, 170 + B), prec)
    with soft.Plan(B, precision=prec) as p:
        clenshaw(p)
        assert p.describe()["dwt_launches"][0]["inverse"] == list(soft.CLENSHAW)
        g = host(p.inverse(to_dev(c, dev, prec)))
    err = relerr(g, oracle.inverse(B, c))
    print(f"B={B} {prec}: {err:.2e}")
    assert err <= TOL[prec]


def test_clenshaw_adjoint_and_batch(oracle, dev):
    """soft_adjoint (the scaled inverse) and a batch of three, against the
    matrix-core path of the same plan."""
    B, n = 16, 3
    c = to_dev(np.stack([inputs.coeffs_decay(B, 180 + f) for f in range(n)]), dev)
    with soft.Plan(B, n) as p:
        want_a, want_i = p.adjoint(c).clone(), p.inverse(c).clone()
        clenshaw(p)
        got_a, got_i = p.adjoint(c), p.inverse(c)
        torch.cuda.synchronize()
        for got, want in ((got_a, want_a), (got_i, want_i)):
            assert float((got - want).abs().max() / want.abs().max()) <= 1e-13


def test_clenshaw_uneven_matches_oracle(oracle, dev):
    Bs, cs = inputs.uneven_batch(8, [2, 8, 32, 64], seed=19)
    with soft.UnevenPlan(Bs) as p:
        clenshaw(p)
        g = host(p.inverse(to_dev(np.concatenate(cs), dev)))
    for f, B in enumerate(Bs):
        N = 2 * B
        gf = g[p.grid_offsets[f]:p.grid_offsets[f + 1]].reshape(N, N, N)
        assert relerr(gf, oracle.inverse(B, cs[f])) <= 1e-11, (f, B)


def test_clenshaw_only_for_the_inverse(dev):
    with soft.Plan(8) as p:
        with pytest.raises(soft.SoftError):
            p.set_dwt_shape(0, 0, *soft.CLENSHAW)


@pytest.mark.parametrize("B", [256, 512])
def test_clenshaw_large_agrees_with_mfma(dev, B):
    """2B = 512 and 1024: the Clenshaw inverse against the matrix-core inverse
    of the same plan (itself pinned to the oracle by the parity tests)."""
    c = to_dev(inputs.coeffs_decay(B, 190 + B), dev)
    with soft.Plan(B) as p:
        want = p.inverse(c)
        clenshaw(p)
        got = p.inverse(c)
        torch.cuda.synchronize()
        err = float((got - want).abs().max() / want.abs().max())
        print(f"B={B}: {err:.2e}")
        assert err <= 1e-12
        del got, want
    torch.cuda.empty_cache()
