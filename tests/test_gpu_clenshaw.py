"""The DWT pair by Clenshaw-type recurrences ("shape" 0x0): the inverse by
Clenshaw's backward summation and the forward by its transpose (the
adjoint-Clenshaw evaluation, sums over beta reduced across lanes), through the
C-ABI, against the oracle and against the matrix-core DWTs.

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


def clenshaw(plan, directions=(1,)):
    for i in range(len(plan.describe()["dwt_launches"])):
        for d in directions:
            plan.set_dwt_shape(i, d, *soft.CLENSHAW)


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


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_split"])
@pytest.mark.parametrize("B", [1, 2, 4, 8, 16, 32, 64, 128])
def test_clenshaw_forward_matches_oracle(oracle, dev, prec, B):
    """The adjoint-Clenshaw forward on random (not band-limited) grids: the
    quadrature sum itself."""
    g = rounded(inputs.grid_random(B, 200 + B), prec)
    with soft.Plan(B, precision=prec) as p:
        clenshaw(p, (0,))
        assert p.describe()["dwt_launches"][0]["forward"] == list(soft.CLENSHAW)
        c = host(p.forward(to_dev(g, dev, prec)))
    err = relerr(c, oracle.forward(B, g))
    print(f"forward B={B} {prec}: {err:.2e}")
    assert err <= TOL[prec]


def test_clenshaw_forward_adjoint_batch_uneven(oracle, dev):
    """soft_adjoint_inverse (unweighted, no V) and a batch of three against the
    matrix-core forward of the same plan; an uneven plan against the oracle."""
    B, n = 16, 3
    g = to_dev(np.stack([inputs.grid_random(B, 210 + f) for f in range(n)]), dev)
    with soft.Plan(B, n) as p:
        want_f, want_a = p.forward(g).clone(), p.adjoint_inverse(g).clone()
        clenshaw(p, (0,))
        got_f, got_a = p.forward(g), p.adjoint_inverse(g)
        torch.cuda.synchronize()
        for got, want in ((got_f, want_f), (got_a, want_a)):
            assert float((got - want).abs().max() / want.abs().max()) <= 1e-13
    Bs, _ = inputs.uneven_batch(8, [2, 8, 32, 64], seed=21)
    gs = [inputs.grid_random(B, 220 + f) for f, B in enumerate(Bs)]
    with soft.UnevenPlan(Bs) as p:
        clenshaw(p, (0, 1))
        c = host(p.forward(to_dev(np.concatenate([x.reshape(-1) for x in gs]), dev)))
    for f, B in enumerate(Bs):
        cf = c[p.coeff_offsets[f]:p.coeff_offsets[f + 1]]
        assert relerr(cf, oracle.forward(B, gs[f])) <= 1e-11, (f, B)


@pytest.mark.parametrize("B", [256, 512])
def test_clenshaw_large_against_oracle(oracle, dev, B):
    """2B = 512 and 1024: both Clenshaw directions against the oracle on
    sampled beta slices (inverse; the long-double oracle at B = 512), the
    round trip, and sampled order pairs of the forward of a random grid."""
    c = inputs.coeffs_decay(B, 230 + B)
    js = (0, B + 3, 2 * B - 1)
    with soft.Plan(B) as p:
        clenshaw(p, (0, 1))
        gd = p.inverse(to_dev(c, dev))
        sl = {j: host(gd[:, j, :]) for j in js}
        cd = host(p.forward(gd))
        del gd
        torch.cuda.empty_cache()
        gr = inputs.grid_random(B, 240 + B)
        cr = host(p.forward(to_dev(gr, dev)))
    torch.cuda.empty_cache()
    prec = "f80" if B == 512 else "f64"
    tol = 1e-9 if B == 512 else 1e-11
    assert relerr(cd, c) <= tol
    for j in js:
        err = relerr(sl[j], oracle.inverse_slice(B, c, j, prec=prec))
        print(f"B={B} inverse slice {j}: {err:.2e}")
        assert err <= tol, j
    pairs = [(0, 0), (B - 1, 1 - B), (-(B // 2), 7), (B // 4, B // 4 - 1)]
    want = oracle.forward_pairs(B, gr, pairs, prec)
    for k, (m, mp) in enumerate(pairs):
        l0 = max(abs(m), abs(mp))
        got = np.array([cr[oracle.coeff_index(l, m, mp)] for l in range(l0, B)])
        err = np.abs(got - want[k, l0:]).max() / np.abs(want).max()
        print(f"B={B} forward pair {(m, mp)}: {err:.2e}")
        assert err <= tol, (m, mp)


@pytest.mark.parametrize("B", [256, 512])
def test_clenshaw_large_agrees_with_mfma(dev, B):
    """2B = 512 and 1024: the Clenshaw inverse and forward against the
    matrix-core DWTs of the same plan (same sums, another order)."""
    c = to_dev(inputs.coeffs_decay(B, 190 + B), dev)
    with soft.Plan(B) as p:
        want = p.inverse(c)
        clenshaw(p)
        got = p.inverse(c)
        torch.cuda.synchronize()
        err = float((got - want).abs().max() / want.abs().max())
        print(f"B={B}: {err:.2e}")
        assert err <= 1e-12
        want_c = p.forward(got).clone()
        clenshaw(p, (0,))
        got_c = p.forward(got)
        torch.cuda.synchronize()
        err = float((got_c - want_c).abs().max() / want_c.abs().max())
        print(f"B={B} forward: {err:.2e}")
        assert err <= 1e-12
        del got, want, got_c, want_c
    torch.cuda.empty_cache()
