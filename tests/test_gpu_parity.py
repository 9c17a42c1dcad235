"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Bar: max |x - x_oracle| / max |x_oracle| over all outputs
  * <= 1e-11 in FP64 for B <= 256 (against the double oracle),
  * <= 1e-9 at B = 512 (against the long-double oracle, sampled).
Inputs are seeded synthetic data from paper_1808_00896_amd.inputs.
"""
import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs
from paper_1808_00896_amd import soft

pytestmark = pytest.mark.gpu

TOL64 = 1e-11


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(dev)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("B", [1, 2, 4, 8, 16, 32, 64])
def test_inverse_matches_oracle(oracle, dev, B):
    c = inputs.coeffs_uniform(B, 10 + B)
    with soft.Plan(B) as p:
        g = to_host(p.inverse(to_dev(c, dev)))
    want = oracle.inverse(B, c)
    assert relerr(g, want) <= TOL64


@pytest.mark.parametrize("B", [1, 2, 4, 8, 16, 32, 64])
def test_forward_matches_oracle(oracle, dev, B):
    """Forward on a random, not band-limited grid: the quadrature sum itself."""
    g = inputs.grid_random(B, 20 + B)
    with soft.Plan(B) as p:
        c = to_host(p.forward(to_dev(g, dev)))
    want = oracle.forward(B, g)
    assert relerr(c, want) <= TOL64


@pytest.mark.parametrize("B", [2, 8, 32])
def test_adjoints_match_oracle(oracle, dev, B):
    c = inputs.coeffs_uniform(B, 30 + B)
    g = inputs.grid_random(B, 40 + B)
    with soft.Plan(B) as p:
        ga = to_host(p.adjoint(to_dev(c, dev)))
        ci = to_host(p.adjoint_inverse(to_dev(g, dev)))
    assert relerr(ga, oracle.adjoint(B, c)) <= TOL64
    assert relerr(ci, oracle.adjoint_inverse(B, g)) <= TOL64


def test_round_trip_B16(oracle, dev):
    """Round trip of uniform[-1, 1] coefficients at B = 16 (inverse, then forward)."""
    B = 16
    c = inputs.coeffs_uniform(B, 0)
    with soft.Plan(B) as p:
        g = p.inverse(to_dev(c, dev))
        c2 = to_host(p.forward(g))
        g = to_host(g)
    assert relerr(g, oracle.inverse(B, c)) <= TOL64
    assert relerr(c2, c) <= TOL64


def test_batched_plan(oracle, dev):
    B, n = 16, 3
    cs = [inputs.coeffs_decay(B, 50 + i) for i in range(n)]
    with soft.Plan(B, batch=n) as p:
        g = p.inverse(to_dev(np.stack(cs), dev))
        c2 = to_host(p.forward(g))
        g = to_host(g)
    for i in range(n):
        assert relerr(g[i], oracle.inverse(B, cs[i])) <= TOL64
        assert relerr(c2[i], cs[i]) <= TOL64


def test_deterministic(dev):
    B = 32
    c = to_dev(inputs.coeffs_decay(B, 60), dev)
    with soft.Plan(B) as p:
        g1 = p.inverse(c).clone()
        g2 = p.inverse(c)
        c1 = p.forward(g1).clone()
        c2 = p.forward(g2)
        torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(c1, c2)


def test_B128_full(oracle, dev):
    """Full comparison at B = 128 (256^3 grid), the spec bandwidth."""
    B = 128
    c = inputs.coeffs_decay(B, 1)
    with soft.Plan(B) as p:
        gd = p.inverse(to_dev(c, dev))
        cd = to_host(p.forward(gd))
        g = to_host(gd)
    want_g = oracle.inverse(B, c)
    assert relerr(g, want_g) <= TOL64
    want_c = oracle.forward(B, want_g)
    assert relerr(cd, want_c) <= TOL64
    assert relerr(cd, c) <= TOL64


def forward_pair_errors(oracle, B, grid, cd, pairs, prec="f64"):
    """Largest error over the listed order pairs of the coefficients cd (the
    HIP forward of grid) against the oracle's forward of the same grid,
    relative to the largest oracle coefficient of those pairs."""
    want = oracle.forward_pairs(B, grid, pairs, prec)
    errs = []
    for p_, (m, mp) in enumerate(pairs):
        l0 = max(abs(m), abs(mp))
        got = np.array([cd[oracle.coeff_index(l, m, mp)] for l in range(l0, B)])
        errs.append(np.abs(got - want[p_, l0:]).max())
    return float(max(errs) / np.abs(want).max())


def test_B256_sampled(oracle, dev):
    """B = 256 (512^3 grid): sampled beta-slices of the inverse against the
    double oracle, the round trip, and sampled order pairs of the forward of a
    random grid."""
    B = 256
    c = inputs.coeffs_decay(B, 2)
    gr = inputs.grid_random(B, 22)
    js = (0, 1, 255, 256, 511)
    with soft.Plan(B) as p:
        gd = p.inverse(to_dev(c, dev))
        sl = {j: to_host(gd[:, j, :]) for j in js}
        cd = to_host(p.forward(gd))
        del gd
        cr = to_host(p.forward(to_dev(gr, dev)))
    for j in js:
        assert relerr(sl[j], oracle.inverse_slice(B, c, j)) <= TOL64, j
    assert relerr(cd, c) <= TOL64
    pairs = [(0, 0), (1, -1), (37, 200), (-128, 5), (255, -255), (-3, 254)]
    assert forward_pair_errors(oracle, B, gr, cr, pairs) <= TOL64


def test_B512_sampled(oracle, dev):
    """B = 512 (1024^3 complex128 grid, 16 GiB): sampled inverse slices against
    the long-double oracle (gate 1e-9), the round trip over all 1.8e8
    coefficients, and sampled order pairs of the forward of a random grid."""
    B = 512
    c = inputs.coeffs_decay(B, 3)
    js = (0, 700)
    with soft.Plan(B) as p:
        gd = p.inverse(to_dev(c, dev))
        sl = {j: to_host(gd[:, j, :]) for j in js}
        cd = to_host(p.forward(gd))
        del gd
        torch.cuda.empty_cache()
        gr = inputs.grid_random(B, 23)
        cr = to_host(p.forward(to_dev(gr, dev)))
        torch.cuda.empty_cache()
    assert relerr(cd, c) <= 1e-9
    for j in js:
        assert relerr(sl[j], oracle.inverse_slice(B, c, j, prec="f80")) <= 1e-9, j
    pairs = [(0, 0), (511, -511), (-300, 17), (64, 63)]
    assert forward_pair_errors(oracle, B, gr, cr, pairs) <= 1e-9


def test_plan_errors_on_gpu(dev):
    with pytest.raises(soft.SoftError):
        soft.Plan(3)
    with pytest.raises(soft.SoftError):
        soft.Plan(2048)
    p = soft.Plan(4)
    with pytest.raises(ValueError):
        p.inverse(torch.zeros(10, dtype=torch.complex128, device=dev))
    with pytest.raises(ValueError):
        p.forward(torch.zeros((8, 8, 8), dtype=torch.complex64, device=dev))
    p.close()
    p.close()


def test_plan_out_of_memory_is_reported(dev):
    """A plan whose workspace cannot fit (64 functions at B = 512: 1.1 TB of
    per-order-pair samples) returns SOFT_ERR_OOM, frees what it took, and the
    device then runs a transform as before."""
    with pytest.raises(soft.SoftError) as err:
        soft.Plan(512, batch=64)
    assert err.value.status == soft.SOFT_ERR_OOM
    B = 8
    c = inputs.coeffs_uniform(B, 7)
    with soft.Plan(B) as p:
        c2 = to_host(p.forward(p.inverse(to_dev(c, dev))))
    assert relerr(c2, c) <= TOL64
