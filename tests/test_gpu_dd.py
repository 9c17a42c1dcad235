"""The double-double Wigner-d recurrence (SOFT_DD_RECURRENCE) through the
C-ABI, against the long-double oracle.

The mode runs eq. "Wigner_d_recurrence" with its coefficients, cos(beta_j)
and the recurrence values in double-double, and leaves the FP64 rounding of
the FFT and of the matrix contraction: its results should sit at the FP64
floor (about 1e-15 of the largest value) at every bandwidth, where the plain
FP64 recurrence loses accuracy with the degree and near beta = 0 and pi
(5.9e-13 on the first beta slice at B = 512).  Bars: max-norm errors and the
per-degree error max|D(l)| / max|c(l)| of the forward of the oracle's grid
(the sampling theorem of Sect. 2.3 gives back the coefficients exactly).
Inputs are seeded synthetic coefficients and grids.
"""
import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs, soft

pytestmark = pytest.mark.gpu

DD_SHAPES = [(1, 1), (2, 1), (4, 1), (8, 1), (2, 2), (4, 2), (8, 2), (16, 1), (4, 4)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(dev)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def degree_errors(got, want, B):
    """max |got - want| / max |want| over each degree's block."""
    out = np.zeros(B)
    for l in range(B):
        s = slice(l * (4 * l * l - 1) // 3, (l + 1) * (4 * (l + 1) ** 2 - 1) // 3)
        out[l] = np.abs(got[s] - want[s]).max() / np.abs(want[s]).max()
    return out


@pytest.mark.parametrize("B", [1, 8, 32, 64])
def test_dd_matches_long_double_oracle(oracle, dev, B):
    """Inverse of decaying coefficients against the oracle's inverse, and the
    forward of the oracle's grid against the coefficients; at B = 64 the plain
    FP64 plan is measured beside it and is at least four times worse."""
    c = inputs.coeffs_decay(B, 500 + B)
    g_o = oracle.inverse(B, c, "f80")
    errs = {}
    for dd in (False, True):
        with soft.Plan(B, dd=dd) as p:
            assert p.describe()["dd_recurrence"] == dd
            g = host(p.inverse(to_dev(c, dev)))
            cf = host(p.forward(to_dev(g_o, dev)))
        errs[dd] = (relerr(g, g_o), relerr(cf, c), float(degree_errors(cf, c, B).max()))
        print(f"B={B} dd={dd}: inverse {errs[dd][0]:.2e}, forward {errs[dd][1]:.2e}, per degree {errs[dd][2]:.2e}")
    assert errs[True][0] <= 2e-15 and errs[True][1] <= 2e-15
    assert errs[True][2] <= 1e-14
    if B == 64:
        assert 4 * errs[True][0] <= errs[False][0]
        assert 4 * errs[True][2] <= errs[False][2]


@pytest.mark.parametrize("B", [16, 64])
def test_every_dd_shape(oracle, dev, B):
    """Each double-double launch shape that covers 2B, pinned for both
    directions, against the oracle; the shapes without a double-double form
    and the Clenshaw forms are refused."""
    c = inputs.coeffs_decay(B, 520 + B)
    gr = inputs.grid_random(B, 530 + B)
    want_g, want_c = oracle.inverse(B, c, "f80"), oracle.forward(B, gr, "f80")
    with soft.Plan(B, dd=True) as p:
        for sh in DD_SHAPES:
            if sh[0] * sh[1] * 64 < 2 * B:
                continue
            p.set_dwt_shape(0, 0, *sh)
            p.set_dwt_shape(0, 1, *sh)
            g = host(p.inverse(to_dev(c, dev)))
            cf = host(p.forward(to_dev(gr, dev)))
            assert relerr(g, want_g) <= 2e-15, sh
            assert relerr(cf, want_c) <= 2e-15, sh
        for sh in ((1, 2), (8, 4), (0, 0)):
            for d in (0, 1):
                with pytest.raises(soft.SoftError):
                    p.set_dwt_shape(0, d, *sh)


def test_dd_tuned_and_uneven(oracle, dev):
    """A tuned plan keeps to the double-double shapes; an uneven plan of six
    bandwidths matches the oracle function by function."""
    with soft.Plan(64, dd=True, tune=True) as p:
        for d in p.describe()["dwt_launches"]:
            assert tuple(d["forward"]) in DD_SHAPES and tuple(d["inverse"]) in DD_SHAPES
    Bs = [2, 64, 1, 16, 32, 8]
    cs = [inputs.coeffs_decay(B, 540 + f) for f, B in enumerate(Bs)]
    with soft.UnevenPlan(Bs, dd=True) as p:
        g = host(p.inverse(to_dev(np.concatenate(cs), dev)))
        goff = p.grid_offsets
    for f, B in enumerate(Bs):
        N = 2 * B
        want = oracle.inverse(B, cs[f], "f80")
        assert relerr(g[goff[f]:goff[f + 1]].reshape(N, N, N), want) <= 2e-15, (f, B)


def test_dd_halves_inplace_graph(dev):
    """Beta halves, in place and as a HIP graph: the inverse bit for bit
    against the plain double-double plan, the forward to the rounding of
    the halves' one addition."""
    B = 128
    c = inputs.coeffs_decay(B, 550)
    with soft.Plan(B, dd=True) as p:
        g0 = p.inverse(to_dev(c, dev))
        c0 = p.forward(g0.clone())
        torch.cuda.synchronize()
    with soft.Plan(B, dd=True, beta_halves=True, inplace_ok=True, graph=True) as q:
        assert q.describe()["dwt_launches"][0]["beta_halves"] == 2
        for _ in range(2):
            g1 = q.inverse(to_dev(c, dev))
            assert torch.equal(g1, g0)
            c1 = q.forward(g1)
            torch.cuda.synchronize()
            assert float((c1 - c0).abs().max() / c0.abs().max()) <= 1e-15


def test_dd_B512_sampled(oracle, dev):
    """B = 512: beta slices at both ends and in the middle against the
    long-double oracle, sampled order pairs of the forward of a random grid,
    and the round trip, each to a few 1e-15, where the plain FP64
    recurrence errs by about 6e-13 on the first slice."""
    B = 512
    c = inputs.coeffs_decay(B, 3)
    js = (0, 1, 512, 1023)
    with soft.Plan(B, dd=True) as p:
        gd = p.inverse(to_dev(c, dev))
        sl = {j: host(gd[:, j, :]) for j in js}
        cd = host(p.forward(gd))
        del gd
        torch.cuda.empty_cache()
        gr = inputs.grid_random(B, 23)
        cr = host(p.forward(to_dev(gr, dev)))
    torch.cuda.empty_cache()
    err_rt = relerr(cd, c)
    print(f"B=512 dd round trip {err_rt:.2e}")
    assert err_rt <= 1e-14
    for j in js:
        err = relerr(sl[j], oracle.inverse_slice(B, c, j, "f80"))
        print(f"B=512 dd inverse slice {j}: {err:.2e}")
        assert err <= 4e-15, j
    pairs = [(0, 0), (511, -511), (-300, 17), (64, 63), (1, -1)]
    want = oracle.forward_pairs(B, gr, pairs, "f80")
    for k, (m, mp) in enumerate(pairs):
        l0 = max(abs(m), abs(mp))
        got = np.array([cr[oracle.coeff_index(l, m, mp)] for l in range(l0, B)])
        err = np.abs(got - want[k, l0:]).max() / np.abs(want).max()
        print(f"B=512 dd forward pair {(m, mp)}: {err:.2e}")
        assert err <= 2e-15, (m, mp)


def test_dd_needs_fp64(dev):
    for prec in ("fp32", "fp32_split"):
        with pytest.raises(soft.SoftError):
            soft.Plan(8, precision=prec, dd=True)
