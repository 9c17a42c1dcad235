"""FP32 / FP32-split modes and plans over mixed bandwidths, through the C-ABI.

Bars (max |x - x_oracle| / max |x_oracle|, oracle in FP64 on the same
FP32-rounded input):
  * SOFT_FP32_SPLIT  <= 1e-6 (the accuracy the split mode is built for),
  * SOFT_FP32        <= 4e-6 (d rounded to FP32 as well),
  * SOFT_FP64 over an uneven plan: <= 1e-11 per function, as for one band.
A function inside an uneven plan whose band keeps the launch shape of a
one-bandwidth plan (2B >= 512) must match that plan bit for bit; smaller
bands run in the shared DWT launch and match to the precision's bar.
Inputs are seeded synthetic data from paper_1808_00896_amd.inputs.
"""
import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs
from paper_1808_00896_amd import soft

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32_split": 1e-6, "fp32": 4e-6}
CDT = {"fp64": np.complex128, "fp32_split": np.complex64, "fp32": np.complex64}


def relerr(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(a, dev, prec):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=CDT[prec])).to(dev)


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rounded(a, prec):
    """The input as the device sees it, widened back to complex128 for the oracle."""
    return np.asarray(a, dtype=CDT[prec]).astype(np.complex128)


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
@pytest.mark.parametrize("B", [1, 4, 16, 64, 128])
def test_fp32_inverse(oracle, dev, prec, B):
    c = rounded(inputs.coeffs_decay(B, 70 + B), prec)
    with soft.Plan(B, precision=prec) as p:
        g = to_host(p.inverse(to_dev(c, dev, prec)))
    err = relerr(g, oracle.inverse(B, c))
    print(f"inverse B={B} {prec}: {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
@pytest.mark.parametrize("B", [2, 16, 64, 128])
def test_fp32_forward(oracle, dev, prec, B):
    g = rounded(inputs.grid_random(B, 80 + B), prec)
    with soft.Plan(B, precision=prec) as p:
        c = to_host(p.forward(to_dev(g, dev, prec)))
    err = relerr(c, oracle.forward(B, g))
    print(f"forward B={B} {prec}: {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
def test_fp32_adjoints(oracle, dev, prec):
    B = 16
    c = rounded(inputs.coeffs_uniform(B, 90), prec)
    g = rounded(inputs.grid_random(B, 91), prec)
    with soft.Plan(B, precision=prec) as p:
        ga = to_host(p.adjoint(to_dev(c, dev, prec)))
        ci = to_host(p.adjoint_inverse(to_dev(g, dev, prec)))
    assert relerr(ga, oracle.adjoint(B, c)) <= TOL[prec]
    assert relerr(ci, oracle.adjoint_inverse(B, g)) <= TOL[prec]


def test_fp32_split_uses_the_tail(dev):
    """The split mode adds the FP32 tail of d: its result differs from the
    plain FP32 one, and both stay within their bars of the FP64 path on the
    same FP32 input.  (The two errors are of the same size: FP32 rounding of
    the data and of the matrix-core sums dominates the rounding of d.)"""
    B = 64
    c = inputs.coeffs_uniform(B, 92)
    with soft.Plan(B) as p:
        ref = to_host(p.inverse(to_dev(rounded(c, "fp32"), dev, "fp64")))
    outs = {}
    for prec in ("fp32", "fp32_split"):
        with soft.Plan(B, precision=prec) as p:
            outs[prec] = to_host(p.inverse(to_dev(c, dev, prec)))
        err = relerr(outs[prec], ref)
        print(f"{prec}: {err:.3e}")
        assert err <= TOL[prec]
    assert not np.array_equal(outs["fp32"], outs["fp32_split"])


@pytest.mark.parametrize("prec", ["fp64", "fp32_split"])
def test_uneven_matches_oracle(oracle, dev, prec):
    """Twelve functions with B drawn from 1..128: one inverse and one forward
    call over all of them, each function checked against the oracle."""
    Bs, cs = inputs.uneven_batch(12, [1, 2, 4, 8, 16, 32, 64, 128], seed=5)
    cs = [rounded(c, prec) for c in cs]
    with soft.UnevenPlan(Bs, precision=prec) as p:
        cflat = to_dev(np.concatenate(cs), dev, prec)
        gflat = p.inverse(cflat)
        c2 = to_host(p.forward(gflat))
        g = to_host(gflat)
        goff, coff = p.grid_offsets, p.coeff_offsets
    for f, B in enumerate(Bs):
        N = 2 * B
        gf = g[goff[f]:goff[f + 1]].reshape(N, N, N)
        assert relerr(gf, oracle.inverse(B, cs[f])) <= TOL[prec], (f, B)
        assert relerr(c2[coff[f]:coff[f + 1]], cs[f]) <= TOL[prec], (f, B)
    # forward of random grids (one per function) against the oracle's forward of the same grids
    gs = [rounded(inputs.grid_random(B, 60 + f), prec) for f, B in enumerate(Bs)]
    with soft.UnevenPlan(Bs, precision=prec) as p:
        cr = to_host(p.forward(to_dev(np.concatenate([x.reshape(-1) for x in gs]), dev, prec)))
    for f in (int(np.argmax(Bs)), int(np.argmin(Bs))):
        B = Bs[f]
        assert relerr(cr[coff[f]:coff[f + 1]], oracle.forward(B, gs[f])) <= TOL[prec], (f, B)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32_split"])
def test_uneven256_config_against_oracle(oracle, dev, prec):
    """The 256-function batch of bandwidths drawn from {16, 32, 64, 128}
    (seed 4, the throughput configuration), in a tuned plan as timed: the
    round trip of every function, and for the first function of each
    bandwidth its inverse, and the forward of a seeded random grid, against
    the oracle (FP64) on the same input as the device sees it."""
    Bs, cs = inputs.uneven_batch(256, [16, 32, 64, 128], seed=4)
    picks = [Bs.index(b) for b in sorted(set(Bs))]
    with soft.UnevenPlan(Bs, precision=prec, tune=True) as p:
        goff, coff = p.grid_offsets, p.coeff_offsets
        cflat = to_dev(np.concatenate(cs), dev, prec)
        gflat = p.inverse(cflat)
        c2 = p.forward(gflat)
        # round trip, every function, compared on the device
        worst = 0.0
        for f in range(len(Bs)):
            a, b = c2[coff[f]:coff[f + 1]], cflat[coff[f]:coff[f + 1]]
            worst = max(worst, float((a - b).abs().max() / b.abs().max()))
        print(f"{prec}: worst round trip over {len(Bs)} functions {worst:.3e}")
        assert worst <= TOL[prec]
        grids = {f: to_host(gflat[goff[f]:goff[f + 1]]) for f in picks}
        # forward of seeded random grids in the picked functions' slots
        gin = torch.zeros_like(gflat)
        rnd = {f: rounded(inputs.grid_random(Bs[f], 400 + f), prec) for f in picks}
        for f in picks:
            gin[goff[f]:goff[f + 1]] = to_dev(rnd[f].reshape(-1), dev, prec)
        cr = p.forward(gin)
        fwd = {f: to_host(cr[coff[f]:coff[f + 1]]) for f in picks}
        del cflat, gflat, c2, gin, cr
    torch.cuda.empty_cache()
    for f in picks:
        B = Bs[f]
        ei = relerr(grids[f].reshape((2 * B,) * 3), oracle.inverse(B, rounded(cs[f], prec)))
        ef = relerr(fwd[f], oracle.forward(B, rnd[f]))
        print(f"{prec} B={B} (function {f}): inverse {ei:.3e} forward {ef:.3e}")
        assert ei <= TOL[prec] and ef <= TOL[prec], (f, B, ei, ef)


def test_uneven_offsets_and_sizes(dev):
    Bs = [4, 1, 8, 4]
    with soft.UnevenPlan(Bs) as p:
        assert p.grid_offsets == [0, 512, 520, 520 + 4096, 520 + 4096 + 512]
        nc = [soft.num_coeffs(b) for b in Bs]
        assert p.coeff_offsets == list(np.concatenate([[0], np.cumsum(nc)]))
        g, c, _ = soft.soft_plan_sizes(p.handle)
        assert (g, c) == (p.grid_offsets[-1], p.coeff_offsets[-1])


@pytest.mark.parametrize("prec", ["fp64", "fp32_split"])
def test_uneven_large_bands_match_single_plans(dev, prec):
    """Bands of 2B >= 128 (here B = 64, 256 and 512) inside an uneven plan
    keep their own DWT launches and FFT passes: bit-identical to
    one-bandwidth plans.  The bands of 2B <= 64 share one launch and agree to
    the precision's bar."""
    Bs = [256, 8, 512, 64, 2] if prec == "fp32_split" else [256, 8, 64, 2]
    cs = [inputs.coeffs_decay(B, 100 + i) for i, B in enumerate(Bs)]
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    with soft.UnevenPlan(Bs, precision=prec) as p:
        gflat = p.inverse(to_dev(np.concatenate(cs), dev, prec))
        cflat = p.forward(gflat)
        torch.cuda.synchronize()
        grids = p.split_grids(gflat)
        coefs = p.split_coeffs(cflat)
        for f, B in enumerate(Bs):
            with soft.Plan(B, precision=prec) as q:
                gs = q.inverse(to_dev(cs[f], dev, prec))
                cs2 = q.forward(gs)
                torch.cuda.synchronize()
                if B >= 64:
                    assert torch.equal(grids[f], gs), B
                    assert torch.equal(coefs[f], cs2), B
                else:
                    assert relerr(to_host(grids[f]), to_host(gs)) <= TOL[prec], B
                    assert relerr(to_host(coefs[f]), to_host(cs2)) <= TOL[prec], B
                del gs, cs2
        assert grids[0].dtype == dt
        del gflat, cflat, grids, coefs
    torch.cuda.empty_cache()


def test_batched_fp32_split_matches_single(dev):
    """A batch of one bandwidth runs the same kernels per function as a plan
    of one function: bit-identical."""
    B, n = 32, 5
    cs = np.stack([inputs.coeffs_decay(B, 110 + i) for i in range(n)])
    with soft.Plan(B, batch=n, precision="fp32_split") as p:
        g = p.inverse(to_dev(cs, dev, "fp32_split"))
        c2 = p.forward(g)
        torch.cuda.synchronize()
        with soft.Plan(B, precision="fp32_split") as q:
            for i in range(n):
                gi = q.inverse(to_dev(cs[i], dev, "fp32_split"))
                assert torch.equal(g[i], gi)
                assert torch.equal(c2[i], q.forward(gi))


def test_uneven_deterministic(dev):
    Bs, cs = inputs.uneven_batch(9, [2, 8, 32, 64], seed=7)
    with soft.UnevenPlan(Bs, precision="fp32_split") as p:
        c = to_dev(np.concatenate(cs), dev, "fp32_split")
        g1 = p.inverse(c).clone()
        g2 = p.inverse(c)
        torch.cuda.synchronize()
        assert torch.equal(g1, g2)
        assert torch.equal(p.forward(g1), p.forward(g2))


def test_precision_dtype_checks(dev):
    with soft.Plan(4, precision="fp32") as p:
        with pytest.raises(ValueError):
            p.inverse(torch.zeros(soft.num_coeffs(4), dtype=torch.complex128, device=dev))
    with pytest.raises(ValueError):
        soft.Plan(4, precision="bf16")
    with pytest.raises(soft.SoftError):
        soft.UnevenPlan([4, 6])


def _covering(nmax):
    return [sh for sh in soft.DWT_SHAPES if sh[0] * sh[1] * 64 >= nmax]


@pytest.mark.parametrize("prec", ["fp64", "fp32_split"])
@pytest.mark.parametrize("B", [16, 64])
def test_every_dwt_shape_matches_oracle(oracle, dev, prec, B):
    """Each built launch shape that covers 2B, pinned in turn for both
    directions: inverse and forward against the oracle."""
    c = rounded(inputs.coeffs_decay(B, 120 + B), prec)
    g = rounded(inputs.grid_random(B, 130 + B), prec)
    want_g, want_c = oracle.inverse(B, c), oracle.forward(B, g)
    with soft.Plan(B, precision=prec) as p:
        for sh in _covering(2 * B):
            p.set_dwt_shape(0, 0, *sh)
            p.set_dwt_shape(0, 1, *sh)
            assert relerr(to_host(p.inverse(to_dev(c, dev, prec))), want_g) <= TOL[prec], sh
            assert relerr(to_host(p.forward(to_dev(g, dev, prec))), want_c) <= TOL[prec], sh


@pytest.mark.parametrize("prec", ["fp64", "fp32_split"])
def test_every_dwt_shape_B256_agrees(dev, prec):
    """At B = 256 every covering shape gives the default shape's result (the
    default is pinned to the oracle by the parity tests) to the precision's
    rounding: same sums, other order."""
    B = 256
    c = to_dev(inputs.coeffs_decay(B, 140), dev, prec)
    with soft.Plan(B, precision=prec) as p:
        ref_g = p.inverse(c).clone()
        ref_c = p.forward(ref_g).clone()
        tol = 1e-13 if prec == "fp64" else 1e-6
        for sh in _covering(2 * B):
            p.set_dwt_shape(0, 0, *sh)
            p.set_dwt_shape(0, 1, *sh)
            g = p.inverse(c)
            assert float((g - ref_g).abs().max() / ref_g.abs().max()) <= tol, sh
            cf = p.forward(ref_g)
            assert float((cf - ref_c).abs().max() / ref_c.abs().max()) <= tol, sh
            del g, cf
    torch.cuda.empty_cache()


def test_set_dwt_shape_rejects_bad_shapes(dev):
    with soft.Plan(64) as p:
        for args in ((1, 0, 2, 1), (0, 2, 2, 1), (0, 0, 1, 1), (0, 0, 3, 1), (0, 0, 16, 2), (0, 0, 2, 0),
                     (0, 1, 0, 1)):
            with pytest.raises(soft.SoftError):
                p.set_dwt_shape(*args)


@pytest.mark.parametrize("prec", ["fp64", "fp32_split"])
def test_tuned_plans_match_oracle(oracle, dev, prec):
    """SOFT_PLAN_TUNE picks a covering shape per launch and direction; the
    tuned one-bandwidth and uneven plans still meet the bar."""
    B = 32
    c = rounded(inputs.coeffs_decay(B, 150), prec)
    with soft.Plan(B, precision=prec, tune=True) as p:
        d = p.describe()
        assert d["dwt_launches"][0]["tuned"]
        for key in ("forward", "inverse"):
            nw, ns = d["dwt_launches"][0][key]
            assert ((nw, ns) in soft.DWT_SHAPES and nw * ns * 64 >= 2 * B) or \
                (nw, ns) == soft.CLENSHAW
        g = to_host(p.inverse(to_dev(c, dev, prec)))
        assert relerr(g, oracle.inverse(B, c)) <= TOL[prec]
    Bs, cs = inputs.uneven_batch(10, [4, 16, 64, 256], seed=9)
    cs = [rounded(x, prec) for x in cs]
    with soft.UnevenPlan(Bs, precision=prec, tune=True) as p:
        d = p.describe()
        assert all(l["tuned"] for l in d["dwt_launches"])
        assert sorted(b["B"] for b in d["bands"]) == sorted(set(Bs))
        gflat = p.inverse(to_dev(np.concatenate(cs), dev, prec))
        c2 = to_host(p.forward(gflat))
        g = to_host(gflat)
    for f, B in enumerate(Bs):
        if B <= 64:
            N = 2 * B
            gf = g[p.grid_offsets[f]:p.grid_offsets[f + 1]].reshape(N, N, N)
            assert relerr(gf, oracle.inverse(B, cs[f])) <= TOL[prec], (f, B)
        assert relerr(c2[p.coeff_offsets[f]:p.coeff_offsets[f + 1]], cs[f]) <= TOL[prec], (f, B)


@pytest.mark.parametrize("prec", ["fp32_split", "fp32"])
def test_fp32_B512_sampled(oracle, dev, prec):
    """B = 512 in the FP32 modes (their own 2B = 1024 launch shapes and the
    complex64 half-height forward alpha pass): sampled beta-slices of the
    inverse against the FP64 oracle on the same FP32-rounded coefficients,
    the round trip, and sampled order pairs of the forward of an FP32-rounded
    random grid against the oracle's forward of the same grid."""
    B = 512
    c = rounded(inputs.coeffs_decay(B, 3), prec)
    js = (0, 511, 700)
    with soft.Plan(B, precision=prec) as p:
        gd = p.inverse(to_dev(c, dev, prec))
        sl = {j: to_host(gd[:, j, :]) for j in js}
        cd = to_host(p.forward(gd))
        del gd
        torch.cuda.empty_cache()
        gr = rounded(inputs.grid_random(B, 4), prec)
        cr = to_host(p.forward(to_dev(gr, dev, prec)))
    torch.cuda.empty_cache()
    assert relerr(cd, c) <= 1e-6
    for j in js:
        assert relerr(sl[j], oracle.inverse_slice(B, c, j)) <= 1e-6, j
    pairs = [(0, 0), (3, -2), (100, 50), (-200, 7), (511, -511)]
    want = oracle.forward_pairs(B, gr, pairs)
    scale = np.abs(want).max()
    for (m, mp), w in zip(pairs, want):
        l0 = max(abs(m), abs(mp))
        ls = np.arange(l0, B)
        got = cr[ls * (4 * ls * ls - 1) // 3 + (m + ls) * (2 * ls + 1) + (mp + ls)]
        assert np.abs(got - w[l0:]).max() / scale <= 1e-6, (m, mp)