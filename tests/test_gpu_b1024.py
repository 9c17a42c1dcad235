"""B = 1024 (2B = 2048 beta samples; a 2048^3 grid, 1.43e9 coefficients),
through the C-ABI with SOFT_INPLACE_OK in all three precisions.  The band
runs in beta halves (S for half of the beta samples at a time), which is what
lets FP64 fit one GPU: 137 GB of grid, 23 GB of coefficients and 82 GB of
plan.  Checked at full size through properties and samples the oracle
computes one by one: the round trip over all coefficients (forward of the
inverse, the sampling theorem of Sect. 2.3) and beta slices of the inverse
against the long-double oracle on the same (rounded) input.  At this
bandwidth some seeds of Sect. 2.2 that matter lie below double precision's
range (the double-build oracle loses d values of order 0.04, see
test_oracle_pins), so the long-double build is the reference; slices 488 and
1560 are among those where the extended-range seeds decide the result, and
the slices cover both beta halves (0, 488 and 1560 in the outer half, 1365 in
the middle one).  Inputs are seeded synthetic coefficients.
"""
import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs, soft

pytestmark = pytest.mark.gpu

B = 1024
SLICES = (0, 488, 1365, 1560)
TOL = {"fp64": 1e-9, "fp64_dd": 1e-14, "fp32": 2e-6, "fp32_split": 2e-6}
SHAPES = {"fp64": ([4, 4], [4, 4]), "fp64_dd": ([8, 2], [8, 2]), "fp32": ([4, 4], [8, 2]),
          "fp32_split": ([4, 4], [16, 1])}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def coeffs():
    print(f"B={B}: drawing {inputs.num_coeffs(B)} coefficients", flush=True)
    return inputs.coeffs_decay(B, 9)


def _max_rel(a, b, chunk=1 << 27):
    """max |a - b| / max |b| over two device vectors, in pieces (no full-size temporaries)."""
    num = den = 0.0
    for i in range(0, a.numel(), chunk):
        num = max(num, float((a[i:i + chunk] - b[i:i + chunk]).abs().max()))
        den = max(den, float(b[i:i + chunk].abs().max()))
    return num / den


@pytest.mark.parametrize("prec", ["fp64", "fp64_dd", "fp32_split", "fp32"])
def test_B1024(oracle, dev, coeffs, prec):
    """fp64_dd: the double-double recurrence (SOFT_DD_RECURRENCE), which
    brings the first beta slice from about 7e-13 to the FP64 floor."""
    dd = prec.endswith("_dd")
    c = coeffs if prec.startswith("fp64") else coeffs.astype(np.complex64)
    with soft.Plan(B, precision=prec.replace("_dd", ""), inplace_ok=True, dd=dd) as p:
        d = p.describe()["dwt_launches"][0]
        assert d["beta_halves"] == 2
        assert (d["forward"], d["inverse"]) == SHAPES[prec]
        cd = torch.from_numpy(c).to(dev)
        print(f"{prec}: inverse", flush=True)
        g = p.inverse(cd)
        slices = {j: g[:, j, :].cpu().numpy().astype(np.complex128) for j in SLICES}
        print(f"{prec}: forward", flush=True)
        c2 = p.forward(g)  # overwrites g (SOFT_INPLACE_OK)
        del g
        torch.cuda.synchronize()
        err_rt = _max_rel(c2, cd)
        del c2, cd
    torch.cuda.empty_cache()
    print(f"B={B} {prec} round trip {err_rt:.2e}", flush=True)
    c = c.astype(np.complex128)
    errs = {}
    for j, sl in slices.items():
        want = oracle.inverse_slice(B, c, j, "f80")
        errs[j] = float(np.abs(sl - want).max() / np.abs(want).max())
        print(f"B={B} {prec} inverse slice {j}: {errs[j]:.2e}", flush=True)
    assert err_rt <= TOL[prec]
    assert max(errs.values()) <= TOL[prec], errs


def test_B1024_in_an_uneven_plan(oracle, dev, coeffs):
    """B = 1024 (in beta halves, extended-range seeds) sharing a plan with
    B = 16 and B = 64 functions, FP32-split in place: the small functions
    equal their single-bandwidth plans bit for bit, and the B = 1024 one
    round-trips."""
    prec = "fp32_split"
    Bs = [16, 1024, 64]
    small = {16: inputs.coeffs_decay(16, 91), 64: inputs.coeffs_decay(64, 92)}
    cs = [small[16], coeffs, small[64]]
    with soft.UnevenPlan(Bs, precision=prec, inplace_ok=True) as p:
        halves = {d["max_2B"]: d["beta_halves"] for d in p.describe()["dwt_launches"]}
        assert halves[2048] == 2 and halves.get(128, 1) == 1
        cd = torch.from_numpy(np.concatenate(cs).astype(np.complex64)).to(dev)
        g = p.inverse(cd)
        gs = {B: g[p.grid_offsets[f]:p.grid_offsets[f + 1]].clone() for f, B in enumerate(Bs) if B < 1024}
        c2 = p.forward(g)
        del g
        torch.cuda.synchronize()
        o = p.coeff_offsets
        err = _max_rel(c2[o[1]:o[2]], cd[o[1]:o[2]])
        c_small = {B: c2[o[f]:o[f + 1]].clone() for f, B in enumerate(Bs) if B < 1024}
        del c2, cd
    torch.cuda.empty_cache()
    print(f"uneven with B=1024 {prec}: round trip {err:.2e}", flush=True)
    assert err <= TOL[prec]
    for B in (16, 64):
        with soft.Plan(B, precision=prec, inplace_ok=True) as q:
            c1 = torch.from_numpy(small[B].astype(np.complex64)).to(dev)
            g1 = q.inverse(c1)
            assert torch.equal(g1.reshape(-1), gs[B]), B
            assert torch.equal(q.forward(g1).reshape(-1), c_small[B]), B
