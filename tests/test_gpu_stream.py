"""Streaming (non-temporal) stores, through the C-ABI.
A launch whose output array exceeds 192 MiB writes it with streaming stores
(the FFT passes and the inverse DWT), except at 2B = 1024.  A store hint changes
no value: 16 functions at B = 64 in one plan (537 MB a pass, streamed) must
equal the same functions transformed one at a time (34 MB a pass, plain
stores) bit for bit, in every transform, for the matrix-core and the Clenshaw
inverse.  B = 128 (268 MB, streamed) is held to the oracle by the parity
tests.  Inputs are seeded synthetic data from paper_1808_00896_amd.inputs.
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


def transforms(plan, c, g):
    out = (plan.inverse(c), plan.forward(g), plan.adjoint(c), plan.adjoint_inverse(g))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32_split"])
@pytest.mark.parametrize("inverse_shape", [None, soft.CLENSHAW])
def test_streamed_batch_equals_single(dev, prec, inverse_shape):
    B, nf = 64, 16
    nc, n3 = inputs.num_coeffs(B), (2 * B) ** 3
    c = torch.from_numpy(np.concatenate([inputs.coeffs_decay(B, 10 + f) for f in range(nf)])).to(dev).to(CDT[prec])
    g = torch.cat([torch.from_numpy(inputs.grid_random(B, 70 + f)).reshape(-1).to(dev).to(CDT[prec])
                   for f in range(nf)])
    with soft.Plan(B, batch=nf, precision=prec) as pb, soft.Plan(B, precision=prec) as p1:
        assert nf * n3 * c.element_size() > 192 * 2 ** 20 > n3 * c.element_size()
        if inverse_shape is not None:
            pb.set_dwt_shape(0, 1, *inverse_shape)
            p1.set_dwt_shape(0, 1, *inverse_shape)
        batched = transforms(pb, c, g)
        for f in range(nf):
            single = transforms(p1, c[f * nc:(f + 1) * nc], g[f * n3:(f + 1) * n3])
            for k, (a, b) in enumerate(zip(batched, single)):
                n = a.numel() // nf
                assert torch.equal(a.reshape(-1)[f * n:(f + 1) * n], b.reshape(-1)), (f, k)
