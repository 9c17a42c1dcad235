"""Stage timers through the C-ABI: every stage, a chosen subset, none."""
import ctypes

import pytest
import torch

from paper_1808_00896_amd import inputs, soft

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def test_stage_timers(dev):
    B = 16
    with soft.Plan(B) as p:
        c = torch.from_numpy(inputs.coeffs_decay(B, 1)).to(dev)
        g = p.inverse(c)

        def step(k=3):
            for _ in range(k):
                p.inverse(c, out=g)
                p.forward(g)
            torch.cuda.synchronize()

        transform_stages = soft.STAGES[:6]
        soft.soft_plan_stage_times(p.handle, reset=True)
        soft.soft_plan_set_timing(p.handle, True)
        step()
        st = soft.soft_plan_stage_times(p.handle, reset=True)
        for name in transform_stages:
            ms, n = st[name]
            assert n == 3 and ms > 0, name

        soft.soft_plan_set_timing_stages(p.handle, ["dwt_inv", "fft_gamma_fwd"])
        step()
        st = soft.soft_plan_stage_times(p.handle, reset=True)
        assert {k for k, (ms, n) in st.items() if n} == {"dwt_inv", "fft_gamma_fwd"}
        assert st["dwt_inv"][1] == 3 and st["fft_gamma_fwd"][1] == 3

        soft.soft_plan_set_timing(p.handle, False)
        step()
        st = soft.soft_plan_stage_times(p.handle, reset=True)
        assert all(n == 0 for ms, n in st.values())

        # a bit past the last stage is rejected
        L = soft.lib()
        assert L.soft_plan_set_timing_stages(ctypes.c_void_p(p.handle), 1 << len(soft.STAGES)) == soft.SOFT_ERR_INVALID
