"""The autotune cache (SOFT_TUNE_CACHE): a tuned plan writes its launch
shapes under its key, a second plan with the same key takes them without
timing, a different key (other bandwidths or precision) tunes anew, and a
damaged file is ignored and rewritten.  Results of a plan with cached shapes
equal those of the plan that tuned them bit for bit (same shapes, same
arithmetic).  The variable is read at plan creation, so the test sets it in
its own process environment and restores it."""
import json
import os

import numpy as np
import pytest
import torch

from paper_1808_00896_amd import inputs, soft

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("SOFT_TUNE_CACHE", str(path))
    return path


def shapes(plan):
    return [(d["forward"], d["inverse"]) for d in plan.describe()["dwt_launches"]]


def test_cache_written_then_used(dev, cache):
    Bs = [16, 64, 64, 128]
    c = torch.from_numpy(np.concatenate([inputs.coeffs_decay(B, 400 + i) for i, B in enumerate(Bs)])).to(dev)
    with soft.UnevenPlan(Bs, tune=True) as p:
        assert p.describe()["tuned_from_cache"] is False
        first = shapes(p)
        g1 = p.inverse(c)
        torch.cuda.synchronize()
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.endswith("|fp64|whole|16x1,64x2,128x1"), key
    assert [tuple(map(list, ((v[0], v[1]), (v[2], v[3])))) for v in val] == first
    with soft.UnevenPlan(Bs, tune=True) as p:
        d = p.describe()
        assert d["tuned_from_cache"] is True and all(l["tuned"] for l in d["dwt_launches"])
        assert shapes(p) == first
        assert torch.equal(p.inverse(c), g1)
    with soft.Plan(64, precision="fp32", tune=True) as p:  # another key: tunes and adds its entry
        assert p.describe()["tuned_from_cache"] is False
    assert len(json.loads(cache.read_text())) == 2


def test_damaged_cache_is_ignored(dev, cache):
    cache.write_text("not json at all\n\"x\": [[1, 2]]\n")
    with soft.Plan(32, tune=True) as p:
        assert p.describe()["tuned_from_cache"] is False
    entries = json.loads(cache.read_text())
    assert list(entries) and all("|fp64|whole|32x1" in k for k in entries)


def test_untuned_plan_ignores_cache(dev, cache):
    with soft.Plan(32) as p:
        assert p.describe()["tuned_from_cache"] is False
    assert not cache.exists()
