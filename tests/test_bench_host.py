"""Host-side parts of bench.py that need no GPU: the algorithmic work model
behind the roofline, the step percentiles, the refusal of several GPUs, the
traffic lookup and the oracle-timing child leg."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_stage_work_fft_bytes():
    """Each FFT pass reads and writes every element once, without the +-B
    frequency row on the side where it is dropped (counted here by brute
    force over the index ranges)."""
    for B in (1, 2, 8, 128):
        N, P = 2 * B, 2 * B - 1
        w = bench.stage_work([B])
        kept_q = sum(1 for q in range(N) if q != B)            # q = m' mod N without +-B
        kept_mm = sum(1 for m in range(-(B - 1), B) for mp in range(-(B - 1), B))
        assert w["fft_gamma_fwd"] == ("hbm", 16.0 * (N ** 3 + N * N * kept_q))
        assert w["fft_alpha_fwd"] == ("hbm", 16.0 * (N * N * kept_q + N * kept_mm))
        assert w["fft_alpha_inv"] == w["fft_alpha_fwd"]
        assert w["fft_gamma_inv"] == w["fft_gamma_fwd"]
        assert P * P == kept_mm


def test_stage_work_dwt_flops():
    """Contraction: 2B samples x (re, im) x FMA per coefficient; recurrence:
    5 flops per step, per sample, over the representatives m >= m' >= 0 from
    l0 = m to B - 1 (enumerated here)."""
    for B in (1, 4, 16, 128):
        N = 2 * B
        ncoef = sum((2 * l + 1) ** 2 for l in range(B))
        steps = sum(B - 1 - m for m in range(B) for mp in range(m + 1))
        kind, flops = bench.stage_work([B])["dwt_fwd"]
        assert kind == "flop"
        assert flops == 2 * N * 2 * ncoef + 5.0 * N * steps
    # several functions add up
    assert bench.stage_work([4, 4, 8])["dwt_inv"][1] == 2 * bench.stage_work([4])["dwt_inv"][1] + \
        bench.stage_work([8])["dwt_inv"][1]


def test_stage_work_fp32_halves_bytes():
    w64, w32 = bench.stage_work([16]), bench.stage_work([16], "fp32_split")
    assert w32["fft_gamma_fwd"][1] * 2 == w64["fft_gamma_fwd"][1]
    assert w32["dwt_fwd"] == w64["dwt_fwd"]


def test_percentiles():
    ms = list(range(1, 101))
    p = bench.percentiles(ms)
    assert p == {"p10": round(float(np.percentile(ms, 10)), 4), "median": 50.5,
                 "p90": round(float(np.percentile(ms, 90)), 4)}
    assert p["p10"] < p["median"] < p["p90"]


def test_traffic_lookup_needs_matching_source():
    assert bench.measured_traffic("dwt_inv", 3) is None          # no such workload
    assert bench.measured_traffic("no_such_stage", 128) is None


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_oracle_child_leg_runs_on_cpu():
    env = dict(os.environ, OMP_NUM_THREADS="1")
    for what in ("inverse", "forward", "inverse_slices"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-leg", f"4:{what}"],
                           capture_output=True, text=True, timeout=120, env=env)
        assert r.returncode == 0, r.stderr
        out = json.loads(r.stdout.strip().splitlines()[-1])
        assert out["seconds"] > 0 and out["threads"] == 1


def test_traffic_lookup_signature():
    assert bench.measured_traffic("fp64_B3_n1", "dwt_inv") is None


def test_err_report_per_degree():
    """deg_rel[l] = max |dx| / max |ref| over degree l's (2l+1)^2 entries, with
    a planted error in one degree only."""
    B = 6
    rng = np.random.default_rng(0)
    ref = rng.standard_normal(bench.num_coeffs(B)) + 1j * rng.standard_normal(bench.num_coeffs(B))
    x = ref.copy()
    l = 4
    start = l * (4 * l * l - 1) // 3
    x[start + 3] += 1e-3
    r = bench.err_report(x, ref, B)
    blk = np.abs(ref[start:start + (2 * l + 1) ** 2]).max()
    assert r["deg_rel"][l] == bench.sig(1e-3 / blk, 2)
    assert all(v == 0.0 for k, v in enumerate(r["deg_rel"]) if k != l)
    assert r["max_rel"] == bench.sig(1e-3 / np.abs(ref).max())
    assert r["l2_rel"] == bench.sig(1e-3 / np.linalg.norm(ref))


def test_coeff_indices_and_pairs_report():
    """The sampled-pair indices are the l-major positions of f°(l, m, m'),
    and entries below a pair's lowest degree are ignored."""
    B = 8
    pairs = bench.sample_pairs(B)
    idx = bench.coeff_indices(B, pairs)
    for p, (m, mp) in enumerate(pairs):
        for l in range(max(abs(m), abs(mp)), B):
            assert idx[p, l] == l * (4 * l * l - 1) // 3 + (m + l) * (2 * l + 1) + (mp + l)
    ref = np.ones((len(pairs), B), dtype=complex)
    x = ref.copy()
    x[:, 0] += 5.0      # degree 0: below the lowest degree of every pair but (0, 0)
    x[0, 0] = ref[0, 0]
    r = bench.pairs_report(x, ref, pairs)
    assert r["max_rel"] == 0.0


def test_stage_of_kernel_names():
    assert bench.stage_of("k_fft<256, 0, 1, double2>") == "fft_gamma_fwd"
    assert bench.stage_of("k_fft_ingrid<1024, 2, -1, float2>") == "fft_alpha_inv"
    assert bench.stage_of("k_fft<64, 3, -1, double2>") == "fft_gamma_inv"
    assert bench.stage_of("k_dwt_fwd<4, 1, 0>") == "dwt_fwd"
    assert bench.stage_of("k_idwt_clenshaw<0, 1>") == "dwt_inv"
    assert bench.stage_of("k_probe_copy") is None


def test_workload_bands():
    assert bench._workload_bands("fp32_split_B128_n16") == ([128] * 16, "fp32_split")
    Bs, prec = bench._workload_bands("fp64_uneven256")
    assert prec == "fp64" and len(Bs) == 256 and set(Bs) == {16, 32, 64, 128}
    assert bench.calls_per_step("fp64_uneven256", "fft_alpha_fwd") == 4
    assert bench.calls_per_step("fp64_uneven256", "dwt_fwd") == 3
    assert bench.calls_per_step("fp64_B512_n1", "dwt_fwd") == 1


def test_only_workloads_parse_and_match_their_legs():
    """Every workload `--only` accepts names its bands and precision, and a
    one-bandwidth workload draws the coefficients its bench leg draws."""
    for w in bench.ONLY_LEGS:
        Bs, prec = bench._workload_bands(w)
        assert prec in ("fp64", "fp32", "fp32_split") and Bs and all(b & (b - 1) == 0 for b in Bs), w
    assert bench.ONLY_SEED == {128: 1, 256: 2, 512: 3}
    assert "fp64_B16_n1" in bench.ONLY_LEGS and bench.SMALL_B == 16
