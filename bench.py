"""Benchmark: SO(3) FFT forward + inverse throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--B 128]

A step is one inverse (coefficients -> grid) followed by one forward (grid ->
coefficients) of one function at bandwidth B in FP64: the whole hot path
(iDWT, two FFT passes, two FFT passes, DWT).  Inputs are
seeded synthetic band-limited coefficients (i.i.d. normal parts scaled by
(1+l)^-1) already resident in HBM when the timed region starts.

Printed: one JSON line with the throughput (fwd+inv per second), the
roofline of the dominant kernel (HIP-event stage timers recorded inside the
library on the launch stream during the timed region), the round-trip error,
the oracle timed on the host cores, and a B = 512 leg.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 (vector and matrix), published
METRIC = "SOFT fwd+inv/sec at B=128 & 512: FP64 plain vs batched FP32-split @ ≤1e-6 err"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {"fft": "fft.hip", "dwt": "dwt.hip"}


def num_coeffs(B):
    return B * (4 * B * B - 1) // 3


def stage_work(B, batch=1):
    """Algorithmic bytes (HBM-bound stages) or flops (DWT) per launch.

    FFT passes: every complex128 element read once and written once, with the
    +-B frequency row absent on the side where it is dropped.  Reorder: the
    coefficients read and written once.  DWT: 8B flops per coefficient for
    the contraction (complex x real over 2B beta samples, FMA = 2 flops) plus
    5 flops per recurrence step per beta sample and symmetry group.
    """
    N, P = 2 * B, 2 * B - 1
    nc = num_coeffs(B)
    steps = sum((m + 1) * (B - 1 - m) for m in range(B))  # recurrence steps over groups m >= m' >= 0
    dwt_flops = 8.0 * B * nc + 5.0 * N * steps
    w = {
        "fft_gamma_fwd": ("hbm", 16.0 * (N ** 3 + N * N * (N - 1))),
        "fft_alpha_fwd": ("hbm", 16.0 * (N * N * (N - 1) + N * P * P)),
        "dwt_fwd": ("flop", dwt_flops),
        "dwt_inv": ("flop", dwt_flops),
        "fft_alpha_inv": ("hbm", 16.0 * (N * P * P + N * N * (N - 1))),
        "fft_gamma_inv": ("hbm", 16.0 * (N * N * (N - 1) + N ** 3)),
    }
    return {k: (kind, v * batch) for k, (kind, v) in w.items()}


def source_digest(kind):
    path = os.path.join(ROOT, "paper_1808_00896_amd", "csrc", KERNEL_SOURCES[kind])
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(stage, B):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None when
    absent or taken on a different version of the kernel source."""
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    rec = data.get(f"B{B}", {}).get(stage)
    if not rec:
        return None
    kind = "fft" if stage.startswith("fft") else "dwt"
    if rec.get("source_sha") != source_digest(kind):
        return None
    return rec.get("bytes_per_launch")


def roofline(stage_ms, B, batch=1):
    work = stage_work(B, batch)
    avg = {k: ms / n for k, (ms, n) in stage_ms.items() if n}
    dom = max(avg, key=avg.get)
    kind, amount = work[dom]
    t = avg[dom] * 1e-3
    if kind == "hbm":
        achieved = amount / t / 1e9
        r = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}
    else:
        achieved = amount / t / 1e12
        r = {"kernel": dom, "bound": "mfma" if dom == "dwt_fwd" else "alu", "achieved": round(achieved, 2),
             "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4)}
    r["avg_launch_ms"] = round(avg[dom], 5)
    r["algorithmic_per_launch"] = amount
    r["traffic"] = measured_traffic(dom, B)
    return r


def per_stage(stage_ms, B, batch=1):
    work = stage_work(B, batch)
    out = {}
    for k, (ms, n) in stage_ms.items():
        if not n:
            continue
        a = ms / n
        kind, amount = work[k]
        rate = amount / (a * 1e-3)
        out[k] = {"ms": round(a, 5), ("GB/s" if kind == "hbm" else "TFLOP/s"):
                  round(rate / 1e9, 1) if kind == "hbm" else round(rate / 1e12, 2)}
    return out


def run_gpu(B, steps, warmup, seed, batch=1):
    import torch
    from paper_1808_00896_amd import inputs, soft

    plan = soft.Plan(B, batch=batch)
    c_host = np.stack([inputs.coeffs_decay(B, seed + i) for i in range(batch)]) if batch > 1 else \
        inputs.coeffs_decay(B, seed)
    c = torch.from_numpy(c_host).cuda()
    grid = torch.empty(plan.grid_shape(), dtype=torch.complex128, device="cuda")
    c2 = torch.empty_like(c)

    def step():
        plan.inverse(c, out=grid)
        plan.forward(grid, out=c2)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    soft.soft_plan_stage_times(plan.handle, reset=True)
    soft.soft_plan_set_timing(plan.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    soft.soft_plan_set_timing(plan.handle, False)
    st = soft.soft_plan_stage_times(plan.handle, reset=True)
    err = float((c2 - c).abs().max() / c.abs().max())
    plan.close()
    del c, c2, grid
    torch.cuda.empty_cache()
    return {"elapsed": t1 - t0, "stages": st, "round_trip_err": err, "c_host": c_host}


def cpu_baseline(B, c_host, budget_s=12.0, max_reps=3):
    from oracle import oracle as O
    reps, t = 0, 0.0
    while reps < max_reps and (reps == 0 or t < budget_s):
        t0 = time.perf_counter()
        g = O.inverse(B, c_host)
        O.forward(B, g)
        t += time.perf_counter() - t0
        reps += 1
    return {"value": round(reps / t, 4), "unit": "fwd+inv/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{reps} x (inverse + forward) at B={B}, FP64 oracle (OpenMP), same coefficients",
            "seconds": round(t, 2)}


def calibrate_copy(gib=1.0):
    """A plain device copy of known size, for scaling the rocprofv3 byte counters."""
    import torch
    n = int(gib * (1 << 30)) // 16
    a = torch.zeros(n, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return 2 * n * 16


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--B", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-b512", action="store_true")
    ap.add_argument("--b512-steps", type=int, default=5)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device copy (byte-counter calibration under rocprofv3)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the transform is built and timed on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    B = args.B
    print(f"[bench] B={B} steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    r = run_gpu(B, args.steps, args.warmup, seed=1)
    ms = r["elapsed"] / args.steps * 1e3
    value = args.steps / r["elapsed"]
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "fwd+inv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded N(0,1)*(1+l)^-1 complex coefficients (band-limited)",
        "config": {"workload": f"one FP64 inverse + forward SO(3) FFT at B={B} "
                               f"({2 * B}^3 complex128 grid, {num_coeffs(B)} coefficients)",
                   "B": B, "batch": 1, "precision": "fp64"},
        "roofline": roofline(r["stages"], B),
        "stages": per_stage(r["stages"], B),
        "round_trip_err": r["round_trip_err"],
    }
    print(f"[bench] B={B}: {value:.1f} fwd+inv/s, round trip {r['round_trip_err']:.2e}", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(B, r["c_host"])
    else:
        out["cpu_baseline"] = None

    if not args.no_b512:
        print("[bench] B=512 leg", file=sys.stderr, flush=True)
        r5 = run_gpu(512, args.b512_steps, 1, seed=3)
        out["b512"] = {"value": round(args.b512_steps / r5["elapsed"], 3), "unit": "fwd+inv/s",
                       "ms_per_step": round(r5["elapsed"] / args.b512_steps * 1e3, 3),
                       "round_trip_err": r5["round_trip_err"], "roofline": roofline(r5["stages"], 512),
                       "stages": per_stage(r5["stages"], 512)}
        print(f"[bench] B=512: {out['b512']['value']} fwd+inv/s", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        out["copy_calibration_bytes"] = calibrate_copy()

    print(json.dumps(out))


if __name__ == "__main__":
    main()
