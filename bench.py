"""Benchmark: SO(3) FFT forward + inverse throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--B 128] [--quick]

A step is one inverse (coefficients -> grid) followed by one forward (grid ->
coefficients) of one function at bandwidth B in FP64: the whole hot path
(iDWT, two FFT passes, two FFT passes, DWT).  Inputs are seeded synthetic
band-limited coefficients (i.i.d. normal parts scaled by (1+l)^-1) already
resident in HBM when the timed region starts.

Printed: one JSON line with the throughput (fwd+inv per second) at B = 128 in
FP64, the roofline of the dominant kernel (HIP-event stage timers recorded
inside the library on the launch stream during the timed region), the
round-trip error, the oracle timed on the host cores, and the legs of the
metric: plain FP64 at B = 512, batched FP32-split at B = 128 and 512, and 256
functions of uneven bandwidth in FP64 / FP32 / FP32-split.  Every reduced-
precision leg reports its error against the FP64 path on the same inputs
(the FP64 path itself is held to 1e-11 / 1e-9 of the oracle by the parity
tests).
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
CSIZE = {"fp64": 16, "fp32": 8, "fp32_split": 8}


def num_coeffs(B):
    return B * (4 * B * B - 1) // 3


def stage_work(Bs, prec="fp64"):
    """Algorithmic bytes (FFT stages) or flops (DWT stages) of one step over
    functions of bandwidths Bs.

    FFT passes: every complex element read once and written once, with the
    +-B frequency row absent on the side where it is dropped.  DWT: 8B flops
    per coefficient for the contraction (complex x real over 2B beta samples,
    FMA = 2 flops) plus 5 flops per recurrence step per beta sample and
    symmetry group.
    """
    cs = CSIZE[prec]
    tot = {k: 0.0 for k in ("fft_gamma_fwd", "fft_alpha_fwd", "dwt_fwd", "dwt_inv", "fft_alpha_inv",
                            "fft_gamma_inv", "match_coeffs", "argmax")}
    for B in Bs:
        N, P = 2 * B, 2 * B - 1
        steps = sum((m + 1) * (B - 1 - m) for m in range(B))  # recurrence steps over groups m >= m' >= 0
        dwt = 8.0 * B * num_coeffs(B) + 5.0 * N * steps
        tot["fft_gamma_fwd"] += cs * (N ** 3 + N * N * (N - 1))
        tot["fft_alpha_fwd"] += cs * (N * N * (N - 1) + N * P * P)
        tot["dwt_fwd"] += dwt
        tot["dwt_inv"] += dwt
        tot["fft_alpha_inv"] += cs * (N * P * P + N * N * (N - 1))
        tot["fft_gamma_inv"] += cs * (N * N * (N - 1) + N ** 3)
        tot["match_coeffs"] += cs * (num_coeffs(B) + 2 * B * B)  # write f°, read a and b
        tot["argmax"] += cs * N ** 3                              # read the grid
    return {k: ("flop" if k.startswith("dwt") else "hbm", v) for k, v in tot.items()}


def source_digest(kind):
    """Hash of a kernel's source file and the shared header it includes."""
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES[kind], "soft_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1808_00896_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


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


def roofline(stage_ms, B):
    """Roofline of the slowest kernel of a one-function FP64 plan (one launch
    per stage per step)."""
    work = stage_work([B])
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
        r = {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 2),
             "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4)}
    r["avg_launch_ms"] = round(avg[dom], 5)
    r["algorithmic_per_launch"] = amount
    r["traffic"] = measured_traffic(dom, B)
    return r


def per_stage(stage_ms, Bs, steps, prec="fp64"):
    """Per stage: ms per step (all launches of the stage) and the algorithmic rate."""
    work = stage_work(Bs, prec)
    out = {}
    for k, (ms, n) in stage_ms.items():
        if not n:
            continue
        a = ms / steps
        kind, amount = work[k]
        rate = amount / (a * 1e-3)
        out[k] = {"ms": round(a, 5), "launches_per_step": n // steps}
        if kind == "hbm":
            out[k]["GB/s"] = round(rate / 1e9, 1)
        else:
            out[k]["TFLOP/s"] = round(rate / 1e12, 2)
    return out


TUNE = True  # plans time their DWT launch shapes at creation (outside the timed region)


def make_plan(Bs, prec, uniform, inplace=False):
    from paper_1808_00896_amd import soft
    if uniform:
        return soft.Plan(Bs[0], batch=len(Bs), precision=prec, tune=TUNE, inplace_ok=inplace)
    return soft.UnevenPlan(Bs, precision=prec, tune=TUNE, inplace_ok=inplace)


def shapes_of(plan):
    return [{"max_2B": l["max_2B"], "forward": l["forward"], "inverse": l["inverse"], "tuned": l["tuned"]}
            for l in plan.describe()["dwt_launches"]]


def percentiles(ms):
    q = np.percentile(np.asarray(ms), [10, 50, 90])
    return {"p10": round(float(q[0]), 4), "median": round(float(q[1]), 4), "p90": round(float(q[2]), 4)}


def timed_steps(plan, c, steps, warmup):
    """Run warmup steps, a short pass with every stage timed (the per-stage
    breakdown, and the slowest kernel), then `steps` timed steps of inverse
    then forward in which only the slowest kernel carries stage events (its
    launch durations for the roofline), so the timed region is perturbed as
    little as possible.  Returns (seconds, breakdown, breakdown steps, the
    slowest kernel's timers from the timed region, grid, round-tripped
    coefficients, per-step ms from HIP events recorded between the steps)."""
    import torch
    from paper_1808_00896_amd import soft
    grid = torch.empty(plan.grid_shape(), dtype=plan.dtype, device="cuda")
    c2 = torch.empty_like(c)

    def step():
        plan.inverse(c, out=grid)
        plan.forward(grid, out=c2)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    soft.soft_plan_stage_times(plan.handle, reset=True)
    soft.soft_plan_set_timing(plan.handle, True)
    kcal = max(3, min(steps, 10))
    for _ in range(kcal):
        step()
    breakdown = soft.soft_plan_stage_times(plan.handle, reset=True)
    avg = {k: ms / n for k, (ms, n) in breakdown.items() if n}
    slowest = max(avg, key=avg.get)
    soft.soft_plan_set_timing_stages(plan.handle, [slowest])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    soft.soft_plan_set_timing(plan.handle, False)
    st = soft.soft_plan_stage_times(plan.handle, reset=True)
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return t1 - t0, breakdown, kcal, {slowest: st[slowest]}, grid, c2, step_ms


def relerr_dev(a, b, chunk=1 << 27):
    """max |a - b| / max |b| over two device tensors of equal size, in FP64,
    chunk by chunk (the grids reach tens of GB)."""
    import torch
    a, b = a.reshape(-1), b.reshape(-1)
    num = den = 0.0
    for s in range(0, b.numel(), chunk):
        x = a[s:s + chunk].to(torch.complex128)
        y = b[s:s + chunk].to(torch.complex128)
        num = max(num, float((x - y).abs().max()))
        den = max(den, float(y.abs().max()))
    return num / den


def run_leg(Bs, prec, steps, warmup, c_host, uniform=True, ref=None, keep_ref=False, inplace=False):
    """Time `steps` fwd+inv of the functions Bs in precision prec.

    ref: dict with the FP64 path's grid and coefficients on the same inputs
    (flat or batched like this plan), for the error report.  keep_ref returns
    this leg's own grid for use as such a reference.  inplace: a
    SOFT_INPLACE_OK plan (its forward overwrites the grid it reads).
    """
    import torch
    plan = make_plan(Bs, prec, uniform, inplace)
    dt = plan.dtype
    c = torch.from_numpy(c_host).to("cuda").to(dt).reshape(plan.coeff_shape())
    el, st, kcal, st_slow, grid, c2, step_ms = timed_steps(plan, c, steps, warmup)
    if inplace:
        plan.inverse(c, out=grid)  # the timed forward overwrote it
    n = len(Bs)
    res = {"functions": n, "precision": prec, "steps": steps,
           "value": round(steps * n / el, 3), "unit": "function fwd+inv/s",
           "ms_per_step": round(el / steps * 1e3, 4),
           "step_ms": percentiles(step_ms),
           "workspace_bytes": plan.workspace_bytes(),
           "round_trip_err": relerr_dev(c2, c),
           "stages": per_stage(st, Bs, kcal, prec),
           "stages_from": f"{kcal} steps with every stage timed, before the timed region",
           "slowest_in_timed_region": {k: {"ms_total": ms, "launches": n} for k, (ms, n) in st_slow.items()},
           "dwt_shapes": shapes_of(plan)}
    out = None
    if ref is not None:
        res["inverse_err_vs_fp64"] = relerr_dev(grid, ref["grid"])
        # forward of the FP64 path's grid, rounded to this precision
        g_in = ref["grid"].to(dt).reshape(plan.grid_shape())
        if inplace:
            g_in = g_in.clone()  # the forward overwrites its input
        plan.forward(g_in, out=c2)
        del g_in
        res["forward_err_vs_fp64"] = relerr_dev(c2, ref["coeffs"])
    if keep_ref:
        # this leg's grid and the forward of it (the last timed step's output)
        out = {"grid": grid.reshape(-1), "coeffs": c2.reshape(-1)}
    plan.close()
    del c, c2, grid
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return res, out


def match_leg(steps, B=128, n=64):
    """Rotational matching of 64 pairs at B = 128: correlation coefficients,
    inverse transform to 64 grids of 256^3, argmax of each.  FP32-split timed;
    the FP64 path run once for the argmax agreement and the grid error.  Each
    precision also times the head without grids (argmax fused into the last
    FFT pass), which must give the same indices."""
    import torch
    from paper_1808_00896_amd import inputs, soft
    a_h, b_h = inputs.sh_pair_batch(n, B, seed=6)
    legs = {}
    ref = None
    for prec in ("fp64", "fp32_split"):
        log(f"match {n} pairs B={B} {prec}")
        m = soft.MatchPlan(B, n, precision=prec, tune=TUNE)
        a = torch.from_numpy(a_h).cuda().to(m.dtype)
        b = torch.from_numpy(b_h).cuda().to(m.dtype)
        grid = torch.empty(m.plan.grid_shape(), dtype=m.dtype, device="cuda")
        idx = torch.empty(n, dtype=torch.int64, device="cuda")
        k = steps if prec == "fp32_split" else 2
        for _ in range(2):
            m.match(a, b, grid, idx)
        torch.cuda.synchronize()
        h = m.plan.handle
        # per-stage breakdown from two calls with every stage timed, then the
        # timed calls without stage events
        soft.soft_plan_stage_times(h, reset=True)
        soft.soft_plan_set_timing(h, True)
        kcal = 2
        for _ in range(kcal):
            m.match(a, b, grid, idx)
        soft.soft_plan_set_timing(h, False)
        st = soft.soft_plan_stage_times(h, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            m.match(a, b, grid, idx)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        r = {"pairs": n, "B": B, "precision": prec, "steps": k, "value": round(n * k / el, 2),
             "unit": "pairs/s (coefficients + inverse + argmax)", "ms_per_step": round(el / k * 1e3, 3),
             "stages": per_stage(st, [B] * n, kcal, prec), "dwt_shapes": shapes_of(m.plan)}
        if ref is None:
            ref = {"grid": grid, "idx": idx.cpu().numpy()}
        else:
            ix = idx.cpu().numpy()
            r["argmax_agree_with_fp64"] = int((ix == ref["idx"]).sum())
            near = 0
            g64 = ref["grid"].reshape(n, -1)
            for f in np.flatnonzero(ix != ref["idx"]):
                g = g64[f]
                gap = float(g[int(ref["idx"][f])].real - g[int(ix[f])].real)
                near += gap <= 2e-6 * float(g.abs().max())
            r["argmax_near_ties"] = int(near)
            r["grid_err_vs_fp64"] = relerr_dev(grid, ref["grid"])
            r["speedup_vs_fp64"] = round(r["value"] / legs[f"match{n}_B{B}_fp64"]["value"], 3)
            del ref
        legs[f"match{n}_B{B}_{prec}"] = r
        # the same head without grids: the argmax fused into the last FFT pass
        idx2 = torch.empty_like(idx)
        k2 = steps if prec == "fp32_split" else 5
        for _ in range(2):
            m.match_index(a, b, idx2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k2):
            m.match_index(a, b, idx2)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t0
        legs[f"match{n}_B{B}_{prec}_index"] = {
            "pairs": n, "B": B, "precision": prec, "steps": k2, "value": round(n * k2 / el2, 2),
            "unit": "pairs/s (coefficients + inverse with the argmax fused into its last pass, no grids)",
            "ms_per_step": round(el2 / k2 * 1e3, 3), "same_index_as_grid_path": bool(torch.equal(idx2, idx)),
            "speedup_vs_grid_path": round(n * k2 / el2 / r["value"], 3)}
        m.close()
        del a, b, grid
        torch.cuda.empty_cache()
    return legs


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gpu_fwd_inv_ms(B, reps):
    """FP64 GPU inverse and forward ms at bandwidth B (library stage timers)."""
    import torch
    from paper_1808_00896_amd import inputs, soft
    with soft.Plan(B, tune=TUNE) as p:
        c = torch.from_numpy(inputs.coeffs_decay(B, 1)).cuda()
        g = p.inverse(c)
        c2 = p.forward(g)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ti = tf = 0.0
        for _ in range(reps):
            s.record(); p.inverse(c, out=g); e.record(); e.synchronize(); ti += s.elapsed_time(e)
            s.record(); p.forward(g, out=c2); e.record(); e.synchronize(); tf += s.elapsed_time(e)
        del c, g, c2
    torch.cuda.empty_cache()
    return ti / reps, tf / reps


def oracle_leg(B, what):
    """Seconds of one oracle call at bandwidth B (run in a child process, so
    OMP_NUM_THREADS applies).  what: "inverse", "forward" or "inverse_slices"
    (the full inverse computed slice by slice, printing progress)."""
    from oracle import oracle as O
    from paper_1808_00896_amd import inputs
    c = inputs.coeffs_decay(B, 1)
    if what == "inverse_slices":
        t = 0.0
        N = 2 * B
        for j in range(N):
            t0 = time.perf_counter()
            O.inverse_slice(B, c, j)
            t += time.perf_counter() - t0
            if (j + 1) % max(1, N // 16) == 0:
                log(f"oracle inverse B={B}: {j + 1}/{N} slices, {t:.1f} s")
        return t
    if what == "forward":
        g = inputs.grid_random(B, 1)
        t0 = time.perf_counter()
        O.forward(B, g)
        return time.perf_counter() - t0
    t0 = time.perf_counter()
    O.inverse(B, c)
    return time.perf_counter() - t0


def oracle_table(Bs_all, Bs_single, slices_B):
    """The FP64 oracle's seconds per inverse and forward at several B, on all
    host threads and on one, beside the GPU's milliseconds for the same calls."""
    import subprocess
    rows = []

    def child(B, what, threads):
        env = dict(os.environ)
        if threads:
            env["OMP_NUM_THREADS"] = str(threads)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-leg", f"{B}:{what}"],
                           env=env, capture_output=True, text=True)
        sys.stderr.write(r.stderr)
        if r.returncode != 0:
            raise RuntimeError(f"oracle leg B={B} {what} failed")
        return json.loads(r.stdout.strip().splitlines()[-1])

    for B in sorted(set(Bs_all) | set(Bs_single) | {slices_B} - {None}):
        gi, gf = gpu_fwd_inv_ms(B, 5 if B >= 256 else 20)
        row = {"B": B, "gpu_inverse_ms": round(gi, 4), "gpu_forward_ms": round(gf, 4)}
        if B in Bs_all:
            for what in ("inverse", "forward"):
                r = child(B, what, None)
                row[f"oracle_{what}_s"] = round(r["seconds"], 3)
                row["threads"] = r["threads"]
                row[f"{what}_ratio"] = round(r["seconds"] * 1e3 / (gi if what == "inverse" else gf), 1)
        if B == slices_B:
            r = child(B, "inverse_slices", None)
            row["oracle_inverse_s"] = round(r["seconds"], 1)
            row["oracle_inverse_how"] = "slice by slice (every beta sample), summed"
            row["threads"] = r["threads"]
            row["inverse_ratio"] = round(r["seconds"] * 1e3 / gi, 1)
        if B in Bs_single:
            for what in ("inverse", "forward"):
                r = child(B, what, 1)
                row[f"oracle_{what}_s_1thread"] = round(r["seconds"], 3)
        log(f"oracle table: {row}")
        rows.append(row)
    return {"cpu": cpu_model(), "nproc": os.cpu_count(), "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "rows": rows}


def ceilings(copy_bytes):
    """What the chip sustains outside this library, for reading the roofline
    fractions: a plain device copy of `copy_bytes` (torch), and FP64 / FP32
    GEMMs of 8192^3 through the vendor BLAS (torch.matmul), best of several."""
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = 1e30
        for _ in range(reps):
            s.record()
            fn()
            e.record()
            e.synchronize()
            t = min(t, s.elapsed_time(e))
        return t

    n = copy_bytes // 16
    a = torch.zeros(n, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    ms = best(lambda: b.copy_(a), 10)
    out = {"copy_bytes": 2 * n * 16, "copy_GB/s": round(2 * n * 16 / ms / 1e6, 1)}
    del a, b
    k = 8192
    for name, dt in (("dgemm", torch.float64), ("sgemm", torch.float32)):
        x = torch.randn(k, k, dtype=dt, device="cuda")
        y = torch.randn(k, k, dtype=dt, device="cuda")
        ms = best(lambda: torch.matmul(x, y), 5)
        out[f"{name}_TFLOP/s"] = round(2 * k ** 3 / ms / 1e9, 1)
        del x, y
    torch.cuda.empty_cache()
    return out


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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--B", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="main B leg only (no B=512, batched or uneven legs)")
    ap.add_argument("--no-b512", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--b512-steps", type=int, default=5)
    ap.add_argument("--batch", type=int, default=16, help="functions per batched FP32-split call at B=128")
    ap.add_argument("--uneven-n", type=int, default=256)
    ap.add_argument("--uneven-steps", type=int, default=5)
    ap.add_argument("--no-match", action="store_true")
    ap.add_argument("--match-steps", type=int, default=10)
    ap.add_argument("--no-tune", action="store_true", help="fixed DWT launch shapes instead of tuned ones")
    ap.add_argument("--oracle-table", action="store_true",
                    help="time the FP64 oracle per direction at B = 16, 128, 256 (all threads; one thread "
                         "at 16 and 128) and the B = 512 inverse slice by slice, beside the GPU, instead of "
                         "the legs")
    ap.add_argument("--oracle-leg", help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device copy (byte-counter calibration under rocprofv3)")
    args = ap.parse_args()
    global TUNE
    TUNE = not args.no_tune
    if args.oracle_leg:
        from oracle import oracle as O
        b, what = args.oracle_leg.split(":")
        print(json.dumps({"seconds": oracle_leg(int(b), what), "threads": O.num_threads()}))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the transform is built and timed on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1808_00896_amd import inputs
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    B = args.B
    log(f"B={B} FP64 steps={args.steps} warmup={args.warmup}")
    c_host = inputs.coeffs_decay(B, 1)
    main_leg, ref128 = run_leg([B], "fp64", args.steps, args.warmup, c_host, keep_ref=True)
    # the roofline needs the per-launch stage times of the one-function plan
    value = main_leg["value"]
    st_ms = {k: (v["ms_total"], v["launches"]) for k, v in main_leg["slowest_in_timed_region"].items()}
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "fwd+inv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded N(0,1)*(1+l)^-1 complex coefficients (band-limited)",
        "config": {"workload": f"one FP64 inverse + forward SO(3) FFT at B={B} "
                               f"({2 * B}^3 complex128 grid, {num_coeffs(B)} coefficients)",
                   "B": B, "batch": 1, "precision": "fp64"},
        "roofline": roofline(st_ms, B),
        "stages": main_leg["stages"],
        "stages_from": main_leg["stages_from"],
        "dwt_shapes": main_leg["dwt_shapes"],
        "round_trip_err": main_leg["round_trip_err"],
        "step_ms": main_leg["step_ms"],
    }
    log(f"B={B}: {value:.1f} fwd+inv/s, round trip {main_leg['round_trip_err']:.2e}")

    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(B, c_host)
    else:
        out["cpu_baseline"] = None

    if args.oracle_table:
        out["oracle_table"] = oracle_table([16, 128, 256], [16, 128], 512)
        print(json.dumps(out))
        return

    legs = {}
    if not args.quick:
        # batched FP32-split at B=128: `batch` copies of the main input, so the
        # FP64 path's grid of the main leg is the reference of every function
        nb = args.batch
        cb = np.tile(c_host, nb)
        refb = {"grid": ref128["grid"].repeat(nb), "coeffs": ref128["coeffs"].repeat(nb)}
        for prec in ("fp64", "fp32", "fp32_split"):
            log(f"B={B} batch={nb} {prec}")
            r, _ = run_leg([B] * nb, prec, max(5, args.steps // 5), 2, cb, ref=None if prec == "fp64" else refb)
            legs[f"B{B}_batch{nb}_{prec}"] = r
        del refb
        legs[f"B{B}_batch{nb}_fp32_split"]["speedup_vs_fp64_single"] = round(
            legs[f"B{B}_batch{nb}_fp32_split"]["value"] / value, 3)
    del ref128
    torch.cuda.empty_cache()

    if not args.quick and not args.no_b512:
        log("B=512 FP64")
        c5 = inputs.coeffs_decay(512, 3)
        r5, ref5 = run_leg([512], "fp64", args.b512_steps, 1, c5, keep_ref=True)
        st5 = {k: (v["ms_total"], v["launches"]) for k, v in r5["slowest_in_timed_region"].items()}
        r5["roofline"] = roofline(st5, 512)
        legs["B512_fp64"] = r5
        log(f"B=512 FP64: {r5['value']} fwd+inv/s")
        for prec in ("fp32", "fp32_split"):
            log(f"B=512 {prec}")
            r, _ = run_leg([512], prec, args.b512_steps, 1, c5, ref=ref5)
            legs[f"B512_{prec}"] = r
        legs["B512_fp32_split"]["speedup_vs_fp64"] = round(legs["B512_fp32_split"]["value"] / r5["value"], 3)
        log("B=512 FP64, SOFT_INPLACE_OK plan")
        r, _ = run_leg([512], "fp64", args.b512_steps, 1, c5, ref=ref5, inplace=True)
        r["speedup_vs_fp64"] = round(r["value"] / r5["value"], 3)
        legs["B512_fp64_inplace"] = r
        del ref5
        torch.cuda.empty_cache()

    if not args.quick and not args.no_uneven:
        n = args.uneven_n
        Bs, cs = inputs.uneven_batch(n, [16, 32, 64, 128], seed=4)
        cu = np.concatenate(cs)
        del cs
        log(f"uneven: {n} functions, B in {{16,32,64,128}}, {cu.size} coefficients")
        ru, refu = run_leg(Bs, "fp64", args.uneven_steps, 1, cu, uniform=False, keep_ref=True)
        legs["uneven256_fp64"] = ru
        for prec in ("fp32", "fp32_split"):
            log(f"uneven {prec}")
            r, _ = run_leg(Bs, prec, args.uneven_steps, 1, cu, uniform=False, ref=refu)
            r["speedup_vs_fp64"] = round(r["value"] / ru["value"], 3)
            legs[f"uneven256_{prec}"] = r
        for k in list(legs):
            if k.startswith("uneven"):
                legs[k]["bandwidths"] = {str(b): Bs.count(b) for b in sorted(set(Bs))}
        del refu
        torch.cuda.empty_cache()

    if not args.quick and not args.no_match:
        legs.update(match_leg(args.match_steps))

    out["legs"] = legs
    if not args.quick:
        log("ceilings")
        out["ceilings"] = ceilings(16 * (2 * B) ** 3)
    if args.calibrate_copy:
        out["copy_calibration_bytes"] = calibrate_copy()

    print(json.dumps(out))


if __name__ == "__main__":
    main()
