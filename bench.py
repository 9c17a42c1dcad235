"""Benchmark: SO(3) FFT forward + inverse throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--B 128] [--quick]
                    [--only LEG] [--summarize-rocprof WORKLOAD]

A step is one inverse (coefficients -> grid) followed by one forward (grid ->
coefficients) of one function at bandwidth B in FP64: the whole hot path
(iDWT, two FFT passes, two FFT passes, DWT).  Inputs are seeded synthetic
band-limited coefficients (i.i.d. normal parts scaled by (1+l)^-1) already
resident in HBM when the timed region starts.

Printed: one JSON line with the throughput (fwd+inv per second) at B = 128 in
FP64, the roofline of the dominant kernel (HIP-event stage timers recorded
inside the library on the launch stream during the timed region), and the
legs of the metric and of the other workloads: B = 16 and B = 256 in FP64,
plain FP64 at B = 512, batched FP32 / FP32-split at B = 128 and 512, 256
functions of uneven bandwidth in FP64 / FP32 / FP32-split, and the
rotational-matching head.  Every leg carries its inverse and forward times
(measured separately), its own roofline, and its error against the FP64
oracle (max-norm, L2 and per degree), which the CPU-baseline leg computes
while it times the oracle: in full at B <= 128, on sampled beta slices and
order pairs at B = 256 and 512.

--summarize-rocprof WORKLOAD turns the rocprofv3 runs of one workload
(kernel trace, FETCH_SIZE and WRITE_SIZE counters, and shader counters of
the matrix cores and the LDS, under gpurun_out/prof/WORKLOAD/) into the
summaries under profiles/ and the per-launch HBM bytes in
profiles/traffic.json; PROFILE_RECIPE below gives the commands.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 (vector and matrix), published
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X FP32 matrix, published (dense)
METRIC = "SOFT fwd+inv/sec at B=128 & 512: FP64 plain vs batched FP32-split @ ≤1e-6 err"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {"fft": "fft.hip", "dwt": "dwt.hip"}
CSIZE = {"fp64": 16, "fp32": 8, "fp32_split": 8}
STAGES = ("fft_gamma_fwd", "fft_alpha_fwd", "dwt_fwd", "dwt_inv", "fft_alpha_inv", "fft_gamma_inv",
          "match_coeffs", "argmax")

# How the committed profiles are made (repository root on the GPU machine, TMPDIR=/tmp),
# for WORKLOAD one of the --only legs:
PROFILE_RECIPE = (
    "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof/{w}/trace -o run -- "
    "python bench.py --only {w} --steps 10 --warmup 2 --no-cpu-baseline",
    "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof/{w}/fetch -o run -- "
    "python bench.py --only {w} --steps 2 --warmup 1 --no-cpu-baseline --calibrate-copy",
    "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof/{w}/write -o run -- "
    "python bench.py --only {w} --steps 2 --warmup 1 --no-cpu-baseline --calibrate-copy",
    "rocprofv3 --pmc {sq} --output-format csv -d gpurun_out/prof/{w}/sq -o run -- "
    "python bench.py --only {w} --steps 2 --warmup 1 --no-cpu-baseline",
    "python bench.py --summarize-rocprof {w}",
)

# Shader counters of the fourth pass (at most 8 SQ and 2 GRBM counters in one
# pass): the matrix-core instructions and their operations of the plan's
# precision (MOPS: units of 512 flop), the matrix cores' busy cycles, the
# LDS instructions and bank-conflict cycles, the FP64 vector FMAs (the
# recurrence) and the GPU's busy cycles.
SQ_COUNTERS = {
    "fp64": "SQ_INSTS_VALU_MFMA_F64 SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_FMA_F64 "
            "SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVE_CYCLES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE",
    "fp32": "SQ_INSTS_VALU_MFMA_F32 SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_BF16 "
            "SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_FMA_F64 SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_BUSY_CYCLES "
            "GRBM_GUI_ACTIVE",
}


def sq_counters_of(workload):
    return SQ_COUNTERS["fp64" if workload.startswith("fp64") else "fp32"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sig(x, d=3):
    """A float rounded to d significant digits (compact JSON)."""
    x = float(x)
    return float(f"{x:.{d}g}") if np.isfinite(x) else x


def num_coeffs(B):
    return B * (4 * B * B - 1) // 3


# ---------------------------------------------------------------------------
# Algorithmic work and rooflines
# ---------------------------------------------------------------------------

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
    tot = {k: 0.0 for k in STAGES}
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
    """Hash of a kernel's source file and the shared header it includes, with
    comments and whitespace runs dropped (an edit of the comments leaves the
    built kernels, and so the measured traffic, unchanged)."""
    h = hashlib.sha256()
    for name in (KERNEL_SOURCES[kind], "soft_internal.h"):
        text = open(os.path.join(ROOT, "paper_1808_00896_amd", "csrc", name)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, stage):
    """HBM bytes per launch of a stage from committed rocprofv3 counter runs
    of the workload, or None when absent or taken on a different version of
    the kernel source."""
    try:
        data = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    rec = data.get(workload, {}).get(stage)
    if not rec:
        return None
    kind = "fft" if stage.startswith("fft") else "dwt"
    if rec.get("source_sha") != source_digest(kind):
        return None
    return rec.get("bytes_per_launch")


def roofline(stage_ms, Bs, prec, workload=None):
    """Roofline of the dominant stage of a plan: its algorithmic work per
    launch (the stage's work per step over its launches per step) over its
    average launch duration.  stage_ms: {stage: (ms_total, launches)} from
    the library's HIP-event timers in the timed region, `steps` steps.
    FFT stages are bound by HBM; the DWT contractions by the FP64 matrix
    cores (FP64) or the FP32 matrix cores (FP32 modes, whose recurrence still
    runs in FP64 on the vector unit)."""
    work = stage_work(Bs, prec)
    timed = {k: v for k, v in stage_ms.items() if not k.startswith("_")}
    avg = {k: ms / n for k, (ms, n) in timed.items() if n}
    dom = max(avg, key=avg.get)
    kind, step_amount = work[dom]
    ms_total, launches = stage_ms[dom]
    steps = stage_ms.get("_steps", None)
    per_step = launches // steps if steps else 1
    amount = step_amount / max(1, per_step)
    t = avg[dom] * 1e-3
    if kind == "hbm":
        achieved = amount / t / 1e9
        r = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}
    else:
        peak = FP64_PEAK_TFLOPS if prec == "fp64" else FP32_MFMA_PEAK_TFLOPS
        achieved = amount / t / 1e12
        r = {"kernel": dom, "bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
             "unit": "TFLOP/s", "frac": round(achieved / peak, 4)}
    r["avg_launch_ms"] = round(avg[dom], 5)
    r["launches_per_step"] = per_step
    r["algorithmic_per_launch"] = amount
    r["traffic"] = measured_traffic(workload, dom) if workload else None
    return r


def per_stage(stage_ms, Bs, steps, prec="fp64"):
    """Per stage: ms per step (all launches of the stage) and the algorithmic rate."""
    work = stage_work(Bs, prec)
    out = {}
    for k, (ms, n) in stage_ms.items():
        if not n or k.startswith("_"):
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


# ---------------------------------------------------------------------------
# Timed legs
# ---------------------------------------------------------------------------

DEV = "cuda"  # device of every tensor the legs allocate
# Bandwidths of the legs besides the headline one: the round trip of one
# small function, the mid-size and the large single transforms, the set the
# uneven batch draws from.
SMALL_B, MID_B, BIG_B = 16, 256, 512
UNEVEN_SET = (16, 32, 64, 128)
TUNE = True  # plans time their DWT launch shapes at creation (outside the timed region)


def make_plan(Bs, prec, uniform, inplace=False, graph=False, dd=False):
    from paper_1808_00896_amd import soft
    if uniform:
        return soft.Plan(Bs[0], batch=len(Bs), precision=prec, tune=TUNE, inplace_ok=inplace, graph=graph, dd=dd)
    return soft.UnevenPlan(Bs, precision=prec, tune=TUNE, inplace_ok=inplace, graph=graph, dd=dd)


def workload_key(Bs, prec, uniform):
    return f"{prec}_B{Bs[0]}_n{len(Bs)}" if uniform else f"{prec}_uneven{len(Bs)}"


def shapes_of(plan):
    return [{"max_2B": l["max_2B"], "forward": l["forward"], "inverse": l["inverse"], "tuned": l["tuned"]}
            for l in plan.describe()["dwt_launches"]]


def percentiles(ms):
    q = np.percentile(np.asarray(ms), [10, 50, 90])
    return {"p10": round(float(q[0]), 4), "median": round(float(q[1]), 4), "p90": round(float(q[2]), 4)}


def timed_steps(plan, c, steps, warmup, fwd_in=None):
    """Run warmup steps, a short pass with every stage timed (the per-stage
    breakdown, and the slowest kernel), then `steps` timed steps of inverse
    then forward in which only the slowest kernel carries stage events (its
    launch durations for the roofline), so the timed region is perturbed as
    little as possible; the host clock around them (after a synchronize on
    both sides) gives the throughput.  A second, shorter pass with HIP events
    on the launch stream between the calls gives the inverse and forward
    times of each step (their percentiles).  The forward reads the inverse's
    output grid, or fwd_in when given (a SOFT_INPLACE_OK plan's forward
    overwrites it).  Returns a dict."""
    import torch
    from paper_1808_00896_amd import soft
    grid = torch.empty(plan.grid_shape(), dtype=plan.dtype, device=DEV)
    c2 = torch.empty_like(c)
    src = grid if fwd_in is None else fwd_in

    def step():
        plan.inverse(c, out=grid)
        plan.forward(src, out=c2)

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
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    soft.soft_plan_set_timing(plan.handle, False)
    st = soft.soft_plan_stage_times(plan.handle, reset=True)
    # the inverse / forward split, from events between the calls
    nsplit = max(1, min(steps, 50))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nsplit + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i in range(nsplit):
        plan.inverse(c, out=grid)
        ev[2 * i + 1].record()
        plan.forward(src, out=c2)
        ev[2 * i + 2].record()
    torch.cuda.synchronize()
    inv_ms = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(nsplit)]
    fwd_ms = [ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) for i in range(nsplit)]
    step_ms = [a + b for a, b in zip(inv_ms, fwd_ms)]
    slow = dict(st)
    slow = {slowest: slow[slowest], "_steps": steps}
    return {"seconds": t1 - t0, "breakdown": breakdown, "kcal": kcal, "slowest": slow, "grid": grid, "c2": c2,
            "step_ms": step_ms, "inv_ms": inv_ms, "fwd_ms": fwd_ms, "nsplit": nsplit}


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


def run_leg(Bs, prec, steps, warmup, c_host, uniform=True, fwd_grid=None, inplace=False, graph=False,
            fwd_sample=None, dd=False):
    """Time `steps` fwd+inv of the functions Bs in precision prec.

    c_host: coefficients (complex128, flat), rounded to the plan's precision
    on the device.  fwd_grid: a device grid (flat, any complex type) that the
    forward reads instead of the inverse's output (rounded to this precision),
    so that reduced-precision legs transform the FP64 path's grid.  inplace:
    a SOFT_INPLACE_OK plan (its forward overwrites the grid it reads, so the
    forward then reads a copy).  graph: a SOFT_PLAN_GRAPH plan (each call a
    replay of its captured kernels; the per-stage pass before the timed
    region runs eagerly, since stage timing needs events between kernels).
    fwd_sample: a device grid (flat) of seeded input for the accuracy report:
    after the timed region the plan's forward reads it (rounded to this
    precision), untimed.  dd: a SOFT_DD_RECURRENCE plan (the double-double
    recurrence; its workload key, and so its traffic record, is its own).
    Returns (record, outputs): outputs holds the device tensors grid, c2
    (flat), fwd_in (flat), the plan offsets and, with fwd_sample, sample_in
    (what the forward read) and sample_out (its coefficients).
    """
    import torch
    plan = make_plan(Bs, prec, uniform, inplace, graph, dd)
    dt = plan.dtype
    c = torch.from_numpy(c_host).to(DEV).to(dt).reshape(plan.coeff_shape())
    fwd_in = None if fwd_grid is None else fwd_grid.to(dt).reshape(plan.grid_shape())
    r = timed_steps(plan, c, steps, warmup, fwd_in=fwd_in)
    if inplace and fwd_grid is None:
        # the timed forwards overwrote the inverse's output: make it again,
        # and the forward of a copy of it, for the error report
        plan.inverse(c, out=r["grid"])
        plan.forward(r["grid"].clone(), out=r["c2"])
    n = len(Bs)
    key = workload_key(Bs, prec, uniform) + ("_dd" if dd else "")
    res = {"functions": n, "precision": prec, "steps": steps, "dd_recurrence": bool(dd),
           "value": round(steps * n / r["seconds"], 3), "unit": "function fwd+inv/s",
           "ms_per_step": round(r["seconds"] / steps * 1e3, 4),
           "step_ms": percentiles(r["step_ms"]),
           "inverse_ms": percentiles(r["inv_ms"]),
           "forward_ms": percentiles(r["fwd_ms"]),
           "workspace_bytes": plan.workspace_bytes(),
           "stages": per_stage(r["breakdown"], Bs, r["kcal"], prec),
           "stages_from": f"{r['kcal']} steps with every stage timed, before the timed region",
           "roofline": roofline(r["slowest"], Bs, prec, key),
           "dwt_shapes": shapes_of(plan), "graph": bool(graph)}
    if fwd_grid is None and not inplace:
        res["round_trip_err"] = relerr_dev(r["c2"], c)
    offs = plan.grid_offsets if hasattr(plan, "grid_offsets") else None
    coffs = plan.coeff_offsets if hasattr(plan, "coeff_offsets") else None
    out = {"grid": r["grid"].reshape(-1), "c2": r["c2"].reshape(-1),
           "fwd_in": (r["grid"] if fwd_in is None else fwd_in).reshape(-1),
           "grid_offsets": offs, "coeff_offsets": coffs}
    if fwd_sample is not None:
        out["sample_in"] = fwd_sample.to(dt).reshape(-1)
        # a SOFT_INPLACE_OK forward overwrites what it reads: give it a copy
        src = out["sample_in"].clone() if inplace else out["sample_in"]
        out["sample_out"] = plan.forward(src.reshape(plan.grid_shape())).reshape(-1)
    plan.close()
    del c
    return res, out


def host(t):
    """A device tensor as a host complex128 numpy array."""
    import torch
    return t.to(torch.complex128).cpu().numpy()


# Accuracy samples gathered by the legs, scored against the oracle by the
# CPU-baseline leg: leg name -> list of dicts.
SAMPLES = {}


def add_full_sample(leg, B, c_in, grid_gpu, fwd_in, c_gpu, oracle_prec="f64"):
    """A whole function: the inverse of c_in and the forward of fwd_in (a
    seeded input grid, host complex128, exactly what the GPU read) against the
    oracle in full; FP64 legs use the long-double oracle ("f80"), whose own
    error is far below theirs (the double oracle's forward of a random grid
    errs by about 1.7e-13 at B = 128)."""
    SAMPLES.setdefault(leg, []).append({"kind": "full", "B": B, "c_in": c_in, "grid_gpu": grid_gpu,
                                        "fwd_in": fwd_in, "c_gpu": c_gpu, "prec": oracle_prec})


def coeff_indices(B, pairs):
    """Flat indices [npairs, B] of f°(l, m, m') for l < B (clamped to the
    pair's lowest degree below it; those entries are ignored)."""
    idx = np.zeros((len(pairs), B), dtype=np.int64)
    for p, (m, mp) in enumerate(pairs):
        l0 = max(abs(m), abs(mp))
        for l in range(B):
            ll = max(l, l0)
            idx[p, l] = ll * (4 * ll * ll - 1) // 3 + (m + ll) * (2 * ll + 1) + (mp + ll)
    return idx


def sample_pairs(B):
    """Order pairs sampled at large B: low, high and mixed orders and signs."""
    h = B // 2
    return [(0, 0), (1, -1), (h, h // 3), (-(B - 1), h), (B - 1, B - 1), (-7, B - 2)]


def sample_slices(B):
    return [0, (2 * B) // 3, 2 * B - 1]


def add_sampled(leg, B, c_in, grid_dev, c2_dev, fwd_in_tag, oracle_prec="f64", slices=None, pairs=None):
    """Sampled at large B: beta slices of the GPU inverse and order pairs of
    the GPU forward of a seeded input grid (HOST_GRIDS[fwd_in_tag], which the
    oracle reads); oracle_prec "f80" scores the slices against the
    long-double oracle (the pairs stay with the double one: a long-double
    forward_pairs at B = 512 takes about half a minute per pair)."""
    import torch
    N = 2 * B
    g = grid_dev.reshape(N, N, N)
    slices = {j: host(g[:, j, :]) for j in (sample_slices(B) if slices is None else slices)}
    pairs = sample_pairs(B) if pairs is None else pairs
    idx = torch.from_numpy(coeff_indices(B, pairs).reshape(-1)).to(c2_dev.device)
    cg = host(c2_dev.reshape(-1)[idx]).reshape(len(pairs), B)
    SAMPLES.setdefault(leg, []).append({"kind": "sampled", "B": B, "c_in": c_in, "slices": slices,
                                        "pairs": pairs, "c_pairs": cg, "fwd_in": fwd_in_tag,
                                        "prec": oracle_prec})


HOST_GRIDS = {}


def err_report(x, ref, B=None):
    """max |x - ref| / max |ref|, ||x - ref|| / ||ref||, and for an l-major
    coefficient vector of bandwidth B the per-degree max |dx(l)| / max |ref(l)|."""
    x = np.asarray(x, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    d = np.abs(x - ref)
    a = np.abs(ref)
    r = {"max_rel": sig(d.max() / a.max()), "l2_rel": sig(np.linalg.norm(x - ref) / np.linalg.norm(ref))}
    if B is not None:
        st = np.array([l * (4 * l * l - 1) // 3 for l in range(B)])
        dl = np.maximum.reduceat(d, st) / np.maximum.reduceat(a, st)
        r["deg_rel"] = [sig(v, 2) for v in dl]
        r["deg_rel_max"] = sig(dl.max())
    return r


def pairs_report(x, ref, pairs):
    """The same over sampled order pairs: rows [npairs, B], entries below a
    pair's lowest degree ignored; deg_rel[l] over the pairs present at l."""
    B = ref.shape[1]
    mask = np.zeros(ref.shape, dtype=bool)
    for p, (m, mp) in enumerate(pairs):
        mask[p, max(abs(m), abs(mp)):] = True
    d = np.where(mask, np.abs(x - ref), 0.0)
    a = np.where(mask, np.abs(ref), 0.0)
    xs, rs = x[mask], ref[mask]
    dl = d.max(axis=0) / np.maximum(a.max(axis=0), 1e-300)
    return {"max_rel": sig(d.max() / a.max()), "l2_rel": sig(np.linalg.norm(xs - rs) / np.linalg.norm(rs)),
            "deg_rel": [sig(v, 2) for v in dl], "deg_rel_max": sig(dl.max()),
            "sampled": f"{len(pairs)} order pairs, all degrees"}


def fingerprint(B, a):
    """Cache key of an input array: B, its shape and a hash of a strided subset."""
    sub = np.ascontiguousarray(np.asarray(a).reshape(-1)[::997])
    return (B, a.shape, hashlib.sha1(sub.view(np.uint8)).hexdigest())


def score_samples(O, cache):
    """Every leg's samples against the FP64 oracle (a few oracle calls per
    input, shared between legs with the same input)."""

    def memo(key, fn):
        if key not in cache:
            cache[key] = fn()
        return cache[key]

    ckey = fingerprint

    out = {}
    for leg, samples in SAMPLES.items():
        rep = []
        for s in samples:
            B = s["B"]
            kc = ckey(B, s["c_in"])
            op = s.get("prec", "f64")
            if s["kind"] == "full":
                gi = memo(("inv", op) + kc, lambda: O.inverse(B, s["c_in"], op))
                cf = memo(("fwd", op) + ckey(B, s["fwd_in"]), lambda: O.forward(B, s["fwd_in"], op))
                inv, fwd = err_report(s["grid_gpu"], gi), err_report(s["c_gpu"], cf, B)
                inv["oracle"] = fwd["oracle"] = op
                rep.append({"B": B, "inverse": inv, "forward": fwd})
            else:
                inv = {}
                worst = {"max_rel": 0.0, "l2_num": 0.0, "l2_den": 0.0}
                for j, sl in s["slices"].items():
                    want = memo(("slice", j, op) + kc, lambda: O.inverse_slice(B, s["c_in"], j, op))
                    e = np.abs(sl - want)
                    worst["max_rel"] = max(worst["max_rel"], e.max() / np.abs(want).max())
                    worst["l2_num"] += float(np.sum(e ** 2))
                    worst["l2_den"] += float(np.sum(np.abs(want) ** 2))
                inv = {"max_rel": sig(worst["max_rel"]), "l2_rel": sig(np.sqrt(worst["l2_num"] / worst["l2_den"])),
                       "sampled": f"beta slices {sorted(s['slices'])} (each max-normed)", "oracle": op}
                g = HOST_GRIDS[s["fwd_in"]]
                want = memo(("pairs", s["fwd_in"], tuple(s["pairs"])),
                            lambda: O.forward_pairs(B, g, s["pairs"]))
                fwd = pairs_report(s["c_pairs"], want, s["pairs"])
                fwd["oracle"] = "f64"
                rep.append({"B": B, "inverse": inv, "forward": fwd})
        out[leg] = rep
    return out


# ---------------------------------------------------------------------------
# Legs of the metric
# ---------------------------------------------------------------------------

def sample_grid(B):
    """The seeded random grid whose forward a leg of bandwidth B reports
    against the oracle (on the device, complex128, flat)."""
    import torch
    from paper_1808_00896_amd import inputs
    return torch.from_numpy(inputs.grid_random(B, 700 + B).reshape(-1)).to(DEV)


def leg_single(B, prec, steps, warmup, c_host, name, legs, sampled=False, grid_tag=None):
    """One function of bandwidth B: timed, then its accuracy sample (the
    inverse of c_host and the forward of a seeded random grid; sampled:
    grid_tag names that grid, as read, in HOST_GRIDS)."""
    log(f"{name}: B={B} {prec} steps={steps}")
    res, out = run_leg([B], prec, steps, warmup, c_host, fwd_sample=sample_grid(B))
    legs[name] = res
    c_in = c_host.astype(np.complex64).astype(np.complex128) if prec != "fp64" else c_host
    fin = host(out.pop("sample_in")).reshape((2 * B,) * 3)
    op = "f80" if prec == "fp64" else "f64"
    if sampled:
        HOST_GRIDS[grid_tag] = fin
        add_sampled(name, B, c_in, out["grid"], out["sample_out"], grid_tag, oracle_prec=op)
    else:
        add_full_sample(name, B, c_in, host(out["grid"]), fin, host(out["sample_out"]), oracle_prec=op)
    return res, out


def main_legs(args, legs):
    """The FP64 single-function legs: B = 16 (round trip), B = 128 (the
    headline), B = 256; forward and inverse timed separately in each."""
    from paper_1808_00896_amd import inputs
    B = args.B
    c_host = inputs.coeffs_decay(B, 1)
    main, out = leg_single(B, "fp64", args.steps, args.warmup, c_host, f"B{B}_fp64", legs)
    main_grid = out["grid"]
    if args.quick:
        return main, main_grid, c_host
    c16 = inputs.coeffs_uniform(SMALL_B, 0)
    leg_single(SMALL_B, "fp64", max(20, args.steps), args.warmup, c16, f"B{SMALL_B}_fp64", legs)
    # the same calls replayed as captured HIP graphs (SOFT_PLAN_GRAPH)
    log(f"B{SMALL_B}_fp64_graph")
    r, _ = run_leg([SMALL_B], "fp64", max(20, args.steps), args.warmup, c16, graph=True)
    r["speedup_vs_eager"] = round(r["value"] / legs[f"B{SMALL_B}_fp64"]["value"], 3)
    legs[f"B{SMALL_B}_fp64_graph"] = r
    c256 = inputs.coeffs_decay(MID_B, 2)
    leg_single(MID_B, "fp64", max(10, args.steps // 5), 2, c256, f"B{MID_B}_fp64", legs, sampled=True,
               grid_tag=f"B{MID_B}_fp64_sample")
    return main, main_grid, c_host


def batch_legs(args, legs, B, c_host, main_grid):
    """`batch` copies of the headline input at B = 128 in FP64, FP32 and
    FP32-split; the reduced-precision forwards read the FP64 path's grid."""
    import torch
    nb = args.batch
    cb = np.tile(c_host, nb)
    gb = main_grid.repeat(nb)
    gs = sample_grid(B).repeat(nb)  # every function's forward sample reads the same seeded grid
    for prec in ("fp64", "fp32", "fp32_split"):
        name = f"B{B}_batch{nb}_{prec}"
        log(f"{name}")
        res, out = run_leg([B] * nb, prec, max(5, args.steps // 5), 2, cb,
                           fwd_grid=None if prec == "fp64" else gb, fwd_sample=gs)
        legs[name] = res
        rnd = (lambda a: a.astype(np.complex64).astype(np.complex128)) if prec != "fp64" else (lambda a: a)
        n3, nc = (2 * B) ** 3, num_coeffs(B)
        for f in (0, nb - 1):
            add_full_sample(name, B, rnd(c_host), host(out["grid"][f * n3:(f + 1) * n3]),
                            host(out["sample_in"][f * n3:(f + 1) * n3]).reshape((2 * B,) * 3),
                            host(out["sample_out"][f * nc:(f + 1) * nc]), oracle_prec="f80" if prec == "fp64" else "f64")
        del out
        torch.cuda.empty_cache()
    del gb, gs


def b512_legs(args, legs):
    """B = 512 in FP64, FP32, FP32-split and FP64 with SOFT_INPLACE_OK; the
    reduced-precision forwards read the FP64 path's grid."""
    import torch
    from paper_1808_00896_amd import inputs
    B = BIG_B
    c5 = inputs.coeffs_decay(B, 3)
    r5, out5 = leg_single(B, "fp64", args.b512_steps, 1, c5, f"B{B}_fp64", legs, sampled=True,
                          grid_tag=f"B{B}_fp64_sample")
    g64 = out5["grid"]
    del out5["sample_out"]
    HOST_GRIDS[f"B{B}_c64_sample"] = HOST_GRIDS[f"B{B}_fp64_sample"].astype(np.complex64).astype(np.complex128)
    c5r = c5.astype(np.complex64).astype(np.complex128)
    for prec in ("fp32", "fp32_split"):
        name = f"B{B}_{prec}"
        log(name)
        r, out = run_leg([B], prec, args.b512_steps, 1, c5, fwd_grid=g64, fwd_sample=sample_grid(B))
        r["inverse_err_vs_fp64_gpu"] = relerr_dev(out["grid"], g64)
        legs[name] = r
        add_sampled(name, B, c5r, out["grid"], out["sample_out"], f"B{B}_c64_sample")
        del out
        torch.cuda.empty_cache()
    for prec in ("fp32", "fp32_split"):
        legs[f"B{B}_{prec}"]["speedup_vs_fp64"] = round(legs[f"B{B}_{prec}"]["value"] / r5["value"], 3)
    log(f"B{B}_fp64_inplace")
    r, out = run_leg([B], "fp64", args.b512_steps, 1, c5, inplace=True)
    r["inverse_err_vs_fp64_gpu"] = relerr_dev(out["grid"], g64)
    r["forward_err_vs_fp64_gpu"] = relerr_dev(out["c2"], out5["c2"])
    r["speedup_vs_fp64"] = round(r["value"] / r5["value"], 3)
    legs[f"B{B}_fp64_inplace"] = r
    del out, out5, g64
    torch.cuda.empty_cache()
    # the double-double recurrence (SOFT_DD_RECURRENCE): the first and last
    # beta slices (where the FP64 recurrence errs most) against the
    # long-double oracle; the FP64 leg's order pairs of the same grid
    name = f"B{B}_fp64_dd"
    log(name)
    r, out = run_leg([B], "fp64", args.b512_steps, 1, c5, dd=True, fwd_sample=sample_grid(B))
    r["speedup_vs_fp64"] = round(r["value"] / r5["value"], 3)
    legs[name] = r
    add_sampled(name, B, c5, out["grid"], out["sample_out"], f"B{B}_fp64_sample", oracle_prec="f80",
                slices=[0, 2 * B - 1])
    del out
    torch.cuda.empty_cache()


def uneven_legs(args, legs):
    """256 functions of bandwidths drawn from {16, 32, 64, 128} in FP64, FP32
    and FP32-split; one function per bandwidth scored against the oracle."""
    import torch
    from paper_1808_00896_amd import inputs
    n = args.uneven_n
    Bs, cs = inputs.uneven_batch(n, list(UNEVEN_SET), seed=4)
    cu = np.concatenate(cs)
    log(f"uneven: {n} functions, B in {UNEVEN_SET}, {cu.size} coefficients")
    picks = [Bs.index(b) for b in sorted(set(Bs))]
    g64 = None
    # forward samples: a seeded random grid for each picked function, zeros elsewhere
    go0 = np.concatenate([[0], np.cumsum([(2 * b) ** 3 for b in Bs])])  # grids back to back
    gs = torch.zeros(int(go0[-1]), dtype=torch.complex128, device=DEV)
    for f in picks:
        gs[go0[f]:go0[f + 1]] = sample_grid(Bs[f])
    for prec in ("fp64", "fp32", "fp32_split"):
        name = f"uneven{n}_{prec}"
        log(name)
        r, out = run_leg(Bs, prec, args.uneven_steps, 1, cu, uniform=False, fwd_grid=g64, fwd_sample=gs)
        legs[name] = r
        go, co = out["grid_offsets"], out["coeff_offsets"]
        for f in picks:
            B = Bs[f]
            c_in = cs[f] if prec == "fp64" else cs[f].astype(np.complex64).astype(np.complex128)
            add_full_sample(name, B, c_in, host(out["grid"][go[f]:go[f + 1]]),
                            host(out["sample_in"][go[f]:go[f + 1]]).reshape((2 * B,) * 3),
                            host(out["sample_out"][co[f]:co[f + 1]]), oracle_prec="f80" if prec == "fp64" else "f64")
        if prec == "fp64":
            g64 = out["grid"].clone()
            ru = r
            del out
            # the same calls replayed as captured HIP graphs (SOFT_PLAN_GRAPH)
            log(f"{name}_graph")
            rg, out = run_leg(Bs, prec, args.uneven_steps, 1, cu, uniform=False, graph=True)
            rg["speedup_vs_eager"] = round(rg["value"] / ru["value"], 3)
            legs[f"{name}_graph"] = rg
        else:
            r["speedup_vs_fp64"] = round(r["value"] / ru["value"], 3)
        del out
        torch.cuda.empty_cache()
    for k in list(legs):
        if k.startswith("uneven"):
            legs[k]["bandwidths"] = {str(b): Bs.count(b) for b in sorted(set(Bs))}
    del g64, gs
    torch.cuda.empty_cache()


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
        a = torch.from_numpy(a_h).to(DEV).to(m.dtype)
        b = torch.from_numpy(b_h).to(DEV).to(m.dtype)
        grid = torch.empty(m.plan.grid_shape(), dtype=m.dtype, device=DEV)
        idx = torch.empty(n, dtype=torch.int64, device=DEV)
        k = steps if prec == "fp32_split" else 2
        for _ in range(2):
            m.match(a, b, grid, idx)
        torch.cuda.synchronize()
        h = m.plan.handle
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


# ---------------------------------------------------------------------------
# CPU baseline (the oracle) and the accuracy it scores
# ---------------------------------------------------------------------------

def cpu_baseline(B, budget_s=12.0, max_reps=3):
    """The FP64 oracle timed on the host cores on a bounded sample of the
    headline workload (inverse of the headline coefficients, forward of the
    headline leg's seeded sample grid, up to max_reps times); its results
    then score every leg's accuracy samples.  Returns (baseline record,
    accuracy record)."""
    from oracle import oracle as O
    main = SAMPLES.get(f"B{B}_fp64", [None])[0]
    reps, t = 0, 0.0
    cache = {}
    while reps < max_reps and (reps == 0 or t < budget_s):
        t0 = time.perf_counter()
        g = O.inverse(B, main["c_in"])
        c = O.forward(B, main["fwd_in"])
        t += time.perf_counter() - t0
        reps += 1
    cache[("inv", "f64") + fingerprint(B, main["c_in"])] = g
    cache[("fwd", "f64") + fingerprint(B, main["fwd_in"])] = c
    base = {"value": round(reps / t, 4), "unit": "fwd+inv/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{reps} x (inverse + forward) at B={B}, FP64 oracle (OpenMP): the inverse of the headline "
                      f"coefficients and the forward of a seeded random grid", "seconds": round(t, 2)}
    t0 = time.perf_counter()
    acc = score_samples(O, cache)
    log(f"oracle scoring of {sum(len(v) for v in acc.values())} samples: {time.perf_counter() - t0:.1f} s")
    return base, acc


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gpu_fwd_inv_ms(B, reps):
    """FP64 GPU inverse and forward ms at bandwidth B (HIP events around each call)."""
    import torch
    from paper_1808_00896_amd import inputs, soft
    with soft.Plan(B, tune=TUNE) as p:
        c = torch.from_numpy(inputs.coeffs_decay(B, 1)).to(DEV)
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


# ---------------------------------------------------------------------------
# Ceilings: what the device sustains, with this library's own probe kernels
# ---------------------------------------------------------------------------

def ceilings(copy_bytes):
    """A streaming copy of `copy_bytes` and arithmetic loops on the FP64
    vector unit and the FP64 / FP32 matrix cores (soft_probe_*), best of
    several launches; vendor-BLAS GEMMs of 8192^3 beside them for context."""
    import torch
    from paper_1808_00896_amd import soft
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
    a = torch.zeros(n, dtype=torch.complex128, device=DEV)
    b = torch.empty_like(a)
    ms = best(lambda: soft.soft_probe_copy(a, b), 10)
    out = {"copy_bytes": n * 16, "stream_copy_GB/s": round(2 * n * 16 / ms / 1e6, 1),
           "stream_copy_frac_of_peak": round(2 * n * 16 / ms / 1e6 / HBM_PEAK_GBS, 4)}
    ms = best(lambda: b.copy_(a), 10)
    out["torch_copy_GB/s"] = round(2 * n * 16 / ms / 1e6, 1)
    del a, b
    blocks = 256 * 8
    sink = torch.zeros(blocks * 256, dtype=torch.float64, device=DEV)
    for kind, name, target in ((soft.PROBE_FMA64, "fp64_fma", 5e11), (soft.PROBE_MFMA64, "fp64_mfma", 5e11),
                               (soft.PROBE_MFMA32, "fp32_mfma", 1e12)):
        per_iter = soft.lib().soft_probe_flop_count(kind, blocks, 1)
        iters = max(1, int(target / per_iter))
        flops = soft.lib().soft_probe_flop_count(kind, blocks, iters)
        ms = best(lambda: soft.soft_probe_flops(kind, blocks, iters, sink), 5)
        out[f"{name}_TFLOP/s"] = round(flops / ms / 1e9, 1)
    peaks = {"fp64_fma": FP64_PEAK_TFLOPS, "fp64_mfma": FP64_PEAK_TFLOPS, "fp32_mfma": FP32_MFMA_PEAK_TFLOPS}
    for k, p in peaks.items():
        out[f"{k}_frac_of_peak"] = round(out[f"{k}_TFLOP/s"] / p, 4)
    del sink
    k = 8192
    for name, dt in (("vendor_dgemm", torch.float64), ("vendor_sgemm", torch.float32)):
        x = torch.randn(k, k, dtype=dt, device=DEV)
        y = torch.randn(k, k, dtype=dt, device=DEV)
        ms = best(lambda: torch.matmul(x, y), 5)
        out[f"{name}_TFLOP/s"] = round(2 * k ** 3 / ms / 1e9, 1)
        del x, y
    torch.cuda.empty_cache()
    return out


def calibrate_copy(gib=1.0):
    """The library's streaming copy of a known size (1 GiB read, 1 GiB
    written), for scaling the rocprofv3 byte counters."""
    import torch
    from paper_1808_00896_amd import soft
    n = int(gib * (1 << 30)) // 16
    a = torch.zeros(n, dtype=torch.complex128, device=DEV)
    b = torch.empty_like(a)
    for _ in range(3):
        soft.soft_probe_copy(a, b)
    torch.cuda.synchronize()
    return n * 16


# ---------------------------------------------------------------------------
# rocprofv3 summaries (profiles/)
# ---------------------------------------------------------------------------

FFT_KIND = {"0": "fft_gamma_fwd", "1": "fft_alpha_fwd", "2": "fft_alpha_inv", "3": "fft_gamma_inv"}


def stage_of(kernel):
    """Library stage of a kernel name, or None."""
    m = re.match(r"k_fft(?:_ingrid)?<\s*\d+\s*,\s*(\d)", kernel)
    if m:
        return FFT_KIND.get(m.group(1))
    if kernel.startswith("k_fft_gamma_inv_argmax"):
        return "fft_gamma_inv"
    if kernel.startswith("k_dwt_fwd"):
        return "dwt_fwd"
    if kernel.startswith("k_dwt_inv") or kernel.startswith("k_idwt_clenshaw"):
        return "dwt_inv"
    if kernel.startswith("k_corr_coeffs"):
        return "match_coeffs"
    if kernel.startswith("k_argmax"):
        return "argmax"
    return None


def _csv_rows(pattern):
    rows = []
    for f in sorted(glob.glob(pattern, recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _short(name, n=56):
    name = re.sub(r"\(.*$", "", name.replace("(anonymous namespace)::", "").replace("soft::", ""))
    name = re.sub(r"^void ", "", name.strip())
    return name[:n]


def _last_dispatches(rows, stage, count):
    """The last `count` dispatches of a stage's kernels (by dispatch id)."""
    picked = [r for r in rows if stage_of(_short(r["Kernel_Name"], 400)) == stage]
    picked.sort(key=lambda r: int(r["Dispatch_Id"]))
    return picked[-count:] if count else []


def summarize_rocprof(workload, trace_steps=10, pmc_steps=2):
    """Write profiles/<workload>_kernel_stats.txt and _hbm_traffic.txt from the
    rocprofv3 runs of PROFILE_RECIPE, and the per-launch HBM bytes of each
    stage into profiles/traffic.json.  Per stage, only the launches of the
    last timed steps count (the plan's launch-shape tuning and the warm-up
    run before them)."""
    base = os.path.join(ROOT, "gpurun_out", "prof", workload)
    srcs = f"fft.hip+soft_internal.h {source_digest('fft')}, dwt.hip+soft_internal.h {source_digest('dwt')}"
    cmds = [c.format(w=workload, sq=sq_counters_of(workload)) for c in PROFILE_RECIPE]
    Bs, prec = _workload_bands(workload)
    work = stage_work(Bs, prec)
    stats = _csv_rows(os.path.join(base, "trace", "**", "*kernel_stats.csv"))
    trace = _csv_rows(os.path.join(base, "trace", "**", "*kernel_trace.csv"))
    if not stats or not trace:
        raise SystemExit(f"no kernel_stats.csv / kernel_trace.csv under {base}/trace")
    lines = [f"# rocprofv3 kernel-trace summary: workload {workload} (bench.py --only {workload})",
             f"# command (repository root, TMPDIR=/tmp): {cmds[0]}",
             f"# kernel sources: {srcs}",
             f"# per stage, the launches of the last {trace_steps} timed steps (durations in microseconds):",
             f"{'stage':14s} {'kernel':44s} {'launches':>8s} {'avg_us':>9s} {'algorithmic':>12s} {'rate':>14s}"]
    avg_of = {}
    for st in STAGES:
        per_step = calls_per_step(workload, st)
        d = _last_dispatches(trace, st, trace_steps * per_step)
        if not d:
            continue
        us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in d]
        avg = sum(us) / len(us)
        names = sorted({_short(r["Kernel_Name"], 44) for r in d})
        avg_of[st] = (names, avg)
        kind, amount = work[st]
        amount /= per_step
        if kind == "hbm":
            rate, algo = f"{amount / avg / 1e3:8.0f} GB/s", f"{amount / 1e6:9.1f} MB"
        else:
            rate, algo = f"{amount / avg / 1e6:7.2f} TFLOP/s", f"{amount / 1e9:8.3f} GF"
        lines.append(f"{st:14s} {names[0]:44s} {len(d):8d} {avg:9.2f} {algo:>12s} {rate:>14s}")
        for nm in names[1:]:
            lines.append(f"{'':14s} {nm:44s}")
    lines += ["#", "# every kernel of the run (rocprofv3 --stats), including the plan-time launch-shape tuning:",
              f"{'kernel':58s} {'stage':14s} {'calls':>6s} {'total_us':>10s} {'avg_us':>10s} {'pct':>6s}"]
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        k = _short(r["Name"], 400)
        lines.append(f"{k[:58]:58s} {stage_of(k) or '-':14s} {int(r['Calls']):6d} "
                     f"{float(r['TotalDurationNs']) / 1e3:10.1f} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['Percentage']):6.2f}")
    with open(os.path.join(ROOT, "profiles", f"{workload}_kernel_stats.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")

    def per_dispatch(sub, counter):
        rows = _csv_rows(os.path.join(base, sub, "**", "*counter_collection.csv"))
        acc = {}
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            key = int(r["Dispatch_Id"])
            if key not in acc:
                acc[key] = dict(r, Counter_Value=0.0)
            acc[key]["Counter_Value"] += float(r["Counter_Value"])
        return list(acc.values())

    fetch = per_dispatch("fetch", "FETCH_SIZE")
    write = per_dispatch("write", "WRITE_SIZE")
    if not fetch or not write:
        log("no counter runs found: kernel trace summary only")
        return

    def mean_kib(rows, pred):
        v = [r["Counter_Value"] for r in rows if pred(_short(r["Kernel_Name"], 400))]
        return sum(v) / len(v) if v else None

    cf = mean_kib(fetch, lambda k: k.startswith("k_probe_copy"))
    cw = mean_kib(write, lambda k: k.startswith("k_probe_copy"))
    if not cf or not cw:
        raise SystemExit("no calibration copy (k_probe_copy) in the counter runs")
    copy_bytes = float(1 << 30)
    ff, fw = copy_bytes / (cf * 1024), copy_bytes / (cw * 1024)
    lines = [f"# HBM traffic per launch from rocprofv3 counters: workload {workload}",
             f"# FETCH_SIZE command: {cmds[1]}", f"# WRITE_SIZE command: {cmds[2]}",
             f"# calibration: the library's 1 GiB streaming copy (k_probe_copy) reads FETCH_SIZE = "
             f"{cf:.0f} KiB and WRITE_SIZE = {cw:.0f} KiB per dispatch,",
             f"#   so bytes = FETCH_SIZE * 1024 * {ff:.3f} + WRITE_SIZE * 1024 * {fw:.3f}",
             f"# kernel sources: {srcs}",
             f"# per stage, the launches of the last {pmc_steps} timed steps; avg_us from the kernel trace",
             f"{'stage':14s} {'kernel':44s} {'fetch_MB':>9s} {'write_MB':>9s} {'total_MB':>9s} {'algo_MB':>9s} "
             f"{'ratio':>6s} {'avg_us':>8s} {'GB/s':>7s}"]
    try:
        traffic = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        traffic = {}
    rec = {}
    for st, (names, avg) in avg_of.items():
        per_step = calls_per_step(workload, st)
        df = _last_dispatches(fetch, st, pmc_steps * per_step)
        dw = _last_dispatches(write, st, pmc_steps * per_step)
        if not df or not dw:
            continue
        fb = sum(r["Counter_Value"] for r in df) / len(df) * 1024 * ff
        wb = sum(r["Counter_Value"] for r in dw) / len(dw) * 1024 * fw
        if work[st][0] == "hbm":
            algo = work[st][1] / per_step
        else:  # DWT: read S (or the coefficients) and write the coefficients (or S)
            algo = sum(CSIZE[prec] * ((2 * B) * (2 * B - 1) ** 2 + num_coeffs(B)) for B in Bs) / per_step
        lines.append(f"{st:14s} {names[0]:44s} {fb / 1e6:9.1f} {wb / 1e6:9.1f} {(fb + wb) / 1e6:9.1f} "
                     f"{algo / 1e6:9.1f} {(fb + wb) / algo:6.3f} {avg:8.2f} {(fb + wb) / avg / 1e3:7.0f}")
        kind = "fft" if st.startswith("fft") else "dwt"
        rec[st] = {"bytes_per_launch": round(fb + wb), "fetch_bytes": round(fb), "write_bytes": round(wb),
                   "algorithmic_bytes": round(algo), "kernels": names, "source_sha": source_digest(kind)}
    traffic[workload] = rec
    with open(os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(traffic, fh, indent=1, sort_keys=True)
        fh.write("\n")
    summarize_sq(workload, base, cmds[3], srcs, avg_of, work, pmc_steps)


def summarize_sq(workload, base, cmd, srcs, avg_of, work, pmc_steps):
    """profiles/<workload>_sq_counters.txt from the shader-counter pass: per
    stage and launch, the matrix-core operations executed (MOPS x 512 flop)
    against the contraction's algorithmic flops 8 B N_c per function (their
    ratio counts the padded lanes: absent members, rows past a group's last
    degree, the split mode's tail), the matrix cores' busy share (busy cycles
    over the launch's duration x 2.4 GHz x 1024 SIMDs), the FP64 vector FMA
    flops (64 lanes x 2 per instruction: the recurrence) against the
    recurrence's algorithmic (5/3) B (B^3 - B), LDS instructions and
    bank-conflict cycles per LDS instruction."""
    rows = _csv_rows(os.path.join(base, "sq", "**", "*counter_collection.csv"))
    if not rows:
        log("no shader-counter run found")
        return
    vals = {}
    for r in rows:
        key = (int(r["Dispatch_Id"]), r["Counter_Name"])
        vals.setdefault(key, [r, 0.0])
        vals[key][1] += float(r["Counter_Value"])
    by_disp = {}
    for (d, name), (r, v) in vals.items():
        by_disp.setdefault(d, {"Kernel_Name": r["Kernel_Name"], "Dispatch_Id": d})[name] = v
    disp = list(by_disp.values())
    names = sq_counters_of(workload).split()
    mops = [n for n in names if "MOPS" in n]
    Bs, _ = _workload_bands(workload)
    contraction = sum(8.0 * B * num_coeffs(B) for B in Bs)
    recurrence = sum(5.0 / 3.0 * B * (B ** 3 - B) for B in Bs)
    lines = [f"# shader counters per launch (rocprofv3 --pmc): workload {workload}",
             f"# command: {cmd}",
             f"# kernel sources: {srcs}",
             f"# per stage, the mean over the launches of the last {pmc_steps} timed steps; avg_us from the kernel trace",
             "# mfma_GF: matrix-core operations executed, sum of " + " + ".join(mops) + " x 512 flop",
             "# busy: SQ_VALU_MFMA_BUSY_CYCLES / (avg_us x 2400 cycles/us x 1024 SIMDs)",
             "# fma64_GF: SQ_INSTS_VALU_FMA_F64 x 128 flop; rec_GF: the recurrence's algorithmic flops",
             f"{'stage':14s} {'avg_us':>8s} {'contr_GF':>8s} {'mfma_GF':>8s} {'ratio':>6s} {'busy':>6s} "
             f"{'rec_GF':>7s} {'fma64_GF':>8s} {'lds_M':>7s} {'confl/lds':>9s}"]
    for st, (_, avg) in avg_of.items():
        per_step = calls_per_step(workload, st)
        d = _last_dispatches(disp, st, pmc_steps * per_step)
        if not d:
            continue

        def mean(n):
            return sum(x.get(n, 0.0) for x in d) / len(d)

        mf = sum(mean(n) for n in mops) * 512.0
        dwt = st.startswith("dwt")
        algo = contraction / per_step if dwt else 0.0
        rec_f = recurrence / per_step if dwt else 0.0
        busy = mean("SQ_VALU_MFMA_BUSY_CYCLES") / (avg * 2400.0 * 1024)
        lds = mean("SQ_INSTS_LDS")
        confl = mean("SQ_LDS_BANK_CONFLICT") / lds if lds else 0.0
        ratio = f"{mf / algo:6.3f}" if algo else f"{'-':>6s}"
        lines.append(f"{st:14s} {avg:8.2f} {algo / 1e9:8.3f} {mf / 1e9:8.3f} {ratio} {busy:6.3f} "
                     f"{rec_f / 1e9:7.3f} {mean('SQ_INSTS_VALU_FMA_F64') * 128 / 1e9:8.3f} {lds / 1e6:7.2f} "
                     f"{confl:9.3f}")
    lines.append("# raw means per launch:")
    for st in avg_of:
        d = _last_dispatches(disp, st, pmc_steps * calls_per_step(workload, st))
        if d:
            lines.append(f"#   {st}: " + ", ".join(f"{n} {sum(x.get(n, 0.0) for x in d) / len(d):.4g}" for n in names))
    with open(os.path.join(ROOT, "profiles", f"{workload}_sq_counters.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _workload_bands(workload):
    m = re.match(r"(fp64|fp32_split|fp32)_B(\d+)_n(\d+)$", workload)
    if m:
        return [int(m.group(2))] * int(m.group(3)), m.group(1)
    m = re.match(r"(fp64|fp32_split|fp32)_uneven(\d+)$", workload)
    if m:
        from paper_1808_00896_amd import inputs
        Bs, _ = inputs.uneven_batch(int(m.group(2)), [16, 32, 64, 128], seed=4)
        return Bs, m.group(1)
    raise SystemExit(f"unknown workload {workload}")


def calls_per_step(workload, stage):
    """Launches of a stage per step: one per band for the FFT passes, one per
    DWT launch group for the DWT; a one-band plan launches each once."""
    Bs, _ = _workload_bands(workload)
    bands = sorted(set(Bs))
    if len(bands) == 1:
        return 1
    if stage.startswith("fft"):
        return len(bands)
    return len({0 if b * 2 <= 64 else b for b in bands})


ONLY_LEGS = ("fp64_B16_n1", "fp64_B128_n1", "fp64_B256_n1", "fp64_B512_n1", "fp32_split_B512_n1", "fp32_B512_n1",
             "fp32_split_B128_n16", "fp32_B128_n16", "fp64_B128_n16", "fp64_uneven256", "fp32_split_uneven256")
# Coefficient seed of a one-bandwidth workload, as its leg draws it.
ONLY_SEED = {128: 1, 256: 2, 512: 3}


def run_only(args):
    """One workload alone, for profiling: `steps` timed steps, no oracle."""
    from paper_1808_00896_amd import inputs
    Bs, prec = _workload_bands(args.only)
    uniform = len(set(Bs)) == 1 and not args.only.startswith(prec + "_uneven")
    if uniform and Bs[0] == SMALL_B:
        c = np.tile(inputs.coeffs_uniform(SMALL_B, 0), len(Bs))
    elif uniform:
        c = np.tile(inputs.coeffs_decay(Bs[0], ONLY_SEED.get(Bs[0], 1)), len(Bs))
    else:
        _, cs = inputs.uneven_batch(len(Bs), [16, 32, 64, 128], seed=4)
        c = np.concatenate(cs)
    res, _ = run_leg(Bs, prec, args.steps, args.warmup, c, uniform=uniform)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--B", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline leg only")
    ap.add_argument("--only", choices=ONLY_LEGS, help="one workload alone (for rocprofv3 runs)")
    ap.add_argument("--no-b512", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--b512-steps", type=int, default=5)
    ap.add_argument("--batch", type=int, default=16, help="functions per batched call at B=128")
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
                    help="also run the library's 1 GiB streaming copy (byte-counter calibration under rocprofv3)")
    ap.add_argument("--summarize-rocprof", metavar="WORKLOAD",
                    help="summarize gpurun_out/prof/WORKLOAD/ into profiles/ (no GPU needed)")
    args = ap.parse_args()
    global TUNE
    TUNE = not args.no_tune
    if args.summarize_rocprof:
        summarize_rocprof(args.summarize_rocprof)
        return
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
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.only:
        res = run_only(args)
        if args.calibrate_copy:
            res["copy_calibration_bytes"] = calibrate_copy()
        print(json.dumps({"only": args.only, **res}))
        return

    B = args.B
    legs = {}
    main_leg, main_grid, c_host = main_legs(args, legs)
    value = main_leg["value"]
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
        "roofline": main_leg["roofline"],
        "stages": main_leg["stages"],
        "stages_from": main_leg["stages_from"],
        "dwt_shapes": main_leg["dwt_shapes"],
        "round_trip_err": main_leg["round_trip_err"],
        "step_ms": main_leg["step_ms"],
        "inverse_ms": main_leg["inverse_ms"],
        "forward_ms": main_leg["forward_ms"],
    }
    log(f"B={B}: {value:.1f} fwd+inv/s, round trip {main_leg['round_trip_err']:.2e}")

    if args.oracle_table:
        out["oracle_table"] = oracle_table([16, 128, 256], [16, 128], 512)
        print(json.dumps(out))
        return

    if not args.quick:
        batch_legs(args, legs, B, c_host, main_grid)
    del main_grid
    torch.cuda.empty_cache()
    if not args.quick and not args.no_b512:
        b512_legs(args, legs)
    if not args.quick and not args.no_uneven:
        uneven_legs(args, legs)
    if not args.quick and not args.no_match:
        legs.update(match_leg(args.match_steps))

    if not args.no_cpu_baseline:
        log("CPU baseline: timing the oracle, then scoring every leg against it")
        out["cpu_baseline"], acc = cpu_baseline(B)
        for leg, rep in acc.items():
            legs.setdefault(leg, {})["err_vs_oracle"] = rep
        out["err_vs_oracle"] = legs[f"B{B}_fp64"]["err_vs_oracle"]
    else:
        out["cpu_baseline"] = None
    legs.pop(f"B{B}_fp64", None)
    out["legs"] = legs
    if not args.quick:
        log("ceilings")
        out["ceilings"] = ceilings(16 * (2 * B) ** 3)
    if args.calibrate_copy:
        out["copy_calibration_bytes"] = calibrate_copy()
    out["summary"] = summary(out, legs)
    print(json.dumps(out))


def summary(out, legs):
    """One compact entry per leg, last in the line (so a tail of it shows
    every leg): v = throughput, ms = median inverse and forward ms, rf = the
    dominant kernel's roofline fraction, inv / fwd = the worst error against
    the oracle over the leg's samples as [max-norm, L2] (inverse) and
    [max-norm, L2, largest per-degree] (forward), x = speedup over the leg's
    FP64 (or eager) counterpart; 3 significant digits."""
    def worst(rep, key, n):
        return [sig(max(r[key].get(k, 0.0) for r in rep), 2) for k in ("max_rel", "l2_rel", "deg_rel_max")[:n]]

    res = {}
    for name, r in legs.items():
        rf = r.get("roofline") or {}
        rep = r.get("err_vs_oracle")
        e = {"v": sig(r["value"]) if r.get("value") is not None else None}
        if r.get("inverse_ms"):
            e["ms"] = [sig(r["inverse_ms"]["median"]), sig(r["forward_ms"]["median"])]
        if rf:
            e["rf"] = sig(rf["frac"], 2)
        if rep:
            e["inv"] = worst(rep, "inverse", 2)
            e["fwd"] = worst(rep, "forward", 3)
        for k in ("speedup_vs_fp64", "speedup_vs_eager"):
            if k in r:
                e["x"] = r[k]
        res[name] = e
    return res


if __name__ == "__main__":
    main()
