"""Benchmark: GStencil/s of the outer-product stencil sweep on one MI355X.

Workload (one bench "step" = one pass of the whole hot path): 2D box
stencils of order r = 1, 2, 3, 4 (9/25/49/81 points) on an 8192 x 8192 FP32
grid, seeded coefficients normalised to sum 1, inputs uniform on [-1, 1),
periodic boundary, 100 Jacobi steps per order -- i.e. four solves of 100
steps.  ``value`` is the whole step's point-steps per second for the
headline path; the gather-form baseline and the other outer-product variants
are timed beside it on the same inputs.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "f16": 2500.0}
DIMS = (8192, 8192)
RADII = (1, 2, 3, 4)
JACOBI_STEPS = 100
INPUT_SEED = 201
COEF_SEED0 = 2100


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2310_16298_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def time_path(st, torch, path, radius, a0_dev, coeffs, reps, warmup, stream):
    """Per-rep wall times (ms, HIP events on the launch stream) of one
    100-step solve."""
    plan = st.Plan(DIMS, radius, st.BOX, coeffs, boundary=st.BC_PERIODIC, dtype=st.F32, path=path)
    x = a0_dev.clone()
    tmp = torch.empty_like(x)
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plan.run_steps(x, tmp, JACOBI_STEPS, stream=stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for s, e in evs:
        s.record(stream)
        plan.run_steps(x, tmp, JACOBI_STEPS, stream=stream)
        e.record(stream)
    torch.cuda.synchronize()
    times = [s.elapsed_time(e) for s, e in evs]
    info = plan.info
    plan.close()
    return times, info


def cpu_baseline(coeffs_by_r, a0) -> dict:
    """The FP64 oracle on the host cores: one Jacobi step of the full grid per
    order (a bounded sample of the same workload), scaled to GStencil/s."""
    import oracle
    oracle.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    used = oracle.set_threads(threads)
    total_pts, total_s = 0, 0.0
    for r in RADII:
        c = coeffs_by_r[r].astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        oracle.run(a0, c, r, 1, 1, 1)
        total_s += time.perf_counter() - t0
        total_pts += DIMS[0] * DIMS[1]
    return {"value": total_pts / total_s / 1e9, "unit": "GStencil/s", "cores": used, "kind": "oracle",
            "sample": f"one Jacobi step of the full {DIMS[0]}x{DIMS[1]} grid for each r in {list(RADII)} "
                      f"(FP64 gather oracle, {used} OpenMP threads, {cpu_model()}), {total_s:.1f} s",
            "seconds": total_s}


def load_traffic(kernel_key: str, src_hash: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    if not ent or ent.get("source_hash") != src_hash:
        return None
    return ent.get("hbm_bytes_per_launch")


def main() -> int:
    global RADII, JACOBI_STEPS
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed bench steps (one step = 4 solves x 100 Jacobi steps)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--headline", default="auto", choices=["auto", "mfma", "gather", "mfma_f16x3", "mfma_bf16x3"])
    ap.add_argument("--paths", default="gather,mfma,mfma_f16x3,mfma_bf16x3,auto")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--radii", default="1,2,3,4", help="orders to run (profiling runs use a subset)")
    ap.add_argument("--jacobi-steps", type=int, default=JACOBI_STEPS,
                    help="Jacobi steps per solve (profiling runs only; the benchmark uses 100)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="first run N plain device copies of one grid (known bytes) for counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU runs are not part of this build.",
              file=sys.stderr)
        return 2

    import torch
    from paper_2310_16298_amd import inputs
    from paper_2310_16298_amd import stencil as st

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    st.load_library()
    name_to_path = {"gather": st.PATH_GATHER, "mfma": st.PATH_MFMA, "mfma_f16x3": st.PATH_MFMA_F16X3,
                    "mfma_bf16x3": st.PATH_MFMA_BF16X3, "auto": st.PATH_AUTO}
    paths = [p for p in args.paths.split(",") if p]
    if args.headline not in paths:
        paths.append(args.headline)

    RADII = tuple(int(v) for v in args.radii.split(","))
    JACOBI_STEPS = args.jacobi_steps
    a0 = inputs.grid(DIMS, seed=INPUT_SEED, dtype=np.float32)
    coeffs = {r: inputs.coefficients(2, r, inputs.BOX, seed=COEF_SEED0 + r, dtype=np.float64) for r in RADII}
    a0_dev = torch.from_numpy(a0).cuda()
    stream = torch.cuda.Stream()
    if args.calibrate_copy:
        dst = torch.empty_like(a0_dev)
        for _ in range(args.calibrate_copy):
            dst.copy_(a0_dev)
        torch.cuda.synchronize()
        print(f"[bench] calibration: {args.calibrate_copy} copies of {a0_dev.numel() * 4} bytes", file=sys.stderr)
    pts_per_solve = DIMS[0] * DIMS[1] * JACOBI_STEPS

    results = {}
    for name in paths:
        per_r = {}
        for r in RADII:
            times, info = time_path(st, torch, name_to_path[name], r, a0_dev, coeffs[r],
                                    args.steps, args.warmup, stream)
            med = float(np.median(times))
            per_r[r] = {"ms_per_solve": med, "gstencil_s": pts_per_solve / (med * 1e-3) / 1e9,
                        "p50_ms": float(np.percentile(times, 50)), "p99_ms": float(np.percentile(times, 99)),
                        "resolved_path": st.PATH_NAMES[info["path"]], "info": info, "times": times}
            print(f"[bench] {name:12s} r={r}: {per_r[r]['gstencil_s']:8.1f} GStencil/s "
                  f"({med:.2f} ms / 100 steps, path={per_r[r]['resolved_path']})", file=sys.stderr, flush=True)
        results[name] = per_r

    head = results[args.headline]
    # one bench step = the four solves; per-step time = sum of the per-order medians
    step_times = [sum(head[r]["times"][k] for r in RADII) for k in range(args.steps)]
    ms_per_step = float(np.median(step_times))
    value = len(RADII) * pts_per_solve / (ms_per_step * 1e-3) / 1e9

    # dominant kernel: the order with the largest share of the step
    r_dom = max(RADII, key=lambda r: head[r]["ms_per_solve"])
    dom = head[r_dom]
    launch_ms = dom["ms_per_solve"] / JACOBI_STEPS
    info = dom["info"]
    bytes_per_launch = info["bytes_per_point"] * DIMS[0] * DIMS[1]
    gbs = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    flops_per_launch = info["useful_flops_per_point"] * DIMS[0] * DIMS[1]
    tflops = flops_per_launch / (launch_ms * 1e-3) / 1e12
    exec_tflops = info["executed_flops_per_point"] * DIMS[0] * DIMS[1] / (launch_ms * 1e-3) / 1e12
    rpath = dom["resolved_path"]
    mfma_dtype = {"mfma": "f32", "mfma_f16x3": "f16", "mfma_bf16x3": "bf16"}.get(rpath)
    # bound: HBM unless the executed matrix work at the unit's peak would take longer than the bytes
    bound = "hbm"
    if mfma_dtype:
        t_mem = bytes_per_launch / (HBM_PEAK_GBS * 1e9)
        t_mfma = info["executed_flops_per_point"] * DIMS[0] * DIMS[1] / (PEAK_TFLOPS[mfma_dtype] * 1e12)
        if t_mfma > t_mem:
            bound = "mfma"
    src_hash = kernel_source_hash()
    kernel_key = f"{rpath}_box_r{r_dom}_f32_{DIMS[0]}x{DIMS[1]}_periodic"
    traffic = load_traffic(kernel_key, src_hash)
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    else:
        peak = PEAK_TFLOPS[mfma_dtype]
        roof = {"bound": "mfma", "achieved": tflops, "peak": peak, "unit": "TFLOP/s", "frac": tflops / peak,
                "executed_tflops": exec_tflops, "hbm_gbs": gbs}
    roof["traffic"] = traffic
    roof["kernel"] = kernel_key
    roof["launch_us"] = launch_ms * 1e3

    line = {
        "metric": "GStencil/s (points·steps/s) + % HBM/MFMA roofline vs gather; p50/p99 latency",
        "value": value,
        "unit": "GStencil/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.headline in ("mfma", "gather") else ("f32+" + (mfma_dtype or "f32")),
        "data": "synthetic",
        "config": {"workload": f"2D box stencils r=1..4, {DIMS[0]}x{DIMS[1]} FP32 grid, periodic, "
                               f"{JACOBI_STEPS} Jacobi steps per order (4 solves per bench step)",
                   "headline_path": args.headline, "input_seed": INPUT_SEED,
                   "coef_seeds": [COEF_SEED0 + r for r in RADII]},
        "roofline": roof,
    }
    line["per_order"] = {name: {str(r): {"gstencil_s": round(v["gstencil_s"], 2), "p50_ms": round(v["p50_ms"], 3),
                                         "p99_ms": round(v["p99_ms"], 3), "path": v["resolved_path"],
                                         "hbm_frac": round(v["gstencil_s"] * 8 / HBM_PEAK_GBS, 4)}
                                 for r, v in res.items()} for name, res in results.items()}
    if "gather" in results:
        line["vs_gather"] = {name: {str(r): round(res[r]["gstencil_s"] / results["gather"][r]["gstencil_s"], 3)
                                    for r in RADII} for name, res in results.items()}
    line["latency_ms"] = {"p50": float(np.percentile(step_times, 50)), "p99": float(np.percentile(step_times, 99))}
    if not args.no_cpu:
        cb = cpu_baseline(coeffs, a0)
        cb.pop("seconds", None)
        line["cpu_baseline"] = cb
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
