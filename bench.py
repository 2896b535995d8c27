"""Benchmark: GStencil/s of the outer-product stencil sweep on one MI355X.

Workload (one bench "step" = one pass of the whole hot path): 2D box
stencils of order r = 1, 2, 3, 4 (9/25/49/81 points) on an 8192 x 8192 FP32
grid, seeded coefficients normalised to sum 1, inputs uniform on [-1, 1),
periodic boundary, 100 Jacobi steps per order -- i.e. four solves of 100
steps.  ``value`` is the whole step's point-steps per second for the
headline path; the gather-form baseline and the other outer-product variants
are timed beside it on the same inputs.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Other configurations (their own JSON line each; not the headline):
    --workload star2d_512   2D five-point star, 512 x 512 FP64, zero halo, 10 steps
    --workload grid3d       3D stars r=1..4 and the 27-point box, 512^3 FP32/FP64, 50 steps
    --workload mixed        BF16x3 / FP16x3 with an FP64 shadow and the CPU FP64 oracle (whole grid),
                            drift check every 50 steps
    --workload batch        many small FP64 grids (Table 3 shapes) per batched launch vs one by one
    --workload tune         autotuner sweep: line option x MFMA block x chunk per radius
    --workload serve        serving loop, Poisson arrivals at 0.5 / 0.8 load: p50/p99 latency
    --workload cover        irregular order-4 stencils: minimum line cover vs box and gather
    --workload tiles        register x workgroup tiles of the n = 4 box outer products (Fig. 4 on MI355X)

The default line also carries ``configs``: the 512^2 FP64 latency case, the
512^3 3D stars and 27-point box (FP32 / FP64, AUTO) and the mixed-precision
pair at 200 steps, a few repetitions each (``--no-configs`` skips them).
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


# Sources of the 2D kernels timed by the default workload: a counter summary
# in profiles/traffic.json is used only while these files are unchanged.
KERNEL_SOURCES_2D = ["device_common.hpp", "stream2d.hpp", "dma2d.hpp", "kernels_2d.hpp", "kernels_split2d.hpp",
                     "mfma_traits.hpp", "kernels_mfma2d.hip", "kernels_split2d.hip", "kernels_gather2d.hip",
                     "kernels_tb2d.hpp", "kernels_tb2d.hip", "kernels_tb2d_box.hip", "kernels_tb2d_star.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2310_16298_amd", "csrc")
    for name in KERNEL_SOURCES_2D:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def hbm_frac(gstencil_s: float, bytes_per_point: int, time_block: int = 1) -> float:
    """Algorithmic HBM bytes per second over the 8 TB/s peak: a launch reads and
    writes the grid once and advances time_block steps."""
    return round(gstencil_s * bytes_per_point / max(1, int(time_block)) / HBM_PEAK_GBS, 4)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def time_path(st, torch, knobs, radius, a0_dev, coeffs, reps, warmup, stream):
    """Per-rep wall times (ms, HIP events on the launch stream) of one
    100-step solve from the seeded grid (restored before each solve, outside
    the timed region); knobs: Plan keyword arguments (path, time_block, ...)."""
    plan = st.Plan(DIMS, radius, st.BOX, coeffs, boundary=st.BC_PERIODIC, dtype=st.F32, **knobs)
    x = a0_dev.clone()
    tmp = torch.empty_like(x)
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            x.copy_(a0_dev)
            plan.run_steps(x, tmp, JACOBI_STEPS, stream=stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    with torch.cuda.stream(stream):
        for s, e in evs:
            x.copy_(a0_dev)
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


def _time_solve(torch, plan, x0, steps, reps, warmup, stream):
    """Wall times (ms) of `steps`-step solves, each from x0 (restored on the
    launch stream before the start event)."""
    x = x0.clone()
    tmp = torch.empty_like(x)
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            x.copy_(x0)
            plan.run_steps(x, tmp, steps, stream=stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    with torch.cuda.stream(stream):
        for s0, e0 in evs:
            x.copy_(x0)
            s0.record(stream)
            plan.run_steps(x, tmp, steps, stream=stream)
            e0.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def workload_star2d_512(args, torch, st, inputs) -> dict:
    """2D five-point star (r = 1), 512 x 512 FP64, centre 1/2, neighbours 1/8,
    zero halo, 10 Jacobi steps: GPU latency p50/p99 and the CPU oracle's time."""
    import oracle
    dims, steps = (512, 512), 10
    c = inputs.diffusion_5pt()
    a0 = inputs.grid(dims, seed=101, dtype=np.float64)
    x0 = torch.from_numpy(a0).cuda()
    stream = torch.cuda.Stream()
    out = {"metric": "10-step solve latency (us) and GStencil/s", "workload":
           "2D 5-point star r=1, 512x512 FP64, zero halo, 10 Jacobi steps, seed 101", "paths": {}}
    for name, knobs in (("gather", {"path": st.PATH_GATHER}), ("mfma", {"path": st.PATH_MFMA}),
                        ("gather_tb5", {"path": st.PATH_GATHER, "time_block": 5}),
                        ("gather_tb8", {"path": st.PATH_GATHER, "time_block": 8}), ("auto", {})):
        plan = st.Plan(dims, 1, st.STAR, c, boundary=st.BC_ZERO, dtype=st.F64, **knobs)
        times = _time_solve(torch, plan, x0, steps, max(args.steps, 20), args.warmup, stream)
        res = plan.run_steps(x0.clone(), torch.empty_like(x0), steps)
        torch.cuda.synchronize()
        want = oracle.run(a0, c, 1, st.STAR, st.BC_ZERO, steps)
        err = float(np.abs(res.cpu().numpy() - want).max())
        out["paths"][name] = {"p50_us": float(np.percentile(times, 50)) * 1e3,
                              "p99_us": float(np.percentile(times, 99)) * 1e3,
                              "gstencil_s": dims[0] * dims[1] * steps / (np.median(times) * 1e-3) / 1e9,
                              "max_abs_err_vs_oracle": err, "block_n": plan.info["block_n"],
                              "time_block": plan.info["time_block"]}
        print(f"[bench] star2d_512 {name}: p50 {out['paths'][name]['p50_us']:.1f} us, "
              f"p99 {out['paths'][name]['p99_us']:.1f} us, err {err:.2e}", file=sys.stderr, flush=True)
        plan.close()
    oracle.build(force=False)
    used = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    t0 = time.perf_counter()
    oracle.run(a0, c, 1, st.STAR, st.BC_ZERO, steps)
    out["cpu_oracle_seconds"] = time.perf_counter() - t0
    out["cpu_oracle_threads"] = used
    return out


def workload_grid3d(args, torch, st, inputs) -> dict:
    """3D stars r = 1..4 and boxes r = 1..4 (27-point box: r = 1) on 512^3,
    FP32 and FP64, zero halo, 50 Jacobi steps: gather vs outer-product paths,
    the two-step time block (`gather_tb2`, where it is built) and AUTO."""
    dims, steps = (512, 512, 512), args.solve_steps or 50
    a64 = inputs.grid(dims, seed=301, dtype=np.float64)
    stream = torch.cuda.Stream()
    out = {"metric": "GStencil/s", "workload": f"3D 512^3, zero halo, {steps} Jacobi steps", "cases": {}}
    cases = [(st.STAR, r) for r in (1, 2, 3, 4)] + [(st.BOX, r) for r in (1, 2, 3, 4)]
    want_cases = set(args.cases.split(",")) if args.cases else None
    want_paths = set(args.paths3d.split(",")) if args.paths3d else None
    for dt, tdt in ((st.F32, np.float32), (st.F64, np.float64)):
        x0 = None
        paths = [("gather", st.PATH_GATHER, 0), ("gather_tb2", st.PATH_GATHER, 2), ("mfma", st.PATH_MFMA, 0),
                 ("auto", st.PATH_AUTO, 0)]
        if dt == st.F32:
            paths += [("mfma_f16x3", st.PATH_MFMA_F16X3, 0), ("mfma_bf16x3", st.PATH_MFMA_BF16X3, 0)]
        for shape, r in cases:
            c = inputs.coefficients(3, r, shape, seed=3100 + 10 * shape + r, dtype=np.float64)
            key = f"{'f32' if dt == st.F32 else 'f64'}_{'box' if shape == st.BOX else 'star'}_r{r}"
            if want_cases is not None and key not in want_cases:
                continue
            if x0 is None:
                x0 = torch.from_numpy(a64.astype(tdt)).cuda()
            out["cases"][key] = {}
            for name, path, tb in paths:
                if want_paths is not None and name not in want_paths:
                    continue
                if shape == st.BOX and r > 1 and (path == st.PATH_AUTO or
                                                  (path == st.PATH_MFMA and dt == st.F64 and r > 2)):
                    continue  # 3D boxes beyond r = 1: gather, outer products (FP64: r <= 2), split products
                if tb and st.desc_check(dims, r, shape, c, boundary=st.BC_ZERO, dtype=dt, path=path,
                                        time_block=tb) != st.OK:
                    continue  # no time-blocked kernel for this stencil
                plan = st.Plan(dims, r, shape, c, boundary=st.BC_ZERO, dtype=dt, path=path, time_block=tb)
                times = _time_solve(torch, plan, x0, steps, args.steps, args.warmup, stream)
                g = dims[0] * dims[1] * dims[2] * steps / (np.median(times) * 1e-3) / 1e9
                bpp = 8 if dt == st.F32 else 16
                out["cases"][key][name] = {"gstencil_s": round(g, 2),
                                           "hbm_frac": hbm_frac(g, bpp, plan.info["time_block"]),
                                           "ms_per_solve": round(float(np.median(times)), 3),
                                           "resolved_path": st.PATH_NAMES[plan.info["path"]],
                                           "time_block": plan.info["time_block"]}
                print(f"[bench] {key} {name}: {g:.1f} GStencil/s", file=sys.stderr, flush=True)
                plan.close()
        x0 = None
        torch.cuda.empty_cache()
    return out


def workload_batch(args, torch, st, inputs) -> dict:
    """Many small FP64 grids of the paper's Table 3 shapes (2D box/star r = 1..3
    at 64^2..512^2, 3D box r = 1, 2 and star r = 1..3 at 8^3..64^3), zero halo,
    10 Jacobi steps: one batched launch per step over 2^24 points of grids of
    one size (a shared plan), for the outer-product (MFMA) and the gather
    path -- their ratio is the MI355X counterpart of Table 3's speedups --
    and, for the AUTO plan, against launching the grids one by one."""
    steps = 10
    total_pts = 1 << 24
    stream = torch.cuda.Stream()
    out = {"metric": "GStencil/s", "workload": "batches of FP64 Table 3 grids, 2^24 points per batch, "
           "zero halo, 10 Jacobi steps", "cases": {}}
    cases = [(2, st.BOX, r) for r in (1, 2, 3)] + [(2, st.STAR, r) for r in (1, 2, 3)]
    cases += [(3, st.BOX, r) for r in (1, 2)] + [(3, st.STAR, r) for r in (1, 2, 3)]

    def timed(batch):
        for _ in range(max(args.warmup, 1)):
            batch.run_steps(steps, stream=stream)
        torch.cuda.synchronize()
        times = []
        for _ in range(max(args.steps, 3)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            batch.run_steps(steps, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        return total_pts * steps / (np.median(times) * 1e-3) / 1e9

    for nd, shape, r in cases:
        sizes = (64, 128, 256, 512) if nd == 2 else (8, 16, 32, 64)
        for n in sizes:
            dims = (n,) * nd
            pts = n ** nd
            count = total_pts // pts
            c = inputs.coefficients(nd, r, shape, seed=8000 + 10 * nd + r + 100 * shape, dtype=np.float64)
            a0 = torch.from_numpy(inputs.grid((count,) + dims, seed=8001, dtype=np.float64)).cuda()
            key = f"{nd}d_{'box' if shape == st.BOX else 'star'}_r{r}_{n}"
            entry = {"grids": count}
            for name, path in (("mfma", st.PATH_MFMA), ("gather", st.PATH_GATHER), ("auto", st.PATH_AUTO)):
                plan = st.Plan(dims, r, shape, c, boundary=st.BC_ZERO, dtype=st.F64, path=path)
                b0 = a0.clone()
                b1 = torch.empty_like(b0)
                batch = st.Batch([plan] * count, list(b0.unbind(0)), list(b1.unbind(0)))
                entry[f"{name}_batched_gstencil_s"] = round(timed(batch), 2)
                if name == "auto":
                    info = batch.info()
                    entry.update({"auto_path": st.PATH_NAMES[plan.info["path"]],
                                  "auto_time_block": plan.info["time_block"], "items": info["items"],
                                  "workgroups": info["blocks"]})
                    # one by one: a sample of the grids, each launched eagerly step by step
                    ns = min(count, 64)
                    x = a0[:ns].clone()
                    y = torch.empty_like(x)
                    os.environ["STENCIL_NO_GRAPH"] = "1"
                    try:
                        for k in range(ns):
                            plan.run_steps(x[k], y[k], steps, stream=stream)
                        torch.cuda.synchronize()
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        for k in range(ns):
                            plan.run_steps(x[k], y[k], steps, stream=stream)
                        e1.record(stream)
                        torch.cuda.synchronize()
                    finally:
                        del os.environ["STENCIL_NO_GRAPH"]
                    entry["auto_one_by_one_gstencil_s"] = round(ns * pts * steps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 3)
                    del x, y
                batch.close()
                plan.close()
                del b0, b1
            entry["mfma_vs_gather"] = round(entry["mfma_batched_gstencil_s"] / entry["gather_batched_gstencil_s"], 3)
            # AUTO (time-blocked classes where the library time-blocks) against
            # the faster one-step path
            entry["auto_vs_one_step"] = round(entry["auto_batched_gstencil_s"] / max(
                entry["mfma_batched_gstencil_s"], entry["gather_batched_gstencil_s"]), 3)
            entry["batched_vs_one_by_one"] = round(entry["auto_batched_gstencil_s"] / entry["auto_one_by_one_gstencil_s"], 1)
            out["cases"][key] = entry
            print(f"[bench] batch {key}: mfma {entry['mfma_batched_gstencil_s']:.1f}, gather "
                  f"{entry['gather_batched_gstencil_s']:.1f}, auto {entry['auto_batched_gstencil_s']:.1f} GStencil/s batched "
                  f"(mfma/gather x{entry['mfma_vs_gather']}); auto one by one {entry['auto_one_by_one_gstencil_s']:.2f} "
                  f"({count} grids)", file=sys.stderr, flush=True)
            del a0
            torch.cuda.empty_cache()
    return out


def workload_tune(args, torch, st, inputs) -> dict:
    """The autotuner over line option x MFMA block x register/workgroup tile x
    time block x chunk, per radius: 2D
    box/star r = 1..4 at 8192^2 FP32 (periodic), 3D star r = 1..4 and the
    27-point box at 512^3 FP32 (zero halo), 2D box/star r = 1..3 at 512^2 FP64
    (zero halo): every measured candidate and the winner."""
    out = {"metric": "ms per Jacobi step of each candidate plan", "cases": {}}
    names = {st.LINES_AUTO: "-", st.LINES_PARALLEL: "p", st.LINES_ORTHOGONAL: "o", st.LINES_HYBRID: "h"}
    specs = [((8192, 8192), st.F32, st.BC_PERIODIC, shape, r) for shape in (st.BOX, st.STAR) for r in (1, 2, 3, 4)]
    specs += [((512, 512, 512), st.F32, st.BC_ZERO, st.STAR, r) for r in (1, 2, 3, 4)]
    specs += [((512, 512, 512), st.F32, st.BC_ZERO, st.BOX, 1)]
    specs += [((512, 512), st.F64, st.BC_ZERO, shape, r) for shape in (st.BOX, st.STAR) for r in (1, 2, 3)]
    for dims, dt, bc, shape, r in specs:
        c = inputs.coefficients(len(dims), r, shape, seed=9500 + r, dtype=np.float64)
        knobs, ms, rows = st.autotune(dims, r, shape, c, boundary=bc, dtype=dt, force=True)
        pts = float(np.prod(dims))
        key = (f"{len(dims)}d_{'box' if shape == st.BOX else 'star'}_r{r}_{'x'.join(map(str, dims))}_"
               f"{'f64' if dt == st.F64 else 'f32'}")
        out["cases"][key] = {
            "winner": {"path": st.PATH_NAMES[knobs["path"]], "lines": names[knobs["lines"]],
                       "block_n": knobs["block_n"], "chunk": knobs["chunk"], "time_block": knobs["time_block"],
                       "reg_rows": knobs["reg_rows"], "tile_width": knobs["tile_width"],
                       "ms_per_step": round(ms, 5), "gstencil_s": round(pts / (ms * 1e-3) / 1e9, 2)},
            "candidates": [{"path": st.PATH_NAMES[row["path"]], "lines": names[row["lines"]],
                            "block_n": row["block_n"], "chunk": row["chunk"], "time_block": row["time_block"],
                            "reg_rows": row["reg_rows"], "tile_width": row["tile_width"],
                            "gstencil_s": round(pts / (row["ms_per_step"] * 1e-3) / 1e9, 2)} for row in rows]}
        w = out["cases"][key]["winner"]
        print(f"[bench] tune {key}: {w['path']} lines={w['lines']} n={w['block_n']} chunk={w['chunk']} "
              f"T={w['time_block']} {w['gstencil_s']} GStencil/s ({len(rows)} candidates)", file=sys.stderr, flush=True)
    out["data_sensitivity"] = data_sensitivity(args, torch, st, inputs)
    return out


def data_sensitivity(args, torch, st, inputs) -> dict:
    """Why the tuner times candidates on seeded data: GStencil/s of a 100-step
    solve (8192^2 FP32 box, periodic) from a zeroed grid and from the seeded
    headline grid, for the MFMA outer products, the one-step gather and the
    library's time block, r = 1..4 (median of --steps runs)."""
    stream = torch.cuda.Stream()
    seeded = torch.from_numpy(inputs.grid(DIMS, seed=INPUT_SEED, dtype=np.float32)).cuda()
    zero = torch.zeros_like(seeded)
    res = {}
    for r in RADII:
        c = inputs.coefficients(2, r, inputs.BOX, seed=COEF_SEED0 + r, dtype=np.float64)
        row = {}
        for name, knobs in (("mfma", {"path": st.PATH_MFMA}), ("gather", {"path": st.PATH_GATHER}),
                            ("auto", {})):
            plan = st.Plan(DIMS, r, st.BOX, c, boundary=st.BC_PERIODIC, dtype=st.F32, **knobs)
            for label, x0 in (("zero", zero), ("seeded", seeded)):
                times = _time_solve(torch, plan, x0, JACOBI_STEPS, max(args.steps, 3), 1, stream)
                row[f"{name}_{label}"] = round(float(DIMS[0] * DIMS[1] * JACOBI_STEPS / (np.median(times) * 1e-3) / 1e9), 1)
            plan.close()
        res[f"box_r{r}"] = row
        print(f"[bench] data sensitivity r={r}: {row}", file=sys.stderr, flush=True)
    return res


def _serve_requests(n, st):
    """Seeded request stream (stream seed 501): 2D/3D 50/50, square/cube side
    log-uniform on [64, 4096] (2D) or [32, 512] (3D), r uniform on 1..4,
    star/box 50/50, steps uniform on 1..200, zero/periodic 50/50, FP32."""
    rng = np.random.default_rng(501)
    reqs = []
    for k in range(n):
        nd = 2 if rng.random() < 0.5 else 3
        lo, hi = (64, 4096) if nd == 2 else (32, 512)
        side = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
        reqs.append({"id": k, "dims": (side,) * nd, "r": int(rng.integers(1, 5)),
                     "shape": st.STAR if rng.random() < 0.5 else st.BOX, "steps": int(rng.integers(1, 201)),
                     "bc": st.BC_ZERO if rng.random() < 0.5 else st.BC_PERIODIC})
    return reqs


def _serve_run(torch, st, inputs, srv, reqs, arrivals, keep_ids=()):
    """Drive the server: submit each request at its arrival time (seconds
    from the start), tick while work is resident or queued, record completion
    times at poll.  Returns (latency_s by id, wall seconds, outputs kept)."""
    stream = srv.stream()
    t0 = time.perf_counter()
    nxt, busy = 0, 0
    by_rid, lat, kept = {}, {}, {}
    total = len(reqs)
    last_note = 0.0
    while len(lat) < total:
        now = time.perf_counter() - t0
        if now - last_note > 10.0:
            print(f"[serve] t={now:.0f}s submitted={nxt} done={len(lat)} of {total}", file=sys.stderr, flush=True)
            last_note = now
        while nxt < total and arrivals[nxt] <= now:
            q = reqs[nxt]
            g = torch.Generator(device="cuda")
            g.manual_seed(5000 + q["id"])
            with torch.cuda.stream(stream):
                x = torch.rand(q["dims"], generator=g, device="cuda", dtype=torch.float32) * 2 - 1
                out = torch.empty_like(x)
            c = inputs.coefficients(len(q["dims"]), q["r"], q["shape"], seed=5000 + q["id"], dtype=np.float64)
            rid = srv.submit(x, out, q["steps"], q["r"], q["shape"], c, boundary=q["bc"])
            by_rid[rid] = (q, out, arrivals[nxt], c, x if q["id"] in keep_ids else None)
            nxt += 1
            busy += 1
        if busy:
            srv.tick()
        elif nxt < total:
            time.sleep(max(0.0, min(arrivals[nxt] - now, 0.0005)))
        for rid in srv.poll():
            q, out, arr, c, x = by_rid.pop(rid)
            lat[q["id"]] = time.perf_counter() - t0 - arr
            busy -= 1
            if q["id"] in keep_ids:
                kept[q["id"]] = (q, c, x.cpu().numpy(), out.cpu().numpy())
    torch.cuda.synchronize()
    return lat, time.perf_counter() - t0, kept


def workload_serve(args, torch, st, inputs) -> dict:
    """Serving: Poisson arrivals of the seeded request stream at offered
    loads 0.5 and 0.8 of the server's calibrated closed-loop throughput;
    p50/p99 of completion - arrival, aggregate GStencil/s, and results of
    sampled requests equal (bitwise) to the same request run alone."""
    n_warm, n_meas = args.serve_warmup, args.serve_requests
    reqs = _serve_requests(n_warm + n_meas, st)
    pts = {q["id"]: float(np.prod(q["dims"])) * q["steps"] for q in reqs}
    out = {"metric": "completion - arrival latency p50/p99 (ms) and aggregate GStencil/s",
           "workload": f"{n_warm} warm-up + {n_meas} measured requests per load; 2D side log-uniform[64,4096], "
                       "3D side log-uniform[32,512], r 1..4, star/box, steps 1..200, zero/periodic, FP32",
           "arena_gib": args.serve_arena_gib, "loads": {}}
    srv = st.Server(args.serve_arena_gib << 30, max_inflight_ticks=4)
    # closed loop: everything arrives at once
    cal = reqs[:min(len(reqs), 150)]
    lat, wall, _ = _serve_run(torch, st, inputs, srv, cal, [0.0] * len(cal))
    thr_req = len(cal) / wall
    thr_pts = sum(pts[q["id"]] for q in cal) / wall
    out["closed_loop"] = {"requests": len(cal), "requests_per_s": round(thr_req, 2),
                          "gstencil_s": round(thr_pts / 1e9, 2)}
    print(f"[bench] serve closed loop: {thr_req:.1f} req/s, {thr_pts / 1e9:.1f} GStencil/s", file=sys.stderr,
          flush=True)
    rng = np.random.default_rng(502)
    for rho in (0.5, 0.8):
        lam = rho * thr_req
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=len(reqs)))
        arrivals -= arrivals[0]
        sample = [q["id"] for q in reqs[n_warm:] if np.prod(q["dims"]) <= 300 * 300][:6]
        lat, wall, kept = _serve_run(torch, st, inputs, srv, reqs, arrivals, keep_ids=set(sample))
        meas = [q["id"] for q in reqs[n_warm:]]
        ms = np.array([lat[i] for i in meas]) * 1e3
        t_first = arrivals[n_warm]
        t_last = max(arrivals[i] + lat[i] for i in meas)
        g = sum(pts[i] for i in meas) / (t_last - t_first) / 1e9
        equal = []
        for rid, (q, c, x, got) in kept.items():
            plan = st.Plan(q["dims"], q["r"], q["shape"], c, boundary=q["bc"], dtype=st.F32)
            xd = torch.from_numpy(x).cuda()
            res = plan.run_steps(xd, torch.empty_like(xd), q["steps"])
            torch.cuda.synchronize()
            equal.append(bool(np.array_equal(res.cpu().numpy(), got)))
            plan.close()
        out["loads"][str(rho)] = {"offered_requests_per_s": round(lam, 2), "p50_ms": round(float(np.percentile(ms, 50)), 3),
                                  "p99_ms": round(float(np.percentile(ms, 99)), 3),
                                  "mean_ms": round(float(ms.mean()), 3), "gstencil_s": round(g, 2),
                                  "hbm_frac_1step_equiv": round(g * 8 / HBM_PEAK_GBS, 4),
                                  "alone_equals_mix": {"checked": len(equal), "equal": int(sum(equal))}}
        print(f"[bench] serve rho={rho}: p50 {np.percentile(ms, 50):.2f} ms, p99 {np.percentile(ms, 99):.2f} ms, "
              f"{g:.1f} GStencil/s, alone==mix {sum(equal)}/{len(equal)}", file=sys.stderr, flush=True)
    srv.close()
    return out


def workload_cover(args, torch, st, inputs) -> dict:
    """Irregular 2D stencils of order 4 on 8192^2 FP32 (periodic, 100 steps):
    the outer-product form over a minimum line cover (GENERAL), the gather
    over the nonzero taps, the AUTO choice between them, and the same weights
    as a box (all 9 lines on MFMA / all 81 taps gathered)."""
    dims, r, steps = (8192, 8192), 4, 100
    w = 2 * r + 1
    z = np.zeros((w, w), dtype=bool)
    pats = {}
    m = z.copy(); m[r, :] = True; m[:, r] = True; m[0, 0] = m[w - 1, w - 1] = True; pats["cross_plus_two_corners"] = m
    m = z.copy(); m[w - 1, :] = True; m[:, 0] = True; pats["l_shape"] = m
    m = z.copy(); m[1, :] = True; m[5, :] = True; m[:, 2] = True; pats["two_rows_one_column"] = m
    pats["random_25pct"] = np.random.default_rng(6100).random((w, w)) < 0.25
    m = z.copy(); np.fill_diagonal(m, True); pats["diagonal"] = m
    m = z.copy(); np.fill_diagonal(m, True); m[np.arange(w), w - 1 - np.arange(w)] = True; pats["both_diagonals"] = m
    if args.patterns:
        pats = {k: v for k, v in pats.items() if k in args.patterns.split(",")}
    a0 = torch.from_numpy(inputs.grid(dims, seed=6000, dtype=np.float32)).cuda()
    stream = torch.cuda.Stream()
    out = {"metric": "GStencil/s", "workload": "2D order-4 irregular stencils, 8192^2 FP32, periodic, 100 steps",
           "cases": {}}
    for name, mask in pats.items():
        c = np.where(mask, np.random.default_rng(6200).uniform(0.05, 1.0, size=(w, w)), 0.0)
        c /= c.sum()
        rows, cols = st.line_cover(c, r)
        res = {"nonzeros": int(mask.sum()), "cover_lines": len(rows) + len(cols)}
        for label, shape, path in (("general_mfma_cover", st.GENERAL, st.PATH_MFMA),
                                   ("general_gather_nonzero_taps", st.GENERAL, st.PATH_GATHER),
                                   ("general_auto", st.GENERAL, st.PATH_AUTO),
                                   ("box_mfma_all_columns", st.BOX, st.PATH_MFMA),
                                   ("box_gather_all_taps", st.BOX, st.PATH_GATHER)):
            plan = st.Plan(dims, r, shape, c, boundary=st.BC_PERIODIC, dtype=st.F32, path=path)
            times = _time_solve(torch, plan, a0, steps, args.steps, args.warmup, stream)
            res[label] = round(float(dims[0] * dims[1] * steps / (np.median(times) * 1e-3) / 1e9), 2)
            if shape == st.GENERAL and path == st.PATH_MFMA:
                res["plan_lines"] = plan.info["mfma_lines"]
            if path == st.PATH_AUTO:
                res["auto_path"] = st.PATH_NAMES[plan.info["path"]]
            plan.close()
        out["cases"][name] = res
        print(f"[bench] cover {name}: {res}", file=sys.stderr, flush=True)
    return out


def workload_cover_sweep(args, torch, st, inputs) -> dict:
    """GENERAL 2D stencils of orders 1..4, FP32 and FP64, 8192^2 periodic, 50
    steps: the nonzero-tap gather, the all-tap gather (the same weights as a
    box), the line cover on MFMA and the AUTO choice, on four patterns of
    growing density (one diagonal, ~25 % and ~45 % random, one row plus one
    column)."""
    dims, steps = (8192, 8192), 50
    stream = torch.cuda.Stream()
    out = {"metric": "GStencil/s", "workload": "2D GENERAL stencils r=1..4, 8192^2 FP32/FP64, periodic, 50 steps",
           "cases": {}}
    for dt, ndt, tag in ((st.F32, np.float32, "f32"), (st.F64, np.float64, "f64")):
        x0 = torch.from_numpy(inputs.grid(dims, seed=6200, dtype=ndt)).cuda()
        for r in (1, 2, 3, 4):
            w = 2 * r + 1
            rng = np.random.default_rng(6300 + r)
            rc = np.zeros((w, w), dtype=bool)
            rc[0, :] = True
            rc[:, w - 1] = True
            pats = {"diagonal": np.eye(w, dtype=bool), "random_25pct": rng.random((w, w)) < 0.25,
                    "random_45pct": rng.random((w, w)) < 0.45, "row_and_column": rc}
            for name, m in pats.items():
                c = np.where(m, 1.0 / max(1, int(m.sum())), 0.0)
                res = {"nonzeros": int(m.sum())}
                for label, shape, path in (("nonzero_tap_gather", st.GENERAL, st.PATH_GATHER),
                                           ("all_tap_gather", st.BOX, st.PATH_GATHER),
                                           ("line_cover_mfma", st.GENERAL, st.PATH_MFMA),
                                           ("auto", st.GENERAL, st.PATH_AUTO)):
                    plan = st.Plan(dims, r, shape, c, boundary=st.BC_PERIODIC, dtype=dt, path=path)
                    times = _time_solve(torch, plan, x0, steps, args.steps, args.warmup, stream)
                    res[label] = round(float(dims[0] * dims[1] * steps / (np.median(times) * 1e-3) / 1e9), 1)
                    if label == "nonzero_tap_gather":
                        res["gather_taps_run"] = int(plan.info["executed_flops_per_point"] // 2)
                    if label == "line_cover_mfma":
                        res["lines"] = plan.info["mfma_lines"]
                    if label == "auto":
                        res["auto_path"] = st.PATH_NAMES[plan.info["path"]]
                    plan.close()
                key = f"{tag}_r{r}_{name}"
                out["cases"][key] = res
                print(f"[bench] cover_sweep {key}: {res}", file=sys.stderr, flush=True)
        del x0
    return out


def workload_general3d(args, torch, st, inputs) -> dict:
    """GENERAL 3D stencils of orders 1..4, FP32 and FP64, 256^3 periodic, 20
    steps: the nonzero-tap gather, the all-tap gather (the same weights as a
    box), the outer products over every line (MFMA) and the AUTO choice, for
    n random nonzero taps (n = 2r+1 on the space diagonal, then 16, 32, 64,
    128 where the box holds them)."""
    dims, steps = (256, 256, 256), 20
    stream = torch.cuda.Stream()
    out = {"metric": "GStencil/s", "workload": "3D GENERAL stencils r=1..4, 256^3 FP32/FP64, periodic, 20 steps",
           "cases": {}}
    for dt, ndt, tag in ((st.F32, np.float32, "f32"), (st.F64, np.float64, "f64")):
        x0 = torch.from_numpy(inputs.grid(dims, seed=6400, dtype=ndt)).cuda()
        for r in (1, 2, 3, 4):
            w = 2 * r + 1
            rng = np.random.default_rng(6500 + r)
            pats = {"space_diagonal": np.zeros((w, w, w), dtype=bool)}
            pats["space_diagonal"][np.arange(w), np.arange(w), np.arange(w)] = True
            for n in (16, 32, 64, 128):
                if n < w ** 3:
                    m = np.zeros(w ** 3, dtype=bool)
                    m[rng.choice(w ** 3, size=n, replace=False)] = True
                    pats[f"random_{n}"] = m.reshape(w, w, w)
            for name, m in pats.items():
                c = np.where(m, 1.0 / max(1, int(m.sum())), 0.0)
                res = {"nonzeros": int(m.sum())}
                cols = [("nonzero_tap_gather", st.GENERAL, st.PATH_GATHER), ("all_tap_gather", st.BOX, st.PATH_GATHER),
                        ("auto", st.GENERAL, st.PATH_AUTO)]
                if dt == st.F32 or r <= 2:  # FP64 3D boxes have outer products up to r = 2
                    cols.insert(2, ("box_mfma", st.BOX, st.PATH_MFMA))
                for label, shape, path in cols:
                    plan = st.Plan(dims, r, shape, c, boundary=st.BC_PERIODIC, dtype=dt, path=path)
                    times = _time_solve(torch, plan, x0, steps, args.steps, args.warmup, stream)
                    res[label] = round(float(np.prod(dims) * steps / (np.median(times) * 1e-3) / 1e9), 1)
                    if label == "nonzero_tap_gather":
                        res["gather_taps_run"] = int(plan.info["executed_flops_per_point"] // 2)
                    if label == "auto":
                        res["auto_path"] = st.PATH_NAMES[plan.info["path"]]
                    plan.close()
                key = f"{tag}_r{r}_{name}"
                out["cases"][key] = res
                print(f"[bench] general3d {key}: {res}", file=sys.stderr, flush=True)
        del x0
    return out


def _drift_run(torch, st, plan, shadow_plan, x0, sh0, checks, every, oracle_states=None):
    """Advance the FP32 state and its FP64 shadow `every` steps at a time;
    at each check the rel-L2 / max-abs of the state against the shadow (GPU)
    and, when given, against the CPU FP64 oracle's state of that step."""
    x = x0.clone()
    tmp = torch.empty_like(x)
    s64 = sh0.clone()
    sh_tmp = torch.empty_like(s64)
    drift = []
    for k in range(checks):
        res = plan.run_steps(x, tmp, every)
        if res.data_ptr() != x.data_ptr():
            x, tmp = tmp, x
        r64 = shadow_plan.run_steps(s64, sh_tmp, every)
        if r64.data_ptr() != s64.data_ptr():
            s64, sh_tmp = sh_tmp, s64
        nrm = st.error_norms(x, s64).cpu().numpy()
        d = {"step": every * (k + 1), "rel_l2": float(np.sqrt(nrm[0] / nrm[1])), "max_abs": float(nrm[2])}
        if oracle_states is not None:
            want = oracle_states[k]
            got = x.cpu().numpy().astype(np.float64)
            diff = got - want
            d["rel_l2_vs_cpu_oracle"] = float(np.sqrt((diff * diff).sum() / (want * want).sum()))
            d["max_abs_vs_cpu_oracle"] = float(np.abs(diff).max())
            d["shadow_vs_cpu_oracle_max_abs"] = float(np.abs(s64.cpu().numpy() - want).max())
        drift.append(d)
    return drift


MIXED_SPECS = [("box2d_r2_4096", (4096, 4096), 2, 1, 401, 4100),   # shape 1 = BOX
               ("star3d_r4_384", (384, 384, 384), 4, 0, 402, 4200)]  # shape 0 = STAR


def workload_tiles(args, torch, st, inputs) -> dict:
    """The unrolling study of Section 4.2 (Fig. 4) on MI355X: the FP32 box
    outer products on n = 4 blocks at 8192^2 (periodic, 50 steps) for every
    register tile (8 / 16 / 32 output rows per wave: two, four or eight 4-row
    accumulator blocks, the i unrolling) and workgroup tile (256 columns: four
    waves side by side; 128: two rows of two waves), r = 1..4."""
    dims, steps = DIMS, 50
    stream = torch.cuda.Stream()
    a0 = torch.from_numpy(inputs.grid(dims, seed=INPUT_SEED, dtype=np.float32)).cuda()
    out = {"metric": "GStencil/s", "workload": f"2D box r=1..4, {dims[0]}x{dims[1]} FP32, periodic, {steps} steps, "
           "MFMA path on n = 4 blocks", "cases": {}}
    for r in RADII:
        c = inputs.coefficients(2, r, inputs.BOX, seed=COEF_SEED0 + r, dtype=np.float64)
        res = {}
        for rows in (8, 16, 32):
            for width in (256, 128):
                plan = st.Plan(dims, r, st.BOX, c, boundary=st.BC_PERIODIC, dtype=st.F32, path=st.PATH_MFMA,
                               reg_rows=rows, tile_width=width)
                times = _time_solve(torch, plan, a0, steps, args.steps, args.warmup, stream)
                res[f"{rows}x{width}"] = round(float(dims[0] * dims[1] * steps / (np.median(times) * 1e-3) / 1e9), 1)
                plan.close()
        out["cases"][f"r{r}"] = res
        print(f"[bench] tiles r={r}: {res}", file=sys.stderr, flush=True)
    return out


def workload_mixed(args, torch, st, inputs) -> dict:
    """BF16x3 / FP16x3 outer products with FP32 state for 200 steps, beside the
    FP32 paths; an FP64 shadow trajectory (FP64 gather path) on the GPU and
    the CPU FP64 oracle on the whole grid; rel-L2 and max-abs of the state
    against both every 50 steps."""
    import oracle
    oracle.build(force=False)
    threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    out = {"metric": "GStencil/s and drift vs FP64 (GPU shadow and CPU oracle, whole grid)", "cases": {},
           "cpu_oracle_threads": threads}
    stream = torch.cuda.Stream()
    nsteps = args.solve_steps or 200
    checks = max(1, nsteps // 50)
    want_cases = set(args.cases.split(",")) if args.cases else None
    want_paths = set(args.paths3d.split(",")) if args.paths3d else None
    for key, dims, r, shape, iseed, cseed in MIXED_SPECS:
        if want_cases is not None and key not in want_cases:
            continue
        nd = len(dims)
        c = inputs.coefficients(nd, r, shape, seed=cseed, dtype=np.float64)
        c32 = c.astype(np.float32).astype(np.float64)
        a32 = inputs.grid(dims, seed=iseed, dtype=np.float32)
        states = None
        out["cases"][key] = {}
        if not args.no_oracle:
            # the CPU oracle's states at steps 50, 100, 150, 200 (whole grid, FP64)
            t0 = time.perf_counter()
            states, cur = [], a32.astype(np.float64)
            for k in range(checks):
                cur = oracle.run(cur, c32, r, shape, st.BC_ZERO, 50)
                states.append(cur)
                print(f"[bench] {key}: CPU oracle at step {50 * (k + 1)} ({time.perf_counter() - t0:.0f} s)",
                      file=sys.stderr, flush=True)
            out["cases"][key]["cpu_oracle_seconds"] = round(time.perf_counter() - t0, 1)
            del cur
        x0 = torch.from_numpy(a32).cuda()
        shadow_plan = st.Plan(dims, r, shape, c32, boundary=st.BC_ZERO, dtype=st.F64, path=st.PATH_GATHER)
        sh = x0.double()
        for name, path in (("mfma_bf16x3", st.PATH_MFMA_BF16X3), ("mfma_f16x3", st.PATH_MFMA_F16X3),
                           ("mfma", st.PATH_MFMA), ("gather", st.PATH_GATHER), ("auto", st.PATH_AUTO)):
            if want_paths is not None and name not in want_paths:
                continue
            plan = st.Plan(dims, r, shape, c, boundary=st.BC_ZERO, dtype=st.F32, path=path)
            times = _time_solve(torch, plan, x0, nsteps, args.steps, args.warmup, stream)
            g = float(np.prod(dims)) * nsteps / (np.median(times) * 1e-3) / 1e9
            entry = {"gstencil_s": round(g, 2), "hbm_frac": hbm_frac(g, 8, plan.info["time_block"]),
                     "resolved_path": st.PATH_NAMES[plan.info["path"]], "time_block": plan.info["time_block"]}
            if name != "auto":
                drift = _drift_run(torch, st, plan, shadow_plan, x0, sh, checks, 50, states)
                entry["drift"] = drift
                msg = f"rel_l2 vs shadow {drift[-1]['rel_l2']:.2e}"
                if states is not None:
                    msg += (f", vs oracle {drift[-1]['rel_l2_vs_cpu_oracle']:.2e} "
                            f"(max_abs {drift[-1]['max_abs_vs_cpu_oracle']:.2e})")
            else:
                msg = f"path {entry['resolved_path']}"
            out["cases"][key][name] = entry
            print(f"[bench] {key} {name}: {g:.1f} GStencil/s; {msg}", file=sys.stderr, flush=True)
            plan.close()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        sh_tmp = torch.empty_like(sh)
        t0.record(stream)
        shadow_plan.run_steps(sh.clone(), sh_tmp, nsteps, stream=stream)
        t1.record(stream)
        torch.cuda.synchronize()
        out["cases"][key][f"fp64_shadow_ms_per_{nsteps}_steps"] = t0.elapsed_time(t1)
        shadow_plan.close()
        del x0, sh, sh_tmp, states
        torch.cuda.empty_cache()
    return out


def config_extras(args, torch, st, inputs) -> dict:
    """The other benchmark configurations in compact form for the default
    line (a few repetitions each):
      star2d_512_fp64 -- 2D five-point star, 512^2 FP64, zero halo, 10 steps:
                         AUTO latency p50/p99 and the CPU oracle's time;
      grid3d_512      -- 3D stars r = 1..4 and the 27-point box, 512^3 FP32
                         and FP64, zero halo, 50 steps, AUTO path;
      mixed_200       -- 2D box r = 2 at 4096^2 and 3D star r = 4 at 384^3,
                         200 steps, BF16x3 / FP16x3 beside the FP32 paths,
                         drift against the FP64 GPU shadow at step 200."""
    import oracle
    stream = torch.cuda.Stream()
    ex = {}
    # config: 512^2 FP64 five-point star
    dims, steps = (512, 512), 10
    c = inputs.diffusion_5pt()
    a0 = inputs.grid(dims, seed=101, dtype=np.float64)
    x0 = torch.from_numpy(a0).cuda()
    plan = st.Plan(dims, 1, st.STAR, c, boundary=st.BC_ZERO, dtype=st.F64)
    times = _time_solve(torch, plan, x0, steps, 50, 5, stream)
    res = plan.run_steps(x0.clone(), torch.empty_like(x0), steps)
    torch.cuda.synchronize()
    oracle.build(force=False)
    used = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    t0 = time.perf_counter()
    want = oracle.run(a0, c, 1, st.STAR, st.BC_ZERO, steps)
    cpu_s = time.perf_counter() - t0
    ex["star2d_512_fp64"] = {"path": st.PATH_NAMES[plan.info["path"]], "time_block": plan.info["time_block"],
                             "p50_us": round(float(np.percentile(times, 50)) * 1e3, 1),
                             "p99_us": round(float(np.percentile(times, 99)) * 1e3, 1),
                             "gstencil_s": round(dims[0] * dims[1] * steps / (np.median(times) * 1e-3) / 1e9, 2),
                             "max_abs_err_vs_oracle": float(np.abs(res.cpu().numpy() - want).max()),
                             "cpu_oracle_s": round(cpu_s, 4), "cpu_threads": used}
    plan.close()
    print(f"[bench] extra star2d_512_fp64: {ex['star2d_512_fp64']}", file=sys.stderr, flush=True)
    # config: 512^3 3D stars and 27-point box, FP32 and FP64, AUTO
    dims, steps = (512, 512, 512), 50
    a64 = inputs.grid(dims, seed=301, dtype=np.float64)
    g3 = {}
    for dt, ndt, tag, bpp in ((st.F32, np.float32, "f32", 8), (st.F64, np.float64, "f64", 16)):
        x0 = torch.from_numpy(a64.astype(ndt)).cuda()
        for shape, r in [(st.STAR, 1), (st.STAR, 2), (st.STAR, 3), (st.STAR, 4), (st.BOX, 1)]:
            c = inputs.coefficients(3, r, shape, seed=3100 + 10 * shape + r, dtype=np.float64)
            plan = st.Plan(dims, r, shape, c, boundary=st.BC_ZERO, dtype=dt)
            times = _time_solve(torch, plan, x0, steps, 3, 1, stream)
            g = float(np.prod(dims)) * steps / (np.median(times) * 1e-3) / 1e9
            tb = plan.info["time_block"]
            g3[f"{tag}_{'box' if shape == st.BOX else 'star'}_r{r}"] = {
                "path": st.PATH_NAMES[plan.info["path"]], "time_block": tb, "gstencil_s": round(g, 1),
                "hbm_frac": hbm_frac(g, bpp, tb)}
            plan.close()
        del x0
        torch.cuda.empty_cache()
    del a64
    ex["grid3d_512"] = g3
    print(f"[bench] extra grid3d_512: {g3}", file=sys.stderr, flush=True)
    # config: mixed precision, 200 steps, drift at 200 against the FP64 shadow
    mx = {}
    for key, dims, r, shape, iseed, cseed in MIXED_SPECS:
        nd = len(dims)
        c = inputs.coefficients(nd, r, shape, seed=cseed, dtype=np.float64)
        c32 = c.astype(np.float32).astype(np.float64)
        x0 = torch.from_numpy(inputs.grid(dims, seed=iseed, dtype=np.float32)).cuda()
        shadow_plan = st.Plan(dims, r, shape, c32, boundary=st.BC_ZERO, dtype=st.F64, path=st.PATH_GATHER)
        sh = x0.double()
        mx[key] = {}
        for name, path in (("mfma_bf16x3", st.PATH_MFMA_BF16X3), ("mfma_f16x3", st.PATH_MFMA_F16X3),
                           ("mfma", st.PATH_MFMA), ("gather", st.PATH_GATHER), ("auto", st.PATH_AUTO)):
            plan = st.Plan(dims, r, shape, c, boundary=st.BC_ZERO, dtype=st.F32, path=path)
            times = _time_solve(torch, plan, x0, 200, 3, 1, stream)
            g = float(np.prod(dims)) * 200 / (np.median(times) * 1e-3) / 1e9
            e = {"gstencil_s": round(g, 1), "hbm_frac": hbm_frac(g, 8, plan.info["time_block"])}
            if name.startswith("mfma_"):
                d = _drift_run(torch, st, plan, shadow_plan, x0, sh, 1, 200)[-1]
                e.update({"rel_l2_200": d["rel_l2"], "max_abs_200": d["max_abs"]})
            if name == "auto":
                e["path"] = st.PATH_NAMES[plan.info["path"]]
                e["time_block"] = plan.info["time_block"]
            mx[key][name] = e
            plan.close()
        shadow_plan.close()
        del x0, sh
        torch.cuda.empty_cache()
    ex["mixed_200"] = mx
    print(f"[bench] extra mixed_200: {mx}", file=sys.stderr, flush=True)
    return ex


def main() -> int:
    global RADII, JACOBI_STEPS
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed bench steps (one step = 4 solves x 100 Jacobi steps)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--headline", default="auto",
                    choices=["auto", "mfma", "gather", "mfma_f16x3", "mfma_bf16x3", "gather_tb", "mfma_tb2", "tuned"])
    ap.add_argument("--paths", default="gather,mfma,mfma_f16x3,mfma_bf16x3,gather_tb,mfma_tb2,tuned,auto",
                    help="gather_tb: time-blocked gather (largest time block); tuned: the autotuner's plan")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations' compact results in the default line")
    ap.add_argument("--radii", default="1,2,3,4", help="orders to run (profiling runs use a subset)")
    ap.add_argument("--jacobi-steps", type=int, default=JACOBI_STEPS,
                    help="Jacobi steps per solve (profiling runs only; the benchmark uses 100)")
    ap.add_argument("--workload", default="box2d", choices=["box2d", "star2d_512", "grid3d", "mixed", "batch", "tune", "serve", "cover", "cover_sweep", "general3d",
                             "tiles"])
    ap.add_argument("--patterns", default="", help="cover workload: comma-separated pattern names (default all)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured requests per offered load")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-arena-gib", type=int, default=64)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="first run N plain device copies of one grid (known bytes) for counter scaling")
    ap.add_argument("--cases", default="", help="grid3d / mixed: comma-separated case keys (default all)")
    ap.add_argument("--paths3d", default="", help="grid3d / mixed: comma-separated path names (default all)")
    ap.add_argument("--solve-steps", type=int, default=0,
                    help="grid3d / mixed: Jacobi steps per solve (profiling runs only; default 50 / 200)")
    ap.add_argument("--no-oracle", action="store_true", help="mixed: skip the CPU oracle (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library runs each plan on one device and bench.py does not launch ranks.",
              file=sys.stderr)
        return 2

    import torch
    from paper_2310_16298_amd import inputs
    from paper_2310_16298_amd import stencil as st

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    st.load_library()
    if args.calibrate_copy:
        # a plain device copy of 2^26 FP32 values (268,435,456 bytes read and written) per repetition:
        # the reference reading for scaling the FETCH_SIZE / WRITE_SIZE counters of the kernels
        src = torch.empty(1 << 26, dtype=torch.float32, device="cuda").uniform_(-1.0, 1.0)
        dst = torch.empty_like(src)
        for _ in range(args.calibrate_copy):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration: {args.calibrate_copy} copies of {src.numel() * 4} bytes", file=sys.stderr)
        del src, dst
    if args.workload != "box2d":
        fn = {"star2d_512": workload_star2d_512, "grid3d": workload_grid3d, "mixed": workload_mixed,
              "batch": workload_batch, "tune": workload_tune, "serve": workload_serve,
              "cover": workload_cover, "cover_sweep": workload_cover_sweep,
              "general3d": workload_general3d, "tiles": workload_tiles}[args.workload]
        res = fn(args, torch, st, inputs)
        res.update({"n_gpus": 1, "data": "synthetic"})
        print(json.dumps(res))
        return 0
    name_to_path = {"gather": st.PATH_GATHER, "mfma": st.PATH_MFMA, "mfma_f16x3": st.PATH_MFMA_F16X3,
                    "mfma_bf16x3": st.PATH_MFMA_BF16X3, "auto": st.PATH_AUTO}
    tb_max = {1: 12, 2: 6, 3: 4, 4: 3}  # largest FP32 time block per order

    def knobs_for(name, r):
        if name == "gather_tb":
            return {"path": st.PATH_GATHER, "time_block": tb_max[r]}
        if name == "mfma_tb2":
            return {"path": st.PATH_MFMA, "time_block": 2}
        if name == "tuned":
            kn, _, _ = st.autotune(DIMS, r, st.BOX, coeffs[r], boundary=st.BC_PERIODIC, dtype=st.F32)
            return kn
        return {"path": name_to_path[name]}
    paths = [p for p in args.paths.split(",") if p]
    if args.headline not in paths:
        paths.append(args.headline)

    RADII = tuple(int(v) for v in args.radii.split(","))
    JACOBI_STEPS = args.jacobi_steps
    a0 = inputs.grid(DIMS, seed=INPUT_SEED, dtype=np.float32)
    coeffs = {r: inputs.coefficients(2, r, inputs.BOX, seed=COEF_SEED0 + r, dtype=np.float64) for r in RADII}
    a0_dev = torch.from_numpy(a0).cuda()
    stream = torch.cuda.Stream()
    pts_per_solve = DIMS[0] * DIMS[1] * JACOBI_STEPS

    results = {}
    for name in paths:
        per_r = {}
        for r in RADII:
            knobs = knobs_for(name, r)
            times, info = time_path(st, torch, knobs, r, a0_dev, coeffs[r], args.steps, args.warmup, stream)
            med = float(np.median(times))
            per_r[r] = {"ms_per_solve": med, "gstencil_s": pts_per_solve / (med * 1e-3) / 1e9,
                        "p50_ms": float(np.percentile(times, 50)), "p99_ms": float(np.percentile(times, 99)),
                        "resolved_path": st.PATH_NAMES[info["path"]], "info": info, "times": times,
                        "knobs": knobs}
            print(f"[bench] {name:12s} r={r}: {per_r[r]['gstencil_s']:8.1f} GStencil/s "
                  f"({med:.2f} ms / 100 steps, path={per_r[r]['resolved_path']}, knobs={knobs})", file=sys.stderr,
                  flush=True)
        results[name] = per_r

    head = results[args.headline]
    # one bench step = the four solves; per-step time = sum of the per-order medians
    step_times = [sum(head[r]["times"][k] for r in RADII) for k in range(args.steps)]
    ms_per_step = float(np.median(step_times))
    value = len(RADII) * pts_per_solve / (ms_per_step * 1e-3) / 1e9

    # dominant kernel: the order with the largest share of the step
    r_dom = max(RADII, key=lambda r: head[r]["ms_per_solve"])
    dom = head[r_dom]
    info = dom["info"]
    # a time-blocked plan advances up to T steps per launch: per launch it
    # reads and writes the grid once and does the arithmetic of its steps
    tb = max(1, int(info.get("time_block", 1)))
    launches = -(-JACOBI_STEPS // tb)
    launch_ms = dom["ms_per_solve"] / launches
    steps_per_launch = JACOBI_STEPS / launches
    bytes_per_launch = info["bytes_per_point"] * DIMS[0] * DIMS[1]
    gbs = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    flops_per_launch = info["useful_flops_per_point"] * DIMS[0] * DIMS[1] * steps_per_launch
    tflops = flops_per_launch / (launch_ms * 1e-3) / 1e12
    exec_tflops = info["executed_flops_per_point"] * DIMS[0] * DIMS[1] * steps_per_launch / (launch_ms * 1e-3) / 1e12
    rpath = dom["resolved_path"]
    mfma_dtype = {"mfma": "f32", "mfma_f16x3": "f16", "mfma_bf16x3": "bf16"}.get(rpath)
    # bound: HBM unless the arithmetic at its unit's peak (matrix cores for the
    # outer products, FP32 vector ALUs for the gather) would take longer than the bytes
    t_mem = bytes_per_launch / (HBM_PEAK_GBS * 1e9)
    bound = "hbm"
    if mfma_dtype:
        t_mfma = exec_tflops * 1e12 * launch_ms * 1e-3 / (PEAK_TFLOPS[mfma_dtype] * 1e12)
        if t_mfma > t_mem:
            bound = "mfma"
    elif flops_per_launch / (PEAK_TFLOPS["f32"] * 1e12) > t_mem:
        bound = "alu"
    src_hash = kernel_source_hash()
    klabel = f"{rpath}_tb{tb}" if tb > 1 else rpath
    kernel_key = f"{klabel}_box_r{r_dom}_f32_{DIMS[0]}x{DIMS[1]}_periodic"
    traffic = load_traffic(kernel_key, src_hash)
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    elif bound == "alu":
        # FP32 vector peak 157.3 TFLOP/s = 256 CUs x 4 SIMDs x 2.4 GHz x 64
        # flop/clock with packed FP32; without packed instructions (never
        # emitted here) a SIMD retires 16 FMAs a clock: 78.6 TFLOP/s
        peak = PEAK_TFLOPS["f32"]
        roof = {"bound": "alu", "achieved": tflops, "peak": peak, "unit": "TFLOP/s", "frac": tflops / peak,
                "peak_unpacked": peak / 2, "frac_unpacked": tflops / (peak / 2), "hbm_gbs": gbs,
                "steps_per_launch": steps_per_launch}
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
        "dtype": "f32+" + mfma_dtype if mfma_dtype in ("bf16", "f16") else "f32",
        "data": "synthetic",
        "config": {"workload": f"2D box stencils r=1..4, {DIMS[0]}x{DIMS[1]} FP32 grid, periodic, "
                               f"{JACOBI_STEPS} Jacobi steps per order (4 solves per bench step)",
                   "headline_path": args.headline, "input_seed": INPUT_SEED, "kernel_sources": kernel_source_hash(),
                   "coef_seeds": [COEF_SEED0 + r for r in RADII]},
        "roofline": roof,
    }
    line["per_order"] = {name: {str(r): {"gstencil_s": round(v["gstencil_s"], 2), "p50_ms": round(v["p50_ms"], 3),
                                         "p99_ms": round(v["p99_ms"], 3), "path": v["resolved_path"],
                                         "time_block": v["info"]["time_block"],
                                         "hbm_frac": hbm_frac(v["gstencil_s"], 8, v["info"]["time_block"])}
                                 for r, v in res.items()} for name, res in results.items()}
    if "gather" in results:
        line["vs_gather"] = {name: {str(r): round(res[r]["gstencil_s"] / results["gather"][r]["gstencil_s"], 3)
                                    for r in RADII} for name, res in results.items()}
    line["latency_ms"] = {"p50": float(np.percentile(step_times, 50)), "p99": float(np.percentile(step_times, 99))}
    if not args.no_cpu:
        cb = cpu_baseline(coeffs, a0)
        cb.pop("seconds", None)
        line["cpu_baseline"] = cb
    if not args.no_configs:
        del a0_dev
        torch.cuda.empty_cache()
        line["configs"] = config_extras(args, torch, st, inputs)
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
