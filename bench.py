"""Benchmark of the gfx950 SmrtLBM stream-collide path on one MI355X.

One benchmark step is one residual window: `--window` time steps of the
fused stream-collide kernel over the whole lattice, then the FP64 residual and
mass check and the export of (rho, u).  The default workload is the
bandwidth-scale case: a 4096 x 4096 periodic Taylor-Green field (u0 = 0.05,
wavenumber 2 pi / N, seeded +-1e-3 density noise), SmrtLBM, FP32 deviation
storage, tau = 0.6.

Printed (one JSON line): MLUPS of the whole job; the roofline of the
stream-collide kernel (its average launch time measured with HIP events on
the stream it runs on; the default kernel advances five time steps per launch
through LDS, reading and writing each node's populations once per launch):
the algorithmic HBM rate against the 8 TB/s peak, the HBM bytes that the
rocprofv3 counters recorded, and the vector-instruction rate against the
issue ceiling (the counter figures when they were taken on the current
kernel source), with "bound" naming the ceiling that binds; the CPU oracle
timed on a bounded sample of the same workload; and, after the timed
region, the rest of the metric: the rates of the other (scheme, tau) pairs,
the 1024^2 cavity's time to the steady-state residual, and the learned warm
start against the cold start.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS & HBM GB/s vs peak; time-to-steady (warm vs cold) at 1e-7 residual"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2409_01076_amd", "csrc", f)
                  for f in ("lbm_kernels.hpp", "smrt_api.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stream_collide.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_stream_collide.json")
# Vector-instruction issue ceiling of the MI355X: 256 CUs x 4 SIMDs, one
# 64-lane wave instruction per SIMD every 4 cycles (16 lanes per cycle) at
# 2.4 GHz.  Packed FP32 instructions are disabled in this build, so every
# FP32 operation is one such instruction.
VALU_PEAK_G = 256 * 4 * 2.4 / 4
# Lane operations of one SmrtLBM node-update in FP32 (collide<SMRT>), an FMA
# or a reciprocal counting as one: 8 pair sums and differences, 4 for the
# density, 4 for the momentum, 2 for 1/rho, 2 for u, 3 products j u, 2 for
# j.u and the equilibrium base, 3 + 4 for the axis and diagonal equilibrium
# parts, 4 + 4 for the odd parts, 5 for the two group sums, 2 for the
# corrections, 4 + 8 to assemble the eight moving populations and 8 for the
# rest population from the density.
SMRT_VALU_OPS = 67
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "f32x": 4}
# moment storage: bytes a node reads and writes per step (3 moments + 2 amplitudes)
MOMENT_NODE_BYTES = {"m64": 40, "m16": 16, "mbf16": 16}


def kernel_source_hash():
    """Hash of the kernel and launch source, to tell whether stored counter
    readings still describe the kernel being timed."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed residual windows")
    ap.add_argument("--warmup", type=int, default=1, help="untimed residual windows")
    ap.add_argument("--window", type=int, default=1000, help="time steps per residual window")
    ap.add_argument("--n", type=int, default=4096, help="lattice side")
    ap.add_argument("--scheme", default="smrt", choices=["smrt", "srt", "trt"])
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16", "bf16", "f32x", "m64", "m16", "mbf16"],
                    help="stored populations (default f32)")
    ap.add_argument("--tau", type=float, default=0.6)
    ap.add_argument("--storages", default="",
                    help="precision: comma-separated storages to compare with FP64 (default: all)")
    ap.add_argument("--launch", default="", help="bx,by,rows of the stream-collide kernel")
    ap.add_argument("--steps-per-launch", type=int, default=0,
                    help="time steps per kernel launch (0: the library's default for the lattice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget")
    ap.add_argument("--workload", default="tg",
                    choices=["tg", "cavity", "precision", "batch", "warmstart", "small", "mlp"],
                    help="tg: periodic Taylor-Green throughput (default); cavity: lid-driven "
                         "cavity run from the cold start to the steady-state residual; "
                         "precision: one cavity in every storage type against FP64; "
                         "batch: many cavities of uneven size and Re run together to steady; "
                         "warmstart: learned warm start against the cold start; "
                         "small: the 64^2 FP64 cavity at Re 100, eager and graph-captured; "
                         "mlp: one training step of the warm-start network on 65,536 rows")
    ap.add_argument("--train", type=int, default=200, help="warmstart: training cavities")
    ap.add_argument("--held-out", type=int, default=50, help="warmstart: evaluation cavities")
    ap.add_argument("--epochs", type=int, default=120, help="warmstart: training epochs")
    ap.add_argument("--count", type=int, default=256, help="batch: number of cavities")
    ap.add_argument("--schedule", default="",
                    help="cavity: precision schedule 'f16:1e-5' = run in that storage until the "
                         "residual falls below the level, then convert to --storage and finish")
    ap.add_argument("--compare-steps", type=int, default=200_000,
                    help="precision: step count at which the storage types are compared")
    ap.add_argument("--re", type=float, default=1000.0, help="cavity Reynolds number")
    ap.add_argument("--tol", type=float, default=1e-7, help="cavity steady-state residual")
    ap.add_argument("--max-steps", type=int, default=None,
                    help="cavity step cap (default 500,000 for the batch workload, 3,000,000 otherwise)")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the six (scheme, tau) rates, the 1024^2 cavity's "
                         "time to steady and the warm-start study")
    ap.add_argument("--copy-only", type=int, default=0, metavar="MIB",
                    help="only run the reference copy kernel over MIB mebibytes (counter calibration)")
    args = ap.parse_args()
    if args.max_steps is None:
        args.max_steps = 500_000 if args.workload == "batch" else 3_000_000
    return args


def copy_only(mib, reps=5):
    import torch
    from paper_2409_01076_amd import smrt
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        smrt.copy_kernel(a, b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kernel_bytes_each_way": n * 4, "launches": reps}), flush=True)


def copy_ceiling(nbytes, reps=10):
    """GB/s (read + write) of the library's plain copy kernel over nbytes."""
    import torch
    from paper_2409_01076_amd import smrt
    n = nbytes // 4 // 16 * 16
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    smrt.copy_kernel(a, b)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        smrt.copy_kernel(a, b)
    e1.record(s)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2 * n * 4 / sec / 1e9


def traffic_record(launch_cells, kernel):
    """Measured HBM bytes per launch of `kernel` from the committed counter
    summary, or None when it is missing, describes another kernel, or was
    taken on other kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if rec.get("cells_per_launch") != launch_cells or rec.get("kernel_name") != kernel:
        return None
    return rec.get("hbm_bytes_per_launch")


def valu_record(launch_cells):
    """VALU wave instructions per launch of the multi-step kernel and per
    node-update of the one-step kernel, from the committed counter record,
    or None when it is missing, describes another lattice, or was taken on
    other kernel source."""
    try:
        with open(VALU_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash() or rec.get("cells") != launch_cells:
        return None
    return rec


def pair_rates(n, steps=1000, storages=("f32",)):
    """GLUPS of the default launch for every (scheme, tau) of the bandwidth
    workload: `steps` time steps timed with HIP events on the solver's stream
    after 100 untimed ones."""
    import torch
    from paper_2409_01076_amd import inputs, smrt
    fields = [torch.from_numpy(a).to("cuda:0") for a in inputs.taylor_green(n, n, u0=0.05, noise=1e-3)]
    out = {}
    for storage in storages:
        for scheme in (("smrt",) if storage.startswith("m") else ("smrt", "srt")):
            for tau in (0.51, 0.6, 1.0):
                with smrt.Solver(n, n, scheme=scheme, boundary="periodic", storage=storage, tau=tau) as s:
                    s.init_fields(*fields)
                    s.step(100)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(s.stream)
                    s.step(steps)
                    e1.record(s.stream)
                    torch.cuda.synchronize()
                    out["%s %s tau=%g" % (storage, scheme, tau)] = round(
                        n * n * steps / (e0.elapsed_time(e1) / 1e3) / 1e9, 2)
    del fields
    return out


def cpu_baseline(args, fields, budget_s):
    """The oracle as it is, on the same workload, for about budget_s seconds."""
    import numpy as np

    import oracle as O
    rho, ux, uy = (a.astype(np.float64) for a in fields)
    L = O.Lattice(args.n, args.n, args.scheme, tau=args.tau, boundary="periodic", tau_s=1.0)
    f = L.init_equilibrium(rho, ux, uy)
    f = L.run(f, 1)
    t0 = time.perf_counter()
    f = L.run(f, 2)
    per_step = (time.perf_counter() - t0) / 2
    # chunks of about a sixth of the budget until the budget has elapsed (the
    # first steps run slower than the rest, so one estimate falls short)
    chunk = int(max(1, round(budget_s / 6 / max(per_step, 1e-3))))
    steps = 0
    t0 = time.perf_counter()
    while steps < 400:
        k = min(chunk, 400 - steps)
        f = L.run(f, k)
        steps += k
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    cells = args.n * args.n * steps
    threads = O.get_threads()
    # one-thread rate on the same lattice: one time step
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        f = L.run(f, 1)
        dt1 = time.perf_counter() - t0
    finally:
        O.set_threads(threads)
    return {"value": cells / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d time steps of the %dx%d periodic Taylor-Green lattice (%s, tau=%g), "
                      "FP64, %.1f s" % (steps, args.n, args.n, args.scheme, args.tau, dt),
            "value_1_thread": args.n * args.n / dt1 / 1e6, "cpu_model": cpu_model()}


def cpu_model():
    """The host CPU's model name, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def small_cavity(args):
    """The 64 x 64 FP64 cavity at Re = 100 (U = 0.1), 2000 steps, SmrtLBM and
    SRT: 4096 nodes, so each launch is bound by launch latency, not by the
    GPU.  Times the steps issued one call at a time and replayed from a
    captured HIP graph (each graph holds an even number of launches, so a
    replay leaves the buffer parity as capture found it) and checks that both
    end bitwise equal."""
    import torch

    from paper_2409_01076_amd import smrt

    n, steps, per_graph = 64, 2000, 200
    out = {"workload": "lid-driven cavity 64x64, Re=100, U=0.1, f64 storage, 2000 steps from the cold start",
           "results": {}}
    side = torch.cuda.Stream()
    for scheme in ("smrt", "srt"):
        with torch.cuda.stream(side):
            warm = smrt.Solver(n, n, scheme=scheme, storage="f64", re=100.0, u_lid=0.1)
            warm.step(per_graph)
            warm.close()
            eager = smrt.Solver(n, n, scheme=scheme, storage="f64", re=100.0, u_lid=0.1)
            replay = smrt.Solver(n, n, scheme=scheme, storage="f64", re=100.0, u_lid=0.1)
        spl = eager.steps_per_launch
        if (per_graph // spl) % 2 or per_graph % spl:
            raise RuntimeError("a graph of %d steps needs an even number of %d-step launches" % (per_graph, spl))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(side)
        with torch.cuda.stream(side):
            eager.step(steps)
        e1.record(side)
        torch.cuda.synchronize()
        eager_us = e0.elapsed_time(e1) * 1e3 / steps
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            replay.step(per_graph)
        torch.cuda.synchronize()
        e0.record(side)
        with torch.cuda.stream(side):
            for _ in range(steps // per_graph):
                g.replay()
        e1.record(side)
        torch.cuda.synchronize()
        graph_us = e0.elapsed_time(e1) * 1e3 / steps
        same = bool(torch.equal(eager.populations(torch.float64), replay.populations(torch.float64)))
        out["results"][scheme] = {"steps_per_launch": spl, "eager_us_per_step": round(eager_us, 3),
                                  "graph_us_per_step": round(graph_us, 3),
                                  "mlups_eager": round(n * n / eager_us, 1), "mlups_graph": round(n * n / graph_us, 1),
                                  "graph_equals_eager": same}
        del g
        eager.close()
        replay.close()
    print(json.dumps(out))


def cavity_to_steady(args, storage=None, quiet=False):
    """Cold-start lid-driven cavity (U = 0.1) run until the windowed residual
    falls below args.tol: steps, wall time and throughput for each scheme.
    Returns the JSON record."""
    import torch
    from paper_2409_01076_amd import smrt
    n = args.n if args.n != 4096 else 1024
    storage = storage or args.storage
    results = {}
    stages = []
    if args.schedule:
        first, level = args.schedule.split(":")
        stages.append((first, float(level)))
    stages.append((storage, args.tol))
    # moment storage holds the SmrtLBM state only
    for scheme in (("smrt",) if storage.startswith("m") else ("smrt", "srt")):
        solver = smrt.Solver(n, n, scheme=scheme, boundary="cavity", storage=stages[0][0],
                             re=args.re, u_lid=0.1, device="cuda:0")
        if args.launch:
            solver.set_launch(*[int(v) for v in args.launch.split(",")])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = [0.0]

        def progress(steps, r):
            if not quiet and time.perf_counter() - last[0] > 20:
                last[0] = time.perf_counter()
                print("# %s step %d residual %.3e" % (scheme, steps, r), file=sys.stderr, flush=True)
        steps, res, status, stage_steps = 0, [], "cap", []
        try:
            for i, (storage, level) in enumerate(stages):
                if i > 0:
                    old = solver
                    solver = old.convert(storage)
                    old.close()
                k, r, ok = solver.run_to_steady(level, args.window, args.max_steps - steps, progress)
                steps += k
                res += r
                stage_steps.append(k)
                if not ok:
                    break
            else:
                status = "steady"
        except smrt.UnstableError:
            steps, status = steps + solver.steps_done, "unstable"
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        results[scheme] = {"steps": steps, "seconds": round(wall, 3), "status": status,
                           "final_residual": res[-1] if res else None,
                           "mlups": round(n * n * steps / wall / 1e6, 1), "tau": solver.tau,
                           "stages": [{"storage": st, "until": lv, "steps": k}
                                      for (st, lv), k in zip(stages, stage_steps)]}
        solver.close()
    s = results["smrt"]
    out = {
        "metric": METRIC, "value": s["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": s["steps"],
        "warmup": 0, "ms_per_step": round(s["seconds"] / max(1, s["steps"]) * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if storage in ("f64", "f32x") else "f32", "data": "synthetic",
        "config": {"workload": "lid-driven cavity %dx%d, Re=%g, U=0.1, %s storage%s, cold start, "
                               "run to windowed residual < %g (window %d)"
                               % (n, n, args.re, storage,
                                  " after " + args.schedule if args.schedule else "", args.tol,
                                  args.window),
                   "schedule": args.schedule or None,
                   "nx": n, "ny": n, "re": args.re, "u_lid": 0.1, "storage": storage,
                   "window": args.window, "tol": args.tol},
        "time_to_steady": results,
    }
    return out


def precision_study(args):
    """The cold-start cavity (U = 0.1) in every storage type, against FP64
    storage (itself within round-off of the CPU oracle): max |du| / U after
    --compare-steps steps and at the step count where FP64 reaches the
    steady-state residual (equal step counts: at R = 1e-7 a field is still
    moving, so states reached at different step counts differ by more than
    the storage does); and each storage's own steps and seconds to the
    residual (or the cap)."""
    import torch
    from paper_2409_01076_amd import smrt
    n = args.n if args.n != 4096 else 2048
    U = 0.1
    ref, ref_steady, n_steady, n_ref, out = None, None, None, None, {}
    storages = ("f64", "f32x", "f32", "f16", "bf16") + (("m16", "mbf16") if args.scheme == "smrt" else ())
    if args.storages:
        wanted = args.storages.split(",")
        if any(w not in storages for w in wanted):
            raise SystemExit("--storages: pick from %s" % ",".join(storages))
        storages = ("f64",) + tuple(w for w in storages if w in wanted and w != "f64")
    for storage in storages:
        s = smrt.Solver(n, n, scheme=args.scheme, boundary="cavity", storage=storage, re=args.re,
                        u_lid=U, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.compare_steps)
        _, ux, uy = s.moments(torch.float64)
        torch.cuda.synchronize()
        t_cmp = time.perf_counter() - t0
        rec = {"seconds_to_compare": round(t_cmp, 3),
               "mlups": round(n * n * args.compare_steps / t_cmp / 1e6, 1)}
        if ref is None:
            ref = (ux, uy)
        else:
            rec["max_du_over_U_at_compare"] = float(max((ux - ref[0]).abs().max(),
                                                         (uy - ref[1]).abs().max())) / U
        m0 = float(n * n)
        rec["mass_drift_at_compare"] = s.mass() / m0 - 1.0
        del ux, uy
        steps, steady_at, t_steady, status, last_r, paused = args.compare_steps, None, None, "cap", None, 0.0
        last = [time.perf_counter()]
        try:
            while steps < args.compare_steps + args.max_steps:
                s.step(args.window)
                steps += args.window
                last_r = s.residual()
                if steady_at is None and last_r < args.tol:
                    steady_at, t_steady, status = steps, time.perf_counter() - t0 - paused, "steady"
                if n_steady is not None and steps == n_steady:
                    t1 = time.perf_counter()
                    _, fx, fy = s.moments(torch.float64)
                    rec["max_du_over_U_at_fp64_steady_steps"] = float(max((fx - ref_steady[0]).abs().max(),
                                                                          (fy - ref_steady[1]).abs().max())) / U
                    del fx, fy
                    torch.cuda.synchronize()
                    paused += time.perf_counter() - t1
                if steady_at is not None and (n_steady is None or steps >= n_steady):
                    break
                if time.perf_counter() - last[0] > 20:
                    last[0] = time.perf_counter()
                    print("# %s step %d residual %.3e" % (storage, steps, last_r), file=sys.stderr, flush=True)
        except smrt.UnstableError:
            status = "unstable"
        torch.cuda.synchronize()
        rec.update({"status": status, "steps_to_steady": steady_at,
                    "seconds_to_steady": round(t_steady, 3) if t_steady is not None else None,
                    "steps_run": steps, "final_residual": last_r})
        if storage == "f64":
            n_steady, n_ref = steady_at, steps
            _, fx, fy = s.moments(torch.float64)
            ref_steady = (fx, fy)
        elif n_steady is None and steps == n_ref:
            # FP64 itself stayed above the residual: compare all at the cap
            _, fx, fy = s.moments(torch.float64)
            rec["max_du_over_U_at_cap"] = float(max((fx - ref_steady[0]).abs().max(),
                                                    (fy - ref_steady[1]).abs().max())) / U
            del fx, fy
        rec["mass_drift_final"] = s.mass() / m0 - 1.0
        s.close()
        out[storage] = rec
        print("# %s %s" % (storage, json.dumps(rec)), file=sys.stderr, flush=True)
    print(json.dumps({"workload": "precision: cavity %dx%d Re=%g U=%g %s, compared at %d steps and at the "
                                  "step count where FP64 reaches the residual %g (window %d, cap %d)"
                                  % (n, n, args.re, U, args.scheme, args.compare_steps, args.tol,
                                     args.window, args.max_steps),
                      "reference": "FP64 storage on the GPU (round-off parity with the FP64 CPU oracle)",
                      "fp64_steady_steps": n_steady, "results": out}), flush=True)


def batch_to_steady(args):
    """args.count cavities, side N = round(64 * 8^u) and Re = 100 * 100^v with
    u, v ~ U(0, 1) from the seed, U = 0.1, all advanced together (one launch
    per step, graph-captured windows, autotuned launch shape) until each is
    steady (windowed residual < args.tol), unstable, or at args.max_steps."""
    import torch
    from paper_2409_01076_amd import inputs, smrt
    n, re = inputs.cavity_batch(args.count, 64, 512, 100.0, 10000.0)
    nodes = n.astype(np.int64) ** 2
    b = smrt.Batch(n, n, scheme=args.scheme, storage=args.storage, re=re, u_lid=0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chosen = b.autotune(steps=20)
    spl_batch = b.steps_per_launch
    tune_steps = b.steps_done
    steps, status, res = b.run(args.tol, args.window, args.max_steps - tune_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.close()
    steps = np.array(steps)
    updates = int((nodes * steps).sum())
    st = np.array(status)
    out = {
        "metric": METRIC, "value": round(updates / wall / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": int(steps.max()), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": "%d lid-driven cavities, N log-uniform [64, 512], Re log-uniform "
                               "[100, 1e4], U=0.1, %s, %s storage, each to residual < %g or %d steps"
                               % (args.count, args.scheme, args.storage, args.tol, args.max_steps),
                   "count": args.count, "seed": inputs.DEFAULT_SEED, "window": args.window,
                   "total_nodes": int(nodes.sum())},
        "cavities_per_second": round(args.count / wall, 3),
        "seconds": round(wall, 3),
        "node_updates": updates,
        "autotuned_launch": {"bx": chosen[0], "by": chosen[1], "grid": chosen[2],
                             "steps_per_launch": spl_batch},
        "steady": int((st == smrt.STEADY).sum()), "unstable": int((st == smrt.UNSTABLE).sum()),
        "capped": int((st == smrt.RUNNING).sum()),
        "per_cavity": [{"n": int(a), "re": round(float(r), 2), "steps": int(k),
                        "status": ["cap", "steady", "unstable"][int(s)],
                        "residual": None if not np.isfinite(x) else float(x)}
                       for a, r, k, s, x in zip(n, re, steps, status, res)],
    }
    print(json.dumps(out), flush=True)


def mlp_step(args, rows=65536):
    """Training steps of the warm-start network (5 layers of width 128,
    16 Fourier features, bf16 matrix cores) on `rows` seeded synthetic points
    and targets: `warmup` untimed steps, then `steps` timed with HIP events on
    the network's stream."""
    import torch
    from paper_2409_01076_amd import warmstart as W
    rng = np.random.default_rng(2409)
    pts = torch.from_numpy(rng.uniform(0, 1, size=(rows, 3)).astype(np.float32)).to("cuda:0")
    tgt = torch.from_numpy(rng.normal(0, 0.5, size=(rows, 3)).astype(np.float32)).to("cuda:0")
    ws = W.WarmStart(fourier=16, width=128, layers=5, batch=rows)
    stream = ws.net.stream

    def timed():
        for _ in range(max(1, args.warmup)):
            ws.net.train_step(pts, tgt, 1e-3)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            ws.net.train_step(pts, tgt, 1e-3)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    fused = ws.net.fused_forward
    ms = timed()
    # the same step with one forward launch per layer
    ws.net.fused_forward = False
    ms_layers = timed()
    ws.close()
    flops = 6.0 * rows * (64 * 128 + 3 * 128 * 128 + 128 * 64)  # forward + two backward products, padded sizes
    return {"workload": "warm-start network training step: %d rows, 5 weight layers of width 128, "
                        "16 Fourier features, bf16 matrix cores, Adam" % rows,
            "steps": args.steps, "ms_per_step": round(ms, 4), "fused_forward": fused,
            "ms_per_step_forward_per_layer": round(ms_layers, 4),
            "tflops_padded": round(flops / (ms * 1e-3) / 1e12, 1)}


def warm_start_study(args, quiet=False):
    """Learned warm start on 256^2 cavities: Re log-uniform in [100, 1e4]
    (seeded); args.train steady fields from the solver train the network on
    the GPU; on args.held_out other Re the cold start and the warm start run
    to the same residual; reports steps, wall time (warm includes inference)
    and the final-field difference max |du| / U per cavity."""
    import torch
    from paper_2409_01076_amd import smrt
    from paper_2409_01076_amd import warmstart as W
    n, U = (args.n if args.n != 4096 else 256), 0.1
    rng = np.random.default_rng(2409010760)
    re_all = 100.0 * 100.0 ** rng.uniform(0, 1, size=args.train + args.held_out)
    re_train, re_test = re_all[:args.train], re_all[args.train:]
    log = (lambda msg: None) if quiet else (lambda msg: print("# " + msg, file=sys.stderr, flush=True))

    def run_batch(res, warm=None):
        b = smrt.Batch([n] * len(res), [n] * len(res), scheme=args.scheme, storage=args.storage,
                       re=res, u_lid=U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if warm is not None:
            for i, r in enumerate(res):
                b.init_fields(i, *warm.predict(n, r, U))
        steps, status, resid = b.run(args.tol, args.window, args.max_steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fields = [[t.cpu().numpy() for t in b.moments(i)] for i in range(len(res))]
        b.close()
        return np.array(steps), np.array(status), fields, wall

    t0 = time.perf_counter()
    tr_steps, tr_status, tr_fields, tr_wall = run_batch(re_train)
    log("training data: %d cavities, %d steady, %.1f s" % (len(re_train), (tr_status == smrt.STEADY).sum(), tr_wall))
    keep = tr_status == smrt.STEADY
    if not keep.any():
        raise SystemExit("no training cavity reached the residual %g within %d steps; raise --max-steps"
                         % (args.tol, args.max_steps))
    pts = np.concatenate([W.cavity_points(n, r) for r, k in zip(re_train, keep) if k])
    tgt = np.concatenate([W.targets(*f, U) for f, k in zip(tr_fields, keep) if k])
    ws = W.WarmStart(fourier=16, width=128, layers=5, batch=65536)
    t1 = time.perf_counter()
    hist = ws.fit(pts, tgt, epochs=args.epochs, lr=2e-3, log=log)
    train_s = time.perf_counter() - t1
    cold_steps, cold_status, cold, cold_wall = run_batch(re_test)
    warm_steps, warm_status, warm, warm_wall = run_batch(re_test, ws)
    ws.close()
    per = []
    for i, r in enumerate(re_test):
        err = max(np.abs(warm[i][1] - cold[i][1]).max(), np.abs(warm[i][2] - cold[i][2]).max()) / U
        per.append({"re": round(float(r), 2), "cold_steps": int(cold_steps[i]), "warm_steps": int(warm_steps[i]),
                    "cold_status": ["cap", "steady", "unstable"][int(cold_status[i])],
                    "warm_status": ["cap", "steady", "unstable"][int(warm_status[i])],
                    "final_max_du_over_U": float(err)})
    both = (cold_status == smrt.STEADY) & (warm_status == smrt.STEADY)
    out = {
        "workload": "learned warm start, %dx%d cavities, Re log-uniform [100, 1e4], %d training / %d "
                    "held-out, U=0.1, %s %s, residual < %g (window %d), cap %d steps"
                    % (n, n, args.train, args.held_out, args.scheme, args.storage, args.tol, args.window,
                       args.max_steps),
        "network": "5 weight layers, width 128, (x, y, log Re) + 16 Fourier features, bf16 MFMA, FP32 accumulation",
        "training_cavities_steady": int(keep.sum()),
        "training_data_seconds": round(tr_wall, 2),
        "training_seconds": round(train_s, 2),
        "training_loss_first_last": [hist[0][1], hist[-1][1]],
        "held_out_both_steady": int(both.sum()),
        "cold_total_steps_both_steady": int(cold_steps[both].sum()),
        "warm_total_steps_both_steady": int(warm_steps[both].sum()),
        "median_step_ratio_warm_over_cold": float(np.median(warm_steps[both] / cold_steps[both])) if both.any() else None,
        "cold_wall_seconds": round(cold_wall, 3),
        "warm_wall_seconds_including_inference": round(warm_wall, 3),
        "max_final_field_diff_over_U": float(max(p["final_max_du_over_U"] for p, b in zip(per, both) if b))
        if both.any() else None,
        "total_seconds": round(time.perf_counter() - t0, 1),
        "per_cavity": per,
    }
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_only:
        copy_only(args.copy_only)
        return

    if args.workload == "cavity":
        print(json.dumps(cavity_to_steady(args)), flush=True)
        return
    if args.workload == "precision":
        precision_study(args)
        return
    if args.workload == "batch":
        batch_to_steady(args)
        return
    if args.workload == "warmstart":
        print(json.dumps(warm_start_study(args)), flush=True)
        return
    if args.workload == "small":
        small_cavity(args)
        return
    if args.workload == "mlp":
        print(json.dumps(mlp_step(args)), flush=True)
        return

    from paper_2409_01076_amd import inputs, smrt

    n, K = args.n, args.window
    fields = inputs.taylor_green(n, n, u0=0.05, noise=1e-3)
    dev = [torch.from_numpy(a).to("cuda:0") for a in fields]
    solver = smrt.Solver(n, n, scheme=args.scheme, boundary="periodic", storage=args.storage,
                         tau=args.tau, tau_s=1.0, device="cuda:0")
    if args.launch:
        solver.set_launch(*[int(v) for v in args.launch.split(",")])
    if args.steps_per_launch:
        solver.set_steps_per_launch(args.steps_per_launch)
    solver.init_fields(*dev)
    del dev
    mass0 = solver.mass()
    stream = solver.stream
    rho_out, ux_out, uy_out = (torch.empty((n, n), dtype=torch.float32, device="cuda:0")
                               for _ in range(3))

    def window(events=None):
        if events is not None:
            events[0].record(stream)
        solver.step(K)
        if events is not None:
            events[1].record(stream)
        r = solver.residual()
        solver.moments_into(rho_out, ux_out, uy_out)
        return r

    for _ in range(args.warmup):
        window()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    residuals = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        residuals.append(window(ev[i]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    window_ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    kernel_ms = window_ms / K
    mass = solver.mass()
    spl = solver.steps_per_launch
    # A window of K steps is q launches of the dominant kernel plus, when spl
    # does not divide K, one launch of the remaining r steps; that launch is
    # timed on its own (same stream, HIP events) and taken out.
    q, r = divmod(K, spl)
    rem_ms = 0.0
    if r:
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            solver.step(r)  # one launch of r steps each
        e1.record(stream)
        torch.cuda.synchronize()
        rem_ms = e0.elapsed_time(e1) / reps
    solver.close()

    cells = n * n
    mom = args.storage in MOMENT_NODE_BYTES
    # The dominant kernel reads d(t) and writes d(t + spl) once per node per
    # launch: 9 loads + 9 stores per node whether it advances one time step
    # (stream_collide) or several through LDS (stream_collide_x2 .. _x5).
    kernel_name = "stream_collide_mom" if mom else ("stream_collide" if spl == 1 else "stream_collide_x%d" % spl)
    launch_ms = (window_ms - rem_ms) / q
    node_bytes = 2 * MOMENT_NODE_BYTES[args.storage] if mom else 18 * STORAGE_BYTES[args.storage]
    alg_bytes = node_bytes * cells
    achieved = alg_bytes / (launch_ms / 1e3) / 1e9
    mlups = cells * K * args.steps / wall / 1e6
    traffic = traffic_record(cells, kernel_name)
    hbm_frac = achieved / HBM_PEAK_GBS
    valu = valu_record(cells) if args.scheme == "smrt" and args.storage == "f32" and spl > 1 else None
    if valu is not None and valu.get("multi_kernel_name") != kernel_name:
        valu = None
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage in ("f64", "f32x", "m64") else "f32",
        "data": "synthetic",
        "config": {
            "workload": "periodic Taylor-Green %dx%d, %s, %s storage, tau=%g, "
                        "step = %d time steps + residual/mass + moments export"
                        % (n, n, args.scheme, args.storage, args.tau, K),
            "nx": n, "ny": n, "scheme": args.scheme, "storage": args.storage, "tau": args.tau,
            "window": K, "u0": 0.05, "density_noise": 1e-3, "seed": inputs.DEFAULT_SEED,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(hbm_frac, 4),
            "traffic": traffic,
            "kernel": kernel_name,
            "time_steps_per_launch": spl,
            "kernel_avg_us": round(launch_ms * 1e3, 2),
            "algorithmic_bytes_per_launch": alg_bytes,
            "algorithmic_unit": ("one node advanced one time step: its 5 moments read and written, %d B"
                                 % node_bytes) if mom else
                                ("one node advanced %d time step%s per launch: 9 reads + 9 writes of %d B"
                                 % (spl, "s" * (spl > 1), STORAGE_BYTES[args.storage])),
        },
        "glups_kernel": round(cells / (kernel_ms / 1e3) / 1e9, 2),
        "copy_kernel_gbs": round(copy_ceiling(alg_bytes // 2), 1),
        "last_residual": residuals[-1],
        "mass_drift": mass / mass0 - 1.0,
    }
    out["roofline"]["frac_of_copy_kernel"] = round(achieved / out["copy_kernel_gbs"], 4)
    if valu is not None:
        # The vector-instruction ceiling.  Algorithmic: the SmrtLBM collision's
        # own arithmetic, SMRT_VALU_OPS lane operations a node-update (moments,
        # equilibrium terms, the two group corrections, the rest population;
        # streaming is data movement), as wave-instruction equivalents (64 lanes
        # each).  Issued: what SQ_INSTS_VALU recorded for this launch (ring
        # recomputation, LDS addressing and conversions too).  The ceiling that
        # the issued instructions come closer to binds.
        alg_insts = SMRT_VALU_OPS / 64.0 * spl * cells
        alg_g = alg_insts / (launch_ms / 1e3) / 1e9
        issued_g = valu["multi_wave_insts_per_launch"] / (launch_ms / 1e3) / 1e9
        hbm = {k: out["roofline"][k] for k in ("achieved", "peak", "unit", "frac")}
        out["roofline"]["hbm"] = hbm
        out["roofline"]["valu"] = {
            "achieved": round(alg_g, 1), "peak": VALU_PEAK_G, "unit": "G wave-instructions/s",
            "frac": round(alg_g / VALU_PEAK_G, 4),
            "algorithmic_wave_insts_per_launch": round(alg_insts),
            "algorithmic_unit": "one node advanced %d time steps: %d x %d lane operations of the SmrtLBM "
                                "collision per node-update, / 64 lanes" % (spl, spl, SMRT_VALU_OPS),
            "issued_wave_insts_per_launch": valu["multi_wave_insts_per_launch"],
            "issued_g": round(issued_g, 1), "issued_frac": round(issued_g / VALU_PEAK_G, 4),
            "source": "SQ_INSTS_VALU, profiles/valu_stream_collide.json",
        }
        if issued_g / VALU_PEAK_G > hbm_frac:
            # the vector ALU binds: report its ceiling at the top level
            out["roofline"].update(bound="alu", achieved=round(alg_g, 1), peak=VALU_PEAK_G,
                                   unit="G wave-instructions/s", frac=round(alg_g / VALU_PEAK_G, 4))
    # the HBM rate one step per launch would need for the same node updates:
    # temporal blocking moves 18 s / spl bytes per node-update instead of 18 s
    out["roofline"]["one_step_equivalent_gbs"] = round(achieved * spl, 1)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, fields, args.cpu_seconds)
    if not args.no_extras:
        # the rest of the metric, after the timed region: the other (scheme,
        # tau) pairs of this workload, the 1024^2 cavity at Re 1000 from the
        # cold start to the residual (binary32 storage with FP64 and with
        # binary32 arithmetic), and learned warm starts against cold starts
        out["glups_pairs"] = pair_rates(n, storages=("f32", "f32x", "m16"))
        import copy
        cav = copy.copy(args)
        cav.n, cav.schedule, cav.launch = 1024, "", ""
        out["time_to_steady_cavity1024"] = {}
        for storage in ("f32x", "f32"):
            rec = cavity_to_steady(cav, storage=storage, quiet=True)
            out["time_to_steady_cavity1024"][storage] = {
                sch: {k: r[k] for k in ("steps", "seconds", "status", "final_residual", "mlups")}
                for sch, r in rec["time_to_steady"].items()}
        out["time_to_steady_cavity1024"]["config"] = ("lid-driven cavity 1024x1024, Re=%g, U=0.1, cold start, run to "
                                                      "windowed residual < %g (window %d); f32x: binary32 storage "
                                                      "with FP64 arithmetic" % (cav.re, cav.tol, cav.window))
        ws = copy.copy(args)
        ws.n, ws.max_steps, ws.storage = 256, 400_000, "f32"
        rec = warm_start_study(ws, quiet=True)
        out["warm_start"] = {k: v for k, v in rec.items() if k != "per_cavity"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
