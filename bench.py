#!/usr/bin/env python3
"""Throughput of the BP RI-OEDG stage on one MI355X.

Metric: DOF-stage updates per second, DOF = 4 variables x (L_k + 1) modes per cell,
one SSP-RK3 step = 3 stages.  A benchmark step is one SSP-RK3 step of the whole
stage path (residual + SSP combination, domain reductions, RIOE, BP limiter,
max wave speed, device-side Delta t) over the resident mesh and state.

Workloads (every mesh is built before the GPU is touched, in spawned processes):
* headline: P2, about 200k cells of a seeded Poisson-disk Delaunay mesh of the unit
  square, four-quadrant Riemann data (rho in [0.14, 1.5], p in [0.03, 1.5]),
  transmissive boundaries, FP64 (the value) and the mixed form (FP32 bulk, FP64
  averages and limiter; "mixed");
* "blast": the near-vacuum blast on a ~1M-cell mesh, FP64 and mixed, each with its
  own roofline object (its state does not fit the 256 MB Infinity Cache);
* "largest": the largest P2 mesh (22,368,256 periodic cells), FP64 and mixed;
* "batch": 64 uneven P1/P2 instances stepped as one batch (full sizes by default);
* "serving": the continuous-batching server on a Poisson request stream of
  1k-2M-cell requests at two arrival rates (p50/p99 latency, aggregate DOF-stage/s);
* "decompositions": Sec. 6's optimal-vs-classical time-step comparison;
* "cpu_baseline": the FP64 C oracle on all usable host cores (and one thread).

Prints one JSON line.  Only one GPU is supported: --gpus N with N > 1 exits.
"""

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, vendor figure
KERNEL_SRC = os.path.join(ROOT, "paper_2409_09620_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")


def log(*a):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def state_bytes_per_cell(k, precision="fp64"):
    """S: the bytes of one cell's state (mixed: FP64 averages, FP32 higher modes)."""
    nm = (k + 1) * (k + 2) // 2
    b_hi = 8 if precision == "fp64" else 4
    return 4 * (8 + (nm - 1) * b_hi)


def algorithmic_bytes_per_cell(k, precision="fp64"):
    """Bytes each pass must move per cell and launch, as the hot-path scope fixes
    them: the residual pass reads the stage input (S), reads u^n in two of three
    stages (2/3 S) and writes the pre-filter state (S), plus 128 B of geometry; the
    filter pass reads the pre-filter state and writes the stage output (2 S) plus
    160 B of geometry.  Neighbour re-reads are cache hits and not counted."""
    S = state_bytes_per_cell(k, precision)
    return {"residual": S + S + (2.0 / 3.0) * S + 128, "filter": 2 * S + 160}


def stored_bytes_per_cell(k, precision="fp64"):
    """The same with the geometry these kernels actually read: the residual J^-1,
    |K| and the edge links (52 B); the filter adds the edge lengths and the two
    limiter points' reference coordinates (108 B)."""
    S = state_bytes_per_cell(k, precision)
    return {"residual": S + S + (2.0 / 3.0) * S + 52, "filter": 2 * S + 108}


def kernel_source_hash(path=KERNEL_SRC):
    """Hash of the kernel source's code: line comments, trailing blanks and empty lines
    are dropped first, so counters stay valid across edits of the comments only.  (The
    kernel source has no block comments and no '//' inside string literals.)"""
    lines = []
    with open(path, encoding="utf-8") as f:
        for line in f:
            code = line.split("//", 1)[0].rstrip()
            if code:
                lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def load_counters(kernel, workload):
    """The committed counter record of `kernel` on `workload` (HBM bytes, VALU
    issue), or None when it was taken on other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get("workloads", {}).get(workload, {}).get(kernel)


def load_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    summary, or None when it was taken on other kernel sources."""
    rec = load_counters(kernel, workload)
    return rec.get("hbm_bytes_per_launch") if rec else None


def load_valu(kernel, workload):
    """VALU issue of `kernel` on `workload` from the committed counter summary:
    instructions per launch (wave-level), the fraction of the SIMDs' cycles spent
    executing them, and the shader clock during the launch; None when absent or
    taken on other kernel sources."""
    rec = load_counters(kernel, workload)
    v = rec.get("valu") if rec else None
    if not v:
        return None
    return {"insts_per_launch": v["insts_per_launch"], "busy_frac": v["busy_frac"], "clock_ghz": v["clock_ghz"]}


def run_gpu(mesh, kind, params, k, steps, warmup, precision="fp64"):
    """Two timed regions of `steps` SSP-RK3 steps each, inputs resident in HBM:
    (a) the production path, each step replayed as one captured HIP graph; its wall
        time gives the throughput;
    (b) the same steps launched eagerly with HIP events around every pass kernel,
        recorded by the library on its stream; gives the per-kernel durations."""
    import torch
    from paper_2409_09620_amd import Solver

    s = Solver(mesh, k, device=0)
    s.init_problem(kind, params, precision=precision)
    for _ in range(warmup):
        s.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.profile(True)
    s.profile_read()                       # reset the accumulators
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        s.step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    prof = s.profile_read()
    s.profile(False)
    d = s.diag()
    s.close()
    return t1 - t0, t3 - t2, prof, d


def batch_tasks(scale):
    """Mesh builders of the 64-instance workload (log-uniform sizes 5k-500k divided
    by `scale`, P1/P2 50/50, two-state data), and the degrees."""
    from synth import workloads
    sizes, degree = workloads.batch_sizes(n_inst=64)
    tasks = [(workloads.batch_instance, (i, max(int(sz) // scale, 64))) for i, sz in enumerate(sizes)]
    return tasks, [int(k) for k in degree]


def run_batch(instances, degree, steps, warmup, precision):
    """The 64 instances stepped as one batch: autotuned schedule, each step one graph
    replay."""
    import torch
    from paper_2409_09620_amd import Batch, Solver
    sols, dof = [], 0
    for i, ((m, kind, p), k) in enumerate(zip(instances, degree)):
        if i % 16 == 0:
            log(f"batch {precision}: initialising instance {i}/{len(instances)}")
        s = Solver(m, k)
        s.init_problem(kind, p, precision=precision)
        sols.append(s)
        dof += m.n_cell * 4 * (k + 1) * (k + 2) // 2
    b = Batch(sols)
    tuned = b.autotune(reps=2)
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    act, st = b.status()
    out = {"value": dof * 3 * steps / el, "ms_per_step": el / steps * 1e3, "instances": len(sols),
           "cells": int(sum(s.nc for s in sols)), "p2_instances": int(sum(1 for k in degree if k == 2)),
           "steps": steps, "schedule": dict(b.schedule(), ms_stage0_tuned=tuned["ms_stage"]),
           "members_active": act, "members_in_error": int((st[:, 1] != 0).sum())}
    b.close()
    for s in sols:
        s.close()
    return out


def serving_tasks(n_req, scale, t_scale):
    from synth import workloads
    specs = workloads.serving_requests(n_req=n_req, rate=1.0, scale=scale, t_scale=t_scale)
    return specs, [(workloads.serving_request, (sp,)) for sp in specs]


def run_serving(specs, built, rates, scale, t_scale, steps_per_tick=8, max_wall=120.0):
    """The continuous-batching server on a seeded request stream (sizes 1k-2M
    divided by `scale`, t_end in [0.05, 0.5] times `t_scale`), once per arrival
    rate.  Request meshes are built before the clock starts (the client's
    payload); upload, host precompute, projection and stepping are timed.  A run
    stops after max_wall seconds (its unfinished requests count as errors)."""
    from paper_2409_09620_amd.serving import Request, Server
    from synth import workloads
    n_req = len(specs)
    out = {}
    for rate in rates:
        reqs = [Request(id=sp["id"], k=sp["k"], n_cell=built[sp["id"]][0].n_cell, t_end=sp["t_end"],
                        build=(lambda b=built[sp["id"]]: b), arrival=sp["arrival"])
                for sp in workloads.serving_requests(n_req=n_req, rate=rate, scale=scale, t_scale=t_scale)]
        log(f"serving: {n_req} requests at {rate:g}/s")
        st = Server(steps_per_tick=steps_per_tick, keep_results=False, progress=lambda m: log("serving", m),
                    max_wall=max_wall).run(reqs)
        out[f"rate_{rate:g}_per_s"] = {
            "p50_ms": st.p50 * 1e3, "p99_ms": st.p99 * 1e3, "mean_ms": st.mean * 1e3,
            "dof_stage_per_s": st.dof_stage_per_s, "wall_s": st.wall, "peak_members": st.peak_members,
            "batch_rebuilds": st.rebuilds, "errors": st.errors, "steps_total": int(sum(r.steps for r in reqs))}
    cells = [b[0].n_cell for b in built.values()]
    out["workload"] = (f"{n_req} requests, sizes log-uniform 1k-2M / {scale} ({min(cells)}-{max(cells)} cells), "
                       f"P1|P2, Riemann|vortex, t_end in [0.05, 0.5] x {t_scale}, Poisson arrivals")
    return out


def run_decompositions(mesh, kind, params, steps_dcw=150):
    """Sec. 6's comparison of the two convex decompositions behind the BP time step:
    the same problem run to the same final time t_end = steps_dcw x the optimal
    decomposition's first Delta t, P1 and P2, FP64.  The mean time step is t_end over
    the number of steps (as in Sec. 6).  Time to solution: the first step (which
    captures the step graph) runs untimed, dg_step_to times the rest, and the total
    is that rate times the number of steps."""
    import torch
    from paper_2409_09620_amd import Solver

    out = {}
    for k in (1, 2):
        s = Solver(mesh, k, device=0)
        s.init_problem(kind, params)
        t_end = steps_dcw * s.diag()["dt"]
        s.close()
        res = {"t_end": t_end}
        for dec in ("dcw", "zxs"):
            s = Solver(mesh, k, device=0)
            s.init_problem(kind, params, decomposition=dec)
            s.step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = s.step_to(t_end)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            d = s.diag()
            steps = n + 1
            res[dec] = {"steps": steps, "mean_dt": t_end / steps, "ms_per_step": (t1 - t0) / n * 1e3,
                        "time_to_solution_s": (t1 - t0) / n * steps, "n_restarts": d["n_restarts"],
                        "n_limited": d["n_limited"]}
            s.close()
        res["mean_dt_ratio_dcw_over_zxs"] = res["dcw"]["mean_dt"] / res["zxs"]["mean_dt"]
        res["time_to_solution_speedup"] = res["zxs"]["time_to_solution_s"] / res["dcw"]["time_to_solution_s"]
        out[f"p{k}"] = res
        log(f"decompositions P{k}: mean dt ratio {res['mean_dt_ratio_dcw_over_zxs']:.4f}, "
            f"time-to-solution speedup {res['time_to_solution_speedup']:.3f}")
    return out


def copy_bandwidth(mib=2048, reps=10):
    """Practical HBM rate for context: a device-to-device copy of `mib` MiB, read plus
    write bytes over the mean time of `reps` copies (HIP events)."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return {"gbs": 2 * n * 8 / t / 1e9, "bytes_per_copy": 2 * n * 8, "kernel": "torch copy_ (device to device)"}


def roofline(prof, k, n_cell, workload, precision="fp64"):
    """The roofline object of the kernel with the largest total time: its
    algorithmic bytes per launch (the hot-path definition's bytes per cell times the
    cells) over its mean launch time, against the 8 TB/s peak; the same with the
    bytes as stored next to it, and the counters' HBM bytes when they were taken on
    these kernel sources."""
    per_cell = algorithmic_bytes_per_cell(k, precision)
    stored = stored_bytes_per_cell(k, precision)
    kernels = {}
    for name, (ms, n) in prof.items():
        if n == 0:
            continue
        avg_s = ms / n / 1e3
        alg = per_cell[name] * n_cell
        kernels[name] = {"avg_us": avg_s * 1e6, "launches": n, "alg_bytes": alg,
                         "gbs": alg / avg_s / 1e9, "gbs_as_stored": stored[name] * n_cell / avg_s / 1e9}
    dom = max(kernels, key=lambda x: kernels[x]["avg_us"] * kernels[x]["launches"])
    kd = kernels[dom]
    traffic = load_traffic(dom, workload)
    return {
        "bound": "hbm",
        "kernel": dom,
        "achieved": round(kd["gbs"], 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(kd["gbs"] / PEAK_HBM_GBS, 4),
        "traffic": traffic,
        "alg_bytes_per_cell": round(per_cell[dom], 1),
        "alg_bytes_per_launch": int(kd["alg_bytes"]),
        "avg_launch_us": round(kd["avg_us"], 2),
        "as_stored": {"bytes_per_cell": round(stored[dom], 1), "achieved": round(kd["gbs_as_stored"], 1),
                      "frac": round(kd["gbs_as_stored"] / PEAK_HBM_GBS, 4)},
        "valu": load_valu(dom, workload),
    }, {n: {kk: (round(v, 2) if isinstance(v, float) else v) for kk, v in kd_.items()}
        for n, kd_ in kernels.items()}


def host_cpu():
    """CPU model (from /proc/cpuinfo) and the processors this process may use."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return model, usable


def cpu_baseline(mesh, kind, params, k, budget_s=12.0, threads=0):
    """The oracle as it stands (FP64, its cell loops on `threads` OpenMP threads, 0
    for every usable processor; results bit for bit those of one thread) on a
    bounded sample of the same workload: whole SSP-RK3 steps from the same initial
    data until about `budget_s` seconds have run (at least one step)."""
    import oracle
    used = oracle.set_threads(threads)
    try:
        o = oracle.Oracle(mesh, k)
        o.init_problem(kind, params)
        steps = 0
        t0 = time.perf_counter()
        while True:
            assert o.step() == 0
            steps += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        t1 = time.perf_counter()
    finally:
        oracle.set_threads(0)
    nm = (k + 1) * (k + 2) // 2
    dof_stages = mesh.n_cell * 4 * nm * 3 * steps
    model, usable = host_cpu()
    return {"value": dof_stages / (t1 - t0), "unit": "DOF-stage updates/s", "cores": used,
            "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps (3 stages each) of the same {mesh.n_cell}-cell P{k} workload "
                      f"from its initial data, C oracle on {used} thread(s) ({t1 - t0:.1f} s)",
            "host_cpu": model, "host_threads": usable}


def build_meshes(jobs, tasks):
    """Runs the mesh builders `tasks` (a list of (function, args)) in `jobs` spawned
    worker processes (none when jobs <= 1); returns their results in order.  Called
    before this process touches the GPU."""
    if jobs <= 1 or len(tasks) <= 1:
        return [fn(*a) for fn, a in tasks]
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=jobs, mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(fn, *a) for fn, a in tasks]
        return [f.result() for f in futs]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=200_000)
    ap.add_argument("--blast-steps", type=int, default=10, help="timed steps of the ~1M-cell blast; 0 skips it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work per CPU figure")
    ap.add_argument("--only-serving", action="store_true", help="run the serving workload alone")
    ap.add_argument("--only-largest", action="store_true",
                    help="run only the largest P2 mesh (22,368,256 periodic cells), FP64 and mixed")
    ap.add_argument("--largest-steps", type=int, default=5,
                    help="timed steps of the largest P2 mesh per precision; 0 skips it")
    ap.add_argument("--only-blast", action="store_true",
                    help="run only the ~1M-cell blast, FP64 and mixed (for counter runs)")
    ap.add_argument("--serving-requests", type=int, default=8, metavar="N",
                    help="serving run with N requests per arrival rate; 0 skips it")
    ap.add_argument("--serving-rates", type=str, default="1,4,16", help="arrival rates per second")
    ap.add_argument("--serving-scale", type=int, default=1, metavar="S",
                    help="serving request sizes 1k-2M divided by S")
    ap.add_argument("--serving-t-scale", type=float, default=1.0,
                    help="serving final times [0.05, 0.5] multiplied by this")
    ap.add_argument("--batch-scale", type=int, default=1, metavar="S",
                    help="64-instance batch with sizes divided by S (1: the full 5k-500k sizes); 0 skips it")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-copy-bandwidth", action="store_true",
                    help="skip the device-to-device copy that measures the practical HBM rate")
    ap.add_argument("--no-decompositions", action="store_true",
                    help="skip the optimal-vs-classical decomposition comparison (Sec. 6)")
    ap.add_argument("--jobs", type=int, default=0,
                    help="processes building the meshes before the GPU is touched (0: up to 16)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized buffer 5 times (reference kernel for HBM counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "copies": 5}), flush=True)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the stage runs on one GPU and is not sharded across GPUs.", file=sys.stderr)
        sys.exit(2)

    from synth import workloads
    jobs = args.jobs if args.jobs > 0 else min(16, host_cpu()[1] or 1)
    k = 2
    nm = (k + 1) * (k + 2) // 2

    # every mesh is built before the GPU is touched (the builders may run in
    # spawned processes)
    t_build = time.perf_counter()
    tasks = []
    only = args.only_blast or args.only_serving or args.only_largest
    if not only:
        tasks.append((workloads.quadrant_delaunay, (args.cells,)))
    if (args.blast_steps > 0 and not only) or args.only_blast:
        tasks.append((workloads.blast_delaunay, ()))
    if not only and args.batch_scale > 0:
        btasks, bdeg = batch_tasks(args.batch_scale)
        tasks += btasks
    else:
        btasks, bdeg = [], []
    if not (args.only_blast or args.only_largest) and args.serving_requests > 0:
        sspecs, stasks = serving_tasks(args.serving_requests, args.serving_scale, args.serving_t_scale)
        tasks += stasks
    else:
        sspecs, stasks = [], []
    log(f"building {len(tasks)} meshes in {jobs} processes")
    built = build_meshes(jobs, tasks)
    log(f"meshes built in {time.perf_counter() - t_build:.1f} s")
    pos = 0
    quad = blastw = None
    if not only:
        quad = built[pos]
        pos += 1
    if (args.blast_steps > 0 and not only) or args.only_blast:
        blastw = built[pos]
        pos += 1
    binst = built[pos:pos + len(btasks)]
    pos += len(btasks)
    sbuilt = {sp["id"]: built[pos + i] for i, sp in enumerate(sspecs)}

    import torch
    from paper_2409_09620_amd import binding
    if not os.path.exists(binding.lib_path()):
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)

    def measure(m, kd, pr, precision, steps, warmup, tag_):
        workload_ = f"{tag_}_{precision}"
        el, eager_, prof_, d_ = run_gpu(m, kd, pr, k, steps, warmup, precision)
        roof_, per_k = roofline(prof_, k, m.n_cell, workload_, precision)
        return {"value": m.n_cell * 4 * nm * 3 * steps / el, "ms_per_step": el / steps * 1e3,
                "ms_per_step_eager_with_events": eager_ / steps * 1e3, "workload": workload_,
                "roofline": roof_, "kernels": per_k,
                "run": {"t": d_["t"], "step": d_["step"], "alpha": d_["alpha"], "n_limited": d_["n_limited"],
                        "n_flat": d_["n_flat"], "n_bad": d_["n_bad"]}}

    def blast(steps):
        bm, bk, bp = blastw
        btag = f"p2_blast_delaunay_{bm.n_cell // 1000}k"
        log(f"blast: {bm.n_cell} cells, {steps} steps per precision")
        return {pr: dict(measure(bm, bk, bp, pr, steps, 2, btag), cells=bm.n_cell, steps=steps)
                for pr in ("fp64", "mixed")}

    if args.only_blast:
        print(json.dumps({"blast": blast(max(args.steps, 1))}), flush=True)
        return
    def largest(steps):
        lm, lk, lp = workloads.largest_periodic()
        log(f"largest mesh: {lm.n_cell} cells, {steps} steps per precision")
        return {pr: dict(measure(lm, lk, lp, pr, steps, 2, "p2_periodic_vortex_22m"), cells=lm.n_cell, steps=steps)
                for pr in ("fp64", "mixed")}

    if args.only_largest:
        print(json.dumps({"largest": largest(max(args.steps, 1))}), flush=True)
        return
    if args.only_serving:
        rates = [float(x) for x in args.serving_rates.split(",") if x]
        print(json.dumps({"serving": run_serving(sspecs, sbuilt, rates, args.serving_scale,
                                                 args.serving_t_scale)}), flush=True)
        return

    mesh, kind, params = quad
    tag = f"p2_quadrant_delaunay_{args.cells // 1000}k"
    log(f"main workload: {mesh.n_cell} cells")
    r64 = measure(mesh, kind, params, "fp64", args.steps, args.warmup, tag)
    rmx = measure(mesh, kind, params, "mixed", args.steps, args.warmup, tag)
    out = {
        "metric": "P2 Euler DG DOF-stage updates/s (FP32 vs FP64) + serving p50/p99 latency",
        "value": r64["value"],
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": r64["workload"], "cells": mesh.n_cell, "degree": k, "dof_per_cell": 4 * nm,
                   "stages_per_step": 3, "precision": "fp64", "mesh": "poisson-disk delaunay",
                   "problem": "four-quadrant riemann", "parallelism": "single-gpu"},
        "roofline": r64["roofline"],
        "kernels": r64["kernels"],
        "ms_per_step_eager_with_events": r64["ms_per_step_eager_with_events"],
        "run": dict(r64["run"], device=torch.cuda.get_device_name(0)),
        "mixed": dict(rmx, dtype="f32 bulk / f64 averages and limiter",
                      speedup_vs_fp64=rmx["value"] / r64["value"]),
    }
    if blastw is not None:
        out["blast"] = blast(args.blast_steps)
    if args.largest_steps > 0:
        out["largest"] = largest(args.largest_steps)
    if not args.no_copy_bandwidth:
        out["measured_copy_bandwidth"] = copy_bandwidth()
    if not args.no_decompositions:
        out["decompositions"] = dict(run_decompositions(mesh, kind, params),
                                     workload=f"{tag}, P1 and P2 FP64, same t_end (150 x the optimal decomposition's first dt)")
    if binst:
        out["batch"] = {pr: run_batch(binst, bdeg, args.batch_steps, 2, pr) for pr in ("fp64", "mixed")}
        out["batch"]["workload"] = (f"64 two-state instances, sizes log-uniform 5k-500k / {args.batch_scale}, "
                                    "P1/P2 50/50, seeded Delaunay")
    if sspecs:
        rates = [float(x) for x in args.serving_rates.split(",") if x]
        out["serving"] = run_serving(sspecs, sbuilt, rates, args.serving_scale, args.serving_t_scale)
    if not args.no_cpu_baseline:
        base = cpu_baseline(mesh, kind, params, k, budget_s=args.cpu_budget, threads=0)
        one = cpu_baseline(mesh, kind, params, k, budget_s=args.cpu_budget / 2, threads=1)
        base["single_thread"] = {"value": one["value"], "cores": 1, "sample": one["sample"]}
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
