"""Benchmark of the matrix-free P1 pressure solve on one MI355X.

Default workload (one step): the 3D unit cube, 160^3 cells x 6 tetrahedra
(24,576,000 tets, 4,173,281 nodes, Morton order), interior nodes jittered
by up to 0.2h, c = 1/rho with rho lognormal(0, 0.5) per element, w = 1e-4,
and one FP64 CG solve to rtol 1e-10 from x0 = 0.  The right-hand side is
b = A_D x* with x* = prod sin(pi x_i), computed once before timing.  The
same system is then solved by FP32-inner defect correction (FP64
corrections), timed after the FP64 region.

Prints one JSON line: GDOF*iter/s (free nodes x CG iterations per second,
whole job), solves/s, p50/p99 solve latency, the roofline of the operator
apply kernel (algorithmic bytes / measured average kernel duration against
the 8 TB/s HBM peak, with the rocprofv3-measured HBM bytes when the
committed record matches the kernel source), the mixed-precision speedup,
two extra legs (the 64^3 cube over w in {1e-6, 1e-3, 1}, and the latency of
the 2D 32 x 32 square at rtol 1e-12) and the CPU oracle timed on the host
(one thread on a bounded sample, and all host cores on the whole solve,
whose solution the GPU's are compared with).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pressure-solve GDOF·iter/s + % HBM peak; solves/s & p50/p99 latency at rtol 1e-10"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2301_08357_amd", "csrc", "pressure.hip")


def measured_traffic(workload, n_tiles, tiled):
    """HBM bytes per apply launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE measurement of this workload (profiles/apply_<workload>_traffic.json),
    if it was taken on the current kernel source and the same launch: the
    tiled kernel over the same number of tiles."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "apply_%s_traffic.json" % workload)
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha or not tiled or rec.get("n_tiles") != n_tiles:
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_info():
    cpu = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cpu


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--tile", type=int, default=-1,
                    help="Morton tile nodes (128/256/512; 0 = the library default, 128; -1 = the size the library's "
                         "tile autotuner picks, on the cube160 line, else the default)")
    ap.add_argument("--inner-rtol", type=float, default=1e-2,
                    help="residual drop of the FP32 inner CG between FP64 corrections (mixed solve)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--workload", default="cube160",
                    choices=["cube160", "cube64", "cube160p", "projection160", "transport160", "timestep160",
                             "batch256", "serve", "copy", "tgv2d32"],
                    help="cube160 (default line) or one of the other synthetic workloads")
    ap.add_argument("--no-extras", action="store_true", help="cube160: skip the cube64 and tgv2d_32 legs")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="single-thread oracle sample length (seconds of CG iterations)")
    ap.add_argument("--requests", type=int, default=10000, help="serving: number of requests")
    ap.add_argument("--budget-gb", type=float, default=0.0, help="serving: HBM budget (0 = 80%% of free)")
    ap.add_argument("--serve-mixed", action="store_true", help="serving: mixed-precision solves")
    ap.add_argument("--lumped", action="store_true", help="cube160/cube160p: lumped (diagonal) mass matrix")
    ap.add_argument("--mu", type=float, default=0.0,
                    help="transport160/timestep160: dynamic viscosity of the transport stage (0: inviscid)")
    ap.add_argument("--lam", type=float, default=0.0,
                    help="transport160/timestep160: thermal conductivity (gas constant R = 1; 0: no heat flux)")
    ap.add_argument("--lader", action="store_true",
                    help="transport160: the second-order LADER step (Sec. 3.2.1) instead of the first-order one")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "cube64":
        return bench_cube64(args)
    if args.workload in ("cube160", "cube160p"):
        return bench_cube160(args)
    if args.workload == "projection160":
        return bench_projection(args)
    if args.workload == "transport160":
        return bench_transport(args)
    if args.workload == "timestep160":
        return bench_timestep(args)
    if args.workload == "batch256":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "copy":
        return bench_copy(args)
    if args.workload == "tgv2d32":
        return bench_tgv2d32(args)


def bench_tgv2d32(args):
    """The small 2D case alone: --steps x 100 single solves of tgv2d_32 (each
    one launch of the one-workgroup solver, a state read and the scatter);
    the line's value is the p50 latency."""
    rec = extra_tgv2d32(args, solves=100 * max(1, args.steps))
    print(json.dumps({"metric": "tgv2d_32 single-solve latency (FP64 CG to rtol 1e-12)",
                      "value": rec["latency_ms_p50"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": rec["workload"]}, **{k: v for k, v in rec.items() if k != "workload"}}))


def tile_flag_of(args):
    """PM_TILE_* flag of --tile (-1, the autotuner, counts as the default here)."""
    import paper_2301_08357_amd as pm
    return {-1: 0, 0: 0, 128: pm.PM_TILE_128, 256: pm.PM_TILE_256, 512: pm.PM_TILE_512}[args.tile]


def bench_cube64(args):
    """The 64^3 cube (1,572,864 tets, 274,625 nodes, no jitter), c = 1/rho
    with rho ~ U[0.5, 2] per element, one FP64 CG solve to rtol 1e-10 from
    x0 = 0 for each w in {1e-6, 1e-3, 1} per step."""
    import torch
    import paper_2301_08357_amd as pm
    from synth import workloads
    dev = torch.device("cuda:0")
    ws = workloads.CUBE64_W
    probs = [workloads.cube64(w) for w in ws]
    m = probs[0].mesh
    tile_flag = tile_flag_of(args)
    flags = pm.PM_FP64 | pm.PM_FP32_INNER | tile_flag
    systems = [pm.PressureSystem.from_problem(p, flags=flags) for p in probs]
    for s in systems:
        s.set_variant(args.variant)
    info = systems[0].info()
    xstar = torch.tensor(probs[0].extra["xstar"], device=dev)
    rhs = [s.apply(xstar) for s in systems]
    torch.cuda.synchronize()

    def step(lat=None, iters=None):
        for s, b in zip(systems, rhs):
            t0 = time.perf_counter()
            r = s.solve(b, rtol=args.rtol, max_iter=20000)
            t1 = time.perf_counter()
            if r.status != 0:
                raise RuntimeError("solve status %d" % r.status)
            if lat is not None:
                lat.append(t1 - t0)
                iters.append(r.iters)
        return r

    for _ in range(args.warmup):
        step()
    for s in systems:
        s.timing_enable(True)
    lat, iters = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        last = step(lat, iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    n_free = info["n_free"]
    dofiter = float(n_free) * float(sum(iters))
    value = dofiter / elapsed / 1e9

    launches, ms = 0, 0.0
    for s in systems:
        n, t = s.timing_read()
        launches += n
        ms += t
    avg_ms = ms / max(launches, 1)
    achieved = info["apply_bytes"] / (avg_ms * 1e-3) / 1e9
    err = float(torch.linalg.norm(last.p - xstar) / torch.linalg.norm(xstar))

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GDOF*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded structured 64^3 Kuhn mesh, rho~U[0.5,2])",
        "config": {
            "workload": "cube64: unit cube 64^3 x 6 tets (1,572,864 tets, 274,625 nodes), c=1/rho, "
                        "rho~U[0.5,2], w in {1e-6,1e-3,1}, FP64 matrix-free CG to rtol %g from x0=0, "
                        "Morton order; one step = one solve per w" % args.rtol,
            "n_nodes": info["n_nodes"], "n_free": n_free, "n_elems": info["n_elems"],
            "w": list(ws), "rtol": args.rtol,
            "iterations_per_solve": iters[: len(ws)],
        },
        "solves_per_s": round(len(lat) / elapsed, 3),
        "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "rel_error_vs_manufactured": err,
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("cube64", info["n_tiles"], args.variant != pm.PM_VARIANT_NODE),
            "kernel": "operator apply (fused CG iteration)",
            "bytes_per_launch": info["apply_bytes"], "avg_launch_us": round(avg_ms * 1e3, 3),
            "launches": launches,
        },
    }
    tr = out["roofline"]["traffic"]
    if tr:
        # the rate of the measured HBM traffic (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a copy)
        out["roofline"]["traffic_achieved"] = round(tr / (avg_ms * 1e-3) / 1e9, 1)
        out["roofline"]["traffic_frac"] = round(tr / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    if not args.no_mixed:
        out["mixed"] = mixed_comparison(systems, rhs, xstar, args, elapsed / len(lat))
    if not args.no_cpu:
        out["cpu_baseline"], x_oracle, b_oracle = cpu_baseline_cube64(probs)
        # error of each GPU solve against the oracle's FP64 solution of the
        # same system (the oracle's right-hand side), per w
        def vs_oracle(xg, xo):
            return float(np.linalg.norm(xg.cpu().numpy() - xo) / np.linalg.norm(xo))
        bo = [torch.tensor(b, device=dev) for b in b_oracle]
        out["error_vs_oracle"] = {
            "fp64": [vs_oracle(s.solve(b, rtol=args.rtol).p, xo) for s, b, xo in zip(systems, bo, x_oracle)]}
        if not args.no_mixed:
            out["error_vs_oracle"]["mixed"] = [
                vs_oracle(s.solve_mixed(b, rtol=args.rtol, inner_rtol=args.inner_rtol).p, xo)
                for s, b, xo in zip(systems, bo, x_oracle)]
    print(json.dumps(out), flush=True)
    for s in systems:
        s.close()


def _common(args, metric_value, unit, ms_per_step, config, extra):
    out = {"metric": METRIC, "value": metric_value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_cube160(args):
    """160^3 x 6 tets, jitter 0.2h, rho lognormal(0, 0.5), w = 1e-4: FP64 CG
    and FP32-inner defect correction, both to rtol 1e-10 (the default line,
    with the cube64 and tgv2d_32 legs and the CPU oracle).  cube160p: the
    same recipe on the fully periodic mesh with merged images; --lumped: the
    lumped mass matrix (these two print the solve and roofline only).  The
    default line takes the Morton tile size the library's autotuner picks for
    the mesh (tuned before the timed region; --tile fixes it instead)."""
    import torch
    import paper_2301_08357_amd as pm
    from synth import workloads
    periodic = args.workload == "cube160p"
    prob = workloads.cube160p() if periodic else workloads.cube160()
    if args.lumped:
        prob = workloads.lumped(prob)
    main_line = not periodic and not args.lumped
    tile_flag = tile_flag_of(args)
    tuning_s = None
    if args.tile == -1 and main_line:
        # the library's tile autotuner (pressure_tune_tile): CG iterations at
        # each Morton tile size, the fastest kept (cached per device and build)
        t_tune = time.perf_counter()
        try:
            tuned, _ = pm.tune_tile(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER, iters=32)
        except OSError:   # no writable cache directory: tune without a cache
            tuned, _ = pm.tune_tile(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER, iters=32, cache=False)
        tile_flag = tuned & 0xF0
        tuning_s = round(time.perf_counter() - t_tune, 2)
    tile_nodes = {0: 128, pm.PM_TILE_128: 128, pm.PM_TILE_256: 256, pm.PM_TILE_512: 512}[tile_flag]
    t_setup = time.perf_counter()
    s = pm.PressureSystem.from_problem(prob, flags=pm.PM_FP64 | pm.PM_FP32_INNER | tile_flag)
    t_setup = time.perf_counter() - t_setup
    s.set_variant(args.variant)
    info = s.info()
    xs = torch.tensor(prob.extra["xstar"], device="cuda")
    b = s.apply(xs)
    for _ in range(args.warmup):
        s.solve(b, rtol=args.rtol)
    s.timing_enable(True)
    torch.cuda.synchronize()
    lat, its = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ta = time.perf_counter()
        r = s.solve(b, rtol=args.rtol)
        lat.append(time.perf_counter() - ta)
        its.append(r.iters)
        if r.status != 0:
            raise RuntimeError("solve status %d" % r.status)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    n, ms = s.timing_read()
    s.timing_enable(False)
    avg = ms / max(n, 1)
    achieved = info["apply_bytes"] / (avg * 1e-3) / 1e9
    value = info["n_free"] * sum(its) / el / 1e9
    err = float(torch.linalg.norm(r.p - xs) / torch.linalg.norm(xs))
    if periodic:
        what = ("cube160p: unit cube 160^3 x 6 tets, periodic along x, y and z with merged images "
                "(24,576,000 tets, 4,096,000 nodes)")
    else:
        what = "cube160: unit cube 160^3 x 6 tets (24,576,000 tets, 4,173,281 nodes)"
    tiled = args.variant != pm.PM_VARIANT_NODE
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload, info["n_tiles"], tiled) if main_line else None,
            "kernel": "operator apply (fused CG iteration)",
            "bytes_per_launch": info["apply_bytes"], "avg_launch_us": round(avg * 1e3, 3), "launches": n}
    if roof["traffic"]:
        # the rate of the measured HBM traffic (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a copy)
        roof["traffic_achieved"] = round(roof["traffic"] / (avg * 1e-3) / 1e9, 1)
        roof["traffic_frac"] = round(roof["traffic_achieved"] / HBM_PEAK_GBS, 4)
    out = {"metric": METRIC, "value": round(value, 4), "unit": "GDOF*iter/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded jittered 160^3 Kuhn mesh, rho lognormal)",
           "config": {"workload": what + ", jitter 0.2h, rho~lognormal(0,0.5), w=1e-4, %s mass, FP64 matrix-free CG "
                                         "to rtol %g from x0=0, b = A x* with x* = prod sin(pi x_i), Morton order; one "
                                         "step = one solve" % ("lumped" if args.lumped else "consistent", args.rtol),
                      "n_nodes": info["n_nodes"], "n_free": info["n_free"], "n_elems": info["n_elems"],
                      "tile_nodes": tile_nodes, "n_tiles": info["n_tiles"],
                      "tile_choice": "autotuner" if tuning_s is not None else "fixed",
                      "rtol": args.rtol, "iterations": its[0]},
           "solves_per_s": round(args.steps / el, 3),
           "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
           "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
           "setup_s": round(t_setup, 2), "tile_tuning_s": tuning_s,
           "rel_error_vs_manufactured": err, "roofline": roof}
    if not args.no_mixed:
        out["mixed"] = mixed_comparison([s], [b], xs, args, el / args.steps)
    if main_line and not args.no_extras:
        out["cube64"] = extra_cube64(args)
        out["tgv2d_32"] = extra_tgv2d32(args)
    if main_line and not args.no_cpu:
        out["cpu_baseline"], out["error_vs_oracle"] = cpu_baseline_cube160(prob, s, args)
        if not args.no_extras:
            out["cpu_baseline"]["other_configs"] = oracle_other_configs(args)
    print(json.dumps(out), flush=True)
    s.close()


def extra_cube64(args, reps=3):
    """The 64^3 cube (no jitter, rho ~ U[0.5, 2]) over w in {1e-6, 1e-3, 1}:
    reps FP64 solves per w to rtol 1e-10, with the apply's roofline."""
    import torch
    import paper_2301_08357_amd as pm
    from synth import workloads
    probs = [workloads.cube64(w) for w in workloads.CUBE64_W]
    systems = [pm.PressureSystem.from_problem(p) for p in probs]
    info = systems[0].info()
    xs = torch.tensor(probs[0].extra["xstar"], device="cuda")
    rhs = [q.apply(xs) for q in systems]
    for q, b in zip(systems, rhs):
        q.solve(b, rtol=args.rtol)
        q.timing_enable(True)
    torch.cuda.synchronize()
    lat, its = [], []
    t0 = time.perf_counter()
    for _ in range(reps):
        for q, b in zip(systems, rhs):
            ta = time.perf_counter()
            r = q.solve(b, rtol=args.rtol)
            lat.append(time.perf_counter() - ta)
            its.append(r.iters)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nl, ms = 0, 0.0
    for q in systems:
        a, t = q.timing_read()
        nl, ms = nl + a, ms + t
        q.close()
    avg = ms / max(nl, 1)
    ach = info["apply_bytes"] / (avg * 1e-3) / 1e9
    return {"workload": "cube64: 64^3 x 6 tets (1,572,864 tets, 274,625 nodes), no jitter, rho~U[0.5,2], "
                        "w in {1e-6,1e-3,1}, FP64 CG to rtol %g, %d solves per w" % (args.rtol, reps),
            "value": round(info["n_free"] * sum(its) / el / 1e9, 4), "unit": "GDOF*iter/s",
            "iterations": its[:3], "solves_per_s": round(len(lat) / el, 2),
            "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                         "avg_launch_us": round(avg * 1e3, 3), "bytes_per_launch": info["apply_bytes"],
                         "traffic": measured_traffic("cube64", info["n_tiles"], True)}}


def extra_tgv2d32(args, solves=300):
    """The 2D unit square, 32 x 32 cells x 2 triangles (2048 tris, 1089
    nodes), jitter 0.2h, c = 1, w = 1e-2, Dirichlet boundary, FP64 CG to
    rtol 1e-12 from x0 = 0: latency of single solves (a latency-bound size).
    The right-hand side is b = A_D p* with p* = sin(pi x) sin(pi y) at the
    nodes (computed by the library, so that the timed path calls nothing
    else)."""
    import torch
    import paper_2301_08357_amd as pm
    from synth import fields, workloads
    prob = workloads.tgv2d(32)
    q = pm.PressureSystem.from_problem(prob)
    b = q.apply(torch.tensor(fields.sine_product(prob.mesh.coords), device="cuda"))
    for _ in range(10):
        q.solve(b, rtol=1e-12)
    torch.cuda.synchronize()
    lat, its = [], []
    t0 = time.perf_counter()
    for _ in range(solves):
        ta = time.perf_counter()
        r = q.solve(b, rtol=1e-12)
        lat.append(time.perf_counter() - ta)
        its.append(r.iters)
    el = time.perf_counter() - t0
    info = q.info()
    nfree = info["n_free"]
    q.close()
    return {"workload": "tgv2d_32: unit square 32x32 x 2 tris (2048 tris, 1089 nodes), jitter 0.2h, c=1, w=1e-2, "
                        "FP64 CG to rtol 1e-12, b = A_D p*, %d single solves" % solves,
            "solves_per_s": round(solves / el, 1), "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 4),
            "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 4), "iterations": its[0],
            "GDOF_iter_per_s": round(nfree * sum(its) / el / 1e9, 4),
            "one_launch_solve": bool(info["one_launch_solve"])}


def oracle_other_configs(args, single_seconds=6.0):
    """The CPU oracle on the other fixed configurations, beside the GPU:
    tgv2d_32 (to rtol 1e-12), cube64 (the three w, to rtol 1e-10) and 16
    meshes of the batched mix (to rtol 1e-10; the GPU solves them as one
    batch at the tuned shape).  Assembly is not timed; each oracle solve runs
    on all host cores and on one thread (the batch subset on one thread over
    its first meshes, about single_seconds)."""
    import torch
    import oracle
    import paper_2301_08357_amd as pm
    from synth import fields, workloads
    cores = len(os.sched_getaffinity(0))

    def solve_all(cases, rtol, threads, budget=None):
        oracle.set_threads(threads)
        t_sum, dofit, iters = 0.0, 0.0, []
        for A, b, nfree, dirichlet in cases:
            ta = time.perf_counter()
            _, st, it, _, _ = oracle.cg(A, b, rtol=rtol, max_iter=20000, dirichlet=dirichlet)
            t_sum += time.perf_counter() - ta
            dofit += nfree * it
            iters.append(it)
            if budget is not None and t_sum > budget:
                break
        oracle.set_threads(1)
        return {"value": round(dofit / t_sum / 1e9, 5), "seconds": round(t_sum, 3), "iterations": iters}

    out = {"cores": cores}
    # tgv2d_32: b = A p* (the oracle's operator), repeated to about 0.2 s
    prob = workloads.tgv2d(32)
    A = oracle.assemble_problem(prob)
    b = A.matvec(fields.sine_product(prob.mesh.coords))
    nf = int((prob.mesh.dirichlet == 0).sum())
    reps = 40
    one = [(A, b, nf, prob.mesh.dirichlet)] * reps
    out["tgv2d_32"] = {"all_cores": solve_all(one, 1e-12, cores), "single_thread": solve_all(one, 1e-12, 1),
                       "solves": reps}
    for k in ("all_cores", "single_thread"):
        rec = out["tgv2d_32"][k]
        rec["latency_ms"] = round(rec["seconds"] / reps * 1e3, 4)
        rec["iterations"] = rec["iterations"][0]
    # cube64: the three w
    cases = []
    for w in workloads.CUBE64_W:
        prob = workloads.cube64(w)
        A = oracle.assemble_problem(prob)
        cases.append((A, A.matvec(prob.extra["xstar"]), int((prob.mesh.dirichlet == 0).sum()), prob.mesh.dirichlet))
    out["cube64"] = {"all_cores": solve_all(cases, args.rtol, cores), "single_thread": solve_all(cases, args.rtol, 1)}
    # 16 meshes of the batched mix, and the GPU's batched solve of the same systems
    params = workloads.batch_params()
    probs = [workloads.batch_problem(i, params) for i in workloads.batch_sample(16, params)]
    cases = []
    for prob in probs:
        A = oracle.assemble_problem(prob)
        cases.append((A, A.matvec(prob.extra["xstar"]), int((prob.mesh.dirichlet == 0).sum()), prob.mesh.dirichlet))
    out["batch16"] = {"all_cores": solve_all(cases, args.rtol, cores),
                      "single_thread": solve_all(cases, args.rtol, 1, budget=single_seconds)}
    systems = [pm.PressureSystem.from_problem(p) for p in probs]
    rhs = [torch.tensor(c[1], device="cuda") for c in cases]
    batch = pm.PressureBatch(systems, tiles_per_slot=8, nodes_per_lane=4)
    batch.solve(rhs, rtol=args.rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_rep, dofit = 3, 0.0
    for _ in range(n_rep):
        code, res = batch.solve(rhs, rtol=args.rtol)
        if code != 0:
            raise RuntimeError("batch16 status %d" % code)
        dofit += sum(c[2] * r.iters for c, r in zip(cases, res))
    el = time.perf_counter() - t0
    out["batch16"]["gpu"] = {"value": round(dofit / el / 1e9, 4), "solves_per_s": round(16 * n_rep / el, 1),
                             "ms_per_batched_solve": round(el / n_rep * 1e3, 3),
                             "iterations": [r.iters for r in res]}
    batch.close()
    for q in systems:
        q.close()
    out["unit"] = "GDOF*iter/s"
    out["note"] = ("oracle: assembled CSR + textbook CG (OpenMP SpMV rows, fixed-order dots on all cores); "
                   "GPU figures for tgv2d_32 and cube64 are the line's tgv2d_32 and cube64 entries")
    return out


def cpu_baseline_cube160(prob, s, args):
    """The CPU oracle (assembled CSR, textbook CG) on the cube160 system:
    one thread on a bounded sample of CG iterations (about --cpu-seconds),
    and all host cores (OpenMP SpMV rows, fixed-order chunked dots) on the
    whole solve to rtol, bounded at about 60 s.  Assembly is not timed.
    Then the GPU solves (FP64 and mixed) of the oracle's right-hand side
    b = A x*, each accepted by the oracle's operator and compared with the
    oracle's solution and with x*."""
    import torch
    import oracle
    m = prob.mesh
    t0 = time.perf_counter()
    A = oracle.assemble_problem(prob)
    t_asm = time.perf_counter() - t0
    xs = prob.extra["xstar"]
    b = A.matvec(xs)
    nfree = int((m.dirichlet == 0).sum())
    cores = len(os.sched_getaffinity(0))

    def timed_cg(k, rtol=1e-300):
        ta = time.perf_counter()
        x, st, it, _, tr = oracle.cg(A, b, rtol=rtol, max_iter=k, dirichlet=m.dirichlet)
        return time.perf_counter() - ta, x, st, it, tr

    oracle.set_threads(1)
    t8 = timed_cg(8)[0]
    k1 = max(8, int(8 * args.cpu_seconds / max(t8, 1e-3)))
    t1, _, _, it1, _ = timed_cg(k1)
    single = nfree * it1 / t1 / 1e9
    oracle.set_threads(cores)
    t8 = timed_cg(8)[0]
    cap = max(8, int(8 * 60.0 / max(t8, 1e-3)))
    ta, x_o, st_o, it_o, tr_o = timed_cg(min(20000, cap), rtol=args.rtol)
    oracle.set_threads(1)
    allc = nfree * it_o / ta / 1e9
    base = {"value": round(allc, 5), "unit": "GDOF*iter/s", "cores": cores, "kind": "oracle",
            "sample": "cube160 FP64 CG (assembled CSR, assembly %.1f s not timed) on all %d host cores: %d iterations "
                      "in %.1f s (%s); one thread: %d iterations in %.1f s = %.5f GDOF*iter/s; %s"
                      % (t_asm, cores, it_o, ta, "converged" if st_o == 0 else "bounded sample", k1, t1, single,
                         cpu_info()),
            "single_thread": {"value": round(single, 5), "iterations": it1, "seconds": round(t1, 2)},
            "all_cores": {"value": round(allc, 5), "iterations": it_o, "seconds": round(ta, 2), "status": st_o}}
    bd = torch.tensor(b, device="cuda")
    checks = {"rhs": "the oracle's b = A x*"}
    for name, res in (("fp64", s.solve(bd, rtol=args.rtol)),
                      ("mixed", None if args.no_mixed else s.solve_mixed(bd, rtol=args.rtol,
                                                                          inner_rtol=args.inner_rtol))):
        if res is None:
            continue
        x = res.p.cpu().numpy()
        rec = {"status": res.status, "iterations": res.iters,
               "oracle_relres": float(np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)),
               "rel_error_vs_xstar": float(np.linalg.norm(x - xs) / np.linalg.norm(xs))}
        if st_o == 0:
            rec["rel_diff_vs_oracle_solution"] = float(np.linalg.norm(x - x_o) / np.linalg.norm(x_o))
        checks[name] = rec
    checks["oracle_iterations"] = it_o
    return base, checks


def bench_projection(args):
    """One projection stage per step (Sec. 3.3-3.5: dual->primal means, N_Pic
    = 2 Picard iterations of weak-problem RHS + FP64 CG + updates, momentum
    on the dual cells) on the cube160 mesh (jitter 0.2h, Dirichlet boundary
    with prescribed P^{n+1}, boundary normal flux), gamma = 1.4, Mach 0.1,
    dt = 0.5 h / Mach (convective CFL 0.5, acoustic CFL 5), synthetic
    dual-cell fields.  Each step starts from the same P^n with dp0 = 0."""
    import torch
    import paper_2301_08357_amd as pm
    from synth import mesh as smesh
    from synth import projection as sproj
    n = 160
    from synth.rng import MASTER_SEED
    m = smesh.structured_mesh(3, n, jitter=0.2, seed=MASTER_SEED)
    gamma, mach = 1.4, 0.1
    dt = 0.5 * (1.0 / n) / mach
    s = pm.PressureSystem(3, m.coords, m.elems, np.ones(m.n_elems), 1.0 / (gamma - 1.0), dt, m.dirichlet, m.lattice)
    t0 = time.perf_counter()
    fv, fe, nb = s.dual_faces()
    t_faces = time.perf_counter() - t0
    inp = sproj.fields(m, fv, fe, gamma=gamma, mach=mach)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    rho, we, wu, p = dev(inp["rho_f"]), dev(inp["we_f"]), dev(inp["wu_f"]), dev(inp["p"])
    pb, bflux = dev(inp["pb"]), dev(inp["bflux"])
    p_out, wu_out = torch.empty_like(p), torch.empty_like(wu)
    h_out = torch.empty(m.n_elems, dtype=torch.float64, device="cuda")

    def stage():
        return s.projection(rho, we, wu, p, gamma, dt, pb=pb, bflux=bflux, n_picard=2, rtol=args.rtol,
                            p_out=p_out, wu_out=wu_out, h_out=h_out)

    for _ in range(args.warmup):
        stage()
    s.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = None
    for _ in range(args.steps):
        _, _, _, its, st = stage()
        if st != 0:
            raise RuntimeError("projection status %d" % st)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    nl, ms = s.timing_read()
    info = s.info()
    avg = ms / max(nl, 1)
    achieved = info["apply_bytes"] / (avg * 1e-3) / 1e9
    total_it = int(sum(int(i) for i in its))
    _common(args, round(info["n_free"] * total_it / el / 1e9, 4), "GDOF*iter/s", round(el * 1e3, 3),
            {"workload": "projection160: cube 160^3 x 6 tets (24,576,000 tets, 4,173,281 nodes, %d dual cells), "
                         "jitter 0.2h; one step = one projection stage, N_Pic = 2, gamma 1.4, Mach 0.1, dt = 0.5h/Mach, "
                         "FP64 CG to rtol %g" % (fv.shape[0], args.rtol),
             "n_faces": int(fv.shape[0]), "n_boundary_faces": int(nb), "cg_iterations": [int(i) for i in its]},
            {"stages_per_s": round(1.0 / el, 3), "dual_faces_setup_s": round(t_faces, 2),
             "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                          "kernel": "operator apply (fused CG iteration)",
                          "bytes_per_launch": info["apply_bytes"], "avg_launch_us": round(avg * 1e3, 3)}})
    s.close()


def bench_transport(args):
    """One first-order transport step per step (Rusanov flux on the dual
    cells, P1 pressure force, gravity, with --mu / --lam the viscous stress
    and the heat flux) on the
    jittered cube160 mesh with the projection-stage input recipe.
    Algorithmic bytes of a step: the dual-cell
    state read and written (2 x 40 B per cell), the element-to-face and
    face-to-slot maps (16 + 8 B), connectivity (16 B per element), vertex
    coordinates and P^n (32 B per node)."""
    import torch
    import paper_2301_08357_amd as pm
    from synth import mesh as smesh
    from synth import projection as sproj
    from synth.rng import MASTER_SEED
    n = 160
    m = smesh.structured_mesh(3, n, jitter=0.2, seed=MASTER_SEED)
    gamma, mach = 1.4, 0.1
    dt = 0.5 * (1.0 / n) / mach
    s = pm.PressureSystem(3, m.coords, m.elems, np.ones(m.n_elems), 1.0 / (gamma - 1.0), dt, m.dirichlet, m.lattice)
    fv, fe, nb = s.dual_faces()
    inp = sproj.fields(m, fv, fe, gamma=gamma, mach=mach)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    rho, wu, we, p = dev(inp["rho_f"]), dev(inp["wu_f"]), dev(inp["we_f"]), dev(inp["p"])
    outs = (torch.empty_like(rho), torch.empty_like(wu), torch.empty_like(we))
    g = np.array([0.0, 0.0, -1.0])

    def step():
        s.transport(rho, wu, we, p, dt, gravity=g, c_alpha=0.0, mu=args.mu, lam=args.lam, r_gas=1.0,
                    rho_out=outs[0], wu_out=outs[1], we_out=outs[2], lader=args.lader)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    F, E, N = int(fv.shape[0]), int(m.n_elems), int(m.n_nodes)
    alg = F * (80 + 8) + E * (16 + 16) + N * 32
    if args.lader:
        # the element gradients of rho and W_u (12 doubles) written once and read once
        alg += E * 2 * 8 * 12
    ach = alg / el / 1e9
    _common(args, round(F / el / 1e9, 4), "Gcell/s", round(el * 1e3, 3),
            {"workload": "transport160: cube 160^3 x 6 tets (24,576,000 tets, %d dual cells), jitter 0.2h; one step = "
                         "one %s transport step (Mach 0.1, dt = 0.5h/Mach, gravity, mu = %g, "
                         "lambda = %g, R = 1)" % (F, "second-order LADER" if args.lader else "first-order Rusanov",
                                                   args.mu, args.lam),
             "n_faces": F, "mu": args.mu, "lambda": args.lam, "lader": bool(args.lader)},
            {"steps_per_s": round(1.0 / el, 3),
             "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                          "kernel": "transport step (gather of P^n, %sone pass per dual cell), wall time per step"
                                    % ("element gradients, " if args.lader else ""),
                          "bytes_per_step": alg}})
    s.close()


def bench_timestep(args):
    """Whole time steps on the jittered cube160 mesh: first-order transport
    (Sec. 3.2), the projection stage with N_Pic = 2 (Sec. 3.3-3.4) and the
    post-projection energy update (Sec. 3.5); each step starts from the
    previous step's state (P, W_u, W_E, rho), Mach 0.1, dt = 0.5h/Mach,
    Dirichlet boundary pressure held at P^n, walls.  The time step follows
    the rule of Sec. 4, dt = CFL r^2 / (|U|_max r + (8/3) (nu + gamma
    lambda / (c_p rho))_max) with CFL = 1/d, nu = mu / rho, R = 1,
    |U|_max and min rho from the initial state and
    r = 0.17 h, the smallest incircle-diameter estimate 2 d |C| / |dC| of
    the jittered Kuhn dual cells (measured on a 10^3 mesh: 0.177 h)."""
    import torch
    import paper_2301_08357_amd as pm
    from synth import mesh as smesh
    from synth import projection as sproj
    from synth.rng import MASTER_SEED
    n = 160
    m = smesh.structured_mesh(3, n, jitter=0.2, seed=MASTER_SEED)
    gamma, mach = 1.4, 0.1
    s = pm.PressureSystem(3, m.coords, m.elems, np.ones(m.n_elems), 1.0 / (gamma - 1.0), 1.0, m.dirichlet, m.lattice)
    fv, fe, nb = s.dual_faces()
    inp = sproj.fields(m, fv, fe, gamma=gamma, mach=mach)
    umax = float(np.max(np.linalg.norm(inp["wu_f"], axis=1) / inp["rho_f"]))
    # dt = CFL r^2 / (|U|_max r + 2 (4/3) (nu_max + gamma lambda / (c_p rho_min))),
    # nu = mu / rho, c_p = gamma R / (gamma - 1) with R = 1
    r = 0.17 * (1.0 / n)
    rmin = float(np.min(inp["rho_f"]))
    cp = gamma / (gamma - 1.0)
    diff = args.mu / rmin + gamma * args.lam / (cp * rmin)
    dt = (1.0 / 3.0) * r * r / (umax * r + (8.0 / 3.0) * diff)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
    st = {"rho": dev(inp["rho_f"]), "wu": dev(inp["wu_f"]), "we": dev(inp["we_f"]), "p": dev(inp["p"])}
    its_all = []

    def step(st):
        # the first Picard solve starts from the previous step's correction
        rho, wu, we = s.transport(st["rho"], st["wu"], st["we"], st["p"], dt, mu=args.mu, lam=args.lam, r_gas=1.0)
        p_new, wu_new, _, its, code = s.projection(rho, we, wu, st["p"], gamma, dt, dp0=st.get("dp"), n_picard=2,
                                                   rtol=args.rtol)
        if code != 0:
            raise RuntimeError("projection status %d" % code)
        its_all.append([int(i) for i in its])
        we_new = s.post_projection(rho, we, wu_new, p_new, gamma, dt)
        return {"rho": rho, "wu": wu_new, "we": we_new, "p": p_new, "dp": p_new - st["p"]}

    for _ in range(args.warmup):
        st = step(st)
    s.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step(st)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    nl, ms = s.timing_read()
    info = s.info()
    avg = ms / max(nl, 1)
    achieved = info["apply_bytes"] / (avg * 1e-3) / 1e9
    timed = its_all[args.warmup:]
    total_it = sum(sum(x) for x in timed)
    _common(args, round(info["n_free"] * total_it / (el * args.steps) / 1e9, 4), "GDOF*iter/s", round(el * 1e3, 3),
            {"workload": "timestep160: cube 160^3 x 6 tets (24,576,000 tets, 4,173,281 nodes, %d dual cells), jitter "
                         "0.2h; one step = transport + projection (N_Pic = 2, FP64 CG to rtol %g, warm start from "
                         "the previous step's correction) + post-projection, Mach 0.1, dt by the rule of Sec. 4 "
                         "with r = 0.17h, mu = %g, lambda = %g, R = 1" % (fv.shape[0], args.rtol, args.mu, args.lam),
             "dt": dt, "mu": args.mu, "lambda": args.lam, "cg_iterations": timed},
            {"time_steps_per_s": round(1.0 / el, 3),
             "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                          "kernel": "operator apply (fused CG iteration)",
                          "bytes_per_launch": info["apply_bytes"], "avg_launch_us": round(avg * 1e3, 3)}})
    s.close()


def bench_copy(args):
    """The practical HBM ceiling and the counter scale: the hand-written
    probe kernels of libstream_probe.so (csrc/stream_probe.hip) copy 1 GiB
    (read 1 GiB, write 1 GiB) and read 1 GiB, over a sweep of grid sizes
    (best of the steps per grid, HIP events on the probe's stream); torch's
    copy_ of the same buffers for comparison.  Under rocprofv3 --pmc the
    counters of the probe kernels (k_copy, k_read) give the FETCH_SIZE /
    WRITE_SIZE readings of a known byte count."""
    import ctypes
    import torch
    from paper_2301_08357_amd import build as pbuild
    if not os.path.exists(pbuild.PROBE_LIB):
        raise RuntimeError("libstream_probe.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(pbuild.PROBE_LIB)
    lib.stream_probe.restype = ctypes.c_int
    lib.stream_probe.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                 ctypes.c_void_p]
    n = 2 ** 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    res = {}
    for kind, name, nbytes in ((0, "copy", 16 * n), (1, "read", 8 * n)):
        best = {}
        for grid in (1024, 2048, 4096, 8192):
            ts = []
            for _ in range(max(args.steps, 3)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                if lib.stream_probe(kind, a.data_ptr(), b.data_ptr(), n, grid, ctypes.c_void_p(st.cuda_stream)):
                    raise RuntimeError("stream_probe failed")
                e1.record(st)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            best[grid] = round(nbytes / min(ts) / 1e9, 1)
        res[name] = {"bytes_per_launch": nbytes, "GB_per_s_by_grid": best, "GB_per_s_best": max(best.values())}
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    res["torch_copy_GB_per_s"] = round(16 * n / el / 1e9, 1)
    print(json.dumps({"workload": "copy (1 GiB probe kernels)", **res}), flush=True)


def _batch_problems(n):
    from synth import workloads
    params = workloads.batch_params(n)
    return [workloads.batch_problem(i, params) for i in range(n)]


def bench_batch(args):
    """256 meshes (2D and 3D), nodes log-uniform in [2e3, 2e5], w log-uniform
    in [1e-6, 1]: one batched FP64 solve of all of them per step, in the
    launch shape picked by the library's autotuner; then the same batch as
    mixed-precision solves (FP32 inner CG, FP64 corrections), timed after."""
    import torch
    import paper_2301_08357_amd as pm
    probs = _batch_problems(256)
    systems = [pm.PressureSystem.from_problem(p, flags=pm.PM_FP64 | pm.PM_FP32_INNER) for p in probs]
    rhs = [s.apply(torch.tensor(p.extra["xstar"], device="cuda")) for s, p in zip(systems, probs)]
    t0 = time.perf_counter()
    tps, npl, tuned_ms = pm.tune_batch(systems, iters=32)
    tune_s = time.perf_counter() - t0
    nfree = np.array([int((p.mesh.dirichlet == 0).sum()) for p in probs])

    def timed(batch):
        for _ in range(args.warmup):
            batch.solve(rhs, rtol=args.rtol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dofit = 0.0
        for _ in range(args.steps):
            code, res = batch.solve(rhs, rtol=args.rtol)
            if code != 0:
                raise RuntimeError("batch status %d" % code)
            dofit += float((nfree * np.array([r.iters for r in res])).sum())
        torch.cuda.synchronize()
        return time.perf_counter() - t0, dofit, res

    batch = pm.PressureBatch(systems, tiles_per_slot=tps, nodes_per_lane=npl)
    el, dofit, res = timed(batch)
    its = np.array([r.iters for r in res])
    ref = [r.p.clone() for r in res]
    # the same solves as one persistent cooperative launch per 16-iteration
    # step (grid barriers between the phases): timed after, checked bit for bit
    batch.set_persistent(True)
    el_p, _, res_p = timed(batch)
    same = all(bool(torch.equal(r.p, q)) and r.iters == int(k) for r, q, k in zip(res_p, ref, its))
    persistent = {"persistent_batch_ms": round(el_p / args.steps * 1e3, 3),
                  "persistent_speedup_vs_graph": round(el / el_p, 3), "persistent_bitwise_equal": same}
    batch.close()
    mixed = {}
    if not args.no_mixed:
        mb = pm.PressureBatch(systems, tiles_per_slot=tps, nodes_per_lane=npl, mixed=True, inner_rtol=args.inner_rtol)
        el_m, dofit_m, res_m = timed(mb)
        diff = max(float(torch.linalg.norm(r.p - q) / torch.linalg.norm(q)) for r, q in zip(res_m, ref))
        mixed = {"mixed_batch_ms": round(el_m / args.steps * 1e3, 3),
                 "mixed_speedup_vs_fp64_batch": round(el / el_m, 3),
                 "mixed_inner_iterations_mean": float(np.mean([r.iters for r in res_m])),
                 "mixed_max_true_relres": max(r.true_relres for r in res_m),
                 "mixed_max_rel_diff_vs_fp64": diff, "mixed_inner_rtol": args.inner_rtol}
        mb.close()
    _common(args, round(dofit / el / 1e9, 4), "GDOF*iter/s", round(el / args.steps * 1e3, 3),
            {"workload": "batch256: 256 meshes (129 2D, 127 3D), nodes log-uniform [2e3,2e5] (10.9M total), "
                         "w log-uniform [1e-6,1], jitter 0.2h, rho~U[0.5,2], FP64 CG to rtol %g; one step = one "
                         "batched solve of all meshes" % args.rtol,
             "n_nodes_total": int(sum(p.mesh.n_nodes for p in probs))},
            dict({"solves_per_s": round(256 * args.steps / el, 2), "iterations_max": int(its.max()),
                  "iterations_mean": float(its.mean()), "graph_iterations_per_replay": 16,
                  "tuned_tiles_per_slot": tps, "tuned_nodes_per_lane": npl,
                  "tuned_ms_per_iteration": round(tuned_ms, 4), "tuning_s": round(tune_s, 2)}, **persistent,
                 **mixed))
    for s in systems:
        s.close()


def bench_serve(args):
    """Serving: Poisson arrivals over the 256-mesh pool (uniform mesh choice),
    each request warm-started from its mesh's previous solution with the rhs
    perturbed by 1 % (normal noise scaled to ||rhs|| / sqrt(N_free)).  The
    main rate is 0.8 x the saturated rate measured in a closed-loop pass;
    0.8 x, 0.5 x and 0.95 x on 2000 requests are extra points (the 0.8 x one
    shows whether the tail grows with the run length).  The same requests
    served one at a time by single FP64 solves give the sequential rate."""
    import torch
    import paper_2301_08357_amd as pm
    from paper_2301_08357_amd.serve import PressureServer, Request
    from synth import fields, workloads
    probs = _batch_problems(256)
    flags = pm.PM_FP64 | (pm.PM_FP32_INNER if args.serve_mixed else 0)
    base, pool = [], []
    for p in probs:
        s = pm.PressureSystem.from_problem(p, flags=flags)
        base.append(s.apply(torch.tensor(p.extra["xstar"], device="cuda")).clone())
        pool.append(s)
    free = [torch.tensor((p.mesh.dirichlet == 0).astype(np.float64), device="cuda") for p in probs]
    scale = [0.01 * float(torch.linalg.norm(b)) / float(f.sum()) ** 0.5 for b, f in zip(base, free)]

    def rhs_fn(req):
        xi = fields.perturbation_torch(workloads.MASTER_SEED, req.rid, probs[req.mesh].mesh.n_nodes, "cuda")
        return base[req.mesh] + scale[req.mesh] * free[req.mesh] * xi

    # sequential baseline: single solves (each handle with its own launch
    # grids), one request at a time, warm starts
    n_seq = min(500, args.requests)
    _, choice = workloads.arrivals(n_seq, 1.0, 256)

    def single(m, b, x0):
        if args.serve_mixed:
            return pool[m].solve_mixed(b, x0=x0, rtol=args.rtol, inner_rtol=args.inner_rtol)
        return pool[m].solve(b, x0=x0, rtol=args.rtol)

    single(0, rhs_fn(Request(rid=4 * 10 ** 6, mesh=0, arrival=0.0)), None)
    last = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, m in enumerate(choice):
        m = int(m)
        r = single(m, rhs_fn(Request(rid=2 * 10 ** 6 + i, mesh=m, arrival=0.0)), last.get(m))
        last[m] = r.p
    torch.cuda.synchronize()
    seq_rate = n_seq / (time.perf_counter() - t0)
    print("serve: sequential single solves %.1f/s" % seq_rate, file=sys.stderr, flush=True)
    del last
    tps, npl, _ = pm.tune_batch(pool, iters=32)
    for s in pool:
        s.close()

    budget = int(args.budget_gb * 2 ** 30) if args.budget_gb > 0 else int(0.8 * torch.cuda.mem_get_info()[0])

    def server():
        return PressureServer(probs, budget, max_in_flight=256, rtol=args.rtol, tiles_per_slot=tps,
                              nodes_per_lane=npl, mixed=args.serve_mixed, inner_rtol=args.inner_rtol)

    # closed loop: saturation rate
    n_cal = min(2000, args.requests)
    _, choice = workloads.arrivals(n_cal, 1.0, 256)
    srv = server()
    srv.run([Request(rid=10 ** 6 + i, mesh=int(m), arrival=0.0) for i, m in enumerate(choice)], rhs_fn)
    sat = srv.stats.solves_per_s
    srv.close()
    print("serve: closed-loop saturation %.1f/s" % sat, file=sys.stderr, flush=True)

    def point(factor, n_req, rid0):
        times, choice = workloads.arrivals(n_req, factor * sat, 256)
        srv = server()
        done = srv.run([Request(rid=rid0 + i, mesh=int(m), arrival=float(t))
                        for i, (t, m) in enumerate(zip(times, choice))], rhs_fn)
        st = srv.stats
        bad = sum(1 for r in done if r.status != 0 or r.true_relres > args.rtol)
        srv.close()
        print("serve: %d requests at %.2f x saturation: %.1f/s, p50 %.1f ms, p99 %.1f ms"
              % (n_req, factor, st.solves_per_s, st.latency_ms["p50"], st.latency_ms["p99"]), file=sys.stderr,
              flush=True)
        return st, bad

    def lat(d):
        return {k: round(v, 3) for k, v in d.items()}

    st, bad = point(0.8, args.requests, 0)
    extra_points = []
    for f in (0.8, 0.5, 0.95):
        e, eb = point(f, min(2000, args.requests), 3 * 10 ** 6 + int(f * 100) * 10 ** 4)
        extra_points.append({"rate_factor": f, "rate_per_s": round(f * sat, 2), "requests": e.n,
                             "solves_per_s": round(e.solves_per_s, 3), "latency_ms_p50": round(e.latency_ms["p50"], 3),
                             "latency_ms_p99": round(e.latency_ms["p99"], 3), "latency_ms_warm": lat(e.latency_ms_warm),
                             "service_ms_mean": round(e.service_ms_mean, 3), "failed": eb})
    kind = "mixed-precision (FP32 inner, FP64 corrections)" if args.serve_mixed else "FP64"
    _common(args, round(st.solves_per_s, 3), "solves/s", round(st.makespan_s * 1e3, 3),
            {"workload": "serve: %d requests, Poisson arrivals at 0.8 x saturation over the 256-mesh pool, warm "
                         "starts, 1%% rhs perturbation, %s solves to rtol %g" % (args.requests, kind, args.rtol),
             "rate_per_s": round(0.8 * sat, 2), "saturation_solves_per_s": round(sat, 2), "budget_bytes": budget,
             "tiles_per_slot": tps, "nodes_per_lane": npl},
            {"latency_ms_p50": round(st.latency_ms["p50"], 3), "latency_ms_p99": round(st.latency_ms["p99"], 3),
             "latency_ms_warm": lat(st.latency_ms_warm), "latency_ms_cold": lat(st.latency_ms_cold),
             "service_ms_mean": round(st.service_ms_mean, 3),
             "mean_iterations_cold": round(st.mean_iters_cold, 1), "mean_iterations_warm": round(st.mean_iters_warm, 1),
             "loads": st.loads, "evictions": st.evictions, "batch_rebuilds": st.rebuilds,
             "max_in_flight": st.max_in_flight_seen, "failed": bad,
             "host_time_s": {"steps": round(st.t_step, 2), "finish": round(st.t_finish, 2),
                             "admit": round(st.t_admit, 2), "rebuild": round(st.t_rebuild, 2)},
             "sequential_solves_per_s": round(seq_rate, 3),
             "speedup_vs_sequential_single_solves": round(st.solves_per_s / seq_rate, 3),
             "extra_points": extra_points})


def mixed_comparison(systems, rhs, xstar, args, fp64_solve_s):
    """The same solves by FP32-inner defect correction (FP64 outer residual,
    dot accumulation and update), timed after the FP64 region."""
    import torch
    ref = [s.solve(b, rtol=args.rtol).p.clone() for s, b in zip(systems, rhs)]
    for s, b in zip(systems, rhs):
        s.solve_mixed(b, rtol=args.rtol, inner_rtol=args.inner_rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inner, outer, worst_res, worst_diff = [], [], 0.0, 0.0
    for _ in range(args.steps):
        for s, b, pr in zip(systems, rhs, ref):
            r = s.solve_mixed(b, rtol=args.rtol, inner_rtol=args.inner_rtol)
            if r.status != 0:
                raise RuntimeError("mixed solve status %d" % r.status)
            inner.append(r.iters)
            outer.append(r.outer)
            worst_res = max(worst_res, r.true_relres)
            worst_diff = max(worst_diff, float(torch.linalg.norm(r.p - pr) / torch.linalg.norm(pr)))
    torch.cuda.synchronize()
    per_solve = (time.perf_counter() - t0) / len(inner)
    return {"solve_ms": round(per_solve * 1e3, 3), "speedup_vs_fp64": round(fp64_solve_s / per_solve, 3),
            "inner_iterations": inner[: len(systems)], "outer_corrections": outer[: len(systems)],
            "inner_rtol": args.inner_rtol, "max_true_relres": worst_res,
            "max_rel_diff_vs_fp64_solution": worst_diff}


def cpu_baseline_cube64(probs, min_seconds=10.0):
    """The CPU oracle (assembled CSR + textbook CG, one thread) on the same
    three systems, one solve each, the round of three repeated until at
    least min_seconds of solve time; assembly is not timed.  Returns the
    baseline record, the oracle's solutions and its right-hand sides
    (caller's node order)."""
    import oracle
    total_dofiter, total_t = 0.0, 0.0
    xs, bs = [], []
    systems = []
    for p in probs:
        A = oracle.assemble_problem(p)
        systems.append((p, A, A.matvec(p.extra["xstar"])))
    rounds = 0
    while rounds == 0 or total_t < min_seconds:
        for p, A, b in systems:
            t0 = time.perf_counter()
            x, st, it, _, _ = oracle.cg(A, b, rtol=1e-10, max_iter=20000, dirichlet=p.mesh.dirichlet)
            total_t += time.perf_counter() - t0
            if rounds == 0:
                xs.append(x)
                bs.append(b)
            total_dofiter += float((p.mesh.dirichlet == 0).sum()) * it
        rounds += 1
    cpu = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(total_dofiter / total_t / 1e9, 5), "unit": "GDOF*iter/s", "cores": 1,
            "kind": "oracle",
            "sample": "one FP64 CG solve per w in {1e-6,1e-3,1} on the same 64^3 mesh, %d rounds "
                      "(%.1f s of CPU time, assembly excluded; one thread of %d available, %s)"
                      % (rounds, total_t, len(os.sched_getaffinity(0)), cpu)}, xs, bs


if __name__ == "__main__":
    main()
