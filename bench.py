"""Benchmark of the matrix-free P1 pressure solve on one MI355X.

Workload (one step): the 3D unit cube, 64^3 cells x 6 tetrahedra
(1,572,864 tets, 274,625 nodes, Morton order), c = 1/rho with
rho ~ U[0.5, 2] per element, and one FP64 CG solve to rtol 1e-10 from
x0 = 0 for each mass weight w in {1e-6, 1e-3, 1}.  The right-hand side is
b = A_D x* with x* = prod sin(pi x_i), computed once before timing.

Prints one JSON line: GDOF*iter/s (free nodes x CG iterations per second,
whole job), solves/s, p50/p99 solve latency, the roofline of the operator
apply kernel (algorithmic bytes / measured average kernel duration against
the 8 TB/s HBM peak) and the CPU oracle timed on a bounded sample.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--tile", type=int, default=0, help="Morton tile nodes (128/256/512; 0 = library default)")
    ap.add_argument("--inner-rtol", type=float, default=1e-4, help="inner tolerance of the mixed solve")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2301_08357_amd as pm
    from synth import workloads

    dev = torch.device("cuda:0")
    ws = workloads.CUBE64_W
    probs = [workloads.cube64(w) for w in ws]
    m = probs[0].mesh
    tile_flag = {0: 0, 128: pm.PM_TILE_128, 256: pm.PM_TILE_256, 512: pm.PM_TILE_512}[args.tile]
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
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "operator apply (fused CG iteration)",
            "bytes_per_launch": info["apply_bytes"], "avg_launch_us": round(avg_ms * 1e3, 3),
            "launches": launches,
        },
    }
    if not args.no_mixed:
        out["mixed"] = mixed_comparison(systems, rhs, xstar, args, elapsed / len(lat))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(probs)
    print(json.dumps(out), flush=True)
    for s in systems:
        s.close()


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


def cpu_baseline(probs):
    """The CPU oracle (assembled CSR + textbook CG, one thread) on the same
    three systems, one solve each; assembly is not timed."""
    import oracle
    total_dofiter, total_t = 0.0, 0.0
    for p in probs:
        A = oracle.assemble_problem(p)
        b = A.matvec(p.extra["xstar"])
        t0 = time.perf_counter()
        x, st, it, _, _ = oracle.cg(A, b, rtol=1e-10, max_iter=20000, dirichlet=p.mesh.dirichlet)
        total_t += time.perf_counter() - t0
        total_dofiter += float((p.mesh.dirichlet == 0).sum()) * it
    return {"value": round(total_dofiter / total_t / 1e9, 5), "unit": "GDOF*iter/s", "cores": 1,
            "kind": "oracle",
            "sample": "one FP64 CG solve per w in {1e-6,1e-3,1} on the same 64^3 mesh "
                      "(%.1f s of CPU time, assembly excluded)" % total_t}


if __name__ == "__main__":
    main()
