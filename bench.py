#!/usr/bin/env python3
"""Throughput of the normal-mode eigensolve on one MI355X.

Workload (one "step"): the three-layer planet (solid inner core r < 0.19,
fluid outer core to 0.55, solid mantle to 1; smooth layered profiles times a
2 % Gaussian random field in the solids; 384,000 tetrahedra; P2 displacement
and P1 pressure, 1.63M displacement DOFs), Cowling approximation: assembly of
the pencil on the device and the polynomial-filtered Lanczos solve for all
eigenpairs with omega^2 in [1, 60] (nev cap 200), residual tolerance 1e-8.

By default the filter runs in FP64 with each mass solve as two FP32
Chebyshev-Jacobi passes joined by an FP64 residual correction (--mass-passes 2,
dtype "f64+f32"); --mass-passes 0 is the all-FP64 solve, --precision fp32 the
FP32 filter.  Every returned pair's residual is computed in FP64.

Prints one JSON line: eigenpairs/s with residual <= tol over the timed steps,
the roofline of the dominant kernel (the fused Chebyshev-Jacobi mass-solve
step inside the filter; mean duration from HIP events recorded by the
library on the solve's stream) and the CPU oracle's rate on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "eigenpairs/s at resid≤1e-8, FP32-filter vs FP64; SpMM HBM GB/s; p99 latency"


def cpu_baseline(gpu_result, gpu_nnzb, args):
    """The oracle (scipy CSR products, Chebyshev-Jacobi mass solve) timed on
    column B-applications of the same planet family at n_half = 8, scaled by
    the node-graph size to the full workload and multiplied by the GPU run's
    B-application count (extrapolated; the oracle's Lanczos and
    Rayleigh-Ritz work is not counted, which favours the oracle)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import planetgen as pg
    from oracle.assemble import Pencil
    from oracle import solve as S
    nh = args.cpu_n_half
    planet = pg.three_layer_planet(n_half=nh)
    with threadpool_limits(limits=1):
        P = Pencil(planet)
        op = S.CowlingOperator(P, minv_tol=args.minv_tol if args.minv_tol > 0 else 0.3 * args.tol, kp_tol=1e-13)
        rng = np.random.default_rng(0)
        X = rng.standard_normal((P.n, 4))
        op.B(X)
        reps = 0
        t0 = time.perf_counter()
        while True:
            op.B(X)
            reps += 1
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
    per_col = dt / (reps * X.shape[1])
    ptr, _ = P.nb.node_graph()
    scale = gpu_nnzb / float(ptr[-1])
    t_solve = per_col * scale * gpu_result.stats["bapps"]
    pairs = int((gpu_result.resid <= args.tol).sum())
    return {
        "value": pairs / t_solve if t_solve > 0 else None,
        "unit": "eigenpairs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("%d x 4-column B-applications (A + Schur + %d-step Chebyshev-Jacobi M^-1) of the oracle on the "
                   "same planet generator at n_half=%d (%d DOF, %.1f s), scaled by node-graph size x%.1f to this "
                   "workload and by its %d column B-applications; single-threaded scipy CSR"
                   % (reps, op.kM, nh, P.n, dt, scale, gpu_result.stats["bapps"])),
        "seconds_per_column_bapp_full_size": per_col * scale,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--n-half", type=int, default=20)
    ap.add_argument("--a", type=float, default=1.0)
    ap.add_argument("--b", type=float, default=60.0)
    ap.add_argument("--nev", type=int, default=200)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--guard", type=float, default=1.0)
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--minv-tol", type=float, default=0.0, help="mass-solve bound (0: library default, 0.3 tol)")
    ap.add_argument("--max-basis", type=int, default=1400)
    ap.add_argument("--mass-passes", type=int, default=2,
                    help="FP64 filter with the mass solve in this many FP32 passes with FP64 residual corrections "
                         "(0: one FP64 pass; ignored with --precision fp32)")
    ap.add_argument("--cpu-n-half", type=int, default=8)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", default="", help="PMC traffic summary of the hot kernel (default: "
                    "profiles/<kernel>_c2_<precision>_b<block>_traffic.json)")
    ap.add_argument("--quiet", action="store_true", help="no per-block progress lines on stderr")
    ap.add_argument("--omega", type=float, default=0.0,
                    help="rotation rate about z: the step also projects the Coriolis term over the window's pairs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import planetgen as pg
    import paper_1906_11082_amd as nm

    nm.load_library()
    torch.cuda.set_device(0)
    planet = pg.three_layer_planet(n_half=args.n_half, omega=(0.0, 0.0, args.omega))
    prec = 1 if args.precision == "fp32" else 0
    if prec:
        args.mass_passes = 0

    rot = {}

    def step():
        P = nm.Pencil(planet)
        r = P.filtered_eig(args.a, args.b, args.nev, args.tol, block=args.block, guard=args.guard,
                           precision=prec, minv_tol=args.minv_tol, max_basis=args.max_basis,
                           verbose=0 if args.quiet else 1, allow_partial=True, mass_passes=args.mass_passes)
        if args.omega != 0.0:
            t = time.perf_counter()
            rr = P.project_rotation(r, args.a, args.b)
            rot.update(count=rr.count, seconds=time.perf_counter() - t,
                       omega_min=float(rr.omega.min()) if rr.count else None,
                       omega_max=float(rr.omega.max()) if rr.count else None)
        return P, r

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for _ in range(args.steps):
        P, r = step()
        res.append(r)
        print("[bench] step done: %d pairs, %.1f s" % (r.count, r.stats["seconds"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T = t1 - t0
    pairs = sum(int((r.resid <= args.tol).sum()) for r in res)
    last = res[-1]
    st = last.stats
    hot_gbs = st["hot_bytes"] / (st["hot_ms"] * 1e-3) / 1e9 if st["hot_ms"] > 0 else None
    traffic = None
    # the sampled kernel: a middle step of the FP64 mass solve, or of an FP32 pass
    hot_prec = "fp32" if prec else ("mixed" if args.mass_passes else "fp64")
    hot = "k_cj_group" if st["block"] >= 32 else "k_cj_step"
    if not args.traffic_json:
        args.traffic_json = os.path.join(ROOT, "profiles", "%s_c2_%s_b%d_traffic.json" % (hot, hot_prec,
                                                                                           st["block"]))
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            tj = json.load(f)
        if tj.get("precision") == hot_prec and tj.get("block") == args.block and \
                tj.get("n_half") == args.n_half:
            traffic = tj.get("hbm_bytes_per_launch")
    out = {
        "metric": METRIC,
        "value": pairs / T,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec else ("f64+f32" if args.mass_passes else "f64"),
        "data": "synthetic",
        "config": {
            "workload": "three-layer planet, %d tets, P2/P1, Cowling, omega^2 in [%g, %g], nev<=%d, tol %g"
                        % (len(planet["tet"]), args.a, args.b, args.nev, args.tol),
            "n_disp": P.info["n_disp"], "n_pres": P.info["n_pres"], "nnzb": P.info["nnzb"],
            "filter_degree": st["degree"], "kM": st["kM"], "block": st["block"], "basis": st["basis"],
            "mass_passes": st["mass_passes"], "mass_pass_steps": st["mass_pass_steps"],
            "column_bapps": st["bapps"], "pairs": last.count, "resid_max": float(last.resid.max()) if last.count else None,
            "lmax": st["lmax"], "solve_seconds": st["seconds"], "filter_seconds": st["filter_seconds"],
            "partial": bool(last.partial),
            "refine_passes": st["refine_passes"], "refine_degree": st["refine_degree"],
            "refine_seconds": st["refine_seconds"], "refine_column_bapps": st["refine_bapps"],
            "omega_z": args.omega, "rotating_modes": rot or None,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": hot_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hot_gbs / HBM_PEAK_GBS if hot_gbs else None,
            "traffic": traffic,
            "kernel": hot + " (fused Chebyshev-Jacobi step of the mass solve)",
            "bytes_per_launch": st["hot_bytes"],
            "mean_launch_ms": st["hot_ms"],
            "sampled_launches": st["hot_samples"],
            "launches": st["hot_launches"],
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(last, P.info["nnzb"], args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
