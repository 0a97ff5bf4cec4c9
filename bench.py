#!/usr/bin/env python3
"""Throughput of the normal-mode eigensolve on one MI355X.

Workload: the rotating three-layer planet (solid inner core r < 0.19, fluid
outer core to 0.55, solid mantle to 1; smooth layered profiles times a 2 %
Gaussian random field in the solids; 384,000 tetrahedra; P2 displacement and
P1 pressure, 1.63M displacement DOFs), Cowling approximation, rotation
Omega = 0.05 along z: all eigenpairs with omega^2 in [1, 60] (nev cap 200,
residual tolerance 1e-8) by the polynomial-filtered Lanczos solve, then the
Coriolis term by projection on those pairs.

One timed "step" is one application of B = M^{-1} A inside the polynomial
filter on the solve's full 32-column block: the Cowling operator (A_G with
the E_G K_p^{-1} E_G^T Schur part), the Chebyshev-Jacobi mass solve and the
fused three-term filter update.  --warmup untimed and --steps timed steps
run as one filter application each (degree = that count), bracketed by
device synchronisations; ms_per_step is the timed one divided by --steps.

The eigenpair rate comes from full solves run in the same command ("legs"):
  fp64   the all-FP64 filter (mass solve one FP64 Chebyshev-Jacobi pass);
  mixed  FP64 filter with every mass solve as two FP32 passes joined by an
         FP64 residual correction;
  fp32   FP32 filter (values, vectors, accumulation) with FP64 Lanczos,
         Rayleigh-Ritz, residuals and a final FP64 refinement.
The first leg named by --legs is the headline (`value`); the others run while
the wall-clock budget allows (a leg that would not fit is reported null with
the reason).  Every returned pair's residual is computed in FP64 against the
FP64 pencil; value = pairs with residual <= tol / (solve + projection) seconds,
with the pencil resident in HBM (assembly timed separately).

Also printed: the roofline of the dominant kernel (a middle Chebyshev-Jacobi
step of the mass solve; mean duration from HIP events the library records on
the solve's stream) and the CPU oracle's rate on a bounded sample.
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
T0 = time.perf_counter()

LEGS = {
    "fp64": dict(precision=0, mass_passes=0, dtype="f64"),
    "mixed": dict(precision=0, mass_passes=2, dtype="f64+f32"),
    "fp32": dict(precision=1, mass_passes=0, dtype="f32+f64"),
}


def kernel_fingerprint():
    """sha256 of the source text of the row-group mass-solve kernel (its
    gather helper and body), so that HBM traffic measured by rocprofv3 on an
    earlier build is reported only while the kernel is unchanged."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_1906_11082_amd", "csrc", "nm_ops.hip")).read()
    i = src.index("// sum over the group's union columns")
    j = src.index("// LDS-tiled Chebyshev-Jacobi step")
    return hashlib.sha256(src[i:j].encode()).hexdigest()


def measured_traffic(kernel, leg, block, n_half):
    """HBM bytes per launch of the hot kernel from the committed rocprofv3
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy's
    readings), or None if there is none for this kernel, leg and size or the
    kernel's source has changed since."""
    path = os.path.join(ROOT, "profiles", "k_cj_group_c2_%s_b%d_traffic.json" % (leg, block))
    try:
        t = json.load(open(path))
    except (OSError, ValueError):
        return None
    if (t.get("kernel") != kernel or t.get("n_half") != n_half or t.get("block") != block
            or t.get("kernel_source_sha256") != kernel_fingerprint()):
        return None
    return t["hbm_bytes_per_launch"]


def hot_kernel_name(st, leg):
    """The template instance of the mass-solve step the leg ran, as the profiler
    names it (rows of 3 x 32 columns: 4 floats or 2 doubles per lane, 4-row
    groups, 4 gathers in flight, the default LDS stage)."""
    if st.get("hot_kernel") != "row-group":
        return None
    return "k_cj_group<float, 4, 4, 4, 0>" if leg in ("mixed", "fp32") else "k_cj_group<double, 2, 4, 4, 0>"


def log(msg):
    print("[bench %6.1fs] %s" % (time.perf_counter() - T0, msg), file=sys.stderr, flush=True)


_ORACLE = {}


def _oracle_worker(args):
    """Column B-applications of the oracle on `ncols` columns for about `seconds`
    (one single-threaded pool process; the oracle pencil is built on first use)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    nh, tol, ncols, seconds, seed = args
    with threadpool_limits(limits=1):
        if nh not in _ORACLE:
            import planetgen as pg
            from oracle.assemble import Pencil
            from oracle import solve as S
            t = time.perf_counter()
            P = Pencil(pg.three_layer_planet(n_half=nh))
            ptr, _ = P.nb.node_graph()
            _ORACLE[nh] = (S.CowlingOperator(P, minv_tol=0.3 * tol, kp_tol=1e-13), int(ptr[-1]),
                           time.perf_counter() - t)
        op, nnzb, t_asm = _ORACLE[nh]
        X = np.random.default_rng(seed).standard_normal((op.n, ncols))
        op.B(X)
        reps, t0 = 0, time.perf_counter()
        while True:
            op.B(X)
            reps += 1
            if time.perf_counter() - t0 > seconds:
                break
        dt = time.perf_counter() - t0
    return dict(cols=reps * ncols, seconds=dt, pid=os.getpid(), n=op.n, nnzb=nnzb, kM=op.kM, kP=op.kP,
                asm=t_asm)


class CpuBaseline:
    """The oracle (scipy CSR products and its own Chebyshev-Jacobi mass solve,
    the same Cowling operator and mass-solve bound as the GPU leg) timed on
    column B-applications of the same planet generator at n_half = cpu_n_half,
    once on one core and then on `cores` cores (one single-threaded process
    per core, 4 columns each), in processes forked before the GPU is touched
    and running while the GPU solves.  Scaled to the workload by node-graph
    size and multiplied by the GPU leg's column B-application count: an
    extrapolated oracle solve time (its Lanczos and Rayleigh-Ritz are not
    counted, which favours the oracle)."""

    def __init__(self, pool, cores, args):
        import threading
        self.pool, self.cores, self.args = pool, cores, args
        self.out = {}
        self.th = threading.Thread(target=self._run, daemon=True)

    def start(self):
        self.th.start()

    def _run(self):
        a = self.args
        self.out["one"] = self.pool.apply(_oracle_worker, ((a.cpu_n_half, a.tol, 4, a.cpu_seconds, 0),))
        self.out["all"] = self.pool.map(_oracle_worker, [(a.cpu_n_half, a.tol, 4, a.cpu_seconds, 1 + i)
                                                         for i in range(self.cores)], chunksize=1)

    def result(self, gpu_stats, pairs, gpu_nnzb):
        self.th.join()
        self.pool.close()
        args, one, outs = self.args, self.out["one"], self.out["all"]
        used = len({o["pid"] for o in outs})  # processes that ran concurrently
        rate_all = sum(o["cols"] / o["seconds"] for o in outs) * used / len(outs)
        per_col_1 = one["seconds"] / one["cols"]
        per_col_all = 1.0 / rate_all
        scale = gpu_nnzb / float(one["nnzb"])
        bapps = gpu_stats["bapps"] + gpu_stats["refine_bapps"]
        t_1 = per_col_1 * scale * bapps
        t_all = per_col_all * scale * bapps
        return {
            "value": pairs / t_all if t_all > 0 else None,
            "unit": "eigenpairs/s",
            "cores": used,
            "kind": "oracle",
            "sample": ("column B-applications (A_G + E_G K_p^-1 E_G^T with a %d-step K_p solve, then the %d-step "
                       "Chebyshev-Jacobi M solve) of the oracle on the same planet generator at n_half=%d (%d DOF, "
                       "nnzb %d), ~%.0f s on 1 core and ~%.0f s on %d cores (one single-threaded process each, 4 "
                       "columns; run while the GPU solved); per-column time scaled by node-graph size x%.2f to "
                       "this workload and multiplied by the headline solve's %d column B-applications "
                       "(extrapolated; Lanczos and Rayleigh-Ritz not counted)"
                       % (one["kP"], one["kM"], args.cpu_n_half, one["n"], one["nnzb"], one["seconds"],
                          max(o["seconds"] for o in outs), used, scale, bapps)),
            "value_1core": pairs / t_1 if t_1 > 0 else None,
            "seconds_per_column_bapp_full_size_1core": per_col_1 * scale,
            "seconds_per_column_bapp_full_size_all_cores": per_col_all * scale,
            "extrapolated_solve_seconds_1core": t_1,
            "extrapolated_solve_seconds_all_cores": t_all,
            "oracle_assembly_seconds": one["asm"],
        }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed B-applications (one filter application)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed B-applications before them")
    ap.add_argument("--legs", default="mixed,fp64,fp32",
                    help="comma-separated solve legs (fp64, mixed, fp32); the first is the headline")
    ap.add_argument("--budget-s", type=float, default=470.0,
                    help="wall-clock budget from process start: later legs that would not fit are skipped")
    ap.add_argument("--n-half", type=int, default=20)
    ap.add_argument("--omega", type=float, default=0.05, help="rotation rate about z (0: no projection)")
    ap.add_argument("--a", type=float, default=1.0)
    ap.add_argument("--b", type=float, default=60.0)
    ap.add_argument("--nev", type=int, default=200)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--guard", type=float, default=1.0)
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--max-basis", type=int, default=1400)
    ap.add_argument("--cpu-n-half", type=int, default=8)
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--cpu-cores", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true", help="no per-block solver lines on stderr")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this program runs on one GPU; --gpus %d is not supported (the multi-GPU sharding is "
              "described in the design notes, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    for x in legs:
        if x not in LEGS:
            ap.error("unknown leg %r" % x)
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's processes are forked before anything touches the GPU; one core stays free
        # for the process that drives the GPU
        import multiprocessing as mp
        cores = max(1, min(args.cpu_cores, (os.cpu_count() or 2) - 1))
        cpu = CpuBaseline(mp.get_context("fork").Pool(cores), cores, args)

    import numpy as np
    import torch
    import planetgen as pg
    import paper_1906_11082_amd as nm

    nm.load_library()
    torch.cuda.set_device(0)
    planet = pg.three_layer_planet(n_half=args.n_half, omega=(0.0, 0.0, args.omega))
    log("planet: %d tets" % len(planet["tet"]))
    torch.cuda.synchronize()
    t = time.perf_counter()
    P = nm.Pencil(planet)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t
    log("assembly %.2f s: n %d, n_p %d, nnzb %d" % (t_asm, P.n, P.n_p, P.info["nnzb"]))

    # ---- timed steps: B-applications of the headline leg's filter on the full block
    head = LEGS[legs[0]]
    lo, hi = P.spectrum_bounds(60, 0x5BD1E995)
    lmin, lmax = lo - 1e-3 * (args.b - args.a), hi
    c, e = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    X = torch.randn(P.n, args.block, dtype=torch.float32 if head["precision"] else torch.float64, device="cuda")
    kw = dict(minv_tol=0.3 * args.tol if not head["precision"] else 1e-7,
              kp_tol=1e-13 if not head["precision"] else 1e-7,
              precision=head["precision"], mass_passes=head["mass_passes"])
    if args.warmup > 0:
        P.filter_apply(nm.filter_coeffs(args.a, args.b, lmin, lmax, args.warmup), c, e, X, **kw)
    mu = nm.filter_coeffs(args.a, args.b, lmin, lmax, max(args.steps, 1))
    torch.cuda.synchronize()
    t = time.perf_counter()
    P.filter_apply(mu, c, e, X, **kw)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t
    ms_per_step = t_steps / max(args.steps, 1) * 1e3
    log("%d B-applications (block %d, %s): %.2f ms each" % (args.steps, args.block, legs[0], ms_per_step))
    if cpu:
        cpu.start()

    # ---- full solves
    results = {}
    first_seconds = None
    for i, name in enumerate(legs):
        L = LEGS[name]
        elapsed = time.perf_counter() - T0
        if i > 0:
            # a later leg is estimated from the headline solve's length (the FP32 filter with its
            # refinement and the all-FP64 solve have measured up to ~1.6x the mixed one)
            est = 1.7 * first_seconds
            if elapsed + est > args.budget_s:
                results[name] = dict(value=None, reason="not run: the estimated %.0f s would exceed the %.0f s "
                                     "budget (%.0f s elapsed)" % (est, args.budget_s, elapsed))
                log("leg %s skipped (estimate %.0f s)" % (name, est))
                continue
        log("leg %s: solve" % name)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = P.filtered_eig(args.a, args.b, args.nev, args.tol, block=args.block, guard=args.guard,
                           precision=L["precision"], max_basis=args.max_basis, lmin=lmin, lmax=lmax,
                           verbose=0 if args.quiet else 1, allow_partial=True, mass_passes=L["mass_passes"])
        rot = None
        if args.omega != 0.0 and r.count:
            rr = P.project_rotation(r, args.a, args.b)
            rot = dict(count=rr.count, omega_min=float(rr.omega.min()) if rr.count else None,
                       omega_max=float(rr.omega.max()) if rr.count else None, seconds=rr.seconds)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t
        if first_seconds is None:
            first_seconds = secs
        st = r.stats
        pairs = int((r.resid <= args.tol).sum())
        results[name] = dict(
            value=pairs / secs, unit="eigenpairs/s", dtype=L["dtype"], seconds=secs, pairs=pairs, count=r.count,
            resid_max=float(r.resid.max()) if r.count else None, partial=bool(r.partial),
            filter_degree=st["degree"], kM=st["kM"], mass_passes=st["mass_passes"],
            mass_pass_steps=st["mass_pass_steps"], block=st["block"], basis=st["basis"],
            column_bapps=st["bapps"], filter_seconds=st["filter_seconds"], refine_passes=st["refine_passes"],
            refine_degree=st["refine_degree"], refine_seconds=st["refine_seconds"],
            refine_column_bapps=st["refine_bapps"], rotating_modes=rot,
            hot_kernel_ms=st["hot_ms"], hot_kernel_bytes=st["hot_bytes"], hot_samples=st["hot_samples"],
            _lam=r.lam, _stats=st)
        log("leg %s: %d pairs <= tol in %.1f s (%.3f eigenpairs/s), resid max %.2e"
            % (name, pairs, secs, pairs / secs, results[name]["resid_max"] or 0.0))
        if i == 0 and cpu:
            cpu = cpu.result(st, pairs, P.info["nnzb"])
            log("cpu baseline: %.3g eigenpairs/s on %d cores" % (cpu["value"], cpu["cores"]))
    # accuracy of each leg against the FP64 leg (eigenvalues of matched pairs)
    ref = results.get("fp64", {}).get("_lam")
    for name, R in results.items():
        lam = R.pop("_lam", None)
        if name != legs[0]:
            R.pop("_stats", None)
        if ref is not None and lam is not None and name != "fp64":
            k = min(len(ref), len(lam))
            R["max_rel_eig_diff_vs_fp64"] = float(np.max(np.abs(lam[:k] - ref[:k]) / np.abs(ref[:k]))) if k else None
    H = results[legs[0]]
    st = H.pop("_stats")
    hot_gbs = st["hot_bytes"] / (st["hot_ms"] * 1e-3) / 1e9 if st["hot_ms"] > 0 else None
    out = {
        "metric": METRIC,
        "value": H["value"],
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": H["dtype"],
        "data": "synthetic",
        "config": {
            "workload": "rotating three-layer planet, %d tets, P2/P1, Cowling, Omega=%g z, omega^2 in [%g, %g], "
                        "nev<=%d, tol %g" % (len(planet["tet"]), args.omega, args.a, args.b, args.nev, args.tol),
            "step": "one B = M^-1 A application inside the filter on the %d-column block (%s leg)"
                    % (args.block, legs[0]),
            "headline_leg": legs[0],
            "n_disp": P.n, "n_pres": P.n_p, "nnzb": P.info["nnzb"], "assembly_seconds": t_asm,
            "lmin": lmin, "lmax": lmax,
        },
        "legs": results,
        "roofline": {
            "bound": "hbm",
            "achieved": hot_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hot_gbs / HBM_PEAK_GBS if hot_gbs else None,
            "traffic": measured_traffic(hot_kernel_name(st, legs[0]), legs[0], args.block, args.n_half),
            "kernel": "middle Chebyshev-Jacobi step of the mass solve (%s leg)" % legs[0],
            "bytes_per_launch": st["hot_bytes"],
            "mean_launch_ms": st["hot_ms"],
            "sampled_launches": st["hot_samples"],
            "launches": st["hot_launches"],
        },
    }
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
