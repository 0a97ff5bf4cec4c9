"""Serving workload: a seeded Poisson stream of eigensolve requests through
the library's request server (continuous batching under an HBM budget).
The solver's per-block log lines (stderr) show each request's progress.

Per request (seeded): a layered planet with T tets drawn log-uniform in
[tmin, tmax] (three-layer generator, n_half = (T / 48)^(1/3)), P1 or P2
displacement, Omega in {0, 0.05, 0.5} along z, 1..max_slices windows of
omega^2 contiguous from 1 upward (width `width` each), nev 20..100 per
window.  Arrivals: exponential gaps with mean 1 / rate.  Reports p50 / p99 of
(completion - arrival), completion taken from the server's own clock, and
eigenpairs with residual <= tol per second over the whole stream.

    python -m paper_1906_11082_amd.serving --requests 16 --tmin 2e4 --tmax 1e5
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def make_stream(args):
    import numpy as np
    rng = np.random.default_rng(args.seed)
    reqs, t = [], 0.0
    for i in range(args.requests):
        t += rng.exponential(1.0 / args.rate)
        T = math.exp(rng.uniform(math.log(args.tmin), math.log(args.tmax)))
        n_half = max(3, int(round((T / 48.0) ** (1.0 / 3.0))))
        order = int(rng.integers(1, 3))
        om = float(rng.choice([0.0, 0.05, 0.5]))
        ns = int(rng.integers(1, args.max_slices + 1))
        nev = [int(rng.integers(20, 101)) for _ in range(ns)]
        wins = [(1.0 + args.width * k, 1.0 + args.width * (k + 1)) for k in range(ns)]
        reqs.append(dict(arrival=t, n_half=n_half, order=order, omega=om, windows=wins, nev=nev,
                         seed=args.seed * 1000 + i))
    return reqs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=2.0)
    ap.add_argument("--tmin", type=float, default=2e4)
    ap.add_argument("--tmax", type=float, default=8e5)
    ap.add_argument("--max-slices", type=int, default=8)
    ap.add_argument("--width", type=float, default=5.0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-active", type=int, default=4)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--mass-passes", type=int, default=0,
                    help="FP64 filters: mass solves as this many FP32 passes with FP64 residual corrections")
    ap.add_argument("--seed", type=int, default=4)
    args = ap.parse_args()
    import numpy as np
    import planetgen as pg
    import paper_1906_11082_amd as nm

    stream = make_stream(args)
    prec = 1 if args.precision == "fp32" else 0
    server = nm.Server(hbm_budget_gb=args.budget_gb, max_active=args.max_active)
    t0 = time.perf_counter()
    tickets = []
    for r in stream:
        planet = pg.three_layer_planet(seed=r["seed"], n_half=r["n_half"], order=r["order"], pres_order=1,
                                       omega=(0.0, 0.0, r["omega"]))
        delay = r["arrival"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        sub = time.perf_counter() - t0
        tickets.append((r, sub, server.submit(planet, r["windows"], r["nev"], args.tol, rotate=r["omega"] > 0,
                                              precision=prec, block=16, verbose=1,
                                              mass_passes=0 if prec else args.mass_passes)))
        print("[serve] submitted request %d (T=%d, P%d, %d windows) at %.2fs"
              % (len(tickets) - 1, len(planet["tet"]), r["order"], len(r["windows"]), sub), file=sys.stderr,
              flush=True)
    lat, pairs, fails = [], 0, 0
    for k, (r, sub, t) in enumerate(tickets):
        res = server.wait(t)
        # the server's own clock: completion minus submission of this request (waits return in
        # ticket order, so the time a wait returns would charge an early finisher for the
        # requests before it), plus any lag of the submission behind the arrival
        lat.append(res["t_end"] - res["t_submit"] + max(0.0, sub - r["arrival"]))
        if res["status"] < 0:
            fails += 1
        pairs += sum(int((s.resid <= args.tol).sum()) for s in res["slices"])
        print("[serve] request %d done: status %d, %d pairs, latency %.2fs"
              % (k, res["status"], sum(s.count for s in res["slices"]), lat[-1]), file=sys.stderr, flush=True)
    total = time.perf_counter() - t0
    server.close()
    lat = np.array(lat)
    print(json.dumps(dict(requests=len(stream), failed=fails, p50_s=float(np.percentile(lat, 50)),
                          p99_s=float(np.percentile(lat, 99)), eigenpairs=pairs, seconds=total,
                          eigenpairs_per_s=pairs / total, precision=args.precision,
                          budget_gb=args.budget_gb, max_active=args.max_active,
                          tets=[args.tmin, args.tmax], rate=args.rate)), flush=True)


if __name__ == "__main__":
    main()
