"""Spectrum slicing and rotation study of a rotating layered planet on one GPU.

    python3 -m paper_1906_11082_amd.slicing_study [--n-half 20] [--slices 4] [--a 1] [--b 60]
        [--omega 0.05] [--omega2 0.0125,0.025,0.1,0.2,0.5] [--nev 260] [--mass-passes 2] [--precision 0] [--guard 1]
        [--skip-slices] [--skip-window] [--skip-rotation] [--save eig.npz]

The three-layer planet (P2/P1, Cowling) rotating about z:

1. spectrum bounds and null-free density-of-states traces (kernel
   polynomial method on B z, so the fluid null space at 0 does not leak into
   the counts; Sec. 6.1's spectrum slicing) give `slices` windows of [a, b]
   with equal estimated eigenvalue counts;
2. the slices are solved in one batched call (or one after another with
   --sequential), each with the two-sided slice filter (damping beyond bands
   of `guard` slice widths on both sides), their filter applications
   concatenated (series zero-padded to the largest degree);
3. the whole window [a, b] is solved once for comparison (unless
   --skip-window): counts, eigenvalues and column B-applications;
4. the Coriolis problem (Sec. 7) is projected on the window's modes at the
   planet's Omega and at the rates of --omega2 (pencils differing only in
   Omega), and compared with first-order splitting (the eigenvalues of
   Lambda^{1/2} + i X^T R X): the difference scales as Omega^2.

Prints progress lines on stderr and one JSON line on stdout.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

T0 = time.time()


def log(msg):
    print("[slices %7.1fs] %s" % (time.time() - T0, msg), file=sys.stderr, flush=True)


def first_order(P, r, nm, np):
    """First-order Coriolis frequencies from the same modes: the eigenvalues
    of Lambda^{1/2} + i X^T R X (Hermitian; for a degenerate multiplet this
    is sqrt(lambda) plus the eigenvalues of i X_g^T R X_g).  They differ from
    the projected quadratic problem's by O(Omega^2)."""
    X = r.X
    RX = P.apply(nm.OP_R, X)
    S = (X.T @ RX).cpu().numpy()
    S = 0.5 * (S - S.T)
    H = np.diag(np.sqrt(r.lam)).astype(complex) + 1j * S
    return np.linalg.eigvalsh(H)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-half", type=int, default=20)
    ap.add_argument("--slices", type=int, default=4)
    ap.add_argument("--a", type=float, default=1.0)
    ap.add_argument("--b", type=float, default=60.0)
    ap.add_argument("--omega", type=float, default=0.05)
    ap.add_argument("--omega2", type=str, default="0.0125,0.025,0.1,0.2,0.5",
                    help="further rotation rates (comma-separated) for the projection on the same modes")
    ap.add_argument("--nev", type=int, default=260)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--mass-passes", type=int, default=2)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--dos-degree", type=int, default=3000)
    ap.add_argument("--skip-window", action="store_true")
    ap.add_argument("--skip-slices", action="store_true")
    ap.add_argument("--skip-rotation", action="store_true")
    ap.add_argument("--guard", type=float, default=1.0, help="slice filter bands, in slice widths")
    ap.add_argument("--sequential", action="store_true",
                    help="solve the slices one after another, each with its own filter degree, instead of one "
                         "batched call (whose series are padded to the largest degree)")
    ap.add_argument("--save", default="", help="write the eigenvalues found to this .npz")
    args = ap.parse_args()
    import numpy as np
    import torch
    import planetgen as pg
    import paper_1906_11082_amd as nm

    torch.cuda.set_device(0)
    d = pg.three_layer_planet(n_half=args.n_half, omega=(0.0, 0.0, args.omega))
    P = nm.Pencil(d)
    log("planet %d tets, n %d, n_p %d" % (len(d["tet"]), P.n, P.n_p))
    kw = dict(block=args.block, mass_passes=args.mass_passes if args.precision == 0 else 0,
              precision=args.precision)
    out = dict(workload="three-layer planet n_half %d (%d tets), P2/P1, Cowling, Omega %g z, window [%g, %g]"
                        % (args.n_half, len(d["tet"]), args.omega, args.a, args.b),
               n_disp=P.n, n_pres=P.n_p, precision=args.precision, mass_passes=kw["mass_passes"], block=args.block)
    t = time.time()
    lo, hi = P.spectrum_bounds(80, 3)
    lmin, lmax = lo - 1e-3 * (args.b - args.a), hi
    out["bounds"] = [lmin, lmax]
    res = {}
    saved = {}
    if not args.skip_slices:
        edges, tau = P.dos_slice_edges(args.a, args.b, args.slices, lmin, lmax, m=args.dos_degree, nvec=32, seed=5,
                                       weighted=True)
        torch.cuda.synchronize()
        out["dos"] = dict(seconds=time.time() - t, degree=args.dos_degree, nvec=32, edges=list(map(float, edges)),
                          estimated_count=nm.dos_count(tau, lmin, lmax, args.a, args.b, weighted=True))
        log("dos edges %s (estimated count %.1f) in %.1f s" % (np.round(edges, 3), out["dos"]["estimated_count"],
                                                                 out["dos"]["seconds"]))
        wins = [(float(edges[i]), float(edges[i + 1])) for i in range(args.slices)]
        t = time.time()
        if args.sequential:
            rs = [P.filtered_eig(a, b, args.nev, args.tol, lmin=lmin, lmax=lmax, null_filter=3, guard=args.guard,
                                 seed=9, verbose=1, **kw) for a, b in wins]
        else:
            rs = P.filtered_eig_slices(wins, args.nev, args.tol, lmin=lmin, lmax=lmax, null_filter=3,
                                       guard=args.guard, seed=9, verbose=1, **kw)
        torch.cuda.synchronize()
        dt = time.time() - t
        lam_s = np.concatenate([r.lam for r in rs])
        bapps = sum(r.stats["bapps"] + r.stats["refine_bapps"] for r in rs)
        out["slices"] = dict(seconds=dt, count=int(len(lam_s)), column_bapps=int(bapps), sequential=args.sequential,
                             guard=args.guard,
                             per_slice=[dict(window=w, count=r.count, degree=r.stats["degree"], basis=r.stats["basis"],
                                             resid_max=float(r.resid.max()) if r.count else None,
                                             bapps=r.stats["bapps"], refine_bapps=r.stats["refine_bapps"])
                                        for w, r in zip(wins, rs)],
                             eigenpairs_per_s=len(lam_s) / dt)
        log("slices: %d pairs in %.1f s, %d column B-applications" % (len(lam_s), dt, bapps))
        res["slices"] = (rs, lam_s)
        saved = {"slices": np.sort(lam_s), "edges": np.asarray(edges)}
    if not args.skip_window:
        t = time.time()
        r = P.filtered_eig(args.a, args.b, args.nev, args.tol, lmin=lmin, lmax=lmax, seed=9, verbose=1, **kw)
        torch.cuda.synchronize()
        dt = time.time() - t
        bapps = r.stats["bapps"] + r.stats["refine_bapps"]
        out["window"] = dict(seconds=dt, count=r.count, column_bapps=int(bapps), degree=r.stats["degree"],
                             basis=r.stats["basis"], resid_max=float(r.resid.max()), eigenpairs_per_s=r.count / dt)
        log("window: %d pairs in %.1f s, %d column B-applications" % (r.count, dt, bapps))
        saved["window"] = r.lam
        if "slices" in res:
            lam_s = res["slices"][1]
            out["slices_vs_window"] = dict(same_count=bool(len(lam_s) == r.count),
                                           max_rel_diff=float(np.abs(np.sort(lam_s) - r.lam).max() / r.lam.max())
                                           if len(lam_s) == r.count else None)
            log("slices vs window: %s" % out["slices_vs_window"])
        # rotation at the planet's Omega and at omega2
        rot = []
        extra = [float(x) for x in args.omega2.split(",") if x.strip()]
        for om_z, pen in (() if args.skip_rotation else [(args.omega, P)] + [(x, None) for x in extra]):
            if pen is None:
                d2 = dict(d)
                d2["omega"] = (0.0, 0.0, om_z)
                pen = nm.Pencil(d2)
            t = time.time()
            rr = pen.project_rotation(r, args.a, args.b)
            torch.cuda.synchronize()
            dt = time.time() - t
            fo = first_order(pen, r, nm, np)
            # nearest first-order value of every projected frequency away from the window ends
            om = np.sort(rr.omega)
            inner = om[(om * om >= 1.05 * args.a) & (om * om <= args.b / 1.05)]
            diff = float(np.abs(inner[:, None] - fo[None, :]).min(axis=1).max()) if len(inner) else None
            rot.append(dict(omega=om_z, modes=rr.count, seconds=dt, omega_min=float(rr.omega.min()),
                            omega_max=float(rr.omega.max()), first_order_max_diff=diff))
            log("Omega %g: %d rotating modes, max |omega - first order| %.3e" % (om_z, rr.count, diff if diff else -1.0))
        out["rotation"] = rot
        # O(Omega^2) check: the difference from first order over Omega^2 stays bounded as Omega falls
        if rot:
            out["second_order_coefficient"] = {("%g" % x["omega"]): x["first_order_max_diff"] / x["omega"] ** 2
                                               for x in rot if x["first_order_max_diff"]}
    if args.save:
        np.savez(args.save, **saved)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
