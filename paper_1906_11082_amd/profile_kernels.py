"""Run the hot kernels at the benchmark configuration, for rocprofv3.

    rocprofv3 --kernel-trace --stats -d <dir> -- python3 -m paper_1906_11082_amd.profile_kernels
    rocprofv3 --pmc FETCH_SIZE -d <dir> -- python3 -m paper_1906_11082_amd.profile_kernels
    rocprofv3 --pmc WRITE_SIZE -d <dir> -- python3 -m paper_1906_11082_amd.profile_kernels

Launches, on the three-layer planet at n_half (default 20): `reps` M-solves
of `steps` Chebyshev-Jacobi steps on a block of `block` columns (so the
middle-step kernel dominates: k_cj_group from 32 columns, k_cj_step for
narrower blocks), one filter application of degree `degree`, and a
plain device copy of `copy_mb` MB (torch) that calibrates the HBM byte
counters.  Prints the algorithmic bytes of one middle-step launch so the
counters can be compared with it.

--mass-passes P (FP64 vectors): the M solves and the filter's M solves run as
P FP32 passes of `steps` (filter: 22) steps with FP64 residual corrections,
so the middle-step kernel is the FP32 one (k_cj_group at 32 columns) next to
k_mix_first, k_mix_resid and k_mix_final.
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-half", type=int, default=20)
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--degree", type=int, default=4)
    ap.add_argument("--copy-mb", type=int, default=1024)
    ap.add_argument("--mass-passes", type=int, default=0)
    args = ap.parse_args()
    if args.mass_passes and args.precision != "fp64":
        ap.error("--mass-passes runs with FP64 vectors")
    import numpy as np
    import torch
    import planetgen as pg
    import paper_1906_11082_amd as nm

    torch.cuda.set_device(0)
    planet = pg.three_layer_planet(n_half=args.n_half)
    P = nm.Pencil(planet)
    prec = 1 if args.precision == "fp32" else 0
    dt = torch.float32 if prec else torch.float64
    s = 4 if (prec or args.mass_passes) else 8
    X = torch.randn(P.n, args.block, dtype=dt, device="cuda")
    mp = args.mass_passes
    for _ in range(args.reps):
        P.apply(nm.OP_MINV, X, kM=args.steps, precision=prec, mass_passes=mp)
    lo, hi = -1.0, 7.1e5
    mu = nm.filter_coeffs(1.0, 60.0, lo, hi, args.degree)
    P.filter_apply(mu, 0.5 * (hi + lo), 0.5 * (hi - lo), X, kM=22 if mp else 45, precision=prec, mass_passes=mp)
    n_copy = args.copy_mb * (1 << 20) // 8
    a = torch.empty(n_copy, dtype=torch.float64, device="cuda").normal_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    nnzb, N, n = P.info["nnzb"], P.info["n_node"], P.info["n_disp"]
    cj = nnzb * (4 + s) + 4 * (N + 1) + s * N + 4 * n * args.block * s
    print("Chebyshev-Jacobi step algorithmic bytes per launch %d (nnzb %d, N %d, block %d, %s%s)"
          % (cj, nnzb, N, args.block, args.precision, ", %d FP32 passes" % mp if mp else ""))
    print("copy kernel bytes per launch %d (read) + %d (write)" % (n_copy * 8, n_copy * 8))


if __name__ == "__main__":
    main()
