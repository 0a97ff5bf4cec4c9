"""Throughput of the self-gravitation N-body sums (Sec. 5) on one GPU.

    python3 -m paper_1906_11082_amd.profile_selfgrav [--n-half 12] [--cols 8] [--reps 5]

Builds the bodies of the three-layer planet at n_half (tetrahedra, surface
and fluid-solid faces), then times nm_selfgrav_apply (charges C X, the
direct N-body sums S q, the scatter C^T) on `cols` columns with HIP events
(the N-body kernel variant from the NM_NBODY environment variable),
and the reference field at the vertices.  Reports pairs per second and the
FP32 rate of the N-body kernel against the 157.3 TFLOP/s FP32 vector peak,
counting per pair and column one FMA (2 flops) and per pair 8 flops for the
distance and its reciprocal square root.  Prints one JSON line.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-half", type=int, default=12)
    ap.add_argument("--cols", type=int, default=8)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import numpy as np
    import torch
    import planetgen as pg
    import paper_1906_11082_amd as nm

    torch.cuda.set_device(0)
    d = pg.three_layer_planet(n_half=args.n_half)
    P = nm.Pencil(d)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    sg = nm.SelfGravity(P, d)
    t1.record()
    torch.cuda.synchronize()
    build_ms = t0.elapsed_time(t1)
    X = torch.randn(P.n, args.cols, dtype=torch.float64, device="cuda")
    sg.apply(X)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(args.reps):
        sg.apply(X)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / args.reps
    nb = sg.n_body
    pairs = float(nb) * nb
    flops = pairs * (2.0 * args.cols + 8.0)
    pts = torch.from_numpy(np.asarray(d["xyz"], np.float64)).cuda()
    sg.field(pts)
    torch.cuda.synchronize()
    t0.record()
    sg.field(pts)
    t1.record()
    torch.cuda.synchronize()
    fms = t0.elapsed_time(t1)
    fpairs = float(pts.shape[0]) * sg.n_tet
    print(json.dumps(dict(
        kernel=os.environ.get("NM_NBODY", "split"),
        workload="self-gravitation of the three-layer planet, %d tets, %d bodies (%d faces), %d columns"
                 % (len(d["tet"]), nb, sg.n_face, args.cols),
        build_ms=build_ms, apply_ms=ms, pairs_per_s=pairs / (ms * 1e-3),
        fp32_tflops=flops / (ms * 1e-3) / 1e12, frac_of_fp32_peak=flops / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
        field_ms=fms, field_pairs_per_s=fpairs / (fms * 1e-3))), flush=True)


if __name__ == "__main__":
    main()
