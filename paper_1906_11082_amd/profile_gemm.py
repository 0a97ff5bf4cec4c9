"""Time the Lanczos block products (nm_gemm_tn / nm_gemm_nn) at a basis shape.

    python3 -m paper_1906_11082_amd.profile_gemm [--n 1633791] [--kmax 1400] [--q 32]

On a random FP64 basis V [n][kmax] (row-major, as the solver stores it) and a
block W [n][q]: C = V[:, :K]^T W and D = V[:, :K] C for K in 200, 800, kmax,
and the Rayleigh-Ritz product V[:, :K]^T V[:, :K] for K in 400, 800, each
beside torch.matmul on the same strided operands (the vendor GEMM).  Times are
means over a few calls between HIP events (nm_gemm_tn's call includes its
partial-sum allocation and its stream synchronisation).  Prints one JSON line.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1633791)
    ap.add_argument("--kmax", type=int, default=1400)
    ap.add_argument("--q", type=int, default=32)
    args = ap.parse_args()
    import torch
    import paper_1906_11082_amd as nm
    torch.manual_seed(0)
    n, q = args.n, args.q
    V = torch.randn(n, args.kmax, dtype=torch.float64, device="cuda")
    W = torch.randn(n, q, dtype=torch.float64, device="cuda")

    def timed(f, reps=5):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    for K in sorted({200, 800, args.kmax}):
        if K > args.kmax:
            continue
        Cm = torch.randn(K, q, dtype=torch.float64, device="cuda")
        D = torch.empty(n, q, dtype=torch.float64, device="cuda")
        out["tn K=%d q=%d" % (K, q)] = (timed(lambda: nm.gemm_tn(V, W, K, q)), timed(lambda: V[:, :K].T @ W))
        out["nn K=%d q=%d" % (K, q)] = (timed(lambda: nm.gemm_nn(V, Cm, D)),
                                        timed(lambda: torch.matmul(V[:, :K], Cm, out=D)))
        print("K %d done" % K, file=sys.stderr, flush=True)
    for K in (400, 800):
        if K > args.kmax:
            continue
        out["tn K=%d q=%d (V^T V)" % (K, K)] = (timed(lambda: nm.gemm_tn(V, V, K, K), 3),
                                                timed(lambda: V[:, :K].T @ V[:, :K], 3))
    res = dict(n=n, kmax=args.kmax, products={k: dict(ms=round(a, 3), torch_matmul_ms=round(b, 3))
                                              for k, (a, b) in out.items()})
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
