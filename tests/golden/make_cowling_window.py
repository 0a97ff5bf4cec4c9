"""Write the oracle's reference eigenvalues of a layered-planet window.

    python tests/golden/make_cowling_window.py [n_half] [a] [b]

Three-layer planet of the seeded generator (default seed) at n_half
(default 6: 10,368 tetrahedra, P2 displacement, P1 pressure), Cowling
pencil with the exact Schur complement: every eigenvalue in [a, b]
(default [1, 60]) by the oracle's window-complete shift-invert solve
(oracle.solve.cowling_window).  Only the oracle computes; the output holds
a digest of the planet arrays so a test can check it describes the same
input.
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import planetgen as pg  # noqa: E402
from oracle.assemble import Pencil  # noqa: E402
from oracle import solve as S  # noqa: E402


def planet_digest(planet):
    h = hashlib.sha256()
    for k in ("xyz", "tet", "region", "rho", "lam", "mu", "gprime", "grad_gprime"):
        h.update(np.ascontiguousarray(planet[k]).tobytes())
    return h.hexdigest()


def main():
    nh = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    a = float(sys.argv[2]) if len(sys.argv) > 2 else 1.0
    b = float(sys.argv[3]) if len(sys.argv) > 3 else 60.0
    planet = pg.three_layer_planet(n_half=nh)
    P = Pencil(planet)
    w, X = S.cowling_window(P, a, b)
    G = X.T @ (P.M @ X)
    orth = float(np.abs(G - np.eye(len(w))).max())
    R = np.column_stack([P.cowling_apply(X[:, i]) for i in range(len(w))]) - (P.M @ X) * w
    res = np.linalg.norm(R, axis=0) / (np.abs(w) * np.linalg.norm(P.M @ X, axis=0))
    out = os.path.join(HERE, "cowling_window_nh%d.txt" % nh)
    with open(out, "w") as f:
        f.write("# oracle.solve.cowling_window: three_layer_planet(n_half=%d), P2/P1, Cowling, window [%r, %r]\n"
                % (nh, a, b))
        f.write("# planet sha256 %s\n" % planet_digest(planet))
        f.write("# n_disp %d n_pres %d count %d max |X^T M X - I| %.2e max residual %.2e\n"
                % (P.n, P.n_p, len(w), orth, res.max()))
        for x in w:
            f.write("%.17e\n" % x)
    print("wrote", out, len(w), "eigenvalues")


if __name__ == "__main__":
    main()
