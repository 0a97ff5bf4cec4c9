"""The GPU solve of the full-size layered planet against the radial (1-D)
oracle of Appendix B (eq. "1Dform")."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_full_size_planet_converges_to_radial_oracle():
    """The three-layer planet at n_half 12 (384,000 tetrahedra, P2/P1, the
    benchmark's planet), Cowling, window [1, 12] on the GPU (block 32, mixed
    mass solve): as many eigenvalues as the radial multiplets stand for, each
    within 2 % of its radial value, and every multiplet at least 2.5 times
    closer than the oracle's n_half 6 solve (discretisation error O(h^2))."""
    import planetgen as pg
    import paper_1906_11082_amd as nm
    from oracle import radial as RD
    lay = RD.layers_from(pg.three_layer_model())
    rows = RD.spectrum(lay, 1.0, 12.0, 10, nel=40, p=3, gravity="cowling")
    ms = RD.multiset(rows)
    w6 = np.loadtxt(os.path.join(HERE, "golden", "cowling_window_nh6.txt"))
    w6 = w6[(w6 >= 1.0) & (w6 <= 12.0)]
    print("\n[case] radial oracle vs n_half 12, window [1, 12]", flush=True)
    d = pg.three_layer_planet(n_half=12)
    G = nm.Pencil(d)
    r = G.filtered_eig(1.0, 12.0, 100, 1e-8, block=32, mass_passes=2, verbose=1)
    print("count %d (radial multiplets stand for %d), degree %d" % (r.count, len(ms), r.stats["degree"]), flush=True)
    assert r.count == len(ms) == len(w6)
    e12 = np.abs(r.lam - ms) / ms
    e6 = np.abs(w6 - ms) / ms
    start = 0
    for wr, l, kind in rows:
        m = int(2 * l + 1)
        a, b = e6[start:start + m].mean(), e12[start:start + m].mean()
        print("%s l=%d radial %.5f: mean rel error n_half 6 %.2e, n_half 12 %.2e"
              % ("ST"[int(kind)], l, wr, a, b), flush=True)
        assert b < a / 2.5
        start += m
    assert e12.max() <= 0.02
