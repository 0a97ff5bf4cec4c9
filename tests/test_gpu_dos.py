"""GPU density of states (kernel polynomial method) against the oracle."""
import numpy as np
import pytest

from conftest import planet as make_planet, pencil as oracle_pencil

pytestmark = pytest.mark.gpu


def test_dos_traces_match_oracle():
    """tau_k from the GPU recurrence equal the oracle's for the same random
    block (1e-9 of the largest, degree 200), and at degree 1200 the count they
    give for [1, 12] is the oracle window's count within the stochastic error
    (Hutchinson, 32 vectors) and the kernel's smoothing at the window ends."""
    import torch
    import paper_1906_11082_amd as nm
    from oracle import dos as D
    from oracle import solve as S
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    O = oracle_pencil("three_layer_planet", n_half=4, order=2, pres_order=1)
    G = nm.Pencil(d)
    lo, hi = G.spectrum_bounds(60, 3)
    lmin, lmax = lo - 0.01, hi
    Zh = np.random.default_rng(8).standard_normal((G.n, 32))
    Z = torch.from_numpy(Zh).cuda()
    m = 200
    tau = G.spectrum_dos(lmin, lmax, m, Z, minv_tol=1e-12, kp_tol=1e-13)
    op = S.CowlingOperator(O, minv_tol=1e-12, kp_tol=1e-13)
    ref = D.kpm_traces(op.B, Zh, lmin, lmax, m)
    err = np.abs(tau - ref).max() / np.abs(ref).max()
    print("dos traces: max rel difference %.2e" % err, flush=True)
    assert err <= 1e-9
    w, _ = S.cowling_window(O, 1.0, 12.0)
    tau = G.spectrum_dos(lmin, lmax, 1200, Z, minv_tol=1e-12, kp_tol=1e-13)
    est = nm.dos_count(tau, lmin, lmax, 1.0, 12.0)
    print("count [1, 12]: estimate %.1f, oracle %d" % (est, len(w)), flush=True)
    assert abs(est - len(w)) <= 6 * np.sqrt(2 * len(w) / 32) + 3
