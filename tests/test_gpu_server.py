"""Request server: continuous batching of eigensolves on one GPU."""
import numpy as np
import pytest

from conftest import planet as make_planet, pencil as oracle_pencil, window_ref, check_against_oracle

pytestmark = pytest.mark.gpu


def _requests():
    return [
        (make_planet("homogeneous_ball", n_half=4, order=1), [(0.5, 40.0)], 30, dict(degree=40, block=8)),
        (make_planet("three_layer_planet", n_half=4, order=2, pres_order=1), [(1.0, 6.0), (6.0, 12.0)], 100,
         dict(block=8)),
        (make_planet("homogeneous_ball", n_half=3, order=2), [(0.5, 30.0)], 20, dict(block=8, precision=1)),
    ]


def _overlaps(res):
    return [(i, j) for i in range(len(res)) for j in range(i + 1, len(res))
            if res[i]["t_start"] < res[j]["t_end"] and res[j]["t_start"] < res[i]["t_end"]]


def test_server_results_same_alone_and_in_the_mix():
    """Each request's eigenvalues and vectors are bit-identical when it runs
    alone and when it runs concurrently with the others; in the mix the
    requests overlap in time."""
    import paper_1906_11082_amd as nm
    reqs = _requests()
    s1 = nm.Server(hbm_budget_gb=100.0, max_active=1)
    alone = [s1.wait(s1.submit(p, w, nev, 1e-8, **kw)) for p, w, nev, kw in reqs]
    s1.close()
    s3 = nm.Server(hbm_budget_gb=100.0, max_active=3)
    tickets = [s3.submit(p, w, nev, 1e-8, **kw) for p, w, nev, kw in reqs]
    mix = [s3.wait(t) for t in tickets]
    s3.close()
    for k, (a, m) in enumerate(zip(alone, mix)):
        print("request %d: status %d/%d, %s pairs, alone %.2fs, mix %.2fs" % (
            k, a["status"], m["status"], [r.count for r in m["slices"]], a["t_end"] - a["t_start"],
            m["t_end"] - m["t_start"]), flush=True)
        assert a["status"] == 0 and m["status"] == 0, (a["error"], m["error"])
        assert len(a["slices"]) == len(m["slices"]) == len(reqs[k][1])
        for ra, rm in zip(a["slices"], m["slices"]):
            assert ra.count == rm.count > 0
            assert np.array_equal(ra.lam, rm.lam)
            assert np.array_equal(ra.X.cpu().numpy(), rm.X.cpu().numpy())
            assert rm.resid.max() <= 1e-8
    assert _overlaps(mix), "no two requests ran concurrently"
    assert not _overlaps(alone)
    # and against the oracle: dense solves of the balls, shift-invert windows of the layered planet
    from oracle import solve as S
    refs = []
    for name, kw in (("homogeneous_ball", dict(n_half=4, order=1)), ("homogeneous_ball", dict(n_half=3, order=2))):
        O = oracle_pencil(name, **kw)
        refs.append((O, S.dense_window(O.AG.toarray(), O.M.toarray(), *(reqs[0 if kw["order"] == 1 else 2][1][0]))))
    O1, (w1, X1) = refs[0]
    check_against_oracle(mix[0]["slices"][0], w1, X1, O1.M, rel=1e-9, resid=1e-8, nev=30)
    O3, (w3, X3) = refs[1]
    check_against_oracle(mix[2]["slices"][0], w3, X3, O3.M, rel=1e-8, resid=1e-8, nev=20, proj=1e-6)
    O2 = oracle_pencil("three_layer_planet", n_half=4, order=2, pres_order=1)
    for (a, b), r in zip(reqs[1][1], mix[1]["slices"]):
        w, X = window_ref("three_layer_planet", a, b, n_half=4, order=2, pres_order=1)
        check_against_oracle(r, w, X, O2.M, rel=1e-9, resid=1e-8)


def test_server_budget_serialises_and_rotation():
    """With a budget below any request's estimate the server still admits the
    head request when nothing runs, so requests run one at a time; a request
    with rotation gets the projected Coriolis modes over its windows."""
    import paper_1906_11082_amd as nm
    d = dict(make_planet("homogeneous_ball", n_half=4, order=1))
    d["omega"] = (0.0, 0.0, 0.2)
    s = nm.Server(hbm_budget_gb=1e-6, max_active=4)
    ts = [s.submit(d, [(0.5, 40.0)], 30, 1e-9, degree=40, block=8, rotate=True) for _ in range(3)]
    res = [s.wait(t) for t in ts]
    s.close()
    assert not _overlaps(res)
    for r in res:
        assert r["status"] == 0 and r["est_bytes"] > 1e3
        assert r["rotation"] is not None and r["rotation"].count > 0
        np.testing.assert_array_equal(r["rotation"].omega, res[0]["rotation"].omega)
    assert res[0]["t_submit"] <= res[1]["t_submit"] <= res[2]["t_submit"]
