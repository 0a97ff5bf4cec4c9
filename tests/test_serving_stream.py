"""Host logic of the serving workload: the seeded request stream (no GPU)."""
import argparse
import math

import numpy as np

from paper_1906_11082_amd.serving import make_stream


def _args(**kw):
    base = dict(requests=64, rate=2.0, tmin=2e4, tmax=8e5, max_slices=8, width=5.0, seed=4)
    base.update(kw)
    return argparse.Namespace(**base)


def test_stream_is_seeded_and_within_ranges():
    a = make_stream(_args())
    b = make_stream(_args())
    assert a == b
    assert len(a) == 64
    arr = np.array([r["arrival"] for r in a])
    assert np.all(np.diff(arr) > 0)
    # Poisson at 2 req/s: mean gap 0.5 s (64 gaps: within 4 standard errors)
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 0.5) < 4 * 0.5 / math.sqrt(64)
    for r in a:
        tets = 48 * r["n_half"] ** 3
        assert 0.5 * 2e4 <= tets <= 1.5 * 8e5
        assert r["order"] in (1, 2) and r["omega"] in (0.0, 0.05, 0.5)
        assert 1 <= len(r["windows"]) <= 8 and len(r["nev"]) == len(r["windows"])
        assert all(20 <= v <= 100 for v in r["nev"])
        lo = [w[0] for w in r["windows"]]
        assert lo[0] == 1.0 and all(w[1] > w[0] for w in r["windows"])
        assert all(r["windows"][k][1] == r["windows"][k + 1][0] for k in range(len(lo) - 1))
    assert make_stream(_args(seed=5)) != a
