import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


_CACHE = {}


def planet(name, **kw):
    """Cached seeded planets shared by the tests of one session."""
    import planetgen as pg
    key = (name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = getattr(pg, name)(**kw)
    return _CACHE[key]


def pencil(name, **kw):
    from oracle.assemble import Pencil
    key = ("pencil", name, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = Pencil(planet(name, **kw))
    return _CACHE[key]


def window_ref(name, a, b, **kw):
    """The oracle's eigenpairs of the Cowling pencil in [a, b] (window-complete
    shift-invert with the exact Schur complement), cached per session."""
    from oracle import solve as S
    key = ("window", name, a, b, tuple(sorted(kw.items())))
    if key not in _CACHE:
        _CACHE[key] = S.cowling_window(pencil(name, **kw), a, b)
    return _CACHE[key]


def clusters(w, rel=1e-6):
    """Index groups of (near-)equal consecutive eigenvalues."""
    import numpy as np
    groups, cur = [], [0]
    for i in range(1, len(w)):
        if w[i] - w[i - 1] <= rel * abs(w[i]):
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    if len(w):
        groups.append(cur)
    return groups


def check_against_oracle(r, w_ref, X_ref, M, rel=1e-9, resid=1e-8, nev=None, proj=1e-7):
    """A GPU result against the oracle's window: the min(nev, count) smallest
    pairs, eigenvalues within rel (relative to the largest), residuals within
    resid, and per cluster of (near-)equal eigenvalues the M-orthogonal
    projectors agree (singular values of X^T M X_ref above 1 - proj); the last
    cluster is skipped when the nev cut may split it."""
    import numpy as np
    k = len(w_ref) if nev is None else min(nev, len(w_ref))
    assert r.count == k, (r.count, k)
    if k == 0:
        return
    w = w_ref[:k]
    err = np.abs(r.lam - w).max() / np.abs(w).max()
    assert err <= rel, err
    assert r.resid.max() <= resid, r.resid.max()
    if X_ref is None:
        return
    X = r.X.cpu().numpy()
    for g in clusters(w):
        if g[-1] == k - 1 and k < len(w_ref):
            continue
        s = np.linalg.svd(X[:, g].T @ (M @ X_ref[:, g]), compute_uv=False)
        assert s.min() > 1 - proj, (g, s)
