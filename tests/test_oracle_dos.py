"""Pins of the oracle's density-of-states estimate and spectrum slices
against exact eigenvalue counts of small pencils (dense solves)."""
import numpy as np
import pytest

from conftest import pencil
from oracle import dos as D
from oracle import solve as S


@pytest.fixture(scope="module")
def ball():
    P = pencil("homogeneous_ball", n_half=3, order=1)
    A, M = P.AG.toarray(), P.M.toarray()
    lam = S.dense_window(A, M, -1.0, 1e9)[0]
    Bd = np.linalg.solve(M, A)
    return P, lam, (lambda X: Bd @ X)


def test_traces_over_all_unit_vectors_are_exact(ball):
    """With z running over the unit vectors scaled by sqrt(n) (so that the
    mean of z z^T is the identity), (1/n) sum z^T T_k z is exactly
    tr T_k = sum_i cos(k arccos t_i)."""
    P, lam, B = ball
    lmin, lmax = -0.01, 1.01 * lam.max()
    tau = D.kpm_traces(B, np.sqrt(P.n) * np.eye(P.n), lmin, lmax, 30)
    ref = D.exact_traces(lam, lmin, lmax, 30)
    assert np.abs(tau - ref).max() <= 1e-10 * np.abs(ref).max()


def test_counts_from_exact_traces(ball):
    """The Jackson-damped series of the indicator applied to exact traces
    counts the eigenvalues of windows whose ends lie in spectral gaps; the
    cumulative count is nondecreasing."""
    P, lam, B = ball
    lmin, lmax = -0.01, 1.01 * lam.max()
    tau = D.exact_traces(lam, lmin, lmax, 1500)
    gaps = np.nonzero(np.diff(lam) > 0.05 * lam[1:])[0]
    checked = 0
    for i in gaps[(lam[gaps] > 1.0) & (lam[gaps] < 200.0)][:6]:
        b = 0.5 * (lam[i] + lam[i + 1])
        a = 0.5
        true = int(((lam >= a) & (lam <= b)).sum())
        est = D.window_count(tau, lmin, lmax, a, b)
        assert abs(est - true) < 0.5, (b, est, true)
        checked += 1
    assert checked >= 3
    xs = np.linspace(0.6, 150.0, 60)
    cum = [D.window_count(tau, lmin, lmax, 0.5, x) for x in xs]
    assert np.all(np.diff(cum) >= -1e-9)


def test_stochastic_estimate_and_slices(ball):
    """Hutchinson's estimate with 64 Gaussian vectors is within a few standard
    deviations of the true count (variance 2 count / s for a projector), and
    equal-count slices of [1, 120] hold about a quarter of the count each."""
    P, lam, B = ball
    lmin, lmax = -0.01, 1.01 * lam.max()
    Z = np.random.default_rng(3).standard_normal((P.n, 64))
    tau = D.kpm_traces(B, Z, lmin, lmax, 300)
    a, b = 1.0, 120.0
    true = int(((lam >= a) & (lam <= b)).sum())
    est = D.window_count(tau, lmin, lmax, a, b)
    assert abs(est - true) <= 5 * np.sqrt(2 * true / 64) + 1.5, (est, true)
    ex = D.slice_edges(D.exact_traces(lam, lmin, lmax, 300), lmin, lmax, a, b, 4)
    assert ex[0] == a and ex[-1] == b and np.all(np.diff(ex) > 0)
    cnt = [((lam >= ex[i]) & (lam < ex[i + 1])).sum() for i in range(4)]
    assert max(abs(c - true / 4) for c in cnt) <= 0.25 * true / 4 + 8, cnt
