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


def test_weighted_traces_over_all_unit_vectors_are_exact(ball):
    """Weighted traces (recurrence started from B z) over the scaled unit
    vectors are exactly sum_i T_k(t_i) lambda_i."""
    P, lam, B = ball
    lmin, lmax = -0.01, 1.01 * lam.max()
    tau = D.kpm_traces(B, np.sqrt(P.n) * np.eye(P.n), lmin, lmax, 30, weighted=True)
    ref = D.exact_traces(lam, lmin, lmax, 30, weighted=True)
    assert np.abs(tau - ref).max() <= 1e-10 * np.abs(ref).max()


def test_weighted_count_ignores_a_null_cluster():
    """A spectrum as wide as the benchmark planet's (to 7e5) with 5000
    eigenvalues exactly 0 (a fluid null space) and multiplets at 10, 20 and
    30 (and 90): from exact traces at degree 3000 the weighted count of [1, 40] is the
    true 21 within one (the multiplets sit farther from the ends than the
    kernel's resolution), the unweighted one is swamped by the null cluster's leak;
    the undamped series of 1/lambda on [1, 40] reproduces 1/lambda inside it,
    and weighted slices split the multiplets."""
    rng = np.random.default_rng(5)
    lam = np.concatenate([np.zeros(5000), np.full(5, 10.0), np.full(7, 20.0), np.full(9, 30.0), np.full(11, 90.0),
                          rng.uniform(100.0, 7.0e5, 400)])
    lmin, lmax, m = -0.5, 7.1e5, 3000
    tw = D.exact_traces(lam, lmin, lmax, m, weighted=True)
    tu = D.exact_traces(lam, lmin, lmax, m)
    est_w = D.window_count(tw, lmin, lmax, 1.0, 40.0, weighted=True)
    est_u = D.window_count(tu, lmin, lmax, 1.0, 40.0)
    # within one eigenvalue: the smoothing of the steep 1/lambda near a = 1
    # costs a fraction of one (0.6 here, 0.24 at degree 5000)
    assert abs(est_w - 21) < 1.0, est_w
    assert est_u > 100, est_u
    # on a narrow interval, where degree 400 resolves it, the undamped series
    # of 1/lambda on [1, 40] is 1/lambda inside the window and 0 outside
    lo2, hi2, m2 = -0.5, 100.0, 400
    co = D.inv_window_coeffs(1.0, 40.0, lo2, hi2, m2) / D.jackson(m2)
    c, e = 0.5 * (hi2 + lo2), 0.5 * (hi2 - lo2)
    for x, want in ((5.0, 0.2), (15.0, 1 / 15.0), (25.0, 0.04), (35.0, 1 / 35.0), (60.0, 0.0), (90.0, 0.0)):
        v = np.polynomial.chebyshev.chebval((x - c) / e, co)
        assert abs(v - want) < 0.01, (x, v, want)
    edges = D.slice_edges(tw, lmin, lmax, 1.0, 40.0, 3, weighted=True)
    cnt = [((lam >= edges[i]) & (lam < edges[i + 1])).sum() for i in range(3)]
    assert cnt == [5, 7, 9], (edges, cnt)
