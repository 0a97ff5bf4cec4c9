"""Density of states of the pencil and spectrum slices (oracle, FP64).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package; the GPU library never does.

Sec. 6.1 solves for the modes in a window with polynomial filtering, and its
spectrum slicing follows the cited EVSL approach, where slice ends come from
a density-of-states estimate.  This module writes that estimate out plainly:

* Eigenvalue counts are traces of spectral projectors.  With B = M^{-1} A,
  t = (lambda - c)/e mapping [lmin, lmax] onto [-1, 1], and the Jackson-damped
  Chebyshev coefficients mu_k = g_k gamma_k of the indicator of [a, b] (the
  filter's own series), the number of eigenvalues in [a, b] is estimated by
  sum_k mu_k tau_k, tau_k = tr T_k((B - c)/e) (kernel polynomial method; the
  Jackson kernel is positive, so with exact traces the smoothed count is
  nondecreasing in b).
* tau_k is estimated by Hutchinson's estimator: for vectors z with
  E[z z^T] = I, E[z^T X z] = tr X for any matrix X, so
  tau_k ~ (1/s) sum_v z_v^T T_k((B - c)/e) z_v; the vectors are inputs (the
  caller draws them).  With z running over all unit vectors times sqrt(n)
  the sum is exact.
* Slices of [a, b] with equal estimated counts: the ends x_i where the
  cumulative count over [a, x_i] reaches i/S of the count over [a, b]
  (bisection).
"""
from __future__ import annotations

import numpy as np

from .solve import filter_coeffs, jackson


def kpm_traces(Bop, Z, lmin, lmax, m):
    """tau_k = (1/s) sum_v z_v^T T_k((B - c)/e) z_v, k = 0..m, for the s
    columns of Z, by the three-term recurrence W_{k+1} = 2 (B - c)/e W_k - W_{k-1}."""
    c, e = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    s = Z.shape[1]
    tau = np.empty(m + 1)
    W0 = Z
    tau[0] = np.einsum("ij,ij->", Z, W0) / s
    if m == 0:
        return tau
    W1 = (Bop(W0) - c * W0) / e
    tau[1] = np.einsum("ij,ij->", Z, W1) / s
    for k in range(2, m + 1):
        W2 = 2.0 * (Bop(W1) - c * W1) / e - W0
        tau[k] = np.einsum("ij,ij->", Z, W2) / s
        W0, W1 = W1, W2
    return tau


def exact_traces(lam, lmin, lmax, m):
    """tau_k = sum_i T_k(t_i) from the eigenvalues themselves (T_k(cos th) = cos k th)."""
    c, e = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    th = np.arccos(np.clip((np.asarray(lam) - c) / e, -1.0, 1.0))
    return np.cos(np.outer(np.arange(m + 1), th)).sum(axis=1)


def window_count(tau, lmin, lmax, a, b):
    """Estimated number of eigenvalues in [a, b]: sum_k mu_k tau_k."""
    m = len(tau) - 1
    mu, _, _ = filter_coeffs(a, b, lmin, lmax, m)
    return float(mu @ tau)


def slice_edges(tau, lmin, lmax, a, b, nslices, iters=60):
    """Ends a = x_0 < x_1 < ... < x_S = b of S slices with equal estimated
    counts (bisection on the cumulative count over [a, x])."""
    total = window_count(tau, lmin, lmax, a, b)
    edges = [a]
    for i in range(1, nslices):
        target = total * i / nslices
        lo, hi = edges[-1], b
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if window_count(tau, lmin, lmax, a, mid) < target:
                lo = mid
            else:
                hi = mid
        edges.append(0.5 * (lo + hi))
    edges.append(b)
    return np.array(edges)


__all__ = ["kpm_traces", "exact_traces", "window_count", "slice_edges", "jackson"]
