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
* Weighted traces for pencils with a large null space: tau_k = tr(T_k(.) B)
  = sum_i T_k(t_i) lambda_i (the recurrence started from B z), in which an
  eigenvalue 0 weighs nothing, and counts of [a, b] (a > 0) with the
  Jackson-damped Chebyshev coefficients of 1/lambda on [a, b]: the kernel's
  finite resolution can then not leak a degenerate cluster at 0 into a low
  window.
"""
from __future__ import annotations

import math

import numpy as np

from .solve import filter_coeffs, jackson


def kpm_traces(Bop, Z, lmin, lmax, m, weighted=False):
    """tau_k = (1/s) sum_v z_v^T T_k((B - c)/e) z_v, k = 0..m, for the s
    columns of Z, by the three-term recurrence W_{k+1} = 2 (B - c)/e W_k - W_{k-1}
    (weighted: started from W_0 = B Z)."""
    c, e = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    s = Z.shape[1]
    tau = np.empty(m + 1)
    W0 = Bop(Z) if weighted else Z
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


def exact_traces(lam, lmin, lmax, m, weighted=False):
    """tau_k = sum_i T_k(t_i) (weighted: sum_i T_k(t_i) lambda_i) from the
    eigenvalues themselves (T_k(cos th) = cos k th)."""
    c, e = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    lam = np.asarray(lam, float)
    th = np.arccos(np.clip((lam - c) / e, -1.0, 1.0))
    T = np.cos(np.outer(np.arange(m + 1), th))
    return (T * lam[None, :]).sum(axis=1) if weighted else T.sum(axis=1)


def inv_window_coeffs(a, b, lmin, lmax, m):
    """Jackson-damped Chebyshev coefficients on [lmin, lmax] of f = 1/lambda
    on [a, b] and 0 elsewhere: with lambda = c + e cos(th),
    c_k = (2/pi) int_{th_b}^{th_a} cos(k th) / (c + e cos th) dth (c_0 halved),
    each by adaptive quadrature."""
    from scipy.integrate import quad
    c, e = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    tha = math.acos(min(1.0, max(-1.0, (a - c) / e)))
    thb = math.acos(min(1.0, max(-1.0, (b - c) / e)))
    co = np.empty(m + 1)
    for k in range(m + 1):
        v, _ = quad(lambda th: math.cos(k * th) / (c + e * math.cos(th)), thb, tha, limit=400,
                    epsabs=1e-14, epsrel=1e-12)
        co[k] = (1.0 if k == 0 else 2.0) / math.pi * v
    return co * jackson(m)


def window_count(tau, lmin, lmax, a, b, weighted=False):
    """Estimated number of eigenvalues in [a, b]: sum_k mu_k tau_k (weighted
    traces: the coefficients of 1/lambda on [a, b])."""
    m = len(tau) - 1
    if weighted:
        return float(inv_window_coeffs(a, b, lmin, lmax, m) @ tau)
    mu, _, _ = filter_coeffs(a, b, lmin, lmax, m)
    return float(mu @ tau)


def slice_edges(tau, lmin, lmax, a, b, nslices, iters=60, weighted=False):
    """Ends a = x_0 < x_1 < ... < x_S = b of S slices with equal estimated
    counts (bisection on the cumulative count over [a, x])."""
    count = lambda x: window_count(tau, lmin, lmax, a, x, weighted)
    total = count(b)
    edges = [a]
    for i in range(1, nslices):
        target = total * i / nslices
        lo, hi = edges[-1], b
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if count(mid) < target:
                lo = mid
            else:
                hi = mid
        edges.append(0.5 * (lo + hi))
    edges.append(b)
    return np.array(edges)


__all__ = ["kpm_traces", "exact_traces", "inv_window_coeffs", "window_count", "slice_edges", "jackson"]
