"""Pins of the oracle's solver pieces: Chebyshev-Jacobi mass solve,
Jackson-Chebyshev filter, Lanczos bounds, filtered Lanczos + Rayleigh-Ritz,
and the closed-form spectrum of the homogeneous elastic ball."""
import math
import os

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sla
import scipy.optimize as so
import scipy.sparse.linalg as spla
import scipy.special as ss

from conftest import planet, pencil
from oracle import solve as S
from oracle.assemble import Pencil

HERE = os.path.dirname(__file__)


# ---------------------------------------------------------------- mass solve
@pytest.mark.parametrize("order", [1, 2])
def test_wathen_bounds_enclose_assembled_spectrum(order):
    P = pencil("three_layer_planet", n_half=3, order=order)
    M = P.Ms.toarray()
    w = sla.eigh(M, np.diag(np.diag(M)), eigvals_only=True)
    lo, hi = S.jacobi_mass_bounds(order)
    assert w.min() >= lo * (1 - 1e-12) and w.max() <= hi * (1 + 1e-12)


@pytest.mark.parametrize("order,tol", [(1, 1e-10), (2, 1e-10), (2, 1e-6)])
def test_cheb_jacobi_error_bound(order, tol):
    P = pencil("three_layer_planet", n_half=4, order=order)
    lo, hi = S.jacobi_mass_bounds(order)
    k = S.cheb_iters(lo, hi, tol)
    rng = np.random.default_rng(1)
    f = rng.standard_normal((P.n, 3))
    y = S.cheb_jacobi(lambda x: P.M @ x, np.repeat(P.Ms.diagonal(), 3), f, k, lo, hi)
    ys = spla.splu(P.M.tocsc()).solve(f)
    e = y - ys
    en = np.sqrt(np.einsum("ij,ij->j", e, P.M @ e))
    xn = np.sqrt(np.einsum("ij,ij->j", ys, P.M @ ys))
    assert np.all(en <= tol * xn)
    # the fixed-k solve is a symmetric operator
    Sx = S.cheb_jacobi(lambda x: P.M @ x, np.repeat(P.Ms.diagonal(), 3), f[:, :2], k, lo, hi)
    assert abs(f[:, 0] @ Sx[:, 1] - f[:, 1] @ Sx[:, 0]) < 1e-13 * np.abs(f[:, 0] @ Sx[:, 0])


@pytest.mark.parametrize("passes,k", [(2, 12), (3, 8)])
def test_refined_mass_solve_error_operator_and_bound(passes, k):
    """Refinement y <- y + S(f - M y) of the k-step solve S: the error after P
    passes is (I - S M)^P applied to M^{-1} f (the error propagated pass by pass
    from the exact solution, not through residuals), its M-norm is at most
    (2 r^k)^P of that of M^{-1} f (I - S M is a polynomial in D^{-1} M,
    self-adjoint in the M-inner product, of norm <= 2 r^k), and the passes in
    float32 with float64 residuals stay within float32 rounding of the last
    correction, 1e-5 (2 r^k)^(P-1), of the float64 refinement."""
    P = pencil("three_layer_planet", n_half=4, order=2)
    lo, hi = S.jacobi_mass_bounds(2)
    d = np.repeat(P.Ms.diagonal(), 3)
    Mop = lambda x: P.M @ x
    M32 = P.M.astype(np.float32)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((P.n, 3))
    xs = spla.splu(P.M.tocsc()).solve(f)
    y = S.cheb_jacobi_refined(Mop, d, f, k, lo, hi, passes)
    e = xs.copy()
    for _ in range(passes):
        e = e - S.cheb_jacobi(Mop, d, Mop(e), k, lo, hi)
    mn = lambda v: np.sqrt(np.einsum("ij,ij->j", v, P.M @ v))
    assert np.all(mn((xs - y) - e) <= 1e-12 * mn(xs))
    kap = hi / lo
    fac = 2 * ((math.sqrt(kap) - 1) / (math.sqrt(kap) + 1)) ** k
    assert np.all(mn(xs - y) <= fac ** passes * mn(xs))
    # one pass is the plain solve
    assert np.array_equal(S.cheb_jacobi_refined(Mop, d, f, k, lo, hi, 1), S.cheb_jacobi(Mop, d, f, k, lo, hi))
    y32 = S.cheb_jacobi_refined(Mop, d, f, k, lo, hi, passes, Mop32=lambda x: M32 @ x)
    rel = np.linalg.norm(y32 - y, axis=0) / np.linalg.norm(y, axis=0)
    assert np.all(rel <= 1e-5 * fac ** (passes - 1))


def test_refined_float32_passes_beat_float32_rounding():
    """At the benchmark's setting (2 passes of 22 steps, bound 1.8e-9) the
    float32 passes reach the float64 bound, while one float32 solve of 44
    steps stops at float32 rounding."""
    P = pencil("three_layer_planet", n_half=4, order=2)
    lo, hi = S.jacobi_mass_bounds(2)
    d = np.repeat(P.Ms.diagonal(), 3)
    M32 = P.M.astype(np.float32)
    f = np.random.default_rng(4).standard_normal((P.n, 2))
    xs = spla.splu(P.M.tocsc()).solve(f)
    y32 = S.cheb_jacobi_refined(lambda x: P.M @ x, d, f, 22, lo, hi, 2, Mop32=lambda x: M32 @ x)
    one32 = S.cheb_jacobi(lambda x: M32 @ x, d.astype(np.float32), f.astype(np.float32), 44,
                          np.float32(lo), np.float32(hi)).astype(np.float64)
    e_ref = np.linalg.norm(y32 - xs, axis=0) / np.linalg.norm(xs, axis=0)
    e_one = np.linalg.norm(one32 - xs, axis=0) / np.linalg.norm(xs, axis=0)
    assert np.all(e_ref <= 1e-8) and np.all(e_one >= 1e-8) and np.all(e_one > 10 * e_ref)


# -------------------------------------------------------------------- filter
def test_jackson_and_window_coefficients():
    g = S.jackson(30)
    assert abs(g[0] - 1.0) < 1e-15
    assert np.all(np.diff(g) < 0) and g[-1] > 0
    a, b = -0.3, 0.45
    gam = S.window_chebyshev(a, b, 12)
    for k in range(13):
        val = si.quad(lambda th: math.cos(k * th), math.acos(b), math.acos(a), epsabs=1e-14)[0]
        ref = (1 if k == 0 else 2) / math.pi * val
        assert abs(gam[k] - ref) < 1e-12


def test_filter_recurrence_matches_scalar_polynomial():
    """p(B) x = sum_i p(lambda_i) (x_i) on a dense B with known eigenpairs;
    Jackson damping keeps 0 <= p <= 1 (positivity of the Jackson kernel)."""
    rng = np.random.default_rng(7)
    n = 40
    lam = np.sort(rng.uniform(0.0, 50.0, n))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = Q @ np.diag(lam) @ Q.T
    mu, c, e = S.filter_coeffs(10.0, 20.0, 0.0, 50.0, 60)
    x = rng.standard_normal((n, 2))
    y = S.filter_apply(lambda v: B @ v, x, mu, c, e)
    p = S.cheb_series(mu, (lam - c) / e)
    ref = Q @ (p[:, None] * (Q.T @ x))
    assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()
    t = np.linspace(-1, 1, 2001)
    pt = S.cheb_series(mu, t)
    assert pt.min() > -1e-12 and pt.max() < 1 + 1e-12
    yn = S.filter_apply(lambda v: B @ v, x, mu, c, e, null_shift=0.0, null_scale=20.0)
    refn = Q @ ((p * lam / 20.0)[:, None] * (Q.T @ x))
    assert np.abs(yn - refn).max() < 1e-12 * np.abs(refn).max()


def test_lanczos_bounds_enclose_dense_extremes():
    P = pencil("homogeneous_ball")
    op = S.CowlingOperator(P)
    tmin, rmin, tmax, rmax = S.lanczos_bounds(op, steps=60)
    w = sla.eigh(P.AG.toarray(), P.M.toarray(), eigvals_only=True)
    assert tmax <= w[-1] * (1 + 1e-12) and w[-1] <= tmax + rmax
    assert tmin >= w[0] - 1e-9


# ------------------------------------------------------------ eigen solutions
def test_inertia_count_matches_lapack():
    P = pencil("homogeneous_ball")
    A, M = P.AG.toarray(), P.M.toarray()
    w = sla.eigh(A, M, eigvals_only=True)
    for sig in (0.5, 10.0, 40.0):
        assert S.inertia_count(A, M, sig) == int((w < sig).sum())


@pytest.mark.parametrize("null", [False, True])
def test_filtered_lanczos_matches_dense(null):
    """C1 workload: lowest 30 eigenpairs in [0.5, 40], degree-40 filter."""
    P = pencil("homogeneous_ball")
    op = S.CowlingOperator(P)
    _, _, tmax, rmax = S.lanczos_bounds(op)
    lmax = (tmax + rmax) * 1.01
    mu, c, e = S.filter_coeffs(0.5, 40.0, 0.0, lmax, 40)
    kw = dict(null_shift=0.0, null_scale=40.0) if null else {}
    lam, X, res, steps = S.filtered_lanczos(op, 0.5, 40.0, 30, 1e-10, mu, c, e, **kw)
    A, M = P.AG.toarray(), P.M.toarray()
    w, Xd = S.dense_window(A, M, 0.5, 40.0)
    n_in = S.inertia_count(A, M, 40.0) - S.inertia_count(A, M, 0.5)
    assert len(w) == n_in and n_in >= 30
    assert np.all(np.abs(lam - w[:30]) <= 1e-10 * w[:30])
    assert res.max() <= 1e-10
    # eigenvectors: M-orthonormal and spanning the dense clusters
    np.testing.assert_allclose(X.T @ M @ X, np.eye(30), atol=1e-9)
    # six rigid modes below the window
    assert S.inertia_count(A, M, 1e-6) - S.inertia_count(A, M, -1e-6) == 6


# -------------------------------------------------------- closed-form spectra
def _toroidal_roots(l, count):
    f = lambda x: (l - 1) * ss.spherical_jn(l, x) - x * ss.spherical_jn(l + 1, x)
    xs = np.linspace(0.5, 12, 4000)
    v = f(xs)
    roots = [so.brentq(f, xs[i], xs[i + 1]) for i in range(len(xs) - 1) if v[i] * v[i + 1] < 0]
    return roots[:count]


def test_paper_1d_values_are_the_toroidal_closed_form():
    """The paper's printed 1-D values for the homogeneous ball are the roots
    of (l-1) j_l(x) - x j_{l+1}(x) = 0 scaled by V_S / (2 pi a)."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "toroidal_1d_paper.txt"))
            if l.strip() and not l.startswith("#")]
    beta, a = 5.7735, 6371.0
    for name, l, n, fm in rows:
        x = _toroidal_roots(int(l), 1)[int(n)]
        f = x * beta / (2 * math.pi * a) * 1e3
        assert abs(f - float(fm)) < 6e-5


@pytest.mark.slow
def test_homogeneous_ball_converges_to_closed_forms():
    """rho = lambda = mu = 1 ball: the 0T2 and 0T3 multiplets and the radial
    mode 0S0 (tan x = 4x/(4 - 3x^2), omega = sqrt(3) x) converge under
    refinement, faster for P2 than P1.  Straight-sided tetrahedra make the
    geometric error of the polyhedral ball O(h^2), which dominates here."""
    x2, x3 = _toroidal_roots(2, 1)[0], _toroidal_roots(3, 1)[0]
    g = lambda x: math.tan(x) - 4 * x / (4 - 3 * x * x)
    x0 = so.brentq(g, 2.3, 2.8)
    exact = {"T2": x2 ** 2, "T3": x3 ** 2, "S0": 3 * x0 ** 2}
    errs = {}
    for order, nh in ((1, 4), (2, 3), (2, 4)):
        P = pencil("homogeneous_ball", order=order, n_half=nh)
        w = spla.eigsh(P.AG.tocsc(), k=60, M=P.M.tocsc(), sigma=3.0, which="LM",
                       return_eigenvectors=False)
        w = np.sort(w)
        w = w[w > 1.0]
        e = {}
        e["T2"] = abs(w[:5].mean() - exact["T2"]) / exact["T2"]
        i0 = np.argmin(np.abs(w - exact["S0"]))
        e["S0"] = abs(w[i0] - exact["S0"]) / exact["S0"]
        near = np.sort(w[np.argsort(np.abs(w - exact["T3"]))[:7]])
        e["T3"] = abs(near.mean() - exact["T3"]) / exact["T3"]
        errs[(order, nh)] = e
    for k in ("T2", "T3", "S0"):
        assert errs[(2, 4)][k] < errs[(2, 3)][k] < 0.05
        assert errs[(2, 4)][k] < 0.02
        assert errs[(2, 4)][k] < errs[(1, 4)][k]


def test_cowling_window_equals_dense_solve():
    """The window-complete shift-invert reference (several shifts, exact
    Schur complement) finds exactly the dense generalised eigenvalues of the
    Cowling pencil in the window, with M-orthonormal vectors, on a small
    three-layer planet; pieces straddle clusters without losing or doubling
    any eigenvalue."""
    import planetgen as pg
    from oracle.assemble import Pencil
    P = Pencil(pg.three_layer_planet(n_half=4, order=1, pres_order=1))
    A, M = P.cowling_dense(), P.M.toarray()
    wd, _ = S.dense_window(A, M, 1.0, 60.0)
    for pieces in (1, 4):
        w, X = S.cowling_window(P, 1.0, 60.0, pieces=pieces, k0=16)
        assert len(w) == len(wd) > 100
        assert np.abs(w - wd).max() <= 1e-11 * wd.max()
        assert np.abs(X.T @ (P.M @ X) - np.eye(len(w))).max() < 1e-10
        R = A @ X - (M @ X) * w
        assert (np.linalg.norm(R, axis=0) / (w * np.linalg.norm(M @ X, axis=0))).max() < 1e-10
