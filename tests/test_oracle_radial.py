"""Pins of the radial (1-D) oracle of Appendix B (eq. "1Dform"), and the 3-D
oracle's convergence to it on the layered planet."""
import math
import os

import numpy as np
import pytest
import scipy.optimize as so
import scipy.special as ss

import planetgen as pg
from oracle import radial as RD

HERE = os.path.dirname(os.path.abspath(__file__))


def _roots(f, lo, hi, count, n=20000):
    xs = np.linspace(lo, hi, n)
    v = f(xs)
    return np.array([so.brentq(f, xs[i], xs[i + 1]) for i in range(n - 1) if v[i] * v[i + 1] < 0][:count])


def _djn(l, x, d):
    """d-th derivative of the spherical Bessel function j_l (the second from
    Bessel's equation)."""
    if d < 2:
        return ss.spherical_jn(l, x, derivative=bool(d))
    return -2.0 / x * ss.spherical_jn(l, x, True) - (1.0 - l * (l + 1) / x ** 2) * ss.spherical_jn(l, x)


def _lamb_determinant(l, w, rho, lam, mu, R=1.0):
    """Traction-free homogeneous elastic ball: u = grad(phi) + curl curl(x psi)
    with phi = j_l(a r) Y, psi = j_l(b r) Y (a = w/V_P, b = w/V_S) gives, in
    the U, V (V along k^{-1} grad_1 Y) normalisation,
      U = A a j_l'(ar) + B k^2 j_l(br)/r,
      V = A k j_l(ar)/r + B k (j_l(br) + br j_l'(br))/r;
    the radial and tangential tractions at r = R,
      (lam + 2 mu) U' + lam (2U - kV)/r  and  mu (V' - V/r + kU/r),
    vanish for a nonzero (A, B): their 2 x 2 determinant (l = 0: the radial
    traction of the A term)."""
    a, b, r = w * math.sqrt(rho / (lam + 2 * mu)), w * math.sqrt(rho / mu), R
    k = math.sqrt(l * (l + 1.0))
    J = lambda x, d=0: _djn(l, x, d)
    U = [a * J(a * r, 1), k * k * J(b * r) / r]
    V = [k * J(a * r) / r, k * (J(b * r) + b * r * J(b * r, 1)) / r]
    dU = [a * a * J(a * r, 2), k * k * (b * J(b * r, 1) / r - J(b * r) / r ** 2)]
    dV = [k * (a * J(a * r, 1) / r - J(a * r) / r ** 2),
          k * ((2 * b * J(b * r, 1) + b * b * r * J(b * r, 2)) / r - (J(b * r) + b * r * J(b * r, 1)) / r ** 2)]
    tr = [(lam + 2 * mu) * dU[j] + lam * (2 * U[j] - k * V[j]) / r for j in range(2)]
    tt = [mu * (dV[j] - V[j] / r + k * U[j] / r) for j in range(2)]
    return tr[0] if l == 0 else tr[0] * tt[1] - tr[1] * tt[0]


def test_toroidal_ball_closed_form():
    """Homogeneous ball: toroidal omega R / V_S are the roots of
    (l - 1) j_l(x) - x j_{l+1}(x) = 0 (traction-free surface)."""
    ball = [RD.Layer(0, 1, 1.0, math.sqrt(3.0), 1.0, False)]
    for l in (1, 2, 5):
        x = _roots(lambda x: (l - 1) * ss.spherical_jn(l, x) - x * ss.spherical_jn(l + 1, x), 0.5, 30.0, 3)
        w = RD.toroidal(ball, l, nel=20, p=3)
        w = w[w > 1e-8][:3]
        assert np.abs(w - x ** 2).max() <= 2e-6 * x[-1] ** 2, (l, w, x ** 2)


@pytest.mark.parametrize("l", [0, 1, 2, 3, 6])
def test_spheroidal_elastic_ball_closed_form(l):
    """Homogeneous elastic ball without gravity (rho 1.3, lambda 2, mu 0.7):
    the four lowest spheroidal omega^2 of degree l are the roots of the
    traction determinant; P3 elements, error falling with refinement."""
    rho, lam, mu = 1.3, 2.0, 0.7
    ex = _roots(lambda w: _lamb_determinant(l, w, rho, lam, mu), 0.05, 30.0, 4, n=30000) ** 2
    ball = [RD.Layer(0, 1, rho, math.sqrt((lam + 2 * mu) / rho), math.sqrt(mu / rho), False)]
    errs = []
    for nel in (10, 20):
        w = RD.Spheroidal(ball, l, nel=nel, p=3, gravity="none").eigenvalues(1e-8, 1e9)[:4]
        errs.append(np.abs(w - ex).max() / ex.max())
    assert errs[1] <= 1e-5 and errs[1] < errs[0] / 8


@pytest.mark.parametrize("l", [0, 1, 2, 4])
def test_fluid_ball_closed_form(l):
    """A fluid ball is bounded by a rigid wall in this formulation (the
    pressure's boundary term only meets a solid): omega R / c are the roots
    of j_l'(x) = 0, c = sqrt(kappa / rho)."""
    c = 1.7
    x = _roots(lambda x: ss.spherical_jn(l, x, True), 0.1, 30.0, 3)
    fb = [RD.Layer(0, 1, 1.1, c, 0.0, True)]
    errs = []
    for nel in (10, 20):
        w = RD.Spheroidal(fb, l, nel=nel, p=3, gravity="none").eigenvalues(1e-6, 1e9)[:3]
        errs.append(np.abs(w - (c * x) ** 2).max() / (c * x[-1]) ** 2)
    assert errs[1] <= 2e-4 and errs[1] < errs[0] / 4


def test_translation_costs_no_energy():
    """A rigid translation (l = 1: U = 1, V = sqrt 2) of a self-gravitating
    planet in hydrostatic equilibrium has zero energy: with the buoyancy term
    and the incremental potential, A x = 0.  Exact (to rounding) for the
    homogeneous ball, whose g and potential are polynomials of the element
    order; for the solid-fluid-solid planet it falls to zero under
    refinement (every fluid, fluid-solid and gravity term takes part)."""
    ball = [RD.Layer(0, 1, 1.0, math.sqrt(3.0), 1.0, False)]
    sp_ = RD.Spheroidal(ball, 1, nel=10, p=3, gravity="full", buoyancy=True)
    A, x = sp_.operator(), sp_.translation()
    assert np.linalg.norm(A @ x) <= 1e-14 * np.linalg.norm(A, 2) * np.linalg.norm(x)
    lay = RD.layers_from(pg.three_layer_model())
    rel = []
    for nel in (10, 20, 40):
        sp_ = RD.Spheroidal(lay, 1, nel=nel, p=3, gravity="full", buoyancy=True)
        A, x = sp_.operator(), sp_.translation()
        rel.append(np.linalg.norm(A @ x) / (np.linalg.norm(A, 2) * np.linalg.norm(x)))
    assert rel[2] < rel[1] / 4 < rel[0] / 16 and rel[2] <= 1e-9
    # without the buoyancy term, or in the Cowling approximation, it is not a
    # zero mode: its Rayleigh quotient is of the order of the low eigenvalues
    for grav, buoy in (("full", False), ("cowling", True)):
        sp_ = RD.Spheroidal(lay, 1, nel=20, p=3, gravity=grav, buoyancy=buoy)
        A, x = sp_.operator(), sp_.translation()
        assert abs(x @ A @ x) / (x @ sp_.M @ x) > 0.01


def test_paper_1d_values_of_the_self_gravitating_ball():
    """The paper's printed 1-D frequencies of its homogeneous ball with
    self-gravitation (four digits) from the radial pencil with the Poisson
    blocks.  Nondimensional units: radius, density and time 1/sqrt(pi G rho)."""
    G, rho0, R = 6.674e-11, 5.51e3, 6371e3
    T = 1.0 / math.sqrt(math.pi * G * rho0)
    vn = lambda v: v * 1e3 * T / R
    ball = [RD.Layer(0, 1, 1.0, vn(10.0), vn(5.7735), False)]
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "spheroidal_1d_paper.txt"))
            if l.strip() and not l.startswith("#")]
    for name, l, n, fm in rows:
        l, n = int(l), int(n)
        w = RD.Spheroidal(ball, l, nel=20, p=3, gravity="full").eigenvalues(1e-6, 1e9)
        idx = n - 1 if l == 1 else n                  # l = 1: the translation (n = 0) has omega = 0
        f = math.sqrt(w[idx]) / (2 * math.pi * T) * 1e3
        assert abs(f - float(fm)) < 6e-5, (name, f, fm)
    # without self-gravitation 0S2 moves well away from the printed value
    w = RD.Spheroidal(ball, 2, nel=20, p=3, gravity="cowling").eigenvalues(1e-6, 1e9)
    assert abs(math.sqrt(w[0]) / (2 * math.pi * T) * 1e3 - 0.4087) > 5e-3


def _fixture(nh):
    return np.loadtxt(os.path.join(HERE, "golden", "cowling_window_nh%d.txt" % nh))


def test_3d_oracle_converges_to_radial():
    """The 3-D oracle's Cowling eigenvalues of the three-layer planet (stored
    windows at n_half 4 and 6, 2 % lateral density perturbation in the solid)
    against the radial oracle of the same layered profiles: the same number
    of eigenvalues in [1, 12] as the radial multiplets stand for, each
    multiplet within 6 % at n_half 6 and closer than at n_half 4."""
    lay = RD.layers_from(pg.three_layer_model())
    rows = RD.spectrum(lay, 1.0, 12.0, 10, nel=40, p=3, gravity="cowling")
    ms = RD.multiset(rows)
    errs = {}
    for nh in (4, 6):
        w = _fixture(nh)
        w = w[(w >= 1.0) & (w <= 12.0)]
        assert len(w) == len(ms), (nh, len(w), len(ms))
        errs[nh] = np.abs(w - ms) / ms
    assert errs[6].max() <= 0.06
    # per multiplet (sorted order groups them: the radial values are well separated here)
    start = 0
    for wr, l, kind in rows:
        m = int(2 * l + 1)
        e4 = errs[4][start:start + m].mean()
        e6 = errs[6][start:start + m].mean()
        assert e6 < 0.7 * e4, (wr, l, kind, e4, e6)
        start += m
