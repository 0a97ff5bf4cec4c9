"""Pins of the oracle's self-gravitation (N-body) operators: self-terms
against closed forms and Monte Carlo, the charges against mass conservation
(divergence theorem), -C^T S C against symmetry and definiteness, and the
reference field of a homogeneous ball against (4/3) pi G rho r."""
import math

import numpy as np
import pytest

from conftest import planet
from oracle import selfgrav as SG
from oracle.assemble import Pencil


def _mc_mean_inv(P, sample, n=400000, seed=0):
    rng = np.random.default_rng(seed)
    x = sample(rng, n)
    return float(np.mean(1.0 / np.linalg.norm(x - P, axis=1)))


def test_triangle_self_term():
    """Equilateral triangle of side a, from its centroid: (4/a) ln(2 + sqrt 3)
    (three pieces, each 2 d asinh(sqrt 3), d = a / (2 sqrt 3)); a scalene
    triangle from its centroid agrees with Monte Carlo."""
    a = 0.37
    A, B, C = np.array([0, 0, 0.]), np.array([a, 0, 0.]), np.array([a / 2, a * math.sqrt(3) / 2, 0.])
    got = SG.triangle_mean_inv_dist_from_point((A + B + C) / 3, A, B, C)
    assert abs(got - 4.0 / a * math.log(2 + math.sqrt(3))) < 1e-12 * got
    A, B, C = np.array([0.1, -0.2, 0.3]), np.array([0.9, 0.1, 0.2]), np.array([0.3, 0.7, -0.4])
    P = (A + B + C) / 3

    def tri(rng, n):
        u, v = rng.random(n), rng.random(n)
        f = u + v > 1
        u[f], v[f] = 1 - u[f], 1 - v[f]
        return A + u[:, None] * (B - A) + v[:, None] * (C - A)
    got = SG.triangle_mean_inv_dist_from_point(P, A, B, C)
    assert abs(got - _mc_mean_inv(P, tri)) < 4e-3 * got


def test_tetrahedron_self_term():
    """Mean of 1/|x - r| over a tetrahedron from its barycentre: the cone
    decomposition agrees with Monte Carlo, and doubling the face rule changes
    nothing; it scales as 1 / size."""
    X = np.array([[0, 0, 0.], [1, 0, 0.], [0.2, 0.9, 0.], [0.3, 0.3, 0.8]])
    P = X.mean(0)

    def tet(rng, n):
        b = rng.dirichlet(np.ones(4), n)
        return b @ X
    got = SG.tet_mean_inv_dist_from_point(P, X)
    assert abs(got - SG.tet_mean_inv_dist_from_point(P, X, n=48)) < 1e-10 * got
    assert abs(got - _mc_mean_inv(P, tet, seed=2)) < 4e-3 * got
    assert abs(SG.tet_mean_inv_dist_from_point(0.5 * P, 0.5 * X) - 2 * got) < 1e-12 * got


def _layered_constant(n_half, order=2):
    """The three-layer planet with one density per layer, so that the density
    jumps only across the fluid-solid interfaces and the surface."""
    d = dict(planet("three_layer_planet", n_half=n_half, order=order, pres_order=1))
    x = np.asarray(d["xyz"])[np.asarray(d["tet"])].mean(1)
    r = np.linalg.norm(x, axis=1)
    d["rho"] = np.where(r < 0.19, 2.3, np.where(r < 0.55, 2.0, 0.8))
    return d


@pytest.mark.parametrize("case", ["ball", "layered"])
def test_charges_conserve_mass(case):
    """With a density constant per layer the charges of any displacement sum
    to zero: int div(rho u) over the layers is cancelled by the surface and
    fluid-solid face terms (divergence theorem, exact for the discrete u)."""
    d = planet("homogeneous_ball", n_half=3, order=2) if case == "ball" else _layered_constant(3)
    P = Pencil(d)
    S = SG.SelfGravity(P)
    col = np.asarray(S.C.sum(axis=0)).ravel()
    assert np.abs(col).max() <= 1e-13 * np.abs(S.C).max()
    assert S.n_face > 0 and (case == "ball" or len(P.nb.fs_faces) > 0)


def test_operator_symmetric():
    """-C^T S C is symmetric and apply() (row-by-row direct sums) equals the
    dense form.  (S itself is symmetric but not definite: a surface face's
    barycentre sits a quarter height above the barycentre of its
    tetrahedron, closer than the two bodies' self-term radii, so the
    point-charge discretisation has a few small negative eigenvalues.)"""
    d = _layered_constant(3, order=1)
    P = Pencil(d)
    S = SG.SelfGravity(P)
    Sd = S.S_dense()
    assert np.abs(Sd - Sd.T).max() == 0.0
    Cd = S.C.toarray()
    K = -Cd.T @ Sd @ Cd
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    U = np.random.default_rng(1).standard_normal((P.n, 3))
    assert np.abs(S.apply(U) - K @ U).max() <= 1e-12 * np.abs(K @ U).max()


def test_reference_field_of_homogeneous_ball():
    """g from element masses (at mesh vertices, the paper's targets): far away
    it is -G M x / |x|^3 (M the exact mesh mass); at interior vertices it
    approaches -(4/3) pi G rho x, the mean error falling with refinement."""
    errs = []
    for nh in (3, 6):
        d = planet("homogeneous_ball", n_half=nh, order=1)
        S = SG.SelfGravity(Pencil(d))
        M = S.mass.sum()
        far = np.array([[10.0, 3.0, -4.0]])
        g = S.reference_field(far)[0]
        ex = -S.G * M * far[0] / np.linalg.norm(far[0]) ** 3
        assert np.linalg.norm(g - ex) <= 1e-4 * np.linalg.norm(ex)
        x = np.asarray(d["xyz"])
        r = np.linalg.norm(x, axis=1)
        pts = x[(r > 0.3) & (r < 0.7)]
        g = S.reference_field(pts)
        ex = -(4.0 / 3.0) * math.pi * S.G * 1.0 * pts
        errs.append(float(np.mean(np.linalg.norm(g - ex, axis=1) / np.linalg.norm(ex, axis=1))))
    assert errs[1] < 0.75 * errs[0] and errs[1] < 0.05, errs
