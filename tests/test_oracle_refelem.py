"""Pins of the oracle's reference-element integrals (Appendix A)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import refelem as R

HERE = os.path.dirname(__file__)


def _golden_masses():
    out, name, scale, rows = {}, None, None, []
    for line in open(os.path.join(HERE, "golden", "reference_mass.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0].startswith("p"):
            if name:
                out[name] = np.array(rows, float) / scale
            name, scale, rows = tok[0], float(tok[1]), []
        else:
            rows.append([float(t) for t in tok])
    out[name] = np.array(rows, float) / scale
    return out


@pytest.mark.parametrize("name,order,nv", [("p1_tet", 1, 4), ("p2_tet", 2, 4),
                                           ("p1_tri", 1, 3), ("p2_tri", 2, 3)])
def test_mass_matches_closed_form(name, order, nv):
    M = R.as_float(R.mass_exact(order, order, nv))
    np.testing.assert_allclose(M, _golden_masses()[name], rtol=0, atol=1e-15)


def test_lagrange_property_and_partition_of_unity():
    for nv in (3, 4):
        for order in (1, 2):
            nodes = R.node_bary(order, nv)
            V = R.eval_basis(order, nv, nodes)
            np.testing.assert_allclose(V, np.eye(len(nodes)), atol=1e-15)
            rng = np.random.default_rng(0)
            b = rng.dirichlet(np.ones(nv), 50)
            np.testing.assert_allclose(R.eval_basis(order, nv, b).sum(1), 1.0, atol=1e-14)


def test_basis_integrals():
    # int of a P2 vertex function is -|K|/20, of an edge function |K|/5 (tet)
    one = {(0, 0, 0, 0): Fraction(1)}
    B = R.lagrange_basis(2, 4)
    ints = [R._simplex_int(R._poly_mul(p, one), 3) for p in B]
    assert ints[:4] == [Fraction(-1, 20)] * 4
    assert ints[4:] == [Fraction(1, 5)] * 6


def _tet_physical():
    X = np.array([[0.1, 0.0, -0.2], [1.3, 0.2, 0.1], [0.2, 0.9, 0.0], [0.3, 0.1, 1.1]])
    Tm = (X[1:] - X[0]).T
    inv = np.linalg.inv(Tm)
    G = np.vstack([-inv.sum(0), inv])
    vol = np.linalg.det(Tm) / 6
    return X, G, vol


def _nodes_xyz(X, order):
    bary = R.node_bary(order, 4)
    return bary @ X


def test_derivative_integrals_exact_on_quadratics():
    """int grad u . grad w over a physical tet for quadratic u, w equals the
    value from a direct cubature (degree-2 integrand, Keast 4-point rule is
    exact for degree 2)."""
    X, G, vol = _tet_physical()
    KK = R.as_float(R.stiff_exact(2, 4))
    S = np.einsum("km,ln,abkl->abmn", G, G, KK) * vol
    xn = _nodes_xyz(X, 2)
    u = lambda x: x[:, 0] ** 2 + 0.5 * x[:, 0] * x[:, 1] - x[:, 2]
    gu = lambda x: np.stack([2 * x[:, 0] + 0.5 * x[:, 1], 0.5 * x[:, 0], -np.ones(len(x))], 1)
    w = lambda x: x[:, 1] * x[:, 2] + 2 * x[:, 0]
    gw = lambda x: np.stack([2 * np.ones(len(x)), x[:, 2], x[:, 1]], 1)
    val = np.einsum("a,abmm,b->", u(xn), S, w(xn))
    a, b = 0.5854101966249685, 0.1381966011250105
    bary = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
    q = bary @ X
    ref = vol * np.mean(np.einsum("pi,pi->p", gu(q), gw(q)))
    assert abs(val - ref) < 1e-12 * abs(ref)


def test_dmass_matches_cubature():
    """int (d_m l_a) l_c: contract with nodal values of a quadratic u and a
    quadratic w and compare with a degree-3 cubature of (d_m u) w."""
    X, G, vol = _tet_physical()
    DM = R.as_float(R.dmass_exact(2, 2, 4))
    P = np.einsum("km,ack->acm", G, DM) * vol
    xn = _nodes_xyz(X, 2)
    u = lambda x: x[:, 0] * x[:, 1] + x[:, 2] ** 2
    du0 = lambda x: x[:, 1]
    w = lambda x: 1 + x[:, 0] - x[:, 1] * x[:, 2]
    val = np.einsum("a,ac,c->", u(xn), P[:, :, 0], w(xn))
    # Keast degree-3 rule (5 points)
    pts = np.array([[0.25] * 4, [0.5, 1 / 6, 1 / 6, 1 / 6], [1 / 6, 0.5, 1 / 6, 1 / 6],
                    [1 / 6, 1 / 6, 0.5, 1 / 6], [1 / 6, 1 / 6, 1 / 6, 0.5]])
    wts = np.array([-0.8, 0.45, 0.45, 0.45, 0.45])
    q = pts @ X
    ref = vol * np.sum(wts * du0(q) * w(q))
    assert abs(val - ref) < 1e-12 * max(1.0, abs(ref))
