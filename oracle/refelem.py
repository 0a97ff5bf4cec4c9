"""Nodal Lagrange bases on simplices and their exact integrals (oracle).

Appendix A builds the element mass and derivative matrices from an
orthonormal modal basis and a Vandermonde matrix; the results are the exact
integrals of products of the nodal (Lagrange) basis functions and of their
derivatives.  This module computes those integrals directly, from the
barycentric form of the Lagrange basis and the simplex monomial formula

    int_K  prod_i lambda_i^{a_i} dx = |K| d! prod_i a_i! / (sum_i a_i + d)!,

in exact rational arithmetic.  Node sets: degree 1 -> the vertices; degree 2
-> vertices then edge midpoints (edges (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)
on a tetrahedron, (0,1),(0,2),(1,2) on a triangle).
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import factorial
import itertools

import numpy as np

TET_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))
TRI_EDGES = ((0, 1), (0, 2), (1, 2))


def _poly_mul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            k = tuple(x + y for x, y in zip(a, b))
            out[k] = out.get(k, 0) + ca * cb
    return out


def _poly_dlam(p, i):
    """Partial derivative with respect to barycentric coordinate i."""
    out = {}
    for a, c in p.items():
        if a[i]:
            k = list(a)
            k[i] -= 1
            k = tuple(k)
            out[k] = out.get(k, 0) + c * a[i]
    return out


def _simplex_int(p, d):
    """Integral over a d-simplex divided by its measure."""
    s = Fraction(0)
    for a, c in p.items():
        num = factorial(d)
        for x in a:
            num *= factorial(x)
        s += Fraction(c) * Fraction(num, factorial(sum(a) + d))
    return s


def _unit(nv, i, power=1):
    a = [0] * nv
    a[i] = power
    return tuple(a)


@lru_cache(None)
def lagrange_basis(order: int, nv: int):
    """Lagrange basis in barycentric form on a simplex with nv vertices."""
    edges = TET_EDGES if nv == 4 else TRI_EDGES
    if order == 1:
        return tuple({_unit(nv, i): Fraction(1)} for i in range(nv))
    if order == 2:
        basis = [{_unit(nv, i, 2): Fraction(2), _unit(nv, i): Fraction(-1)} for i in range(nv)]
        for i, j in edges:
            a = [0] * nv
            a[i] = a[j] = 1
            basis.append({tuple(a): Fraction(4)})
        return tuple(basis)
    raise ValueError("order must be 1 or 2")


def node_bary(order: int, nv: int):
    """Barycentric coordinates of the nodes, [Np, nv]."""
    edges = TET_EDGES if nv == 4 else TRI_EDGES
    pts = [np.eye(nv)[i] for i in range(nv)]
    if order == 2:
        pts += [(np.eye(nv)[i] + np.eye(nv)[j]) / 2 for i, j in edges]
    return np.array(pts)


@lru_cache(None)
def mass_exact(order_a: int, order_b: int, nv: int):
    """[Na, Nb] exact Fractions: int l^a_i l^b_j / |K|."""
    A, B = lagrange_basis(order_a, nv), lagrange_basis(order_b, nv)
    return tuple(tuple(_simplex_int(_poly_mul(p, q), nv - 1) for q in B) for p in A)


@lru_cache(None)
def dmass_exact(order_a: int, order_b: int, nv: int):
    """[Na, Nb, nv]: int (d l^a_i / d lambda_k) l^b_j / |K|."""
    A, B = lagrange_basis(order_a, nv), lagrange_basis(order_b, nv)
    return tuple(tuple(tuple(_simplex_int(_poly_mul(_poly_dlam(p, k), q), nv - 1)
                             for k in range(nv)) for q in B) for p in A)


@lru_cache(None)
def stiff_exact(order: int, nv: int):
    """[N, N, nv, nv]: int (d l_i / d lambda_k)(d l_j / d lambda_l) / |K|."""
    A = lagrange_basis(order, nv)
    return tuple(tuple(tuple(tuple(_simplex_int(_poly_mul(_poly_dlam(p, k), _poly_dlam(q, l)), nv - 1)
                                   for l in range(nv)) for k in range(nv)) for q in A) for p in A)


def as_float(t):
    return np.array(t, dtype=object).astype(np.float64)


def eval_basis(order: int, nv: int, bary):
    """Values of the basis at barycentric points [P, nv] -> [P, N]."""
    B = lagrange_basis(order, nv)
    out = np.zeros((bary.shape[0], len(B)))
    for n, p in enumerate(B):
        for a, c in p.items():
            out[:, n] += float(c) * np.prod(bary ** np.array(a), axis=1)
    return out
