"""Self-gravitation as an N-body problem (oracle, FP64).

Test infrastructure only (see the package docstring).

Sec. 5 of the paper evaluates the gravitational potential of the planet, and
its perturbation by a displacement, as N-body sums over the elements:

* Reference field (Sec. 5.1): with the element masses m_k = rho_k |K_k| at
  the barycentres r_k, Phi0(x) = -G sum_k m_k / |x - r_k| and
  g(x) = -G sum_k m_k (x - r_k) / |x - r_k|^3 (the printed exponent 3/2 on
  the distance is read as 3, the field of a point mass).
* Incremental potential (Sec. 5.2, eqs. "ph1body0", "ph1surface0",
  "ph1body2", "ph1surface2"): the bodies are the tetrahedra, with charge
  q_k(u) = int_K div(rho_k u) dx = rho_k int_K div u dx, and the faces where
  the density jumps -- the outer surface, q_l(u) = int_E (nu . u)[rho]^+_-
  = -rho_k int_E nu . u (nu outward, vacuum outside), and the fluid-solid
  faces, q_l(u) = int_E (nu^{f->s} . u^s) rho^s + (nu^{s->f} . u^f) rho^f,
  each side with its own displacement and density.  The potential at body
  i is S_i(u) = G q_i / R_i + sum_{j != i} G q_j / |r_i - r_j| with the
  self-terms 1/R_k = mean over K of 1/|r_k - x| (eq. "k2local") and 1/R_l
  = mean over E of 1/|r_l - x| (eq. "l2local").
* The weak form (eqs. "phi1solid", "phi1fluidsolid") is
  -sum_i q_i(v) S_i(u): the matrix -C^T S C of eq. "eigfull", C the map
  u -> (q_i), S the matrix of the N-body sums.

Here C is a sparse matrix (bodies x displacement DOFs) and S a dense one,
for small meshes.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import refelem as re_
from .assemble import tet_geometry, FACES

G_NONDIM = 1.0 / math.pi


# ----------------------------------------------------------- self-terms
def _gauss_triangle(n):
    """Collapsed Gauss-Legendre rule on the unit right triangle: points
    (s, t) with s, t >= 0, s + t <= 1, weights summing to 1/2."""
    x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    u, v = np.meshgrid(x, x, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    s = u.ravel()
    t = (v * (1.0 - u)).ravel()
    ww = (wu * wv * (1.0 - u)).ravel()
    return s, t, ww


def triangle_mean_inv_dist_from_point(P, A, B, C):
    """Mean over the triangle ABC of 1/|x - P| for P in the triangle's plane
    (P inside): split at P into three triangles and integrate in polar
    coordinates about P, where each piece's radial integral is the distance
    to its far edge: int_theta d / cos(theta - theta0) dtheta."""
    def piece(P, X, Y):
        # triangle with apex P and far edge XY: d * [ln(sec + tan)] between the edge end angles
        e = Y - X
        L = np.linalg.norm(e)
        t = e / L
        foot = X + np.dot(P - X, t) * t
        d = np.linalg.norm(P - foot)
        if d < 1e-300:
            return 0.0
        s1 = np.dot(X - foot, t) / d
        s2 = np.dot(Y - foot, t) / d
        return d * (np.arcsinh(s2) - np.arcsinh(s1))
    area = 0.5 * np.linalg.norm(np.cross(B - A, C - A))
    tot = piece(P, A, B) + piece(P, B, C) + piece(P, C, A)
    return abs(tot) / area


def tet_mean_inv_dist_from_point(P, X, n=24):
    """Mean over the tetrahedron X[4] of 1/|x - P| for P inside: the
    tetrahedron is the union of the four cones from P over its faces, and
    over a cone of height h above face F, int 1/|x - P| dx = (h/2) int_F
    dA/|y - P| (radial coordinate from P); the face integrals, of a smooth
    integrand since h > 0, by a collapsed Gauss rule of n x n points."""
    s, t, w = _gauss_triangle(n)
    vol = abs(np.dot(X[1] - X[0], np.cross(X[2] - X[0], X[3] - X[0]))) / 6.0
    tot = 0.0
    for a, b, c in FACES:
        A, B, C = X[a], X[b], X[c]
        nrm = np.cross(B - A, C - A)
        area2 = np.linalg.norm(nrm)
        h = abs(np.dot(P - A, nrm)) / area2
        Y = A[None, :] + s[:, None] * (B - A)[None, :] + t[:, None] * (C - A)[None, :]
        f = 1.0 / np.linalg.norm(Y - P[None, :], axis=1)
        tot += 0.5 * h * area2 * np.dot(w, f)
    return tot / vol


# ----------------------------------------------------------- bodies and C
def outer_faces(tet):
    """Faces of exactly one tetrahedron: rows (tet, local face)."""
    keys = np.concatenate([np.sort(tet[:, list(f)], 1) for f in FACES])
    owner = np.concatenate([np.arange(len(tet))] * 4)
    lf = np.repeat(np.arange(4), len(tet))
    _, inv, cnt = np.unique(keys, axis=0, return_inverse=True, return_counts=True)
    one = cnt[inv.ravel()] == 1
    o = np.lexsort((lf[one], owner[one]))
    return np.stack([owner[one][o], lf[one][o]], 1)


class SelfGravity:
    """Bodies, the charge map C and the N-body matrix S of a planet and its
    displacement numbering (an oracle Pencil)."""

    def __init__(self, pencil, G=G_NONDIM):
        P = pencil
        pl = P.p
        nb = P.nb
        xyz = np.asarray(pl["xyz"], float)
        tet = np.asarray(pl["tet"], np.int64)
        region = np.asarray(pl["region"])
        rho = np.asarray(pl["rho"], float)
        order = P.order
        self.G = G
        n = P.n
        vol, Gr = tet_geometry(xyz, tet)
        T = len(tet)
        # --- tetrahedra: q_k = rho_k sum_a (int_K grad l_a) . u_a
        basis = re_.lagrange_basis(order, 4)
        nd = len(basis)
        mbar = np.array([[float(re_._simplex_int(re_._poly_dlam(p, k), 3)) for k in range(4)] for p in basis])
        gint = np.einsum("t,ak,tkj->taj", vol, mbar, Gr)          # int_K d_j l_a, [T, nd, 3]
        en = nb.elem_node
        rows = [np.repeat(np.arange(T), nd * 3)]
        cols = [(3 * en[:, :, None] + np.arange(3)[None, None, :]).ravel()]
        vals = [(rho[:, None, None] * gint).ravel()]
        bary = xyz[tet].mean(1)
        self.n_tet = T
        # --- faces: outer surface (solid side) and fluid-solid faces (both sides)
        fbasis = re_.lagrange_basis(order, 3)
        fint = np.array([float(re_._simplex_int(p, 2)) for p in fbasis])  # int_E l_a / |E|

        def face_data(t, f):
            a, b, c = FACES[f]
            X = xyz[tet[t]]
            nrm = np.cross(X[b] - X[a], X[c] - X[a])
            area = 0.5 * np.linalg.norm(nrm)
            nu = nrm / (2 * area)
            opp = [q for q in range(4) if q not in (a, b, c)][0]
            if np.dot(nu, X[a] - X[opp]) < 0:
                nu = -nu                                            # outward from tet t
            loc = nb.face_nodes(t, f, order, "u")
            return area, nu, en[t][loc], (X[a] + X[b] + X[c]) / 3.0

        fb = []  # (centre, vertices)
        row = T
        of = outer_faces(tet)
        for t, f in of:
            area, nu, nodes, cen = face_data(t, f)
            coef = -rho[t] * area * fint                            # [rho]^+_- = 0 - rho_t, nu outward
            rows.append(np.full(3 * len(nodes), row))
            cols.append((3 * nodes[:, None] + np.arange(3)[None, :]).ravel())
            vals.append((coef[:, None] * nu[None, :]).ravel())
            fb.append((cen, xyz[tet[t]][list(FACES[f])]))
            row += 1
        for st, sf, ft in nb.fs_faces:
            area, nu_s, nodes_s, cen = face_data(st, sf)             # nu_s: outward from the solid = s -> f
            # the fluid tetrahedron's face with the same vertices
            vs = set(tet[st][list(FACES[sf])])
            ff = [q for q, fc in enumerate(FACES) if set(tet[ft][list(fc)]) == vs][0]
            _, nu_f, nodes_f, _ = face_data(ft, ff)                # outward from the fluid = f -> s
            # the face nodes of both sides in a common order (by geometric node)
            gs = nb.geom[st][nb.face_nodes(st, sf, order, "u")]
            gf = nb.geom[ft][nb.face_nodes(ft, ff, order, "u")]
            perm = [int(np.nonzero(gf == g)[0][0]) for g in gs]
            nodes_f = nodes_f[perm]
            # (nu^{f->s} . u^s) rho^s + (nu^{s->f} . u^f) rho^f: nu^{f->s} = nu_f, nu^{s->f} = nu_s
            for nodes, nu, r in ((nodes_s, nu_f, rho[st]), (nodes_f, nu_s, rho[ft])):
                coef = r * area * fint
                rows.append(np.full(3 * len(nodes), row))
                cols.append((3 * nodes[:, None] + np.arange(3)[None, :]).ravel())
                vals.append((coef[:, None] * nu[None, :]).ravel())
            fb.append((cen, xyz[tet[st]][list(FACES[sf])]))
            row += 1
        self.n_face = row - T
        self.nb_ = row
        self.C = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(row, n))
        self.C.sum_duplicates()
        # --- body positions and self-terms
        self.pos = np.concatenate([bary, np.array([c for c, _ in fb]).reshape(-1, 3)])
        inv_r = np.empty(row)
        X = xyz[tet]
        for k in range(T):
            inv_r[k] = tet_mean_inv_dist_from_point(bary[k], X[k])
        for i, (cen, V3) in enumerate(fb):
            inv_r[T + i] = triangle_mean_inv_dist_from_point(cen, V3[0], V3[1], V3[2])
        self.inv_R = inv_r
        self.mass = rho * vol

    def S_dense(self):
        """G / |r_i - r_j| off the diagonal, G / R_i on it."""
        d = np.linalg.norm(self.pos[:, None, :] - self.pos[None, :, :], axis=2)
        np.fill_diagonal(d, 1.0)
        S = self.G / d
        np.fill_diagonal(S, self.G * self.inv_R)
        return S

    def potential(self, q):
        """S q by direct summation (rows of S one at a time: no dense matrix)."""
        out = np.empty_like(q)
        for i in range(len(q)):
            d = np.linalg.norm(self.pos - self.pos[i], axis=1)
            d[i] = 1.0
            w = self.G / d
            w[i] = self.G * self.inv_R[i]
            out[i] = w @ q
        return out

    def apply(self, U):
        """-C^T S C U (the self-gravitation term of eq. "eigfull")."""
        q = self.C @ U
        return -(self.C.T @ self.potential(q))

    def reference_field(self, x):
        """g at points x [P, 3] from the element masses at the barycentres."""
        bary = self.pos[:self.n_tet]
        d = x[:, None, :] - bary[None, :, :]
        r = np.linalg.norm(d, axis=2)
        return -self.G * np.einsum("k,pkj,pk->pj", self.mass, d, 1.0 / r ** 3)
