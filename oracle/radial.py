"""Spherically symmetric planets by a radial (1-D) finite-element method
(oracle, FP64).

Test infrastructure only (see the package docstring).

Appendix B reduces the weak forms of Sec. 4 to one radial coordinate: for a
spherically symmetric planet the displacement of one spherical-harmonic
degree l separates as

    spheroidal  u = U(r) Y r_hat + V(r) k^{-1} grad_1 Y,    k = sqrt(l(l+1)),
    toroidal    u = W(r) k^{-1} (-r_hat x grad_1 Y),

(grad_1 the gradient on the unit sphere), the pressure as P(r) Y and the
incremental potential as S(r) Y, and eq. "1Dform" is the resulting pencil
(A_G + E_G K_p^{-1} E_G^T - C^T S^{-1} C, M) with every block a 1-D integral
(Tables "radialresults" and "radialresults1").  This module discretises it
with continuous Lagrange elements of order p on each solid or fluid region
(pressure of order p - 1, potential of order p on the whole ball).

Forms, integrated over the unit sphere (r^2 dr is the radial measure, g the
magnitude of the reference gravity, g' = -g r_hat, dg = dg/dr):

* elasticity (the standard isotropic form):
    lambda E1(v) E1(u) + 2 mu r^2 U_v' U_u' + mu E3(v) E3(u)
    + 2 mu [2 U_v U_u - k (U_v V_u + V_v U_u) + (k^2 - 1) V_v V_u]
  with E1 = r U' + 2U - kV (r times the divergence) and E3 = r V' - V + kU;
* the symmetrised solid gravity terms of Sec. 4 (those the 3-D assembly
  uses, g' = -grad Phi0), reduced by the same separation:
    rho [(dg r^2 - 2 g r) U_v U_u + g k r (U_v V_u + V_v U_u)];
* on a fluid-solid boundary, the solid's face term S{(v.g')(nu.u)[rho]^f}:
    -(nu.r_hat) g rho_f r^2 U_v U_u   (nu the solid's outward normal);
* the fluid blocks: K_p = int P' P / kappa r^2 dr, A_dg = int U_v (P' + rho g
  P / kappa) r^2 + k V_v P r dr, E_FS = (nu.r_hat) U_v^s P r^2 at each
  fluid-solid boundary point; the buoyancy block A_f = int N^2 rho U_v U_u
  r^2 dr with N^2 = -g (rho'/rho + rho g / kappa) is included on request
  (the 3-D assembly takes N^2 = 0);
* self-gravitation (eq. "1Dform" with the Poisson blocks of Table
  "radialresults1"): C = int rho (S' U r^2 + k S V r) dr,
  S = (4 pi G)^{-1} [int (S'_v S'_u r^2 + k^2 S_v S_u) dr + (l + 1) R S_v(R) S_u(R)],
  the last term being the exterior integral over r > R, where the potential
  decays as r^{-(l+1)} (the special treatment the paper refers to).
* mass: rho (U_v U_u + V_v V_u) r^2, and rho W_v W_u r^2 for toroidal modes;
  toroidal energy mu [(r W_v' - W_v)(r W_u' - W_u) + (k^2 - 2) W_v W_u].

The reduction of the gravity and self-gravitation terms is pinned by the
tests: a translated self-gravitating planet costs no energy (l = 1), the
paper's printed 1-D values of its homogeneous ball, closed forms for the
homogeneous elastic ball (spheroidal and toroidal) and for a fluid ball.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

G_NONDIM = 1.0 / math.pi


# ----------------------------------------------------------------- the model
class Layer:
    """One layer r0 < r < r1 with polynomial profiles (numpy Polynomial in r)
    of density, V_P and V_S, solid or fluid."""

    def __init__(self, r0, r1, rho, vp, vs, fluid):
        P = np.polynomial.Polynomial
        self.r0, self.r1 = float(r0), float(r1)
        self.rho = rho if isinstance(rho, P) else P(np.atleast_1d(rho))
        self.vp = vp if isinstance(vp, P) else P(np.atleast_1d(vp))
        self.vs = vs if isinstance(vs, P) else P(np.atleast_1d(vs))
        self.fluid = bool(fluid)

    def kappa(self, r):
        mu = 0.0 if self.fluid else self.rho(r) * self.vs(r) ** 2
        return self.rho(r) * self.vp(r) ** 2 - 4.0 * mu / 3.0

    def lam_mu(self, r):
        mu = np.zeros_like(r) if self.fluid else self.rho(r) * self.vs(r) ** 2
        return self.rho(r) * self.vp(r) ** 2 - 2.0 * mu, mu


def layers_from(model):
    """Layers of a planet-generator RadialModel (outer radii, profiles, fluid flags)."""
    out, r0 = [], 0.0
    for i, r1 in enumerate(model.radii):
        out.append(Layer(r0, r1, model.rho[i], model.vp[i], model.vs[i], model.fluid[i]))
        r0 = r1
    return out


class Gravity:
    """g(r) = G m(r) / r^2 with m(r) = 4 pi int_0^r rho s^2 ds (exact for
    polynomial densities), and dg/dr = 4 pi G rho - 2 g / r."""

    def __init__(self, layers, G):
        self.layers, self.G = layers, G
        self.prim, acc = [], 0.0
        s2 = np.polynomial.Polynomial([0, 0, 1])
        for L in layers:
            Pm = (L.rho * s2).integ()
            self.prim.append((Pm, acc - Pm(L.r0)))
            acc += Pm(L.r1) - Pm(L.r0)

    def g(self, r, i):
        Pm, off = self.prim[i]
        m = 4.0 * math.pi * (Pm(r) + off)
        return self.G * m / r ** 2

    def dg(self, r, i):
        return 4.0 * math.pi * self.G * self.layers[i].rho(r) - 2.0 * self.g(r, i) / r


# ----------------------------------------------------------- 1-D elements
def _lagrange(p, x):
    """Values and derivatives of the p + 1 equispaced Lagrange polynomials on
    [0, 1] at points x: arrays [len(x), p + 1]."""
    nodes = np.linspace(0.0, 1.0, p + 1)
    V = np.vander(nodes, p + 1, increasing=True)
    C = np.linalg.inv(V)                         # column j: coefficients of l_j
    X = np.vander(x, p + 1, increasing=True)
    dX = np.zeros_like(X)
    dX[:, 1:] = X[:, :-1] * np.arange(1, p + 1)
    return X @ C, dX @ C


class Mesh1D:
    """Elements of each layer (nel per layer, or nel scaled by thickness),
    grouped in regions: maximal runs of layers of one kind.  Nodes are
    continuous within a region; the potential's nodes are continuous over
    the whole ball."""

    def __init__(self, layers, nel, p, nq=None):
        self.layers, self.p = layers, p
        R = layers[-1].r1
        self.R = R
        self.elems = []                          # (layer index, a, b)
        for i, L in enumerate(layers):
            ne = max(1, int(round(nel * (L.r1 - L.r0) / R)))
            e = np.linspace(L.r0, L.r1, ne + 1)
            self.elems += [(i, e[j], e[j + 1]) for j in range(ne)]
        # regions
        self.region = []
        reg = -1
        for q, (i, a, b) in enumerate(self.elems):
            if q == 0 or layers[i].fluid != layers[self.elems[q - 1][0]].fluid:
                reg += 1
            self.region.append(reg)
        self.n_region = reg + 1
        self.region_fluid = [layers[self.elems[self.region.index(g)][0]].fluid for g in range(self.n_region)]
        nq = nq or (p + 8)
        xg, wg = np.polynomial.legendre.leggauss(nq)
        self.xq, self.wq = 0.5 * (xg + 1.0), 0.5 * wg

    def region_nodes(self, order, fluid=None):
        """Per element: global node indices of an order-`order` continuous field
        living on the regions of the given kind (all regions if fluid is None);
        elements outside get None.  Returns (list, node count)."""
        out, nxt, prev_reg, last = [], 0, None, None
        for q, (i, a, b) in enumerate(self.elems):
            g = self.region[q]
            if fluid is not None and self.region_fluid[g] != fluid:
                out.append(None)
                prev_reg = None
                continue
            if fluid is not None and g != prev_reg:
                start = nxt                      # a new region: fresh first node
                nxt += 1
            elif q == 0 or prev_reg is None:
                start = nxt
                nxt += 1
            else:
                start = last
            ids = [start] + list(range(nxt, nxt + order))
            nxt += order
            last = ids[-1]
            out.append(np.array(ids))
            prev_reg = g
        return out, nxt


def _fs_points(mesh):
    """Fluid-solid boundary points: (radius, solid element's end node side,
    index of the solid element, index of the fluid element, nu.r_hat) with
    nu the solid's outward normal (+1 when the solid lies inside)."""
    pts = []
    for q in range(len(mesh.elems) - 1):
        g0, g1 = mesh.region[q], mesh.region[q + 1]
        if g0 != g1:
            r = mesh.elems[q][2]
            if mesh.region_fluid[g0]:            # fluid inside, solid outside
                pts.append((r, q + 1, "first", q, "last", -1.0))
            else:                                # solid inside, fluid outside
                pts.append((r, q, "last", q + 1, "first", +1.0))
    return pts


# ------------------------------------------------------------ spheroidal
class Spheroidal:
    """Assembled blocks of eq. "1Dform" for degree l.

    gravity: "none", "cowling" (the reference-gravity terms) or "full"
    (plus the incremental potential).  buoyancy: include A_f.
    DOF layout of u: per node of the solid field [U, V], then per node of the
    fluid field [U, V] (U only for l = 0)."""

    def __init__(self, layers, l, nel=40, p=3, gravity="cowling", buoyancy=False, G=G_NONDIM):
        self.layers, self.l, self.p = layers, int(l), p
        k = math.sqrt(l * (l + 1.0))
        self.k = k
        mesh = Mesh1D(layers, nel, p)
        self.mesh = mesh
        grav = Gravity(layers, G)
        nc = 1 if l == 0 else 2                  # components per node
        sn, ns = mesh.region_nodes(p, fluid=False)
        fn, nf = mesh.region_nodes(p, fluid=True)
        pn, npp = mesh.region_nodes(max(1, p - 1), fluid=True)
        gn, ng = mesh.region_nodes(p, fluid=None)
        n = nc * (ns + nf)
        self.n, self.n_p, self.n_s = n, npp, ng
        A = np.zeros((n, n))
        Mm = np.zeros((n, n))
        Af = np.zeros((n, n))
        E = np.zeros((n, npp))
        Kp = np.zeros((npp, npp))
        Cm = np.zeros((ng, n))
        Sm = np.zeros((ng, ng))
        fourpiG = 4.0 * math.pi * G
        use_g = gravity in ("cowling", "full")

        def dofs(nodes, off):
            # [U dofs], [V dofs]
            U = off + nc * nodes
            Vd = U + 1 if nc == 2 else None
            return U, Vd

        for q, (i, a, b) in enumerate(mesh.elems):
            L = layers[i]
            h = b - a
            r = a + h * mesh.xq
            w = h * mesh.wq
            phi, dphi = _lagrange(p, mesh.xq)
            dphi = dphi / h
            rho = L.rho(r)
            g = grav.g(r, i) if use_g else np.zeros_like(r)
            dg = grav.dg(r, i) if use_g else np.zeros_like(r)
            if L.fluid:
                U, Vd = dofs(fn[q], nc * ns)
            else:
                U, Vd = dofs(sn[q], 0)
            # mass
            mloc = np.einsum("q,qa,qb->ab", w * rho * r * r, phi, phi)
            A_ix = np.ix_
            Mm[A_ix(U, U)] += mloc
            if Vd is not None:
                Mm[A_ix(Vd, Vd)] += mloc
            if not L.fluid:
                lam, mu = L.lam_mu(r)
                # E1 = r U' + 2 U - k V ; E3 = r V' - V + k U  as [q, dof] on (U, V)
                E1u = r[:, None] * dphi + 2.0 * phi
                E1v = -k * phi
                E3u = k * phi
                E3v = r[:, None] * dphi - phi
                blocks = {}
                blocks["UU"] = (np.einsum("q,qa,qb->ab", w * lam, E1u, E1u)
                                + np.einsum("q,qa,qb->ab", w * 2 * mu * r * r, dphi, dphi)
                                + np.einsum("q,qa,qb->ab", w * mu, E3u, E3u)
                                + np.einsum("q,qa,qb->ab", w * 4 * mu, phi, phi))
                if Vd is not None:
                    blocks["UV"] = (np.einsum("q,qa,qb->ab", w * lam, E1u, E1v)
                                    + np.einsum("q,qa,qb->ab", w * mu, E3u, E3v)
                                    - np.einsum("q,qa,qb->ab", w * 2 * mu * k, phi, phi))
                    blocks["VV"] = (np.einsum("q,qa,qb->ab", w * lam, E1v, E1v)
                                    + np.einsum("q,qa,qb->ab", w * mu, E3v, E3v)
                                    + np.einsum("q,qa,qb->ab", w * 2 * mu * (k * k - 1), phi, phi))
                if use_g:
                    blocks["UU"] = blocks["UU"] + np.einsum("q,qa,qb->ab", w * rho * (dg * r * r - 2 * g * r), phi, phi)
                    if Vd is not None:
                        blocks["UV"] = blocks["UV"] + np.einsum("q,qa,qb->ab", w * rho * g * k * r, phi, phi)
                A[A_ix(U, U)] += blocks["UU"]
                if Vd is not None:
                    A[A_ix(U, Vd)] += blocks["UV"]
                    A[A_ix(Vd, U)] += blocks["UV"].T
                    A[A_ix(Vd, Vd)] += blocks["VV"]
            else:
                kap = L.kappa(r)
                pp = max(1, p - 1)
                psi, dpsi = _lagrange(pp, mesh.xq)
                dpsi = dpsi / h
                P = pn[q]
                Kp[A_ix(P, P)] += np.einsum("q,qa,qb->ab", w * r * r / kap, psi, psi)
                E[A_ix(U, P)] += (np.einsum("q,qa,qc->ac", w * r * r, phi, dpsi)
                                  + np.einsum("q,qa,qc->ac", w * rho * g * r * r / kap, phi, psi))
                if Vd is not None:
                    E[A_ix(Vd, P)] += np.einsum("q,qa,qc->ac", w * k * r, phi, psi)
                if buoyancy and use_g:
                    drho = L.rho.deriv()(r)
                    N2 = -g * (drho / rho + rho * g / kap)
                    Af[A_ix(U, U)] += np.einsum("q,qa,qb->ab", w * N2 * rho * r * r, phi, phi)
            if gravity == "full":
                Sn = gn[q]
                Sm[A_ix(Sn, Sn)] += (np.einsum("q,qa,qb->ab", w * r * r, dphi, dphi)
                                     + np.einsum("q,qa,qb->ab", w * k * k, phi, phi)) / fourpiG
                Cm[A_ix(Sn, U)] += np.einsum("q,qa,qb->ab", w * rho * r * r, dphi, phi)
                if Vd is not None:
                    Cm[A_ix(Sn, Vd)] += np.einsum("q,qa,qb->ab", w * rho * k * r, phi, phi)
        # fluid-solid boundary points
        for (rb, qs, ss, qf, sf_, nur) in _fs_points(mesh):
            s_node = sn[qs][0 if ss == "first" else -1]
            p_node = pn[qf][0 if sf_ == "first" else -1]
            Us = nc * s_node
            E[Us, p_node] += nur * rb * rb
            if use_g:
                # density of the fluid side at rb and g there (continuous in r)
                Lf = layers[mesh.elems[qf][0]]
                gi = mesh.elems[qs][0]
                A[Us, Us] += -nur * grav.g(rb, gi) * Lf.rho(rb) * rb * rb
        # buoyancy jumps at fluid-fluid layer interfaces: [rho]^+_- g U_v U_u r^2
        if buoyancy and use_g:
            for q in range(len(mesh.elems) - 1):
                i0, i1 = mesh.elems[q][0], mesh.elems[q + 1][0]
                if i0 != i1 and layers[i0].fluid and layers[i1].fluid:
                    rb = mesh.elems[q][2]
                    u = nc * ns + nc * fn[q][-1]
                    A[u, u] += (layers[i1].rho(rb) - layers[i0].rho(rb)) * grav.g(rb, i0) * rb * rb
        if gravity == "full":
            last = gn[len(mesh.elems) - 1][-1]
            Sm[last, last] += (l + 1) * mesh.R / fourpiG
        self.AG = A + Af
        self.M = Mm
        self.EG, self.Kp = E, Kp
        self.C, self.S = Cm, Sm
        self.gravity = gravity
        self.nc, self.ns_nodes, self.nf_nodes = nc, ns, nf

    def operator(self):
        """The dense matrix of eq. "1Dform"."""
        A = self.AG.copy()
        if self.n_p:
            A += self.EG @ np.linalg.solve(self.Kp, self.EG.T)
        if self.gravity == "full":
            A -= self.C.T @ np.linalg.solve(self.S, self.C)
        return 0.5 * (A + A.T)

    def translation(self):
        """The l = 1 field of a uniform translation: U = 1, V = k (= sqrt 2)
        at every displacement node."""
        assert self.l == 1
        x = np.zeros(self.n)
        x[0::2] = 1.0
        x[1::2] = self.k
        return x

    def eigenvalues(self, a=None, b=None):
        w = sla.eigh(self.operator(), self.M, eigvals_only=True)
        if a is not None:
            w = w[(w >= a) & (w <= b)]
        return w


def toroidal(layers, l, nel=40, p=3):
    """Toroidal eigenvalues omega^2 of degree l >= 1, each solid region on its
    own (fluid regions carry no toroidal motion)."""
    k2 = l * (l + 1.0)
    mesh = Mesh1D(layers, nel, p)
    sn, ns = mesh.region_nodes(p, fluid=False)
    A = np.zeros((ns, ns))
    Mm = np.zeros((ns, ns))
    for q, (i, a, b) in enumerate(mesh.elems):
        L = layers[i]
        if L.fluid:
            continue
        h = b - a
        r = a + h * mesh.xq
        w = h * mesh.wq
        phi, dphi = _lagrange(p, mesh.xq)
        dphi = dphi / h
        _, mu = L.lam_mu(r)
        e = r[:, None] * dphi - phi
        ix = np.ix_(sn[q], sn[q])
        A[ix] += np.einsum("q,qa,qb->ab", w * mu, e, e) + np.einsum("q,qa,qb->ab", w * mu * (k2 - 2), phi, phi)
        Mm[ix] += np.einsum("q,qa,qb->ab", w * L.rho(r) * r * r, phi, phi)
    return np.sort(sla.eigh(A, Mm, eigvals_only=True))


def spectrum(layers, a, b, lmax, nel=40, p=3, gravity="cowling", buoyancy=False, G=G_NONDIM):
    """All eigenvalues omega^2 in [a, b] of degrees 0..lmax as rows (omega^2,
    l, kind) with kind 0 spheroidal, 1 toroidal; each stands for 2l + 1
    eigenvalues of the 3-D problem."""
    rows = []
    for l in range(lmax + 1):
        for w in Spheroidal(layers, l, nel, p, gravity, buoyancy, G).eigenvalues(a, b):
            rows.append((w, l, 0))
        if l >= 1:
            for w in toroidal(layers, l, nel, p):
                if a <= w <= b:
                    rows.append((w, l, 1))
    rows.sort()
    return np.array(rows).reshape(-1, 3)


def multiset(rows):
    """The 3-D eigenvalues the radial spectrum stands for: each row repeated
    2l + 1 times, sorted."""
    return np.sort(np.repeat(rows[:, 0], (2 * rows[:, 1] + 1).astype(int)))
