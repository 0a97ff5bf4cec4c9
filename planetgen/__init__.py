"""Seeded synthetic planets: meshes, materials and the reference gravity field.

This module produces the *inputs* of the normal-mode eigenproblem and holds
none of the method's arithmetic (no element matrices, no operators, no
solvers).  Both the CPU oracle and the GPU library consume what it returns.

Mesh.  A "cubed ball": the cube grid [-n, n]^3 is split into Freudenthal
(Kuhn) tetrahedra, six per cell, and every integer infinity-norm shell of
the grid is mapped onto a sphere whose radius is a piecewise-linear function
of the shell index.  Region interfaces are shells, so every interface of the
layered planet is a triangulated sphere and each tetrahedron lies in exactly
one layer.  Interior vertices are jittered uniformly in a ball of radius
``jitter`` times their mean incident edge length; vertices on an interface
or on the surface are jittered tangentially and projected back onto their
sphere.  A tetrahedron whose jitter makes it inverted is re-drawn.

Local node order of an element (used for every per-element-node array):
vertices 0..3 in the order of ``tet[k]``, then for quadratic elements the
edge midpoints of edges (0,1), (0,2), (0,3), (1,2), (1,3), (2,3).

Units follow the usual nondimensionalisation of planetary normal-mode codes:
radius 1, density unit rho_bar, frequency unit sqrt(pi G rho_bar), hence
G = 1/pi and 4 pi G = 4.
"""
from __future__ import annotations

import itertools
import numpy as np

G_NONDIM = 1.0 / np.pi
P2_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))

SOLID, FLUID = 0, 1


# ----------------------------------------------------------------------------
# mesh
# ----------------------------------------------------------------------------
def _kuhn_tets(n_half: int):
    """Mirrored Freudenthal (Kuhn) triangulation of the cells of [-n, n]^3.

    In each cell the six tetrahedra share the diagonal that runs from the
    corner nearest the centre to the farthest one, so every tetrahedron has a
    vertex on the inner shell of its cell and none is flattened when shells
    are mapped onto spheres.  The mirrored triangulation is conforming."""
    m = 2 * n_half + 1
    c = np.arange(-n_half, n_half)
    I, J, K = np.meshgrid(c, c, c, indexing="ij")
    cells = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
    sgn = np.where(cells >= 0, 1, -1)
    inner = np.where(cells >= 0, cells, cells + 1)
    vid = lambda p: ((p[:, 0] + n_half) * m + (p[:, 1] + n_half)) * m + (p[:, 2] + n_half)
    eye = np.eye(3, dtype=np.int64)
    cshell = (np.abs(cells + 0.5).max(1) + 0.5).astype(np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        p0 = inner
        p1 = p0 + sgn[:, perm[0], None] * eye[perm[0]]
        p2 = p1 + sgn[:, perm[1], None] * eye[perm[1]]
        p3 = p2 + sgn[:, perm[2], None] * eye[perm[2]]
        a, b, d = p1 - p0, p2 - p0, p3 - p0
        neg = np.einsum("ij,ij->i", a, np.cross(b, d)) < 0
        t = np.stack([vid(p0), vid(p1), vid(p2), vid(p3)], 1)
        t[neg] = t[neg][:, [0, 2, 1, 3]]
        tets.append(t)
    T = np.stack(tets, 1).reshape(-1, 4)
    S = np.repeat(cshell, 6)
    return T.astype(np.int32), S


def _signed_volumes(xyz, tet):
    a = xyz[tet[:, 1]] - xyz[tet[:, 0]]
    b = xyz[tet[:, 2]] - xyz[tet[:, 0]]
    c = xyz[tet[:, 3]] - xyz[tet[:, 0]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def cubed_ball(n_half: int, shells, seed: int, jitter: float = 0.1):
    """Seeded jittered tetrahedral mesh of a layered ball.

    shells: increasing ((level, radius), ...); the last level must be n_half.
    Returns xyz f64[V,3], tet i32[T,4] (positively oriented), layer i8[T].
    """
    levels = [0] + [int(l) for l, _ in shells]
    radii = [0.0] + [float(r) for _, r in shells]
    assert levels[-1] == n_half and all(np.diff(levels) > 0)
    m = 2 * n_half + 1
    g = np.arange(-n_half, n_half + 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([I.ravel(), J.ravel(), K.ravel()], 1).astype(np.float64)
    lev = np.abs(P).max(1)
    r = np.interp(lev, levels, radii)
    nrm = np.linalg.norm(P, axis=1)
    xyz = np.zeros_like(P)
    nz = nrm > 0
    xyz[nz] = P[nz] / nrm[nz, None] * r[nz, None]
    tet, cshell = _kuhn_tets(n_half)
    layer = np.searchsorted(np.asarray(levels[1:]), cshell, side="left").astype(np.int8)

    # mean incident edge length per vertex
    e = np.concatenate([tet[:, [a, b]] for a, b in P2_EDGES])
    e = np.unique(np.sort(e, 1), axis=0)
    L = np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1)
    V = xyz.shape[0]
    hsum = np.bincount(e[:, 0], L, V) + np.bincount(e[:, 1], L, V)
    hcnt = np.bincount(e[:, 0], None, V) + np.bincount(e[:, 1], None, V)
    h = hsum / np.maximum(hcnt, 1)
    on_shell = np.isin(lev, levels[1:])

    rng = np.random.Generator(np.random.PCG64(seed))
    base = xyz.copy()

    def draw(ids):
        d = rng.standard_normal((len(ids), 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        d *= (rng.random(len(ids)) ** (1.0 / 3.0) * jitter * h[ids])[:, None]
        p = base[ids] + d
        s = on_shell[ids]
        if s.any():
            rr = r[ids][s]
            q = p[s]
            q /= np.linalg.norm(q, axis=1)[:, None]
            p[s] = q * rr[:, None]
        return p

    ids = np.arange(V)
    xyz = draw(ids)
    for _ in range(20):
        bad = _signed_volumes(xyz, tet) <= 0
        if not bad.any():
            break
        vb = np.unique(tet[bad].ravel())
        xyz[vb] = draw(vb)
    else:
        bad = _signed_volumes(xyz, tet) <= 0
        vb = np.unique(tet[bad].ravel())
        xyz[vb] = base[vb]
    assert (_signed_volumes(xyz, tet) > 0).all(), "mesh has inverted tetrahedra"
    return xyz, tet, layer


def element_node_coords(xyz, tet, order: int):
    """Coordinates of the local nodes of every element, f64[T, Np, 3]."""
    X = xyz[tet]  # [T,4,3]
    if order == 1:
        return X
    mids = [(X[:, a] + X[:, b]) * 0.5 for a, b in P2_EDGES]
    return np.concatenate([X, np.stack(mids, 1)], 1)


# ----------------------------------------------------------------------------
# material fields
# ----------------------------------------------------------------------------
def gaussian_random_field(points, seed: int, corr_len: float = 0.1, n_features: int = 2048,
                          chunk: int = 2048):
    """Unit-variance Gaussian random field with squared-exponential correlation
    (random Fourier features), evaluated at points [P,3].  The phases are
    evaluated in float32 after reduction to [-pi, pi]; the field is an input
    and only needs to be smooth and reproducible."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = (rng.standard_normal((n_features, 3)) / corr_len).astype(np.float32)
    ph = (rng.random(n_features) * 2.0 * np.pi).astype(np.float32)
    out = np.empty(points.shape[0])
    s = np.sqrt(2.0 / n_features)
    buf = np.empty((chunk, n_features), np.float32)
    tmp = np.empty((chunk, n_features), np.float32)
    inv2pi = np.float32(1.0 / (2.0 * np.pi))
    twopi = np.float32(2.0 * np.pi)
    pts = points.astype(np.float32)
    for i in range(0, pts.shape[0], chunk):
        q = pts[i:i + chunk]
        b, t = buf[:len(q)], tmp[:len(q)]
        np.multiply(q[:, 0:1], k[:, 0], out=b)
        b += q[:, 1:2] * k[:, 1]
        b += q[:, 2:3] * k[:, 2]
        b += ph
        np.multiply(b, inv2pi, out=t)
        np.rint(t, out=t)
        t *= twopi
        b -= t
        np.cos(b, out=b)
        out[i:i + len(q)] = s * b.sum(1, dtype=np.float64)
    return out


class RadialModel:
    """Layered radial model: per layer, polynomials (coefficients in powers
    of r, lowest first) for density, V_P and V_S, plus a solid/fluid flag."""

    def __init__(self, radii, rho, vp, vs, fluid):
        self.radii = np.asarray(radii, float)  # outer radius of each layer
        self.rho = [np.polynomial.Polynomial(c) for c in rho]
        self.vp = [np.polynomial.Polynomial(c) for c in vp]
        self.vs = [np.polynomial.Polynomial(c) for c in vs]
        self.fluid = list(fluid)
        # enclosed mass integrals m(r) = int_0^r rho s^2 ds, continuous in r
        self._mint = []
        acc = 0.0
        lo = 0.0
        s2 = np.polynomial.Polynomial([0, 0, 1])
        for i, R in enumerate(self.radii):
            P = (self.rho[i] * s2).integ()
            self._mint.append((P, acc - P(lo)))
            acc = acc + P(R) - P(lo)
            lo = R

    def enclosed(self, r, layer):
        out = np.empty_like(r)
        for i, (P, off) in enumerate(self._mint):
            s = layer == i
            out[s] = P(r[s]) + off
        return out

    def gravity(self, x, layer):
        """g' = -grad(Phi0) for the radial mean density (centrifugal term
        omitted) and its gradient d_i g'_j at points x [P,3] of given layers.
        Returns (g [P,3], dg [P,3,3])."""
        r = np.linalg.norm(x, axis=1)
        rs = np.maximum(r, 1e-300)
        m = self.enclosed(r, layer)
        rho = np.empty_like(r)
        for i in range(len(self.radii)):
            s = layer == i
            rho[s] = self.rho[i](r[s])
        fourpiG = 4.0 * np.pi * G_NONDIM
        small = r < 1e-12
        g_over_r = np.where(small, fourpiG * rho / 3.0, fourpiG * m / rs ** 3)
        gmag = g_over_r * r
        dgdr = fourpiG * rho - 2.0 * g_over_r
        xh = np.where(small[:, None], 0.0, x / rs[:, None])
        gvec = -gmag[:, None] * xh
        eye = np.eye(3)[None]
        xx = xh[:, :, None] * xh[:, None, :]
        dg = -(g_over_r[:, None, None] * (eye - xx) + dgdr[:, None, None] * xx)
        dg[small] = -(g_over_r[small, None, None] * eye[0])
        return gvec, dg

    def sample(self, x, layer):
        r = np.linalg.norm(x, axis=1)
        rho, vp, vs = (np.empty_like(r) for _ in range(3))
        for i in range(len(self.radii)):
            s = layer == i
            rho[s] = self.rho[i](r[s])
            vp[s] = self.vp[i](r[s])
            vs[s] = self.vs[i](r[s])
        return rho, vp, vs


def three_layer_model():
    """Smooth layered profiles shaped like a terrestrial planet (solid inner
    core, fluid outer core, solid mantle) in nondimensional units."""
    return RadialModel(
        radii=[0.19, 0.55, 1.0],
        rho=[[2.35, 0.0, -0.6], [2.20, 0.0, -0.8], [1.50, -0.89]],
        vp=[[2.05, 0.0, -0.5], [1.55, 0.0, -0.9], [2.98, -1.78]],
        vs=[[0.65, 0.0, -0.3], [0.0], [1.56, -0.91]],
        fluid=[False, True, False],
    )


def two_layer_model():
    """Mars-like body: fluid core r < 0.5 and a solid mantle."""
    return RadialModel(
        radii=[0.5, 1.0],
        rho=[[1.95, 0.0, -0.6], [1.30, -0.6]],
        vp=[[1.40, 0.0, -0.8], [2.40, -1.30]],
        vs=[[0.0], [1.30, -0.70]],
        fluid=[True, False],
    )


def _materials(model, xyz, tet, layer, seed, grf_amp, order, gravity=True):
    bary = xyz[tet].mean(1)
    rho, vp, vs = model.sample(bary, layer.astype(np.int64))
    region = np.array([FLUID if model.fluid[l] else SOLID for l in range(len(model.radii))],
                      np.int8)[layer]
    if grf_amp:
        # the field multiplies rho, lambda and mu alike (velocities unchanged)
        d = gaussian_random_field(bary, seed + 7919)
        rho = rho * np.where(region == SOLID, 1.0 + grf_amp * d, 1.0)
    mu = np.where(region == FLUID, 0.0, rho * vs ** 2)
    lam = rho * vp ** 2 - 2.0 * mu
    out = dict(xyz=xyz, tet=tet, region=region, layer=layer, rho=rho, lam=lam, mu=mu,
               gprime=None, grad_gprime=None)
    if gravity:
        en = element_node_coords(xyz, tet, order)
        T, Np, _ = en.shape
        lay = np.repeat(layer.astype(np.int64), Np)
        g, dg = model.gravity(en.reshape(-1, 3), lay)
        out["gprime"] = g.reshape(T, Np, 3)
        out["grad_gprime"] = dg.reshape(T, Np, 3, 3)
    return out


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def homogeneous_ball(seed: int = 1906, n_half: int = 4, order: int = 1, jitter: float = 0.1):
    """Homogeneous elastic ball, radius 1, rho = lambda = mu = 1, no gravity,
    no rotation (~3k tets at n_half = 4)."""
    xyz, tet, layer = cubed_ball(n_half, [(n_half, 1.0)], seed, jitter)
    T = tet.shape[0]
    one = np.ones(T)
    return dict(xyz=xyz, tet=tet, region=np.zeros(T, np.int8), layer=layer, rho=one.copy(),
                lam=one.copy(), mu=one.copy(), gprime=None, grad_gprime=None,
                disp_order=order, pres_order=1, omega=(0.0, 0.0, 0.0))


def three_layer_planet(seed: int = 1906, n_half: int = 20, order: int = 2, pres_order: int = 1,
                       grf_amp: float = 0.02, jitter: float = 0.05, omega=(0.0, 0.0, 0.0),
                       gravity: bool = True):
    """Solid inner core r < 0.19, fluid outer core to 0.55, solid mantle to 1.
    Interface shells are placed so that the radial spacing is nearly uniform.
    Vertex jitter 5 % of the local edge length: larger jitter creates the
    flattest elements, which set the top of the spectrum."""
    l1 = max(1, int(round(n_half * 0.19)))
    l2 = max(l1 + 1, int(round(n_half * 0.55)))
    xyz, tet, layer = cubed_ball(n_half, [(l1, 0.19), (l2, 0.55), (n_half, 1.0)], seed, jitter)
    d = _materials(three_layer_model(), xyz, tet, layer, seed, grf_amp, order, gravity)
    d.update(disp_order=order, pres_order=pres_order, omega=tuple(float(w) for w in omega))
    return d


def mars_like(seed: int = 1906, n_half: int = 30, order: int = 2, pres_order: int = 1,
              grf_amp: float = 0.05, jitter: float = 0.05, omega=(0.0, 0.0, 0.1),
              gravity: bool = True):
    """Two-layer body: fluid core r < 0.5, solid mantle with lateral
    heterogeneity."""
    l1 = max(1, int(round(n_half * 0.5)))
    xyz, tet, layer = cubed_ball(n_half, [(l1, 0.5), (n_half, 1.0)], seed, jitter)
    d = _materials(two_layer_model(), xyz, tet, layer, seed, grf_amp, order, gravity)
    d.update(disp_order=order, pres_order=pres_order, omega=tuple(float(w) for w in omega))
    return d


def start_block(n: int, ncols: int, seed: int, col0: int = 0):
    """Seeded N(0,1) start vectors, column c drawn from its own stream so a
    column is the same whatever block it is requested in.  f64[n, ncols]."""
    out = np.empty((n, ncols))
    for c in range(ncols):
        rng = np.random.Generator(np.random.PCG64([seed, col0 + c]))
        out[:, c] = rng.standard_normal(n)
    return out
