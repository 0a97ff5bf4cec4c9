"""Pins of the oracle's assembled matrices (Sec. 4.2 table, Appendix A):
closed forms, invariants and brute force."""
import numpy as np
import pytest
import scipy.linalg as sla

import planetgen as pg
from conftest import planet
from oracle.assemble import Pencil, tet_geometry, omega_cross
from oracle.mesh import FACES


def _dof_field(P, f):
    """Nodal DOF vector (3 * node + comp) of a vector field f(x)."""
    nb = P.nb
    xyz = P.p["xyz"]
    gx = np.concatenate([xyz, 0.5 * (xyz[nb.edges[:, 0]] + xyz[nb.edges[:, 1]])]) if len(nb.edges) else xyz
    return f(gx[nb.node_geom]).ravel()


def _rigid_modes(P):
    out = []
    for k in range(3):
        out.append(_dof_field(P, lambda x, k=k: np.tile(np.eye(3)[k], (len(x), 1))))
        out.append(_dof_field(P, lambda x, k=k: np.cross(np.eye(3)[k][None], x)))
    return out


def test_symmetry_definiteness_skew():
    d = dict(planet("three_layer_planet", n_half=4, order=2))
    d["omega"] = (0.1, -0.2, 0.3)
    P = Pencil(d)
    for Mtx in (P.AG, P.Kp):
        assert abs(Mtx - Mtx.T).max() <= 1e-14 * abs(Mtx).max()
    assert abs(P.R + P.R.T).max() <= 1e-15 * abs(P.R).max()
    np.linalg.cholesky(P.Ms.toarray())
    np.linalg.cholesky(P.Kp.toarray())


@pytest.mark.parametrize("order", [1, 2])
def test_rigid_modes_no_gravity(order):
    """Without gravity the six rigid motions are in the kernel of the full
    Cowling operator A_G + E_G K_p^{-1} E_G^T (solid ball and layered planet)."""
    for d in (planet("homogeneous_ball", order=order),
              planet("three_layer_planet", n_half=4, order=order, gravity=False)):
        P = Pencil(d)
        kp = P.kp_direct() if P.n_p else None
        nA = abs(P.AG).max()
        for r in _rigid_modes(P):
            y = P.cowling_apply(r, kp)
            assert np.abs(y).max() <= 1e-12 * nA * np.abs(r).max()


def test_patch_test_and_energy():
    """u = Gx on a homogeneous P1 ball: interior rows of A u vanish and
    u^T A u = sum |K| (lambda (tr G)^2 + 2 mu |sym G|^2)."""
    d = planet("homogeneous_ball")
    P = Pencil(d)
    Gm = np.array([[0.3, -0.1, 0.2], [0.05, -0.4, 0.1], [0.2, 0.3, 0.15]])
    u = _dof_field(P, lambda x: x @ Gm.T)
    y = (P.AG @ u).reshape(-1, 3)
    r = np.linalg.norm(P.p["xyz"], axis=1)
    interior = r < 0.999
    assert np.abs(y[interior]).max() < 1e-13 * np.abs(P.AG).max()
    Gs = 0.5 * (Gm + Gm.T)
    vol = P.vol.sum()
    energy = vol * (np.trace(Gm) ** 2 + 2 * (Gs ** 2).sum())
    assert abs(u @ (P.AG @ u) - energy) < 1e-12 * energy


def test_mass_and_coriolis_moments():
    d = dict(planet("three_layer_planet", n_half=4, order=2))
    d["omega"] = (0.0, 0.0, 0.37)
    P = Pencil(d)
    tx = _dof_field(P, lambda x: np.tile([1.0, 0, 0], (len(x), 1)))
    ty = _dof_field(P, lambda x: np.tile([0, 1.0, 0], (len(x), 1)))
    mass = (d["rho"] * P.vol).sum()
    assert abs(tx @ (P.M @ tx) - mass) < 1e-12 * mass
    assert abs(tx @ (P.R @ ty) + 0.37 * mass) < 1e-12 * mass


def test_p1_element_stiffness_bmatrix():
    """One P1 tetrahedron: the oracle's blocks equal the engineering
    strain-displacement form K = |K| B^T C B (Voigt notation)."""
    xyz = np.array([[0.0, 0, 0], [1.1, 0.1, 0], [0.2, 0.9, 0.1], [0.1, 0.2, 1.3]])
    d = dict(xyz=xyz, tet=np.array([[0, 1, 2, 3]], np.int32), region=np.zeros(1, np.int8),
             rho=np.array([2.0]), lam=np.array([1.7]), mu=np.array([0.6]), gprime=None,
             grad_gprime=None, disp_order=1, pres_order=1, omega=(0, 0, 0))
    P = Pencil(d)
    vol, G = tet_geometry(xyz, d["tet"])
    B = np.zeros((6, 12))
    for a in range(4):
        gx, gy, gz = G[0, a]
        B[:, 3 * a:3 * a + 3] = [[gx, 0, 0], [0, gy, 0], [0, 0, gz], [gy, gx, 0], [0, gz, gy], [gz, 0, gx]]
    lam, mu = 1.7, 0.6
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[:3, :3] += 2 * mu * np.eye(3)
    C[3:, 3:] = mu * np.eye(3)
    K = vol[0] * B.T @ C @ B
    np.testing.assert_allclose(P.AG.toarray(), K, atol=1e-14 * np.abs(K).max())


def _moments(xyz, tet):
    """Exact int 1, int x_i, int x_i x_j over each tetrahedron."""
    X = xyz[tet]
    vol = np.abs(np.einsum("ti,ti->t", X[:, 1] - X[:, 0],
                           np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]))) / 6
    m1 = vol[:, None] * X.mean(1)
    s = X.sum(1)
    m2 = vol[:, None, None] / 20.0 * (np.einsum("tai,taj->tij", X, X) + s[:, :, None] * s[:, None, :])
    return vol, m1, m2


def test_gravity_terms_closed_form():
    """Homogeneous P2 ball with the linear field g' = -c x: the symmetrised
    gravity form of a_2^s between affine fields u = Gx + t and v = Hx + s is
    integrated exactly by the nodal formulas of Appendix A; compare with the
    analytic integral from exact tetrahedral moments."""
    d = dict(planet("homogeneous_ball", order=2))
    c = 1.3
    en = pg.element_node_coords(d["xyz"], d["tet"], 2)
    d["gprime"] = -c * en
    d["grad_gprime"] = np.broadcast_to(-c * np.eye(3), en.shape + (3,)).copy()
    rho = 0.8
    d["rho"] = np.full(len(d["tet"]), rho)
    P1 = Pencil(d)
    d0 = dict(d, gprime=None, grad_gprime=None)
    Ag = P1.AG - Pencil(d0).AG
    rng = np.random.default_rng(3)
    Gm, H = rng.standard_normal((3, 3)), rng.standard_normal((3, 3))
    t, s = rng.standard_normal(3), rng.standard_normal(3)
    u = _dof_field(P1, lambda x: x @ Gm.T + t)
    v = _dof_field(P1, lambda x: x @ H.T + s)
    vol, m1, m2 = _moments(d["xyz"], d["tet"])
    I0, I1, I2 = vol.sum(), m1.sum(0), m2.sum(0)
    # integrals of products of affine functions (a.x + a0)(b.x + b0)
    def prod(A, a0, B, b0):
        return np.einsum("i,j,ij->", A, B, I2) + a0 * B @ I1 + b0 * A @ I1 + a0 * b0 * I0
    # g' = -c x; g'.u = -c x.(Gx+t); div v = tr H; u.(grad v).g' = g'^T H u
    def L(Gu, tu, Hv, sv):
        # (div v)(g'.u) rho - u.(grad g').v rho - u.(grad v).g' rho
        t1 = np.trace(Hv) * (-c) * sum(prod(np.eye(3)[i], 0.0, Gu[i], tu[i]) for i in range(3))
        t2 = c * sum(prod(Gu[i], tu[i], Hv[i], sv[i]) for i in range(3))
        t3 = c * sum(prod(np.eye(3)[i], 0.0, (Hv @ Gu)[i], (Hv @ tu)[i]) for i in range(3))
        return rho * (t1 + t2 + t3)
    ref = 0.5 * (L(Gm, t, H, s) + L(H, s, Gm, t))
    val = v @ (Ag @ u)
    assert abs(val - ref) < 1e-11 * max(1.0, abs(ref))


def test_fs_face_term_closed_form():
    """Layered P2 planet, synthetic linear g' = -c x: the symmetrised
    fluid-solid face term int S{(v.g')(nu.u)} [rho]^f between affine fields
    equals a degree-3 triangle cubature over the fluid-solid faces."""
    d = dict(planet("three_layer_planet", n_half=4, order=2))
    c = 0.7
    en = pg.element_node_coords(d["xyz"], d["tet"], 2)
    d["gprime"] = -c * en
    d["grad_gprime"] = np.zeros(en.shape + (3,))
    d["mu"] = d["mu"] * 0 + np.where(d["region"] == 0, 1.0, 0.0)
    Pg = Pencil(d)
    P0 = Pencil(dict(d, gprime=None, grad_gprime=None))
    rng = np.random.default_rng(5)
    Gm, H = rng.standard_normal((3, 3)), rng.standard_normal((3, 3))
    t, s = rng.standard_normal(3), rng.standard_normal(3)
    # gravity volume part is removed by using the same grad g' = 0 and
    # evaluating the volume terms separately is avoided: restrict fields to
    # the solid copies and subtract the volume contribution computed with
    # the same oracle on a planet whose fluid-solid faces are removed.
    u = _dof_field(Pg, lambda x: x @ Gm.T + t)
    v = _dof_field(Pg, lambda x: x @ H.T + s)
    ns = Pg.nb.n_solid
    u[3 * ns:] = 0
    v[3 * ns:] = 0
    d_all_solid = dict(d, region=np.zeros_like(d["region"]), mu=np.ones(len(d["tet"])))
    # volume terms of the solid tets only: assemble on the all-solid planet
    # and restrict to solid tets by zeroing rho of the fluid tets
    d_vol = dict(d_all_solid, rho=np.where(d["region"] == 0, d["rho"], 0.0))
    Pv = Pencil(d_vol)
    Pv0 = Pencil(dict(d_vol, gprime=None, grad_gprime=None))
    uv = _dof_field(Pv, lambda x: x @ Gm.T + t)
    vv = _dof_field(Pv, lambda x: x @ H.T + s)
    vol_part = vv @ ((Pv.AG - Pv0.AG) @ uv)
    face_part = v @ ((Pg.AG - P0.AG) @ u) - vol_part
    # cubature over the faces
    tet, xyz = d["tet"], d["xyz"]
    qb = np.array([[1 / 3, 1 / 3, 1 / 3], [0.6, 0.2, 0.2], [0.2, 0.6, 0.2], [0.2, 0.2, 0.6]])
    qw = np.array([-27 / 48, 25 / 48, 25 / 48, 25 / 48])
    ref = 0.0
    for st, sf, ft in Pg.nb.fs_faces:
        A, B, C = (xyz[tet[st][q]] for q in FACES[sf])
        o = xyz[tet[st][sf]]
        nvec = np.cross(B - A, C - A)
        area = 0.5 * np.linalg.norm(nvec)
        nvec /= 2 * area
        if np.dot(nvec, A - o) < 0:
            nvec = -nvec
        for b, w in zip(qb, qw):
            x = b[0] * A + b[1] * B + b[2] * C
            g = -c * x
            uu, vvv = Gm @ x + t, H @ x + s
            ref += w * area * d["rho"][ft] * 0.5 * ((vvv @ g) * (nvec @ uu) + (uu @ g) * (nvec @ vvv))
    assert abs(face_part - ref) < 1e-10 * max(1.0, abs(ref))


def test_coupling_divergence_theorem():
    """E_G^T of a uniform translation (same on both sides of the fluid-solid
    interfaces) vanishes without gravity: int grad(v^p).t over the fluid
    cancels the face integrals of v^p nu.t.  With g' the p = 1 row sum is
    -int_F (g'.t) rho / kappa."""
    d = planet("three_layer_planet", n_half=4, order=2, gravity=False)
    P = Pencil(d)
    t = np.array([0.3, -0.5, 0.8])
    u = _dof_field(P, lambda x: np.tile(t, (len(x), 1)))
    r = P.EG.T @ u
    assert np.abs(r).max() < 1e-14 * np.abs(P.EG).max() * 10
    dg = dict(planet("three_layer_planet", n_half=4, order=2))
    c = 0.9
    en = pg.element_node_coords(dg["xyz"], dg["tet"], 2)
    dg["gprime"] = -c * en
    dg["grad_gprime"] = np.zeros(en.shape + (3,))
    Pg = Pencil(dg)
    u = _dof_field(Pg, lambda x: np.tile(t, (len(x), 1)))
    got = (Pg.EG.T @ u).sum()
    fl = dg["region"] == 1
    vol, m1, _ = _moments(dg["xyz"], dg["tet"])
    kappa = dg["lam"] + 2 * dg["mu"] / 3
    ref = (c * (dg["rho"] / kappa)[fl, None] * m1[fl]).sum(0) @ t
    assert abs(got - ref) < 1e-12 * max(1.0, abs(ref))
    assert abs(Pg.Kp.sum() - (vol[fl] / kappa[fl]).sum()) < 1e-12 * Pg.Kp.sum()


def test_cowling_essential_spectrum_dimension():
    """Cowling with N^2 = 0: fluid-only displacements with E_G^T u = 0 are
    exact zero modes (the discrete essential spectrum); their number is
    3 N_f - rank(E_G restricted to the fluid)."""
    d = planet("three_layer_planet", n_half=3, order=1)
    P = Pencil(d)
    A = P.cowling_dense()
    M = P.M.toarray()
    w = sla.eigh(A, M, eigvals_only=True)
    ns = P.nb.n_solid
    Ef = P.EG.toarray()[3 * ns:]
    nf = Ef.shape[0]
    rank = np.linalg.matrix_rank(Ef)
    nzero = int((np.abs(w) < 1e-9 * np.abs(w).max()).sum())
    assert nzero >= nf - rank
    # and the count of zeros is exactly that (no other zero modes besides
    # the fluid kernel, up to the rigid rotations of the spherical layers)
    assert nzero - (nf - rank) <= 6
