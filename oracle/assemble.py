"""Element matrices and global assembly (oracle, FP64).

Follows the table of implicit matrix definitions (Sec. 4.2) and the element
formulas of Appendix A:

* A_G (stiffness with gravity, solid block A_sg; the fluid block A_f is zero
  because the buoyancy term vanishes for N^2 = 0 and no fluid-fluid
  interface exists):
    - elasticity  int grad(v) : c : grad(u), isotropic c (lambda, mu);
    - the symmetrised gravity terms of a_2^s,
        S{ (div v)(g'.u) rho - u.(grad g').v rho - u.(grad v).g' rho },
      with g' and grad g' interpolated at the element nodes exactly as the
      diagonal matrices D_{g'} of Appendix A do;
    - the symmetrised fluid-solid face term S{ (v.g')(nu.u) [rho]^f }.
* M_s  scalar mass int rho l_a l_b (M = M_s (x) I_3).
* R    Coriolis int rho v.(Omega x u) = M_s (x) [Omega]_x.
* K_p  = -A_p = int kappa^{-1} l^p_a l^p_b  (SPD; the paper's A_p carries the
  minus sign).
* E_G  = [E_FS ; A_dg] (n x n_p):
    A_dg  int v^f.grad p - (v^f.g') p rho / kappa   (fluid tetrahedra),
    E_FS  int (v^s.nu^{s->f}) p                      (fluid-solid faces).

Every integral is exact for affine tetrahedra (refelem), so the nodal
formulas of Appendix A and the direct integrals used here coincide.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import refelem as re_
from .mesh import Numbering, FACES

LEVI = np.zeros((3, 3, 3))
for _i, _j, _k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    LEVI[_i, _j, _k] = 1.0
    LEVI[_i, _k, _j] = -1.0


def omega_cross(omega):
    """[Omega]_x with ([Omega]_x u)_i = (Omega x u)_i."""
    return -np.einsum("ijk,k->ij", LEVI, np.asarray(omega, float))


def tet_geometry(xyz, tet):
    """Volumes |K| and barycentric gradients G[T, 4, 3] (row k = grad lambda_k)."""
    X = xyz[tet]
    Tm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], 2)  # columns
    det = np.linalg.det(Tm)
    if (det <= 0).any():
        raise ValueError("tetrahedron %d has non-positive Jacobian" % int(np.argmax(det <= 0)))
    inv = np.linalg.inv(Tm)  # rows: grad lambda_1..3
    G = np.concatenate([-inv.sum(1, keepdims=True), inv], 1)
    return det / 6.0, G


def face_geometry(xyz, tet, st, sf):
    """Area and outward unit normal of local face sf of tetrahedra st."""
    a, b, c = (np.array([FACES[f][q] for f in sf]) for q in range(3))
    X = xyz[tet[st]]
    idx = np.arange(len(st))
    Xa, Xb, Xc = X[idx, a], X[idx, b], X[idx, c]
    Xo = X[idx, sf]
    n = np.cross(Xb - Xa, Xc - Xa)
    area = 0.5 * np.linalg.norm(n, axis=1)
    n /= (2.0 * area)[:, None]
    flip = np.einsum("ij,ij->i", n, Xa - Xo) < 0
    n[flip] *= -1.0
    return area, n


class Ref:
    def __init__(self, order, pres_order):
        self.MM = re_.as_float(re_.mass_exact(order, order, 4))
        self.KK = re_.as_float(re_.stiff_exact(order, 4))
        self.DM = re_.as_float(re_.dmass_exact(order, order, 4))          # [a,c,k]: d_k l_a * l_c
        self.Mp = re_.as_float(re_.mass_exact(pres_order, pres_order, 4))
        self.Mfp = re_.as_float(re_.mass_exact(order, pres_order, 4))    # [a,c]
        self.DMpf = re_.as_float(re_.dmass_exact(pres_order, order, 4))  # [c,a,k]: d_k lp_c * l_a
        self.M2 = re_.as_float(re_.mass_exact(order, order, 3))
        self.M2sp = re_.as_float(re_.mass_exact(order, pres_order, 3))


def element_stiffness(vol, G, lam, mu, ref):
    """Elasticity blocks K[T, a, j, b, n] (test node a comp j, trial node b
    comp n) of int d_i v_j c_ijmn d_m u_n with isotropic c:
    K = lam S[a,b,j,n] + mu S[a,b,n,j] + mu delta_jn sum_m S[a,b,m,m],
    S[a,b,m,n] = int d_m l_a d_n l_b."""
    S = np.einsum("t,tkm,tln,abkl->tabmn", vol, G, G, ref.KK)
    tr = np.einsum("tabmm->tab", S)
    L = lam[:, None, None, None, None]
    U = mu[:, None, None, None, None]
    return (L * np.einsum("tabjn->tajbn", S) + U * np.einsum("tabnj->tajbn", S)
            + U * np.einsum("tab,jn->tajbn", tr, np.eye(3)))


def element_gravity(vol, G, rho, g, dg, ref):
    """Symmetrised gravity blocks [T, a, i, c, j] from g'[T,Np,3] and
    grad g'[T,Np,3,3] (dg[.., i, j] = d_i g'_j) given at element nodes."""
    P = np.einsum("t,tkm,ack->tacm", vol, G, ref.DM)  # int d_m l_a * l_c
    Mk = vol[:, None, None] * ref.MM
    t1 = np.einsum("taci,tcj->taicj", P, g)                   # (div v)(g'.u)
    t2 = -np.einsum("taij,tac->taicj", dg, Mk)                 # -u.(grad g').v
    t3 = -np.einsum("tacj,tci->taicj", P, g)                   # -u.(grad v).g'
    Gm = rho[:, None, None, None, None] * (t1 + t2 + t3)
    return 0.5 * (Gm + Gm.transpose(0, 3, 4, 1, 2))


def _coo_blocks(rows_node, cols_node, blocks):
    """Expand node-level 3x3 blocks [T,a,i,c,j] to scalar COO triplets."""
    T, na, _, nc, _ = blocks.shape
    i3 = np.arange(3)
    r = (3 * rows_node[:, :, None, None, None] + i3[None, None, :, None, None])
    c = (3 * cols_node[:, None, None, :, None] + i3[None, None, None, None, :])
    r = np.broadcast_to(r, blocks.shape).ravel()
    c = np.broadcast_to(c, blocks.shape).ravel()
    return r, c, blocks.ravel()


class Pencil:
    """All assembled matrices of one planet (scipy CSR, DOF numbering
    3 * node + component)."""

    def __init__(self, planet, omega=None, chunk=20000):
        self.p = planet
        xyz = np.asarray(planet["xyz"], float)
        tet = np.asarray(planet["tet"], np.int64)
        region = np.asarray(planet["region"])
        order, porder = int(planet["disp_order"]), int(planet["pres_order"])
        self.nb = nb = Numbering(tet, region, len(xyz), order, porder)
        self.ref = ref = Ref(order, porder)
        self.order, self.porder = order, porder
        self.N, self.n, self.n_p = nb.N, 3 * nb.N, nb.n_pres
        self.omega = np.zeros(3) if omega is None else np.asarray(omega, float)
        if omega is None and "omega" in planet:
            self.omega = np.asarray(planet["omega"], float)
        rho = np.asarray(planet["rho"], float)
        lam = np.asarray(planet["lam"], float)
        mu = np.asarray(planet["mu"], float)
        gp, dgp = planet.get("gprime"), planet.get("grad_gprime")
        nd = 4 if order == 1 else 10
        if gp is not None:
            gp = np.asarray(gp, float)[:, :nd]
            dgp = np.asarray(dgp, float)[:, :nd]
        vol, Gr = tet_geometry(xyz, tet)
        self.vol = vol
        solid = region == 0
        R, C, V = [], [], []
        Rm, Cm, Vm = [], [], []
        for s in range(0, len(tet), chunk):
            sl = slice(s, s + chunk)
            en = nb.elem_node[sl]
            # mass (all tets)
            me = (rho[sl] * vol[sl])[:, None, None] * ref.MM
            Rm.append(np.repeat(en, nd, 1).ravel())
            Cm.append(np.tile(en, (1, nd)).ravel())
            Vm.append(me.ravel())
            sol = np.nonzero(solid[sl])[0]
            if len(sol):
                vs, Gs = vol[sl][sol], Gr[sl][sol]
                K = element_stiffness(vs, Gs, lam[sl][sol], mu[sl][sol], ref)
                if gp is not None:
                    K = K + element_gravity(vs, Gs, rho[sl][sol], gp[sl][sol], dgp[sl][sol], ref)
                r, c, v = _coo_blocks(en[sol], en[sol], K)
                R.append(r); C.append(c); V.append(v)
        # fluid-solid face gravity term (solid side)
        fs = nb.fs_faces
        if gp is not None and len(fs):
            st, sf, ft = fs[:, 0], fs[:, 1], fs[:, 2]
            area, nu = face_geometry(xyz, tet, st, sf)
            loc = np.array([nb.face_nodes(a, b, order, "u") for a, b in zip(st, sf)])
            un = nb.elem_node[st[:, None], loc]
            gf = gp[st[:, None], loc]                                # [F, nf, 3]
            M2 = area[:, None, None] * ref.M2
            Fb = rho[ft][:, None, None, None, None] * np.einsum("fai,fac,fj->faicj", gf, M2, nu)
            Fb = 0.5 * (Fb + Fb.transpose(0, 3, 4, 1, 2))
            r, c, v = _coo_blocks(un, un, Fb)
            R.append(r); C.append(c); V.append(v)
        n = self.n
        if R:
            self.AG = sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))),
                                    shape=(n, n))
        else:
            self.AG = sp.csr_matrix((n, n))
        self.AG.sum_duplicates()
        self.Ms = sp.csr_matrix((np.concatenate(Vm), (np.concatenate(Rm), np.concatenate(Cm))),
                                shape=(self.N, self.N))
        self.Ms.sum_duplicates()
        self.M = sp.kron(self.Ms, sp.identity(3), format="csr")
        self.R = sp.kron(self.Ms, sp.csr_matrix(omega_cross(self.omega)), format="csr")
        self._fluid(xyz, tet, region, rho, lam, mu, gp, vol, Gr)

    def _fluid(self, xyz, tet, region, rho, lam, mu, gp, vol, Gr):
        nb, ref = self.nb, self.ref
        fl = np.nonzero(region != 0)[0]
        n, n_p = self.n, self.n_p
        if n_p == 0:
            self.Kp = sp.csr_matrix((0, 0))
            self.EG = sp.csr_matrix((n, 0))
            return
        kappa = lam[fl] + 2.0 * mu[fl] / 3.0
        ep = nb.elem_pres[fl]
        npp = ep.shape[1]
        ke = (vol[fl] / kappa)[:, None, None] * ref.Mp
        self.Kp = sp.csr_matrix((ke.ravel(), (np.repeat(ep, npp, 1).ravel(), np.tile(ep, (1, npp)).ravel())),
                                shape=(n_p, n_p))
        self.Kp.sum_duplicates()
        # A_dg: (v_j at node a, p at node c)
        en = nb.elem_node[fl]
        nd = en.shape[1]
        Q = np.einsum("t,tkj,cak->tajc", vol[fl], Gr[fl], ref.DMpf)        # int l_a d_j lp_c
        blk = Q.copy()
        if gp is not None:
            Mfp = vol[fl][:, None, None] * ref.Mfp
            blk -= np.einsum("t,taj,tac->tajc", rho[fl] / kappa, gp[fl], Mfp)
        r = (3 * en[:, :, None, None] + np.arange(3)[None, None, :, None])
        c = np.broadcast_to(ep[:, None, None, :], blk.shape)
        R, C, V = [np.broadcast_to(r, blk.shape).ravel()], [c.ravel()], [blk.ravel()]
        fs = nb.fs_faces
        if len(fs):
            st, sf = fs[:, 0], fs[:, 1]
            area, nu = face_geometry(xyz, tet, st, sf)
            locu = np.array([nb.face_nodes(a, b, self.order, "u") for a, b in zip(st, sf)])
            locp = np.array([nb.face_nodes(a, b, self.porder, "p") for a, b in zip(st, sf)])
            un = nb.elem_node[st[:, None], locu]
            pn = nb.pid[nb.geom[st[:, None], locp]]
            M2 = area[:, None, None] * ref.M2sp
            e = np.einsum("fac,fj->fajc", M2, nu)
            r = 3 * un[:, :, None, None] + np.arange(3)[None, None, :, None]
            R.append(np.broadcast_to(r, e.shape).ravel())
            C.append(np.broadcast_to(pn[:, None, None, :], e.shape).ravel())
            V.append(e.ravel())
        self.EG = sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(n, n_p))
        self.EG.sum_duplicates()

    # ------------------------------------------------------------ operators
    def cowling_apply(self, x, kp_solve=None):
        """y = (A_G + E_G K_p^{-1} E_G^T) x  (eq. "cowling": A_G - E_G A_p^{-1} E_G^T)."""
        y = self.AG @ x
        if self.n_p:
            if kp_solve is None:
                kp_solve = self.kp_direct()
            y = y + self.EG @ kp_solve(self.EG.T @ x)
        return y

    def kp_direct(self):
        import scipy.sparse.linalg as spla
        lu = spla.splu(self.Kp.tocsc())
        return lambda r: lu.solve(r)

    def cowling_dense(self):
        A = self.AG.toarray()
        if self.n_p:
            E = self.EG.toarray()
            A = A + E @ np.linalg.solve(self.Kp.toarray(), E.T)
        return 0.5 * (A + A.T)
