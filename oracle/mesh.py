"""Node numbering and sparsity patterns (oracle; integer work, bit-exact).

The paper collects nodal values of u^s, u^f and p into vectors (Sec. 4.2)
and uses elements that are non-conforming across fluid-solid boundaries
(Sec. 4.1): a node on such a boundary carries an independent solid and a
fluid displacement.  It assembles "using standard techniques" (Appendix A)
and fixes no numbering.  The numbering rules used here (a reading, shared
as a specification with the GPU library, not as code):

1. Geometric nodes: vertices 0..V-1 in input order, then (degree 2) one node
   per edge, edges ordered lexicographically by (min vertex, max vertex).
2. Displacement nodes: a geometric node has a solid copy if it belongs to a
   solid tetrahedron and a fluid copy if it belongs to a fluid one.  All
   solid copies come first, ordered by geometric id, then all fluid copies.
   Displacement DOF = 3 * node + component.
3. Pressure nodes: geometric nodes of the pressure degree that belong to a
   fluid tetrahedron, ordered by geometric id.
4. Node graph: displacement nodes i ~ j when some tetrahedron holds both
   (a tetrahedron holds the copies of its own side); the diagonal is always
   present; columns strictly increasing; no value-based pruning.
5. Pressure graph: pressure nodes sharing a fluid tetrahedron.
6. E_G pattern (displacement node, pressure node): pairs sharing a fluid
   tetrahedron, plus (solid copy, pressure node) pairs on a common
   fluid-solid face.
"""
from __future__ import annotations

import numpy as np

from .refelem import TET_EDGES

FACES = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))  # face i is opposite vertex i


class Numbering:
    def __init__(self, tet, region, n_vert, disp_order, pres_order):
        tet = np.asarray(tet, np.int64)
        region = np.asarray(region)
        self.T = tet.shape[0]
        self.V = int(n_vert)
        self.disp_order, self.pres_order = disp_order, pres_order
        need_edges = max(disp_order, pres_order) == 2
        if need_edges:
            e = np.concatenate([np.sort(tet[:, [a, b]], 1) for a, b in TET_EDGES])
            uniq, inv = np.unique(e, axis=0, return_inverse=True)
            self.edges = uniq
            tet_edge = inv.reshape(len(TET_EDGES), self.T).T + self.V
            self.geom = np.concatenate([tet, tet_edge], 1)  # [T,10]
        else:
            self.edges = np.zeros((0, 2), np.int64)
            self.geom = tet.copy()
        self.n_geom = self.V + len(self.edges)
        nd = 4 if disp_order == 1 else 10
        npp = 4 if pres_order == 1 else 10
        gdisp = self.geom[:, :nd]
        solid = region == 0
        fluid = ~solid
        has_s = np.zeros(self.n_geom, bool)
        has_f = np.zeros(self.n_geom, bool)
        has_s[np.unique(gdisp[solid])] = True
        has_f[np.unique(gdisp[fluid])] = True
        sid = np.full(self.n_geom, -1, np.int64)
        fid = np.full(self.n_geom, -1, np.int64)
        sid[has_s] = np.arange(has_s.sum())
        self.n_solid = int(has_s.sum())
        fid[has_f] = self.n_solid + np.arange(has_f.sum())
        self.N = self.n_solid + int(has_f.sum())
        self.sid, self.fid = sid, fid
        self.node_geom = np.concatenate([np.nonzero(has_s)[0], np.nonzero(has_f)[0]])
        self.elem_node = np.where(solid[:, None], sid[gdisp], fid[gdisp])  # [T,nd]
        # pressure nodes
        gp = self.geom[:, :npp]
        has_p = np.zeros(self.n_geom, bool)
        has_p[np.unique(gp[fluid])] = True
        pid = np.full(self.n_geom, -1, np.int64)
        pid[has_p] = np.arange(has_p.sum())
        self.n_pres = int(has_p.sum())
        self.pid = pid
        self.elem_pres = np.where(fluid[:, None], pid[gp], -1)
        self.region = region
        self.fs_faces = self._fs_faces(tet, region)

    @staticmethod
    def _fs_faces(tet, region):
        """Faces shared by a solid and a fluid tetrahedron:
        rows (solid tet, local face of the solid tet, fluid tet)."""
        T = tet.shape[0]
        keys, owner, lf = [], [], []
        for f, (a, b, c) in enumerate(FACES):
            keys.append(np.sort(tet[:, [a, b, c]], 1))
            owner.append(np.arange(T))
            lf.append(np.full(T, f))
        keys = np.concatenate(keys)
        owner = np.concatenate(owner)
        lf = np.concatenate(lf)
        order = np.lexsort((owner, keys[:, 2], keys[:, 1], keys[:, 0]))
        k = keys[order]
        same = np.all(k[1:] == k[:-1], axis=1)
        i = np.nonzero(same)[0]
        t0, t1 = owner[order][i], owner[order][i + 1]
        f0, f1 = lf[order][i], lf[order][i + 1]
        s0 = region[t0] == 0
        s1 = region[t1] == 0
        fs = s0 != s1
        st = np.where(s0, t0, t1)[fs]
        sf = np.where(s0, f0, f1)[fs]
        ft = np.where(s0, t1, t0)[fs]
        o = np.lexsort((sf, st))
        return np.stack([st[o], sf[o], ft[o]], 1)

    # ---------------------------------------------------------------- graphs
    @staticmethod
    def _csr_from_pairs(r, c, nrows):
        key = np.unique(r.astype(np.int64) * (1 << 32) + c.astype(np.int64))
        rows = key >> 32
        cols = (key & 0xFFFFFFFF).astype(np.int64)
        ptr = np.zeros(nrows + 1, np.int64)
        np.add.at(ptr, rows + 1, 1)
        return np.cumsum(ptr), cols

    def node_graph(self):
        en = self.elem_node
        nd = en.shape[1]
        r = np.repeat(en, nd, axis=1).ravel()
        c = np.tile(en, (1, nd)).ravel()
        diag = np.arange(self.N)
        return self._csr_from_pairs(np.concatenate([r, diag]), np.concatenate([c, diag]), self.N)

    def pres_graph(self):
        fl = self.region != 0
        ep = self.elem_pres[fl]
        k = ep.shape[1]
        r = np.repeat(ep, k, axis=1).ravel()
        c = np.tile(ep, (1, k)).ravel()
        diag = np.arange(self.n_pres)
        return self._csr_from_pairs(np.concatenate([r, diag]), np.concatenate([c, diag]), self.n_pres)

    def face_nodes(self, tet_id, local_face, order, kind):
        """Element-local node indices of a face (tri order: 3 vertices, then
        edges (0,1),(0,2),(1,2) of the face)."""
        a, b, c = FACES[local_face]
        loc = [a, b, c]
        if order == 2:
            eidx = {tuple(sorted(e)): 4 + i for i, e in enumerate(TET_EDGES)}
            loc += [eidx[tuple(sorted((a, b)))], eidx[tuple(sorted((a, c)))],
                    eidx[tuple(sorted((b, c)))]]
        return loc

    def eg_pattern(self):
        fl = np.nonzero(self.region != 0)[0]
        en = self.elem_node[fl]
        ep = self.elem_pres[fl]
        r = np.repeat(en, ep.shape[1], axis=1).ravel()
        c = np.tile(ep, (1, en.shape[1])).ravel()
        rs, cs = [r], [c]
        for st, sf, ft in self.fs_faces:
            un = self.elem_node[st][self.face_nodes(st, sf, self.disp_order, 'u')]
            # pressure nodes of the face, via geometric ids
            gface = self.geom[st][self.face_nodes(st, sf, self.pres_order, 'p')]
            pn = self.pid[gface]
            rs.append(np.repeat(un, len(pn)))
            cs.append(np.tile(pn, len(un)))
        return self._csr_from_pairs(np.concatenate(rs), np.concatenate(cs), self.N)
