"""Pins of the oracle's numbering and patterns against brute force."""
import itertools

import numpy as np
import pytest

from conftest import planet
from oracle.mesh import Numbering, FACES
from oracle.assemble import tet_geometry
from oracle.refelem import TET_EDGES


def _brute(d, order, porder):
    tet = [tuple(int(v) for v in t) for t in d["tet"]]
    reg = [int(r) for r in d["region"]]
    V = len(d["xyz"])
    edges = sorted({tuple(sorted((t[a], t[b]))) for t in tet for a, b in TET_EDGES}) if max(order, porder) == 2 else []
    eid = {e: V + i for i, e in enumerate(edges)}

    def gnodes(t, o):
        g = list(t)
        if o == 2:
            g += [eid[tuple(sorted((t[a], t[b])))] for a, b in TET_EDGES]
        return g

    solid_g = sorted({g for t, r in zip(tet, reg) if r == 0 for g in gnodes(t, order)})
    fluid_g = sorted({g for t, r in zip(tet, reg) if r == 1 for g in gnodes(t, order)})
    sid = {g: i for i, g in enumerate(solid_g)}
    fid = {g: len(solid_g) + i for i, g in enumerate(fluid_g)}
    node = lambda g, r: sid[g] if r == 0 else fid[g]
    pres_g = sorted({g for t, r in zip(tet, reg) if r == 1 for g in gnodes(t, porder)})
    pid = {g: i for i, g in enumerate(pres_g)}
    N = len(solid_g) + len(fluid_g)
    graph = {(i, i) for i in range(N)}
    for t, r in zip(tet, reg):
        ns = [node(g, r) for g in gnodes(t, order)]
        graph |= {(i, j) for i in ns for j in ns}
    # fluid-solid faces
    fmap = {}
    for k, t in enumerate(tet):
        for f, (a, b, c) in enumerate(FACES):
            fmap.setdefault(tuple(sorted((t[a], t[b], t[c]))), []).append(k)
    fs = [ks for ks in fmap.values() if len(ks) == 2 and reg[ks[0]] != reg[ks[1]]]
    eg = set()
    for t, r in zip(tet, reg):
        if r == 1:
            eg |= {(node(g, 1), pid[p]) for g in gnodes(t, order) for p in gnodes(t, porder)}
    for ks in fs:
        s = ks[0] if reg[ks[0]] == 0 else ks[1]
        fv = set(tet[ks[0]]) & set(tet[ks[1]])
        gs = [g for g in gnodes(tet[s], order)
              if g in fv or (g >= V and set(edges[g - V]) <= fv)]
        ps = [g for g in gnodes(tet[s], porder)
              if g in fv or (g >= V and set(edges[g - V]) <= fv)]
        eg |= {(node(g, 0), pid[p]) for g in gs for p in ps}
    pg_ = set()
    for t, r in zip(tet, reg):
        if r == 1:
            ps = [pid[g] for g in gnodes(t, porder)]
            pg_ |= {(i, j) for i in ps for j in ps}
    return dict(N=N, ns=len(solid_g), np=len(pres_g), graph=graph, eg=eg, pgraph=pg_, nfs=len(fs))


def _pairs(ptr, col):
    return {(i, int(c)) for i in range(len(ptr) - 1) for c in col[ptr[i]:ptr[i + 1]]}


@pytest.mark.parametrize("order,porder", [(1, 1), (2, 1), (2, 2)])
def test_numbering_matches_brute_force(order, porder):
    d = planet("three_layer_planet", n_half=3, order=order, pres_order=porder)
    nb = Numbering(d["tet"], d["region"], len(d["xyz"]), order, porder)
    bf = _brute(d, order, porder)
    assert nb.N == bf["N"] and nb.n_solid == bf["ns"] and nb.n_pres == bf["np"]
    ptr, col = nb.node_graph()
    assert _pairs(ptr, col) == bf["graph"]
    assert all(np.all(np.diff(col[ptr[i]:ptr[i + 1]]) > 0) for i in range(nb.N))
    ptr, col = nb.eg_pattern()
    assert _pairs(ptr, col) == bf["eg"]
    ptr, col = nb.pres_graph()
    assert _pairs(ptr, col) == bf["pgraph"]
    assert len(nb.fs_faces) == bf["nfs"]


def test_fs_faces_are_solid_fluid():
    d = planet("three_layer_planet", n_half=4, order=2)
    nb = Numbering(d["tet"], d["region"], len(d["xyz"]), 2, 1)
    tet = d["tet"]
    for st, sf, ft in nb.fs_faces:
        assert d["region"][st] == 0 and d["region"][ft] == 1
        fv = {int(tet[st][q]) for q in FACES[sf]}
        assert fv <= set(int(v) for v in tet[ft])


def test_volume_divergence_theorem():
    """Sum of |K| equals the volume enclosed by the boundary triangulation
    (divergence theorem, (1/3) sum over boundary faces of x . n dA)."""
    d = planet("three_layer_planet", n_half=6, order=1)
    xyz, tet = d["xyz"], d["tet"]
    vol, _ = tet_geometry(xyz, tet)
    faces = {}
    for k, t in enumerate(tet):
        for f, (a, b, c) in enumerate(FACES):
            key = tuple(sorted((t[a], t[b], t[c])))
            faces.setdefault(key, []).append((k, f))
    V = 0.0
    for key, occ in faces.items():
        if len(occ) == 1:
            k, f = occ[0]
            a, b, c = (xyz[tet[k][q]] for q in FACES[f])
            o = xyz[tet[k][f]]
            n = np.cross(b - a, c - a)
            if np.dot(n, a - o) < 0:
                n = -n
            V += np.dot(a, n) / 6.0
    assert abs(vol.sum() - V) < 1e-12 * V
    assert abs(V - 4 * np.pi / 3) < 0.03 * 4 * np.pi / 3
