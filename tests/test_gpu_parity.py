"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Integer work (numbering, CSR patterns) must match bit for bit; floating-point
results within tolerances derived from the arithmetic (stated per test)."""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import planet as make_planet
from oracle.assemble import Pencil as OPencil
from oracle import solve as S

pytestmark = pytest.mark.gpu

CASES = [
    ("homogeneous_ball", dict(n_half=4, order=1)),
    ("homogeneous_ball", dict(n_half=3, order=2)),
    ("three_layer_planet", dict(n_half=4, order=2, pres_order=1)),
    ("three_layer_planet", dict(n_half=3, order=2, pres_order=2)),
    ("three_layer_planet", dict(n_half=4, order=1, pres_order=1)),
]
IDS = ["ball-P1", "ball-P2", "layered-P2P1", "layered-P2P2", "layered-P1P1"]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


_PAIRS = {}


def pair(name, kw):
    import paper_1906_11082_amd as nm
    key = (name, tuple(sorted(kw.items())))
    if key not in _PAIRS:
        d = dict(make_planet(name, **kw))
        d["omega"] = (0.03, -0.02, 0.11)
        print("\n[case] %s %s" % (name, kw), flush=True)
        _PAIRS[key] = (nm.Pencil(d), OPencil(d), d)
    return _PAIRS[key]


def _csr(ptr, col, val, shape):
    return sp.csr_matrix((val, col, ptr), shape=shape)


@pytest.mark.parametrize("name,kw", CASES, ids=IDS)
def test_numbering_and_patterns_bit_exact(torch_cuda, name, kw):
    import paper_1906_11082_amd as nm
    G, O, d = pair(name, kw)
    nb = O.nb
    assert G.info["n_node"] == nb.N and G.info["n_solid"] == nb.n_solid
    assert G.info["n_pres"] == nb.n_pres and G.info["n_geom"] == nb.n_geom
    assert G.info["n_fs_faces"] == len(nb.fs_faces)
    ng, pgm = G.nodes()
    assert np.array_equal(ng, nb.node_geom)
    assert np.array_equal(pgm, np.nonzero(nb.pid >= 0)[0])
    ptr, col, _, _ = G.export_csr(nm.MAT_M)
    optr, ocol = nb.node_graph()
    assert np.array_equal(ptr, optr) and np.array_equal(col, ocol)
    if nb.n_pres:
        ptr, col, _, _ = G.export_csr(nm.MAT_KP)
        optr, ocol = nb.pres_graph()
        assert np.array_equal(ptr, optr) and np.array_equal(col, ocol)
        ptr, col, _, _ = G.export_csr(nm.MAT_EG)
        optr, ocol = nb.eg_pattern()
        rows = [col[ptr[3 * i]:ptr[3 * i + 1]] for i in range(nb.N)]
        orows = [ocol[optr[i]:optr[i + 1]] for i in range(nb.N)]
        assert all(np.array_equal(r, o) for r, o in zip(rows, orows))


@pytest.mark.parametrize("name,kw", CASES, ids=IDS)
def test_matrix_values(torch_cuda, name, kw):
    """Assembled values: every entry within 1e-13 of the largest entry of the
    matrix (sums of a handful of element terms in a different order)."""
    import paper_1906_11082_amd as nm
    G, O, d = pair(name, kw)
    for which, ref in [(nm.MAT_AG, O.AG), (nm.MAT_M, O.Ms), (nm.MAT_R, O.R)] + \
            ([(nm.MAT_KP, O.Kp), (nm.MAT_EG, O.EG)] if O.n_p else []):
        ptr, col, val, shape = G.export_csr(which)
        A = _csr(ptr, col, val, shape)
        diff = abs(A - ref).max()
        scale = abs(ref).max()
        assert diff <= 1e-13 * scale, (which, diff, scale)


def _rand(torch, rows, cols, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn(rows, cols, generator=g, dtype=torch.float64)


@pytest.mark.parametrize("name,kw", CASES, ids=IDS)
@pytest.mark.parametrize("ncols", [1, 5, 16])
def test_operators(torch_cuda, name, kw, ncols):
    """Sparse products and fixed-step Chebyshev-Jacobi solves equal the
    oracle's: per entry within 1e-12 of the result's largest entry."""
    torch = torch_cuda
    import paper_1906_11082_amd as nm
    G, O, d = pair(name, kw)
    X = _rand(torch, O.n, ncols, 1)
    Xd = X.cuda()
    x = X.numpy()

    def close(y, ref, tol=1e-12):
        y = y.cpu().numpy()
        assert np.abs(y - ref).max() <= tol * max(np.abs(ref).max(), 1e-300)

    close(G.apply(nm.OP_AG, Xd), O.AG @ x)
    close(G.apply(nm.OP_M, Xd), O.M @ x)
    close(G.apply(nm.OP_R, Xd), O.R @ x)
    lo, hi = S.jacobi_mass_bounds(O.order)
    for k in (2, 7, 30):
        ref = S.cheb_jacobi(lambda v: O.M @ v, np.repeat(O.Ms.diagonal(), 3), x, k, lo, hi)
        close(G.apply(nm.OP_MINV, Xd, kM=k), ref)
    if O.n_p:
        P = _rand(torch, O.n_p, ncols, 2)
        p = P.numpy()
        close(G.apply(nm.OP_EGT, Xd), O.EG.T @ x)
        close(G.apply(nm.OP_EG, P.cuda(), out_rows=O.n), O.EG @ p)
        close(G.apply(nm.OP_KP, P.cuda()), O.Kp @ p)
        plo, phi = S.jacobi_mass_bounds(O.porder)
        kp = lambda r, k: S.cheb_jacobi(lambda v: O.Kp @ v, O.Kp.diagonal(), r, k, plo, phi)
        close(G.apply(nm.OP_KPINV, P.cuda(), kP=9), kp(p, 9))
        refA = O.AG @ x + O.EG @ kp(O.EG.T @ x, 11)
        close(G.apply(nm.OP_A, Xd, kP=11), refA)
        close(G.apply(nm.OP_B, Xd, kP=11, kM=12),
              S.cheb_jacobi(lambda v: O.M @ v, np.repeat(O.Ms.diagonal(), 3), refA, 12, lo, hi))


@pytest.mark.parametrize("name,kw", CASES[:3], ids=IDS[:3])
@pytest.mark.parametrize("null", [False, True])
def test_filter_application(torch_cuda, name, kw, null):
    """One polynomial-filter application p(B) X (degree 25, 7 columns) against
    the oracle's recurrence with the same coefficients and inner steps:
    within 1e-11 of the result's largest entry."""
    torch = torch_cuda
    G, O, d = pair(name, kw)
    op = S.CowlingOperator(O)
    kM, kP = 14, 13
    op.kM = kM
    if O.n_p:
        plo, phi = S.jacobi_mass_bounds(O.porder)
        op.kp_solve = lambda r: S.cheb_jacobi(lambda v: O.Kp @ v, O.Kp.diagonal(), r, kP, plo, phi)
    lmax = 1.2 * S.lanczos_bounds(op, steps=30)[2]
    mu, c, e = S.filter_coeffs(2.0, 30.0, 0.0, lmax, 25)
    X = _rand(torch, O.n, 7, 3)
    kw2 = dict(null_shift=0.0, null_scale=30.0) if null else {}
    Y = G.filter_apply(mu, c, e, X.cuda(), kM=kM, kP=kP, **kw2).cpu().numpy()
    ref = S.filter_apply(op.B, X.numpy(), mu, c, e, **kw2)
    assert np.abs(Y - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("name,kw", CASES[:3], ids=IDS[:3])
def test_fp32_operators(torch_cuda, name, kw):
    """FP32 values, vectors and accumulation: relative error ~ 1e-6."""
    torch = torch_cuda
    import paper_1906_11082_amd as nm
    G, O, d = pair(name, kw)
    X = _rand(torch, O.n, 6, 4)
    x = X.numpy()
    y = G.apply(nm.OP_AG, X.float().cuda(), precision=1).double().cpu().numpy()
    ref = O.AG @ x
    assert np.abs(y - ref).max() <= 2e-5 * np.abs(ref).max()
    lo, hi = S.jacobi_mass_bounds(O.order)
    y = G.apply(nm.OP_MINV, X.float().cuda(), kM=20, precision=1).double().cpu().numpy()
    ref = S.cheb_jacobi(lambda v: O.M @ v, np.repeat(O.Ms.diagonal(), 3), x, 20, lo, hi)
    assert np.abs(y - ref).max() <= 2e-5 * np.abs(ref).max()


def test_assembly_is_deterministic(torch_cuda):
    import paper_1906_11082_amd as nm
    d = dict(make_planet("three_layer_planet", n_half=4, order=2))
    A1 = nm.Pencil(d).export_csr(nm.MAT_AG)
    A2 = nm.Pencil(d).export_csr(nm.MAT_AG)
    for a, b in zip(A1[:3], A2[:3]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("ncols", [3, 8, 16, 32])
def test_row_group_kernel_matches_per_row(torch_cuda, ncols, monkeypatch):
    """The row-group mass-solve kernel (4 or 8 consecutive internal rows per lane, union
    columns with zero-padded coefficients) and the LDS-tile kernel (32 or 64
    rows per tile, 128- or 64-byte row chunks) sum each row in the same
    column order as the per-row kernel: FP64 and FP32 results are
    bit-identical, including the ragged last group and tile."""
    torch = torch_cuda
    import paper_1906_11082_amd as nm
    d = dict(make_planet("three_layer_planet", n_half=5, order=2, pres_order=1))
    pens = {}
    for tag, on, R, tiles, tr in (("row", "0", "4", "0", "32"), ("g4", "2", "4", "0", "32"),
                                  ("g8", "2", "8", "0", "32"), ("t32", "0", "4", "1", "32"),
                                  ("t64", "0", "4", "1", "64")):
        monkeypatch.setenv("NM_ROW_GROUPS", on)
        monkeypatch.setenv("NM_GROUP_ROWS", R)
        monkeypatch.setenv("NM_TILES", tiles)
        monkeypatch.setenv("NM_TILE_ROWS", tr)
        pens[tag] = nm.Pencil(d)
    N = pens["row"].info["n_node"]
    assert N % 4 != 0 or N % 8 != 0
    X = _rand(torch, pens["row"].info["n_disp"], ncols, 5).cuda()
    mu = nm.filter_coeffs(2.0, 30.0, 0.0, 4.0e3, 9)
    c, e = 2.0e3, 2.0e3
    ref_m = pens["row"].apply(nm.OP_MINV, X, kM=17)
    ref_f = pens["row"].filter_apply(mu, c, e, X, kM=6, kP=5)
    X32 = X.float()
    ref_32 = pens["row"].apply(nm.OP_MINV, X32, kM=17, precision=1)
    N = pens["row"].info["n_node"]
    assert N % 64 != 0
    for tag in ("g4", "g8", "t32", "t64"):
        assert torch.equal(pens[tag].apply(nm.OP_MINV, X, kM=17), ref_m), tag
        assert torch.equal(pens[tag].filter_apply(mu, c, e, X, kM=6, kP=5), ref_f), tag
        assert torch.equal(pens[tag].apply(nm.OP_MINV, X32, kM=17, precision=1), ref_32), tag
