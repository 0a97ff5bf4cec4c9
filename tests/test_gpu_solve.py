"""GPU eigensolves against the oracle's reference solutions."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from conftest import planet as make_planet
from oracle.assemble import Pencil as OPencil
from oracle import solve as S
from oracle import rotation as RT

pytestmark = pytest.mark.gpu


def _clusters(w, rel=1e-6):
    groups, cur = [], [0]
    for i in range(1, len(w)):
        if w[i] - w[i - 1] <= rel * abs(w[i]):
            cur.append(i)
        else:
            groups.append(cur)
            cur = [i]
    groups.append(cur)
    return groups


def _check_vectors(X, Xref, M, w):
    """Eigenvectors: per cluster of (near-)equal eigenvalues the M-orthogonal
    projectors agree (any orthonormal basis of a cluster is correct)."""
    for g in _clusters(w):
        if len(g) and g[-1] == len(w) - 1:
            continue  # the last cluster may be cut by nev
        A, B = X[:, g], Xref[:, g]
        s = np.linalg.svd(A.T @ (M @ B), compute_uv=False)
        assert s.min() > 1 - 1e-7, (g, s)


def test_c1_ball_matches_dense():
    """Homogeneous ball, P1, ~3k tets: lowest 30 pairs in [0.5, 40] with the
    degree-40 filter; eigenvalues within 1e-10 relative, residuals <= 1e-10."""
    import paper_1906_11082_amd as nm
    d = make_planet("homogeneous_ball", n_half=4, order=1)
    print("\n[case] C1 ball", flush=True)
    G = nm.Pencil(d)
    r = G.filtered_eig(0.5, 40.0, 30, 1e-10, degree=40, block=8)
    O = OPencil(d)
    A, M = O.AG.toarray(), O.M.toarray()
    w, Xr = S.dense_window(A, M, 0.5, 40.0)
    assert r.count == 30
    assert np.abs(r.lam - w[:30]).max() <= 1e-10 * w[29]
    assert r.resid.max() <= 1e-10
    X = r.X.cpu().numpy()
    np.testing.assert_allclose(X.T @ M @ X, np.eye(30), atol=1e-9)
    _check_vectors(X, Xr[:, :30], O.M, w[:30])


def _cowling_reference(O, sigma, k):
    """Eigenvalues of the Cowling pencil nearest sigma: ARPACK shift-invert
    (scipy eigsh), the shifted solve done exactly by a sparse LU of the
    saddle-point system [[A_G - s M, E_G], [E_G^T, -K_p]] (exact Schur
    complement)."""
    n, n_p = O.n, O.n_p
    K = sp.bmat([[O.AG - sigma * O.M, O.EG], [O.EG.T, -O.Kp]], format="csc")
    lu = spla.splu(K)
    kp = O.kp_direct()
    Aop = spla.LinearOperator((n, n), matvec=lambda x: O.cowling_apply(x, kp), dtype=float)
    Sop = spla.LinearOperator((n, n), matvec=lambda f: lu.solve(np.concatenate([f, np.zeros(n_p)]))[:n],
                              dtype=float)
    lam, V = spla.eigsh(Aop, k=k, M=O.M, sigma=sigma, OPinv=Sop, which="LM", tol=1e-13)
    order = np.argsort(lam)
    return lam[order], V[:, order]


def test_layered_cowling_matches_shift_invert():
    """Three-layer planet (solid/fluid/solid), P2 displacement + P1 pressure,
    gravity, Cowling: all pairs in [1, 12] within 1e-9 relative of the
    oracle's exact-Schur shift-invert solution."""
    import paper_1906_11082_amd as nm
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    print("\n[case] layered P2/P1 n_half=4", flush=True)
    G = nm.Pencil(d)
    r = G.filtered_eig(1.0, 12.0, 200, 1e-9, block=8, verbose=1)
    O = OPencil(d)
    lam, _ = _cowling_reference(O, 6.0, min(3 * max(r.count, 10), 80))
    ref = lam[(lam >= 1.0) & (lam <= 12.0)]
    assert r.count == len(ref) and r.count > 0
    assert np.abs(r.lam - ref).max() <= 1e-9 * ref.max()
    assert r.resid.max() <= 1e-9


def test_fp32_filter_refined_to_fp64_accuracy():
    """FP32 filter (values, vectors, accumulation) + FP64 Lanczos, Rayleigh-Ritz
    and low-pass refinement: residual <= 1e-8 and eigenvalues within 1e-8
    relative of the FP64 solve; without the refinement the FP32 residual
    floor is higher."""
    import paper_1906_11082_amd as nm
    d = make_planet("homogeneous_ball", n_half=4, order=1)
    G = nm.Pencil(d)
    r64 = G.filtered_eig(0.5, 40.0, 30, 1e-10, degree=40, block=8)
    r32 = G.filtered_eig(0.5, 40.0, 30, 1e-8, degree=40, block=8, precision=1)
    print("fp32 refined: resid max %.2e passes %d degree %d" % (r32.resid.max(), r32.stats["refine_passes"],
                                                               r32.stats["refine_degree"]), flush=True)
    assert r32.count == 30 and r32.stats["refine_passes"] >= 1
    assert r32.resid.max() <= 1e-8
    assert np.abs(r32.lam - r64.lam).max() <= 1e-8 * r64.lam.max()
    O = OPencil(d)
    X32, X64 = r32.X.cpu().numpy(), r64.X.cpu().numpy()
    for g in _clusters(r64.lam):
        if g[-1] == 29:
            continue
        sv = np.linalg.svd(X32[:, g].T @ (O.M @ X64[:, g]), compute_uv=False)
        assert sv.min() > 1 - 1e-6, (g, sv)
    raw = G.filtered_eig(0.5, 40.0, 30, 1e-8, degree=40, block=8, precision=1, refine=-1, allow_partial=True)
    print("fp32 unrefined: resid max %.2e" % raw.resid.max(), flush=True)
    assert raw.stats["refine_passes"] == 0 and raw.resid.max() > r32.resid.max()


def test_fp32_layered_cowling_refined():
    """Three-layer planet, P2/P1, Cowling: the FP32-filter path with FP64
    refinement finds all pairs in [1, 12] within 1e-8 relative of the exact-Schur
    shift-invert reference, residuals <= 1e-8."""
    import paper_1906_11082_amd as nm
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    print("\n[case] layered P2/P1 n_half=4 FP32 filter", flush=True)
    G = nm.Pencil(d)
    r = G.filtered_eig(1.0, 12.0, 200, 1e-8, block=8, precision=1, verbose=1)
    O = OPencil(d)
    lam, _ = _cowling_reference(O, 6.0, min(3 * max(r.count, 10), 80))
    ref = lam[(lam >= 1.0) & (lam <= 12.0)]
    assert r.count == len(ref) and r.count > 0
    assert np.abs(r.lam - ref).max() <= 1e-8 * ref.max()
    assert r.resid.max() <= 1e-8


def test_rotation_projection_matches_oracle():
    """Projected Coriolis problem from the GPU basis: the oracle's projection
    of the same basis gives the same frequencies (1e-12), and R = 0 gives
    omega = sqrt(lambda)."""
    import paper_1906_11082_amd as nm
    d = dict(make_planet("homogeneous_ball", n_half=4, order=1))
    d["omega"] = (0.0, 0.0, 0.2)
    G = nm.Pencil(d)
    r = G.filtered_eig(0.5, 40.0, 30, 1e-10, degree=40, block=8)
    rot = G.project_rotation(r, 4.0, 36.0)
    O = OPencil(d)
    X = r.X.cpu().numpy()
    om, U, _ = RT.project_rotation(r.lam, X, lambda V: O.R @ V, 4.0, 36.0)
    assert rot.count == len(om)
    assert np.abs(rot.omega - np.sort(om)).max() <= 1e-12 * om.max()
    Ug = rot.U.cpu().numpy()
    Mx = O.M
    Gm = Ug.conj().T @ (Mx @ Ug) - 2j * (Ug.conj().T @ (O.R @ Ug)) / (rot.omega[:, None] + rot.omega[None, :])
    np.testing.assert_allclose(Gm, np.eye(rot.count), atol=1e-9)
    d0 = dict(d, omega=(0.0, 0.0, 0.0))
    G0 = nm.Pencil(d0)
    r0 = G0.filtered_eig(0.5, 40.0, 30, 1e-10, degree=40, block=8)
    rot0 = G0.project_rotation(r0, 0.5, 40.0)
    assert np.abs(rot0.omega - np.sqrt(r0.lam)).max() <= 1e-13 * np.sqrt(r0.lam).max()


def test_empty_window_returns_no_pairs():
    import paper_1906_11082_amd as nm
    d = make_planet("homogeneous_ball", n_half=3, order=1)
    G = nm.Pencil(d)
    r = G.filtered_eig(0.01, 0.05, 5, 1e-8, degree=30, block=4, max_basis=40, allow_partial=True)
    assert r.count == 0


@pytest.mark.parametrize("mass_passes", [0, 2])
def test_slices_batched_equal_alone(mass_passes):
    """Spectrum slicing with shared filter applications: two windows solved
    together (one Lanczos per window, their filter blocks concatenated with
    one Chebyshev series per column) give bit-identical eigenvalues to each
    window solved alone with the same bounds and start block; also with the
    mass solve in FP32 passes."""
    import paper_1906_11082_amd as nm
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    print("\n[case] slices layered P2/P1 n_half=4, mass_passes %d" % mass_passes, flush=True)
    G = nm.Pencil(d)
    lo, hi = G.spectrum_bounds()
    lmin, lmax = lo - 0.01, hi
    wins = [(1.0, 6.0), (6.0, 12.0)]
    rs = G.filtered_eig_slices(wins, 100, 1e-9, block=8, lmin=lmin, lmax=lmax, seed=7, mass_passes=mass_passes)
    assert len(rs) == 2
    for i, (a, b) in enumerate(wins):
        seed_i = (7 + 0x9E3779B97F4A7C15 * (i + 1)) % (1 << 64)
        r1 = G.filtered_eig(a, b, 100, 1e-9, block=8, lmin=lmin, lmax=lmax, seed=seed_i, mass_passes=mass_passes)
        assert r1.stats["mass_passes"] == rs[i].stats["mass_passes"] == mass_passes
        print("slice %d: %d pairs, batched degree %d, alone degree %d" % (i, r1.count, rs[i].stats["degree"],
                                                                        r1.stats["degree"]), flush=True)
        assert r1.count == rs[i].count > 0
        assert np.array_equal(r1.lam, rs[i].lam)
        assert np.array_equal(r1.resid, rs[i].resid)
        assert rs[i].resid.max() <= 1e-9
    # together the windows cover [1, 12] once
    allw = np.concatenate([r.lam for r in rs])
    ref = G.filtered_eig(1.0, 12.0, 200, 1e-9, block=8, lmin=lmin, lmax=lmax)
    assert len(allw) == ref.count
    assert np.abs(np.sort(allw) - ref.lam).max() <= 1e-9 * ref.lam.max()


def test_autotune_picks_a_block_and_solves():
    """The autotuner times the mass-solve step for block widths 8..64 and both
    kernels; the solve then uses the chosen width and finds the same pairs."""
    import paper_1906_11082_amd as nm
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    G = nm.Pencil(d)
    ref = G.filtered_eig(1.0, 12.0, 200, 1e-9, block=8)
    blk, us = G.autotune(0)
    print("autotune: block %d, %.3f us per column-step" % (blk, us), flush=True)
    assert blk in (8, 16, 32, 64) and us > 0
    r = G.filtered_eig(1.0, 12.0, 200, 1e-9, verbose=1)
    assert r.stats["block"] == min(blk, 48)  # capped at nev / 4 in multiples of 8
    assert r.count == ref.count
    assert np.abs(r.lam - ref.lam).max() <= 1e-9 * ref.lam.max()


def test_autotune_times_group_sizes_and_keeps_fp32_coefficients(capfd, monkeypatch):
    """The FP32 autotuner also times row groups of 4 and 8 rows (the block
    size of the grouped format), rebuilding the groups and their FP32
    coefficients as it goes; afterwards the mixed-precision mass solve at 32
    columns (the grouped kernel with whatever group size won) still equals the
    per-row FP32 passes bit for bit (and the FP64 solve within the passes'
    error bound, (2 r^12)^2 = 3.2e-5 in the M-norm)."""
    import torch
    import paper_1906_11082_amd as nm
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    monkeypatch.setenv("NM_ROW_GROUPS", "0")
    P0 = nm.Pencil(d)
    rng = np.random.default_rng(3)
    F = torch.from_numpy(rng.standard_normal((P0.n, 32))).cuda()
    Y_row = P0.apply(nm.OP_MINV, F, kM=12, mass_passes=2).cpu().numpy()
    monkeypatch.delenv("NM_ROW_GROUPS")
    G = nm.Pencil(d)
    Y64 = G.apply(nm.OP_MINV, F, kM=40).cpu().numpy()
    monkeypatch.setenv("NM_AUTOTUNE_VERBOSE", "1")
    blk, us = G.autotune(1)
    err = capfd.readouterr().err
    print(err, flush=True)
    for rows in (4, 8):
        for pe in (0, 1):
            assert "kernel=group tile_rows=0 group_rows=%d persistent=%d" % (rows, pe) in err
    Y = G.apply(nm.OP_MINV, F, kM=12, mass_passes=2).cpu().numpy()
    assert np.array_equal(Y, Y_row)
    assert np.abs(Y - Y64).max() <= 1e-3 * np.abs(Y64).max()


def test_persistent_group_step_equals_one_launch_per_share(monkeypatch):
    """The persistent form of the row-group step (as many workgroups as the
    GPU holds, each sweeping its XCD's shares in order) computes every share
    exactly as the one-workgroup-per-share launch: FP64 and mixed mass solves
    at 32 and 64 columns on the 83k-tet planet (2,877 and 5,753 shares, more
    than the persistent grid holds, so workgroups take several) and a whole
    mixed-precision solve on a small planet are bit-identical."""
    import torch
    import paper_1906_11082_amd as nm
    big = make_planet("three_layer_planet", n_half=12, order=2, pres_order=1)
    small = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    rng = np.random.default_rng(5)
    out = {}
    for persist in ("0", "1"):
        monkeypatch.setenv("NM_PERSIST", persist)
        G = nm.Pencil(big)
        for b in (32, 64):
            if persist == "0":
                out[("F", b)] = rng.standard_normal((G.n, b))
            F = torch.from_numpy(out[("F", b)]).cuda()
            out[(persist, b, "fp64")] = G.apply(nm.OP_MINV, F, kM=14).cpu().numpy()
            out[(persist, b, "mixed")] = G.apply(nm.OP_MINV, F, kM=12, mass_passes=2).cpu().numpy()
        del G
        r = nm.Pencil(small).filtered_eig(1.0, 12.0, 200, 1e-9, block=32, mass_passes=2)
        out[(persist, "lam")] = r.lam
    for b in (32, 64):
        for leg in ("fp64", "mixed"):
            assert np.array_equal(out[("0", b, leg)], out[("1", b, leg)]), (b, leg)
    assert np.array_equal(out[("0", "lam")], out[("1", "lam")])


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replayed_filter_equals_eager(monkeypatch, precision):
    """Small problems capture one filter application in a HIP graph and replay
    it for every Lanczos block, with the orthogonalisation and Rayleigh-Ritz
    running eagerly between the replays: the solve is bit-identical to the
    eager one."""
    import paper_1906_11082_amd as nm
    d = make_planet("homogeneous_ball", n_half=4, order=1)
    G = nm.Pencil(d)
    out = {}
    for g in ("0", "1"):
        monkeypatch.setenv("NM_GRAPH", g)
        out[g] = G.filtered_eig(0.5, 40.0, 30, 1e-9, degree=40, block=8, precision=precision)
    assert out["1"].count == out["0"].count == 30
    assert np.array_equal(out["1"].lam, out["0"].lam)
    assert np.array_equal(out["1"].X.cpu().numpy(), out["0"].X.cpu().numpy())
    assert out["1"].stats["basis"] >= 24  # several blocks, so several replays


def test_blow_up_restarts_with_a_larger_bound():
    """A spectrum bound lambda_max far below the spectrum makes the filtered
    vectors blow up; the solve restarts on an enlarged interval and finds the
    same pairs as the dense oracle."""
    import paper_1906_11082_amd as nm
    d = make_planet("homogeneous_ball", n_half=4, order=1)
    G = nm.Pencil(d)
    r = G.filtered_eig(0.5, 40.0, 30, 1e-10, degree=40, block=8, lmin=-0.01, lmax=100.0, verbose=1)
    O = OPencil(d)
    w, _ = S.dense_window(O.AG.toarray(), O.M.toarray(), 0.5, 40.0)
    assert r.count == 30 and r.stats["lmax"] > 1000.0
    assert np.abs(r.lam - w[:30]).max() <= 1e-10 * w[29]


@pytest.mark.parametrize("case", ["ball", "layered"])
def test_rigorous_spectrum_bound(case):
    """The Gershgorin bound of nm_spectrum_bound_rigorous lies above every
    eigenvalue of the pencil (the oracle's dense solve) and within a small
    factor of the largest; the Lanczos estimate lies between them."""
    import scipy.linalg as sla
    import paper_1906_11082_amd as nm
    if case == "ball":
        d = make_planet("homogeneous_ball", n_half=3, order=2)
    else:
        d = make_planet("three_layer_planet", n_half=3, order=2, pres_order=1)
    G = nm.Pencil(d)
    O = OPencil(d)
    A = O.cowling_dense() if O.n_p else O.AG.toarray()
    lam_max = sla.eigh(A, O.M.toarray(), eigvals_only=True)[-1]
    bound = G.spectrum_bound_rigorous()
    lo, est = G.spectrum_bounds(80, 3)
    print("%s: lambda_max %.6g, Lanczos estimate %.6g, rigorous bound %.6g (x%.2f)"
          % (case, lam_max, est, bound, bound / lam_max), flush=True)
    assert bound >= lam_max * (1 - 1e-12)
    assert bound <= 20 * lam_max
    assert lam_max * (1 - 1e-6) <= est <= bound
