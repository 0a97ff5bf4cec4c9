"""Self-gravitation on the GPU (N-body sums, FP32 pair terms with FP64
accumulation) against the oracle's FP64 operators."""
import numpy as np
import pytest

from conftest import planet as make_planet

pytestmark = pytest.mark.gpu


def _planets():
    return [("homogeneous_ball", dict(n_half=3, order=2)), ("three_layer_planet", dict(n_half=3, order=2, pres_order=1))]


@pytest.mark.parametrize("case", [0, 1])
def test_selfgrav_operator_matches_oracle(case):
    """-C^T S C X on the GPU equals the oracle's to 1e-5 (relative, per column;
    FP32 pair terms), with the same bodies and self-terms (1e-12)."""
    import torch
    import paper_1906_11082_amd as nm
    from oracle.assemble import Pencil as OPencil
    from oracle import selfgrav as SG
    name, kw = _planets()[case]
    d = make_planet(name, **kw)
    G = nm.Pencil(d)
    sg = nm.SelfGravity(G, d)
    O = OPencil(d)
    so = SG.SelfGravity(O)
    assert (sg.n_tet, sg.n_face) == (so.n_tet, so.n_face)
    ir = sg.inv_R()
    assert np.abs(ir[:sg.n_tet] - so.inv_R[:so.n_tet]).max() <= 1e-12 * so.inv_R.max()
    assert np.abs(np.sort(ir[sg.n_tet:]) - np.sort(so.inv_R[so.n_tet:])).max() <= 1e-12 * so.inv_R.max()
    X = np.random.default_rng(4).standard_normal((O.n, 5))
    Y = sg.apply(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = so.apply(X)
    err = (np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)).max()
    print("%s: bodies %d (%d faces), max rel column error %.2e" % (name, sg.n_body, sg.n_face, err), flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("kernel", ["simple", "split"])
def test_nbody_kernels_match_oracle(monkeypatch, kernel):
    """Both N-body kernels (one target per lane; the default: two per lane
    with LDS-staged sources split into runs over several workgroups and
    reduced in order) on 5, 8, 12 and 16 columns (whole and partial column
    groups, several workgroups of targets, a partial last source tile, 16 to
    4 source runs) equal the oracle's operator to 1e-5."""
    import torch
    import paper_1906_11082_amd as nm
    from oracle.assemble import Pencil as OPencil
    from oracle import selfgrav as SG
    monkeypatch.setenv("NM_NBODY", kernel)
    d = make_planet("three_layer_planet", n_half=3, order=2, pres_order=1)
    G = nm.Pencil(d)
    sg = nm.SelfGravity(G, d)
    so = SG.SelfGravity(OPencil(d))
    assert sg.n_body > 512 and sg.n_body % 256
    for nc in (5, 8, 12, 16):
        X = np.random.default_rng(nc).standard_normal((G.n, nc))
        Y = sg.apply(torch.from_numpy(X).cuda()).cpu().numpy()
        ref = so.apply(X)
        err = (np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)).max()
        print("%s, %d columns: max rel column error %.2e" % (kernel, nc, err), flush=True)
        assert err <= 1e-5


def test_reference_field_matches_oracle():
    """g at the vertices from the element masses: GPU (FP32 pairs) equals the
    oracle's FP64 sums to 1e-5 of the largest."""
    import torch
    import paper_1906_11082_amd as nm
    from oracle.assemble import Pencil as OPencil
    from oracle import selfgrav as SG
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    G = nm.Pencil(d)
    sg = nm.SelfGravity(G, d)
    so = SG.SelfGravity(OPencil(d))
    x = np.asarray(d["xyz"])
    g = sg.field(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = so.reference_field(x)
    assert np.abs(g - ref).max() <= 1e-5 * np.abs(ref).max()


def test_self_gravitating_solve_matches_dense():
    """Three-layer planet (P1/P1, Cowling pencil plus self-gravitation, eq.
    "eigfull" without rotation): the filtered Lanczos on the GPU with the
    N-body term attached finds the eigenvalues of the dense oracle pencil
    (A_G + E_G K_p^-1 E_G^T - C^T S C, M) in the window to 1e-6 (FP32 pairs)."""
    import paper_1906_11082_amd as nm
    from oracle.assemble import Pencil as OPencil
    from oracle import selfgrav as SG
    from oracle import solve as S
    d = make_planet("three_layer_planet", n_half=3, order=1, pres_order=1)
    G = nm.Pencil(d)
    sg = nm.SelfGravity(G, d)
    sg.attach()
    r = G.filtered_eig(2.0, 30.0, 200, 1e-6, block=8, allow_partial=True)
    O = OPencil(d)
    so = SG.SelfGravity(O)
    Cd = so.C.toarray()
    A = O.cowling_dense() - Cd.T @ so.S_dense() @ Cd
    w, _ = S.dense_window(0.5 * (A + A.T), O.M.toarray(), 2.0, 30.0)
    print("self-gravitating: %d pairs (dense %d), resid max %.2e" % (r.count, len(w), r.resid.max()), flush=True)
    assert r.count == len(w) > 10
    assert np.abs(r.lam - w).max() <= 1e-6 * w.max()
    sg.attach(False)
