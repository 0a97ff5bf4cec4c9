"""Mass solve in FP32 Chebyshev-Jacobi passes with FP64 residual corrections
(mass_passes): against the same refinement written out with the FP64 solve,
against an FP64 filter, and in a full solve against the FP64 solve."""
import numpy as np
import pytest

from conftest import planet as make_planet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def layered():
    import torch
    import paper_1906_11082_amd as nm
    d = make_planet("three_layer_planet", n_half=4, order=2, pres_order=1)
    print("\n[case] layered P2/P1 n_half=4, mixed mass solve", flush=True)
    return torch, nm, d, nm.Pencil(d)


def _rand(torch, n, b, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn(n, b, generator=g, dtype=torch.float64).cuda()


def _rate(G):
    kap = G.info["minv_hi"] / G.info["minv_lo"]
    return (np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)


@pytest.mark.parametrize("passes,k,ncols", [(2, 12, 12), (3, 9, 12), (4, 7, 12), (2, 12, 5)])
def test_mixed_solve_is_the_refinement_of_the_fp64_solve(layered, passes, k, ncols):
    """P FP32 passes of k steps equal, up to FP32 rounding of the corrections,
    y <- y + S(f - M y) repeated P times from y = 0 with S the k-step FP64
    solve; the rounding left is that of one FP32 pass times the error factor
    of the passes after it.  Both are within the refinement's bound of M^-1 f.
    5 columns: rows of 15 entries (one entry per lane)."""
    torch, nm, d, G = layered
    n = G.info["n_disp"]
    F = _rand(torch, n, ncols, 5 + passes)
    Y = G.apply(nm.OP_MINV, F, kM=k, mass_passes=passes)
    y = torch.zeros_like(F)
    for _ in range(passes):
        y = y + G.apply(nm.OP_MINV, F - G.apply(nm.OP_M, y), kM=k)
    fac = 2 * _rate(G) ** k
    rel = ((Y - y).norm(dim=0) / y.norm(dim=0)).max().item()
    print("passes %d k %d: |mixed - fp64 refinement| %.2e (factor %.2e)" % (passes, k, rel, fac), flush=True)
    assert rel <= 1e-5 * fac ** (passes - 1)
    exact = G.apply(nm.OP_MINV, F, kM=90)
    err = ((Y - exact).norm(dim=0) / exact.norm(dim=0)).max().item()
    assert err <= 100 * fac ** passes


def test_mixed_solve_matches_oracle_refinement(layered):
    """The GPU passes against the oracle's refinement of its own Chebyshev-Jacobi
    solve on the same planet and right-hand sides: within 1e-5 of the pass
    factor of the FP64 definition (the FP32 rounding of the second pass's
    correction), and as close to the oracle's float32-pass model."""
    torch, nm, d, G = layered
    from oracle.assemble import Pencil as OPencil
    from oracle import solve as S
    O = OPencil(d)
    lo, hi = S.jacobi_mass_bounds(2)
    assert abs(lo - G.info["minv_lo"]) <= 1e-14 and abs(hi - G.info["minv_hi"]) <= 1e-12
    F = np.random.default_rng(11).standard_normal((O.n, 8))
    Y = G.apply(nm.OP_MINV, torch.from_numpy(F).cuda(), kM=12, mass_passes=2).cpu().numpy()
    dg = np.repeat(O.Ms.diagonal(), 3)
    ref = S.cheb_jacobi_refined(lambda x: O.M @ x, dg, F, 12, lo, hi, 2)
    M32 = O.M.astype(np.float32)
    ref32 = S.cheb_jacobi_refined(lambda x: O.M @ x, dg, F, 12, lo, hi, 2, Mop32=lambda x: M32 @ x)
    fac = 2 * _rate(G) ** 12
    rel = (np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)).max()
    rel32 = (np.linalg.norm(Y - ref32, axis=0) / np.linalg.norm(ref, axis=0)).max()
    print("oracle: |gpu - fp64 refinement| %.2e, |gpu - float32-pass model| %.2e" % (rel, rel32), flush=True)
    assert rel <= 1e-5 * fac and rel32 <= 1e-5 * fac


def test_mixed_filter_matches_fp64_filter(layered):
    """A degree-8 filter with the mixed solve (2 passes of 20 steps, bound
    1.3e-8) against the FP64 filter with a 90-step FP64 solve."""
    torch, nm, d, G = layered
    n = G.info["n_disp"]
    lo, hi = G.spectrum_bounds()
    mu = nm.filter_coeffs(1.0, 12.0, lo, hi, 8)
    c, e = 0.5 * (hi + lo), 0.5 * (hi - lo)
    X = _rand(torch, n, 8, 21)
    Ym = G.filter_apply(mu, c, e, X, kM=20, mass_passes=2)
    Y64 = G.filter_apply(mu, c, e, X, kM=90)
    rel = ((Ym - Y64).norm(dim=0) / Y64.norm(dim=0)).max().item()
    print("filter: |mixed - fp64| %.2e" % rel, flush=True)
    assert rel <= 1e-6


def test_mixed_solve_matches_fp64_solve(layered):
    """The Cowling window [1, 12] of the layered planet with the mixed mass solve
    inside the filter: the same pairs as the FP64 solve, eigenvalues within
    1e-9 relative, every residual <= 1e-9 (after the FP64 refinement)."""
    torch, nm, d, G = layered
    r64 = G.filtered_eig(1.0, 12.0, 200, 1e-9, block=8)
    rm = G.filtered_eig(1.0, 12.0, 200, 1e-9, block=8, mass_passes=2, verbose=1)
    print("mixed solve: %d pairs, resid max %.2e, %d passes of %d steps, refine passes %d" % (
        rm.count, rm.resid.max(), rm.stats["mass_passes"], rm.stats["mass_pass_steps"],
        rm.stats["refine_passes"]), flush=True)
    assert rm.stats["mass_passes"] == 2 and rm.stats["mass_pass_steps"] >= 2
    assert rm.count == r64.count and rm.count > 0
    assert np.abs(rm.lam - r64.lam).max() <= 1e-9 * r64.lam.max()
    assert rm.resid.max() <= 1e-9


def test_mixed_solve_rejects_fp32_filter_and_bad_pass_counts(layered):
    torch, nm, d, G = layered
    X = _rand(torch, G.info["n_disp"], 4, 3)
    for kw in (dict(mass_passes=1), dict(mass_passes=9), dict(mass_passes=2, precision=1)):
        with pytest.raises(nm.NMError) as ei:
            G.apply(nm.OP_MINV, X.float() if kw.get("precision") else X, kM=8, **kw)
        assert ei.value.status == -1
