"""The dense block products of the filtered Lanczos (Sec. 6.2: Gram-Schmidt
projections against the basis, Cholesky Gram matrices, Rayleigh-Ritz
matrices) on the FP64 matrix cores, through nm_gemm_tn / nm_gemm_nn, against
numpy's FP64 products.

Bound: both sides sum the same products in different orders, so each entry
differs by at most about 2 K eps sum_k |a_k b_k| (K terms, eps = 2^-53); the
tests allow 4 K eps times that sum."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def nm_torch():
    import torch
    import paper_1906_11082_amd as nm
    assert torch.cuda.is_available()
    return nm, torch


def _check(got, ref, absprod, K):
    err = np.abs(got - ref)
    bound = 4 * max(K, 1) * EPS * absprod + 1e-300
    assert np.all(err <= bound), "max err/bound %.3g" % (err / bound).max()


# (n, K, q, extra leading-dimension columns): ragged tiles, one chunk and many,
# the Lanczos shapes (K up to the basis size, q the block width or K itself)
TN_CASES = [(1, 1, 1, 0), (7, 5, 3, 2), (1000, 37, 5, 3), (4099, 100, 32, 0), (3, 70, 70, 1),
            (20000, 200, 64, 11), (50000, 300, 17, 0), (70001, 129, 129, 5)]


@pytest.mark.parametrize("n,K,q,pad", TN_CASES)
def test_gemm_tn_matches_numpy(nm_torch, n, K, q, pad):
    nm, torch = nm_torch
    rng = np.random.default_rng(n * 7 + K)
    A = rng.standard_normal((n, K + pad))
    B = rng.standard_normal((n, q + pad)) * 1e3
    Ad, Bd = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    C1 = nm.gemm_tn(Ad, Bd, K, q).cpu().numpy()
    C2 = nm.gemm_tn(Ad, Bd, K, q).cpu().numpy()
    assert np.array_equal(C1, C2), "the chunked sum must not depend on scheduling"
    ref = A[:, :K].T @ B[:, :q]
    _check(C1, ref, np.abs(A[:, :K]).T @ np.abs(B[:, :q]), n)


NN_CASES = [(1, 1, 1, 0), (7, 5, 3, 2), (1000, 37, 5, 3), (4099, 100, 32, 0), (3, 70, 70, 1),
            (20000, 200, 64, 11), (50000, 300, 17, 0), (70001, 129, 129, 5), (300, 0, 8, 0)]


@pytest.mark.parametrize("n,K,q,pad", NN_CASES)
def test_gemm_nn_matches_numpy(nm_torch, n, K, q, pad):
    nm, torch = nm_torch
    rng = np.random.default_rng(n * 11 + K)
    A = rng.standard_normal((n, K + pad))
    Cm = rng.standard_normal((K, q))
    D0 = rng.standard_normal((n, q + pad))
    Ad = torch.tensor(A, device="cuda")
    # beta 0: D is not read (NaN stays out)
    Dd = torch.full((n, q + pad), float("nan"), dtype=torch.float64, device="cuda")
    got = nm.gemm_nn(Ad, torch.tensor(Cm), Dd, alpha=1.0, beta=0.0).cpu().numpy()
    ref = A[:, :K] @ Cm
    _check(got[:, :q], ref, np.abs(A[:, :K]) @ np.abs(Cm), K)
    if pad:
        assert np.isnan(got[:, q:]).all(), "columns past q must be left alone"
    # the projection update D <- D - A C
    Dd = torch.tensor(D0, device="cuda")
    got = nm.gemm_nn(Ad, torch.tensor(Cm), Dd, alpha=-1.0, beta=1.0).cpu().numpy()
    ref = D0[:, :q] - A[:, :K] @ Cm
    _check(got[:, :q], ref, np.abs(D0[:, :q]) + np.abs(A[:, :K]) @ np.abs(Cm), K + 1)
    assert np.array_equal(got[:, q:], D0[:, q:])


def test_gemm_empty_sizes(nm_torch):
    """n = 0 gives a zero Gram matrix; q = 0 and K = 0 products are no-ops or
    scale D by beta."""
    nm, torch = nm_torch
    A = torch.zeros((0, 8), dtype=torch.float64, device="cuda")
    B = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    assert np.array_equal(nm.gemm_tn(A, B).cpu().numpy(), np.zeros((8, 4)))
    A = torch.ones((50, 3), dtype=torch.float64, device="cuda")
    D = torch.full((50, 2), 2.0, dtype=torch.float64, device="cuda")
    D = nm.gemm_nn(A[:, :0], torch.zeros((0, 2), dtype=torch.float64), D, alpha=1.0, beta=0.5)
    assert np.array_equal(D.cpu().numpy(), np.ones((50, 2)))
