"""Pins of the oracle's Coriolis projection (Sec. 7)."""
import numpy as np
import pytest

from conftest import pencil, planet
from oracle import rotation as RT
from oracle import solve as S
from oracle.assemble import Pencil, omega_cross
import scipy.sparse as sp


def _modes():
    P = pencil("homogeneous_ball")
    A, M = P.AG.toarray(), P.M.toarray()
    lam, X = S.dense_window(A, M, 0.5, 60.0)
    return P, lam, X


def _Rop(P, Om):
    Rm = sp.kron(P.Ms, sp.csr_matrix(omega_cross(Om)), format="csr")
    return lambda X: Rm @ X


def test_no_rotation_gives_sqrt_lambda():
    P, lam, X = _modes()
    om, U, _ = RT.project_rotation(lam, X, _Rop(P, (0, 0, 0)), 0.5, 60.0)
    np.testing.assert_allclose(np.sort(om), np.sqrt(lam), rtol=1e-13)


def test_plus_minus_pairs_and_orthonormality():
    P, lam, X = _modes()
    Rop = _Rop(P, (0.02, -0.01, 0.3))
    S_ = X.T @ Rop(X)
    H = RT.projected_problem(lam, 0.5 * (S_ - S_.T))
    w = np.linalg.eigvalsh(H)
    np.testing.assert_allclose(np.sort(w), np.sort(-w), atol=1e-12 * np.abs(w).max())
    om, U, S2 = RT.project_rotation(lam, X, Rop, 5.0, 40.0)
    M = P.M
    Rm = lambda v: Rop(v)
    G = U.conj().T @ (M @ U) - 2j * (U.conj().T @ Rm(U)) / (om[:, None] + om[None, :])
    np.testing.assert_allclose(G, np.eye(len(om)), atol=1e-10)


def test_first_order_toroidal_splitting():
    """0T2 multiplet: first-order Coriolis shifts are m Omega / (l (l+1)),
    m = -2..2, for any spherically symmetric model (the jittered polyhedral
    ball is nearly so)."""
    P, lam, X = _modes()
    U = X[:, 6:11] if lam[0] < 1.0 else X[:, :5]
    om0 = 0.2
    d = RT.first_order_splitting(U, _Rop(P, (0, 0, om0)))
    ref = om0 * np.arange(-2, 3) / 6.0
    assert np.abs(np.sort(d) - ref).max() < 0.03 * om0 / 3


def test_projection_matches_first_order_at_small_rate():
    """Projected rotating frequencies of the 0T2 multiplet against
    quasi-degenerate first-order theory, eigenvalues of
    diag(omega_0,i) + i U^T R U (the jitter splits the multiplet slightly):
    the discrepancy is O(Omega^2), so halving Omega divides it by about 4."""
    P, lam, X = _modes()
    errs = []
    for om0 in (0.02, 0.01):
        Rop = _Rop(P, (0, 0, om0))
        om, U, _ = RT.project_rotation(lam, X, Rop, 0.5, 60.0)
        U5 = X[:, :5]
        S5 = U5.T @ Rop(U5)
        S5 = 0.5 * (S5 - S5.T)
        ref = np.linalg.eigvalsh(np.diag(np.sqrt(lam[:5])) + 1j * S5)
        got = np.sort(om)[:5]
        errs.append(np.abs(got - ref).max())
    assert errs[1] < errs[0] / 3.0
    assert errs[0] < 0.01 * 0.02


def _small_ball(om):
    d = dict(planet("homogeneous_ball", n_half=3, order=1))
    d["omega"] = om
    P = Pencil(d)
    return P, P.AG.toarray(), P.M.toarray(), P.R.toarray()


def test_exact_qep_without_rotation_is_sqrt_lambda():
    """R = 0: the QEP's positive frequencies are the square roots of the
    pencil's eigenvalues in the window, and every companion eigenvalue is real."""
    P, A, M, R = _small_ball((0.0, 0.0, 0.0))
    w, U = RT.qep_exact(A, M, R, 4.0, 40.0)
    lam, _ = S.dense_window(A, M, 4.0, 40.0)
    assert len(w) == len(lam) > 10
    assert np.abs(w - np.sqrt(lam)).max() <= 1e-10 * w.max()
    assert RT.qep_residual(A, M, R, w, U).max() < 1e-10


def test_exact_qep_real_spectrum_and_first_order_splitting():
    """Gyroscopic QEP (A semidefinite, R skew): the companion spectrum is real
    and modes solve the QEP with orthonormality eq. "orthonormalcond".  Near
    an isolated cluster the exact frequencies approach the degenerate
    first-order theory, eig(diag(sqrt lambda) + i U^T R U), with an error that
    falls ~4x when Omega halves (second order in Omega)."""
    errs = []
    for oz in (0.08, 0.04):
        P, A, M, R = _small_ball((0.0, 0.0, oz))
        n = A.shape[0]
        L = np.block([[np.zeros((n, n)), np.eye(n)], [np.linalg.solve(M, A), 2j * np.linalg.solve(M, R)]])
        ev = np.linalg.eigvals(L)
        assert np.abs(ev.imag).max() <= 1e-8 * np.abs(ev).max()
        lam, X = S.dense_window(A, M, 0.5, 80.0)
        # the lowest toroidal-like cluster: the first eigenvalue group well separated from the next
        gaps = np.diff(lam)
        i0 = 0
        j = i0 + 1
        while j < len(lam) and gaps[j - 1] < 0.03 * lam[j]:
            j += 1
        cl = slice(i0, j)
        lo, hi = lam[cl].min(), lam[cl].max()
        w, U = RT.qep_exact(A, M, R, 0.97 * lo, 1.03 * hi)
        Xc = X[:, cl]
        Sc = Xc.T @ (R @ Xc)
        Heff = np.diag(np.sqrt(lam[cl])) + 1j * 0.5 * (Sc - Sc.T)
        pred = np.sort(np.linalg.eigvalsh(Heff))
        assert len(w) == len(pred) >= 3
        assert RT.qep_residual(A, M, R, w, U).max() < 1e-9
        G = U.conj().T @ (M @ U) - 2j * (U.conj().T @ (R @ U)) / (w[:, None] + w[None, :])
        assert np.abs(G - np.eye(len(w))).max() < 1e-8
        errs.append(np.abs(w - pred).max())
    assert 3.0 < errs[0] / errs[1] < 5.5, errs
