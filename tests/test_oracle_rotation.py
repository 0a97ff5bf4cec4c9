"""Pins of the oracle's Coriolis projection (Sec. 7)."""
import numpy as np
import pytest

from conftest import pencil
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
