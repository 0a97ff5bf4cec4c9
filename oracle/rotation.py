"""Coriolis QEP by projection on non-rotating modes (oracle, FP64).

Sec. 7: omega^2 M u - 2 i omega R u - A u = 0 (eq. "simplequad"), with R
real skew-symmetric (2iR Hermitian).  With X_e the M-orthonormal eigenvectors
of A X_e = M X_e Lambda_e (eq. "linearpb") and u = X_e y, the linearised
2n pencil [[0, A], [A, 2iR]] z = omega [[A, 0], [0, M]] z, z = [u; omega u],
projected on diag(X_e, X_e) gives (eq. "sublinear0")

    [[0, L], [L, 2iS]] [y; omega y] = omega [[L, 0], [0, I]] [y; omega y],
    L = Lambda_e, S = X_e^T R X_e.

Scaling by diag(L^{-1/2}, I) turns it into the Hermitian standard problem
[[0, L^{1/2}], [L^{1/2}, 2iS]] w = omega w, w = [L^{1/2} y; omega y].
Modes are normalised by eq. "orthonormalcond":
u^H M u - (2 i / (2 omega)) u^H R u = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def projected_problem(lam, S):
    """Hermitian 2m x 2m matrix of the projected linearisation."""
    m = len(lam)
    r = np.sqrt(lam)
    H = np.zeros((2 * m, 2 * m), complex)
    H[:m, m:] = np.diag(r)
    H[m:, :m] = np.diag(r)
    H[m:, m:] = 2j * S
    return H


def project_rotation(lam, X, Rop, a, b):
    """Rotating eigenfrequencies omega > 0 with omega^2 in [a, b] and their
    complex modes (columns of U, normalised by the orthonormality condition).
    Rop(X) applies the Coriolis matrix R to the columns of X."""
    S = X.T @ Rop(X)
    S = 0.5 * (S - S.T)
    H = projected_problem(lam, S)
    w, Z = sla.eigh(H)
    m = len(lam)
    keep = (w > 0) & (w * w >= a) & (w * w <= b)
    om = w[keep]
    Y = Z[:m, keep] / np.sqrt(lam)[:, None]
    # orthonormality condition: y^H y - (i/omega) y^H S y = 1
    nrm = np.real(np.einsum("ik,ik->k", Y.conj(), Y)
                  - 1j / om * np.einsum("ik,ij,jk->k", Y.conj(), S, Y))
    Y = Y / np.sqrt(nrm)[None, :]
    U = X @ Y
    # phase: entry of largest magnitude real and positive
    idx = np.argmax(np.abs(U), axis=0)
    ph = U[idx, np.arange(U.shape[1])]
    U = U * (np.abs(ph) / ph)[None, :]
    return om, U, S


def first_order_splitting(U, Rop):
    """First-order frequency shifts of a degenerate multiplet with
    M-orthonormal basis U: eigenvalues of i U^T R U."""
    S = U.T @ Rop(U)
    S = 0.5 * (S - S.T)
    return np.linalg.eigvalsh(1j * S)


def qep_exact(A, M, R, a, b):
    """The rotating modes of the full discrete QEP (eq. "simplequad"),
    omega^2 M u - 2 i omega R u - A u = 0, with omega > 0 and omega^2 in
    [a, b]: eigenvalues of the first companion form
    [[0, I], [M^{-1} A, 2 i M^{-1} R]] acting on [u; omega u] (dense, numpy),
    ascending, with their modes normalised by eq. "orthonormalcond"
    (u^H M u - (i / omega) u^H R u = 1).  Unlike the projection, nothing is
    left out: rigid motions and the fluid null space of A couple too."""
    n = A.shape[0]
    Mi = np.linalg.inv(M)
    L = np.block([[np.zeros((n, n)), np.eye(n)], [Mi @ A, 2j * (Mi @ R)]])
    w, Z = np.linalg.eig(L)
    scale = np.abs(w).max()
    sel = (np.abs(w.imag) <= 1e-8 * scale) & (w.real > 0)
    w, Z = w[sel].real, Z[:, sel]
    keep = (w * w >= a) & (w * w <= b)
    w, U = w[keep], Z[:n, keep]
    o = np.argsort(w)
    w, U = w[o], U[:, o]
    nrm = np.real(np.einsum("ik,ik->k", U.conj(), M @ U) - 1j / w * np.einsum("ik,ik->k", U.conj(), R @ U))
    U = U / np.sqrt(nrm)[None, :]
    idx = np.argmax(np.abs(U), axis=0)
    ph = U[idx, np.arange(U.shape[1])]
    U = U * (np.abs(ph) / ph)[None, :]
    return w, U


def qep_residual(A, M, R, omega, U):
    """|| omega^2 M u - 2 i omega R u - A u || / (omega^2 || M u ||) per mode."""
    Rr = (M @ U) * omega ** 2 - 2j * (R @ U) * omega - A @ U
    return np.linalg.norm(Rr, axis=0) / (omega ** 2 * np.linalg.norm(M @ U, axis=0))
