"""Pencil operators, polynomial filter and filtered Lanczos (oracle, FP64).

* The Cowling pencil (eq. "cowling"): A x = omega^2 M x with
  A = A_G + E_G K_p^{-1} E_G^T, M = M_s (x) I_3 (Sec. 6.1, eq. "gep").
* The paper accesses A, M and M^{-1} only through matrix-vector products
  (Sec. 6.1).  M^{-1} here: Chebyshev iteration preconditioned by the
  diagonal of M, on the interval that bounds the spectrum of D^{-1} M
  element by element (the same iteration serves K_p^{-1}); its iterative
  refinement y <- y + S(f - M y) over several passes, in float64 or with
  float32 passes (the library's mass_passes).
* Polynomial filtering (Sec. 2.5 remark, Sec. 6.1): a Jackson-damped
  Chebyshev expansion of the indicator of the window, applied by the
  three-term recurrence, optionally times the factor (B - lambda_0)/s that
  annihilates an exactly degenerate null space at lambda_0.
* Lanczos in the M-inner product on p(B), full reorthogonalisation, and
  Rayleigh-Ritz with the original pencil (A, M).
* Dense reference solve and Sylvester-inertia counts for small problems.
"""
from __future__ import annotations

import math
import numpy as np
import scipy.linalg as sla

# Element bounds of the spectrum of D^{-1} M (D = diag M): the extreme
# generalised eigenvalues of (M_e, diag M_e) of one reference element
# (identical for every affine element and any positive element weight).
def jacobi_mass_bounds(order: int):
    from . import refelem
    M = refelem.as_float(refelem.mass_exact(order, order, 4))
    w = sla.eigh(M, np.diag(np.diag(M)), eigvals_only=True)
    return float(w[0]), float(w[-1])


def cheb_iters(lo: float, hi: float, tol: float) -> int:
    """Smallest k with 2 r^k <= tol, r = (sqrt(kappa)-1)/(sqrt(kappa)+1)."""
    kap = hi / lo
    r = (math.sqrt(kap) - 1.0) / (math.sqrt(kap) + 1.0)
    return max(1, int(math.ceil(math.log(2.0 / tol) / math.log(1.0 / r))))


def cheb_jacobi(Mop, diag, f, k, lo, hi):
    """k steps of the Chebyshev iteration for M y = f from y = 0 with
    preconditioner diag(M) (Saad, Iterative Methods, Alg. 12.1): returns
    y_k, a polynomial of degree k-1 in D^{-1}M applied to D^{-1} f."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    dinv = (1.0 / diag).reshape((-1,) + (1,) * (f.ndim - 1))
    x = np.zeros_like(f)
    r = f.copy()
    d = dinv * r / theta
    for it in range(k):
        x = x + d
        if it == k - 1:
            break
        r = r - Mop(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * dinv * r
        rho = rho_new
    return x


def cheb_jacobi_refined(Mop, diag, f, k, lo, hi, passes, Mop32=None):
    """Iterative refinement of the k-step solve S = cheb_jacobi: from y = 0,
    `passes` times y <- y + S(f - M y), so M^{-1} f - y = (I - S M)^passes M^{-1} f.
    The paper fixes only that M^{-1} is applied through products with M
    (Sec. 6.1); this is the reading the library's mass_passes option computes.
    With Mop32 (M in float32) each S runs in float32 on the float32-rounded
    residual while the residuals and the sum stay float64, as the library's
    passes do (a model of their rounding, not of their summation order)."""
    y = np.zeros_like(f)
    r = f.copy()
    for p in range(passes):
        if Mop32 is None:
            d = cheb_jacobi(Mop, diag, r, k, lo, hi)
        else:
            d = cheb_jacobi(Mop32, diag.astype(np.float32), r.astype(np.float32), k,
                            np.float32(lo), np.float32(hi)).astype(np.float64)
        y = y + d
        if p + 1 < passes:
            r = f - Mop(y)
    return y


# ------------------------------------------------------------------ filter
def jackson(m: int):
    """Jackson damping factors g_0..g_m."""
    th = math.pi / (m + 2)
    k = np.arange(m + 1)
    return ((1.0 - k / (m + 2)) * math.sin(th) * np.cos(k * th)
            + math.cos(th) * np.sin(k * th) / (m + 2)) / math.sin(th)


def window_chebyshev(alpha: float, beta: float, m: int):
    """Chebyshev coefficients of the indicator of [alpha, beta] in [-1, 1]."""
    ta, tb = math.acos(max(-1.0, min(1.0, alpha))), math.acos(max(-1.0, min(1.0, beta)))
    k = np.arange(1, m + 1)
    g = np.empty(m + 1)
    g[0] = (ta - tb) / math.pi
    g[1:] = 2.0 * (np.sin(k * ta) - np.sin(k * tb)) / (math.pi * k)
    return g


def filter_coeffs(a, b, lmin, lmax, m):
    """mu_k = g_k gamma_k for the window [a, b] mapped from [lmin, lmax]."""
    c, e = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    return jackson(m) * window_chebyshev((a - c) / e, (b - c) / e, m), c, e


def cheb_series(mu, t):
    """Scalar p(t) = sum_k mu_k T_k(t) by the three-term recurrence."""
    t = np.asarray(t, float)
    T0, T1 = np.ones_like(t), t
    s = mu[0] * T0 + (mu[1] * T1 if len(mu) > 1 else 0.0)
    for k in range(2, len(mu)):
        T0, T1 = T1, 2.0 * t * T1 - T0
        s = s + mu[k] * T1
    return s


def filter_apply(Bop, V, mu, c, e, null_shift=None, null_scale=1.0):
    """Y = p(B) V (and, with null_shift l0, Y = ((B - l0)/s) p(B) V)."""
    if null_shift is not None:
        V = (Bop(V) - null_shift * V) / null_scale
    W0 = V
    Y = mu[0] * W0
    if len(mu) == 1:
        return Y
    W1 = (Bop(W0) - c * W0) / e
    Y = Y + mu[1] * W1
    for k in range(2, len(mu)):
        W2 = 2.0 * (Bop(W1) - c * W1) / e - W0
        Y = Y + mu[k] * W2
        W0, W1 = W1, W2
    return Y


# ---------------------------------------------------------------- operators
class CowlingOperator:
    """Matrix-free access to the pencil: A x, M x, M^{-1} x, B x = M^{-1} A x."""

    def __init__(self, pencil, minv_tol=1e-13, kp_tol=1e-14, kp_exact=False):
        self.P = pencil
        lo, hi = jacobi_mass_bounds(pencil.order)
        self.m_lo, self.m_hi = lo, hi
        self.kM = cheb_iters(lo, hi, minv_tol)
        self.Md = np.repeat(pencil.Ms.diagonal(), 3)
        self.n = pencil.n
        if pencil.n_p:
            plo, phi = jacobi_mass_bounds(pencil.porder)
            self.kP = cheb_iters(plo, phi, kp_tol)
            kd = pencil.Kp.diagonal()
            if kp_exact:
                self.kp_solve = pencil.kp_direct()
            else:
                self.kp_solve = lambda r: cheb_jacobi(lambda x: pencil.Kp @ x, kd, r, self.kP, plo, phi)
        self.n_A = 0

    def A(self, x):
        self.n_A += 1
        y = self.P.AG @ x
        if self.P.n_p:
            y = y + self.P.EG @ self.kp_solve(self.P.EG.T @ x)
        return y

    def M(self, x):
        return self.P.M @ x

    def Minv(self, f):
        return cheb_jacobi(self.M, self.Md, f, self.kM, self.m_lo, self.m_hi)

    def B(self, x):
        return self.Minv(self.A(x))


def lanczos_bounds(op, steps=60, seed=12345):
    """Extreme Ritz values of B from Lanczos in the M-inner product, with the
    residual norms |beta_k s_k| of the extreme Ritz pairs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = op.n
    v = rng.standard_normal(n)
    v /= math.sqrt(v @ op.M(v))
    V = [v]
    al, be = [], []
    vprev, bprev = np.zeros(n), 0.0
    for j in range(steps):
        w = op.B(v) - bprev * vprev
        a = w @ op.M(v)
        w = w - a * v
        for u in V:  # full reorthogonalisation
            w = w - (w @ op.M(u)) * u
        b = math.sqrt(max(w @ op.M(w), 0.0))
        al.append(a); be.append(b)
        if b < 1e-14 * abs(a):
            break
        vprev, v, bprev = v, w / b, b
        V.append(v)
    k = len(al)
    th, S = sla.eigh_tridiagonal(np.array(al), np.array(be[:k - 1]))
    res = np.abs(be[k - 1] * S[-1, :])
    return th[0], res[0], th[-1], res[-1]


# ------------------------------------------------------------- dense oracle
def dense_window(A, M, a, b):
    """All eigenpairs of the dense pencil with a <= lambda <= b, ascending,
    M-orthonormal (scipy / LAPACK)."""
    w, X = sla.eigh(A, M, subset_by_value=(a, b))
    return w, X


def cowling_window(pencil, a, b, pieces=None, k0=48, tol=1e-13, permc_spec="MMD_AT_PLUS_A"):
    """All eigenpairs of the Cowling pencil (eq. "cowling": A_G + E_G K_p^{-1}
    E_G^T with the exact Schur complement) with a <= lambda <= b, a > 0,
    ascending, M-orthonormal: shift-invert Lanczos (ARPACK through scipy) at
    the midpoint of each of `pieces` equal sub-intervals of [a, b], the
    shifted solve done by one sparse LU of the saddle-point system
    [[A_G - s M, E_G], [E_G^T, -K_p]].  Shift-invert returns the k
    eigenvalues nearest the shift; k grows until the farthest of them lies
    outside the sub-interval, so every eigenvalue inside it is found (the
    exactly degenerate fluid null space at 0 lies farther from every shift
    than the sub-interval's ends)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    n, n_p = pencil.n, pencil.n_p
    kp = pencil.kp_direct() if n_p else None
    Aop = spla.LinearOperator((n, n), matvec=lambda x: pencil.cowling_apply(x, kp), dtype=float)
    pieces = pieces or max(1, int(math.ceil((b - a) / 12.0)))
    edges = np.linspace(a, b, pieces + 1)
    lams, vecs = [], []
    for i in range(pieces):
        lo, hi = edges[i], edges[i + 1]
        s, r = 0.5 * (lo + hi), 0.5 * (hi - lo)
        if n_p:
            K = sp.bmat([[pencil.AG - s * pencil.M, pencil.EG], [pencil.EG.T, -pencil.Kp]], format="csc")
        else:
            K = (pencil.AG - s * pencil.M).tocsc()
        lu = spla.splu(K, permc_spec=permc_spec)
        Sop = spla.LinearOperator((n, n), dtype=float,
                                  matvec=lambda f: lu.solve(np.concatenate([f, np.zeros(n_p)]))[:n])
        k = k0
        while True:
            k = min(k, n - 2)
            w, V = spla.eigsh(Aop, k=k, M=pencil.M, sigma=s, OPinv=Sop, which="LM", tol=tol)
            if np.abs(w - s).max() > r * (1 + 1e-9) or k >= n - 2:
                break
            k *= 2
        keep = (w >= lo) & ((w < hi) if i + 1 < pieces else (w <= hi))
        lams.append(w[keep])
        vecs.append(V[:, keep])
    w = np.concatenate(lams)
    X = np.concatenate(vecs, axis=1)
    o = np.argsort(w)
    return w[o], X[:, o]


def inertia_count(A, M, sigma):
    """Number of eigenvalues of (A, M) below sigma (Sylvester's law of
    inertia on the dense LDL^T factorisation of A - sigma M)."""
    L, D, perm = sla.ldl(A - sigma * M)
    return int((np.linalg.eigvalsh(D) < 0).sum())


# ------------------------------------------------------------ filtered Lanczos
def filtered_lanczos(op, a, b, nev, tol, mu, c, e, null_shift=None, null_scale=1.0,
                     max_iter=None, check_every=10, seed=1, v0=None):
    """Lanczos on C = p(B) in the M-inner product with full (twice-iterated)
    reorthogonalisation; every check_every steps Rayleigh-Ritz with (A, M)
    on the Lanczos basis.  Returns (lambda, X, resid, n_steps)."""
    n = op.n
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(n) if v0 is None else v0.copy()
    v /= math.sqrt(v @ op.M(v))
    C = lambda x: filter_apply(op.B, x, mu, c, e, null_shift, null_scale)
    max_iter = max_iter or n
    V = np.empty((n, 0))
    MV = np.empty((n, 0))
    AV = np.empty((n, 0))
    al, be = [], []
    last_count = -1
    out = None
    for j in range(max_iter):
        V = np.column_stack([V, v])
        Mv = op.M(v)
        MV = np.column_stack([MV, Mv])
        AV = np.column_stack([AV, op.A(v)])
        w = C(v)
        h = MV.T @ w
        w = w - V @ h
        h2 = MV.T @ w
        w = w - V @ h2
        al.append(h[-1] + h2[-1])
        bt = math.sqrt(max(w @ op.M(w), 0.0))
        be.append(bt)
        done = (j + 1) % check_every == 0 or j + 1 == max_iter or bt < 1e-13
        if done:
            Ha = V.T @ AV
            Hm = V.T @ MV
            th, Y = sla.eigh(0.5 * (Ha + Ha.T), 0.5 * (Hm + Hm.T))
            sel = (th >= a) & (th <= b)
            X = V @ Y[:, sel]
            lam = th[sel]
            R = AV @ Y[:, sel] - (MV @ Y[:, sel]) * lam
            MX = MV @ Y[:, sel]
            res = np.linalg.norm(R, axis=0) / (np.abs(lam) * np.linalg.norm(MX, axis=0))
            # Ritz values of C and their residual estimates
            k = len(al)
            mth, S = sla.eigh_tridiagonal(np.array(al), np.array(be[:k - 1]))
            mres = np.abs(be[k - 1] * S[-1, :])
            pa = min(cheb_series(mu, np.array([(a - c) / e, (b - c) / e])) *
                     (np.array([a, b]) - (null_shift or 0.0)) / null_scale
                     if null_shift is not None else
                     cheb_series(mu, np.array([(a - c) / e, (b - c) / e])))
            big = mth >= pa
            c_conv = np.all(mres[big] <= 1e-9 * max(abs(mth).max(), 1e-300))
            count = int(sel.sum())
            ok = count > 0 and np.all(res <= tol) and c_conv and count == last_count
            last_count = count
            out = (lam, X, res, j + 1)
            if ok or bt < 1e-13:
                break
        v = w / bt
    lam, X, res, steps = out
    k = min(nev, len(lam))
    return lam[:k], X[:, :k], res[:k], steps
