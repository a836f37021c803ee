"""Deflated restarted Hermitian Lanczos methods of the paper: Lan-DR, MinRes-DR, D-CG, D-MinRes.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper (abstract; Section 1, closing paragraph; Section 2) describes the
methods and defers their definitions to its Ref. [3], which is not available.
The steps below are the published algorithms the paper names, specialised to
Hermitian A, in the paper's notation (m = Krylov dimension, k = deflated
eigenvectors):

Lan-DR(m,k) -- restarted Lanczos whose linear solve is the Galerkin/FOM solve
    T_m d = c (the "CG implementation of the Lanczos algorithm"), restarted
    with the k Ritz vectors of smallest Ritz value plus the next Lanczos
    vector (thick restart).  The projected matrix after a restart is an
    arrowhead: diag(theta) with coupling row beta_m * G[m, :k].
MinRes-DR(m,k) -- the same Lanczos space with the minimum-residual (least
    squares) solve d = argmin ||c - Tbar_m d|| and the k harmonic Ritz vectors
    of smallest |theta| (T_m g = mu Tbar_m^H Tbar_m g, theta = 1/mu), restarted
    GMRES-DR style with the orthonormalised [[G_k; 0], q], q spanning the
    orthogonal complement of range(Tbar_m).
D-CG / D-MinRes -- for every later right-hand side a Galerkin projection over
    the stored eigenvectors Y at the beginning, H d = Y^H r0 with
    H = Y^H A Y, x0 += Y d, followed by CG (normal equations) or MinRes.

Readings (paper silent): every Lanczos step is fully re-orthogonalised by
classical Gram-Schmidt applied twice (the paper's periodic re-orthogonalisation
over the kept vectors is the weaker special case); the first right-hand side
runs past linear convergence until every kept eigenpair has residual
<= eig_tol * ||A||_est or the MVP count reaches past_conv_factor (<= 2, Section 2,
last paragraph) times the count at linear convergence.  ||A||_est is the largest
infinity norm of the projected matrices T_m seen so far (a bound on ||A||
within the Krylov space); every cycle ends with a check of the true residual
that costs ``res_mvp`` MVPs (one application of M for the Wilson systems).
The solution returned is the cycle-end iterate with the smallest true residual:
once the linear system has met tol the further cycles serve the eigenvectors
(Section 2, last paragraph), and at the FP64 residual floor (near 1e-11 for the
normal equations of a near-critical lattice) their corrections can move the
residual up or down by small factors.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import krylov


def _nrm(u):
    return float(np.sqrt(np.real(np.vdot(u, u))))


def _cgs2(V, w):
    """Orthogonalise w against the columns of V twice; return (w, summed coefficients)."""
    h = V.conj().T @ w
    w = w - V @ h
    h2 = V.conj().T @ w
    w = w - V @ h2
    return w, h + h2


class _Stopper:
    """Stopping rule for the first right-hand side (linear convergence, then eigenvectors)."""

    def __init__(self, tol, k, eig_tol, past_conv_factor, max_mvp):
        self.tol, self.k, self.eig_tol = tol, k, eig_tol
        self.factor, self.max_mvp = past_conv_factor, max_mvp
        self.mvp_lin = None
        self.rule = None

    def done(self, relres, rho, anorm, mvp):
        if self.mvp_lin is None and relres <= self.tol:
            self.mvp_lin = mvp
        if self.mvp_lin is not None:
            if self.k == 0:
                self.rule = "linear"
                return True
            if np.all(rho <= self.eig_tol * anorm):
                self.rule = "eigen"
                return True
            if mvp >= self.factor * self.mvp_lin:
                self.rule = "mvp_factor"
                return True
        if mvp >= self.max_mvp:
            self.rule = "max_mvp"
            return True
        return False


def _lanczos_extend(A, V, Tb, j0, m, apv, mvp, bnorm_tiny):
    """Extend the basis from column j0 to m (in place). Returns (m_used, mvp, breakdown)."""
    for j in range(j0, m):
        w = A(V[:, j])
        mvp += apv
        w, h = _cgs2(V[:, : j + 1], w)
        Tb[j, j] = np.real(h[j])
        # symmetric coupling: full arrow column right after a restart, else the tridiagonal entry
        Tb[:j, j] = Tb[j, :j]
        beta = _nrm(w)
        Tb[j + 1, j] = beta
        if beta <= bnorm_tiny:
            return j + 1, mvp, True
        V[:, j + 1] = w / beta
    return m, mvp, False


def lan_dr(A, bA, m, k, tol, residual=None, eig_tol=1e-12, past_conv_factor=2.0,
           max_mvp=100000, apv=1, x0=None, mvp0=0, res_mvp=1):
    """Lan-DR(m,k) for Hermitian positive definite A (callable on vectors).

    ``residual(x)`` is the relative residual used for convergence (for the
    normal equations it is ||b - M x||/||b||); by default ||bA - A x||/||bA||.
    ``apv`` is the number of MVPs per application of A (2 for M^dag M).
    Returns (x, eig, info) with eig = dict(vals, vecs, rho).
    """
    if not (0 <= k < m):
        raise ValueError("need 0 <= k < m")
    n = bA.shape[0]
    bn = _nrm(bA)
    if residual is None:
        residual = lambda x: _nrm(bA - A(x)) / bn
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    mvp = mvp0
    if x0 is None:
        r = bA.copy()
    else:
        r = bA - A(x)
        mvp += apv
    beta0 = _nrm(r)
    if beta0 == 0.0:
        return x, dict(vals=np.zeros(0), vecs=np.zeros((n, 0), complex), rho=np.zeros(0)), \
            dict(mvp=mvp, cycles=0, relres=0.0, history=[0.0], rule="zero_rhs", mvp_lin=0)
    V = np.zeros((n, m + 1), dtype=np.complex128)
    V[:, 0] = r / beta0
    Tb = np.zeros((m + 1, m))
    c = np.zeros(m + 1)
    c[0] = beta0
    j0 = 0
    stop = _Stopper(tol, k, eig_tol, past_conv_factor, max_mvp)
    hist, cycles = [], 0
    anorm = 0.0
    best = (np.inf, x)
    while True:
        mm, mvp, brk = _lanczos_extend(A, V, Tb, j0, m, apv, mvp, 1e-14 * max(anorm, 1e-300) if anorm else 0.0)
        Tm = Tb[:mm, :mm]
        beta_m = Tb[mm, mm - 1]
        d = np.linalg.solve(Tm, c[:mm])
        x = x + V[:, :mm] @ d
        theta, G = np.linalg.eigh(Tm)
        anorm = max(anorm, float(np.abs(Tm).sum(axis=1).max()))
        order = np.lexsort((np.arange(mm), theta))  # algebraically smallest, stable
        keep = order[:k]
        rho = np.abs(beta_m * G[mm - 1, keep])
        relres = residual(x)
        mvp += res_mvp
        hist.append(relres)
        cycles += 1
        if relres < best[0]:
            best = (relres, x.copy())
        if brk or stop.done(relres, rho, anorm, mvp):
            break
        # thick restart: V_k <- V_m G_k, v_{k+1} <- v_{m+1}; arrowhead T-bar
        Vn = np.zeros_like(V)
        Vn[:, :k] = V[:, :m] @ G[:, keep]
        Vn[:, k] = V[:, m]
        V = Vn
        Tb = np.zeros((m + 1, m))
        Tb[np.arange(k), np.arange(k)] = theta[keep]
        Tb[k, :k] = beta_m * G[m - 1, keep]
        c = np.zeros(m + 1)
        c[k] = -beta_m * d[m - 1]
        j0 = k
    vecs = V[:, :mm] @ G[:, keep]
    eig = dict(vals=theta[keep].copy(), vecs=vecs, rho=rho)
    return best[1], eig, dict(mvp=mvp, cycles=cycles, relres=best[0], history=hist,
                              rule=stop.rule if not brk else "breakdown", mvp_lin=stop.mvp_lin)


def _harmonic_ritz(Tb):
    """Harmonic Ritz pairs of T-bar: T_m g = mu (Tbar^H Tbar) g, theta = 1/mu."""
    m = Tb.shape[1]
    Tm = Tb[:m, :m]
    mu, G = sla.eigh(Tm, Tb.T @ Tb)
    with np.errstate(divide="ignore"):
        theta = np.where(mu != 0.0, 1.0 / mu, np.inf)
    return theta, G


def minres_dr(A, bA, m, k, tol, residual=None, eig_tol=1e-12, past_conv_factor=2.0,
              max_mvp=100000, apv=1, x0=None, mvp0=0, res_mvp=1):
    """MinRes-DR(m,k) for Hermitian (indefinite) A.  Returns (x, eig, info)."""
    if not (0 <= k < m):
        raise ValueError("need 0 <= k < m")
    n = bA.shape[0]
    bn = _nrm(bA)
    if residual is None:
        residual = lambda x: _nrm(bA - A(x)) / bn
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    mvp = mvp0
    if x0 is None:
        r = bA.copy()
    else:
        r = bA - A(x)
        mvp += apv
    beta0 = _nrm(r)
    if beta0 == 0.0:
        return x, dict(vals=np.zeros(0), vecs=np.zeros((n, 0), complex), rho=np.zeros(0)), \
            dict(mvp=mvp, cycles=0, relres=0.0, history=[0.0], rule="zero_rhs", mvp_lin=0)
    V = np.zeros((n, m + 1), dtype=np.complex128)
    V[:, 0] = r / beta0
    Tb = np.zeros((m + 1, m))
    c = np.zeros(m + 1)
    c[0] = beta0
    j0 = 0
    stop = _Stopper(tol, k, eig_tol, past_conv_factor, max_mvp)
    hist, cycles = [], 0
    anorm = 0.0
    H = np.zeros((0, 0))
    S = np.zeros((0, 0))
    lam = np.zeros(0)
    rho = np.zeros(0)
    best = (np.inf, x)
    while True:
        mm, mvp, brk = _lanczos_extend(A, V, Tb, j0, m, apv, mvp, 1e-14 * anorm if anorm else 0.0)
        if brk:  # invariant subspace: the square problem is exact
            d = np.linalg.solve(Tb[:mm, :mm], c[:mm])
            x = x + V[:, :mm] @ d
            relres = residual(x)
            mvp += res_mvp
            hist.append(relres)
            cycles += 1
            theta, G = np.linalg.eigh(Tb[:mm, :mm])
            order = np.lexsort((np.arange(mm), np.abs(theta)))[:k]
            vecs = V[:, :mm] @ G[:, order]
            return x, dict(vals=theta[order], vecs=vecs, rho=np.zeros(len(order))), \
                dict(mvp=mvp, cycles=cycles, relres=relres, history=hist, rule="breakdown",
                     mvp_lin=stop.mvp_lin)
        d, *_ = np.linalg.lstsq(Tb, c, rcond=None)
        x = x + V[:, :m] @ d
        s = c - Tb @ d
        theta, G = _harmonic_ritz(Tb)
        anorm = max(anorm, float(np.abs(Tb[:m, :m]).sum(axis=1).max()))
        order = np.lexsort((theta, np.abs(theta)))  # smallest |theta|, ties by theta
        keep = order[:k]
        # orthogonal complement of range(Tbar): last column of a complete QR
        Qc, _ = np.linalg.qr(Tb, mode="complete")
        q = Qc[:, m]
        P = np.zeros((m + 1, k + 1))
        P[:m, :k] = G[:, keep]
        P[:, k] = q
        Q, _ = np.linalg.qr(P)
        Tn = Q.T @ Tb @ Q[:m, :k]
        H = Tn[:k, :k]
        lam, S = np.linalg.eigh(H)
        rho = np.abs(Tn[k, :k] @ S)
        relres = residual(x)
        mvp += res_mvp
        hist.append(relres)
        cycles += 1
        if relres < best[0]:
            best = (relres, x.copy())
        # restart: V_{k+1} <- V_{m+1} Q, Tbar <- Q^H Tbar Q, c <- Q^H s
        V = np.concatenate([V @ Q, np.zeros((n, m - k), dtype=np.complex128)], axis=1)
        Tb = np.zeros((m + 1, m))
        Tb[: k + 1, :k] = Tn
        c = np.zeros(m + 1)
        c[: k + 1] = Q.T @ s
        j0 = k
        if stop.done(relres, rho, anorm, mvp):
            break
    vecs = V[:, :k] @ S
    eig = dict(vals=lam, vecs=vecs, rho=rho, harmonic=theta[keep].copy())
    return best[1], eig, dict(mvp=mvp, cycles=cycles, relres=best[0], history=hist, rule=stop.rule,
                              mvp_lin=stop.mvp_lin)


# --------------------------------------------------------------------------
# Later right-hand sides: Galerkin projection at the beginning, then CG / MinRes
# --------------------------------------------------------------------------

def projection_matrix(A, Y):
    """H = Y^H A Y, built with k applications of A (FP64)."""
    AY = np.stack([A(Y[:, i]) for i in range(Y.shape[1])], axis=1) if Y.shape[1] else Y
    return Y.conj().T @ AY


def galerkin_projection(Y, H, r):
    """d = H^-1 Y^H r; returns the correction Y d."""
    if Y.shape[1] == 0:
        return np.zeros_like(r)
    d = np.linalg.solve(H, Y.conj().T @ r)
    return Y @ d


def d_cg(A, b, Y, H, tol, x0=None, maxiter=100000):
    """D-CG for Hermitian positive definite A: projection, then CG."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - A(x) if x0 is not None else b.copy()
    x = x + galerkin_projection(Y, H, r)
    return krylov.cg(A, b, x0=x, tol=tol, maxiter=maxiter)


def d_cg_normal(M, Mdag, b, Y, H, tol, x0=None, maxiter=100000):
    """D-CG on M^dag M x = M^dag b: projection of the normal-equation residual, then CGLS.

    Y are eigenvectors of M^dag M and H = Y^H M^dag M Y.
    """
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    rA = Mdag(b - M(x))
    x = x + galerkin_projection(Y, H, rA)
    x, info = krylov.cgls(M, Mdag, b, x0=x, tol=tol, maxiter=maxiter)
    info["mvp"] += 2 if x0 is None else 3
    return x, info


def d_minres(A, b, Y, H, tol, x0=None, maxiter=100000):
    """D-MinRes for Hermitian (indefinite) A: projection, then MinRes."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - A(x) if x0 is not None else b.copy()
    x = x + galerkin_projection(Y, H, r)
    return krylov.minres(A, b, x0=x, tol=tol, maxiter=maxiter)
