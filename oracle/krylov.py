"""Unrestarted Krylov solvers of Section 1 (Eq. 1): CG, CG on the normal equations, MinRes.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* ``cg``     -- Hestenes-Stiefel conjugate gradient for Hermitian positive definite A.
* ``cgls``   -- CG applied to M^dag M x = M^dag b (the paper's "CG normal equations",
                two MVPs per iteration, Section 2), written so that it carries the
                residual r = b - M x of the original system.
* ``minres`` -- Paige-Saunders minimum residual for Hermitian (possibly indefinite)
                A: Lanczos three-term recurrence plus Givens QR of the tridiagonal.

Every solver stops on a relative residual and returns (x, info) with the
per-iteration residual-norm history (the paper's figures are residual norm
against iterations/MVPs) and the count of operator applications.
"""
from __future__ import annotations

import numpy as np


def _dot(u, v):
    return np.vdot(u, v)


def _nrm(u):
    return float(np.sqrt(np.real(np.vdot(u, u))))


def cg(A, b, x0=None, tol=1e-10, maxiter=10000, true_residual=True):
    """Conjugate gradient for Hermitian positive definite A (callable).

    Stops when ||b - A x|| / ||b|| <= tol (recurrence residual), then, if
    ``true_residual``, recomputes the residual explicitly for the report.
    """
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = _nrm(b)
    if bn == 0.0:
        return np.zeros_like(b), dict(iters=0, mvp=0, history=[0.0], relres=0.0)
    r = b - A(x) if x0 is not None else b.copy()
    mvp = 1 if x0 is not None else 0
    p = r.copy()
    rr = np.real(_dot(r, r))
    hist = [np.sqrt(rr) / bn]
    it = 0
    while it < maxiter and hist[-1] > tol:
        q = A(p)
        mvp += 1
        alpha = rr / np.real(_dot(p, q))
        x += alpha * p
        r -= alpha * q
        rr_new = np.real(_dot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr) / bn)
    rel = _nrm(b - A(x)) / bn if true_residual else hist[-1]
    return x, dict(iters=it, mvp=mvp, history=hist, relres=rel)


def cgls(M, Mdag, b, x0=None, tol=1e-10, maxiter=10000):
    """CG on M^dag M x = M^dag b, tracking r = b - M x (two MVPs per iteration).

    Recurrences (CGLS form): s = M^dag r, p = s; per iteration
    q = M p, alpha = |s|^2/|q|^2, x += alpha p, r -= alpha q, s = M^dag r,
    beta = |s_new|^2/|s|^2, p = s + beta p.  Stops on ||r||/||b|| <= tol, which is
    the paper's residual "for convergence of M^-1 itself" (Section 2).
    """
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = _nrm(b)
    if bn == 0.0:
        return np.zeros_like(b), dict(iters=0, mvp=0, history=[0.0], relres=0.0)
    mvp = 0
    if x0 is not None:
        r = b - M(x)
        mvp += 1
    else:
        r = b.copy()
    s = Mdag(r)
    mvp += 1
    p = s.copy()
    ss = np.real(_dot(s, s))
    hist = [_nrm(r) / bn]
    it = 0
    while it < maxiter and hist[-1] > tol:
        q = M(p)
        qq = np.real(_dot(q, q))
        alpha = ss / qq
        x += alpha * p
        r -= alpha * q
        s = Mdag(r)
        mvp += 2
        ss_new = np.real(_dot(s, s))
        p = s + (ss_new / ss) * p
        ss = ss_new
        it += 1
        hist.append(_nrm(r) / bn)
    rel = _nrm(b - M(x)) / bn
    return x, dict(iters=it, mvp=mvp, history=hist, relres=rel)


def minres(A, b, x0=None, tol=1e-10, maxiter=10000):
    """Paige-Saunders MinRes for Hermitian A (callable), possibly indefinite.

    Lanczos: beta_{j+1} v_{j+1} = A v_j - alpha_j v_j - beta_j v_{j-1}; the
    (j+1) x j tridiagonal is reduced by Givens rotations G_j = [[c, s], [-s, c]],
    and the solution is advanced along d_j = (v_j - delta_j d_{j-1} - eps_j d_{j-2})/gamma_j.
    |eta| after each step is the norm of the minimised residual.
    """
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = _nrm(b)
    if bn == 0.0:
        return np.zeros_like(b), dict(iters=0, mvp=0, history=[0.0], relres=0.0)
    mvp = 0
    if x0 is not None:
        r0 = b - A(x)
        mvp += 1
    else:
        r0 = b.copy()
    beta1 = _nrm(r0)
    hist = [beta1 / bn]
    if beta1 == 0.0:
        return x, dict(iters=0, mvp=mvp, history=hist, relres=0.0)
    v_prev = np.zeros_like(b)
    v = r0 / beta1
    beta = 0.0              # coupling beta_j to the previous Lanczos vector
    c_old, s_old = 1.0, 0.0  # rotation G_{j-2}
    c, s = 1.0, 0.0          # rotation G_{j-1}
    d1 = np.zeros_like(b)    # d_{j-1}
    d2 = np.zeros_like(b)    # d_{j-2}
    eta = beta1
    it = 0
    while it < maxiter and hist[-1] > tol:
        w = A(v)
        mvp += 1
        w = w - beta * v_prev
        alpha = float(np.real(_dot(v, w)))
        w = w - alpha * v
        beta_next = _nrm(w)
        # apply G_{j-2} and G_{j-1} to the new column (beta_j, alpha_j, beta_{j+1})
        eps = s_old * beta
        delta_t = c_old * beta
        delta = c * delta_t + s * alpha
        gbar = -s * delta_t + c * alpha
        gamma = np.hypot(gbar, beta_next)
        if gamma == 0.0:
            break
        c_new, s_new = gbar / gamma, beta_next / gamma
        d = (v - delta * d1 - eps * d2) / gamma
        tau = c_new * eta
        x += tau * d
        eta = -s_new * eta
        d2, d1 = d1, d
        c_old, s_old, c, s = c, s, c_new, s_new
        it += 1
        hist.append(abs(eta) / bn)
        if beta_next == 0.0:
            break
        v_prev, v = v, w / beta_next
        beta = beta_next
    rel = _nrm(b - A(x)) / bn
    return x, dict(iters=it, mvp=mvp, history=hist, relres=rel)


def residual_polynomial_values(history_solver: str, theta: np.ndarray, lam: np.ndarray):
    """Value of the residual polynomial p(lambda) = prod(1 - lambda/theta_i) at ``lam``.

    For CG the zeros theta_i are the Ritz values of the Lanczos tridiagonal
    T_m; for MinRes they are the harmonic Ritz values (Section 1, Figs. 1 and 3).
    p(0) = 1 by construction.
    """
    lam = np.asarray(lam, dtype=np.float64)
    p = np.ones_like(lam)
    for t in theta:
        p = p * (1.0 - lam / t)
    return p


def lanczos_tridiagonal(A, r0, m):
    """m steps of Lanczos from r0 (full reorthogonalisation), returning T-bar ((m+1) x m)."""
    n = r0.shape[0]
    V = np.zeros((n, m + 1), dtype=np.complex128)
    T = np.zeros((m + 1, m))
    V[:, 0] = r0 / _nrm(r0)
    for j in range(m):
        w = A(V[:, j])
        for _ in range(2):
            h = V[:, : j + 1].conj().T @ w
            w = w - V[:, : j + 1] @ h
            if _ == 0:
                T[j, j] = np.real(h[j])
            else:
                T[j, j] += np.real(h[j])
        if j > 0:
            T[j - 1, j] = T[j, j - 1]
        T[j + 1, j] = _nrm(w)
        V[:, j + 1] = w / T[j + 1, j]
    return T, V
