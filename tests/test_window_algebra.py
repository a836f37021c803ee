"""The windowed MinRes reformulation used by the batched solver, modelled in FP64 numpy: the
Lanczos vectors are kept unnormalised (u_j = n_j v_j), each Givens rotation's (tau, delta, eps,
gamma, n_j) is recorded, and every W iterations the search directions
d_j = (u_j / n_j - delta_j d_{j-1} - eps_j d_{j-2}) / gamma_j are carried as coefficient
vectors over (d_{J-1}, d_J, u_{J+1..J+W}), giving the window's share sum_j tau_j d_j of the
solution and the last two directions.  After any number of iterations and for any window the
result equals the oracle's Paige-Saunders MinRes (three-term direction update every
iteration).  This pins the algebra; the kernels themselves are checked on the GPU against the
fused form and against dense solves."""
import math

import numpy as np
import pytest

from oracle import krylov


def _windowed_minres(A, b, iters, W):
    n = b.size
    R = W + 2
    ring = np.zeros((R, n), complex)
    eta = np.linalg.norm(b)
    ring[1] = b / eta                     # u_1 (normalised), u_0 = 0 in slot 0
    S = dict(beta=0.0, cold=1.0, sold=0.0, c=1.0, s=0.0, eta=eta, ncur=1.0, nprev=1.0)
    d1 = np.zeros(n, complex)             # d_J
    d2 = np.zeros(n, complex)             # d_{J-1}
    e = np.zeros(n, complex)
    rot = []
    J = 0

    def flush():
        nonlocal d1, d2, e, J, rot
        L = len(rot)
        basis = [d2, d1] + [ring[(J + k) % R] for k in range(1, L + 1)]
        nb = L + 2
        dm2, dm1, cx = np.eye(nb)[0], np.eye(nb)[1], np.zeros(nb)
        for i, (tau, delta, eps, gamma, nj) in enumerate(rot, start=1):
            d = (np.eye(nb)[1 + i] / nj - delta * dm1 - eps * dm2) / gamma
            cx += tau * d
            dm2, dm1 = dm1, d
        B = np.array(basis)
        e, d1, d2 = e + cx @ B, dm1 @ B, dm2 @ B
        J += L
        rot = []

    for j in range(iters):
        u = ring[(j + 1) % R]
        w = A(u / S["ncur"])
        alpha = float(np.real(np.vdot(u, w))) / S["ncur"]
        un = w - (alpha / S["ncur"]) * u - (S["beta"] / S["nprev"]) * ring[j % R]
        ring[(j + 2) % R] = un
        bnext = np.linalg.norm(un)
        eps = S["sold"] * S["beta"]
        dt = S["cold"] * S["beta"]
        delta = S["c"] * dt + S["s"] * alpha
        gbar = -S["s"] * dt + S["c"] * alpha
        gamma = math.hypot(gbar, bnext)
        cn, sn = gbar / gamma, bnext / gamma
        tau = cn * S["eta"]
        S.update(eta=-sn * S["eta"], cold=S["c"], sold=S["s"], c=cn, s=sn, beta=bnext, nprev=S["ncur"], ncur=bnext)
        rot.append((tau, delta, eps, gamma, S["nprev"]))
        if (j + 1) % W == 0:
            flush()
    flush()
    return e, abs(S["eta"])


def _problem(n=400, seed=11):
    rng = np.random.default_rng(seed)
    H = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = H + H.conj().T                     # Hermitian, indefinite
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return H, b


@pytest.mark.parametrize("W", [1, 2, 3, 8, 64])
@pytest.mark.parametrize("iters", [1, 2, 5, 16, 37, 65])
def test_windowed_update_equals_three_term_minres(W, iters):
    """Up to 65 iterations on a 400 x 400 matrix (before the Lanczos vectors lose
    orthogonality, past which the two Lanczos orderings drift apart whatever the window)."""
    H, b = _problem()
    A = lambda v: H @ v  # noqa: E731
    x_ref, info = krylov.minres(A, b, tol=0.0, maxiter=iters)
    assert info["iters"] == iters
    x, eta = _windowed_minres(A, b, iters, W)
    assert np.linalg.norm(x - x_ref) <= 1e-11 * np.linalg.norm(x_ref)
    # |eta| is the norm of the minimised residual, as in the oracle's history
    assert abs(eta / np.linalg.norm(b) - info["history"][-1]) <= 1e-12
    assert abs(np.linalg.norm(b - H @ x) - eta) <= 1e-9 * np.linalg.norm(b)


@pytest.mark.parametrize("W", [2, 3, 8, 64])
def test_window_length_only_regroups_the_update(W):
    """Over the same Lanczos run (130 iterations, past the loss of orthogonality), every window
    length gives the per-iteration (W = 1) solution to rounding."""
    H, b = _problem()
    A = lambda v: H @ v  # noqa: E731
    x1, eta1 = _windowed_minres(A, b, 130, 1)
    x, eta = _windowed_minres(A, b, 130, W)
    assert np.linalg.norm(x - x1) <= 1e-11 * np.linalg.norm(x1)
    assert eta == eta1
