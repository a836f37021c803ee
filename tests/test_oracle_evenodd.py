"""Pins of the even-odd (Schur complement) oracle (CPU only): the dense block definition of the
Schur complement, the solution of the full system, det M = det Mhat, the eigenvalue map
mu -> mu (2 - mu) from the spectrum of M, gamma5-hermiticity, and the deflated solvers on the
even-site system against dense algebra."""
import json
import os

import numpy as np
import pytest

from lattice_inputs import gaussian_spinor, su3_links
from oracle import deflated, dirac, evenodd, krylov

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(dims, seed, kappa):
    U = su3_links(dims, seed)
    op = dirac.WilsonOperator(U, dims, kappa)
    eo = evenodd.EvenOdd(U, dims, kappa)
    return U, op, eo


def _perm(eo):
    return np.concatenate([12 * s[:, None] + np.arange(12) for s in eo.sites], axis=None).reshape(-1)


def test_parity_and_half_order():
    dims = (4, 2, 2, 6)
    p = evenodd.parity(dims)
    V = int(np.prod(dims))
    assert p.sum() == V // 2
    s = np.arange(V)
    x, y, z, t = s % 4, (s // 4) % 2, (s // 8) % 2, s // 16
    assert np.array_equal(p, (x + y + z + t) % 2)
    # with an even x extent the half-field position of a site is site // 2
    for par in (0, 1):
        assert np.array_equal(np.nonzero(p == par)[0] // 2, np.arange(V // 2))
    with pytest.raises(ValueError):
        evenodd.EvenOdd(su3_links((3, 2, 2, 2), 1), (3, 2, 2, 2), 0.1)


def test_hopping_only_connects_opposite_parities_and_blocks_are_dense_schur():
    dims = (2, 2, 2, 4)
    U, op, eo = _setup(dims, 3, 0.12)
    M = dirac.dense(op.M, op.n)
    P = _perm(eo)
    Mp = M[np.ix_(P, P)]
    n = eo.n
    assert np.allclose(Mp[:n, :n], np.eye(n)) and np.allclose(Mp[n:, n:], np.eye(n))
    S = Mp[:n, :n] - Mp[:n, n:] @ np.linalg.solve(Mp[n:, n:], Mp[n:, :n])
    Sm = dirac.dense(eo.Mhat, n)
    assert np.max(np.abs(S - Sm)) < 1e-13
    # det M = det(M_oo) det(Schur) = det Mhat
    assert abs(np.linalg.slogdet(M)[1] - np.linalg.slogdet(Sm)[1]) < 1e-10


def test_schur_spectrum_is_mu_times_two_minus_mu():
    """Each eigenvalue pair mu, 2 - mu of M (the hopping term's spectrum is symmetric) gives the
    eigenvalue mu (2 - mu) = 1 - kappa^2 lambda^2 of Mhat."""
    dims = (2, 2, 2, 4)
    U, op, eo = _setup(dims, 4, 0.13)
    mu = np.linalg.eigvals(dirac.dense(op.M, op.n))
    want = mu * (2 - mu)
    got = np.linalg.eigvals(dirac.dense(eo.Mhat, eo.n))
    # every eigenvalue of Mhat appears in the map of M's spectrum, which holds each one twice
    d = np.abs(got[:, None] - want[None, :]).min(axis=1)
    assert d.max() < 1e-9
    cnt = (np.abs(want[:, None] - got[None, :]) < 1e-8).sum(axis=0)
    assert np.all(cnt >= 2)


def test_gamma5_hermiticity_and_adjoint():
    dims = (2, 2, 2, 4)
    U, op, eo = _setup(dims, 5, 0.14)
    S = dirac.dense(eo.Mhat, eo.n)
    Sd = dirac.dense(eo.Mhat_dag, eo.n)
    assert np.max(np.abs(Sd - S.conj().T)) < 1e-13
    G = dirac.dense(eo.g5Mhat, eo.n)
    assert np.max(np.abs(G - G.conj().T)) < 1e-13


@pytest.fixture(scope="module")
def c1eo():
    with open(os.path.join(GOLDEN, "kappa.json")) as fh:
        e = json.load(fh)["4x4x4x4"]
    dims = tuple(e["dims"])
    U = su3_links(dims, e["seed"], e["eps"])
    return dict(e=e, dims=dims, U=U, op=dirac.WilsonOperator(U, dims, e["kappa"]),
                eo=evenodd.EvenOdd(U, dims, e["kappa"]))


def test_schur_solution_equals_full_solution(c1eo):
    """prepare -> dense solve of Mhat -> reconstruct gives the solution of M x = b (4^4, near
    critical), and the full residual equals the even-site one."""
    op, eo = c1eo["op"], c1eo["eo"]
    b = gaussian_spinor(c1eo["dims"], 100)
    S = dirac.dense(eo.Mhat, eo.n)
    bh = eo.prepare(b).ravel()
    xe = np.linalg.solve(S, bh)
    x = eo.reconstruct(b, xe)
    M = dirac.dense(op.M, op.n)
    xd = np.linalg.solve(M, b.ravel())
    assert np.linalg.norm(x.ravel() - xd) / np.linalg.norm(xd) < 1e-10
    # an approximate even solution: the full residual is the Schur residual on the even sites
    xa = xe + 1e-6 * gaussian_spinor(c1eo["dims"], 7).ravel()[: eo.n]
    r = b.ravel() - op.M(eo.reconstruct(b, xa).ravel())
    re, ro = eo.split(r)
    assert np.max(np.abs(ro)) < 1e-14
    assert np.allclose(re.ravel(), bh - eo.Mhat(xa), atol=1e-14)


def test_deflated_solvers_on_the_even_system(c1eo):
    """Lan-DR / D-CG on Mhat^dag Mhat and MinRes-DR on gamma5 Mhat: solutions equal the dense
    solve and kept eigenvalues equal the dense spectrum of the Schur form (4^4)."""
    eo = c1eo["eo"]
    b = gaussian_spinor(c1eo["dims"], 100)
    bh = eo.prepare(b).ravel()
    S = dirac.dense(eo.Mhat, eo.n)
    xs = np.linalg.solve(S, bh)
    res = lambda v: np.linalg.norm(bh - eo.Mhat(v)) / np.linalg.norm(bh)
    x, eig, info = deflated.lan_dr(eo.MhatdagMhat, eo.Mhat_dag(bh), 40, 12, 1e-11, residual=res, apv=2,
                                  mvp0=1, max_mvp=20000)
    assert info["relres"] <= 1e-11 and np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8
    ev = np.linalg.eigvalsh(S.conj().T @ S)[:12]
    assert np.max(np.abs(np.sort(eig["vals"]) - ev) / ev) < 1e-8
    x2, eig2, info2 = deflated.minres_dr(eo.g5Mhat, eo.g5(bh), 40, 12, 1e-12, residual=res, max_mvp=20000)
    assert info2["relres"] <= 1e-12 and np.linalg.norm(x2 - xs) / np.linalg.norm(xs) < 1e-8
    evg = np.sort(np.abs(np.linalg.eigvalsh(np.tile([1.0] * 6 + [-1.0] * 6, eo.Vh)[:, None] * S)))[:6]
    assert np.max(np.abs(np.sort(np.abs(eig2["vals"]))[:6] - evg) / evg) < 1e-8
    # a later rhs: D-CG over the Lan-DR eigenvectors converges faster than plain CGLS
    b2 = eo.prepare(gaussian_spinor(c1eo["dims"], 101)).ravel()
    H = deflated.projection_matrix(eo.MhatdagMhat, eig["vecs"])
    xd, idc = deflated.d_cg_normal(eo.Mhat, eo.Mhat_dag, b2, eig["vecs"], H, 1e-10)
    _, ipl = krylov.cgls(eo.Mhat, eo.Mhat_dag, b2, tol=1e-10)
    assert idc["relres"] <= 1e-10 and idc["iters"] < ipl["iters"]
