"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: closed forms,
algebraic identities, library routines (scipy/LAPACK), dense solves on tiny
lattices, special cases that reduce to a textbook method, and the counts the
paper prints for its diagonal examples (Section 1).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from lattice_inputs import (diag_spectrum_indefinite, diag_spectrum_positive, gaussian_spinor, gaussian_vector,
                            su3_links, volume)
from oracle import deflated, dirac, krylov

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- gamma matrices and links
def test_gamma_algebra():
    g = dirac.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * (mu == nu) * np.eye(4))
        for s in (+1, -1):
            assert np.linalg.matrix_rank(np.eye(4) + s * g[mu]) == 2
    assert np.allclose(dirac.GAMMA5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims,seed", [((2, 2, 2, 2), 0), ((4, 4, 4, 4), 3)])
def test_links_are_su3(dims, seed):
    U = su3_links(dims, seed)
    eye = np.einsum("smij,smkj->smik", U, U.conj())
    assert np.max(np.abs(eye - np.eye(3))) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-14
    # the field is not trivial: eps = 0.5 moves links well away from 1
    assert np.mean(np.abs(U - np.eye(3))) > 0.05


# ---------------------------------------------------------------- Wilson operator
def test_free_field_closed_form():
    """Dense M^dag M at U = 1 has the closed-form plane-wave spectrum (x12 multiplicity)."""
    dims = (2, 2, 2, 4)
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), complex)
    U[:] = np.eye(3)
    for kappa in (0.11, 0.124):
        op = dirac.WilsonOperator(U, dims, kappa)
        ev = np.linalg.eigvalsh(dirac.dense(op.MdagM, op.n))
        assert np.max(np.abs(ev - dirac.free_mdagm_spectrum(dims, kappa))) < 1e-13
        # gamma5 M: +-sqrt(M^dag M(p)), each sign with multiplicity 6
        evg = np.sort(np.linalg.eigvalsh(dirac.dense(op.g5M, op.n)))
        lam = np.sqrt(dirac.free_mdagm_spectrum(dims, kappa)[::2])
        assert np.max(np.abs(evg - np.sort(np.concatenate([lam, -lam])))) < 1e-13


def test_gamma5_hermiticity_and_adjoint():
    dims = (2, 2, 2, 2)
    U = su3_links(dims, 7)
    op = dirac.WilsonOperator(U, dims, 0.13)
    M = dirac.dense(op.M, op.n)
    Md = dirac.dense(op.Mdag, op.n)
    G = dirac.dense(op.g5M, op.n)
    assert np.max(np.abs(Md - M.conj().T)) < 1e-15
    assert np.max(np.abs(G - G.conj().T)) < 1e-15
    assert np.max(np.abs(dirac.dense(op.MdagM, op.n) - Md @ M)) < 1e-14


def test_gauge_covariance():
    """M[U^g](g psi) = g M[U] psi with U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    dims = (4, 2, 3, 4)
    V = volume(dims)
    U = su3_links(dims, 1)
    g = su3_links(dims, 2, eps=2.0)[:, 0]  # a random SU(3) matrix per site
    sh = (dims[3], dims[2], dims[1], dims[0])
    gs = g.reshape(sh + (3, 3))
    Ug = np.empty_like(U)
    for mu in range(4):
        gfwd = np.roll(gs, -1, axis=3 - mu).reshape(V, 3, 3)
        Ug[:, mu] = g @ U[:, mu] @ gfwd.conj().transpose(0, 2, 1)
    psi = gaussian_spinor(dims, 3)
    gpsi = np.einsum("sab,sxb->sxa", g, psi)
    lhs = dirac.wilson(Ug, gpsi, dims, 0.14)
    rhs = np.einsum("sab,sxb->sxa", g, dirac.wilson(U, psi, dims, 0.14))
    assert np.max(np.abs(lhs - rhs)) < 1e-13


def test_hopping_neighbour_structure():
    """A point source at site s spreads only to s and its 8 neighbours (periodic)."""
    dims = (4, 3, 5, 2)
    V = volume(dims)
    U = su3_links(dims, 4)
    b = np.zeros((V, 4, 3), complex)
    s = 1 + 4 * (2 + 3 * (3 + 5 * 1))
    b[s, 1, 2] = 1.0
    out = dirac.hopping(U, b, dims)
    nz = set(np.nonzero(np.abs(out).sum(axis=(1, 2)))[0])
    x, y, z, t = 1, 2, 3, 1
    nb = set()
    for d, L in zip(range(4), dims):
        for step in (1, -1):
            c = [x, y, z, t]
            c[d] = (c[d] + step) % L
            nb.add(c[0] + 4 * (c[1] + 3 * (c[2] + 5 * c[3])))
    assert nz == nb


def test_c_transcription_equals_numpy():
    """The OpenMP C loops (used where numpy is too slow) give the numpy transcription's M."""
    from oracle import cwilson
    dims = (4, 3, 5, 6)
    U = su3_links(dims, 1)
    b = gaussian_spinor(dims, 2).ravel()
    a = dirac.WilsonOperator(U, dims, 0.13)
    c = cwilson.CWilson(U, dims, 0.13)
    for f in ("M", "Mdag", "g5M", "MdagM"):
        assert np.max(np.abs(getattr(a, f)(b) - getattr(c, f)(b))) < 1e-14


# ---------------------------------------------------------------- diagonal examples (Section 1)
def test_indefinite_example_has_22_negatives():
    d = diag_spectrum_indefinite(5)
    assert d.shape == (1000,) and int((d < 0).sum()) == 22


@pytest.mark.parametrize("which", ["positive", "indefinite"])
def test_cg_minres_match_scipy(which):
    """Iterates after j steps equal scipy's CG / MinRes (a library routine) on the diagonal examples.

    MinRes is compared before the Lanczos vectors lose orthogonality (j <= 40); past that point
    every unreorthogonalised implementation is delayed by its own rounding.
    """
    lam = diag_spectrum_positive() if which == "positive" else diag_spectrum_indefinite()
    A = lambda v: lam * v
    b = np.random.default_rng(9).standard_normal(1000)  # real: scipy's minres is real-only
    Aop = spla.LinearOperator((1000, 1000), matvec=A, dtype=float)
    for j in (10, 25, 40):
        xs, _ = spla.minres(Aop, b, rtol=1e-300, maxiter=j)
        xo, _ = krylov.minres(A, b, tol=0, maxiter=j)
        assert np.linalg.norm(xs - xo) / np.linalg.norm(xs) < 1e-8
    for j in (10, 60, 150):
        xs, _ = spla.cg(Aop, b, rtol=1e-300, atol=0, maxiter=j)
        xo, _ = krylov.cg(A, b, tol=0, maxiter=j)
        assert np.linalg.norm(xs - xo) / np.linalg.norm(xs) < 1e-10
    # same stopping rule ||r|| <= tol ||b||: same iteration count
    it = [0]
    spla.cg(Aop, b, rtol=1e-8, atol=0, maxiter=2000, callback=lambda *_: it.__setitem__(0, it[0] + 1))
    x, info = krylov.cg(A, b, tol=1e-8, maxiter=2000)
    assert abs(info["iters"] - it[0]) <= 2
    xm, im = krylov.minres(A, b, tol=1e-8, maxiter=2000)
    assert im["relres"] <= 1.01e-8
    assert np.max(np.abs(xm - b / lam)) / np.max(np.abs(b / lam)) < 1e-5
    # the paper: MinRes converges slightly faster than CG on both examples (Figs. 2 and 4)
    assert im["iters"] <= info["iters"]


@pytest.mark.parametrize("which", ["positive", "indefinite"])
def test_minres_residual_never_above_cg(which):
    """MinRes minimises ||r|| over the same Krylov space CG iterates in (Eq. 1)."""
    lam = diag_spectrum_positive() if which == "positive" else diag_spectrum_indefinite()
    A = lambda v: lam * v
    b = gaussian_vector(1000, 2)
    _, i1 = krylov.cg(A, b, tol=1e-10, maxiter=400)
    _, i2 = krylov.minres(A, b, tol=1e-10, maxiter=400)
    n = min(len(i1["history"]), len(i2["history"]))
    assert np.all(np.array(i2["history"][:n]) <= np.array(i1["history"][:n]) * (1 + 1e-8))


def test_cg_a_norm_error_monotone():
    lam = diag_spectrum_positive()
    b = gaussian_vector(1000, 4)
    xs = b / lam
    errs = []
    for j in range(0, 120, 10):
        x, _ = krylov.cg(lambda v: lam * v, b, tol=0, maxiter=j)
        e = x - xs
        errs.append(np.sqrt(np.real(np.vdot(e, lam * e))))
    assert all(a >= b_ for a, b_ in zip(errs, errs[1:]))


@pytest.mark.parametrize("j", [10, 40, 70])
def test_residual_polynomials(j):
    """r_j = p_j(A) b with p(0) = 1: CG zeros at the Ritz values of T_j, MinRes zeros at the
    harmonic Ritz values (the polynomials of Figs. 1 and 3)."""
    lam = diag_spectrum_positive()
    A = lambda v: lam * v
    b = np.ones(1000, complex)
    T, _ = krylov.lanczos_tridiagonal(A, b, j)
    x, _ = krylov.cg(A, b, tol=0, maxiter=j)
    p = krylov.residual_polynomial_values("cg", np.linalg.eigvalsh(T[:j, :j]), lam)
    r = b - A(x)
    assert np.linalg.norm(r - p * b) / np.linalg.norm(r) < 1e-10
    x, _ = krylov.minres(A, b, tol=0, maxiter=j)
    mu = sla.eigh(T[:j, :j], T.T @ T, eigvals_only=True)
    p = krylov.residual_polynomial_values("minres", 1 / mu, lam)
    r = b - A(x)
    assert np.linalg.norm(r - p * b) / np.linalg.norm(r) < 1e-9
    assert krylov.residual_polynomial_values("cg", np.array([2.0, 5.0]), np.array([0.0]))[0] == 1.0


def test_knee_after_deflation_of_small_eigenvalues():
    """Super-linear convergence after about 125 iterations on the indefinite example (Fig. 4)."""
    lam = diag_spectrum_indefinite()
    b = gaussian_vector(1000, 3)
    _, info = krylov.minres(lambda v: lam * v, b, tol=1e-10, maxiter=600)
    l10 = np.log10(info["history"])
    early = (l10[100] - l10[20]) / 80
    late = (l10[250] - l10[150]) / 100
    assert late < 4 * early < 0


def test_cgls_matches_dense_solve():
    dims = (2, 2, 2, 2)
    U = su3_links(dims, 5)
    op = dirac.WilsonOperator(U, dims, 0.12)
    b = gaussian_spinor(dims, 6).ravel()
    x, info = krylov.cgls(op.M, op.Mdag, b, tol=1e-12)
    xd = np.linalg.solve(dirac.dense(op.M, op.n), b)
    assert info["relres"] <= 1e-12
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


# ---------------------------------------------------------------- Lan-DR / MinRes-DR special cases
def test_landr_first_cycle_is_m_cg_steps():
    """One Lan-DR cycle is the Galerkin (FOM) solve on K_m, i.e. CG after m steps."""
    lam = diag_spectrum_positive()
    A = lambda v: lam * v
    b = gaussian_vector(1000, 10)
    m = 40
    x1, _, info = deflated.lan_dr(A, b, m, 10, 1e-14, max_mvp=m + 1)
    assert info["cycles"] == 1
    xc, _ = krylov.cg(A, b, tol=0, maxiter=m)
    assert np.linalg.norm(x1 - xc) / np.linalg.norm(xc) < 1e-10


def test_minresdr_first_cycle_is_m_minres_steps():
    lam = diag_spectrum_indefinite()
    A = lambda v: lam * v
    b = gaussian_vector(1000, 11)
    m = 30  # before the unreorthogonalised MinRes recurrence drifts
    x1, _, info = deflated.minres_dr(A, b, m, 10, 1e-14, max_mvp=m + 1)
    assert info["cycles"] == 1
    xm, _ = krylov.minres(A, b, tol=0, maxiter=m)
    assert np.linalg.norm(x1 - xm) / np.linalg.norm(xm) < 1e-11


def test_landr_exact_spectrum_of_positive_example():
    """Lan-DR(60,20) on diag(0.1, 1, ..., 999): x = b / lambda and the 20 smallest eigenvalues."""
    lam = diag_spectrum_positive()
    A = lambda v: lam * v
    b = gaussian_vector(1000, 7)
    x, eig, info = deflated.lan_dr(A, b, 60, 20, 1e-12)
    assert info["relres"] <= 1e-12
    assert np.max(np.abs(x - b / lam)) / np.max(np.abs(b / lam)) < 1e-10
    assert np.max(np.abs(eig["vals"] - lam[:20]) / lam[:20]) < 1e-10
    Y = eig["vecs"]
    assert np.max(np.abs(Y.conj().T @ Y - np.eye(20))) < 1e-12
    # the residual norms from the projected matrix equal the explicit ones
    R = lam[:, None] * Y - Y * eig["vals"]
    assert np.allclose(np.linalg.norm(R, axis=0), eig["rho"], atol=1e-10 * lam.max())
    assert info["mvp"] <= 2 * info["mvp_lin"] + 61  # at most a factor of two, plus the last cycle


def test_minresdr_exact_spectrum_of_indefinite_example():
    lam = diag_spectrum_indefinite()
    A = lambda v: lam * v
    b = gaussian_vector(1000, 8)
    x, eig, info = deflated.minres_dr(A, b, 80, 20, 1e-12)
    assert info["relres"] <= 1e-12
    assert np.max(np.abs(x - b / lam)) / np.max(np.abs(b / lam)) < 1e-9
    want = np.sort(np.abs(lam))[:10]
    got = np.sort(np.abs(eig["vals"]))[:10]
    assert np.max(np.abs(got - want) / want) < 1e-9
    Y = eig["vecs"]
    assert np.max(np.abs(Y.conj().T @ Y - np.eye(20))) < 1e-12
    R = lam[:, None] * Y - Y * eig["vals"]
    assert np.allclose(np.linalg.norm(R, axis=0), eig["rho"], atol=1e-10 * np.abs(lam).max())


def test_harmonic_ritz_two_forms_agree():
    """T_m g = mu Tbar^T Tbar g (theta = 1/mu) equals eig(T_m + beta_m^2 T_m^-1 e_m e_m^T)."""
    lam = diag_spectrum_indefinite()
    T, _ = krylov.lanczos_tridiagonal(lambda v: lam * v, gaussian_vector(1000, 1), 40)
    theta, _ = deflated._harmonic_ritz(T)
    Tm = T[:40, :40]
    em = np.zeros(40)
    em[-1] = 1.0
    other = np.linalg.eigvals(Tm + T[40, 39] ** 2 * np.outer(np.linalg.solve(Tm, em), em))
    assert np.allclose(np.sort(theta), np.sort(other.real), rtol=1e-8, atol=1e-10)


def test_deflated_with_k0_is_plain():
    lam = diag_spectrum_indefinite()
    A = lambda v: lam * v
    b = gaussian_vector(1000, 12)
    Y = np.zeros((1000, 0), complex)
    H = np.zeros((0, 0))
    x1, i1 = deflated.d_minres(A, b, Y, H, 1e-10)
    x2, i2 = krylov.minres(A, b, tol=1e-10)
    assert i1["iters"] == i2["iters"] and np.allclose(x1, x2, rtol=0, atol=1e-14)
    lam_p = diag_spectrum_positive()
    x3, i3 = deflated.d_cg(lambda v: lam_p * v, b, Y, H, 1e-10)
    x4, i4 = krylov.cg(lambda v: lam_p * v, b, tol=1e-10)
    assert i3["iters"] == i4["iters"]


def test_projection_over_exact_eigenvectors_solves_in_span():
    """b in span(Y) with exact eigenvectors: the Galerkin projection alone solves the system."""
    lam = diag_spectrum_positive()
    A = lambda v: lam * v
    Y = np.eye(1000, dtype=complex)[:, :15]
    H = deflated.projection_matrix(A, Y)
    b = Y @ (gaussian_vector(15, 3))
    x, info = deflated.d_cg(A, b, Y, H, 1e-12)
    assert info["iters"] == 0 and info["relres"] < 1e-14
    x, info = deflated.d_minres(A, b, Y, H, 1e-12)
    assert info["iters"] == 0


def test_deflation_speeds_up_later_rhs():
    lam = diag_spectrum_indefinite()
    A = lambda v: lam * v
    _, eig, _ = deflated.minres_dr(A, gaussian_vector(1000, 1), 80, 30, 1e-10)
    H = deflated.projection_matrix(A, eig["vecs"])
    b2 = gaussian_vector(1000, 2)
    _, i_d = deflated.d_minres(A, b2, eig["vecs"], H, 1e-10)
    _, i_p = krylov.minres(A, b2, tol=1e-10)
    assert i_d["relres"] <= 1e-10 and i_d["iters"] < 0.6 * i_p["iters"]


# ---------------------------------------------------------------- the 4^4 near-critical lattice
@pytest.fixture(scope="module")
def c1():
    with open(os.path.join(GOLDEN, "kappa.json")) as fh:
        e = json.load(fh)["4x4x4x4"]
    dims = tuple(e["dims"])
    U = su3_links(dims, e["seed"], e["eps"])
    op = dirac.WilsonOperator(U, dims, e["kappa"])
    M = dirac.dense(op.M, op.n)
    return dict(e=e, op=op, M=M, G=np.diag(np.tile([1.0] * 6 + [-1.0] * 6, op.V)) @ M)


def test_kappa_golden_hits_target(c1):
    ev = np.linalg.eigvalsh(c1["G"])
    mn = np.min(np.abs(ev))
    assert abs(mn - c1["e"]["target"]) <= 0.05 * c1["e"]["target"]
    assert c1["e"]["kappa"] < c1["e"]["dip_kappa"]  # lower side of the first dip


def test_landr_on_lattice_vs_dense(c1):
    op, M = c1["op"], c1["M"]
    b = gaussian_spinor(op.dims, 100).ravel()
    # the normal equations square the condition number: the true residual floors near 1e-11
    x, eig, info = deflated.lan_dr(op.MdagM, op.Mdag(b), 60, 20, 1e-11,
                                  residual=lambda x: np.linalg.norm(b - op.M(x)) / np.linalg.norm(b),
                                  apv=2, mvp0=1, max_mvp=20000)
    xd = np.linalg.solve(M, b)
    assert info["relres"] <= 1e-11
    assert info["relres"] == min(info["history"])
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
    ev = np.linalg.eigvalsh(M.conj().T @ M)[:20]
    assert np.max(np.abs(np.sort(eig["vals"]) - ev) / ev) < 1e-8


def test_minresdr_on_lattice_vs_dense(c1):
    op, G = c1["op"], c1["G"]
    b = gaussian_spinor(op.dims, 100).ravel()
    x, eig, info = deflated.minres_dr(op.g5M, op.g5(b), 60, 20, 1e-12,
                                     residual=lambda x: np.linalg.norm(b - op.M(x)) / np.linalg.norm(b),
                                     max_mvp=20000)
    assert info["relres"] <= 1e-12
    xd = np.linalg.solve(c1["M"], b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
    ev = np.linalg.eigvalsh(G)
    want = np.sort(np.abs(ev))[:10]
    got = np.sort(np.abs(eig["vals"]))[:10]
    assert np.max(np.abs(got - want) / want) < 1e-8


# ---------------------------------------------------------------- kappa search on large lattices
def _dense_min_abs_eig_g5m(U, dims, kappa):
    op = dirac.WilsonOperator(U, dims, kappa)
    G = dirac.dense(op.g5M, op.n)
    return float(np.min(np.abs(np.linalg.eigvalsh(G))))


@pytest.mark.parametrize("dims,seed,check", [((2, 2, 2, 2), 1, 40), ((4, 4, 4, 4), 3, 200)])
def test_lanczos_min_eig_against_dense_spectrum(c1, dims, seed, check):
    """The plain Lanczos estimate of lambda_min(M^dag M) that fixes kappa on large lattices
    equals the smallest eigenvalue of the dense M^dag M (4^4: the near-critical C1 field)."""
    from oracle import kappa as kap
    from oracle.cwilson import CWilson
    k = c1["e"]["kappa"] if dims == (4, 4, 4, 4) else 0.13
    U = su3_links(dims, seed, 0.5)
    op = CWilson(U, dims, k)
    th, steps = kap.lanczos_min_eig(op.MdagM, op.n, check=check)
    M = c1["M"] if dims == (4, 4, 4, 4) else dirac.dense(dirac.WilsonOperator(U, dims, k).M, op.n)
    lmin = float(np.linalg.eigvalsh(M.conj().T @ M)[0])
    # Ritz values approach lambda_min from above; the stop rule leaves < 1e-3 relative
    assert th >= lmin * (1 - 1e-9) and (th - lmin) / lmin < 1e-3, (th, lmin, steps)


def test_lanczos_min_eig_against_arpack_6x6x6x6():
    """On 6^4 (n = 15552, beyond a dense eigensolve) the estimate agrees with ARPACK's smallest
    algebraic eigenvalue of M^dag M (a library routine over the same operator)."""
    from oracle import kappa as kap
    from oracle.cwilson import CWilson
    dims = (6, 6, 6, 6)
    op = CWilson(su3_links(dims, 0, 0.5), dims, 0.12)
    lo = spla.LinearOperator((op.n, op.n), matvec=op.MdagM, dtype=np.complex128)
    ref = float(spla.eigsh(lo, k=1, which="SA", tol=1e-10, v0=gaussian_vector(op.n, 4), ncv=40)[0][0])
    th, _ = kap.lanczos_min_eig(op.MdagM, op.n)
    assert abs(th - ref) / ref < 1e-3, (th, ref)


def test_search_large_lands_on_target_of_dense_spectrum(c1):
    """The secant search used for the large lattices, run on 4^4, returns a kappa on the lower
    side of the first dip whose dense min|lambda(gamma5 M)| is the target (a missing square root
    or an early Lanczos stop would land elsewhere)."""
    from oracle import kappa as kap
    e = c1["e"]
    dims = tuple(e["dims"])
    target = 2e-2
    res = kap.search_large(dims, target, seed=e["seed"], eps=e["eps"], k0=0.135, k1=0.14, log=lambda m: None)
    assert res["kappa"] < e["dip_kappa"]
    got = _dense_min_abs_eig_g5m(su3_links(dims, e["seed"], e["eps"]), dims, res["kappa"])
    assert abs(got - target) <= 0.06 * target, (res, got)


# ---------------------------------------------------------------- D-CG on the normal equations
def _svd_operator(n, seed):
    """M = Q1 diag(s) Q2^H with known right singular vectors Q2 (eigenvectors of M^dag M)."""
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    s = np.geomspace(1e-3, 2.0, n)
    M = (Q1 * s) @ Q2.conj().T
    return M, Q2, s


def test_d_cg_normal_with_k0_is_cgls():
    M, _, _ = _svd_operator(120, 21)
    Mf, Mh = (lambda v: M @ v), (lambda v: M.conj().T @ v)
    b = gaussian_vector(120, 22)
    x1, i1 = deflated.d_cg_normal(Mf, Mh, b, np.zeros((120, 0), complex), np.zeros((0, 0)), 1e-10)
    x2, i2 = krylov.cgls(Mf, Mh, b, tol=1e-10)
    assert i1["iters"] == i2["iters"] and i1["history"] == i2["history"]
    assert np.allclose(x1, x2, rtol=0, atol=1e-14)


def test_d_cg_normal_exact_eigenvectors_solve_in_span():
    """M^dag b in span(Y) for exact eigenvectors Y of M^dag M: the projection of the
    normal-equation residual alone gives x, and CGLS takes no iteration."""
    n, k = 150, 12
    M, Q2, s = _svd_operator(n, 23)
    Y = Q2[:, :k]
    A = lambda v: M.conj().T @ (M @ v)
    H = deflated.projection_matrix(A, Y)
    xt = Y @ gaussian_vector(k, 24)
    b = M @ xt
    x, info = deflated.d_cg_normal(lambda v: M @ v, lambda v: M.conj().T @ v, b, Y, H, 1e-12)
    assert info["iters"] == 0 and info["relres"] < 1e-12
    assert np.linalg.norm(x - xt) / np.linalg.norm(xt) < 1e-10


def test_d_cg_normal_galerkin_condition_and_lattice_solution(c1):
    """After the projection the normal-equation residual M^dag (b - M x0) is orthogonal to Y
    (Galerkin condition); on the 4^4 lattice with the 20 lowest dense eigenvectors of M^dag M
    the deflated solve equals the dense solution and needs fewer iterations than CGLS."""
    from oracle.cwilson import CWilson
    M = c1["M"]
    op = CWilson(su3_links(c1["op"].dims, c1["e"]["seed"], c1["e"]["eps"]), c1["op"].dims, c1["e"]["kappa"])
    lam, Z = np.linalg.eigh(M.conj().T @ M)
    Y = Z[:, :20]
    H = deflated.projection_matrix(op.MdagM, Y)
    b = gaussian_spinor(c1["op"].dims, 102).ravel()
    x0, i0 = deflated.d_cg_normal(op.M, op.Mdag, b, Y, H, 1e-10, maxiter=0)
    assert i0["iters"] == 0
    g = Y.conj().T @ op.Mdag(b - op.M(x0))
    assert np.max(np.abs(g)) < 1e-12 * np.linalg.norm(op.Mdag(b))
    x, info = deflated.d_cg_normal(op.M, op.Mdag, b, Y, H, 1e-12)
    xd = np.linalg.solve(M, b)
    assert info["relres"] <= 1e-12 and np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
    # plain CGLS has not converged after twice the deflated iteration count
    _, ip = krylov.cgls(op.M, op.Mdag, b, tol=1e-12, maxiter=2 * info["iters"])
    assert ip["relres"] > 1e-12
