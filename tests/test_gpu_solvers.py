"""Solver-level parity of the HIP library with the FP64 oracle (GPU).

C1 workload: 4^4 near-critical lattice (links seed and kappa from the oracle's
kappa search), Lan-DR(60,20) on M^dag M then D-CG, and MinRes-DR(60,20) on
gamma5 M then D-MinRes, for Gaussian right-hand sides.  Both sides run on the
same seeded arrays; the solution is also compared with a dense LU solve and
the eigenvalues with a dense eigendecomposition.
"""
import numpy as np
import pytest

from lattice_inputs import gaussian_spinor, su3_links
from oracle import deflated, dirac, krylov

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def c1dense(c1_config):
    op = dirac.WilsonOperator(c1_config["links"], c1_config["dims"], c1_config["kappa"])
    M = dirac.dense(op.M, op.n)
    g5 = np.tile([1.0] * 6 + [-1.0] * 6, op.V)
    return dict(op=op, M=M, ev_mdagm=np.linalg.eigvalsh(M.conj().T @ M), ev_g5m=np.linalg.eigvalsh(g5[:, None] * M))


def _oracle_relres(op, b, x):
    return np.linalg.norm(b.ravel() - op.M(np.ravel(x))) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def landr_run(gpu_ctx, c1_config, c1dense):
    from paper_0901_3163_amd import deflan
    op = deflan.Operator(gpu_ctx, c1_config["dims"], c1_config["links"], c1_config["kappa"], deflan.DL_MDAGM)
    b = gaussian_spinor(c1_config["dims"], 100)
    x, eig, st = op.solve_first(b, 60, 20, 1e-11)
    ora = c1dense["op"]
    bb = b.ravel()
    xo, eo, io = deflated.lan_dr(ora.MdagM, ora.Mdag(bb), 60, 20, 1e-11,
                                 residual=lambda v: np.linalg.norm(bb - ora.M(v)) / np.linalg.norm(bb),
                                 apv=2, mvp0=1, max_mvp=20000)
    return dict(op=op, b=b, x=x, eig=eig, st=st, xo=xo, eo=eo, io=io)


def test_landr_solution_parity(landr_run, c1dense):
    r = landr_run
    assert r["st"]["status"] == 0
    assert r["st"]["relres"] <= 1e-11
    assert _oracle_relres(c1dense["op"], r["b"], r["x"]) <= 1e-11
    xd = np.linalg.solve(c1dense["M"], r["b"].ravel())
    assert _rel(r["x"], xd) < 1e-8
    assert _rel(r["x"], r["xo"]) < 1e-8
    # same stopping rule on both sides (at most one cycle apart)
    assert abs(r["st"]["mvp"] - r["io"]["mvp"]) <= 2 * 61
    assert r["st"]["stop_rule"] == r["io"]["rule"]
    assert r["st"]["mvp"] <= 2 * r["st"]["mvp_lin"] + 2 * 61  # at most a factor of two (Section 2)


def test_landr_eigen_parity(landr_run, c1dense):
    r = landr_run
    ev, res = r["eig"].info()
    want = c1dense["ev_mdagm"][:20]
    assert np.max(np.abs(np.sort(ev) - want) / want) < 1e-8
    assert np.max(np.abs(np.sort(ev) - np.sort(r["eo"]["vals"])) / want) < 1e-8
    # reported residuals equal the oracle's ||A y - lambda y|| on the returned vectors
    Y = r["eig"].vectors().reshape(20, -1)
    ora = c1dense["op"]
    for i in range(20):
        rr = np.linalg.norm(ora.MdagM(Y[i]) - ev[i] * Y[i])
        assert abs(rr - res[i]) <= 1e-12 + 1e-6 * rr
    assert np.max(np.abs(Y.conj() @ Y.T - np.eye(20))) < 1e-12
    # well-separated low modes: the same eigenvector up to a phase
    Yo = r["eo"]["vecs"].T
    for i in range(5):
        assert abs(np.vdot(Yo[i], Y[np.argsort(ev)[i]])) > 1 - 1e-8


@pytest.mark.parametrize("tol", [1e-10, 1e-11])
def test_dcg_later_rhs(landr_run, c1dense, tol):
    from paper_0901_3163_amd import deflan
    r = landr_run
    dims = r["b"].shape
    B = np.stack([gaussian_spinor((4, 4, 4, 4), 101 + i) for i in range(3)])
    X, sts, rc = r["op"].solve_next(B, r["eig"], tol)
    assert rc == deflan.DL_OK
    ora = c1dense["op"]
    Yo = r["eo"]["vecs"]
    Ho = deflated.projection_matrix(ora.MdagM, Yo)
    for i in range(3):
        assert sts[i]["relres"] <= tol
        assert _oracle_relres(ora, B[i], X[i]) <= tol
        xd = np.linalg.solve(c1dense["M"], B[i].ravel())
        assert _rel(X[i], xd) < (1e-8 if tol <= 1e-11 else 1e-6)
        xo, io = deflated.d_cg_normal(ora.M, ora.Mdag, B[i].ravel(), Yo, Ho, tol)
        # iteration counts of GPU D-CG and oracle D-CG agree closely
        assert abs(sts[i]["iters"] - io["iters"]) <= max(8, 0.1 * io["iters"])
    # deflation pays: plain CG on the normal equations needs several times more iterations
    X0, st0, _ = r["op"].solve_next(B[:1], None, tol)
    assert st0[0]["iters"] > 3 * sts[0]["iters"]


@pytest.fixture(scope="module")
def minresdr_run(gpu_ctx, c1_config, c1dense):
    from paper_0901_3163_amd import deflan
    op = deflan.Operator(gpu_ctx, c1_config["dims"], c1_config["links"], c1_config["kappa"], deflan.DL_G5M)
    b = gaussian_spinor(c1_config["dims"], 100)
    x, eig, st = op.solve_first(b, 60, 20, 1e-12)
    ora = c1dense["op"]
    bb = b.ravel()
    xo, eo, io = deflated.minres_dr(ora.g5M, ora.g5(bb), 60, 20, 1e-12,
                                    residual=lambda v: np.linalg.norm(bb - ora.M(v)) / np.linalg.norm(bb),
                                    max_mvp=20000)
    return dict(op=op, b=b, x=x, eig=eig, st=st, xo=xo, eo=eo, io=io)


def test_minresdr_solution_parity(minresdr_run, c1dense):
    r = minresdr_run
    assert r["st"]["status"] == 0 and r["st"]["relres"] <= 1e-12
    assert _oracle_relres(c1dense["op"], r["b"], r["x"]) <= 1e-12
    xd = np.linalg.solve(c1dense["M"], r["b"].ravel())
    assert _rel(r["x"], xd) < 1e-8
    assert _rel(r["x"], r["xo"]) < 1e-8
    assert abs(r["st"]["mvp"] - r["io"]["mvp"]) <= 2 * 61
    assert r["st"]["stop_rule"] == r["io"]["rule"]


def test_minresdr_eigen_parity(minresdr_run, c1dense):
    r = minresdr_run
    ev, res = r["eig"].info()
    want = np.sort(np.abs(c1dense["ev_g5m"]))[:12]
    got = np.sort(np.abs(ev))[:12]
    assert np.max(np.abs(got - want) / want) < 1e-8
    assert np.max(np.abs(np.sort(ev) - np.sort(r["eo"]["vals"])) / np.abs(np.sort(ev))) < 1e-6
    Y = r["eig"].vectors().reshape(20, -1)
    assert np.max(np.abs(Y.conj() @ Y.T - np.eye(20))) < 1e-12
    ora = c1dense["op"]
    for i in range(20):
        rr = np.linalg.norm(ora.g5M(Y[i]) - ev[i] * Y[i])
        assert abs(rr - res[i]) <= 1e-12 + 1e-6 * rr


@pytest.mark.parametrize("tol", [1e-10, 1e-12])
def test_dminres_later_rhs(minresdr_run, c1dense, tol):
    r = minresdr_run
    B = np.stack([gaussian_spinor((4, 4, 4, 4), 101 + i) for i in range(3)])
    X, sts, rc = r["op"].solve_next(B, r["eig"], tol)
    assert rc == 0
    ora = c1dense["op"]
    Yo = r["eo"]["vecs"]
    Ho = deflated.projection_matrix(ora.g5M, Yo)
    for i in range(3):
        assert sts[i]["relres"] <= tol
        assert _oracle_relres(ora, B[i], X[i]) <= tol
        xd = np.linalg.solve(c1dense["M"], B[i].ravel())
        assert _rel(X[i], xd) < (1e-8 if tol <= 1e-12 else 1e-6)
        xo, io = deflated.d_minres(ora.g5M, ora.g5(B[i].ravel()), Yo, Ho, tol)
        assert abs(sts[i]["iters"] - io["iters"]) <= max(8, 0.1 * io["iters"])


def test_plain_solvers_match_oracle_iteration_counts(gpu_ctx, c1_config, c1dense):
    """eig = NULL: plain CG (normal equations) and MinRes, same iterations as the oracle's."""
    from paper_0901_3163_amd import deflan
    ora = c1dense["op"]
    b = gaussian_spinor(c1_config["dims"], 104)
    for kind in (deflan.DL_MDAGM, deflan.DL_G5M):
        op = deflan.Operator(gpu_ctx, c1_config["dims"], c1_config["links"], c1_config["kappa"], kind)
        X, sts, rc = op.solve_next(b[None], None, 1e-10)
        if kind == deflan.DL_MDAGM:
            _, io = krylov.cgls(ora.M, ora.Mdag, b.ravel(), tol=1e-10, maxiter=20000)
        else:
            _, io = krylov.minres(ora.g5M, ora.g5(b.ravel()), tol=1e-10, maxiter=20000)
        # the GPU polls the residual every 8 iterations
        assert io["iters"] <= sts[0]["iters"] <= io["iters"] + 8
        assert _oracle_relres(ora, b, X[0]) <= 1e-10
        op.close()


# ---------------------------------------------------------------- edge cases
def test_edge_cases(gpu_ctx, c1_config):
    from paper_0901_3163_amd import deflan
    dims, U, kappa = c1_config["dims"], c1_config["links"], c1_config["kappa"]
    op = deflan.Operator(gpu_ctx, dims, U, kappa, deflan.DL_G5M)
    zero = np.zeros((256, 4, 3), complex)
    x, eig, st = op.solve_first(zero, 20, 5, 1e-10)
    assert st["status"] == 0 and np.all(x == 0) and eig.k == 0
    X, sts, rc = op.solve_next(np.zeros((0, 256, 4, 3), complex), None, 1e-10)
    assert rc == 0 and X.shape[0] == 0
    X, sts, rc = op.solve_next(zero[None], None, 1e-10)
    assert rc == 0 and np.all(X == 0)
    b = gaussian_spinor(dims, 7)
    for m, k in ((10, 10), (10, 12), (5000, 3)):
        with pytest.raises(deflan.DeflanError) as ei:
            op.solve_first(b, m, k, 1e-10)
        assert ei.value.code == deflan.DL_E_INVALID
    with pytest.raises(deflan.DeflanError) as ei:
        op.solve_first(b, 20, 5, -1.0)
    assert ei.value.code == deflan.DL_E_INVALID
    bad = b.copy()
    bad[3, 1, 2] = np.nan
    with pytest.raises(deflan.DeflanError) as ei:
        op.solve_first(bad, 20, 5, 1e-10)
    assert ei.value.code == deflan.DL_E_NONFINITE
    # a handle built for one operator is rejected by another
    _, e1, _ = op.solve_first(b, 20, 4, 1e-6)
    other = deflan.Operator(gpu_ctx, dims, U, kappa * 0.99, deflan.DL_G5M)
    with pytest.raises(deflan.DeflanError) as ei:
        other.solve_next(b[None], e1, 1e-10)
    assert ei.value.code == deflan.DL_E_MISMATCH
    # max_mvp reached: NOT_CONVERGED with the best iterate and statistics filled in
    X, sts, rc = op.solve_next(b[None], None, 1e-10, max_mvp=30)
    assert rc == deflan.DL_NOT_CONVERGED and sts[0]["status"] == 1 and 0 < sts[0]["relres"] < 1
    other.close()
    op.close()


def test_k0_first_rhs_is_restarted_minres_and_fom(gpu_ctx, c1_config):
    from paper_0901_3163_amd import deflan
    from oracle import dirac as D
    dims, U = c1_config["dims"], c1_config["links"]
    kappa = 0.12  # far from critical: restarted methods converge quickly
    ora = D.WilsonOperator(U, dims, kappa)
    b = gaussian_spinor(dims, 9)
    for kind in (deflan.DL_MDAGM, deflan.DL_G5M):
        op = deflan.Operator(gpu_ctx, dims, U, kappa, kind)
        x, eig, st = op.solve_first(b, 30, 0, 1e-10)
        assert st["status"] == 0 and st["stop_rule"] == "linear" and eig.k == 0
        assert _oracle_relres(ora, b, x) <= 1e-10
        op.close()


def test_device_pointers_match_host_path(gpu_ctx, c1_config):
    import torch
    from paper_0901_3163_amd import deflan
    dims, U, kappa = c1_config["dims"], c1_config["links"], c1_config["kappa"]
    op_h = deflan.Operator(gpu_ctx, dims, U, kappa, deflan.DL_G5M)
    op_d = deflan.Operator(gpu_ctx, dims, torch.from_numpy(U).cuda(), kappa, deflan.DL_G5M)
    b = gaussian_spinor(dims, 5)
    xh, eh, sh = op_h.solve_first(b, 30, 8, 1e-10)
    xd, ed, sd = op_d.solve_first(torch.from_numpy(b).cuda(), 30, 8, 1e-10)
    assert np.array_equal(xh, xd.cpu().numpy())  # deterministic reductions: bitwise equal
    B = np.stack([gaussian_spinor(dims, 6)])
    Xh, _, _ = op_h.solve_next(B, eh, 1e-10)
    Xd, _, _ = op_d.solve_next(torch.from_numpy(B).cuda(), ed, 1e-10)
    assert np.array_equal(Xh, Xd.cpu().numpy())


def test_ragged_lattice_solvers(gpu_ctx):
    """V = 120 sites (a ragged last tile): MinRes-DR and Lan-DR against the oracle's dense solve."""
    from paper_0901_3163_amd import deflan
    dims = (3, 4, 5, 2)
    U = su3_links(dims, 21)
    kappa = 0.13
    ora = dirac.WilsonOperator(U, dims, kappa)
    M = dirac.dense(ora.M, ora.n)
    b = gaussian_spinor(dims, 22)
    xd = np.linalg.solve(M, b.ravel())
    for kind, tol in ((deflan.DL_G5M, 1e-12), (deflan.DL_MDAGM, 1e-11)):
        op = deflan.Operator(gpu_ctx, dims, U, kappa, kind)
        x, eig, st = op.solve_first(b, 30, 8, tol)
        assert st["status"] == 0 and _rel(x, xd) < 1e-9
        X, sts, rc = op.solve_next(gaussian_spinor(dims, 23)[None], eig, tol)
        assert rc == 0 and _oracle_relres(ora, gaussian_spinor(dims, 23), X[0]) <= tol
        op.close()


def test_cg_on_indefinite_gamma5_m(gpu_ctx, c1_config, c1dense):
    """CG on gamma5 M (Hermitian indefinite: the combination Section 3 advises against, Fig. 7):
    plain CG and D-CG over the 20 lowest eigenvectors reach tol on the GPU and in the oracle
    (CG on the same matrix, right-hand side gamma5 b, the same eigenvectors and their FP64
    Galerkin matrix).  The recurrence is unstable on an indefinite spectrum, so rounding order
    moves the iterates: the iteration counts agree within 15%, and the eigenvectors still cut
    them, as the paper observes."""
    from paper_0901_3163_amd import deflan
    c1 = c1_config
    dims = c1["dims"]
    ora = c1dense["op"]
    op = deflan.Operator(gpu_ctx, dims, c1["links"], c1["kappa"], deflan.DL_G5M)
    b = gaussian_spinor(dims, 130)
    bb = b.ravel()
    g5b = ora.g5(bb)
    X0, s0, rc0 = op.solve_next(b[None], None, 1e-10, method=deflan.DL_METHOD_CG)
    assert rc0 == deflan.DL_OK and s0[0]["relres"] <= 1e-10
    assert _oracle_relres(ora, b, X0[0]) <= 1.0001e-10
    _, io = krylov.cg(ora.g5M, g5b, tol=1e-10, maxiter=20000)
    assert io["relres"] <= 1.0001e-10
    assert abs(s0[0]["iters"] - io["iters"]) <= 0.15 * io["iters"], (s0[0]["iters"], io["iters"])
    # deflated: the 20 eigenvectors of smallest |lambda| of the dense gamma5 M (oracle side),
    # handed to the library as a handle
    g5 = np.tile([1.0] * 6 + [-1.0] * 6, ora.V)
    lam, Z = np.linalg.eigh(g5[:, None] * c1dense["M"])
    Y = Z[:, np.argsort(np.abs(lam))[:20]]
    eig = op.eig_create(np.ascontiguousarray(Y.T).reshape(20, *b.shape))
    X1, s1, rc1 = op.solve_next(b[None], eig, 1e-10, method=deflan.DL_METHOD_CG)
    assert rc1 == deflan.DL_OK and s1[0]["relres"] <= 1e-10
    assert _oracle_relres(ora, b, X1[0]) <= 1.0001e-10
    assert _rel(X1[0], np.linalg.solve(c1dense["M"], bb)) < 1e-7
    H = deflated.projection_matrix(ora.g5M, Y)
    _, io1 = deflated.d_cg(ora.g5M, g5b, Y, H, 1e-10)
    assert io1["relres"] <= 1.0001e-10
    assert abs(s1[0]["iters"] - io1["iters"]) <= 0.15 * io1["iters"] + 5, (s1[0]["iters"], io1["iters"])
    assert s1[0]["iters"] < 0.8 * s0[0]["iters"]
    # D-MinRes on the same rhs and eigenvectors for comparison (Section 3: MinRes is the method for gamma5 M)
    X2, s2, _ = op.solve_next(b[None], eig, 1e-10)
    assert s2[0]["iters"] <= s1[0]["iters"]
    with pytest.raises(deflan.DeflanError):  # the CG option is for the FP64 one-rhs path
        op.solve_next(b[None], eig, 1e-10, storage=deflan.DL_FP32, batched=1, method=deflan.DL_METHOD_CG)
    with pytest.raises(deflan.DeflanError):
        op.solve_next(b[None], eig, 1e-10, method=5)
    eig.close()
    op.close()
