"""The remaining configurations at full size, each checked on outputs the oracle computes one by
one (the C Wilson matrix of the oracle on the GPU's results):

* the plain-method configuration (16^3x32, min|lambda| ~ 1e-4): the first rhs solved tightly,
  its error bounded through the condition number, and every one of the 60 eigenpairs;
* the learned-guess configuration (16^3x32, kappa tuned on field 10): a network trained on two
  fields and applied on a field it never saw, with the D-CG start it gives;
* the precision configuration (24^3x48): D-CG over the Lan-DR(200,100) eigenvectors themselves;
* the batching configuration: 8^4, 12^4, 16^3x32 and 20^3x40 with k = 40, 60, 80, 100 in one
  work-list batch of 64 rhs.
"""
import json
import os

import numpy as np
import pytest

from lattice_inputs import gaussian_spinor, net_weights, su3_links
from oracle import cwilson

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _kappa(name):
    with open(os.path.join(ROOT, "tests", "golden", "kappa.json")) as fh:
        return json.load(fh)[name]


def _relres(cw, b, x):
    b = np.asarray(b).ravel()
    return np.linalg.norm(b - cw.M(np.asarray(x).ravel())) / np.linalg.norm(b)


def test_plain_configuration_solution_and_every_eigenpair(gpu_ctx):
    """MinRes-DR(120,60) on gamma5 M to 4e-13: the oracle's residual of x, the error bound
    ||x - x*|| / ||x*|| <= cond(M) relres with cond(M) <= (1 + 8 kappa) / min|lambda(gamma5 M)|,
    and all 60 Rayleigh quotients, residual norms and the orthonormality of the vectors."""
    import torch
    from paper_0901_3163_amd import deflan
    e = _kappa("16x16x16x32")
    dims, kappa = tuple(e["dims"]), e["kappa"]
    U = su3_links(dims, e["seed"], e["eps"])
    cw = cwilson.CWilson(U, dims, kappa)
    op = deflan.Operator(gpu_ctx, dims, torch.from_numpy(U).cuda(), kappa, deflan.DL_G5M)
    b1 = gaussian_spinor(dims, 200)
    tol = 4e-13
    x1, eig, st1 = op.solve_first(torch.from_numpy(b1).cuda(), 120, 60, tol)
    x1 = x1.cpu().numpy()
    r1 = _relres(cw, b1, x1)
    assert st1["status"] == 0 and r1 <= 1.001 * tol, (st1, r1)
    evals, resid = eig.info()
    lmin = float(np.min(np.abs(evals)))
    cond = (1 + 8 * kappa) / lmin
    assert cond * r1 <= 1e-8, (cond, r1)
    Y = eig.vectors().reshape(60, -1)
    G = Y.conj() @ Y.T
    assert np.max(np.abs(G - np.eye(60))) < 1e-10
    for i in range(60):
        ay = cw.g5M(Y[i])
        lam = float(np.real(np.vdot(Y[i], ay)))
        assert abs(lam - evals[i]) <= 1e-12 + 1e-10 * abs(evals[i]), i
        assert abs(np.linalg.norm(ay - evals[i] * Y[i]) - resid[i]) <= 1e-12 + 1e-8 * resid[i], i
    eig.close()
    op.close()


def test_learned_configuration_transfers_to_an_unseen_field(gpu_ctx):
    """Fields 10 and 11 train the network (64 D-CG pairs each, projected loss); on held-out field
    20 the learned start needs fewer D-CG iterations than the projection alone, and every
    solution (BF16 batched D-CG with the guess) has an oracle residual <= 1e-10."""
    import torch
    from lattice_inputs import gaussian_spinors_device
    from paper_0901_3163_amd import deflan
    e = _kappa("16x16x16x32/seed10")
    dims, kappa, tol = tuple(e["dims"]), e["kappa"], 1e-10
    net = deflan.Net(gpu_ctx, net_weights(7))
    fields = {}
    for seed in (10, 11, 20):
        U = su3_links(dims, seed, e["eps"])
        op = deflan.Operator(gpu_ctx, dims, torch.from_numpy(U).cuda(), kappa, deflan.DL_MDAGM)
        _, eig, st = op.solve_first(torch.from_numpy(gaussian_spinor(dims, 1000 + seed)).cuda(), 100, 50, tol,
                                    reorth=deflan.DL_REORTH_KEPT)
        assert st["status"] == 0
        eig.lower(deflan.DL_FP32)
        fields[seed] = (U, op, eig)
    kw = dict(storage=deflan.DL_BF16, batched=1, eig_storage=deflan.DL_FP32)
    for ep in range(2):
        for seed in (10, 11):
            _, op, eig = fields[seed][:3]
            if ep == 0:
                B = gaussian_spinors_device(dims, 20000 + 1000 * seed, 64)
                X, sts, rc = op.solve_next(B, eig, tol, **kw)
                assert rc == deflan.DL_OK
                fields[seed] = fields[seed] + (B, X)
            B, X = fields[seed][3], fields[seed][4]
            net.set_projection(eig)
            losses = net.train(op, B, X, batch=6, steps=100, lr=3e-3)
            assert np.all(np.isfinite(losses))
    net.set_projection(None)
    U, op, eig = fields[20][:3]
    B = gaussian_spinors_device(dims, 40000 + 1000 * 20, 16)
    # the same cycle drop for both starts (by default a learned start runs 1e-3 cycles, the
    # projection-only start 1e-5), so that the comparison isolates the network
    Xp, sp, rcp = op.solve_next(B, eig, tol, inner_drop=1e-3, **kw)
    Xn, sn, rcn = op.solve_next(B, eig, tol, net=net, net_prec=deflan.DL_BF16, inner_drop=1e-3, **kw)
    assert rcp == rcn == deflan.DL_OK
    cw = cwilson.CWilson(U, dims, kappa)
    Bh, Xh = B.cpu().numpy(), Xn.cpu().numpy()
    for i in range(16):
        assert _relres(cw, Bh[i], Xh[i]) <= 1.0001 * tol, i
    assert all(s["guess"] == 1 for s in sn)
    it_n, it_p = sum(s["iters"] for s in sn), sum(s["iters"] for s in sp)
    assert it_n < it_p, (it_n, it_p)
    for f in fields.values():
        f[2].close()
        f[1].close()
    net.close()


def test_precision_configuration_over_landr_eigenvectors(gpu_ctx):
    """24^3x48 near critical: Lan-DR(200,100) on M^dag M (the paper's re-orthogonalisation over the
    kept vectors), its 100 eigenvectors lowered to FP32, then D-CG for 12 Gaussian rhs with BF16
    storage: every solution's oracle residual <= 1e-10, and agreement with plain FP64 D-CG."""
    import torch
    from paper_0901_3163_amd import deflan
    e = _kappa("24x24x24x48")
    dims, kappa = tuple(e["dims"]), e["kappa"]
    U = su3_links(dims, e["seed"], e["eps"])
    cw = cwilson.CWilson(U, dims, kappa)
    op = deflan.Operator(gpu_ctx, dims, torch.from_numpy(U).cuda(), kappa, deflan.DL_MDAGM)
    _, eig, st = op.solve_first(torch.from_numpy(gaussian_spinor(dims, 299)).cuda(), 200, 100, 1e-10,
                                reorth=deflan.DL_REORTH_KEPT)
    assert st["status"] == 0
    evals, _ = eig.info()
    # the smallest eigenvalue of M^dag M is the square of the kappa search's min|lambda|
    assert abs(np.sqrt(np.min(evals)) - e["min_abs_eig"]) <= 0.01 * e["min_abs_eig"]
    eig.lower(deflan.DL_FP32)
    B = torch.from_numpy(np.stack([gaussian_spinor(dims, 300 + i) for i in range(12)])).cuda()
    X, sts, rc = op.solve_next(B, eig, 1e-10, storage=deflan.DL_BF16, batched=1, eig_storage=deflan.DL_FP32)
    assert rc == deflan.DL_OK
    X64, _, rc64 = op.solve_next(B[:2], eig, 1e-10)
    assert rc64 == deflan.DL_OK
    Bh, Xh, X64 = B.cpu().numpy(), X.cpu().numpy(), X64.cpu().numpy()
    for i in range(12):
        assert _relres(cw, Bh[i], Xh[i]) <= 1.0001e-10, i
    for i in range(2):
        assert np.linalg.norm(Xh[i] - X64[i]) / np.linalg.norm(X64[i]) < 1e-6
    eig.close()
    op.close()


def test_batching_configuration_four_lattices_in_one_worklist(gpu_ctx):
    """8^4, 12^4, 16^3x32, 20^3x40 (links seed 0, kappa 0.145) with k = 40, 60, 80, 100 Lan-DR
    eigenvectors, 16 Gaussian rhs each, solved together by the work-list batch in FP32 and BF16
    storage: every solution's oracle residual <= 1e-10."""
    import torch
    from paper_0901_3163_amd import deflan
    kappa = 0.145
    lats = [((8, 8, 8, 8), 40), ((12, 12, 12, 12), 60), ((16, 16, 16, 32), 80), ((20, 20, 20, 40), 100)]
    items, keep = [], []
    for j, (dims, k) in enumerate(lats):
        U = su3_links(dims, 0)
        op = deflan.Operator(gpu_ctx, dims, torch.from_numpy(U).cuda(), kappa, deflan.DL_MDAGM)
        _, eig, st = op.solve_first(torch.from_numpy(gaussian_spinor(dims, 390 + j)).cuda(), k + 40, k, 1e-10,
                                    reorth=deflan.DL_REORTH_KEPT)
        assert st["status"] == 0
        eig.lower(deflan.DL_FP32)
        B = torch.from_numpy(np.stack([gaussian_spinor(dims, 400 + 16 * j + i) for i in range(16)])).cuda()
        items.append((op, eig, B, 1e-10))
        keep.append((dims, U))
    for storage in (deflan.DL_FP32, deflan.DL_BF16):
        Xs, sts, rc = deflan.solve_next_multi(gpu_ctx, items, storage=storage, eig_storage=deflan.DL_FP32)
        assert rc == deflan.DL_OK
        for (dims, U), (op, eig, B, tol), X, st in zip(keep, items, Xs, sts):
            cw = cwilson.CWilson(U, dims, kappa)
            Bh, Xh = B.cpu().numpy(), X.cpu().numpy()
            for i in range(16):
                assert st[i]["relres"] <= tol and _relres(cw, Bh[i], Xh[i]) <= 1.0001 * tol, (dims, storage, i)
    for op, eig, _, _ in items:
        eig.close()
        op.close()
