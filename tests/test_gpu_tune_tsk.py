"""The contraction autotuner (GPU): every kind tunes to a shape of its candidate set, and every
launch shape -- forced through DEFLAN_TSK_SHAPE -- gives the contraction's result: the
update and the basis rebuild bit for bit equal across shapes, the dots within the rounding of
their partial sums (FP64) or of FP32 accumulation (matrix cores), against plain numpy."""
import numpy as np
import pytest

from oracle import lowp

pytestmark = pytest.mark.gpu

# (kind, n, nv, nw): a ragged length of several tiles, the basis sizes the solvers use
KEYS = [(0, 12 * 4096 + 37, 40, 12), (1, 12 * 4096 + 36, 60, 16), (2, 12 * 4096 + 36, 100, 5),
        (3, 12 * 4096 + 37, 60, 16), (4, 12 * 4096 + 37, 60, 7), (5, 12 * 4096 + 37, 121, 60)]


@pytest.mark.parametrize("kind,n,nv,nw", KEYS)
def test_tuner_picks_a_candidate(gpu_ctx, kind, n, nv, nw):
    from paper_0901_3163_amd import deflan
    g, t, us = gpu_ctx.tune_tsk(kind, n, nv, nw, reps=3)
    assert us > 0 and g >= 1
    if kind in (deflan.DL_TSK_DOTS32, deflan.DL_TSK_DOTS16):
        assert t in (2, 4, 8)
    elif kind == deflan.DL_TSK_COMBINE:
        assert t in (0, 1, 2, 3)
    else:
        assert t == 0


def test_tuner_rejects_bad_keys(gpu_ctx):
    from paper_0901_3163_amd import deflan
    for args in [(6, 100, 4, 4), (deflan.DL_TSK_DOTS64, 100, 65, 4), (deflan.DL_TSK_DOTS16, 100, 129, 4),
                 (deflan.DL_TSK_UPD64, 100, 4, 17), (deflan.DL_TSK_COMBINE, 0, 4, 4)]:
        with pytest.raises(deflan.DeflanError):
            gpu_ctx.tune_tsk(*args)


def _fields(n, nv, nw, seed):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((nv, n)) + 1j * rng.standard_normal((nv, n))
    W = rng.standard_normal((nw, n)) + 1j * rng.standard_normal((nw, n))
    X = rng.standard_normal((nw, n)) + 1j * rng.standard_normal((nw, n))
    return V, W, X


# grid, tile: one block, a few blocks, more than the default (clamped), odd counts
SHAPES = ["1,4", "7,2", "64,8", "1000,4", "100000,2"]


@pytest.mark.parametrize("shape", SHAPES)
def test_fp64_dots_in_every_shape(gpu_ctx, monkeypatch, shape):
    """Two launches (64 and 6 basis vectors), a ragged length: C = V^H W within the rounding of
    FP64 partial sums, and the update X + V C^T (with those coefficients) within FP64 rounding."""
    from paper_0901_3163_amd import deflan
    n, nv, nw = 12 * 4096 + 37, 70, 13
    V, W, X = _fields(n, nv, nw, 3)
    monkeypatch.setenv("DEFLAN_TSK_SHAPE", shape + ",0")
    C, Xs = deflan.dl_tsk_project_multi(gpu_ctx, V, W, X)
    Cr = W @ V.conj().T  # C[r][j] = <V_j, W_r>
    bound = 1e-14 * np.sqrt(n) * np.outer(np.linalg.norm(W, axis=1), np.linalg.norm(V, axis=1))
    assert np.all(np.abs(C - Cr) <= bound)
    Xr = X + C @ V
    assert np.max(np.abs(Xs - Xr)) <= 1e-12 * np.max(np.abs(Xr))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_update_gives_the_same_bits_in_every_grid(gpu_ctx, monkeypatch, prec):
    """X += V D over an FP64 or FP32 basis: the dots keep their (remembered) shape, the update's
    grid goes from one block to 8192 blocks, and every result has the same bits."""
    from paper_0901_3163_amd import deflan
    n, nv, nw = 12 * 4096 + 36, 140, 9  # two update launches (128 + 12 basis vectors)
    V, W, X = _fields(n, nv, nw, 4)
    kind = 3 if prec == "fp64" else 4
    ref = None
    for g in (1, 13, 512, 2048, 8192):
        monkeypatch.setenv("DEFLAN_TSK_SHAPE", f"{g},0,{kind}")
        if prec == "fp64":
            C, Xs = deflan.dl_tsk_project_multi(gpu_ctx, V, W, X)
        else:
            C, Xs = deflan.dl_tsk_project_lowp(gpu_ctx, 1, V, W, X)
        if ref is None:
            ref = (C, Xs)
        assert np.array_equal(C, ref[0]) and np.array_equal(Xs, ref[1]), g


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_matrix_core_dots_in_every_shape(gpu_ctx, monkeypatch, prec, shape):
    """More than 64 and more than 128 basis vectors (one to three launches per call), a ragged
    length; the FP32-accumulation bound of the default shape holds in every shape."""
    from paper_0901_3163_amd import deflan
    n, nv, nw = 12 * 4096 + 36, 130, 11
    V, W, X = _fields(n, nv, nw, 5)
    monkeypatch.setenv("DEFLAN_TSK_SHAPE", shape)
    C, Xo = deflan.dl_tsk_project_lowp(gpu_ctx, 1 if prec == "fp32" else 2, V, W, X)
    q = lowp.rounding(prec)
    Cr = lowp.contraction(V, W, prec)
    bound = 4e-6 * np.outer(np.linalg.norm(q(W), axis=1), np.linalg.norm(q(V), axis=1))
    assert np.all(np.abs(C - Cr) <= bound), float(np.max(np.abs(C - Cr) / bound))
    V32 = lowp.round_f32(V)
    Xr = X + Cr @ V32
    assert np.all(np.abs(Xo - Xr) <= bound @ np.abs(V32) + 1e-13 * np.abs(Xr))


def test_matrix_core_row_tiles_give_the_same_bits(gpu_ctx, monkeypatch):
    """At one grid size the row tiling does not change any block's accumulation order."""
    from paper_0901_3163_amd import deflan
    n, nv, nw = 12 * 4096 + 36, 100, 16
    V, W, _ = _fields(n, nv, nw, 9)
    out = []
    for t in (2, 4, 8):
        monkeypatch.setenv("DEFLAN_TSK_SHAPE", f"96,{t}")
        out.append(deflan.dl_tsk_project_lowp(gpu_ctx, 2, V, W)[0])
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[1], out[2])


@pytest.mark.parametrize("nv,ny", [(121, 60), (300, 20), (9, 1)])
def test_rebuild_gives_the_same_bits_in_every_shape(gpu_ctx, monkeypatch, nv, ny):
    """Y = V G with 8 or 16 outputs per block, 2-D or XCD-grouped block numbering, grids of 8 to
    8192 blocks (16 outputs per block needs nv <= 256: clamped to the default otherwise)."""
    from paper_0901_3163_amd import deflan
    n = 12 * 4096 + 37
    V, _, _ = _fields(n, nv, 1, nv + ny)
    G = np.random.default_rng(ny).standard_normal((nv, ny))
    Yr = G.T @ V
    ref = None
    for shape in ["2048,0", "8,1", "1000,1", "1000,2", "8192,3", "3,3"]:
        monkeypatch.setenv("DEFLAN_TSK_SHAPE", shape)
        Y = deflan.dl_tsk_combine(gpu_ctx, V, G)
        Y = Y.cpu().numpy() if hasattr(Y, "cpu") else Y
        assert np.allclose(Y, Yr, rtol=0, atol=1e-12 * np.max(np.abs(Yr)))
        if ref is None:
            ref = Y
        assert np.array_equal(Y, ref), shape


def test_solver_results_with_tuning_off_and_on(gpu_ctx, c1_config, monkeypatch):
    """A batched D-CG with FP32 eigenvectors, with every contraction in its default shape and in
    forced non-default shapes, reaches tol and the same solution within the tolerance's reach."""
    from lattice_inputs import gaussian_spinor
    from paper_0901_3163_amd import deflan
    from oracle import dirac
    dims, U, kappa = c1_config["dims"], c1_config["links"], c1_config["kappa"]
    op = deflan.Operator(gpu_ctx, dims, U, kappa, deflan.DL_MDAGM)
    _, eig, _ = op.solve_first(gaussian_spinor(dims, 100), 60, 20, 1e-10)
    eig.lower(deflan.DL_FP32)
    B = np.stack([gaussian_spinor(dims, 500 + i) for i in range(6)])
    ora = dirac.WilsonOperator(U, dims, kappa)
    xs = []
    for shape in [None, "1,2", "5,8"]:
        if shape is None:
            monkeypatch.delenv("DEFLAN_TSK_SHAPE", raising=False)
            monkeypatch.setenv("DEFLAN_AUTOTUNE", "0")
        else:
            monkeypatch.setenv("DEFLAN_TSK_SHAPE", shape)
        X, sts, rc = op.solve_next(B, eig, 1e-10, storage=deflan.DL_BF16, batched=1, eig_storage=deflan.DL_FP32)
        assert rc == deflan.DL_OK
        for i in range(len(B)):
            r = np.linalg.norm(B[i].ravel() - ora.M(X[i].ravel())) / np.linalg.norm(B[i])
            assert r <= 1.0001e-10, (shape, i, r)
        xs.append(X)
    for X in xs[1:]:
        assert np.linalg.norm(X - xs[0]) / np.linalg.norm(xs[0]) < 1e-6
    eig.close()
    op.close()
