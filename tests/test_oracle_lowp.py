"""Pins of the rounding and lowered-projection oracle (CPU only).

Rounding is pinned to values fixed by round-to-nearest-even and to torch's own
bfloat16 conversion; the lowered projection to the paper's projection (the special
case of no rounding), to the closed form over exact eigenvectors and to the
Galerkin orthogonality it is built on.  The last test shows on a matrix with
near-critical small eigenvalues what the library's design rests on: a basis
rounded to BF16 no longer deflates, the FP32 rounding does, and contracting
against BF16 while correcting on the FP32 basis loses nothing.
"""
import numpy as np
import pytest

from oracle import deflated, lowp


def test_bf16_ties_and_halfway_cases():
    one = 1.0
    ulp = 2.0 ** -7  # bfloat16 spacing at 1
    cases = [
        (one, one),
        (one + ulp / 2, one),                      # tie, even neighbour is 1
        (one + 1.5 * ulp, one + 2 * ulp),          # tie, even neighbour is 1 + 2 ulp
        (one + ulp / 2 + 2.0 ** -20, one + ulp),   # just above the tie
        (one + ulp / 2 - 2.0 ** -20, one),         # just below the tie
        (-(one + 1.5 * ulp), -(one + 2 * ulp)),
        (3.0 * 2.0 ** -130, 3.0 * 2.0 ** -130),     # a binary32 subnormal with 2 significant bits
        (0.0, 0.0),
    ]
    x = np.array([c[0] for c in cases])
    got = lowp.round_bf16(x + 0j).real
    assert np.array_equal(got, np.array([c[1] for c in cases]))
    # BF16 goes through binary32: a value that binary32 rounds up onto a tie is then rounded to even
    v = 1.0 + ulp / 2 - 2.0 ** -30  # binary32 rounds this to 1 + ulp/2 exactly
    assert np.float32(v) == np.float32(one + ulp / 2)
    assert lowp.round_bf16(np.array([v + 0j])).real[0] == one


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    z = x.astype(np.float64) + 1j * x[::-1].astype(np.float64)
    got = lowp.round_bf16(z)
    assert np.array_equal(got.real, want) and np.array_equal(got.imag, want[::-1])


def test_fp32_rounding_is_binary32():
    rng = np.random.default_rng(4)
    z = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    r = lowp.round_f32(z)
    assert np.all(np.abs(r.real - z.real) <= np.abs(z.real) * 2.0 ** -24)
    assert np.array_equal(r.real.astype(np.float32).astype(np.float64), r.real)
    assert np.array_equal(lowp.round_f32(r), r)


def test_contraction_of_rounded_fields():
    rng = np.random.default_rng(5)
    V = rng.standard_normal((7, 50)) + 1j * rng.standard_normal((7, 50))
    W = rng.standard_normal((3, 50)) + 1j * rng.standard_normal((3, 50))
    C = lowp.contraction(V, W, "bf16")
    for r in range(3):
        for j in range(7):
            v, w = lowp.round_bf16(V[j]), lowp.round_bf16(W[r])
            assert abs(C[r, j] - sum(np.conj(v[i]) * w[i] for i in range(50))) < 1e-12
    assert np.allclose(lowp.contraction(V, W, "fp64"), W @ V.conj().T, rtol=0, atol=1e-12)


def _hermitian(n, evals, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return (Q * evals) @ Q.conj().T, Q


def test_projection_special_cases():
    n, k = 120, 6
    lam = np.concatenate([np.geomspace(1e-4, 1e-2, k), np.linspace(0.5, 4.0, n - k)])
    A, Q = _hermitian(n, lam, 6)
    Y = Q[:, :k]
    r = np.random.default_rng(7).standard_normal(n) + 0j
    # exact eigenvectors: d = Lambda^-1 Y^H r
    H = lowp.gram(lambda v: A @ v, Y)
    corr = lowp.lowered_projection(Y, Y, H, r, "fp64")
    assert np.allclose(corr, Y @ ((Y.conj().T @ r) / lam[:k]), rtol=1e-10, atol=1e-12)
    # no rounding: the paper's projection (the D-CG oracle's)
    Yg = lowp.round_f32(Y)
    Hg = lowp.gram(lambda v: A @ v, Yg)
    assert np.allclose(lowp.lowered_projection(Yg, Yg, Hg, r, "fp64"), deflated.galerkin_projection(Yg, Hg, r),
                       rtol=1e-12, atol=1e-12)
    # Galerkin orthogonality on any basis: Yg^H (r - A corr) = 0
    c2 = lowp.lowered_projection(Yg, Yg, Hg, r, "fp64")
    assert np.max(np.abs(Yg.conj().T @ (r - A @ c2))) < 1e-10 * np.linalg.norm(r)


def _defl_iters(A, b, Yc, Yg, prec, tol=1e-8, drop=1e-2):
    """CG restarted every `drop` residual reduction from the true residual, with the lowered
    projection at every restart; returns the CG iterations to ||b - A x|| <= tol ||b||."""
    Hg = lowp.gram(lambda v: A @ v, Yg)
    x = np.zeros_like(b)
    total = 0
    bn = np.linalg.norm(b)
    while True:
        x = x + lowp.lowered_projection(Yc, Yg, Hg, b - A @ x, prec)
        r = b - A @ x
        if np.linalg.norm(r) <= tol * bn:
            return total
        p, rr, r0 = r.copy(), np.vdot(r, r).real, np.linalg.norm(r)
        while True:
            q = A @ p
            a = rr / np.vdot(p, q).real
            x, r = x + a * p, r - a * q
            rn = np.vdot(r, r).real
            total += 1
            if np.sqrt(rn) <= drop * r0 or np.linalg.norm(b - A @ x) <= tol * bn or total > 5000:
                break
            p, rr = r + (rn / rr) * p, rn
        if total > 5000:
            return total


def test_bf16_basis_does_not_deflate_near_critical_modes():
    """Smallest eigenvalues 1e-6..1e-4 (below eps_bf16^2 ||A|| ~ 1e-5 ... 4e-5, above eps_f32^2 ||A||)."""
    n, k = 400, 8
    lam = np.concatenate([np.geomspace(1e-6, 1e-4, k), np.linspace(0.05, 4.0, n - k)])
    A, Q = _hermitian(n, lam, 8)
    Y = Q[:, :k]
    b = np.random.default_rng(9).standard_normal(n) + 1j * np.random.default_rng(10).standard_normal(n)
    it64 = _defl_iters(A, b, Y, Y, "fp64")
    it32 = _defl_iters(A, b, lowp.round_f32(Y), lowp.round_f32(Y), "fp32")
    split = _defl_iters(A, b, lowp.round_bf16(Y), lowp.round_f32(Y), "bf16")
    b16 = _defl_iters(A, b, lowp.round_bf16(Y), lowp.round_bf16(Y), "bf16")
    none = _defl_iters(A, b, Y[:, :0], Y[:, :0], "fp64")
    assert it32 <= it64 + 2 and split <= it64 + 2
    assert b16 > 1.5 * it64 and none > 1.5 * it64
