"""Pins of the network oracle (learned initial guess) against what the mathematics fixes (CPU only).

The transport is pinned to the Wilson hopping term (itself pinned to closed forms)
and to a coordinate-loop brute force; the hand-written backward pass to central
finite differences of the forward pass, layer by layer; the whole network to
gauge covariance and to phase and scale equivariance.
"""
import numpy as np
import pytest

from lattice_inputs import gaussian_spinor, point_source, su3_links, volume
from oracle import dirac, ptc

DIMS = (4, 2, 3, 4)


def _rand_act(V, C, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((V, C, 3)) + 1j * rng.standard_normal((V, C, 3))


def test_transport_reassembles_wilson_hopping():
    """sum_mu (1 - g_mu) T_{+mu} + (1 + g_mu) T_{-mu} on spin-as-channel equals the hopping term."""
    U = su3_links(DIMS, 1)
    psi = gaussian_spinor(DIMS, 2)
    out = np.zeros_like(psi)
    for h in range(1, 9):
        mu, s = ptc.HOPS[h]
        proj = np.eye(4) - s * dirac.GAMMA[mu]
        out += np.einsum("st,vtc->vsc", proj, ptc.transport(U, psi, DIMS, h))
    assert np.max(np.abs(out - dirac.hopping(U, psi, DIMS))) < 1e-13


def test_transport_coordinate_loops():
    lx, ly, lz, lt = DIMS
    U = su3_links(DIMS, 4)
    a = _rand_act(volume(DIMS), 2, 5)

    def site(x, y, z, t):
        return (x % lx) + lx * ((y % ly) + ly * ((z % lz) + lz * (t % lt)))

    for h in range(1, 9):
        mu, s = ptc.HOPS[h]
        got = ptc.transport(U, a, DIMS, h)
        step = [0, 0, 0, 0]
        step[mu] = 1
        for t in range(lt):
            for z in range(lz):
                for y in range(ly):
                    for x in range(lx):
                        c = (x, y, z, t)
                        here = site(*c)
                        if s > 0:
                            nb = site(*[c[d] + step[d] for d in range(4)])
                            want = U[here, mu] @ a[nb].T
                        else:
                            nb = site(*[c[d] - step[d] for d in range(4)])
                            want = U[nb, mu].conj().T @ a[nb].T
                        assert np.max(np.abs(got[here] - want.T)) < 1e-14


def test_transport_adjoint_is_reverse_hop():
    U = su3_links(DIMS, 6)
    a, b = _rand_act(volume(DIMS), 3, 7), _rand_act(volume(DIMS), 3, 8)
    for h in range(9):
        lhs = np.vdot(a, ptc.transport(U, b, DIMS, h))
        rhs = np.vdot(ptc.transport(U, a, DIMS, ptc.reverse_hop(h)), b)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _gauge_transform(U, dims, seed):
    """U_mu(x) -> g(x) U_mu(x) g(x + mu)^dag with random SU(3) g."""
    g = su3_links(dims, seed)[:, 0]
    V = volume(dims)
    lx, ly, lz, lt = dims
    sh = (lt, lz, ly, lx)
    gg = g.reshape(sh + (3, 3))
    Ug = np.empty_like(U)
    for mu in range(4):
        gnb = np.roll(gg, -1, axis=3 - mu).reshape(V, 3, 3)
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.transpose(gnb, (0, 2, 1)))
    return g, Ug


def test_gauge_covariance():
    U = su3_links(DIMS, 9)
    w = ptc.init_weights(11, scale=1.0)
    b = gaussian_spinor(DIMS, 12)
    g, Ug = _gauge_transform(U, DIMS, 13)
    gb = np.einsum("vab,vsb->vsa", g, b)
    lhs = ptc.forward(Ug, w, gb, DIMS)
    rhs = np.einsum("vab,vsb->vsa", g, ptc.forward(U, w, b, DIMS))
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(rhs))
    # a gauge-variant map (transport with the untransformed links) fails the same test
    bad = ptc.forward(U, w, gb, DIMS)
    assert np.max(np.abs(bad - rhs)) > 1e-3 * np.max(np.abs(rhs))


def test_phase_and_scale_equivariance():
    U = su3_links(DIMS, 14)
    w = ptc.init_weights(15, scale=1.0)
    b = gaussian_spinor(DIMS, 16)
    y = ptc.forward(U, w, b, DIMS)
    ph = np.exp(0.7j)
    assert np.max(np.abs(ptc.forward(U, w, ph * b, DIMS) - ph * y)) < 1e-13 * np.max(np.abs(y))
    assert np.max(np.abs(ptc.forward(U, w, 3.5 * b, DIMS) - 3.5 * y)) < 1e-13 * 3.5 * np.max(np.abs(y))
    # the non-linearity is not complex-linear: doubling the hidden pre-activations does not double the output
    assert np.max(np.abs(ptc.nonlin(2 * y) - 2 * ptc.nonlin(y))) > 1e-2


def test_zero_last_layer_gives_zero_guess():
    U = su3_links(DIMS, 17)
    w = ptc.init_weights(18)
    n12 = 9 * 16 * 4 + 9 * 16 * 16
    w[n12:] = 0
    b = gaussian_spinor(DIMS, 19)
    assert np.max(np.abs(ptc.forward(U, w, b, DIMS))) == 0.0
    # then the loss is ||M x||^2 / ||b||^2 = 1 for x = M^-1 b, computed here by a dense solve
    op = dirac.WilsonOperator(U, DIMS, 0.12)
    Md = dirac.dense(op.M, op.n)
    x = np.linalg.solve(Md, b.ravel()).reshape(b.shape)
    M = lambda v: op.M(v.ravel()).reshape(v.shape)
    Mdag = lambda v: op.Mdag(v.ravel()).reshape(v.shape)
    L, _ = ptc.loss_and_grad(U, w, b, x, DIMS, M, Mdag)
    assert abs(L - 1.0) < 1e-12


@pytest.mark.parametrize("layer", [0, 1, 2, None])
def test_gradient_matches_central_differences(layer):
    """Directional derivative of the loss along random complex directions in one layer (or all)."""
    U = su3_links(DIMS, 20)
    w = ptc.init_weights(21, scale=1.0)
    b = gaussian_spinor(DIMS, 22)
    x = gaussian_spinor(DIMS, 23) * 0.3
    op = dirac.WilsonOperator(U, DIMS, 0.12)
    M = lambda v: op.M(v.ravel()).reshape(v.shape)
    Mdag = lambda v: op.Mdag(v.ravel()).reshape(v.shape)
    L, G = ptc.loss_and_grad(U, w, b, x, DIMS, M, Mdag)
    rng = np.random.default_rng(24 + (layer or 0))
    d = rng.standard_normal(w.shape) + 1j * rng.standard_normal(w.shape)
    if layer is not None:
        sizes = [9 * ptc.WIDTHS[l + 1] * ptc.WIDTHS[l] for l in range(3)]
        lo = sum(sizes[:layer])
        mask = np.zeros(w.shape, bool)
        mask[lo:lo + sizes[layer]] = True
        d[~mask] = 0
    eps = 1e-6

    def loss(wv):
        r = M(ptc.forward(U, wv, b, DIMS) - x)
        return np.real(np.vdot(r, r)) / np.real(np.vdot(b, b))

    fd = (loss(w + eps * d) - loss(w - eps * d)) / (2 * eps)
    an = np.sum(np.real(G) * np.real(d) + np.imag(G) * np.imag(d))
    assert abs(fd - an) <= 1e-7 * max(abs(fd), 1e-3 * L)


def test_input_scale_is_the_rms_over_the_support():
    V = volume(DIMS)
    b = gaussian_spinor(DIMS, 30)
    assert abs(ptc.input_scale(b) - np.sqrt(np.sum(np.abs(b) ** 2) / V)) < 1e-14 * ptc.input_scale(b)
    p = 2.5 * point_source(DIMS, 7, 1, 2)
    assert ptc.input_scale(p) == 2.5
    q = np.zeros_like(b)
    q[3] = b[3]
    q[10] = b[10]
    assert abs(ptc.input_scale(q) ** 2 - (np.sum(np.abs(b[3]) ** 2) + np.sum(np.abs(b[10]) ** 2)) / 2) < 1e-13
    assert ptc.input_scale(np.zeros_like(b)) == 0.0
    # a point source reaches the network as a unit delta: its guess is O(1) at the source
    U = su3_links(DIMS, 31)
    y = ptc.forward(U, ptc.init_weights(32, scale=1.0), point_source(DIMS, 0, 0, 0), DIMS)
    assert 1e-2 < np.linalg.norm(y[0]) < 1e2


def test_forward_with_rounded_middle_layer():
    """With the identity as rounding it is the pinned forward pass; with BF16 rounding of the
    16 -> 16 layer's operands it stays within the rounding's reach of it."""
    from oracle import lowp
    U = su3_links(DIMS, 40)
    w = ptc.init_weights(41, scale=1.0)
    b = gaussian_spinor(DIMS, 42)
    y = ptc.forward(U, w, b, DIMS)
    assert np.array_equal(ptc.forward_lowp(U, w, b, DIMS, lambda z: z), y)
    yb = ptc.forward_lowp(U, w, b, DIMS, lowp.round_bf16)
    rel = np.linalg.norm(yb - y) / np.linalg.norm(y)
    assert 1e-5 < rel < 2e-2


def _proj_setup(k):
    U = su3_links(DIMS, 20)
    w = ptc.init_weights(21, scale=1.0)
    b = gaussian_spinor(DIMS, 22)
    x = gaussian_spinor(DIMS, 23) * 0.3
    op = dirac.WilsonOperator(U, DIMS, 0.12)
    M = lambda v: op.M(v.ravel()).reshape(v.shape)
    Mdag = lambda v: op.Mdag(v.ravel()).reshape(v.shape)
    Md = dirac.dense(op.M, op.n)
    lam, Z = np.linalg.eigh(Md.conj().T @ Md)
    Y = Z[:, :k]
    H = Y.conj().T @ (Md.conj().T @ (Md @ Y))
    return U, w, b, x, M, Mdag, Md, lam, Y, H


def test_projected_loss_closed_form_over_exact_eigenvectors():
    """Over exact eigenvectors y_i of M^dag M (eigenvalues sigma_i^2) the projection removes
    sigma_i^2 |y_i^H d|^2 from ||M d||^2 (the A-orthogonal projection's Pythagoras), and over the
    whole eigenbasis nothing is left."""
    U, w, b, x, M, Mdag, Md, lam, Y, H = _proj_setup(40)
    d = (ptc.forward(U, w, b, DIMS) - x).ravel()
    bn2 = np.real(np.vdot(b, b))
    want = (np.linalg.norm(Md @ d) ** 2 - np.sum(lam[:40] * np.abs(Y.conj().T @ d) ** 2)) / bn2
    L, _ = ptc.loss_and_grad(U, w, b, x, DIMS, M, Mdag, Y=Y, H=H)
    assert abs(L - want) <= 1e-12 * abs(want)
    L0, _ = ptc.loss_and_grad(U, w, b, x, DIMS, M, Mdag)
    assert L < L0
    full = np.linalg.eigh(Md.conj().T @ Md)[1]
    Hf = full.conj().T @ (Md.conj().T @ (Md @ full))
    Lf, Gf = ptc.loss_and_grad(U, w, b, x, DIMS, M, Mdag, Y=full, H=Hf)
    assert Lf < 1e-20 and np.max(np.abs(Gf)) < 1e-8


@pytest.mark.parametrize("layer", [0, 2, None])
def test_projected_gradient_matches_central_differences(layer):
    """The backward pass of the projected loss (seeded with M^dag M d') against central
    differences of the projected loss over a basis that is not an eigenbasis (random orthonormal)."""
    U, w, b, x, M, Mdag, Md, lam, _, _ = _proj_setup(1)
    rng = np.random.default_rng(25)
    Y, _ = np.linalg.qr(rng.standard_normal((Md.shape[0], 30)) + 1j * rng.standard_normal((Md.shape[0], 30)))
    A = Md.conj().T @ Md
    H = Y.conj().T @ A @ Y
    L, G = ptc.loss_and_grad(U, w, b, x, DIMS, M, Mdag, Y=Y, H=H)
    d = rng.standard_normal(w.shape) + 1j * rng.standard_normal(w.shape)
    if layer is not None:
        sizes = [9 * ptc.WIDTHS[l + 1] * ptc.WIDTHS[l] for l in range(3)]
        lo = sum(sizes[:layer])
        mask = np.zeros(w.shape, bool)
        mask[lo:lo + sizes[layer]] = True
        d[~mask] = 0
    eps = 1e-6
    P = np.eye(A.shape[0]) - Y @ np.linalg.solve(H, Y.conj().T @ A)  # dense projector, built apart

    def loss(wv):
        e = P @ (ptc.forward(U, wv, b, DIMS) - x).ravel()
        return np.linalg.norm(Md @ e) ** 2 / np.real(np.vdot(b, b))

    assert abs(loss(w) - L) <= 1e-12 * L
    fd = (loss(w + eps * d) - loss(w - eps * d)) / (2 * eps)
    an = np.sum(np.real(G) * np.real(d) + np.imag(G) * np.imag(d))
    assert abs(fd - an) <= 1e-7 * max(abs(fd), 1e-3 * L)
