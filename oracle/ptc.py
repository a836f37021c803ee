"""Gauge-covariant parallel-transport convolution network for the learned initial guess (FP64 numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not in the paper: the learned guess is an addition to D-CG / D-MinRes whose
output is refined by the paper's Galerkin projection and Krylov solve.  The
network follows the published gauge-equivariant convolution idea (Lehner and
Wettig, 2023); the reading used here:

* activations are colour triplets per site and channel, shape [V, C, 3]; the
  input spinor b[V, 4 spin, 3 colour] is a 4-channel activation;
* a layer maps psi_out[o](x) = sum_h sum_i W_h[o, i] (T_h psi_in[i])(x) over the nine
  hops h in {0, +x, -x, +y, -y, +z, -z, +t, -t} with T_0 = 1,
  (T_{+mu} psi)(x) = U_mu(x) psi(x + mu), (T_{-mu} psi)(x) = U_mu(x - mu)^dag psi(x - mu);
* channel widths 4 -> 16 -> 16 -> 4, nonlinearity f(z) = z / sqrt(1 + |z|^2) per
  site and channel (|z| the gauge-invariant colour norm) after layers 1 and 2;
* net(b) = s * N(b / s) with s the root-mean-square site norm of b over the sites
  where b is nonzero (s = ||b|| / sqrt(V) for a source without zeros, |b(x0)| for a
  point source), so the guess scales with b and every source reaches the network at
  unit scale.

Loss on a pair (b, x) with M x = b: L = ||M (net(b) - x)||^2 / ||b||^2, the error in
the M^dag M norm.  Gradients use the real-gradient convention G = dL/dRe + i dL/dIm.
The backward pass is written out by hand (adjoint of T_h is T_{-h}).
"""
from __future__ import annotations

import numpy as np

from lattice_inputs import net_weights

WIDTHS = (4, 16, 16, 4)
HOPS = [(None, 0), (0, 1), (0, -1), (1, 1), (1, -1), (2, 1), (2, -1), (3, 1), (3, -1)]


def reverse_hop(h: int) -> int:
    """Index of the hop whose transport is the adjoint of hop h."""
    mu, s = HOPS[h]
    return 0 if mu is None else HOPS.index((mu, -s))


def n_weights(widths=WIDTHS) -> int:
    return sum(9 * widths[l + 1] * widths[l] for l in range(len(widths) - 1))


def split_weights(w, widths=WIDTHS):
    """Flat complex vector -> per-layer arrays [9, C_out, C_in]."""
    out, off = [], 0
    for l in range(len(widths) - 1):
        n = 9 * widths[l + 1] * widths[l]
        out.append(np.asarray(w[off:off + n]).reshape(9, widths[l + 1], widths[l]))
        off += n
    return out


def init_weights(seed: int, widths=WIDTHS, scale=0.3) -> np.ndarray:
    """Seeded complex Gaussian weights (the shared input generator)."""
    return net_weights(seed, widths, scale)


def _shape(dims):
    lx, ly, lz, lt = dims
    return (lt, lz, ly, lx)


def transport(U, psi, dims, h):
    """(T_h psi)(x) for psi [V, C, 3]."""
    mu, s = HOPS[h]
    if mu is None:
        return psi.copy()
    sh = _shape(dims)
    ax = 3 - mu
    p = psi.reshape(sh + psi.shape[1:])
    u = U.reshape(sh + (4, 3, 3))[..., mu, :, :]
    if s > 0:
        q = np.roll(p, -1, axis=ax)
        out = np.einsum("TZYXab,TZYXcb->TZYXca", u, q)
    else:
        q = np.roll(p, 1, axis=ax)
        ub = np.roll(u, 1, axis=ax)
        out = np.einsum("TZYXba,TZYXcb->TZYXca", ub.conj(), q)
    return out.reshape(psi.shape)


def layer(U, W, psi, dims):
    """psi_out[x, o] = sum_h sum_i W[h, o, i] T_h psi[x, i]."""
    out = np.zeros((psi.shape[0], W.shape[1], 3), dtype=np.complex128)
    for h in range(9):
        out += np.einsum("oi,xic->xoc", W[h], transport(U, psi, dims, h))
    return out


def nonlin(z):
    n2 = np.sum(np.abs(z) ** 2, axis=-1, keepdims=True)
    return z / np.sqrt(1.0 + n2)


def nonlin_backward(z, g):
    """G_z = gfac G_f + 2 gfac' Re<G_f, z> z with gfac(s) = (1+s)^-1/2."""
    n2 = np.sum(np.abs(z) ** 2, axis=-1, keepdims=True)
    gf = 1.0 / np.sqrt(1.0 + n2)
    dgf = -0.5 * (1.0 + n2) ** -1.5
    re = np.real(np.sum(np.conj(g) * z, axis=-1, keepdims=True))
    return gf * g + 2.0 * dgf * re * z


def input_scale(b):
    """Root-mean-square site norm of b over its nonzero sites (0 for b = 0)."""
    site_n2 = np.sum(np.abs(b) ** 2, axis=(1, 2))
    nz = np.count_nonzero(site_n2)
    return 0.0 if nz == 0 else float(np.sqrt(np.sum(site_n2) / nz))


def forward(U, w, b, dims, keep=False):
    """net(b) for b [V, 4, 3]; with keep=True also the intermediate activations."""
    Ws = split_weights(w)
    s = input_scale(b)
    a0 = b / s
    z1 = layer(U, Ws[0], a0, dims)
    a1 = nonlin(z1)
    z2 = layer(U, Ws[1], a1, dims)
    a2 = nonlin(z2)
    a3 = layer(U, Ws[2], a2, dims)
    y = s * a3
    if keep:
        return y, dict(s=s, a0=a0, z1=z1, a1=a1, z2=z2, a2=a2)
    return y


def layer_rounded(U, W, psi, dims, rnd):
    """layer() with its operands rounded by rnd: the weights and every transported input."""
    out = np.zeros((psi.shape[0], W.shape[1], 3), dtype=np.complex128)
    for h in range(9):
        out += np.einsum("oi,xic->xoc", rnd(W[h]), rnd(transport(U, psi, dims, h)))
    return out


def forward_lowp(U, w, b, dims, rnd):
    """net(b) with the 16 -> 16 layer computed by layer_rounded (the other layers exact)."""
    Ws = split_weights(w)
    s = input_scale(b)
    a1 = nonlin(layer(U, Ws[0], b / s, dims))
    a2 = nonlin(layer_rounded(U, Ws[1], a1, dims, rnd))
    return s * layer(U, Ws[2], a2, dims)


def weight_grad(U, g_out, psi_in, dims):
    """G_W[h, o, i] = sum_x sum_c G_out[x, o, c] conj(T_h psi_in)[x, i, c]."""
    return np.stack([np.einsum("xoc,xic->oi", g_out, np.conj(transport(U, psi_in, dims, h))) for h in range(9)])


def layer_backward_data(U, W, g_out, dims):
    """G_in = sum_h T_{-h} (W_h^H G_out)."""
    g = np.zeros((g_out.shape[0], W.shape[2], 3), dtype=np.complex128)
    for h in range(9):
        g += transport(U, np.einsum("oi,xoc->xic", np.conj(W[h]), g_out), dims, reverse_hop(h))
    return g


def loss_and_grad(U, w, b, x, dims, M, Mdag, Y=None, H=None):
    """L = ||M (net(b) - x)||^2 / ||b||^2 and its real gradient w.r.t. the weights.

    M, Mdag: callables on [V, 4, 3] spinors.  With a basis Y ([12 V, k], orthonormal columns)
    and H = Y^H M^dag M Y, the error d = net(b) - x is first replaced by what the D-CG start
    (guess, then the Galerkin projection over Y, Section 2) leaves of it,
    d' = d - Y H^-1 Y^H M^dag M d.  That map is the M^dag M-orthogonal projector Q onto the
    complement of span Y, so Q^H A Q = A Q (A = M^dag M) and the gradient of ||M Q d||^2 with
    respect to d is A Q d = M^dag (M d'): the backward pass below is the same in both cases.
    """
    Ws = split_weights(w)
    y, c = forward(U, w, b, dims, keep=True)
    bn2 = np.real(np.vdot(b, b))
    d = y - x
    if Y is not None and Y.shape[1] > 0:
        g = Y.conj().T @ Mdag(M(d)).ravel()
        d = d - (Y @ np.linalg.solve(H, g)).reshape(d.shape)
    r = M(d)
    L = float(np.real(np.vdot(r, r)) / bn2)
    g_y = 2.0 * Mdag(r) / bn2
    g3 = c["s"] * g_y
    gW3 = weight_grad(U, g3, c["a2"], dims)
    g_a2 = layer_backward_data(U, Ws[2], g3, dims)
    g_z2 = nonlin_backward(c["z2"], g_a2)
    gW2 = weight_grad(U, g_z2, c["a1"], dims)
    g_a1 = layer_backward_data(U, Ws[1], g_z2, dims)
    g_z1 = nonlin_backward(c["z1"], g_a1)
    gW1 = weight_grad(U, g_z1, c["a0"], dims)
    return L, np.concatenate([gW1.ravel(), gW2.ravel(), gW3.ravel()])
