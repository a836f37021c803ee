"""Wilson-Dirac operator of the paper's lattice tests (Section 2), FP64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper designates M as "the Wilson matrix" and solves through
M^dag M x = M^dag b (positive definite, Lan-DR / D-CG, Fig. 5) and through
gamma5 M x = gamma5 b (Hermitian indefinite, MinRes-DR / D-MinRes, Fig. 6).
It fixes no convention; the reading used here (hopping-parameter form, chiral
gamma basis, periodic boundaries) is

    (M psi)(x) = psi(x) - kappa * sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                          + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]

so that kappa_c is near 1/8 for weak fields (the paper's kappa_c = 0.1572 at
beta = 6 belongs to the same normalisation).  The implementation is a direct
transcription with full 4x4 gamma matrices and np.roll shifts -- no
spin-projection trick -- so that it stays independent of the GPU stencil.

Spinor arrays are complex128 [V][4][3]; links complex128 [V][4][3][3];
site = x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# Gamma matrices, chiral (DeGrand-Rossi) basis; gamma5 = g1 g2 g3 g4 = diag(1,1,-1,-1)
# --------------------------------------------------------------------------
_i = 1j
GAMMA = np.array([
    [[0, 0, 0, _i], [0, 0, _i, 0], [0, -_i, 0, 0], [-_i, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, _i, 0], [0, 0, 0, -_i], [-_i, 0, 0, 0], [0, _i, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
EYE4 = np.eye(4, dtype=np.complex128)


def _shape(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return lt, lz, ly, lx


def _axis(mu: int) -> int:
    # array axes are (t, z, y, x, ...): direction mu = 0 (x) is axis 3, mu = 3 (t) is axis 0
    return 3 - mu


def hopping(links: np.ndarray, psi: np.ndarray, dims, dagger: bool = False) -> np.ndarray:
    """D psi = sum_mu [(1 -/+ g_mu) U_mu(x) psi(x+mu) + (1 +/- g_mu) U_mu(x-mu)^dag psi(x-mu)].

    ``psi`` may carry a trailing batch axis: shape [V,4,3] or [V,4,3,B].
    With ``dagger`` the projector signs swap (gamma5 D gamma5 = D^dag).
    """
    batched = psi.ndim == 4
    p = psi if batched else psi[..., None]
    sh = _shape(dims)
    u = links.reshape(sh + (4, 3, 3))
    p = p.reshape(sh + (4, 3, p.shape[-1]))
    out = np.zeros_like(p)
    sgn = -1.0 if not dagger else 1.0
    for mu in range(4):
        ax = _axis(mu)
        umu = u[..., mu, :, :]
        fwd = np.roll(p, -1, axis=ax)
        uf = np.einsum("TZYXab,TZYXsbn->TZYXsan", umu, fwd)
        out += np.einsum("st,TZYXtan->TZYXsan", EYE4 + sgn * GAMMA[mu], uf)
        ub = np.roll(umu, 1, axis=ax)
        bwd = np.roll(p, 1, axis=ax)
        ubw = np.einsum("TZYXba,TZYXsbn->TZYXsan", ub.conj(), bwd)
        out += np.einsum("st,TZYXtan->TZYXsan", EYE4 - sgn * GAMMA[mu], ubw)
    out = out.reshape((-1, 4, 3, out.shape[-1]))
    return out if batched else out[..., 0]


def gamma5(psi: np.ndarray) -> np.ndarray:
    """Multiply by gamma5 on the spin index (axis 1)."""
    if psi.ndim == 4:
        return np.einsum("st,vtcn->vscn", GAMMA5, psi)
    return np.einsum("st,vtc->vsc", GAMMA5, psi)


def wilson(links, psi, dims, kappa: float) -> np.ndarray:
    """M psi = psi - kappa D psi."""
    return psi - kappa * hopping(links, psi, dims)


def wilson_dag(links, psi, dims, kappa: float) -> np.ndarray:
    """M^dag psi = psi - kappa D^dag psi."""
    return psi - kappa * hopping(links, psi, dims, dagger=True)


def g5wilson(links, psi, dims, kappa: float) -> np.ndarray:
    """gamma5 M psi (Hermitian, indefinite)."""
    return gamma5(wilson(links, psi, dims, kappa))


def mdagm(links, psi, dims, kappa: float) -> np.ndarray:
    """M^dag M psi (Hermitian positive definite)."""
    return wilson_dag(links, wilson(links, psi, dims, kappa), dims, kappa)


class WilsonOperator:
    """Callable operators on flat complex vectors of length 12 V."""

    def __init__(self, links, dims, kappa: float):
        self.links = np.asarray(links, dtype=np.complex128)
        self.dims = tuple(int(d) for d in dims)
        self.kappa = float(kappa)
        self.V = int(np.prod(self.dims))
        self.n = 12 * self.V

    def _wrap(self, f, v):
        shp = v.shape
        if v.ndim == 1:
            out = f(self.links, v.reshape(self.V, 4, 3), self.dims, self.kappa)
        else:  # (n, B) column batch
            out = f(self.links, v.reshape(self.V, 4, 3, shp[-1]), self.dims, self.kappa)
        return out.reshape(shp)

    def M(self, v):
        return self._wrap(wilson, v)

    def Mdag(self, v):
        return self._wrap(wilson_dag, v)

    def g5M(self, v):
        return self._wrap(g5wilson, v)

    def MdagM(self, v):
        return self._wrap(mdagm, v)

    def g5(self, v):
        shp = v.shape
        if v.ndim == 1:
            return gamma5(v.reshape(self.V, 4, 3)).reshape(shp)
        return gamma5(v.reshape(self.V, 4, 3, shp[-1])).reshape(shp)


def dense(apply, n: int, batch: int = 256) -> np.ndarray:
    """Dense matrix of a linear map on C^n, built column by column."""
    a = np.zeros((n, n), dtype=np.complex128)
    for j0 in range(0, n, batch):
        j1 = min(n, j0 + batch)
        e = np.zeros((n, j1 - j0), dtype=np.complex128)
        e[np.arange(j0, j1), np.arange(j1 - j0)] = 1.0
        a[:, j0:j1] = apply(e)
    return a


def free_mdagm_spectrum(dims, kappa: float) -> np.ndarray:
    """Closed-form eigenvalues of M^dag M for U = 1 (periodic), each with multiplicity 12.

    A plane wave psi(x) = exp(i p.x) u gives M(p) = 1 - 2 kappa sum cos p_mu
    + 2 i kappa sum gamma_mu sin p_mu, so M^dag M(p) = (1 - 2 kappa sum cos p_mu)^2
    + 4 kappa^2 sum sin^2 p_mu, with p_mu = 2 pi n_mu / L_mu.
    """
    grids = np.meshgrid(*[2 * np.pi * np.arange(L) / L for L in dims], indexing="ij")
    c = sum(np.cos(g) for g in grids)
    s2 = sum(np.sin(g) ** 2 for g in grids)
    lam = (1 - 2 * kappa * c) ** 2 + 4 * kappa ** 2 * s2
    return np.sort(np.repeat(lam.ravel(), 12))
