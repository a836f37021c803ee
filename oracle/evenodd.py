"""Even-odd (Schur complement) form of the Wilson matrix, FP64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not in the paper, which solves with "the Wilson matrix" itself (Section 2); this is the
usual production form of the same linear system, one step below the stencil.  With
sites split by parity p(x) = (x + y + z + t) mod 2 (every extent even), the hopping term D
of M = 1 - kappa D only connects opposite parities, so in (even, odd) blocks

    M = [[1, -kappa D_eo], [-kappa D_oe, 1]],

and M x = b is equivalent to the even-site system

    Mhat x_e = bhat_e,   Mhat = 1 - kappa^2 D_eo D_oe,   bhat_e = b_e + kappa D_eo b_o,

followed by x_o = b_o + kappa D_oe x_e.  Mhat^dag = gamma5 Mhat gamma5 (gamma5 commutes with
parity), so gamma5 Mhat is Hermitian and Mhat^dag Mhat is positive definite: the forms the
deflated methods iterate on.  A half field holds the sites of one parity in increasing
full-site order (site = x + Lx (y + Ly (z + Lz t))), [V/2][4][3].
"""
from __future__ import annotations

import numpy as np

from . import dirac


def parity(dims) -> np.ndarray:
    """p(site) = (x + y + z + t) mod 2 for every site, in full-site order."""
    lx, ly, lz, lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return ((x + y + z + t) % 2).ravel()


def check_dims(dims):
    if any(int(d) % 2 for d in dims):
        raise ValueError("the even-odd form needs every lattice extent even")


class EvenOdd:
    """The blocks of M and the even-site Schur complement on half fields ([V/2][4][3] or flat)."""

    def __init__(self, links, dims, kappa: float):
        check_dims(dims)
        self.links = np.asarray(links, dtype=np.complex128)
        self.dims = tuple(int(d) for d in dims)
        self.kappa = float(kappa)
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        self.n = 12 * self.Vh
        p = parity(self.dims)
        self.sites = (np.nonzero(p == 0)[0], np.nonzero(p == 1)[0])

    def split(self, psi):
        """Full field -> (even half, odd half)."""
        f = np.asarray(psi).reshape(self.V, 4, 3)
        return f[self.sites[0]].copy(), f[self.sites[1]].copy()

    def merge(self, pe, po):
        """(even half, odd half) -> full field [V][4][3]."""
        f = np.zeros((self.V, 4, 3), dtype=np.complex128)
        f[self.sites[0]] = np.asarray(pe).reshape(self.Vh, 4, 3)
        f[self.sites[1]] = np.asarray(po).reshape(self.Vh, 4, 3)
        return f

    def hop(self, half, src, dagger=False):
        """D_{dst,src} applied to a half field of parity src: the full hopping term of the
        field that is `half` on the src sites and zero elsewhere, read on the other parity."""
        f = np.zeros((self.V, 4, 3), dtype=np.complex128)
        f[self.sites[src]] = np.asarray(half).reshape(self.Vh, 4, 3)
        g = dirac.hopping(self.links, f, self.dims, dagger=dagger)
        return g[self.sites[1 - src]]

    def _cols(self, f, v):
        """f on a half field, or on every column of an (n, B) batch."""
        v = np.asarray(v)
        if v.ndim == 2 and v.shape[0] == self.n:
            return np.stack([f(v[:, j]) for j in range(v.shape[1])], axis=1)
        return f(v)

    def Mhat(self, v):
        """Mhat v = v - kappa^2 D_eo D_oe v on even half fields (flat or [V/2][4][3])."""
        def one(w):
            h = np.asarray(w).reshape(self.Vh, 4, 3)
            return (h - self.kappa ** 2 * self.hop(self.hop(h, 0), 1)).reshape(np.shape(w))
        return self._cols(one, v)

    def Mhat_dag(self, v):
        def one(w):
            h = np.asarray(w).reshape(self.Vh, 4, 3)
            return (h - self.kappa ** 2 * self.hop(self.hop(h, 0, dagger=True), 1, dagger=True)).reshape(np.shape(w))
        return self._cols(one, v)

    def g5(self, v):
        return self._cols(lambda w: dirac.gamma5(np.asarray(w).reshape(self.Vh, 4, 3)).reshape(np.shape(w)), v)

    def g5Mhat(self, v):
        return self.g5(self.Mhat(v))

    def MhatdagMhat(self, v):
        return self.Mhat_dag(self.Mhat(v))

    def prepare(self, b):
        """bhat_e = b_e + kappa D_eo b_o for a full right-hand side b."""
        be, bo = self.split(b)
        return be + self.kappa * self.hop(bo, 1)

    def reconstruct(self, b, xe):
        """The full solution from the even-site one: x_o = b_o + kappa D_oe x_e."""
        _, bo = self.split(b)
        xe = np.asarray(xe).reshape(self.Vh, 4, 3)
        return self.merge(xe, bo + self.kappa * self.hop(xe, 0))
