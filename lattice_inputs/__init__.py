"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only *draws* inputs; it holds none of the solver or operator
arithmetic.  Both sides (the FP64 oracle and the HIP library) receive the same
numpy arrays produced here.

Host layouts (interleaved complex128, C order):

* links  ``U[site][mu][row][col]`` with ``site = x + Lx*(y + Ly*(z + Lz*t))``
  and ``mu = 0..3`` for the x, y, z, t directions;
* spinor ``psi[site][spin][colour]`` (4 spin x 3 colour = 12 complex per site).

The paper's lattice runs use quenched beta=6.0 ensembles (Section 2), which are
not available; a near-identity random SU(3) field stands in for them:
``U = exp(i * eps * X)`` with X a Gaussian traceless Hermitian 3x3 matrix per
link, ``X = sum_a w_a lambda_a / 2`` (Gell-Mann lambda_a, w_a ~ N(0,1)).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "gell_mann", "su3_links", "gaussian_spinor", "point_source",
    "diag_spectrum_positive", "diag_spectrum_indefinite", "gaussian_vector",
]


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0, 0, 1] = lam[0, 1, 0] = 1
    lam[1, 0, 1], lam[1, 1, 0] = -1j, 1j
    lam[2, 0, 0], lam[2, 1, 1] = 1, -1
    lam[3, 0, 2] = lam[3, 2, 0] = 1
    lam[4, 0, 2], lam[4, 2, 0] = -1j, 1j
    lam[5, 1, 2] = lam[5, 2, 1] = 1
    lam[6, 1, 2], lam[6, 2, 1] = -1j, 1j
    lam[7, 0, 0] = lam[7, 1, 1] = 1 / np.sqrt(3)
    lam[7, 2, 2] = -2 / np.sqrt(3)
    return lam


def su3_links(dims, seed: int, eps: float = 0.5) -> np.ndarray:
    """Random SU(3) links U = exp(i eps X), complex128 [V][4][3][3].

    X = sum_a w_a lambda_a / 2 with w ~ default_rng(seed).standard_normal((V,4,8)).
    The exponential is taken through the eigendecomposition of the Hermitian X,
    so U is unitary and det U = exp(i eps tr X) = 1 up to rounding.
    """
    vol = volume(dims)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((vol, 4, 8))
    x = np.einsum("sma,aij->smij", w, gell_mann()) / 2.0
    ev, vec = np.linalg.eigh(x)
    phase = np.exp(1j * eps * ev)
    u = np.einsum("smij,smj,smkj->smik", vec, phase, vec.conj())
    return np.ascontiguousarray(u)


def gaussian_spinor(dims, seed: int) -> np.ndarray:
    """Complex Gaussian spinor field, re/im ~ N(0,1), complex128 [V][4][3]."""
    vol = volume(dims)
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((vol, 4, 3))
    im = rng.standard_normal((vol, 4, 3))
    return re + 1j * im


def gaussian_spinors_device(dims, seed: int, n: int, device="cuda"):
    """n complex Gaussian spinor fields [n][V][4][3] (re, im ~ N(0,1)), complex128, drawn on a
    torch device by torch's seeded generator: the bulk right-hand sides of the benchmark (thousands
    of fields, where host draws would dominate the run)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    x = torch.randn((n, volume(dims), 4, 3, 2), generator=g, device=device, dtype=torch.float64)
    return torch.view_as_complex(x)


def point_source(dims, site: int, spin: int, colour: int) -> np.ndarray:
    """Unit spin-colour point source e_{site, spin, colour}, complex128 [V][4][3]."""
    b = np.zeros((volume(dims), 4, 3), dtype=np.complex128)
    b[site, spin, colour] = 1.0
    return b


def gaussian_vector(n: int, seed: int, complex_: bool = True) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if complex_:
        return rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return rng.standard_normal(n).astype(np.complex128)


def diag_spectrum_positive() -> np.ndarray:
    """Eigenvalues 0.1, 1, 2, ..., 999 of the first diagonal example (Section 1)."""
    return np.concatenate([[0.1], np.arange(1.0, 1000.0)])


def diag_spectrum_indefinite(seed: int = 5) -> np.ndarray:
    """N(0,1) + 2.0 diagonal of the second example (Section 1), dimension 1000.

    The paper's draw has 22 negative entries; default_rng(5) reproduces that count.
    """
    return np.random.default_rng(seed).standard_normal(1000) + 2.0


def net_weights(seed: int, widths=(4, 16, 16, 4), scale: float = 0.3) -> np.ndarray:
    """Seeded complex Gaussian weights of the learned-guess network: per layer an array
    [9 hops][C_out][C_in] with entries of variance scale^2 / (9 C_in), layers concatenated."""
    rng = np.random.default_rng(seed)
    ws = []
    for l in range(len(widths) - 1):
        cin, cout = widths[l], widths[l + 1]
        sd = scale / np.sqrt(9 * cin)
        ws.append(sd * (rng.standard_normal((9, cout, cin)) + 1j * rng.standard_normal((9, cout, cin))) / np.sqrt(2))
    return np.concatenate([w.ravel() for w in ws])
