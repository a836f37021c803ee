"""Rounded storage of fields and of the deflation basis (plain numpy, FP64 arithmetic).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper runs its later right-hand sides with the Galerkin projection over the
stored eigenvectors (Section 2: H d = Y^H r, x += Y d, H = Y^H A Y).  Storing Y
in a narrower format changes which basis that projection uses; this module
writes out what the rounded variants compute, from their definitions:

* round_f32 / round_bf16: IEEE binary32 rounding of each real part, and bfloat16
  (8 exponent bits, 7 fraction bits) obtained from the binary32 value by
  round-to-nearest-even on the upper 16 bits.
* lowered_projection: the coefficients come from a contraction basis Yc and a
  rounded residual, c = Yc^H q(r); the correction is taken on a Galerkin basis Yg
  with its own matrix Hg = Yg^H A Yg, x += Yg Hg^-1 c.  With Yc = Yg = Y and no
  rounding this is the paper's projection.
"""
from __future__ import annotations

import numpy as np


def round_f32(z: np.ndarray) -> np.ndarray:
    """Each real and imaginary part rounded to the nearest binary32 value (ties to even)."""
    z = np.asarray(z, dtype=np.complex128)
    return z.astype(np.complex64).astype(np.complex128)


def _bf16_bits(x32: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of binary32 values to their upper 16 bits (finite inputs)."""
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return (u << np.uint64(16)).astype(np.uint32).view(np.float32)


def round_bf16(z: np.ndarray) -> np.ndarray:
    """Each real and imaginary part rounded to binary32, then to bfloat16 (ties to even)."""
    z = np.asarray(z, dtype=np.complex128)
    re = _bf16_bits(np.ascontiguousarray(z.real, dtype=np.float32)).astype(np.float64)
    im = _bf16_bits(np.ascontiguousarray(z.imag, dtype=np.float32)).astype(np.float64)
    return re + 1j * im


def rounding(prec: str):
    """The rounding map of a storage name ('fp64', 'fp32', 'bf16')."""
    return {"fp64": lambda z: np.asarray(z, dtype=np.complex128), "fp32": round_f32, "bf16": round_bf16}[prec]


def contraction(V: np.ndarray, W: np.ndarray, prec: str) -> np.ndarray:
    """C[r, j] = <q(V_j), q(W_r)> for rows V_j, W_r, q the rounding of prec; exact FP64 sums
    of the products of the rounded values."""
    q = rounding(prec)
    return q(W) @ q(V).conj().T


def gram(A, Y: np.ndarray) -> np.ndarray:
    """H = Y^H A Y (columns of Y), k applications of A."""
    if Y.shape[1] == 0:
        return np.zeros((0, 0), dtype=np.complex128)
    AY = np.stack([A(Y[:, i]) for i in range(Y.shape[1])], axis=1)
    return Y.conj().T @ AY


def lowered_projection(Yc: np.ndarray, Yg: np.ndarray, Hg: np.ndarray, r: np.ndarray, prec: str) -> np.ndarray:
    """The correction Yg Hg^-1 (Yc^H q(r)) (columns of Yc, Yg), q the rounding of prec."""
    if Yg.shape[1] == 0:
        return np.zeros_like(r)
    c = Yc.conj().T @ rounding(prec)(r)
    return Yg @ np.linalg.solve(Hg, c)
