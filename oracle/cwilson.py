"""ctypes wrapper of the plain-C oracle Wilson matrix (oracle/c/wilson_ref.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The same operator as
oracle.dirac (pinned against it in tests/test_oracle.py), compiled with gcc
and OpenMP so that the kappa search and the CPU baseline can run on lattices
where the numpy transcription is too slow.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "wilson_ref.c")
LIB = os.path.join(HERE, "c", "libwilson_ref.so")


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", SRC, "-o", LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _lib.wilson_ref.restype = None
        _lib.wilson_ref.argtypes = [C.POINTER(C.c_int), C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int]
    return _lib


class CWilson:
    """M, M^dag, gamma5 M, M^dag M on flat complex vectors of length 12 V."""

    def __init__(self, links, dims, kappa):
        self.U = np.ascontiguousarray(links, dtype=np.complex128)
        self.dims = (C.c_int * 4)(*[int(d) for d in dims])
        self.kappa = float(kappa)
        self.V = int(np.prod(dims))
        self.n = 12 * self.V
        self.lib = _load()

    def _apply(self, v, which):
        v = np.ascontiguousarray(v, dtype=np.complex128)
        out = np.empty_like(v)
        self.lib.wilson_ref(self.dims, self.U.ctypes.data, v.ctypes.data, out.ctypes.data, self.kappa, which)
        return out

    def M(self, v):
        return self._apply(v, 0)

    def Mdag(self, v):
        return self._apply(v, 1)

    def g5M(self, v):
        return self._apply(v, 2)

    def MdagM(self, v):
        return self._apply(self._apply(v, 0), 1)
