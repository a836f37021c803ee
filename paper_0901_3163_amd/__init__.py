"""deflan: deflated Hermitian Lanczos solvers (Lan-DR, MinRes-DR, D-CG, D-MinRes)
for the Wilson-Dirac matrix on MI355X (gfx950), after Abdel-Rehim, Morgan,
Nicely and Wilcox, arXiv:0901.3163.

The compute path is the HIP library ``libdeflan.so`` (C ABI in
``include/deflan.h``); ``deflan`` is its thin ctypes binding.
"""
from . import deflan  # noqa: F401  (raises ImportError if libdeflan.so is missing)
from .deflan import (Context, Operator, Eig, DeflanError, DL_MDAGM, DL_G5M, DL_FP64, DL_FP32, DL_BF16,  # noqa: F401
                     DL_APPLY_M, DL_APPLY_MDAG, DL_APPLY_G5M, DL_APPLY_MDAGM)
