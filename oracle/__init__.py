"""FP64 CPU oracle for the deflated Hermitian Lanczos methods (arXiv:0901.3163).

TEST INFRASTRUCTURE ONLY.  Nothing in the library path may import, call or
link anything in this package: it exists so that ``tests/``, the smoke check
and the CPU-baseline leg of the benchmark can compare the HIP library against a
plain, slow, obviously-correct implementation.  It shares no code, tables or
helpers with the GPU path; the only thing both sides share is the seeded input
arrays drawn by ``lattice_inputs``.

Contents
--------
dirac     -- gamma matrices (chiral basis), Wilson matrix M, gamma5 M, M^dag M,
             dense builders and the free-field closed form.
krylov    -- CG, CGLS (CG on the normal equations), MinRes (Paige-Saunders).
deflated  -- Lan-DR(m,k), MinRes-DR(m,k), D-CG and D-MinRes.
kappa     -- the kappa search that fixes the near-critical mass of the
             synthetic lattice workloads.
ptc       -- the gauge-covariant parallel-transport convolution network used
             for the learned initial guess (forward and hand-written backward).
lowp      -- binary32 and bfloat16 rounding, the contraction of rounded fields and
             the Galerkin projection over a rounded eigenvector basis.

All arithmetic is complex128/float64 with inner product <u, v> = sum conj(u) v.
"""
