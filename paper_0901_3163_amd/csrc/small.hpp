// Launchers of the one-workgroup FP64 small dense kernels (small.hip).
#pragma once
#include "internal.hpp"

namespace dl {

// Symmetric eigendecomposition (A destroyed): ev ascending, Z[i*n + l] = l-th eigenvector.
size_t small_eigh_work(int n);
void small_eigh(hipStream_t s, int n, double* A, double* Z, double* ev, double* work);

// Lan-DR(m,k) cycle end.  Tb ((m+1) x m with leading dimension ld >= m, lower
// triangle) and c (m+1) are
// replaced by the next cycle's arrowhead system.  d (m): Galerkin solution of
// T_m d = c; Gk (m x k): kept Ritz vectors of T_m; theta/rho (k): Ritz values
// and residual norms |beta_m G[m-1, i]|.  info: [||T_m||_inf, beta_m, |beta_m d_m|, rotations].
size_t landr_work(int m);
void landr_cycle(hipStream_t s, int m, int ld, int k, double* Tb, double* c, double* work, double* d, double* Gk,
                 double* theta, double* rho, double* info);

// MinRes-DR(m,k) cycle end.  d (m): least-squares solution; Q ((m+1) x (k+1)):
// orthonormal restart basis; lam/S (k, k x k): Rayleigh-Ritz pairs of the
// restarted projected matrix; rho (k): their residual norms; hth (k): kept
// harmonic Ritz values.  info: [||T_m||_inf, beta_m, ||c - Tbar d||, rotations].
size_t minresdr_work(int m);
void minresdr_cycle(hipStream_t s, int m, int k, double* Tb, double* c, double* work, double* d, double* Q,
                    double* lam, double* S, double* rho, double* hth, double* info);

// Galerkin projection solves with H = Y^H A Y (k x k complex Hermitian).
// proj_setup: E, Z (2k x 2k), lamr (2k), work (4*(k+1) doubles).
void proj_setup(hipStream_t s, int k, const double2* Hc, double* E, double* Z, double* lamr, double* work);
// d[r] = H^-1 c[r] for r < nrhs; c, d: [nrhs][k] complex.
void proj_solve(hipStream_t s, int k, int nrhs, const double* Z, const double* lamr, const double2* c, double2* d);

}  // namespace dl
