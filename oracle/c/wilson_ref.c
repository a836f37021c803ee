/*
 * Plain C transcription of the Wilson matrix (the oracle's; test
 * infrastructure only -- nothing in the library path links this file).
 *
 *   (M psi)(x) = psi(x) - kappa * sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                                         + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *
 * Straight loops over sites with the full 4x4 gamma matrices of the chiral
 * basis (no spin projection), so it shares nothing with the GPU stencil.
 * Layouts are the host layouts: psi[V][4][3], U[V][4][3][3] interleaved
 * complex128, site = x + Lx*(y + Ly*(z + Lz*t)).  OpenMP over sites.
 */
#include <complex.h>
#include <stddef.h>

typedef double complex cplx;

static const cplx I_ = I;

static void gammas(cplx g[4][4][4]) {
  for (int m = 0; m < 4; ++m)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) g[m][a][b] = 0;
  /* g1 */ g[0][0][3] = I_;  g[0][1][2] = I_;  g[0][2][1] = -I_; g[0][3][0] = -I_;
  /* g2 */ g[1][0][3] = -1;  g[1][1][2] = 1;   g[1][2][1] = 1;   g[1][3][0] = -1;
  /* g3 */ g[2][0][2] = I_;  g[2][1][3] = -I_; g[2][2][0] = -I_; g[2][3][1] = I_;
  /* g4 */ g[3][0][2] = 1;   g[3][1][3] = 1;   g[3][2][0] = 1;   g[3][3][1] = 1;
}

/* which: 0 M, 1 M^dag, 2 gamma5 M */
void wilson_ref(const int* dims, const cplx* U, const cplx* in, cplx* out, double kappa, int which) {
  const long Lx = dims[0], Ly = dims[1], Lz = dims[2], Lt = dims[3];
  const long V = Lx * Ly * Lz * Lt;
  const long L[4] = {Lx, Ly, Lz, Lt};
  const long stride[4] = {1, Lx, Lx * Ly, Lx * Ly * Lz};
  cplx g[4][4][4];
  gammas(g);
  const double sf = (which == 1) ? 1.0 : -1.0; /* forward projector 1 + sf g_mu */
#pragma omp parallel for schedule(static)
  for (long s = 0; s < V; ++s) {
    long c[4] = {s % Lx, (s / Lx) % Ly, (s / (Lx * Ly)) % Lz, s / (Lx * Ly * Lz)};
    cplx acc[4][3];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 3; ++b) acc[a][b] = 0;
    for (int mu = 0; mu < 4; ++mu) {
      const long fw = s + (c[mu] == L[mu] - 1 ? (1 - L[mu]) * stride[mu] : stride[mu]);
      const long bw = s + (c[mu] == 0 ? (L[mu] - 1) * stride[mu] : -stride[mu]);
      const cplx* Uf = U + (s * 4 + mu) * 9;
      const cplx* Ub = U + (bw * 4 + mu) * 9;
      const cplx* pf = in + fw * 12;
      const cplx* pb = in + bw * 12;
      cplx uf[4][3], ub[4][3];
      for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
          cplx t1 = 0, t2 = 0;
          for (int b = 0; b < 3; ++b) {
            t1 += Uf[a * 3 + b] * pf[sp * 3 + b];
            t2 += conj(Ub[b * 3 + a]) * pb[sp * 3 + b];
          }
          uf[sp][a] = t1;
          ub[sp][a] = t2;
        }
      for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
          cplx t = uf[sp][a] + ub[sp][a];
          for (int q = 0; q < 4; ++q) t += sf * g[mu][sp][q] * uf[q][a] - sf * g[mu][sp][q] * ub[q][a];
          acc[sp][a] += t;
        }
    }
    for (int sp = 0; sp < 4; ++sp)
      for (int a = 0; a < 3; ++a) {
        cplx r = in[s * 12 + sp * 3 + a] - kappa * acc[sp][a];
        if (which == 2 && sp >= 2) r = -r;
        out[s * 12 + sp * 3 + a] = r;
      }
  }
}
