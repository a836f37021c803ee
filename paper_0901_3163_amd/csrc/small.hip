// Small dense FP64 problems of the restart and deflation steps, each solved by
// one workgroup of 1024 threads on matrices of order m <= 512 held in global
// memory (they stay resident in L2).
//
//  * jacobi_eigh -- cyclic Jacobi for real symmetric matrices with the
//    round-robin (circle) pairing: every round applies n/2 disjoint rotations
//    at once, so A <- J^T A J splits into independent 2x2 blocks and the round
//    needs two barriers.  Rotations are skipped when |a_pq| is below
//    eps * sqrt(|a_pp a_qq|) (relative accuracy for small eigenvalues); sweeps
//    stop when a sweep applies no rotation.
//  * k_landr_cycle -- end of a Lan-DR(m,k) cycle: Galerkin solve T_m d = c,
//    Ritz pairs of T_m, the k algebraically smallest kept, the arrowhead
//    projected matrix and right-hand side of the next cycle.
//  * k_minresdr_cycle -- end of a MinRes-DR(m,k) cycle: Householder QR of the
//    (m+1) x m matrix Tbar, least-squares d, the residual direction q spanning
//    range(Tbar)^perp, harmonic Ritz pairs from R^-T T_m R^-1 y = mu y
//    (Tbar^T Tbar = R^T R, theta = 1/mu), k smallest |theta| kept, the
//    orthonormal restart basis Q of [[G_k; 0], q], Q^T Tbar Q and Q^T s.
//  * k_proj_setup / k_proj_solve -- the Galerkin projection H d = c of
//    D-CG / D-MinRes with H = Y^H A Y complex Hermitian, solved through the
//    eigendecomposition of its real symmetric embedding [[Hr, -Hi], [Hi, Hr]].
//
// All projected matrices of the Hermitian Lanczos process are real: alpha_j
// and beta_j are real, and the restart matrices are real combinations.
#include "internal.hpp"
#include "small.hpp"

namespace dl {

constexpr int kSmallThreads = 1024;

__device__ __forceinline__ double blk_reduce(double v, double* red, bool is_max) {
  // result broadcast to all threads
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = is_max ? fmax(v, o) : v + o;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = is_max ? -1.0 : 0.0;
  for (int w = 0; w < nw; ++w) r = is_max ? fmax(r, red[w]) : r + red[w];
  __syncthreads();
  return r;
}

// Eigendecomposition of the symmetric n x n matrix A (destroyed; eigenvalues
// end on its diagonal), Z <- eigenvectors (columns).  rot: n/2+1 double4.
__device__ void jacobi_eigh(int n, double* A, int lda, double* Z, int ldz, double4* rot, double* red,
                            int* nrot) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    const int i = e / n, j = e % n;
    Z[(long)i * ldz + j] = (i == j) ? 1.0 : 0.0;
  }
  if (n <= 1) { __syncthreads(); return; }
  const int np = n + (n & 1), half = np / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double dm = 0.0;
    for (int i = tid; i < n; i += nt) dm = fmax(dm, fabs(A[(long)i * lda + i]));
    dm = blk_reduce(dm, red, true);
    double offmax = 0.0;
    for (int e = tid; e < n * n; e += nt) {
      const int i = e / n, j = e % n;
      if (i != j) offmax = fmax(offmax, fabs(A[(long)i * lda + j]));
    }
    offmax = blk_reduce(offmax, red, true);
    const double scale = fmax(dm, offmax);
    if (tid == 0) *nrot = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      for (int t = tid; t < half; t += nt) {
        int p, q;
        if (t == 0) { p = np - 1; q = r; }
        else { p = (r + t) % (np - 1); q = (r - t + np - 1) % (np - 1); }
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double app = A[(long)p * lda + p], aqq = A[(long)q * lda + q], apq = A[(long)p * lda + q];
          const double aa = fabs(apq);
          if (aa > 2.220446049250313e-16 * sqrt(fabs(app * aqq)) && aa > 1e-18 * scale && aa > 1e-300) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            atomicAdd(nrot, 1);
          }
        }
        rot[t] = make_double4((double)p, (double)q, c, s);
      }
      __syncthreads();
      for (int e = tid; e < half * half; e += nt) {
        const int t1 = e / half, t2 = e % half;
        const double4 r1 = rot[t1], r2 = rot[t2];
        if (r1.w == 0.0 && r2.w == 0.0) continue;
        const int p1 = (int)r1.x, q1 = (int)r1.y, p2 = (int)r2.x, q2 = (int)r2.y;
        const bool q1ok = q1 < n, q2ok = q2 < n;
        const double c1 = r1.z, s1 = r1.w, c2 = r2.z, s2 = r2.w;
        const double a_pp = A[(long)p1 * lda + p2];
        const double a_pq = q2ok ? A[(long)p1 * lda + q2] : 0.0;
        const double a_qp = q1ok ? A[(long)q1 * lda + p2] : 0.0;
        const double a_qq = (q1ok && q2ok) ? A[(long)q1 * lda + q2] : 0.0;
        const double b_pp = c1 * a_pp - s1 * a_qp, b_pq = c1 * a_pq - s1 * a_qq;
        const double b_qp = s1 * a_pp + c1 * a_qp, b_qq = s1 * a_pq + c1 * a_qq;
        double n_pp = c2 * b_pp - s2 * b_pq, n_pq = s2 * b_pp + c2 * b_pq;
        double n_qp = c2 * b_qp - s2 * b_qq, n_qq = s2 * b_qp + c2 * b_qq;
        if (t1 == t2) { n_pq = 0.0; n_qp = 0.0; }
        A[(long)p1 * lda + p2] = n_pp;
        if (q2ok) A[(long)p1 * lda + q2] = n_pq;
        if (q1ok) A[(long)q1 * lda + p2] = n_qp;
        if (q1ok && q2ok) A[(long)q1 * lda + q2] = n_qq;
      }
      for (int e = tid; e < n * half; e += nt) {
        const int i = e / half, t = e % half;
        const double4 rr = rot[t];
        if (rr.w == 0.0) continue;
        const int p = (int)rr.x, q = (int)rr.y;
        const double zp = Z[(long)i * ldz + p], zq = Z[(long)i * ldz + q];
        Z[(long)i * ldz + p] = rr.z * zp - rr.w * zq;
        Z[(long)i * ldz + q] = rr.w * zp + rr.z * zq;
      }
      __syncthreads();
    }
    const int done = (*nrot == 0);
    __syncthreads();
    if (done) break;
  }
}

// perm[rank] = i with ranks by (key ascending, index ascending).
__device__ void rank_sort(int n, const double* key, int* perm) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double ki = key[i];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double kj = key[j];
      r += (kj < ki) || (kj == ki && j < i);
    }
    perm[r] = i;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSmallThreads)
k_small_eigh(int n, double* A, double* Z, double* ev, double* work) {
  __shared__ double red[kSmallThreads / 64];
  __shared__ int nrot;
  double4* rot = reinterpret_cast<double4*>(work);
  double* key = work + 4 * (n / 2 + 1);
  int* perm = reinterpret_cast<int*>(key + n);
  double* Zt = key + 2 * n;
  jacobi_eigh(n, A, n, Zt, n, rot, red, &nrot);
  for (int i = threadIdx.x; i < n; i += blockDim.x) key[i] = A[(long)i * n + i];
  __syncthreads();
  rank_sort(n, key, perm);
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, l = e % n;
    Z[(long)i * n + l] = Zt[(long)i * n + perm[l]];
  }
  for (int l = threadIdx.x; l < n; l += blockDim.x) ev[l] = key[perm[l]];
}

size_t small_eigh_work(int n) { return 4 * (size_t)(n / 2 + 1) + 2 * (size_t)n + (size_t)n * n + 8; }

void small_eigh(hipStream_t s, int n, double* A, double* Z, double* ev, double* work) {
  hipLaunchKernelGGL(k_small_eigh, dim3(1), dim3(kSmallThreads), 0, s, n, A, Z, ev, work);
  DL_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Lan-DR cycle end.  Tb: (m+1) x m row-major (lower triangle valid), c: m+1.
// Outputs: d (m), Gk (m x k, ld k), info[0..]: see small.hpp.
__global__ void __launch_bounds__(kSmallThreads)
k_landr_cycle(int m, int ld, int k, double* Tb, double* c, double* work, double* d, double* Gk, double* theta,
              double* rho, double* info) {
  __shared__ double red[kSmallThreads / 64];
  __shared__ int nrot;
  const int tid = threadIdx.x, nt = blockDim.x;
  double4* rot = reinterpret_cast<double4*>(work);  // m/2+1
  double* A = work + 4 * (m / 2 + 1);  // m*m
  double* Z = A + (long)m * m;         // m*m
  double* ev = Z + (long)m * m;        // m
  double* y = ev + m;                  // m
  int* perm = reinterpret_cast<int*>(y + m);  // m ints
  for (int e = tid; e < m * m; e += nt) {
    const int i = e / m, j = e % m;
    A[e] = (i >= j) ? Tb[(long)i * ld + j] : Tb[(long)j * ld + i];
  }
  __syncthreads();
  double rs = 0.0;
  for (int i = tid; i < m; i += nt) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += fabs(A[(long)i * m + j]);
    rs = fmax(rs, s);
  }
  const double anorm = blk_reduce(rs, red, true);
  const double beta_m = Tb[(long)m * ld + (m - 1)];
  jacobi_eigh(m, A, m, Z, m, rot, red, &nrot);
  for (int i = tid; i < m; i += nt) ev[i] = A[(long)i * m + i];
  __syncthreads();
  // d = Z diag(1/ev) Z^T c
  for (int i = tid; i < m; i += nt) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += Z[(long)j * m + i] * c[j];
    y[i] = s / ev[i];
  }
  __syncthreads();
  for (int j = tid; j < m; j += nt) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += Z[(long)j * m + i] * y[i];
    d[j] = s;
  }
  rank_sort(m, ev, perm);  // contains a barrier; d visible after it
  for (int e = tid; e < m * k; e += nt) {
    const int j = e / k, l = e % k;
    Gk[e] = Z[(long)j * m + perm[l]];
  }
  for (int l = tid; l < k; l += nt) {
    theta[l] = ev[perm[l]];
    rho[l] = fabs(beta_m * Z[(long)(m - 1) * m + perm[l]]);
  }
  const double dm = d[m - 1];
  __syncthreads();
  for (long e = tid; e < (long)(m + 1) * ld; e += nt) Tb[e] = 0.0;
  for (int i = tid; i <= m; i += nt) c[i] = 0.0;
  __syncthreads();
  for (int l = tid; l < k; l += nt) {
    Tb[(long)l * ld + l] = ev[perm[l]];
    Tb[(long)k * ld + l] = beta_m * Z[(long)(m - 1) * m + perm[l]];
  }
  if (tid == 0) {
    c[k] = -beta_m * dm;
    info[0] = anorm;
    info[1] = beta_m;
    info[2] = fabs(beta_m * dm);  // norm of the (normal-equation) FOM residual
    info[3] = (double)nrot;
  }
}

size_t landr_work(int m) { return 2 * (size_t)m * m + 3 * (size_t)m + 4 * (size_t)(m / 2 + 1) + 16; }

void landr_cycle(hipStream_t s, int m, int ld, int k, double* Tb, double* c, double* work, double* d, double* Gk,
                 double* theta, double* rho, double* info) {
  hipLaunchKernelGGL(k_landr_cycle, dim3(1), dim3(kSmallThreads), 0, s, m, ld, k, Tb, c, work, d, Gk, theta, rho,
                     info);
  DL_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// MinRes-DR cycle end.  Outputs: d (m), Q ((m+1) x (k+1), ld k+1), lam (k),
// S (k x k, ld k), rho (k), hth (k harmonic theta), info.
__global__ void __launch_bounds__(kSmallThreads)
k_minresdr_cycle(int m, int k, double* Tb, double* c, double* work, double* d, double* Q, double* lam,
                 double* S, double* rho, double* hth, double* info) {
  __shared__ double red[kSmallThreads / 64];
  __shared__ int nrot;
  __shared__ double sh_alpha, sh_tau, sh_v0;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m1 = m + 1, k1 = k + 1;
  double4* rot = reinterpret_cast<double4*>(work);  // m/2+1
  double* F = work + 4 * (m / 2 + 1);    // (m+1) x m : full Tbar
  double* R = F + (long)m1 * m;          // (m+1) x m : Householder QR in place
  double* A = R + (long)m1 * m;          // m x m
  double* Z = A + (long)m * m;           // m x m
  double* W = Z + (long)m * m;           // m x m
  double* tau = W + (long)m * m;         // m
  double* vh = tau + m;                  // m   (head element of each reflector)
  double* e = vh + m;                    // m+1
  double* s = e + m1;                    // m+1
  double* q = s + m1;                    // m+1
  double* key = q + m1;                  // m
  int* perm = reinterpret_cast<int*>(key + m);        // m ints (m doubles reserved)

  // 1. full Tbar from its lower triangle; anorm = ||T_m||_inf
  for (long t = tid; t < (long)m1 * m; t += nt) {
    const int i = t / m, j = t % m;
    const double v = (i >= j || i == m) ? Tb[(long)i * m + j] : Tb[(long)j * m + i];
    F[t] = v;
    R[t] = v;
  }
  __syncthreads();
  double rs = 0.0;
  for (int i = tid; i < m; i += nt) {
    double a = 0.0;
    for (int j = 0; j < m; ++j) a += fabs(F[(long)i * m + j]);
    rs = fmax(rs, a);
  }
  const double anorm = blk_reduce(rs, red, true);

  // 2. Householder QR: H_j = I - tau_j v_j v_j^T, v_j = (v0, R[j+1..m][j])
  for (int j = 0; j < m; ++j) {
    double ss = 0.0;
    for (int i = j + 1 + tid; i <= m; i += nt) ss += R[(long)i * m + j] * R[(long)i * m + j];
    ss = blk_reduce(ss, red, false);
    if (tid == 0) {
      const double x0 = R[(long)j * m + j];
      const double nrm = sqrt(ss + x0 * x0);
      if (nrm == 0.0) {
        sh_alpha = 0.0; sh_tau = 0.0; sh_v0 = 1.0;
      } else {
        const double alpha = x0 >= 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        sh_alpha = alpha; sh_v0 = v0;
        sh_tau = 2.0 / (v0 * v0 + ss);
      }
      tau[j] = sh_tau;
      vh[j] = sh_v0;
    }
    __syncthreads();
    const double tj = sh_tau, v0 = sh_v0;
    for (int l = j + 1 + tid; l < m; l += nt) {
      double w = v0 * R[(long)j * m + l];
      for (int i = j + 1; i <= m; ++i) w += R[(long)i * m + j] * R[(long)i * m + l];
      w *= tj;
      R[(long)j * m + l] -= w * v0;
      for (int i = j + 1; i <= m; ++i) R[(long)i * m + l] -= w * R[(long)i * m + j];
    }
    __syncthreads();
    if (tid == 0) R[(long)j * m + j] = sh_alpha;
    __syncthreads();
  }
  // 3. e = Q_R^T c
  for (int i = tid; i <= m; i += nt) e[i] = c[i];
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    double w = 0.0;
    for (int i = j + 1 + tid; i <= m; i += nt) w += R[(long)i * m + j] * e[i];
    w = blk_reduce(w, red, false);
    const double ej = e[j];
    __syncthreads();
    w = tau[j] * (w + vh[j] * ej);
    if (tid == 0) e[j] -= w * vh[j];
    for (int i = j + 1 + tid; i <= m; i += nt) e[i] -= w * R[(long)i * m + j];
    __syncthreads();
  }
  // 4. d = R^-1 e[0..m-1] (column-oriented back substitution)
  for (int j = m - 1; j >= 0; --j) {
    if (tid == 0) d[j] = e[j] / R[(long)j * m + j];
    __syncthreads();
    const double dj = d[j];
    for (int i = tid; i < j; i += nt) e[i] -= R[(long)i * m + j] * dj;
    __syncthreads();
  }
  // 5. s = c - Tbar d
  for (int i = tid; i <= m; i += nt) {
    double a = c[i];
    for (int j = 0; j < m; ++j) a -= F[(long)i * m + j] * d[j];
    s[i] = a;
  }
  // 6. q = Q_R e_m
  for (int i = tid; i <= m; i += nt) q[i] = (i == m) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = m - 1; j >= 0; --j) {
    double w = 0.0;
    for (int i = j + 1 + tid; i <= m; i += nt) w += R[(long)i * m + j] * q[i];
    w = blk_reduce(w, red, false);
    const double qj = q[j];
    __syncthreads();
    w = tau[j] * (w + vh[j] * qj);
    if (tid == 0) q[j] -= w * vh[j];
    for (int i = j + 1 + tid; i <= m; i += nt) q[i] -= w * R[(long)i * m + j];
    __syncthreads();
  }
  // 7. S = R^-T T_m R^-1 (R: upper m x m part of the QR)
  for (int i = tid; i < m; i += nt) {  // W row i: W R = T_m
    for (int j = 0; j < m; ++j) {
      double a = F[(long)i * m + j];
      for (int l = 0; l < j; ++l) a -= W[(long)i * m + l] * R[(long)l * m + j];
      W[(long)i * m + j] = a / R[(long)j * m + j];
    }
  }
  __syncthreads();
  for (int j = tid; j < m; j += nt) {  // A column j: R^T A = W
    for (int i = 0; i < m; ++i) {
      double a = W[(long)i * m + j];
      for (int l = 0; l < i; ++l) a -= R[(long)l * m + i] * A[(long)l * m + j];
      A[(long)i * m + j] = a / R[(long)i * m + i];
    }
  }
  __syncthreads();
  for (int t = tid; t < m * m; t += nt) {
    const int i = t / m, j = t % m;
    if (i < j) {
      const double a = 0.5 * (A[(long)i * m + j] + A[(long)j * m + i]);
      A[(long)i * m + j] = a;
      A[(long)j * m + i] = a;
    }
  }
  __syncthreads();
  // 8. harmonic Ritz: eig(A) -> mu, y ; theta = 1/mu
  jacobi_eigh(m, A, m, Z, m, rot, red, &nrot);
  // 9. keep the k smallest |theta| (ties: theta ascending, then index)
  for (int i = tid; i < m; i += nt) {
    const double mu = A[(long)i * m + i];
    key[i] = (mu != 0.0) ? 1.0 / mu : INFINITY;
  }
  __syncthreads();
  for (int i = tid; i < m; i += nt) {
    const double ki = key[i], ai = fabs(ki);
    int r = 0;
    for (int j = 0; j < m; ++j) {
      const double kj = key[j], aj = fabs(kj);
      r += (aj < ai) || (aj == ai && (kj < ki || (kj == ki && j < i)));
    }
    perm[r] = i;
  }
  __syncthreads();
  // 10. g_l = R^-1 y_l into Q[:, l] (row m zero); Q[:, k] = q
  for (int l = tid; l < k; l += nt) {
    const int col = perm[l];
    for (int i = m - 1; i >= 0; --i) {
      double a = Z[(long)i * m + col];
      for (int j = i + 1; j < m; ++j) a -= R[(long)i * m + j] * Q[(long)j * k1 + l];
      Q[(long)i * k1 + l] = a / R[(long)i * m + i];
    }
    Q[(long)m * k1 + l] = 0.0;
    hth[l] = key[col];
  }
  for (int i = tid; i <= m; i += nt) Q[(long)i * k1 + k] = q[i];
  __syncthreads();
  // 11. orthonormalise the k+1 columns (classical Gram-Schmidt, twice)
  double* h = W;  // k+1 coefficients
  for (int j = 0; j <= k; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = tid; i < j; i += nt) {
        double a = 0.0;
        for (int r = 0; r <= m; ++r) a += Q[(long)r * k1 + i] * Q[(long)r * k1 + j];
        h[i] = a;
      }
      __syncthreads();
      for (int r = tid; r <= m; r += nt) {
        double a = Q[(long)r * k1 + j];
        for (int i = 0; i < j; ++i) a -= h[i] * Q[(long)r * k1 + i];
        Q[(long)r * k1 + j] = a;
      }
      __syncthreads();
    }
    double nn = 0.0;
    for (int r = tid; r <= m; r += nt) nn += Q[(long)r * k1 + j] * Q[(long)r * k1 + j];
    nn = blk_reduce(nn, red, false);
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int r = tid; r <= m; r += nt) Q[(long)r * k1 + j] *= inv;
    __syncthreads();
  }
  // 12. X = Tbar Q[:m, :k] ((m+1) x k in W), Tn = Q^T X ((k+1) x k in A, ld k)
  for (long t = tid; t < (long)m1 * k; t += nt) {
    const int i = t / k, l = t % k;
    double a = 0.0;
    for (int j = 0; j < m; ++j) a += F[(long)i * m + j] * Q[(long)j * k1 + l];
    W[t] = a;
  }
  __syncthreads();
  for (long t = tid; t < (long)k1 * k; t += nt) {
    const int a_ = t / k, l = t % k;
    double a = 0.0;
    for (int i = 0; i <= m; ++i) a += Q[(long)i * k1 + a_] * W[(long)i * k + l];
    A[t] = a;
  }
  // 13. cn = Q^T s (into e)
  for (int a_ = tid; a_ <= k; a_ += nt) {
    double a = 0.0;
    for (int i = 0; i <= m; ++i) a += Q[(long)i * k1 + a_] * s[i];
    e[a_] = a;
  }
  __syncthreads();
  // 14. Rayleigh-Ritz in span V_k: H = sym(Tn[:k,:k]) = S diag(lam) S^T; rho = |Tn[k,:] S|
  for (int t = tid; t < k * k; t += nt) {
    const int i = t / k, j = t % k;
    W[t] = 0.5 * (A[(long)i * k + j] + A[(long)j * k + i]);
  }
  __syncthreads();
  jacobi_eigh(k, W, k, Z, k, rot, red, &nrot);
  for (int i = tid; i < k; i += nt) key[i] = W[(long)i * k + i];
  __syncthreads();
  rank_sort(k, key, perm);
  for (int t = tid; t < k * k; t += nt) {
    const int i = t / k, l = t % k;
    S[t] = Z[(long)i * k + perm[l]];
  }
  for (int l = tid; l < k; l += nt) {
    lam[l] = key[perm[l]];
    double a = 0.0;
    for (int i = 0; i < k; ++i) a += A[(long)k * k + i] * Z[(long)i * k + perm[l]];
    rho[l] = fabs(a);
  }
  __syncthreads();
  // 15. next cycle: Tbar <- Tn (rows 0..k), c <- Q^T s
  for (long t = tid; t < (long)m1 * m; t += nt) Tb[t] = 0.0;
  for (int i = tid; i <= m; i += nt) c[i] = 0.0;
  __syncthreads();
  for (long t = tid; t < (long)k1 * k; t += nt) {
    const int i = t / k, j = t % k;
    Tb[(long)i * m + j] = A[t];
  }
  for (int i = tid; i <= k; i += nt) c[i] = e[i];
  if (tid == 0) {
    double sn = 0.0;
    for (int i = 0; i <= m; ++i) sn += s[i] * s[i];
    info[0] = anorm;
    info[1] = F[(long)m * m + (m - 1)];
    info[2] = sqrt(sn);
    info[3] = (double)nrot;
  }
}

size_t minresdr_work(int m) {
  return 2 * (size_t)(m + 1) * m + 3 * (size_t)m * m + 2 * (size_t)m + 3 * (size_t)(m + 1) + 2 * (size_t)m +
         4 * (size_t)(m / 2 + 1) + 16;
}

void minresdr_cycle(hipStream_t s, int m, int k, double* Tb, double* c, double* work, double* d, double* Q,
                    double* lam, double* S, double* rho, double* hth, double* info) {
  hipLaunchKernelGGL(k_minresdr_cycle, dim3(1), dim3(kSmallThreads), 0, s, m, k, Tb, c, work, d, Q, lam, S, rho,
                     hth, info);
  DL_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Projection matrix setup: Hc = complex k x k (interleaved, Hc[i*k+j] = <y_i, A y_j>)
// -> real embedding E (2k x 2k) -> Z (2k x 2k), lamr (2k).
__global__ void __launch_bounds__(kSmallThreads)
k_proj_setup(int k, const double2* Hc, double* E, double* Z, double* lamr, double* work) {
  __shared__ double red[kSmallThreads / 64];
  __shared__ int nrot;
  const int n = 2 * k;
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int i = t / k, j = t % k;
    const double2 a = Hc[(long)i * k + j], b = Hc[(long)j * k + i];
    const double hr = 0.5 * (a.x + b.x), hi = 0.5 * (a.y - b.y);  // Hermitian part
    E[(long)i * n + j] = hr;
    E[(long)(i + k) * n + (j + k)] = hr;
    E[(long)i * n + (j + k)] = -hi;
    E[(long)(i + k) * n + j] = hi;
  }
  __syncthreads();
  jacobi_eigh(n, E, n, Z, n, reinterpret_cast<double4*>(work), red, &nrot);
  for (int i = threadIdx.x; i < n; i += blockDim.x) lamr[i] = E[(long)i * n + i];
}

void proj_setup(hipStream_t s, int k, const double2* Hc, double* E, double* Z, double* lamr, double* work) {
  hipLaunchKernelGGL(k_proj_setup, dim3(1), dim3(kSmallThreads), 0, s, k, Hc, E, Z, lamr, work);
  DL_HIP(hipGetLastError());
}

// d = H^-1 c for nrhs right-hand sides (c, d: [nrhs][k] complex); one block per rhs.
__global__ void __launch_bounds__(256)
k_proj_solve(int k, const double* Z, const double* lamr, const double2* c, double2* d) {
  extern __shared__ double sm[];
  const int n = 2 * k;
  const double2* cr = c + (long)blockIdx.x * k;
  double2* dr = d + (long)blockIdx.x * k;
  double* u = sm;  // n
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double a = 0.0;
    for (int r = 0; r < n; ++r) {
      const double2 cv = cr[r % k];
      a += Z[(long)r * n + i] * (r < k ? cv.x : cv.y);
    }
    u[i] = a / lamr[i];
  }
  __syncthreads();
  for (int r = threadIdx.x; r < k; r += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int i = 0; i < n; ++i) {
      re += Z[(long)r * n + i] * u[i];
      im += Z[(long)(r + k) * n + i] * u[i];
    }
    dr[r] = make_double2(re, im);
  }
}

void proj_solve(hipStream_t s, int k, int nrhs, const double* Z, const double* lamr, const double2* c, double2* d) {
  if (k <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_proj_solve, dim3(nrhs), dim3(256), 2 * k * sizeof(double), s, k, Z, lamr, c, d);
  DL_HIP(hipGetLastError());
}

}  // namespace dl
