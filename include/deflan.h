/*
 * deflan.h -- C ABI of libdeflan.so: deflated Hermitian Lanczos solvers for the
 * Wilson-Dirac matrix on one MI355X (gfx950) GPU.
 *
 * Method: A. M. Abdel-Rehim, R. B. Morgan, D. Nicely, W. Wilcox, "Deflated
 * Hermitian Lanczos Methods for Multiple Right-Hand Sides" (arXiv:0901.3163).
 * The abstract states the problem the two solve calls implement: solve a
 * Hermitian system for the first right-hand side while computing eigenvectors
 * of small eigenvalues (Lan-DR for the positive definite form, MinRes-DR for the
 * indefinite form), then project over those eigenvectors for every additional
 * right-hand side (D-CG, D-MinRes).
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice:   dims = {Lx, Ly, Lz, Lt}, each >= 2, periodic in all directions;
 *            site = x + Lx*(y + Ly*(z + Lz*t)), V = Lx*Ly*Lz*Lt sites.
 * Spinor:    interleaved complex128, [V][4 spin][3 colour] (12 complex per site),
 *            i.e. 24 doubles per site.  "N" below is 12*V complex numbers.
 * Links:     interleaved complex128, [V][4 mu][3 row][3 col]; mu = 0..3 is x,y,z,t.
 * Operator:  (M psi)(x) = psi(x) - kappa * sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
 *                          + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *            with the chiral gamma basis, gamma5 = diag(1, 1, -1, -1) on spin.
 *            (The paper names "the Wilson matrix" M without conventions, Section 2.)
 * Memory:    DL_HOST    -- pointers are host memory; the library copies.
 *            DL_DEVICE  -- pointers are device memory on the context's device, in
 *                          the same interleaved host layout (e.g. a torch complex128
 *                          tensor's data_ptr()); the library reads/writes them on
 *                          the context's stream.
 * Ownership: the caller owns every array it passes; handles returned through
 *            an out-pointer belong to the caller and are freed by the matching
 *            *_destroy call.  One context per host thread.
 * Errors:    every int-returning call returns a DL_* status; on a negative
 *            status nothing has been written through out-pointers and
 *            dl_last_error() describes the failure (thread-local).  No C++
 *            exception crosses this boundary.
 */
#ifndef DEFLAN_H
#define DEFLAN_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define DL_OK             0
#define DL_NOT_CONVERGED  1   /* outputs are filled with the best iterate */
#define DL_E_INVALID     -1   /* bad argument (null pointer, size, option) */
#define DL_E_HIP         -2   /* HIP runtime error */
#define DL_E_NOMEM       -3   /* device allocation failed */
#define DL_E_BREAKDOWN   -4   /* Krylov breakdown that could not be resolved */
#define DL_E_NONFINITE   -5   /* NaN / Inf in input or in a reduction */
#define DL_E_MISMATCH    -6   /* eigenvector handle does not belong to this operator */

/* ---- enumerations -------------------------------------------------------- */
/* The Hermitian form the solvers iterate on (Section 2):
 *   DL_MDAGM: M^dag M x = M^dag b -- Lan-DR (first rhs) and D-CG (later rhs);
 *   DL_G5M:   gamma5 M x = gamma5 b -- MinRes-DR (first rhs) and D-MinRes.
 * In both cases the user solves M x = b and the reported residual is
 * ||b - M x|| / ||b||, the paper's "residual norm for convergence of M^-1". */
#define DL_MDAGM 0
#define DL_G5M   1
/* Flag OR'ed into the kind of dl_op_create: the even-odd (Schur complement) form of the same
 * system (not in the paper; the usual production form, one step below the stencil).  With
 * sites split by parity p(x) = (x + y + z + t) mod 2 (every extent even), M x = b is the
 * even-site system Mhat x_e = bhat_e, Mhat = 1 - kappa^2 D_eo D_oe, bhat_e = b_e + kappa D_eo b_o,
 * then x_o = b_o + kappa D_oe x_e (dl_eo_prepare, dl_eo_reconstruct).  Such an operator acts on
 * even half fields, [V/2][4][3] complex128 holding the even sites in increasing site order
 * (half index = site / 2): dl_apply applies Mhat, Mhat^dag, gamma5 Mhat, Mhat^dag Mhat, and the
 * solvers, eigenvector handles and dl_op_size (12 V / 2) work on that system, the Hermitian forms
 * being Mhat^dag Mhat (Lan-DR, D-CG) and gamma5 Mhat (MinRes-DR, D-MinRes; gamma5 Mhat is
 * Hermitian since Mhat^dag = gamma5 Mhat gamma5), and tol is relative to ||bhat_e||.  Not for
 * the network or the multi-lattice batch (DL_E_INVALID). */
#define DL_EVEN_ODD 16

#define DL_FP64 0
#define DL_FP32 1
#define DL_BF16 2

/* Inner method of the one-rhs-at-a-time FP64 path (dl_next_opts.method). */
#define DL_METHOD_DEFAULT 0   /* D-CG (CGLS) for DL_MDAGM, D-MinRes for DL_G5M */
#define DL_METHOD_CG      1   /* CG on the Hermitian form; for DL_G5M that is CG on the indefinite
                                 gamma5 M, the combination Section 3 advises against (Fig. 7) */

#define DL_HOST   0
#define DL_DEVICE 1

/* which operator dl_apply applies */
#define DL_APPLY_M     0
#define DL_APPLY_MDAG  1
#define DL_APPLY_G5M   2
#define DL_APPLY_MDAGM 3

/* Re-orthogonalisation of the Lanczos vectors of the first right-hand side (dl_first_opts.reorth) */
#define DL_REORTH_FULL 0   /* every step: classical Gram-Schmidt against the whole basis (default) */
#define DL_REORTH_KEPT 1   /* the paper's policy (Section 2, last paragraph): each step orthogonalises
                              against the two previous Lanczos vectors, the first step after
                              a restart against the whole basis, and every reorth_period steps the
                              new vector is also orthogonalised against the vectors kept at
                              the last restart.  Reads 2k instead of 2j fields per step (k kept, j the
                              basis size), so it is cheaper for k well below m.
                              In both policies a Gram-Schmidt pass is repeated only when the first
                              removed more than half of the vector's squared norm (the test of
                              Daniel, Gragg, Kaufman and Stewart with eta = 1/sqrt(2), decided on the
                              device): against the kept vectors, nearly never. */

/* stop rules reported in dl_stats.stop_rule for dl_solve_first */
#define DL_STOP_LINEAR     0  /* k = 0: stopped at linear convergence */
#define DL_STOP_EIGEN      1  /* every kept eigen-residual <= eig_tol * ||A||_est */
#define DL_STOP_MVP_FACTOR 2  /* MVPs reached past_conv_factor x MVPs at linear convergence */
#define DL_STOP_MAX_MVP    3  /* MVP cap reached (status DL_NOT_CONVERGED if not converged) */
#define DL_STOP_BREAKDOWN  4  /* invariant subspace found: exact solve */

typedef struct dl_ctx dl_ctx;
typedef struct dl_op  dl_op;
typedef struct dl_eig dl_eig;
typedef struct dl_net dl_net;

/* Options for the first right-hand side.  Pass NULL for the defaults. */
typedef struct {
  double eig_tol;           /* eigen-residual target relative to ||A||_est; default 1e-12 */
  double past_conv_factor;  /* run past linear convergence up to this MVP factor; default 2.0
                               (the paper: "at most a factor of two in MVPs", Section 2) */
  long   max_mvp;           /* hard cap on MVPs; default 1000000 */
  int    reorth;            /* DL_REORTH_FULL (0, default) or DL_REORTH_KEPT */
  int    reorth_period;     /* DL_REORTH_KEPT: steps between orthogonalisations against the kept
                               vectors; 0 = default 1.  On the near-critical 4^4 lattice and the
                               indefinite diagonal example of Section 1 a period of 2 or more
                               already lets the kept eigenvectors lose orthogonality (MinRes-DR)
                               or the recurrence diverge (Lan-DR, period 4), so 1 is the default. */
} dl_first_opts;

/* Options for later right-hand sides.  Pass NULL for the defaults. */
typedef struct {
  int    storage;           /* DL_FP64 (default): plain FP64 D-CG / D-MinRes.
                               DL_FP32 / DL_BF16: low-precision Krylov storage and Dslash,
                               FP32 arithmetic, FP64 reliable updates and FP64 true residual.
                               A BF16 batch whose cycle stalls above its target (modes below
                               what BF16 resolves, e.g. a near-critical field with too little
                               deflation) continues with FP32 storage and FP32 cycle settings. */
  int    reliable_every;    /* batched path: the inner solve restarts from the FP64 residual
                               b - M x64, with a new projection over the eigenvectors, after each
                               inner_drop reduction; within such a cycle D-CG also makes a reliable
                               update every reliable_every iterations (x64 += e, r = b - M x64 in
                               FP64, search direction kept).  0 = default: 8 for D-CG with DL_BF16
                               storage, else 50; < 0 = no reliable updates.  With DL_BF16 a D-CG
                               cycle also ends when its residual has not reached a new low (by
                               10%) for 200 iterations. */
  int    batched;           /* 0: one rhs after another; 1: all rhs advance together through
                               the multi-rhs kernels (links read once per site for all rhs) */
  int    x0_given;          /* 1: X holds initial guesses on entry (default 0: x0 = 0) */
  long   max_mvp;           /* per-rhs MVP cap; default 1000000 */
  dl_net* net;              /* learned initial guess (batched path only; NULL = projection only):
                               x0 = net(b), then the Galerkin projection; per rhs the library keeps
                               whichever of that and the projection-only start has the smaller
                               true residual ||b - M x0|| (costs one extra projection per rhs) */
  int    graph;             /* batched path: 1 = replay each block of 8 inner iterations as a
                               captured HIP graph (fewer launches for small lattices); ignored
                               while kernel timing (dl_timing) is on.  Default 0.  D-MinRes
                               then runs its fused form (see minres_window), which moves more
                               data per iteration: on large lattices graph replay is slower. */
  double inner_drop;        /* batched path: residual reduction that ends an inner cycle (then
                               FP64 residual, projection, restart); 0 = default: 1e-4 with DL_FP32
                               storage; with DL_BF16 (whose rounding limits one cycle) 1e-2 for
                               D-MinRes, and for D-CG (whose reliable updates carry it further;
                               much longer cycles let the deflated modes back) 1e-5 from the
                               projection-only start and 1e-3 with a net (the drops measured
                               fastest for each start on near-critical fields) */
  int    eig_storage;       /* batched path: eigenvectors the Galerkin projection reads.  DL_FP64
                               (0, default): the handle's FP64 basis.  DL_FP32 / DL_BF16: the
                               lowered copies made by dl_eig_lower (DL_E_INVALID if missing):
                               c = Y^H r on the matrix cores against the FP32 / BF16 rounding of
                               Y and r, then x += Y32 H32^-1 c in FP64 over the FP32 rounding Y32
                               (H32 = Y32^H A Y32).  The BF16 contraction leaves about
                               1.6e-3 ||r|| / sqrt(n) in each deflated mode (n complex elements per
                               field), so it suits cycles whose inner_drop is well above
                               1.6e-3 sqrt(k / n): BF16 storage, or FP32 storage on large lattices.
                               DL_BF16 is for the gamma5 M form only (DL_E_INVALID with M^dag M,
                               where the residual sees that error amplified by 1/sigma_min(M)). */
  int    net_prec;          /* learned guess inference: DL_FP32 (default; 0 reads as DL_FP32) or
                               DL_BF16 (as dl_net_apply_prec) */
  int    method;            /* FP64 one-rhs path: DL_METHOD_DEFAULT or DL_METHOD_CG (the Galerkin
                               projection at the start is the same; breakdown p^H A p = 0 ends a
                               cycle, which restarts from the true residual) */
  int    minres_window;     /* batched D-MinRes without graph replay: the Lanczos vectors of a
                               cycle are kept in a ring and every minres_window iterations one
                               pass adds their share of the solution (the iteration's own pass
                               then moves 4 fields instead of 9).  0 = default: 64, halved down
                               to 8 while the ring (minres_window + 2 fields per rhs) exceeds
                               24 GiB; 1..64 = that window; < 0 = the fused short-recurrence
                               form (the form graph replay uses).  > 64: DL_E_INVALID.  Both
                               forms compute the same iterates up to rounding. */
} dl_next_opts;

/* Per-solve statistics. */
typedef struct {
  int    status;            /* DL_OK or DL_NOT_CONVERGED */
  int    stop_rule;         /* DL_STOP_* (solve_first) */
  int    cycles;            /* restart cycles (solve_first) */
  int    guess;             /* solve_next with a network: 1 if the learned start was kept */
  long   mvp;               /* applications of M or M^dag (M^dag M counts 2; gamma5 is free) */
  long   mvp_lin;           /* MVPs when the linear system first met tol (solve_first) */
  long   iters;             /* Krylov iterations */
  double relres;            /* true ||b - M x|| / ||b||, recomputed in FP64 at return */
  double time_s;            /* wall time of the call */
  /* Residual history (the paper's plots of residual norm against MVPs, Figs. 2 and 4-7).
   * INPUT fields, read before the call writes the struct: history points to caller memory of
   * history_cap (mvp, relres) pairs, i.e. 2 * history_cap doubles (host memory), or is NULL
   * (no history; history_cap is then ignored).  Set both to 0 in a fresh struct.  OUTPUT:
   * history_len = pairs written (at most history_cap; later points are dropped).  Points:
   *   dl_solve_first: the true residual at the end of every restart cycle;
   *   dl_solve_next, one rhs at a time (FP64): the residual after the projection, then the
   *     recurrence residual (CG) or |eta| (MinRes) of every iteration, and the true residual
   *     that closes every inner run;
   *   dl_solve_next batched / dl_solve_next_multi: the true residual at the start of every
   *     inner cycle and the inner estimate at every host check (every 8 to 64 iterations).
   * relres is relative to ||b||; mvp counts MVPs of that right-hand side so far. */
  double* history;
  int    history_cap;
  int    history_len;
} dl_stats;

/* ---- library ----------------------------------------------------------- */
/* Message describing the last non-OK status on this thread ("" if none). */
const char* dl_last_error(void);
/* ABI version (major*100 + minor). */
int dl_version(void);

/* ---- context ------------------------------------------------------------ */
/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (NULL: the library creates its own stream).
 * Device memory: the library keeps the device buffers it frees (solver work
 * fields, handles closed) in a per-device cache and reuses them for requests of
 * the same rounded size, holding at most an eighth of the device's memory; a
 * failed allocation releases the cache and retries once. */
int  dl_ctx_create(int device, void* hip_stream, dl_ctx** out);
/* Wait for the context's stream, release the context, and return the device's
 * cached buffers to HIP (buffers of live operators and handles stay theirs). */
void dl_ctx_destroy(dl_ctx* ctx);
/* Block until all work queued by the library on the context's stream is done. */
int  dl_ctx_sync(dl_ctx* ctx);
/* Kernel timing: when enabled, every launch of the kernel families below is
 * bracketed by HIP events on the context's stream and its duration summed.
 * name: "wilson" (every M / M^dag / gamma5 M launch with FP32 or BF16 spinors),
 * "wilson64" (every FP64 launch: the FP64 solvers, and the true residuals and
 * projections of the batched path), "tsk_dots" (V^H w), "tsk_update" (V c / V Y),
 * "small" (one-workgroup FP64 problems).  dl_kernel_time returns launches, total
 * milliseconds and (bytes may be NULL) the algorithmic bytes those launches moved
 * -- for the stencils the input spinors, links and output spinors counted once:
 * 576 + 384 * nrhs B/site in FP64, 288 + 192 * nrhs (FP32 spinors) or 288 + 96 * nrhs
 * (BF16 spinors) B/site with FP32 links, nrhs counting the active rhs of a launch --
 * since the last reset (dl_timing resets). */
int  dl_timing(dl_ctx* ctx, int enable);
int  dl_kernel_time(dl_ctx* ctx, const char* name, long* launches, double* total_ms, double* bytes);

/* ---- operator ----------------------------------------------------------- */
/* Create the operator A of the paper for links U, hopping parameter kappa and
 * Hermitian form `kind` (DL_MDAGM or DL_G5M, optionally | DL_EVEN_ODD).  The links are converted once to
 * the device's site-major tiled layout (FP64, plus FP32/BF16 copies on first
 * use).  Errors: DL_E_INVALID for dims < 2, kappa not finite, unknown kind. */
int  dl_op_create(dl_ctx* ctx, const int dims[4], const double* links, int mem,
                  double kappa, int kind, dl_op** out);
void dl_op_destroy(dl_op* op);
/* Number of complex entries N = 12 V of one spinor. */
long dl_op_size(const dl_op* op);
/* Even-odd operators (DL_EVEN_ODD): bhat ([V/2][4][3]) = b_e + kappa D_eo b_o for a whole-lattice
 * right-hand side b ([V][4][3]), and the whole-lattice solution x from the even-site solution
 * xe: x_e = xe, x_o = b_o + kappa D_oe xe (FP64).  All pointers DL_HOST or all DL_DEVICE;
 * DL_E_INVALID for an operator without DL_EVEN_ODD. */
int  dl_eo_prepare(dl_op* op, const double* b, double* bhat, int mem);
int  dl_eo_reconstruct(dl_op* op, const double* b, const double* xe, double* x, int mem);
/* The operator's fingerprint: a hash of dims, kappa, kind and every link as stored on the
 * device (so the same links give the same value whether they came from host or device
 * memory, and a change of any one link changes it).  Eigenvector handles carry the
 * fingerprint of the operator they were built for (DL_E_MISMATCH elsewhere). */
int  dl_op_fingerprint(const dl_op* op, unsigned long long* out);

/* out = op(in) with op one of DL_APPLY_* (FP64).  in/out are N complex each
 * and may not alias. */
int  dl_apply(dl_op* op, int which, const double* in, double* out, int mem);

/* ---- first right-hand side: Lan-DR(m,k) / MinRes-DR(m,k) --------------- */
/* Solves M x = b through the op's Hermitian form with Lan-DR(m,k) (DL_MDAGM)
 * or MinRes-DR(m,k) (DL_G5M) from x0 = 0, keeping k eigenvectors of smallest
 * eigenvalue (regular Ritz for Lan-DR, harmonic Ritz for MinRes-DR,
 * Section 2), and runs past linear convergence to refine them (Section 2,
 * last paragraph).  On return x holds the solution, *eig_out (if eig_out is
 * not NULL and k > 0) the k eigenpairs, and *stats the counters.
 * Requires 0 <= k < m <= N and tol > 0.  b = 0 gives x = 0 and DL_OK. */
int  dl_solve_first(dl_op* op, const double* b, double* x, int mem, int m, int k,
                    double tol, const dl_first_opts* opts, dl_eig** eig_out,
                    dl_stats* stats);

/* ---- later right-hand sides: D-CG / D-MinRes ----------------------------- */
/* Solves M X[i] = B[i] for i < nrhs (B, X: [nrhs][V][4][3] complex128) by a
 * Galerkin projection over the eigenvectors of `eig` at the beginning
 * (Section 2), then CG on the normal equations (DL_MDAGM) or MinRes on
 * gamma5 M (DL_G5M) until ||b - M x||/||b|| <= tol.  eig may be NULL (no
 * deflation: plain CG / MinRes).  stats, if not NULL, has nrhs entries.
 * nrhs = 0 is a no-op.  DL_E_MISMATCH if eig was built for another operator. */
int  dl_solve_next(dl_op* op, const dl_eig* eig, int nrhs, const double* B,
                   double* X, int mem, double tol, const dl_next_opts* opts,
                   dl_stats* stats);

/* Measurement: average duration (ms) of one launch of the Wilson stencil
 * `which` (DL_APPLY_M, _MDAG or _G5M) in precision `prec` (DL_FP64 / DL_FP32)
 * applied to nrhs zero-filled device fields at once, over `reps` back-to-back
 * launches timed with HIP events; *bytes (may be NULL) receives the
 * algorithmic bytes of one launch (links once, each input and output spinor
 * once).  Allocates and frees its own fields. */
int  dl_bench_wilson(dl_op* op, int which, int prec, int nrhs, int reps, double* avg_ms, double* bytes);

/* Measurement: average duration (ms) of the library's streaming copy kernel moving `bytes`
 * bytes (rounded down to 16-byte elements) between two device buffers, over `reps`
 * event-timed launches (each moves 2 * bytes through HBM: one read, one write): the practical
 * bandwidth ceiling the stencil is compared with.  Allocates and frees its own buffers. */
int  dl_bench_copy(dl_ctx* ctx, long bytes, int reps, double* avg_ms);

/* Autotuner: time every launch shape of the Wilson stencil (threads per block,
 * occupancy hint, block order) for this operator's lattice in precision `prec`
 * with `nrhs` right-hand sides (reps event-timed launches each), keep the
 * fastest for the process and append it to the tuning cache file
 * ($DEFLAN_TUNE_CACHE, else $HOME/.cache/deflan/tune.txt).  Without an explicit
 * call the library tunes on first use (DEFLAN_AUTOTUNE=0: default shape).
 * variant / order / best_us (may be NULL) receive the choice and its time. */
int  dl_tune_wilson(dl_op* op, int prec, int nrhs, int reps, int* variant, int* order, double* best_us);

/* Contraction kinds of dl_tune_tsk. */
#define DL_TSK_DOTS64   0  /* C = V^H W, FP64 basis and columns (nv <= 64, nw <= 16)            */
#define DL_TSK_DOTS32   1  /* C = V^H W on the matrix cores, FP32 storage (nv <= 128, nw <= 16)  */
#define DL_TSK_DOTS16   2  /* the same with BF16 storage                                         */
#define DL_TSK_UPD64    3  /* X += V D, FP64 basis (nv <= 512, nw <= 16)                         */
#define DL_TSK_UPD32    4  /* X += V D, FP32 basis, FP64 products                                */
#define DL_TSK_COMBINE  5  /* Y = V G, G real nv x nw (the basis rebuild; nv, nw <= 512)         */

/* Autotuner of the tall-skinny contractions (the Galerkin projection c = V^H r and x += V d over
 * the eigenvectors, the re-orthogonalisation, and the basis rebuild Y = V G at a thick restart,
 * section 2): time every launch shape of contraction `kind` for fields of n complex numbers, nv
 * basis vectors and nw columns (outputs) -- grid size; for the matrix-core dots also 2, 4 or 8
 * tiles of 16 basis vectors per launch; for the rebuild 8 or 16 outputs per block and blocks
 * grouped per XCD -- with reps event-timed launches each on zero-filled device buffers the call
 * allocates, keep the fastest for the process and append it to the tuning cache file.  Without
 * an explicit call each shape is tuned on first use of its key (never inside graph capture;
 * DEFLAN_AUTOTUNE=0: the default shape).  The update and the rebuild give the same bits in every
 * shape; the dots' FP64 partial sums follow the grid, so their last bits do.  grid / tile /
 * best_us (may be NULL) receive the choice and its time in microseconds. */
int  dl_tune_tsk(dl_ctx* ctx, int kind, long n, int nv, int nw, int reps, int* grid, int* tile, double* best_us);

/* One operator's share of a multi-lattice batch. */
typedef struct {
  dl_op*        op;         /* operator (all items: the same context and the same kind) */
  const dl_eig* eig;        /* eigenvectors of op for the Galerkin projection, or NULL */
  int           nrhs;       /* right-hand sides of this item (0: the item is skipped) */
  const double* B;          /* [nrhs][V][4][3] complex128 right-hand sides */
  double*       X;          /* [nrhs][V][4][3] complex128 solutions (initial guesses if x0_given) */
  double        tol;        /* relative true-residual target of this item's rhs */
} dl_batch_item;

/* Later right-hand sides of several operators (lattices of different sizes) solved
 * together by the batched mixed-precision path (D-CG or D-MinRes as in dl_solve_next,
 * Section 2): every vector stage is one launch over all lattices and rhs, with per-rhs
 * scalars and convergence masks.  The stencil stage is either one work-list launch over all
 * lattices or one launch per lattice in its tuned shape; the library times both when it sets
 * the batch up and keeps the faster (the environment variable DEFLAN_MULTI_STENCIL =
 * "list" or "lattice" forces one).  opts NULL: DL_FP32 storage, batched; a non-NULL opts must
 * ask for DL_FP32 or DL_BF16 storage and batched = 1, and no network; the operators are
 * whole-lattice ones (no DL_EVEN_ODD).  stats (may be NULL) gets one entry per rhs in item
 * order.  All pointers of all items are host (DL_HOST) or all device (DL_DEVICE).  Returns
 * DL_NOT_CONVERGED if any rhs missed its tol. */
int  dl_solve_next_multi(dl_ctx* ctx, int nitems, const dl_batch_item* items, int mem,
                         const dl_next_opts* opts, dl_stats* stats);

/* out_j = op(in_j) for nrhs fields ([nrhs][V][4][3] complex128), op = M, M^dag or gamma5 M
 * (which = DL_APPLY_M, DL_APPLY_MDAG, DL_APPLY_G5M), by the multi-rhs stencil of the batched
 * solver: links read once per site for all fields.  prec DL_FP32 rounds the input and the
 * links to FP32, computes in FP32 and widens the result.  The launch shape is the tuned one
 * (the environment variable DEFLAN_WILSON_VARIANT = "v" or "v,o" forces one). */
int  dl_apply_batched(dl_op* op, int which, int prec, int nrhs, const double* in, double* out, int mem);

/* ---- eigenvector handle ---------------------------------------------------- */
/* Build a handle from k caller-supplied orthonormal vectors V ([k][V][4][3]);
 * H = V^H A V is formed with k MVPs in FP64. */
int  dl_eig_create(dl_op* op, int k, const double* V, int mem, dl_eig** out);
/* k, the eigenvalues (Rayleigh quotients of A) and eigen-residual norms. */
int  dl_eig_info(const dl_eig* eig, int* k, double* evals, double* resid);
/* Copy the k eigenvectors out ([k][V][4][3] complex128). */
int  dl_eig_vectors(const dl_eig* eig, double* V, int mem);
/* Lowered copies of the eigenvectors for the batched projection (Section 2's Galerkin
 * projection over a rounded basis; dl_next_opts.eig_storage selects them).  prec DL_FP32:
 * Y32 = fp32(Y) and H32 = Y32^H A Y32 (k MVPs in FP64 on the widened Y32) -- Y32 is the
 * projection basis.  DL_BF16: also Y16 = bf16(Y), read (with a BF16 rounding of the
 * residual) by the contraction c = Y^H r, 4 bytes per complex instead of 8; the correction
 * stays on Y32, since a basis rounded to BF16 no longer spans the near-null modes of a
 * near-critical A to the accuracy deflation needs (eps_bf16^2 ||A|| exceeds the smallest
 * eigenvalues).  A handle lowered to DL_BF16 serves eig_storage DL_FP32 as well; lowering it
 * to DL_FP32 releases Y16.  DL_FP64 releases the copies.  The FP64 basis is kept (dl_eig_vectors and
 * the FP64 paths still use it).  eig must belong to op (DL_E_MISMATCH).  *mvp (may be NULL)
 * receives the MVPs used. */
int  dl_eig_lower(dl_op* op, dl_eig* eig, int prec, long* mvp);
void dl_eig_destroy(dl_eig* eig);
/* Checkpoint of a handle (the point of the method, abstract: eigenvectors computed with the
 * first right-hand side serve every later one, also in a later process).  dl_eig_save writes
 * the k FP64 eigenvectors (interleaved complex128, [k][V][4][3]), the eigenvalues, residual
 * norms, the eigendecomposition of H = Y^H A Y that the projection uses, and the operator's
 * fingerprint, dims, kappa and kind, to the file `path` (created or truncated; about
 * 16 * 12 * V * k bytes).  dl_eig_load reads such a file for op: DL_E_MISMATCH if it was saved
 * for another operator (dims, kappa, kind or links differ), DL_E_INVALID if it is not a
 * complete handle file.  The loaded handle equals the saved one bit for bit (a solve with it
 * gives the same iterates); its lowered copies (dl_eig_lower) are not saved.  No MVPs. */
int  dl_eig_save(const dl_eig* eig, const char* path);
int  dl_eig_load(dl_op* op, const char* path, dl_eig** out);

/* ---- learned initial guess ---------------------------------------------------
 * Not part of the paper's method: an optional starting vector for the later
 * right-hand sides, refined by the paper's Galerkin projection (Section 2) and
 * Krylov solve.  A gauge-covariant parallel-transport convolution network in FP32:
 * features are colour triplets per site and channel (the spinor b is 4 channels,
 * one per spin); layer l maps
 *     out[o](x) = sum_h sum_i W_h[o][i] (T_h in[i])(x),
 * h over {0, +x, -x, +y, -y, +z, -z, +t, -t}, T_0 = 1, (T_{+mu} a)(x) = U_mu(x) a(x+mu),
 * (T_{-mu} a)(x) = U_mu(x-mu)^dag a(x-mu); widths 4 -> 16 -> 16 -> 4 with
 * f(z) = z / sqrt(1 + |z|^2) (colour norm per site and channel) after layers 1 and 2.
 * net(b) = s N(b / s) with s the root-mean-square site norm of b over the sites where b is
 * nonzero (||b|| / sqrt(V) for a source without zeros, |b(x0)| for a point source).
 * Weights: complex128 interleaved, layers concatenated, each [9 hops][C_out][C_in]
 * in the hop order above; dl_net_num_weights() complex numbers in all.
 * A network belongs to one context; its scratch grows to the largest batch used. */
int  dl_net_num_weights(void);
/* Create a network with the given weights (host, rounded to FP32). */
int  dl_net_create(dl_ctx* ctx, const double* weights, dl_net** out);
/* Copy the current weights out (host, complex128). */
int  dl_net_get_weights(const dl_net* net, double* weights);
/* Replace the weights (host) and reset the optimiser state. */
int  dl_net_set_weights(dl_net* net, const double* weights);
void dl_net_destroy(dl_net* net);
/* Y = net(B) for nrhs fields B ([nrhs][V][4][3] complex128) on op's lattice and links. */
int  dl_net_apply(dl_net* net, dl_op* op, int nrhs, const double* B, double* Y, int mem);
/* The same with prec DL_FP32 (as dl_net_apply) or DL_BF16: the 16 -> 16 layer's channel mixing
 * with its transported inputs and weights rounded to BF16 on the matrix cores (FP32
 * accumulation; transports, the other layers and the non-linearity stay FP32).  Inference
 * only: training uses the FP32 forward pass. */
int  dl_net_apply_prec(dl_net* net, dl_op* op, int prec, int nrhs, const double* B, double* Y, int mem);
/* loss = (1/n) sum_j ||M (net(b_j) - x_j)||^2 / ||b_j||^2 over n pairs (B, X), with M in FP32;
 * grad (host complex128, may be NULL) = dloss/dRe W + i dloss/dIm W.  b_j = 0 is invalid. */
int  dl_net_loss_grad(dl_net* net, dl_op* op, int n, const double* B, const double* X, int mem,
                      double* loss, double* grad);
/* Train on the error the D-CG start leaves (eig != NULL) or on the raw error (eig = NULL, the
 * default).  With eig, every later dl_net_loss_grad / dl_net_train on eig's operator replaces
 * d = net(b_j) - x_j by d' = d - Y H^-1 Y^H M^dag M d (Y the eigenvectors of eig, H = Y^H M^dag M Y):
 * the error left after the Galerkin projection that follows the guess (Section 2), in the norm
 * CG minimises, instead of the raw error, much of which the projection removes anyway.  eig must
 * be a DL_MDAGM handle of this context, must outlive those calls, and must belong to the operator
 * they are given (DL_E_MISMATCH otherwise); call again with the next field's handle when training
 * moves to another gauge field. */
int  dl_net_set_projection(dl_net* net, const dl_eig* eig);
/* `steps` Adam steps (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the same loss; step s uses
 * the pairs [g*batch, (g+1)*batch) with g = s mod (n / batch).  losses ([steps], host, may
 * be NULL) receives each step's minibatch loss before the update.  1 <= batch <= n. */
int  dl_net_train(dl_net* net, dl_op* op, int n, const double* B, const double* X, int mem,
                  int batch, int steps, double lr, double* losses);

/* ---- kernel-level entry points (used by the parity tests) --------------- */
/* c = V^H w for nv vectors V ([nv][N]) and one vector w ([N]); c: nv complex.
 * Then, if `subtract`, w <- w - V c in place.  All pointers DL_HOST or DL_DEVICE. */
int  dl_tsk_project(dl_ctx* ctx, long n, int nv, const double* V, double* w,
                    double* c, int subtract, int mem);
/* The same projection for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): V, w and c are DEVICE
 * pointers on ctx's device (layouts as dl_tsk_project), and the call allocates nothing -- the
 * reduction partials live in a fixed array of the library that every GPU it runs on holds for
 * the life of the process (8 MiB).  Limit: 2 * nv * ceil(n / 2048) <= 1048576 (every nv <= 512
 * up to n = 2^21, nv <= 134 at n = 7962624); larger sizes return DL_E_INVALID.  The array is
 * shared by every call on that GPU: calls that overlap on one GPU (several threads or streams
 * at once) race and give wrong results.  Results equal dl_tsk_project's bit for bit. */
int  dl_tsk_project_noalloc(dl_ctx* ctx, long n, int nv, const double* V, double* w, double* c, int subtract);
/* Several columns at once (the batched deflation projection): C[r][j] = <V_j, W_r> for nv
 * vectors V ([nv][n] complex) and nw <= 16 columns W ([nw][n]); C: [nw][nv] complex.  If X
 * ([nw][n]) is not NULL, then X_r += sum_j C[r][j] V_j.  V streams once for all columns. */
int  dl_tsk_project_multi(dl_ctx* ctx, long n, int nv, const double* V, int nw, const double* W,
                          double* C, double* X, int mem);
/* The matrix-core contraction of dl_next_opts.eig_storage: C[r][j] = <q(V_j), q(W_r)> for
 * nv <= 512 vectors V ([nv][n] complex128) and nw <= 16 columns W ([nw][n]), q = rounding to
 * prec (DL_FP32 or DL_BF16, nearest even; BF16 via FP32) done on the device; FP32 matrix-core
 * products and block sums, FP64 partial sums; C: [nw][nv] complex128.  If X ([nw][n]) is not
 * NULL, X_r += sum_j C[r][j] fp32(V_j) in FP64 (the update basis of the lowered projection).
 * All pointers DL_HOST or DL_DEVICE. */
int  dl_tsk_project_lowp(dl_ctx* ctx, int prec, long n, int nv, const double* V, int nw,
                         const double* W, double* C, double* X, int mem);
/* Y = V G for V ([nv][n] complex) and real G ([nv][ny], row-major); Y: [ny][n]. */
int  dl_tsk_combine(dl_ctx* ctx, long n, int nv, const double* V, const double* G,
                    int ny, double* Y, int mem);
/* Eigen-decomposition of a real symmetric n x n matrix A (row-major, host) by
 * the device's one-workgroup Jacobi solver: evals ascending, Z[i][j] = j-th
 * eigenvector's i-th entry. n <= 512. */
int  dl_small_eigh(dl_ctx* ctx, int n, const double* A, double* evals, double* Z);

#ifdef __cplusplus
}
#endif
#endif /* DEFLAN_H */
