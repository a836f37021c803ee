// Operator, eigenvector-handle and solver declarations of libdeflan.
#pragma once
#include <map>
#include <vector>

#include "internal.hpp"

struct dl_op {
  dl_ctx* ctx = nullptr;
  dl::Lattice lat{};
  double kappa = 0.0;
  int kind = DL_MDAGM;
  dl::DBuf<double2> U;          // FP64 links, tiled
  dl::DBuf<float2> U32;         // FP32 links, tiled (made on first use)
  uint64_t fingerprint = 0;     // dims, kappa, kind and a hash of the links
  std::map<int, dl::WilsonCfg> wcfg;  // tuned stencil launch shape per (precision, batch size)
};

struct dl_eig {
  dl_ctx* ctx = nullptr;
  dl::Lattice lat{};
  uint64_t fingerprint = 0;
  double kappa = 0.0;
  int kind = 0;
  int k = 0;
  long nc = 0;
  dl::DBuf<double2> Y;          // k tiled fields, contiguous (stride nc)
  dl::DBuf<double> Zr, lamr;    // eigendecomposition of the real embedding of H = Y^H A Y
  std::vector<double> evals;    // Rayleigh quotients y_i^H A y_i
  std::vector<double> resid;    // ||A y_i - lambda_i y_i||
  // Lowered copies for the batched projection (lo_prec = DL_FP32 or DL_BF16 once built): the
  // FP32 rounding Y32 is the Galerkin basis (x += Y32 H32^-1 c, with H32 = Y32^H A Y32 built in
  // FP64); c = Y^H r is contracted against Y32 (DL_FP32) or against the BF16 rounding Y16.
  int lo_prec = DL_FP64;
  dl::DBuf<float2> Y32;
  dl::DBuf<dl::bf2> Y16;
  dl::DBuf<double> Zr32, lamr32;
};

namespace dl {

bool verbose();  // DEFLAN_VERBOSE set: progress lines on stderr

// Residual history requested by the caller (dl_stats.history): per right-hand side, the
// (mvp, relres) points appended in order, at most cap[r] of them.
struct History {
  std::vector<int> cap;
  std::vector<std::vector<double>> pts;
  explicit History(int nrhs = 0) : cap(nrhs, 0), pts(nrhs) {}
  bool want(int r) const { return r >= 0 && r < (int)cap.size() && cap[r] > 0; }
  bool any() const {
    for (int c : cap) if (c > 0) return true;
    return false;
  }
  void add(int r, double mvp, double relres) {
    if (!want(r) || (long)pts[r].size() >= 2L * cap[r]) return;
    pts[r].push_back(mvp);
    pts[r].push_back(relres);
  }
};

// Scratch owned by one solve: device scalars, reduction partials, small work.
struct Scratch {
  DBuf<double> sc;     // 256 device scalars
  DBuf<double> part;   // reduction partials
  size_t part_n = 0;
  void ensure_part(size_t n) {
    if (n > part_n) { part.alloc(n); part_n = n; }
  }
};

// out = A in for the operator's Hermitian form (tmp: one field for M^dag M).
// Returns MVPs used.
int apply_A(dl_op* op, const double2* in, double2* out, double2* tmp);
// out = M in (which: 0 M, 1 M^dag, 2 gamma5 M), timed as "wilson"; returns the partial count
// per rhs of a fused reduction (0 if red == 0).
int apply_wilson(dl_op* op, int which, const double2* in, double2* out, int red = 0, double* part = nullptr);

// Stencil launch shape for (precision, batch size): the tuned choice (tuning on first use
// unless DEFLAN_AUTOTUNE=0), and the explicit tuner.
WilsonCfg wilson_cfg(dl_op* op, int prec, int nrhs);
WilsonCfg tune_wilson(dl_op* op, int prec, int nrhs, int reps, double* best_us);
bool autotune_enabled();  // false when DEFLAN_AUTOTUNE=0

// hist (may be nullptr): residual history of the solve's right-hand sides.
int solve_first(dl_op* op, const double2* b, double2* x, int m, int k, double tol, const dl_first_opts& o,
                dl_eig** eig_out, dl_stats* st, History* hist = nullptr);
int solve_next(dl_op* op, const dl_eig* eig, int nrhs, const double2* B, double2* X, double tol,
               const dl_next_opts& o, dl_stats* st, History* hist = nullptr);
int solve_next_batched(dl_op* op, const dl_eig* eig, int nrhs, const double2* B, double2* X, double tol,
                       const dl_next_opts& o, dl_stats* st, History* hist = nullptr);
// Several operators (lattices) in one batch: item i's fields are contiguous after item i-1's.
struct MultiItem {
  dl_op* op;
  const dl_eig* eig;
  int nrhs;
  double tol;
};
int solve_next_multi(const std::vector<MultiItem>& items, const double2* B, double2* X, const dl_next_opts& o,
                     dl_stats* st, History* hist = nullptr);
dl_eig* eig_build(dl_op* op, int k, DBuf<double2>&& Y, long* mvp);
// Build the lowered copies of eig for prec (DL_FP32 or DL_BF16); k MVPs for H32 (once: a second
// call with the same prec does nothing, DL_FP64 drops the copies).  Returns MVPs used.
long eig_lower(dl_op* op, dl_eig* eig, int prec);
const float2* op_links32_public(dl_op* op);  // FP32 links of the operator (made on first use)

}  // namespace dl
