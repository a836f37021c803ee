// Launchers of the tall-skinny basis contractions (tsk.hip).
#pragma once
#include <functional>
#include <vector>

#include "internal.hpp"

namespace dl {

// Launch shapes of the contractions, chosen by the autotuner per (architecture, kind, n, nv,
// nw).  grid: blocks (dots: at most the default count, so partial buffers sized by the
// *_nblocks functions hold them); tile: kind-specific (matrix-core dots: row tiles of 16 basis
// vectors per launch, 2, 4 or 8; rebuild: outputs per block 8 or 16 (bit 1) and blocks grouped
// per XCD (bit 0); others 0).  Every shape of the update and the rebuild gives the same bits;
// the dots' partial sums follow the grid, so their rounding does.
enum TskKind { TK_DOTS64 = 0, TK_DOTS32, TK_DOTS16, TK_UPD64, TK_UPD32, TK_COMBINE, TK_COUNT };
struct TskCfg {
  int grid = 0;
  int tile = 0;
};
// The shape for a key: DEFLAN_TSK_SHAPE (grid,tile or grid,tile,kind) when set, else the remembered choice, else (outside
// graph capture, unless DEFLAN_AUTOTUNE=0) the fastest of cands timed through launch (reps
// event-timed launches each after a warm-up; cands[0] is the default).  reps > 0 forces the
// timing and replaces a remembered choice.  launch must leave the caller's results unchanged.
TskCfg tsk_choose(hipStream_t s, int kind, long n, int nv, int nw, const std::vector<TskCfg>& cands,
                  const std::function<void(const TskCfg&)>& launch, int reps = 0, double* best_us = nullptr);
// Tune one key on buffers of its own (dl_tune_tsk).
TskCfg tsk_tune(hipStream_t s, int kind, long n, int nv, int nw, int reps, double* best_us);

// Partial count tsk_dots uses for length n (partials are [2*nv][nblocks]).
int tsk_nblocks(long n);
// part <- partials of c = V^H w (sum with sum_partials(part, nb, 2*nv, c)). Returns nb.
// with_norm: partial column 2*nv holds ||w||^2 (part needs 2*(nv+1)*nb doubles).  gate (device,
// may be NULL): *gate == 0 skips the pass, leaving zero partials.
int tsk_dots(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
             const double2* w, double* part, const double* gate = nullptr, int with_norm = 0);
// w <- w + sgn * V c, c: nv complex in device memory; *gate == 0 (gate non-null) skips it.
void tsk_update(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                const double2* c, double sgn, double2* w, const double* gate = nullptr);
// The DGKS test after a first Gram-Schmidt pass with coefficients c (nv complex) of a vector w
// of squared norm *wn2: *gate = 1 (a second pass is needed) when ||c||^2 > (1 - eta2) *wn2.
void tsk_dgks_gate(hipStream_t s, const double* c, int nv, const double* wn2, double eta2, double* gate);
// Y_l (+)= sum_j G[j*ldg + l] V_j for l < ny; output l at obase + (oslot ? oslot[l] : l) * old.
void tsk_combine(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                 const double* G, int ldg, int ny, double2* obase, long old, const int* oslot,
                 int accumulate);

// Several columns at once (nw <= 16 fields W_r / X_r at stride ldw / ldx; nv <= 64 for the
// dots): part <- partials of c[r*nv + j] = <V_j, W_r> (sum with
// sum_partials(part, np, 2*nv*nw, c)), returns np (<= 2048, so part needs 2*nv*nw*2048
// doubles); columns with active[r] == 0 (active may be NULL) read as zero.
int tsk_dots_multi(hipStream_t s, long n, int nv, const double2* base, long ld, const double2* W, long ldw, int nw,
                   const int* active, double* part);
// X_r += sum_j D[r*nv + j] V_j for r < nw with active[r] != 0 (any nv; 128 vectors per launch).
void tsk_update_multi(hipStream_t s, long n, int nv, const double2* base, long ld, const double2* D, int nw,
                      const int* active, double2* X, long ldx);
int tsk_multi_nblocks(long n);
// The same update over an FP32-stored basis (FP64 products and sums).
void tsk_update_multi32(hipStream_t s, long n, int nv, const float2* base, long ld, const double2* D, int nw,
                        const int* active, double2* X, long ldx);

// Matrix-core form of the multi-column dots over FP32- or BF16-stored fields (FP32
// accumulation, FP64 partials): part <- partials of c[r*nv + j] = <V_j, W_r> for nv <= 128,
// nw <= 16 (sum with sum_partials(part, np, 2*nv*nw, c)); returns np <= tsk_lowp_nblocks(n, prec)
// (<= 2048, so part needs 2*nv*nw*2048 doubles; the tuned grid picks np).  Fields must be 16-byte aligned, with ld and
// ldw multiples of the elements per 16 bytes (2 for FP32, 4 for BF16).
int tsk_dots_lowp(hipStream_t s, long n, int nv, const float2* base, long ld, const float2* W, long ldw, int nw,
                  const int* active, double* part);
int tsk_dots_lowp(hipStream_t s, long n, int nv, const bf2* base, long ld, const bf2* W, long ldw, int nw,
                  const int* active, double* part);
int tsk_lowp_nblocks(long n, int prec);

// c = V^H w (and w -= V c if subtract) with the partials in the library's fixed per-device
// array; device pointers only; no allocation (noalloc.hip).
int tsk_project_noalloc(dl_ctx* ctx, long n, int nv, const double2* V, double2* w, double2* c, int subtract);

}  // namespace dl
