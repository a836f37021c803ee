// Launchers of the tall-skinny basis contractions (tsk.hip).
#pragma once
#include "internal.hpp"

namespace dl {

// Partial count tsk_dots uses for length n (partials are [2*nv][nblocks]).
int tsk_nblocks(long n);
// part <- partials of c = V^H w (sum with sum_partials(part, nb, 2*nv, c)). Returns nb.
int tsk_dots(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
             const double2* w, double* part);
// w <- w + sgn * V c, c: nv complex in device memory.
void tsk_update(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                const double2* c, double sgn, double2* w);
// Y_l (+)= sum_j G[j*ldg + l] V_j for l < ny; output l at obase + (oslot ? oslot[l] : l) * old.
void tsk_combine(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                 const double* G, int ldg, int ny, double2* obase, long old, const int* oslot,
                 int accumulate);

}  // namespace dl
