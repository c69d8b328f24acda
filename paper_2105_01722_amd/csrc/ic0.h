// IC(0) baseline for the element systems of the PCG path (Sec. 7.1).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "pcg.h"

namespace gdw {

// Level sets of the two triangular solves of an IC(0) factor on the GD stencil of
// (N, p): lv = forward rows [nn], forward starts [nfw + 1], backward rows [nn], backward
// starts [nbw + 1].
void ic0_levels(int N, int p, std::vector<int>& lv, int* nfw, int* nbw);

// For every element: A = S_K (op 0) or M_J (op 1) in the upper-half stencil layout, U its
// IC(0) factor (of S_hat's stencil entries for op 0), then x = IC(0)-PCG solution of
// S_hat x = b (op 0) or M_J x = b (op 1) from x = 0; its[e] = iterations.  bad / fail
// (device ints, preset by the caller) receive the smallest element id whose factor broke
// down / whose solve reached maxit.  A, U: [nel][nst] workspace; lv: device copy of the
// level tables.
hipError_t launch_ic0(const PcgGeom& g, const PcgElem& el, int op, long nel, double* A, double* U,
                      const int* lv, int nfw, int nbw, const double* b, double* x, double rtol,
                      int maxit, int* its, int* bad, int* fail, hipStream_t st);

}  // namespace gdw
