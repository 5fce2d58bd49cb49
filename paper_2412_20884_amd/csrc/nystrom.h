// Internal interface of the Nystrom preconditioner, shared by the batched PCG and the implicit
// integrator's fixed-point map.
#pragma once

#include "common.h"

namespace gpk {

// Scratch bytes nystrom_apply needs for n rows, a rank-`rank` factor and r columns.
size_t nystrom_apply_scratch(int64_t n, int rank, int r);

// z = P^{-1} v for the r columns of v (n x r, leading dimension r):
//   P^{-1} v_c = v_c + U ((lam_rank + mu_c) / (lam + mu_c) - 1) U^T v_c,
//   mu_c = sigma^2(theta) + shift_c (shift may be NULL).  z must not alias v.
template <typename T>
hipError_t nystrom_apply(int64_t n, int rank, const T *U, const double *lam, const double *theta,
                         int nth, const double *shift, int r, const T *v, T *z, char *scratch,
                         hipStream_t s);

}  // namespace gpk
