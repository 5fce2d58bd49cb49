// Chebyshev-amplitude kernel (GP_SE_CHEB): entry points behind gp_kmatvec / gp_quadform_grad,
// called after their argument checks.
#pragma once

#include "common.h"
#include "gpk.h"

namespace gpk {

// N_cheb^d for a GP_SE_CHEB description, or -1 if N_cheb < 1 or N_cheb^d > 64.
int cheb_terms(const gp_kernel *k);
size_t cheb_workspace_size(const gp_kernel *k, int64_t n, int r);
gp_status cheb_kmatvec(const gp_kernel *k, int64_t n, const void *X, const double *theta, int r,
                       const void *V, int64_t ldv, const double *col_shift, void *out,
                       int64_t ldo, void *ws, size_t ws_bytes, hipStream_t s);
gp_status cheb_quadform_grad(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                             int r, const void *U, int64_t ldu, const void *V, int64_t ldv,
                             const double *w, double *grad, double *quad, void *AU, int64_t ldau,
                             void *AV, int64_t ldav, void *ws, size_t ws_bytes, hipStream_t s);

}  // namespace gpk
