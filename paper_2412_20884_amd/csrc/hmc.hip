// HMC leapfrog trajectories (placeholder until the CG/leapfrog kernels land).
#include "gpk.h"
#include "pass.h"

namespace gpk {
gp_status fail(gp_status st, const char *fmt, ...);
}

extern "C" {

size_t gp_hmc_workspace_size(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b) {
  (void)k; (void)p; (void)b;
  return 0;
}

gp_status gp_hmc_leapfrog(const gp_kernel *k, const gp_hmc_params *p, const gp_batch *b,
                          const void *X, const void *y, const void *phi, double *theta,
                          double *pi, void *x_warm, const double *u_accept, double *H0,
                          double *H1, int32_t *accepted, int32_t *status, int32_t *cg_iters,
                          void *ws, size_t ws_bytes, hipStream_t stream) {
  (void)k; (void)p; (void)b; (void)X; (void)y; (void)phi; (void)theta; (void)pi; (void)x_warm;
  (void)u_accept; (void)H0; (void)H1; (void)accepted; (void)status; (void)cg_iters; (void)ws;
  (void)ws_bytes; (void)stream;
  return gpk::fail(GP_ERR_UNSUPPORTED, "gp_hmc_leapfrog is not available in this build");
}

}
