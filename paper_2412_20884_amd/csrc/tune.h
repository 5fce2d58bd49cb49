// Autotuner table shared by the product dispatch (api.hip) and the tuner (tune.hip).
#pragma once

#include <vector>

#include "gpk.h"
#include "pass.h"

namespace gpk {

struct TuneKey {
  int op;    // 0 product (gp_kmatvec), 1 with gradient (gp_quadform_grad), 2 trajectory launch
  int prec, kind, dp, rb, nb;  // precision, kind, padded d, padded R, floor(log2 N); for op 2
                               // dp is the batch's largest padded d, rb the kernel variant
                               // (preconditioned 1, Chebyshev 2, GP_BF16X 4), nb of the largest N
};

struct TuneCfg {
  int splits;  // column splits of the pair grid
  int ib;      // matrix-core kernel: 16-row blocks per wave (1 or 2)
  float ms;    // measured time of one call (ms)
  // trajectory launches (op 2): waves per SIMD of the persistent kernel's register allocation,
  // and the product jobs' columns per trip for chains with d <= 8 and d > 8 (0: default)
  int waves = 0, cpt_lo = 0, cpt_hi = 0;
};

TuneKey tune_key(int op, int prec, int kind, int d, int rpass, int64_t n);
bool tune_lookup(const TuneKey &k, TuneCfg *out);
void tune_store(const TuneKey &k, const TuneCfg &c);
// Candidate configurations for a problem (defined in api.hip next to the planner).
std::vector<TuneCfg> tune_candidates(const gp_kernel *k, int64_t n, int r, int with_grad);
// While tuning, force the planner to use `c` (nullptr: back to the table / defaults).
void tune_force(const TuneCfg *c);

}  // namespace gpk
