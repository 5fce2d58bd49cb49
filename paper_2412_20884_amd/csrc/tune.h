// Autotuner table shared by the product dispatch (api.hip) and the tuner (tune.hip).
#pragma once

#include <vector>

#include "gpk.h"
#include "pass.h"

namespace gpk {

struct TuneKey {
  int op;    // 0 product (gp_kmatvec), 1 with gradient (gp_quadform_grad)
  int prec, kind, dp, rb, nb;  // precision, kind, padded d, padded R, floor(log2 N)
};

struct TuneCfg {
  int splits;  // column splits of the pair grid
  int ib;      // matrix-core kernel: 16-row blocks per wave (1 or 2)
  float ms;    // measured time of one call (ms)
};

TuneKey tune_key(int op, int prec, int kind, int d, int rpass, int64_t n);
bool tune_lookup(const TuneKey &k, TuneCfg *out);
void tune_store(const TuneKey &k, const TuneCfg &c);
// Candidate configurations for a problem (defined in api.hip next to the planner).
std::vector<TuneCfg> tune_candidates(const gp_kernel *k, int64_t n, int r, int with_grad);
// While tuning, force the planner to use `c` (nullptr: back to the table / defaults).
void tune_force(const TuneCfg *c);

}  // namespace gpk
