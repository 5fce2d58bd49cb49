// VALU pair kernels instantiated for double.
#define GPK_T double
#define GPK_SUFFIX f64
#define GPK_LAUNCH_PASS launch_pass_f64
#define GPK_LAUNCH_STAGE launch_stage_f64
#include "pair_valu.inc"
