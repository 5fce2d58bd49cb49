// VALU pair kernels instantiated for float.
#define GPK_T float
#define GPK_SUFFIX f32
#define GPK_LAUNCH_PASS launch_pass_f32
#define GPK_LAUNCH_STAGE launch_stage_f32
#include "pair_valu.inc"
