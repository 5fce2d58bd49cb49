// HMC trajectory kernels instantiated for float.
#define GPK_T float
#define GPK_SUFFIX hmc_f32
#define GPK_HMC_KICKOFF hmc_kickoff_f32
#define GPK_HMC_TILES hmc_tiles_f32
#define GPK_HMC_EPILOGUE hmc_epilogue_f32
#define GPK_HMC_GATHER hmc_gather_f32
#define GPK_HMC_PERSISTENT hmc_persistent_f32
#define GPK_HMC_CHAIN_BYTES hmc_chain_bytes_f32
#define GPK_HMC_RESET hmc_reset_f32
#define GPK_HMC_CHECK hmc_check_f32
#define GPK_HMC_PHI_POLES hmc_phi_poles_f32
#define GPK_XM 1
#include "hmc_kernels.inc"
