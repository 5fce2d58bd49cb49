// HMC trajectory kernels instantiated for double.
#define GPK_T double
#define GPK_SUFFIX hmc_f64
#define GPK_HMC_KICKOFF hmc_kickoff_f64
#define GPK_HMC_TILES hmc_tiles_f64
#define GPK_HMC_EPILOGUE hmc_epilogue_f64
#define GPK_HMC_GATHER hmc_gather_f64
#define GPK_HMC_PERSISTENT hmc_persistent_f64
#define GPK_HMC_CHAIN_BYTES hmc_chain_bytes_f64
#define GPK_HMC_RESET hmc_reset_f64
#define GPK_HMC_CHECK hmc_check_f64
#define GPK_HMC_PHI_POLES hmc_phi_poles_f64
#define GPK_XM 0
#include "hmc_kernels.inc"
