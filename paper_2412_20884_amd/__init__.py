"""gpk: matrix-free kernel products, quadratic-form gradients and HMC leapfrog trajectories for
determinant-free fully Bayesian Gaussian process regression, on hand-written gfx950 HIP kernels.

The compute path is the C-ABI library libgpk.so (declared in include/gpk.h); `gpk` is its
argument-marshalling binding.  Importing this package does not load the library; the first
call does, and fails loudly if it has not been built.
"""
__all__ = ["gpk", "inputs"]
