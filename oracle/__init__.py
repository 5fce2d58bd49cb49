"""FP64 CPU oracle for the determinant-free fully Bayesian GPR hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute anything in this package: only the tests, the package's smoke check
and the benchmark's CPU-baseline leg use it. It shares no code with the HIP
path: it builds the kernel matrix densely (in row blocks for large N) with
numpy/scipy in float64 and is written from the paper's formulas alone.

Modules
  gp         kernel matrix A(theta), matrix-free product, quadratic-form values
             and theta-gradients (Section 2, eq. kerdef/kernmat; Section 1 SE
             kernel; Section 3.2.1, capacity (3)).
  hmc        exact solve, potential U_phi, force via the frozen-x trick,
             Stormer-Verlet leapfrog, Hamiltonian and Metropolis decision
             (Section 3.2, eq. U, eq. xtheta, eq. u; Section 3.2.2; Algorithm 1).
  posterior  exact (Cholesky-determinant) log posterior, eq. P, and the
             Gaussian-integral identity behind the pseudofermion trick
             (Section 3, eq. extendeddensity).
  poles      pole expansion of A^{-1/2} (Section 3.1, eq. pex; Appendix A).
  stats      integrated autocorrelation time and moving-window statistics
             (Appendix C; Section 4.1).
"""
from . import gp, hmc, posterior, poles, stats  # noqa: F401
