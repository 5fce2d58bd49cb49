// Weights and shifts of the pole expansion A^{-1/2} ~ sum_j w_j (A + lambda_j I)^{-1} (Section
// 3.1, eq. pex; Appendix A, eq. msqdisc), host and device.
//
// With m <= lambda_min(A), M >= lambda_max(A), k^2 = m / M and K' = K(1 - k^2), the nodes
// t_j = i (j - 1/2) K' / N_p are purely imaginary; Jacobi's imaginary transformation turns sn,
// cn, dn of modulus k at i u into sc, 1 / cn and dc of the complementary parameter 1 - k^2 at u,
// so every shift and weight is real:
//     lambda_j = m sc^2(u_j | 1 - k^2),   w_j = 2 K' sqrt(m) / (pi N_p) dn(u_j) / cn^2(u_j).
// K' = pi / (2 AGM(1, k)); sn, cn, dn from the descending AGM (Landen) scale followed by the
// backward angle recursion.  The scale depends on k only, so it is formed once per spectrum and
// shared by the N_p nodes.  Nodes past K'/2 are evaluated at their reflection K' - u (also a
// node) so that cn never cancels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace gpk {

constexpr int kAgmMax = 63;  // most levels of the descending scale (quadratic convergence)

// K(1 - k^2) for 0 < k <= 1 from the arithmetic-geometric mean of 1 and k.
__host__ __device__ inline double ellk_complement(double k) {
  double a = 1.0, b = k;
  for (int it = 0; it < 64 && fabs(a - b) > 1e-16 * a; ++it) {
    const double an = 0.5 * (a + b);
    b = sqrt(a * b);
    a = an;
  }
  return M_PI / (2.0 * a);
}

// The descending scale of parameter mpar = 1 - k^2: a_0 = 1, c_0 = sqrt(mpar), b_0 = k,
// a_{n+1} = (a_n + b_n) / 2, b_{n+1} = sqrt(a_n b_n), c_{n+1} = (a_n - b_n) / 2 until c_n is
// negligible.  a and c hold kAgmMax entries; returns the last level N.
__host__ __device__ inline int agm_scale(double k, double *a, double *c) {
  a[0] = 1.0;
  c[0] = sqrt((1.0 - k) * (1.0 + k));
  double b = k;
  int n = 0;
  while (fabs(c[n]) > 1e-17 * a[n] && n < kAgmMax - 1) {
    const double an = 0.5 * (a[n] + b);
    c[n + 1] = 0.5 * (a[n] - b);
    b = sqrt(a[n] * b);
    a[n + 1] = an;
    ++n;
  }
  return n;
}

// sn, cn, dn(u | 1 - k^2) from the scale of agm_scale (N levels): phi_N = 2^N a_N u,
// phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2; sn = sin(phi_0), cn = cos(phi_0),
// dn = cos(phi_0) / cos(phi_1 - phi_0).  N = 0 (mpar = 0) gives the circular functions.
__host__ __device__ inline void jacobi_scaled(const double *a, const double *c, int n, double u,
                                              double *sn, double *cn, double *dn) {
  double phi = ldexp(a[n] * u, n);
  double phi_next = phi;  // phi_1 once the recursion ends
  for (int j = n; j >= 1; --j) {
    phi_next = phi;
    phi = 0.5 * (phi + asin(c[j] * sin(phi) / a[j]));
  }
  *sn = sin(phi);
  *cn = cos(phi);
  *dn = n >= 1 ? cos(phi) / cos(phi_next - phi) : 1.0;
}

// Weight and shift of node j of np for the spectrum [m, M], given k = sqrt(m / M), K' and the
// scale (a, c, n) of k.
__host__ __device__ inline void pole_node(double m, double M, int np, int j, double k, double kp,
                                          const double *a, const double *c, int n, double *w,
                                          double *shift) {
  const double scale = 2.0 * kp * sqrt(m) / (M_PI * np);
  double sn, cn, dn;
  if (2 * j + 1 <= np) {  // u_j <= K'/2: direct
    jacobi_scaled(a, c, n, (j + 0.5) * kp / np, &sn, &cn, &dn);
    *shift = m * (sn / cn) * (sn / cn);
    *w = scale * dn / (cn * cn);
  } else {
    // u_j > K'/2, where cn(u_j) -> 0 would lose relative accuracy: reflect to v = K' - u_j
    // (itself a node), sn(u) = cd(v), cn(u) = k sd(v), dn(u) = k nd(v), so that
    // m sc^2(u) = M cn^2(v) / sn^2(v) and dn(u) / cn^2(u) = dn(v) / (k sn^2(v))
    jacobi_scaled(a, c, n, (np - j - 0.5) * kp / np, &sn, &cn, &dn);
    *shift = M * (cn / sn) * (cn / sn);
    *w = scale * dn / (k * sn * sn);
  }
}

}  // namespace gpk
