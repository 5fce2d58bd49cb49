"""Writes tests/golden/e1_grid_marginals.json and e1_cheb_grid_marginals.json from the oracle only.

The E1 data (Section 4.1) on the paper's [-3,3]^2 grid with sigma^2 = 0.1 fixed: with the
paper's own kernel, the Chebyshev-amplitude SE kernel with N_cheb = 2 coefficients (Theta_0,
Theta_1) free and 2 l^2 = 1 fixed; and with the isotropic SE kernel's (log alpha, log l) free.
Stores the normalised marginal densities and CDFs (trapezoid rule) used by the statistical
sampler tests.  Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import posterior  # noqa: E402


def e1_data():
    spec = json.load(open(os.path.join(HERE, "e1_problem.json")))
    n = spec["N"]
    X = (spec["x_lo"] + (spec["x_hi"] - spec["x_lo"]) * np.arange(n) / n)[:, None]
    y = np.full(n, spec["y_value"])
    axis = np.linspace(spec["grid_lo"], spec["grid_hi"], spec["grid_n"])
    return spec, X, y, axis


def cheb_base(spec):
    """theta = (Theta_0, Theta_1, log l, log sigma^2) with 2 l^2 = two_l2."""
    return np.array([0.0, 0.0, 0.5 * np.log(0.5 * spec["two_l2"]), np.log(spec["sigma2"])])


def main():
    spec, X, y, axis = e1_data()
    logp = posterior.grid_log_posterior(X, "cheb", y, cheb_base(spec), (0, 1), (axis, axis))
    (m0, m1), (c0, c1) = posterior.grid_marginals(logp, (axis, axis))
    out = {"source": "oracle.posterior via tests/golden/make_golden.py", "axis": axis.tolist(),
           "marginal_theta0": m0.tolist(), "marginal_theta1": m1.tolist(),
           "cdf_theta0": c0.tolist(), "cdf_theta1": c1.tolist()}
    with open(os.path.join(HERE, "e1_cheb_grid_marginals.json"), "w") as f:
        json.dump(out, f, indent=0)
    base = np.array([0.0, 0.0, np.log(spec["sigma2"])])
    logp = posterior.grid_log_posterior(X, "iso", y, base, (0, 1), (axis, axis))
    (m0, m1), (c0, c1) = posterior.grid_marginals(logp, (axis, axis))
    out = {"source": "oracle.posterior via tests/golden/make_golden.py", "axis": axis.tolist(),
           "marginal_log_alpha": m0.tolist(), "marginal_log_l": m1.tolist(),
           "cdf_log_alpha": c0.tolist(), "cdf_log_l": c1.tolist()}
    with open(os.path.join(HERE, "e1_grid_marginals.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("written")


if __name__ == "__main__":
    main()
