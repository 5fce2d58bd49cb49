"""Seeded synthetic workloads, shared by the tests, the benchmark and the smoke check.

This module only draws numbers: it holds none of the method's arithmetic (no kernel values,
no products, no solves).  Every array is float64 on the host; callers cast to the device
precision.  Streams are independent per (workload, purpose) through numpy's PCG64 seeded with
an entropy list [workload_seed, purpose].

Workloads (shapes and distributions of the five benchmark configurations):
  small_fp64  N=1024, X ~ U[0,1]^2, y = sin(2 pi x1) cos(2 pi x2) + 0.1 N(0,1), isotropic SE,
              theta = (0, log 0.2, log 0.01); 8 N(0,1) right-hand sides; 100 leapfrog steps of 1e-2.
  ard8        N=65,536, X ~ N(0, I_8), ARD SE, alpha = 1, l_k log-uniform on [0.3, 3],
              sigma^2 = 1e-2; 16 N(0,1) right-hand sides and 16 upstream gradients.
  large3      N=2^20, X ~ U[0,1]^3, isotropic SE, l = 0.05, alpha = 1, sigma^2 = 1e-3;
              32 N(0,1) auxiliary vectors.
  batched     64 instances, N_b uniform integers in [2048, 32768], d_b in {4, 8, 16},
              X ~ N(0, I_d), ARD SE, l_k log-uniform on [0.3, 3], alpha = 1, sigma^2 = 0.1 (the
              noise variance of the paper's synthetic scaling runs), y = prod_k cos(x_k) +
              0.1 N(0,1); 8 chains each; 20-step trajectories of step 1e-3.
  ard64       N=262,144, X ~ N(0, I_64), ARD SE, l_k log-uniform on [0.5, 8], alpha = 1,
              sigma^2 = 1e-2; 16 chains x 50 leapfrog steps of step 3e-5.
"""
from __future__ import annotations

import numpy as np

# purpose ids: one independent stream per purpose
P_X, P_YNOISE, P_THETA, P_V, P_U, P_PI, P_UACC, P_XI, P_SHAPE = range(9)

WORKLOAD_SEEDS = {"small_fp64": 0, "ard8": 2, "large3": 3, "batched": 4, "ard64": 5, "cheb2d": 6}


def rng(seed, purpose):
    return np.random.default_rng([int(seed), int(purpose)])


def uniform_points(n, d, seed):
    return rng(seed, P_X).uniform(0.0, 1.0, size=(n, d))


def normal_points(n, d, seed):
    return rng(seed, P_X).standard_normal((n, d))


def normal_matrix(n, r, seed, purpose=P_V):
    return rng(seed, purpose).standard_normal((n, r))


def theta_iso(alpha, ell, sigma2):
    return np.array([np.log(alpha), np.log(ell), np.log(sigma2)], dtype=np.float64)


def theta_ard_loguniform(d, lo, hi, seed, alpha=1.0, sigma2=1e-2):
    ell = np.exp(rng(seed, P_THETA).uniform(np.log(lo), np.log(hi), size=d))
    return np.concatenate([[np.log(alpha)], np.log(ell), [np.log(sigma2)]])


def y_sincos(X, seed, noise=0.1):
    e = rng(seed, P_YNOISE).standard_normal(X.shape[0])
    return np.sin(2 * np.pi * X[:, 0]) * np.cos(2 * np.pi * X[:, 1]) + noise * e


def y_prodcos(X, seed, noise=0.1):
    e = rng(seed, P_YNOISE).standard_normal(X.shape[0])
    return np.prod(np.cos(X), axis=1) + noise * e


def small_fp64(n=1024, r=8):
    s = WORKLOAD_SEEDS["small_fp64"]
    X = uniform_points(n, 2, s)
    return {
        "kind": "iso", "X": X, "y": y_sincos(X, s),
        "theta": theta_iso(1.0, 0.2, 0.01),
        "V": normal_matrix(n, r, s, P_V), "U": normal_matrix(n, r, s, P_U),
        "pi": rng(s, P_PI).standard_normal(3), "u": rng(s, P_UACC).uniform(),
        "xi": rng(s, P_XI).standard_normal(n),
        "dt": 1e-2, "n_steps": 100,
    }


def ard8(n=65536, r=16):
    s = WORKLOAD_SEEDS["ard8"]
    X = normal_points(n, 8, s)
    return {
        "kind": "ard", "X": X, "theta": theta_ard_loguniform(8, 0.3, 3.0, s),
        "V": normal_matrix(n, r, s, P_V), "G": normal_matrix(n, r, s, P_U),
    }


def large3(n=1 << 20, r=32):
    s = WORKLOAD_SEEDS["large3"]
    return {
        "kind": "iso", "X": uniform_points(n, 3, s), "theta": theta_iso(1.0, 0.05, 1e-3),
        "Z": normal_matrix(n, r, s, P_V),
    }


def batched(n_inst=64, chains=8, n_lo=2048, n_hi=32768, dims=(4, 8, 16), n_steps=20, sigma2=0.1):
    s = WORKLOAD_SEEDS["batched"]
    g = rng(s, P_SHAPE)
    ns = g.integers(n_lo, n_hi, endpoint=True, size=n_inst)
    ds = g.choice(np.asarray(dims), size=n_inst)
    inst = []
    for b in range(n_inst):
        sb = 1000 + b
        X = normal_points(int(ns[b]), int(ds[b]), sb)
        theta = theta_ard_loguniform(int(ds[b]), 0.3, 3.0, sb, sigma2=sigma2)
        inst.append({
            "X": X, "y": y_prodcos(X, sb), "theta": theta,
            "xi": rng(sb, P_XI).standard_normal((chains, int(ns[b]))),
            "pi": rng(sb, P_PI).standard_normal((chains, len(theta))),
            "u": rng(sb, P_UACC).uniform(size=chains),
        })
    return {"kind": "ard", "instances": inst, "chains": chains, "dt": 1e-3, "n_steps": n_steps}


def ard64(n=262144, chains=16, n_steps=50):
    s = WORKLOAD_SEEDS["ard64"]
    X = normal_points(n, 64, s)
    return {
        "kind": "ard", "X": X, "y": y_prodcos(X, s),
        "theta": theta_ard_loguniform(64, 0.5, 8.0, s),
        "xi": rng(s, P_XI).standard_normal((chains, n)),
        "pi": rng(s, P_PI).standard_normal((chains, 66)),
        "u": rng(s, P_UACC).uniform(size=chains),
        "dt": 3e-5, "n_steps": n_steps, "chains": chains,
    }


def cheb2d(n=3000, n_cheb=4, chains=10, n_updates=10, n_steps=3, dt=0.03, ell=0.3, sigma2=0.1):
    """Stand-in for the satellite-data run of Section 4.3: N points in [-1, 1]^2, half uniform and
    half in 8 tight Gaussian clusters (the measurements there cluster geographically), y a
    de-meaned smooth field plus noise; the Chebyshev-amplitude kernel with N_cheb^2 coefficients
    (small N(0, 0.1) draws), log l and log sigma^2; B chains, each HMC update a fresh xi, pi and
    u per chain and N_int leapfrog steps of dt."""
    s = WORKLOAD_SEEDS["cheb2d"]
    g = rng(s, P_X)
    nu = n // 2
    centres = g.uniform(-0.8, 0.8, size=(8, 2))
    lab = g.integers(0, 8, size=n - nu)
    X = np.concatenate([g.uniform(-1.0, 1.0, size=(nu, 2)),
                        np.clip(centres[lab] + 0.05 * g.standard_normal((n - nu, 2)), -1.0, 1.0)])
    y = y_sincos(0.5 * (X + 1.0), s)
    nt = n_cheb ** 2 + 2
    theta = np.concatenate([0.1 * rng(s, P_THETA).standard_normal(n_cheb ** 2),
                            [np.log(ell), np.log(sigma2)]])
    return {
        "kind": "cheb", "n_cheb": n_cheb, "X": X, "y": y - y.mean(), "theta": theta,
        "xi": rng(s, P_XI).standard_normal((n_updates, chains, n)),
        "pi": rng(s, P_PI).standard_normal((n_updates, chains, nt)),
        "u": rng(s, P_UACC).uniform(size=(n_updates, chains)),
        "dt": dt, "n_steps": n_steps, "chains": chains, "n_updates": n_updates,
    }


def iso_problem(n, d, seed, ell=0.2, sigma2=1e-2, alpha=1.0, r=4, dist="uniform"):
    """A generic seeded problem for parity tests at arbitrary sizes."""
    X = uniform_points(n, d, seed) if dist == "uniform" else normal_points(n, d, seed)
    return {
        "kind": "iso", "X": X, "theta": theta_iso(alpha, ell, sigma2),
        "V": normal_matrix(n, r, seed, P_V), "U": normal_matrix(n, r, seed, P_U),
        "y": y_prodcos(X, seed), "xi": rng(seed, P_XI).standard_normal(n),
    }


def ard_problem(n, d, seed, lo=0.3, hi=3.0, sigma2=1e-2, r=4):
    X = normal_points(n, d, seed)
    return {
        "kind": "ard", "X": X, "theta": theta_ard_loguniform(d, lo, hi, seed, sigma2=sigma2),
        "V": normal_matrix(n, r, seed, P_V), "U": normal_matrix(n, r, seed, P_U),
        "y": y_prodcos(X, seed), "xi": rng(seed, P_XI).standard_normal(n),
    }
