"""Benchmark of the hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-leapfrog] [--no-leapfrog-full]
                    [--no-cpu] [--no-ard8] [--no-ard64] [--no-precond] [--no-implicit] [--no-small]
                    [--no-cheb2d]

A step is one fused gp_quadform_grad pass over the large3 workload (N = 2^20 points uniform in
[0,1]^3, isotropic SE kernel l = 0.05, alpha = 1, sigma^2 = 1e-3, 32 N(0,1) auxiliary vectors Z):
A Z, q_c = z_c^T A z_c and grad_theta sum_c q_c in one pass over all N^2 pairs.  Inputs are
resident in HBM before the timed region.  The value is pair evaluations per second (N^2 per
step).  The JSON line also carries the roofline of the dominant kernel (the matrix-core pair
kernel); the FP64 oracle timed on a bounded row slab of the same workload on the host cores,
which also checks rows of the timed outputs, and the oracle's exact-solve leapfrog on the FP64
workload; identities of the timed outputs; the HMC leapfrog legs on the batched workload (64
instances, 8 chains each, 20-step trajectories; phi by the device Gibbs refresh): graph replay,
Nystrom-preconditioned graph replay and plain mode on a subset, and all 64 instances in one
preconditioned launch; the ARD d = 8 forward/backward rates; the d = 64 workload in the bfloat16
cross-term precision; plain against Nystrom-preconditioned CG; the FP64 workload in three modes;
the Chebyshev-kernel stand-in of the paper's satellite-data run; and one implicit-midpoint
trajectory.  Every leg states its error against an FP64 reference.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-evals/s for K_θV + ∇θ at N=2^20; HMC leapfrog steps/s batched vs plain"
FLOP_PER_PAIR = 143          # 4R + 3d + 6 with R = 32, d = 3 (isotropic, U = V)
PEAK_F16_MFMA = 2.5e15       # dense fp16 matrix-core peak, FLOP/s
PEAK_F32_VECTOR = 157.3e12   # fp32 vector peak, FLOP/s
# Issue bound of the pair kernel. Per 64-lane pair slot (one pair per lane of a wave) the SQ
# counters of pair_mfma<3,32,1,2> on this workload count 13.62 VALU instructions besides the MFMAs
# (11.62 plain FP32 ones, one v_exp_f32, one v_cvt_pkrtz_f16_f32) and 1.5 v_mfma_f32_16x16x32_f16.
# An issue-rate probe (profiles/issue_costs_gfx950.md) measured, in shader cycles per wave instruction: 2.2
# for plain FP32 VALU with VGPR operands, 8.3 for v_exp_f32, 4.15 for v_cvt_pkrtz_f16_f32, and
# ~16 added per MFMA when the VALU is saturated (the two do not overlap then). 1024 SIMDs at the
# 2.4 GHz peak clock.
SLOT_VALU, SLOT_EXP, SLOT_CVT, SLOT_MFMA = 11.62, 1.0, 1.0, 1.5
CYC_VALU, CYC_EXP, CYC_CVT, CYC_MFMA = 2.2, 8.3, 4.15, 16.0
SLOT_CYCLES = SLOT_VALU * CYC_VALU + SLOT_EXP * CYC_EXP + SLOT_CVT * CYC_CVT + SLOT_MFMA * CYC_MFMA
ISSUE_BOUND_PAIRS = 1024 * 2.4e9 * 64 / SLOT_CYCLES


def log(msg):
    print(msg, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pair_mfma_large3_traffic.md")
KERNEL_SOURCES = ["paper_2412_20884_amd/csrc/pair_mfma.hip", "paper_2412_20884_amd/csrc/pass.h",
                  "paper_2412_20884_amd/csrc/common.h"]


def measured_traffic():
    """HBM bytes per launch of the pair kernel from the committed rocprofv3 counter summary, or
    None when the kernel sources have changed since the counters were taken."""
    import hashlib

    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_sources_sha256"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    h = hashlib.sha256()
    for src in KERNEL_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if fields.get("kernel_sources_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def bench_large3(steps, warmup, tune=True, tune_load=None, tune_save=None):
    import torch

    from paper_2412_20884_amd import gpk, inputs

    dev = "cuda:0"
    w = inputs.large3()
    n, r = w["X"].shape[0], w["Z"].shape[1]
    tuned = None
    if tune_load:
        gpk.tune_load(tune_load)
        tuned = {"table": tune_load, "loaded": True}
        log(f"tuning table loaded from {tune_load}")
    elif tune:
        t0 = time.perf_counter()
        gpk.tune("iso", 3, n, r, torch.float32, with_grad=True)
        tuned = {"seconds": time.perf_counter() - t0}
        if tune_save:
            gpk.tune_save(tune_save)
            tuned["table"] = tune_save
        log(f"tuned in {tuned['seconds']:.1f} s")
    X = torch.tensor(w["X"], dtype=torch.float32, device=dev)
    Z = torch.tensor(w["Z"], dtype=torch.float32, device=dev)
    th = torch.tensor(w["theta"], dtype=torch.float64, device=dev)
    k = gpk.make_kernel("iso", X)
    ws = torch.empty(gpk.workspace_size(k, n, r), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        return gpk.quadform_grad(X, th, Z, Z, None, "iso", want_AU=True, ws=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        res = step()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in ev]
    return {"w": w, "res": res, "wall": wall, "per_call": per, "n": n, "r": r, "tuned": tuned}


def parity_sample(b):
    """Identities of the timed outputs that hold at any size (no reference computation): the
    alpha-gradient equals sum_c q_c - sigma^2 |Z|^2 and the sigma^2-gradient equals sigma^2 |Z|^2.
    Rows of A Z are checked against the oracle inside the CPU baseline leg."""
    w, res = b["w"], b["res"]
    Z = np.asarray(w["Z"], np.float32).astype(np.float64)
    s2 = float(np.exp(w["theta"][2]))
    zz = float(np.sum(Z * Z))
    g = res["grad"].cpu().numpy()
    q = res["quad"].cpu().numpy()
    err_alpha = abs(g[0] - (q.sum() - s2 * zz)) / abs(g[0])
    err_sigma = abs(g[2] - s2 * zz) / abs(g[2])
    return {"rel_err_grad_alpha_identity": float(err_alpha), "rel_err_grad_sigma2": float(err_sigma)}


def cpu_baseline(budget_s=15.0, gpu_res=None):
    """The FP64 oracle on a row slab of the large3 workload (all 2^20 columns); the same slab
    checks the timed GPU pass (rows of A Z, componentwise); and the oracle's exact-solve
    leapfrog on the FP64 N = 1024 workload, timed (a different algorithm: Cholesky per step)."""
    from oracle import gp as ogp
    from paper_2412_20884_amd import inputs

    w = inputs.large3()
    X = np.asarray(w["X"], np.float32).astype(np.float64)
    Z = np.asarray(w["Z"], np.float32).astype(np.float64)
    n = X.shape[0]
    workers = max(1, min(16, os.cpu_count() or 1))
    rows = np.arange(workers * 4)
    t0 = time.perf_counter()
    ogp.quadform_grad(X, w["theta"], "iso", Z, Z, rows=rows, workers=workers)
    t1 = time.perf_counter() - t0
    m = int(max(len(rows), min(n, len(rows) * budget_s / max(t1, 1e-3))))
    m = (m // workers) * workers
    rows = np.arange(m)
    t0 = time.perf_counter()
    slab = ogp.quadform_grad(X, w["theta"], "iso", Z, Z, rows=rows, workers=workers)
    t = time.perf_counter() - t0
    parity = None
    if gpu_res is not None:
        k = min(m, 64)
        got = gpu_res["AU"][:k].double().cpu().numpy()
        ref = slab["AU"][:k]
        absref = ogp.matvec(X, w["theta"], "iso", np.abs(Z), rows=np.arange(k))
        parity = {"rows": k, "componentwise_rel_err_AZ": float(np.max(np.abs(got - ref) / absref)),
                  "col_rel_err_AZ": float(np.max(np.linalg.norm(got - ref, axis=0) /
                                                 np.linalg.norm(ref, axis=0)))}
    # the oracle's trajectory on the FP64 workload (phi an exact conditional draw by the
    # oracle's own Cholesky factor), timed
    from scipy.linalg import cho_factor, solve_triangular

    from oracle import hmc as ohmc
    sw = inputs.small_fp64()
    Lc = cho_factor(ogp.a_matrix(sw["X"], sw["theta"], "iso"), lower=True)[0]
    phi = solve_triangular(np.tril(Lc).T, sw["xi"], lower=False)
    t0 = time.perf_counter()
    ohmc.leapfrog(sw["X"], "iso", sw["y"], phi, sw["theta"], sw["pi"], sw["dt"], sw["n_steps"])
    t_lf = time.perf_counter() - t0
    cpu = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key = key.strip()
                if key in ("model name", "vendor_id", "cpu family", "model", "stepping", "cpu MHz") \
                        and key not in cpu:
                    cpu[key] = val.strip()
    except OSError:
        pass
    return {"value": m * n / t, "unit": "pair-evals/s", "cores": workers,
            "threads": {"workers": workers, "blas_omp": os.environ.get("OMP_NUM_THREADS"),
                        "host_cpus_visible": os.cpu_count()},
            "cpu_model": cpu.get("model name", "unknown"),
            "cpu_id": {k: cpu.get(k) for k in ("vendor_id", "cpu family", "model", "stepping", "cpu MHz")},
            "kind": "oracle",
            "sample": f"rows 0..{m - 1} of the large3 workload against all {n} columns "
                      f"(FP64 numpy, {t:.1f} s wall), fused A Z + q + grad",
            "parity_of_timed_gpu_pass": parity,
            "leapfrog_small_fp64": {"chain_steps_per_s": sw["n_steps"] / t_lf, "seconds": t_lf,
                                    "algorithm": "exact Cholesky solves per step (not CG), FP64 numpy",
                                    "workload": "N=1024, d=2, one chain, 100 leapfrog steps of 1e-2"}}


def trajectory_tune_entries():
    """The trajectory entries (op 2) of the library's tuning table, as saved."""
    import json
    import tempfile

    from paper_2412_20884_amd import gpk

    with tempfile.NamedTemporaryFile("r", suffix=".json") as f:
        gpk.tune_save(f.name)
        entries = json.load(open(f.name))["entries"]
    keep = ("dp", "rb", "nb", "waves", "cpt_lo", "cpt_hi", "ms")
    return [{k: e[k] for k in keep} | {"prec": e["prec"]} for e in entries if e["op"] == 2]


def bench_leapfrog(modes=("graph", "graph_nystrom", "plain"), subset=8, group=0, rwm=True,
                   precond_rank=128, tune=True):
    """Chain-leapfrog-steps/s on the batched workload, batched (graph replay) vs plain.

    subset = k takes every k-th instance (k = 1: all 64 instances). group = g > 0 runs the
    batched modes as consecutive persistent launches over g instances each (all chains of
    those instances), with a progress line per launch; 0 runs every instance in one launch.
    Mode graph_nystrom is graph mode with every solve preconditioned by a rank-`precond_rank`
    Nystrom factor per instance, built once at the instance's theta_0 (timed separately).
    rwm = False leaves out the random-walk Metropolis leg.
    """
    import torch

    from paper_2412_20884_amd import gpk, inputs

    dev = "cuda:0"
    wl = inputs.batched()
    C = wl["chains"]
    inst = wl["instances"][::subset]
    ns = [len(b["y"]) for b in inst]
    ds = [b["X"].shape[1] for b in inst]
    offs = np.cumsum([0] + ns[:-1])
    xoffs = np.cumsum([0] + [a * b for a, b in zip(ns, ds)][:-1])
    X = torch.tensor(np.concatenate([b["X"].ravel() for b in inst]), dtype=torch.float32, device=dev)[:, None]
    y = torch.tensor(np.concatenate([b["y"] for b in inst]), dtype=torch.float32, device=dev)
    # phi | theta_0 for every chain by the Gibbs refresh (pole expansion, multi-shift CG), one
    # call per instance with its 8 chains' xi as the right-hand sides; timed as its own leg
    phi = torch.empty(sum(ns) * C, dtype=torch.float32, device=dev)
    t_phi, it_phi, cols = 0.0, [], 0
    for bi, b in enumerate(inst):
        Xb = X[xoffs[bi]:xoffs[bi] + ns[bi] * ds[bi]].view(ns[bi], ds[bi])
        xi = torch.tensor(b["xi"].T.copy(), dtype=torch.float32, device=dev)
        thb = torch.tensor(b["theta"], dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gpk.phi_refresh(Xb, thb, xi, "ard", tol=1e-6, maxit=3000)
        torch.cuda.synchronize()
        t_phi += time.perf_counter() - t0
        if np.any(r["status"].cpu().numpy() != 0):
            raise RuntimeError(f"phi refresh did not converge on instance {bi}")
        it_phi.append(int(r["iters"].max()))
        cols += C
        phi[C * offs[bi]:C * (offs[bi] + ns[bi])] = r["phi"].t().contiguous().view(-1)
    refresh = {"chains_refreshed_per_s": cols / t_phi, "seconds": t_phi,
               "multishift_cg_iterations": it_phi, "n_poles": 15, "tol": 1e-6,
               "workload": "phi = A(theta_0)^{-1/2} xi for the 8 chains of each instance of the subset "
                           "below (one call per instance, 8 right-hand sides), FP32"}
    # the same refresh for every chain of every instance in one launch of the batched refresh,
    # each chain as its own system (the form the sampler needs once chains' theta differ)
    xi_all = torch.tensor(np.concatenate([b["xi"].ravel() for b in inst]), dtype=torch.float32, device=dev)
    th_all = torch.tensor(np.concatenate([np.tile(b["theta"], C) for b in inst]), dtype=torch.float64,
                          device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = gpk.phi_refresh_chains(X, th_all, xi_all, "ard", ns, offs, C, d=ds, x_offsets=xoffs, tol=1e-6,
                                maxit=3000, mode=gpk.BATCHED)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    if np.any(rb["status"].cpu().numpy() != 0):
        raise RuntimeError("batched phi refresh did not converge")
    dphi = (rb["phi"] - phi).norm().item() / phi.norm().item()
    refresh["one_launch_all_chains"] = {
        "chains_refreshed_per_s": cols / t_b, "seconds": t_b,
        "max_multishift_iterations": int(rb["iters"].max()),
        "rel_diff_vs_per_instance_calls": dphi,
        "note": "gp_phi_refresh_chains, BATCHED mode: every chain's product is its own R = 1 job "
                "(the per-instance calls share one R = 8 product between an instance's chains)"}
    log(f"phi refresh: {refresh}")
    th0 = np.concatenate([np.tile(b["theta"], C) for b in inst])
    pi0 = np.concatenate([b["pi"].ravel() for b in inst])
    u = torch.tensor(np.concatenate([b["u"] for b in inst]), dtype=torch.float64, device=dev)
    out = {}
    ref_theta = None
    U_all = lam_all = None
    if tune:
        # the trajectory launch (register allocation, columns per trip) for this batch's class,
        # with and without the preconditioned variant
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if any(m != "graph_nystrom" and m != "plain" for m in modes):
            gpk.tune_hmc("ard", ns, C, ds)
        if "graph_nystrom" in modes:
            gpk.tune_hmc("ard", ns, C, ds, precond_rank=precond_rank)
        out["autotune"] = {"seconds": time.perf_counter() - t0, "chosen": trajectory_tune_entries()}
        log(f"leapfrog autotune: {out['autotune']}")
    if "graph_nystrom" in modes:
        Us, lams = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for bi, b in enumerate(inst):
            Xb = X[xoffs[bi]:xoffs[bi] + ns[bi] * ds[bi]].view(ns[bi], ds[bi])
            om = torch.tensor(inputs.rng(1000 + bi, inputs.P_V).standard_normal((ns[bi], precond_rank)),
                              dtype=torch.float32, device=dev)
            U, lam = gpk.nystrom(Xb, torch.tensor(b["theta"], dtype=torch.float64, device=dev), om, "ard")
            Us.append(U)
            lams.append(lam)
        U_all, lam_all = torch.cat(Us).contiguous(), torch.cat(lams).contiguous()
        torch.cuda.synchronize()
        out["nystrom_build"] = {"rank": precond_rank, "seconds": time.perf_counter() - t0,
                                "instances": len(inst)}
        del Us
    for mode in modes:
        m = {"plain": gpk.PLAIN, "batched": gpk.BATCHED, "graph": gpk.GRAPH,
             "graph_nystrom": gpk.GRAPH}[mode]
        th = torch.tensor(th0, dtype=torch.float64, device=dev)
        pi = torch.tensor(pi0, dtype=torch.float64, device=dev)
        x = torch.zeros(sum(ns) * C, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        kw = dict(n_steps=wl["n_steps"], dt=wl["dt"], cg_tol=1e-6, cg_maxit=2000, mode=m)
        pre = mode == "graph_nystrom"
        if mode == "plain":
            # one instance per call so progress is visible; the library runs chains one at a time
            t = 0.0
            sts, itl, accs = [], [], []
            toff = 0
            for bi in range(len(ns)):
                nth = ds[bi] + 2
                thb = th[toff:toff + C * nth]
                pib = pi[toff:toff + C * nth]
                xb = x[C * offs[bi]:C * (offs[bi] + ns[bi])]
                Xb = X[xoffs[bi]:xoffs[bi] + ns[bi] * ds[bi]]
                t0 = time.perf_counter()
                r = gpk.hmc_leapfrog(Xb, y[offs[bi]:offs[bi] + ns[bi]], phi[C * offs[bi]:C * (offs[bi] + ns[bi])],
                                     thb, pib, xb, "ard", [ns[bi]], [0], C, d=[ds[bi]],
                                     u=u[bi * C:(bi + 1) * C], **kw)
                torch.cuda.synchronize()
                t += time.perf_counter() - t0
                sts.append(r["status"].cpu().numpy())
                itl.append(r["cg_iters"].cpu().numpy())
                accs.append(r["accepted"].cpu().numpy())
                toff += C * nth
                log(f"  plain instance {bi}: N={ns[bi]} d={ds[bi]} cumulative {t:.1f} s")
            st = np.concatenate(sts)
            its = np.concatenate(itl)
            acc = np.concatenate(accs)
        elif group > 0:
            # consecutive persistent launches over `group` instances each
            t = 0.0
            sts, itl, accs = [], [], []
            toff = 0
            for g0 in range(0, len(ns), group):
                gi = list(range(g0, min(len(ns), g0 + group)))
                nth_g = sum(C * (ds[b] + 2) for b in gi)
                r0, r1 = offs[gi[0]], offs[gi[-1]] + ns[gi[-1]]
                x0_, x1_ = xoffs[gi[0]], xoffs[gi[-1]] + ns[gi[-1]] * ds[gi[-1]]
                t0 = time.perf_counter()
                pg = (U_all[r0:r1], lam_all[gi[0] * precond_rank:(gi[-1] + 1) * precond_rank]) if pre else None
                r = gpk.hmc_leapfrog(X[x0_:x1_], y[r0:r1], phi[C * r0:C * r1], th[toff:toff + nth_g],
                                     pi[toff:toff + nth_g], x[C * r0:C * r1], "ard", [ns[b] for b in gi],
                                     [offs[b] - r0 for b in gi], C, d=[ds[b] for b in gi],
                                     x_offsets=[xoffs[b] - x0_ for b in gi], u=u[gi[0] * C:(gi[-1] + 1) * C],
                                     precond=pg, **kw)
                torch.cuda.synchronize()
                t += time.perf_counter() - t0
                sts.append(r["status"].cpu().numpy())
                itl.append(r["cg_iters"].cpu().numpy())
                accs.append(r["accepted"].cpu().numpy())
                toff += nth_g
                log(f"  {mode} instances {gi[0]}..{gi[-1]}: cumulative {t:.1f} s")
            st = np.concatenate(sts)
            its = np.concatenate(itl)
            acc = np.concatenate(accs)
        else:
            # one launch for every chain; the scheduler's progress word (pinned host memory) is
            # read while it runs, so that a long launch prints progress
            prog = torch.zeros(1, dtype=torch.int32).pin_memory()
            t0 = time.perf_counter()
            res = gpk.hmc_leapfrog(X, y, phi, th, pi, x, "ard", ns, offs, C, d=ds, x_offsets=xoffs, u=u,
                                   precond=(U_all, lam_all) if pre else None,
                                   progress=prog if m != gpk.PLAIN else None, **kw)
            done_ev = torch.cuda.Event()
            done_ev.record()
            last = t0
            while not done_ev.query():
                time.sleep(0.002)
                if time.perf_counter() - last > 20.0:
                    last = time.perf_counter()
                    log(f"  {mode}: {int(prog[0])} of {len(ns) * C} chains finished, {last - t0:.0f} s")
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            st = res["status"].cpu().numpy()
            its = res["cg_iters"].cpu().numpy()
            acc = res["accepted"].cpu().numpy()
        if mode != "plain":
            # true residual |y - A(theta) x| / |y| of the solves the accepted chains return (a
            # rejected chain gets its warm start back), A x by the FP64 product
            worst, toff, c = 0.0, 0, 0
            for bi in range(len(ns)):
                nth = ds[bi] + 2
                Xb = X[xoffs[bi]:xoffs[bi] + ns[bi] * ds[bi]].view(ns[bi], ds[bi]).double()
                yb = y[offs[bi]:offs[bi] + ns[bi]].double()
                for h in range(C):
                    if acc[c]:
                        xh = x[C * offs[bi] + h * ns[bi]:C * offs[bi] + (h + 1) * ns[bi]].double()
                        Ax = gpk.kmatvec(Xb, th[toff + h * nth:toff + (h + 1) * nth], xh, "ard")
                        worst = max(worst, float(torch.linalg.norm(yb - Ax) / torch.linalg.norm(yb)))
                    c += 1
                toff += C * nth
            out_res = worst
        thn = th.cpu().numpy()
        # pairs evaluated by the CG products alone (one N_b^2 sweep per iteration): a lower bound
        # on the work, since force passes, residual restarts and energies come on top
        cg_pairs = float(np.sum(its.astype(np.float64) * np.repeat(np.asarray(ns, np.float64) ** 2, C)))
        out[mode] = {"chain_steps_per_s": len(st) * wl["n_steps"] / t, "seconds": t,
                     "cg_pair_evals_per_s_lower_bound": cg_pairs / t,
                     "mean_cg_iters_per_solve": float(its.mean() / (wl["n_steps"] + 2)),
                     "accept_rate": float(np.mean(acc)),
                     "flagged_chains": int((st != 0).sum())}
        if mode != "plain":
            out[mode]["max_true_rel_residual_accepted"] = out_res
        if ref_theta is None:
            ref_theta = thn
        else:
            out[mode]["max_abs_theta_diff_vs_" + modes[0]] = float(np.max(np.abs(thn - ref_theta)))
        log(f"leapfrog {mode}: {out[mode]}")
        torch.cuda.empty_cache()
    if "graph" in out and "plain" in out:
        out["speedup_batched_vs_plain"] = out["graph"]["chain_steps_per_s"] / out["plain"]["chain_steps_per_s"]
    if rwm:
        # random-walk Metropolis on the same chains: 20 graph-mode updates, proposal scale 0.05,
        # xi ~ N(0, I) and u ~ U(0, 1) drawn here (seeded), the solve carried as the warm start
        n_upd, scale = 20, 0.05
        g = np.random.default_rng(20240)
        th = torch.tensor(th0, dtype=torch.float64, device=dev)
        x = torch.zeros(sum(ns) * C, dtype=torch.float32, device=dev)
        xis = torch.tensor(g.normal(size=(n_upd, th.numel())), dtype=torch.float64, device=dev)
        us = torch.tensor(g.uniform(size=(n_upd, len(ns) * C)), dtype=torch.float64, device=dev)
        xi = torch.empty_like(th)
        uu = torch.empty(len(ns) * C, dtype=torch.float64, device=dev)
        acc_n, its_n, flagged = 0, 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_upd):
            xi.copy_(xis[k])
            uu.copy_(us[k])
            r = gpk.rwm(X, y, phi, th, xi, x, "ard", ns, offs, C, d=ds, x_offsets=xoffs, u=uu, dt=scale,
                        cg_tol=1e-6, cg_maxit=2000, mode=gpk.GRAPH)
            acc_n += r["accepted"].sum()
            its_n += r["cg_iters"].sum()
            flagged += (r["status"] != 0).sum()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        nchain = len(ns) * C
        out["rwm_graph"] = {"chain_updates_per_s": nchain * n_upd / t, "seconds": t, "updates": n_upd,
                            "proposal_scale": scale, "accept_rate": float(acc_n.item()) / (nchain * n_upd),
                            "mean_cg_iters_per_update": float(its_n.item()) / (nchain * n_upd),
                            "flagged_chains": int(flagged.item())}
        log(f"rwm graph: {out['rwm_graph']}")
    out["phi_refresh"] = refresh
    out["workload"] = (f"batched: instances 0,{subset},{2 * subset},.. ({len(inst)} of 64; N_b in [2048, 32768], "
                       f"d_b in {{4,8,16}}), ARD SE, sigma^2=0.1, 8 chains each, {wl['n_steps']} leapfrog "
                       f"steps, dt {wl['dt']:g}, CG tol 1e-6, FP32, phi from the device Gibbs refresh; "
                       + (f"batched modes as persistent launches over {group} instances each; " if group > 0 else "")
                       + f"N_b = {ns}, d_b = {ds}")
    return out


def bench_ard64(n_chain_steps=5, chains=16, dt=None, plain_chains=2):
    """The d = 64 workload with GP_BF16X (bfloat16 cross term, compensated norms): rates of the
    product (R = 1, one CG iteration) and of the fused force pass (R = 2, [x | phi] with
    w = (-1/2, 1/2)) through the product entry points, their error against FP64, and the
    trajectories: every chain's phi from one device Gibbs refresh (the chains share theta_0, so one
    multi-shift call with one column per chain), then all chains in one graph-replayed persistent
    launch, against the plain mode (per-op launches) on the first `plain_chains` chains of the
    same inputs."""
    import torch

    from paper_2412_20884_amd import gpk, inputs

    dev = "cuda:0"
    wl = inputs.ard64(chains=max(chains, 1))
    n = wl["X"].shape[0]
    X = torch.tensor(wl["X"], dtype=torch.float32, device=dev)
    th = torch.tensor(wl["theta"], dtype=torch.float64, device=dev)
    y = torch.tensor(wl["y"], dtype=torch.float32, device=dev)
    V = torch.tensor(wl["xi"][:2].T.copy(), dtype=torch.float32, device=dev)
    w = torch.tensor([-0.5, 0.5], dtype=torch.float64, device=dev)
    out = {"workload": "ard64: N=262,144 points N(0, I_64), ARD SE (66 hyperparameters, l_k "
                       "log-uniform [0.5, 8]), sigma^2=1e-2, GP_BF16X", "N": n, "d": 64}
    ws = torch.empty(gpk.workspace_size(gpk.make_kernel("ard", X, "bf16x"), n, 2), dtype=torch.uint8, device=dev)
    for name, fn in (("kmatvec_r1", lambda: gpk.kmatvec(X, th, V[:, :1].contiguous(), "ard", prec="bf16x", ws=ws)),
                     ("force_pass_r2", lambda: gpk.quadform_grad(X, th, V, V, w, "ard", prec="bf16x", ws=ws))):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        out[name] = {"seconds": t, "pair_evals_per_s": n * n / t}
        log(f"ard64 {name}: {out[name]}")
    # error against the library's FP64 path (direct differences): the whole product and its
    # off-diagonal part (K - alpha I) V against that part's own norm
    got = gpk.kmatvec(X, th, V, "ard", prec="bf16x", ws=ws).double()
    Vd = V.double()
    ref = gpk.kmatvec(X.double(), th, Vd, "ard")
    torch.cuda.synchronize()
    diag = float(np.exp(wl["theta"][0]) + np.exp(wl["theta"][-1]))
    od_g, od_r = got - diag * Vd, ref - diag * Vd
    out["error_vs_fp64"] = {
        "product": float(((got - ref).norm(dim=0) / ref.norm(dim=0)).max()),
        "offdiagonal_part": float(((od_g - od_r).norm(dim=0) / od_r.norm(dim=0)).max()),
        "offdiagonal_norm_over_column": float((od_r.norm(dim=0) / ref.norm(dim=0)).min()),
        "budget": 3e-3, "reference": "the library's FP64 kernels on the same inputs, all rows"}
    log(f"ard64 error vs FP64: {out['error_vs_fp64']}")
    del got, ref, Vd, od_g, od_r, ws
    if chains < 1:
        return out
    dt = dt or wl["dt"]
    # phi for every chain at theta_0: one refresh, one column per chain
    xi = torch.tensor(wl["xi"][:chains].T.copy(), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ph = gpk.phi_refresh(X, th, xi, "ard", prec="bf16x", tol=1e-6, maxit=500)
    torch.cuda.synchronize()
    t_phi = time.perf_counter() - t0
    phi = ph["phi"].T.contiguous().view(-1)  # [chain][n]
    out["phi_refresh"] = {"seconds": t_phi, "chains": chains, "iterations": int(ph["iters"].max())}
    log(f"ard64 phi refresh: {out['phi_refresh']}")
    th0 = np.tile(wl["theta"], chains)
    pi0 = wl["pi"][:chains].ravel()
    u = torch.tensor(wl["u"][:chains], dtype=torch.float64, device=dev)
    res = {}
    for mode, nch in (("graph", chains), ("plain", min(plain_chains, chains))):
        thc = torch.tensor(th0[:66 * nch], dtype=torch.float64, device=dev)
        pi = torch.tensor(pi0[:66 * nch], dtype=torch.float64, device=dev)
        x = torch.zeros(nch * n, dtype=torch.float32, device=dev)
        md = gpk.GRAPH if mode == "graph" else gpk.PLAIN
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gpk.hmc_leapfrog(X.view(-1, 1), y, phi[:nch * n], thc, pi, x, "ard", [n], [0], nch,
                             d=[64], u=u[:nch], n_steps=n_chain_steps, dt=dt, cg_tol=1e-6,
                             cg_maxit=500, mode=md, prec="bf16x")
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        dh = (r["H1"] - r["H0"]).cpu().numpy()
        res[mode] = {"theta": thc.cpu().numpy(), "H1": r["H1"].cpu().numpy()}
        out[f"trajectories_{mode}"] = {
            "chains": nch, "chain_steps": nch * n_chain_steps, "seconds": t,
            "chain_steps_per_s": nch * n_chain_steps / t,
            "cg_iterations_per_chain": float(r["cg_iters"].double().mean()),
            "accept_rate": float(r["accepted"].double().mean()),
            "status_nonzero": int((r["status"] != 0).sum()),
            "dH_range": [float(dh.min()), float(dh.max())]}
        log(f"ard64 trajectories {mode}: {out[f'trajectories_{mode}']}")
    k = 66 * min(plain_chains, chains)
    out["graph_vs_plain"] = {
        "max_abs_theta_diff": float(np.max(np.abs(res["graph"]["theta"][:k] - res["plain"]["theta"]))),
        "note": "the same matrix-core tiles in both modes, one job per launch in plain mode"}
    out["speedup_batched_vs_plain"] = (out["trajectories_graph"]["chain_steps_per_s"]
                                       / out["trajectories_plain"]["chain_steps_per_s"])
    out["trajectory_workload"] = (f"{chains} chains x {n_chain_steps} leapfrog steps of dt {dt:g}, "
                                  f"CG tol 1e-6, phi from the device Gibbs refresh")
    return out


def bench_precond(rank=200):
    """Solves A x = y on the ard8 workload (N = 65,536, d = 8, FP32, sigma^2 = 1e-2): plain CG
    against CG preconditioned by a rank-`rank` randomized Nystrom factor, same tolerance."""
    import torch

    from paper_2412_20884_amd import gpk, inputs

    dev = "cuda:0"
    w = inputs.ard8(r=1)
    n = w["X"].shape[0]
    X = torch.tensor(w["X"], dtype=torch.float32, device=dev)
    th = torch.tensor(w["theta"], dtype=torch.float64, device=dev)
    y = torch.tensor(w["V"][:, 0], dtype=torch.float32, device=dev)
    om = torch.tensor(inputs.normal_matrix(n, rank, inputs.WORKLOAD_SEEDS["ard8"], inputs.P_XI),
                      dtype=torch.float32, device=dev)
    out = {"workload": f"ard8: N={n}, d=8, ARD SE, sigma^2=1e-2, FP32; A x = y to relative residual "
                       f"1e-6; Nystrom rank {rank}", "rank": rank}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = gpk.pcg_solve(X, th, y, "ard", tol=1e-6, maxit=5000)
    torch.cuda.synchronize()
    out["cg"] = {"seconds": time.perf_counter() - t0, "iterations": int(plain["iters"][0]),
                 "status": int(plain["status"][0])}
    log(f"precond: plain CG {out['cg']}")
    t0 = time.perf_counter()
    U, lam = gpk.nystrom(X, th, om, "ard")
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    pre = gpk.pcg_solve(X, th, y, "ard", U=U, lam=lam, tol=1e-6, maxit=5000)
    torch.cuda.synchronize()
    out["nystrom_pcg"] = {"build_seconds": t_build, "solve_seconds": time.perf_counter() - t0,
                          "iterations": int(pre["iters"][0]), "status": int(pre["status"][0]),
                          "lam_top": float(lam[0]), "lam_last": float(lam[-1])}
    diff = (plain["x"] - pre["x"]).double().norm() / plain["x"].double().norm()
    out["solution_rel_diff"] = float(diff)
    out["speedup_total"] = out["cg"]["seconds"] / (t_build + out["nystrom_pcg"]["solve_seconds"])
    log(f"precond: Nystrom PCG {out['nystrom_pcg']}, speedup {out['speedup_total']:.2f}")
    return out


def bench_small_fp64(tol=1e-6):
    """The FP64 workload (N = 1024, d = 2, isotropic SE): one chain, 100 leapfrog steps of 1e-2
    after a device phi refresh, in the plain, batched and graph modes."""
    import torch

    from paper_2412_20884_amd import gpk, inputs

    dev = "cuda:0"
    wl = inputs.small_fp64()
    n = wl["X"].shape[0]
    X = torch.tensor(wl["X"], dtype=torch.float64, device=dev)
    y = torch.tensor(wl["y"], dtype=torch.float64, device=dev)
    th0 = torch.tensor(wl["theta"], dtype=torch.float64, device=dev)
    ph = gpk.phi_refresh(X, th0, torch.tensor(wl["xi"], dtype=torch.float64, device=dev), "iso",
                         tol=1e-12, maxit=2000)
    torch.cuda.synchronize()
    phi = ph["phi"].contiguous()
    u = torch.tensor([wl["u"]], dtype=torch.float64, device=dev)
    out = {"workload": f"small_fp64: N={n}, d=2, iso SE, FP64, one chain, {wl['n_steps']} leapfrog "
                       f"steps of dt {wl['dt']:g}, CG tol {tol:g}, phi by the device refresh",
           "phi_refresh_iterations": int(ph["iters"][0])}
    for name, mode in (("plain", gpk.PLAIN), ("batched", gpk.BATCHED), ("graph", gpk.GRAPH)):
        th = th0.clone()
        pi = torch.tensor(wl["pi"], dtype=torch.float64, device=dev)
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        t0 = time.perf_counter()
        r = gpk.hmc_leapfrog(X.view(-1, 1), y, phi, th, pi, x, "iso", [n], [0], 1, d=[2], u=u,
                             n_steps=wl["n_steps"], dt=wl["dt"], cg_tol=tol, cg_maxit=3000, mode=mode)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[name] = {"chain_steps_per_s": wl["n_steps"] / t, "seconds": t,
                     "mean_cg_iters_per_solve": int(r["cg_iters"][0]) / (wl["n_steps"] + 2),
                     "dH": float(r["H1"][0] - r["H0"][0]), "accepted": int(r["accepted"][0]),
                     "status": int(r["status"][0])}
        log(f"small_fp64 {name}: {out[name]}")
        if name == "graph":
            th_gpu, pi_gpu = th.cpu().numpy(), pi.cpu().numpy()
    # error of the production-tolerance trajectory against the same trajectory with the solves
    # at 1e-13 (the FP64 path; the oracle's exact-solve trajectory is matched to 1e-8 in the tests)
    th = th0.clone()
    pi = torch.tensor(wl["pi"], dtype=torch.float64, device=dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    gpk.hmc_leapfrog(X.view(-1, 1), y, phi, th, pi, x, "iso", [n], [0], 1, d=[2], n_steps=wl["n_steps"],
                     dt=wl["dt"], cg_tol=1e-13, cg_maxit=5000, mode=gpk.GRAPH)
    torch.cuda.synchronize()
    out["graph_vs_tight_fp64"] = {"max_abs_theta_err": float(np.max(np.abs(th_gpu - th.cpu().numpy()))),
                                  "max_abs_pi_err": float(np.max(np.abs(pi_gpu - pi.cpu().numpy()))),
                                  "note": f"CG tolerance {tol:g} against 1e-13, same inputs"}
    log(f"small_fp64 error: {out['graph_vs_tight_fp64']}")
    return out


def bench_ard8(reps=5):
    """The ARD workload (N = 65,536, d = 8, FP32, R = 16): the autograd forward A(theta) V and
    its hand-written backward (one gp_quadform_grad pass with U = G, V = V: theta-gradient and
    A G), pair-evals/s and flop rate by the counting convention (forward 3d + 2 + 2R = 58 flop
    per pair, backward 4R + 6d + 4 = 116), and the error against the library's FP64 path
    (componentwise for the products, condition-scaled for the gradient)."""
    import torch

    from paper_2412_20884_amd import gpk, inputs

    dev = "cuda:0"
    wl = inputs.ard8()
    n, d = wl["X"].shape
    r = wl["V"].shape[1]
    X32 = np.asarray(wl["X"], np.float32)
    V32 = np.asarray(wl["V"], np.float32)
    G32 = np.asarray(wl["G"], np.float32)
    X = torch.tensor(X32, device=dev)
    V = torch.tensor(V32, device=dev)
    G = torch.tensor(G32, device=dev)
    th = torch.tensor(wl["theta"], dtype=torch.float64, device=dev)
    ws = torch.empty(gpk.workspace_size(gpk.make_kernel("ard", X), n, r), dtype=torch.uint8, device=dev)
    out = {"workload": f"ard8: N={n} points N(0, I_8), ARD SE (l_k log-uniform [0.3, 3]), sigma^2=1e-2, "
                       f"FP32, R={r}: forward A V and backward (grad_theta, A G) of KMatVec", "N": n, "d": d}
    res = {}
    for name, fn, flop in (
            ("forward", lambda: gpk.kmatvec(X, th, V, "ard", ws=ws), 3 * d + 2 + 2 * r),
            ("backward", lambda: gpk.quadform_grad(X, th, G, V, None, "ard", want_quad=False,
                                                   want_AU=True, ws=ws), 4 * r + 6 * d + 4)):
        res[name] = fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        t = float(np.median(ts))
        out[name] = {"seconds": t, "pair_evals_per_s": n * n / t, "flop_per_pair": flop,
                     "tflop_per_s": flop * n * n / t / 1e12,
                     "frac_of_fp16_mfma_peak": flop * n * n / t / PEAK_F16_MFMA,
                     "kernel": "pair_mfma (R = 16: fp16 hi/lo matrix-core contractions)"}
    # error against the library's FP64 path on the same (rounded) inputs
    Xd, Vd, Gd = X.double(), V.double(), G.double()
    ref_f = gpk.kmatvec(Xd, th, Vd, "ard")
    abs_f = gpk.kmatvec(Xd, th, Vd.abs(), "ard")
    ref_b = gpk.quadform_grad(Xd, th, Gd, Vd, None, "ard", want_quad=False, want_AU=True)
    abs_b = gpk.quadform_grad(Xd, th, Gd.abs(), Vd.abs(), None, "ard", want_quad=False, want_AU=True)
    torch.cuda.synchronize()
    out["error_vs_fp64_path"] = {
        "forward_componentwise": float(((res["forward"].double() - ref_f).abs() / abs_f).max()),
        "backward_AG_componentwise": float(((res["backward"]["AU"].double() - ref_b["AU"]).abs()
                                            / abs_b["AU"]).max()),
        "grad_theta_condition_scaled": float(((res["backward"]["grad"] - ref_b["grad"]).abs()
                                              / abs_b["grad"]).max()),
        "reference": "the library's FP64 kernels on the same inputs (checked against the oracle "
                     "at 1e-11 in the tests)"}
    log(f"ard8: {out}")
    return out


def bench_cheb2d(tol=1e-6, rank=500, refresh_every=5):
    """The Section 4.3 stand-in (N = 3000, d = 2, Chebyshev-amplitude kernel, N_cheb = 4, B = 10
    chains, N_int = 3 leapfrog steps of 0.03, FP64): each HMC update refreshes phi for every chain
    at its current theta on the device, then runs the 10 chains' trajectories in one graph-mode
    call (persistent launch replayed).  Run twice: with plain CG, and with the paper's rank-500
    Nystrom preconditioner rebuilt every five updates (at chain 0's theta, shared by the chains)
    and used by both the trajectory solves and the phi refresh."""
    import torch

    from paper_2412_20884_amd import gpk, inputs

    dev = "cuda:0"
    wl = inputs.cheb2d()
    n, nc, C, nu = wl["X"].shape[0], wl["n_cheb"], wl["chains"], wl["n_updates"]
    nt = wl["theta"].size
    X = torch.tensor(wl["X"], dtype=torch.float64, device=dev)
    y = torch.tensor(wl["y"], dtype=torch.float64, device=dev)
    xi = torch.tensor(wl["xi"], dtype=torch.float64, device=dev)
    omega = torch.tensor(inputs.rng(inputs.WORKLOAD_SEEDS["cheb2d"], inputs.P_V).standard_normal((n, rank)),
                         dtype=torch.float64, device=dev)

    def run(use_precond):
        th = torch.tensor(np.tile(wl["theta"], C), dtype=torch.float64, device=dev)
        x = torch.zeros(n * C, dtype=torch.float64, device=dev)
        phi = torch.empty(n * C, dtype=torch.float64, device=dev)
        xib = torch.empty(n * C, dtype=torch.float64, device=dev)
        pi = torch.empty(C * nt, dtype=torch.float64, device=dev)
        u = torch.empty(C, dtype=torch.float64, device=dev)
        acc, cg, ph_it, dH, t_phi, t_nys = 0, 0, 0, [], 0.0, 0.0
        pre, res, ph_out = None, None, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(nu):
            if use_precond and k % refresh_every == 0:
                t1 = time.perf_counter()
                U, lam = gpk.nystrom(X, th[:nt], omega, "cheb", n_cheb=nc)
                pre = (U, lam)
                torch.cuda.synchronize()
                t_nys += time.perf_counter() - t1
            t1 = time.perf_counter()
            if use_precond:
                # the paper's form: the shifted systems of each chain by preconditioned CG
                for c in range(C):
                    r = gpk.phi_refresh(X, th[c * nt:(c + 1) * nt], xi[k, c], "cheb", tol=tol,
                                        maxit=3000, n_cheb=nc, precond=pre)
                    phi[c * n:(c + 1) * n] = r["phi"].reshape(-1)
                    ph_it += int(r["iters"][0])
                    if int(r["status"][0]) != 0:
                        raise RuntimeError(f"cheb2d: phi refresh of chain {c} failed at update {k}")
            else:
                # every chain at its own theta in one graph-replayed launch (multi-shift CG)
                xib.copy_(xi[k].reshape(-1))
                ph_out = gpk.phi_refresh_chains(X.view(-1, 1), th, xib, "cheb", [n], [0], C, d=[2],
                                                tol=tol, maxit=3000, n_cheb=nc, mode=gpk.GRAPH,
                                                out=phi, outputs=ph_out)
                st = ph_out["status"].cpu().numpy()
                if np.any(st != 0):
                    raise RuntimeError(f"cheb2d: batched phi refresh status {st.tolist()} at update {k}")
                ph_it += int(ph_out["iters"].sum())
            torch.cuda.synchronize()
            t_phi += time.perf_counter() - t1
            pi.copy_(torch.from_numpy(wl["pi"][k].ravel()))
            u.copy_(torch.from_numpy(wl["u"][k]))
            res = gpk.hmc_leapfrog(X.view(-1, 1), y, phi, th, pi, x, "cheb", [n], [0], C, d=[2], u=u,
                                   n_steps=wl["n_steps"], dt=wl["dt"], cg_tol=tol, cg_maxit=3000,
                                   mode=gpk.GRAPH, n_cheb=nc, precond=pre, outputs=res)
            torch.cuda.synchronize()
            st = res["status"].cpu().numpy()
            if np.any(st != 0):
                raise RuntimeError(f"cheb2d: trajectory status {st.tolist()} at update {k}")
            acc += int(res["accepted"].sum())
            cg += int(res["cg_iters"].sum())
            dH += (res["H1"] - res["H0"]).cpu().numpy().tolist()
        t = time.perf_counter() - t0
        steps = nu * C * wl["n_steps"]
        return {"chain_leapfrog_steps_per_s": steps / t, "seconds": t, "phi_refresh_seconds": t_phi,
                "nystrom_build_seconds": t_nys, "updates_per_s": nu * C / t,
                "accept_rate": acc / (nu * C),
                "mean_cg_iters_per_solve": cg / (nu * C * (wl["n_steps"] + 2)),
                "mean_phi_iters": ph_it / (nu * C), "max_abs_dH": float(np.max(np.abs(dH))),
                "theta_final": th.cpu().numpy()}

    # the refresh alone at the chains' start theta: per-chain calls against one batched launch
    th0 = torch.tensor(np.tile(wl["theta"], C), dtype=torch.float64, device=dev)
    xi0 = xi[0].reshape(-1).contiguous()
    phi_a = torch.empty(n * C, dtype=torch.float64, device=dev)
    gpk.phi_refresh_chains(X.view(-1, 1), th0, xi0, "cheb", [n], [0], C, d=[2], tol=tol, maxit=3000,
                           n_cheb=nc, mode=gpk.BATCHED)  # warm-up (workspace, first launch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(C):
        r = gpk.phi_refresh(X, th0[c * nt:(c + 1) * nt], xi[0, c], "cheb", tol=tol, maxit=3000, n_cheb=nc)
        phi_a[c * n:(c + 1) * n] = r["phi"].reshape(-1)
    torch.cuda.synchronize()
    t_per = time.perf_counter() - t0
    t0 = time.perf_counter()
    rb = gpk.phi_refresh_chains(X.view(-1, 1), th0, xi0, "cheb", [n], [0], C, d=[2], tol=tol,
                                maxit=3000, n_cheb=nc, mode=gpk.BATCHED)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    refresh_cmp = {"per_chain_calls_seconds": t_per, "one_launch_seconds": t_one,
                   "speedup": t_per / t_one,
                   "rel_diff": (rb["phi"] - phi_a).norm().item() / phi_a.norm().item(),
                   "iterations": rb["iters"].cpu().numpy().tolist(),
                   "note": f"{C} chains at the start theta, FP64, multi-shift CG to tol {tol:g}: "
                           "gp_phi_refresh per chain against one gp_phi_refresh_chains launch"}
    log(f"cheb2d refresh: {refresh_cmp}")
    plain = run(False)
    prec = run(True)
    dtheta = float(np.max(np.abs(plain.pop("theta_final") - prec.pop("theta_final"))))
    out = {"workload": f"cheb2d: N={n}, d=2 (half uniform on [-1,1]^2, half in 8 clusters), "
                       f"Chebyshev-amplitude SE, N_cheb={nc} ({nt} hyperparameters), FP64, {C} chains, "
                       f"{nu} updates of {wl['n_steps']} leapfrog steps of dt {wl['dt']:g}, CG tol {tol:g}, "
                       "phi refreshed for every chain at every update on the device (plain CG run: all "
                       "chains in one graph-replayed gp_phi_refresh_chains launch; preconditioned run: "
                       "per chain, preconditioned CG per pole), trajectories in graph mode",
           "phi_refresh_per_chain_vs_one_launch": refresh_cmp,
           "graph_plain_cg": plain,
           f"graph_nystrom_rank{rank}_every{refresh_every}": prec,
           "max_abs_theta_diff_between_the_two": dtheta}
    log(f"cheb2d: {out}")
    return out


def bench_implicit(rank=50):
    """One chain of the batched workload's first instance: a 20-step implicit-midpoint trajectory
    (Anderson depth 10, Nystrom-based R of rank `rank`) against the plain-mode leapfrog
    trajectory of the same chain, same dt and CG tolerance."""
    import torch

    from paper_2412_20884_amd import gpk, inputs

    dev = "cuda:0"
    wl = inputs.batched()
    b = wl["instances"][0]
    n, d = b["X"].shape
    X = torch.tensor(b["X"], dtype=torch.float32, device=dev)
    y = torch.tensor(b["y"], dtype=torch.float32, device=dev)
    th0 = torch.tensor(b["theta"], dtype=torch.float64, device=dev)
    phi = gpk.phi_refresh(X, th0, torch.tensor(b["xi"][0], dtype=torch.float32, device=dev), "ard",
                          tol=1e-6, maxit=3000)["phi"].contiguous()
    om = torch.tensor(inputs.normal_matrix(n, rank, 1000, inputs.P_V), dtype=torch.float32, device=dev)
    out = {"workload": f"batched instance 0: N={n}, d={d}, ARD SE, sigma^2=0.1, FP32, one chain, "
                       f"{wl['n_steps']} steps of dt {wl['dt']:g}; implicit: Anderson depth 10, Nystrom "
                       f"rank {rank} for R, fixed-point tol 1e-4, linear tol 1e-6"}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U, lam = gpk.nystrom(X, th0, om, "ard")
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    th, pi = th0.clone(), torch.tensor(b["pi"][0], dtype=torch.float64, device=dev)
    x = torch.zeros(n, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    r = gpk.hmc_implicit(X, y, phi, th, pi, x, "ard", n_steps=wl["n_steps"], dt=wl["dt"], history=10,
                         tol=1e-4, maxit=500, cg_tol=1e-6, U=U, lam=lam)
    torch.cuda.synchronize()
    t_imp = time.perf_counter() - t0
    out["implicit"] = {"seconds": t_imp, "nystrom_build_seconds": t_build,
                       "chain_steps_per_s": wl["n_steps"] / (t_imp + t_build),
                       "fixed_point_iterations": int(r["iters"][0]), "status": int(r["status"][0]),
                       "dH": float(r["H1"][0] - r["H0"][0])}
    th, pi = th0.clone(), torch.tensor(b["pi"][0], dtype=torch.float64, device=dev)
    x = torch.zeros(n, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    r = gpk.hmc_leapfrog(X.view(-1, 1), y, phi, th, pi, x, "ard", [n], [0], 1, d=[d],
                         n_steps=wl["n_steps"], dt=wl["dt"], cg_tol=1e-6, cg_maxit=3000, mode=gpk.PLAIN)
    torch.cuda.synchronize()
    t_lf = time.perf_counter() - t0
    out["leapfrog_plain"] = {"seconds": t_lf, "chain_steps_per_s": wl["n_steps"] / t_lf,
                             "cg_iterations": int(r["cg_iters"][0]), "status": int(r["status"][0]),
                             "dH": float(r["H1"][0] - r["H0"][0])}
    log(f"implicit: {out['implicit']}; leapfrog plain: {out['leapfrog_plain']}")
    return out


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of a known size, run under the same profiler command so its
    FETCH_SIZE / WRITE_SIZE readings calibrate the counters (bytes per counter unit)."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_bytes_each_way": nbytes, "copies": 3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-leapfrog", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--leapfrog-modes", default="graph,graph_nystrom,plain")
    ap.add_argument("--leapfrog-precond-rank", type=int, default=128)
    ap.add_argument("--no-leapfrog-full", action="store_true",
                    help="leave out the one-launch run of all 64 batched instances (~2.5 min)")
    ap.add_argument("--leapfrog-subset", type=int, default=16)
    ap.add_argument("--leapfrog-group", type=int, default=0,
                    help="instances per persistent launch in the batched modes (0: all in one)")
    ap.add_argument("--no-rwm", action="store_true", help="leave out the random-walk Metropolis leg")
    ap.add_argument("--ard64-chains", type=int, default=16, help="chains of the d = 64 trajectory leg")
    ap.add_argument("--ard64-steps", type=int, default=5, help="leapfrog steps per d = 64 trajectory")
    ap.add_argument("--ard64-plain-chains", type=int, default=2,
                    help="chains of the d = 64 leg's plain-mode comparison")
    ap.add_argument("--ard64-dt", type=float, default=None, help="leapfrog step of the d = 64 leg")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-ard64", action="store_true")
    ap.add_argument("--no-ard8", action="store_true", help="leave out the ARD d = 8 forward/backward leg")
    ap.add_argument("--no-precond", action="store_true")
    ap.add_argument("--no-implicit", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="leave out the FP64 N = 1024 leg")
    ap.add_argument("--no-cheb2d", action="store_true",
                    help="leave out the Chebyshev-kernel N = 3000 leg")
    ap.add_argument("--tune-load", default=None, help="load a saved tuning table instead of tuning")
    ap.add_argument("--tune-save", default=None, help="write the tuning table found here to this path")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; multi-GPU sharding is a design "
                          "note (chains/instances split with no communication, large-N row shards "
                          "with a ring pass of column blocks)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    if args.copy_calibration:
        log(f"copy calibration: {copy_calibration()}")
    log("large3: generating inputs and warming up")
    b = bench_large3(args.steps, args.warmup, tune=not args.no_tune, tune_load=args.tune_load,
                     tune_save=args.tune_save)
    n = b["n"]
    t_step = float(np.median(b["per_call"]))
    value = n * n * args.steps / b["wall"]
    pairs_per_s_kernel = n * n / t_step
    achieved = FLOP_PER_PAIR * pairs_per_s_kernel
    log(f"large3: median call {t_step * 1e3:.2f} ms, {pairs_per_s_kernel:.4e} pair-evals/s")
    par = parity_sample(b)
    log(f"parity sample: {par}")
    line = {
        "metric": METRIC, "value": value, "unit": "pair-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["wall"] / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (the two R-contractions as fp16 hi/lo splits, 3 MFMA products each, f32 accumulate)",
        "data": "synthetic",
        "config": {"workload": "large3: N=2^20 points uniform in [0,1]^3, isotropic SE l=0.05, alpha=1, "
                               "sigma^2=1e-3, 32 N(0,1) auxiliary vectors; fused A Z + z_c^T A z_c + grad_theta",
                   "N": n, "d": 3, "R": b["r"], "pairs_per_step": n * n},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_F16_MFMA / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_F16_MFMA, "traffic": measured_traffic(),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "pair_mfma<3,32,1> (fp16 hi/lo split, 3 products per contraction)",
                     "flop_per_pair": FLOP_PER_PAIR,
                     "issue_bound_cycles_per_pair_slot": SLOT_CYCLES,
                     "issue_bound_pair_evals_per_s": ISSUE_BOUND_PAIRS,
                     "frac_of_issue_bound": pairs_per_s_kernel / ISSUE_BOUND_PAIRS},
        "parity": par,
        "autotune": b["tuned"],
    }
    if not args.no_cpu:
        log("cpu baseline: timing the FP64 oracle on a row slab")
        line["cpu_baseline"] = cpu_baseline(args.cpu_budget, b["res"])
    if not args.no_leapfrog:
        line["leapfrog"] = bench_leapfrog(tuple(args.leapfrog_modes.split(",")), args.leapfrog_subset,
                                          args.leapfrog_group, not args.no_rwm,
                                          args.leapfrog_precond_rank)
    if not args.no_leapfrog_full:
        # the whole batched workload (64 instances x 8 chains, 20 steps) in one persistent launch,
        # Nystrom-preconditioned, graph-replayed, its launch configuration tuned for its own class
        # (512 chains)
        line["leapfrog_full"] = bench_leapfrog(("graph_nystrom",), 1, 0, False,
                                               args.leapfrog_precond_rank)
    if not args.no_ard8:
        line["ard8_fwd_bwd"] = bench_ard8()
    if not args.no_ard64:
        line["ard64_bf16x"] = bench_ard64(args.ard64_steps, args.ard64_chains, args.ard64_dt,
                                          args.ard64_plain_chains)
    if not args.no_precond:
        line["nystrom_precond"] = bench_precond()
    if not args.no_implicit:
        line["implicit_midpoint"] = bench_implicit()
    if not args.no_small:
        line["small_fp64"] = bench_small_fp64()
    if not args.no_cheb2d:
        line["cheb2d"] = bench_cheb2d()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
