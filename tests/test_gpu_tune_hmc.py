"""The trajectory autotuner (gp_tune_hmc): it picks the persistent kernel's register allocation
(waves per SIMD) and the product jobs' columns per trip for a batch class, and no choice changes
any result, so a tuned trajectory equals the default one bit for bit."""
import numpy as np
import pytest
import torch

from paper_2412_20884_amd import gpk, inputs as I
from tests.gpu_util import DEV, host, rounded, to_dev

pytestmark = pytest.mark.gpu


def batch(specs, chains, dtype, seed, kind="ard"):
    ns = [n for n, _ in specs]
    ds = [d for _, d in specs]
    Xs, ys, ths = [], [], []
    for s, (n, d) in enumerate(specs):
        p = I.ard_problem(n, d, seed + s, lo=0.5, hi=3.0, sigma2=0.1)
        Xs.append(rounded(p["X"], dtype).ravel())
        ys.append(rounded(p["y"], dtype))
        ths.append(np.concatenate([p["theta"]] * chains))
    g = np.random.default_rng(seed)
    phi = np.concatenate([g.normal(size=n * chains) * 0.3 for n in ns])
    pi = g.normal(size=sum(len(t) for t in ths)) * 0.3
    return ns, ds, np.concatenate(Xs), np.concatenate(ys), phi, np.concatenate(ths), pi


def run(b, chains, dtype, mode, prec=None):
    ns, ds, X, y, phi, th, pi = b
    offs = np.cumsum([0] + ns[:-1])
    xoffs = np.cumsum([0] + [n * d for n, d in zip(ns, ds)][:-1])
    thd, pid = to_dev(th, torch.float64), to_dev(pi, torch.float64)
    xd = torch.zeros(sum(ns) * chains, dtype=dtype, device=DEV)
    u = to_dev(np.full(len(ns) * chains, 0.5), torch.float64)
    r = gpk.hmc_leapfrog(to_dev(X, dtype).reshape(-1, 1), to_dev(y, dtype), to_dev(phi, dtype), thd,
                         pid, xd, "ard", ns, offs, chains, d=ds, x_offsets=xoffs, u=u, n_steps=3,
                         dt=2e-3, cg_tol=1e-6, cg_maxit=2000, mode=mode, prec=prec)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items() if v is not None}
    out["theta"], out["pi"], out["x"] = host(thd), host(pid), host(xd)
    return out


@pytest.mark.parametrize("dtype,prec,specs", [
    (torch.float32, None, [(1500, 3), (900, 6), (700, 16)]),
    (torch.float64, None, [(800, 2), (600, 5)]),
    (torch.float32, "bf16x", [(1100, 40)]),
])
def test_tuned_trajectory_equals_default(tmp_path, dtype, prec, specs):
    saved = tmp_path / "table.json"
    gpk.tune_save(saved)
    try:
        gpk.tune_clear()
        chains = 2
        b = batch(specs, chains, dtype, 70)
        ref = {m: run(b, chains, dtype, m, prec) for m in (gpk.BATCHED, gpk.GRAPH)}
        n = gpk.tune_hmc("ard", [n for n, _ in specs], chains, [d for _, d in specs], dtype=dtype,
                         prec=prec)
        assert n == 1
        text = (tmp_path / "after.json")
        gpk.tune_save(text)
        assert '"op": 2' in text.read_text()
        for m in (gpk.BATCHED, gpk.GRAPH):
            got = run(b, chains, dtype, m, prec)
            for key in ("theta", "pi", "H0", "H1", "accepted", "status", "x", "cg_iters"):
                np.testing.assert_array_equal(got[key], ref[m][key], err_msg=key)
        assert np.all(ref[gpk.BATCHED]["status"] == 0)
    finally:
        gpk.tune_clear()
        gpk.tune_load(saved)
