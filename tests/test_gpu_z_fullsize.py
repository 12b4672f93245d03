"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

For every workload bench.py can time, the batched solve runs exactly as the
benchmark runs it (same generator, sketch, route, mode and tolerance, from
bench.build_workload / bench.pick_mode) and is checked against the CPU oracle:
the whole batch where the oracle's direct QR solve takes seconds, every 16th
problem of the ragged batch, and an a-posteriori error bound (gradient in
extended precision, refined with the generator's planted factors) for the
100000 x 10000 low-rank workload, whose direct solve takes minutes.
"""

import sys
import time

import numpy as np
import pytest
import torch

import bench
import oracle
import workloads as W
from paper_2203_07329_amd import tik

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL_MIXED = 1e-8     # target forward error of the mixed mode
TOL_F64 = 1e-10      # target forward error of the FP64 path


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _run(name, mode_pref=None, tol=None):
    t0 = time.perf_counter()
    plist, cfg = bench.build_workload(name, tik, W, "cuda:0")
    say(f"[{name}] generated {len(plist)} problem(s) in {time.perf_counter() - t0:.1f}s")
    pr = tik.Problems.from_numpy([p.A for p in plist], [p.b for p in plist])
    lams = np.stack([p.lams for p in plist])
    svec = [p.s for p in plist]
    mode, btol = bench.pick_mode(tik, pr, cfg, svec, lams, plist[0].alpha, mode_pref or cfg["mode"])
    sk = tik.sketch(pr, cfg["embed"], svec, 0, sketch_dtype=cfg["sdt"])
    pc = tik.precond(sk, lams, cfg["route"], plist[0].alpha)
    res = tik.Solver(pr, pc, mode)(tol or btol, bench.MAXIT)
    torch.cuda.synchronize()
    st = res.status.cpu().numpy()
    Xs = [res.x_numpy(k) for k in range(len(plist))]
    say(f"[{name}] mode {mode} solved; iterations max {res.iters.cpu().numpy().max()}")
    return plist, cfg, mode, Xs, st


def _check(name, plist, cfg, Xs, bound):
    if cfg["check"] == "certify":
        p = plist[0]
        t0 = time.perf_counter()
        err = oracle.certify_planted(p.A, p.b, p.lams, Xs[0], p.sigma, p.V)
        say(f"[{name}] certified in {time.perf_counter() - t0:.1f}s: max bound {err.max():.2e}")
        assert np.all(err <= bound), err
        return
    idx = range(len(plist)) if cfg["check"] == "full" else range(0, len(plist), 16)
    worst = 0.0
    for k in idx:
        p = plist[k]
        err = oracle.rel_err(Xs[k], oracle.solve(p.A, p.b, p.lams))
        worst = max(worst, float(err.max()))
        assert np.all(err <= bound), (k, err)
    say(f"[{name}] {len(list(idx))} problem(s) checked against the oracle: max rel err {worst:.2e}")


@pytest.mark.parametrize("name", ["over_gauss", "under_scaled", "lowsd", "ragged"])
def test_fullsize_benchmark_configuration(name):
    plist, cfg, mode, Xs, st = _run(name)
    assert np.all(st == tik.ST_CONVERGED), st
    _check(name, plist, cfg, Xs, TOL_MIXED)


def test_fullsize_over_gauss_fp64_batched():
    """The FP64 path at its target forward error: kappa(A) = 1e8, N = 32."""
    plist, cfg, mode, Xs, st = _run("over_gauss", "f64", tol=1e-13)
    assert mode == tik.F64_BATCHED
    assert np.all(st <= tik.ST_MAXIT), st
    _check("over_gauss f64", plist, cfg, Xs, TOL_F64)
