"""tik_lsqr_batch_static (static device workspace, nothing allocated) against
tik_lsqr_batch on the same inputs, through the C ABI: two calls in a row, the
second with a smaller problem, and the size limit."""

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2203_07329_amd import tik

pytestmark = pytest.mark.gpu


def _setup(plist, embed, s=None, route=tik.ROUTE_CHOL):
    pr = tik.Problems.from_numpy([p.A for p in plist], [p.b for p in plist])
    sk = tik.sketch(pr, embed, s or [p.s for p in plist], 2)
    pc = tik.precond(sk, np.stack([p.lams for p in plist]), route, 2.0)
    return pr, sk, pc


@pytest.mark.parametrize("mode", [tik.F64_BATCHED, tik.MIXED_BATCHED])
def test_static_matches_workspace_call(mode):
    cases = [
        [W.over_svd(m=2000, n=100, N=10)],                                  # larger first
        W.ragged(nprob=3, m_lo=400, m_hi=900, n_lo=10, n_hi=40, N=4),       # then smaller
    ]
    for plist in cases:
        embed = tik.SRHT if plist[0].A.dtype == np.float64 else tik.GAUSS
        pr, sk, pc = _setup(plist, embed)
        ref = tik.lsqr_batch(pr, pc, mode, 1e-12, 300)
        got = tik.lsqr_batch_static(pr, pc, mode, 1e-12, 300)
        torch.cuda.synchronize()
        assert np.array_equal(got.status.cpu().numpy(), ref.status.cpu().numpy())
        assert np.array_equal(got.iters.cpu().numpy(), ref.iters.cpu().numpy())
        for k, p in enumerate(plist):
            Xg, Xr = got.x_numpy(k), ref.x_numpy(k)
            assert np.max(oracle.rel_err(Xg, Xr)) <= 1e-12
            print("problem", k, "bitwise equal to the workspace call:", np.array_equal(Xg, Xr))
            Xo = oracle.solve(p.A, p.b, p.lams)
            tolerance = 1e-10 if mode == tik.F64_BATCHED else 1e-8
            assert np.all(oracle.rel_err(Xg, Xo) <= tolerance)


def test_static_rejects_large_solves():
    # m * N * 8 bytes of one long vector alone exceed the 64 MiB array
    rng = np.random.default_rng(0)
    m, n, N = 300000, 8, 32
    A = np.asfortranarray(rng.standard_normal((m, n)).astype(np.float32))
    b = rng.standard_normal(m)
    pr = tik.Problems.from_numpy([A], [b])
    sk = tik.sketch(pr, tik.GAUSS, [4 * n], 0)
    pc = tik.precond(sk, np.logspace(-6, -1, N)[None, :])
    with pytest.raises(tik.TikError) as e:
        tik.lsqr_batch_static(pr, pc, tik.F64_BATCHED, 1e-10, 50)
    assert e.value.rc == tik.ENOTSUP and "static workspace" in str(e.value)
