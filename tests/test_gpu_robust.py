"""Robustness variants on the GPU, through the C ABI, against the oracle:

* the breakdown fallback of the Cholesky route: where chol(C + lam I) breaks
  down, R comes from the Householder QR of [Y; sqrt(lam) I] (the BP2
  preconditioner of Section 4.1), forced from the host with a pivot
  threshold on a well-conditioned problem, and met naturally where
  kappa(C + lam I) exceeds 1/u;
* the blind statistical-dimension workflow of Section 3.1.2: an oversized
  sketch whose size knows nothing of sd, sd_hat from its singular values,
  each lambda truncated to s_i = alpha ceil(sd_hat_i), then (Algorithm 3
  step 1 with the estimate) a second sketch of size alpha ceil(sd_hat_N).
"""

import contextlib
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2203_07329_amd import tik

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def option(name, value):
    old = tik.get_option(name)
    tik.set_option(name, value)
    try:
        yield
    finally:
        tik.set_option(name, old)


def test_qr_fallback_forced_from_host():
    p = W.over_svd()                                       # 2000 x 100, N = 10, SRHT s = 400
    pr = tik.Problems.from_numpy([p.A], [p.b])
    sk = tik.sketch(pr, tik.SRHT, [p.s], 3)
    with option("chol_pivot_ulps", 1 << 50):               # a pivot below 1/8 of its diagonal breaks down
        pq = tik.precond(sk, p.lams)
    st = pq.status[0]
    print("precond status with the forced threshold:", st)
    assert not np.any(st == tik.ST_NOTPD)
    qi = np.flatnonzero(st == tik.ST_QR)
    assert qi.size >= 3, st
    Y = sk.Y(0)
    for i in qi:
        Ri = pq.data(0, i)
        assert np.array_equal(np.tril(Ri, -1), np.zeros_like(Ri))
        Ro = oracle.bp2_precond(Y, p.lams[i])
        Ri_pos = Ri * np.sign(np.diag(Ri))[None, :]       # the QR's diagonal signs, absorbed
        ref = np.linalg.inv(Ro)
        assert np.linalg.norm(Ri_pos - ref) <= 1e-13 * np.linalg.cond(Ro) * np.linalg.norm(ref), i
    res = tik.lsqr_batch(pr, pq, tik.F64_BATCHED, 1e-13, 300)
    torch.cuda.synchronize()
    assert np.all(res.status.cpu().numpy() == tik.ST_CONVERGED)
    Xo = oracle.solve(p.A, p.b, p.lams)
    err = oracle.rel_err(res.x_numpy(0), Xo)
    print("QR-route errors", err)
    assert np.all(err <= 1e-10), err
    # the Cholesky factors of the same sketch solve the same problems
    pc = tik.precond(sk, p.lams)
    assert np.all(pc.status == tik.ST_CONVERGED)
    rc = tik.lsqr_batch(pr, pc, tik.F64_BATCHED, 1e-13, 300)
    assert np.all(oracle.rel_err(res.x_numpy(0), rc.x_numpy(0)) <= 1e-10)


@pytest.mark.parametrize("mode", [tik.F64_BATCHED, tik.MIXED_BATCHED])
def test_qr_fallback_natural_breakdown(mode):
    """sigma down to 1e-10 and lambda <= 1e-20: kappa(C + lam I) >= 1e19, so the
    Cholesky factorization of the sketched Gram matrix breaks down; the QR route
    still gives a good preconditioner.  kappa(B) is 1e10 here, so no method reaches
    1e-10: the bar is the oracle's own distance to the closed form."""
    p = W.over_svd(m=2000, n=100, N=4, sig_lo=1e-10, lam_lo=1e-26, lam_hi=1e-20)
    pr = tik.Problems.from_numpy([p.A], [p.b])
    sk = tik.sketch(pr, tik.SRHT, [p.s], 5)
    pc = tik.precond(sk, p.lams)
    st = pc.status[0]
    print("precond status:", st)
    assert not np.any(st == tik.ST_NOTPD)
    assert np.any(st == tik.ST_QR)
    res = tik.lsqr_batch(pr, pc, mode, 1e-14, 300)
    torch.cuda.synchronize()
    assert np.all(res.status.cpu().numpy() == tik.ST_CONVERGED)
    X = res.x_numpy(0)
    Xo = oracle.solve(p.A, p.b, p.lams)
    c = p.U.T @ p.b
    Xc = np.stack([p.V @ (p.sigma / (p.sigma ** 2 + lam) * c) for lam in p.lams], axis=1)
    err, ref = oracle.rel_err(X, Xo), oracle.rel_err(Xo, Xc)
    print("iterations", res.iters.cpu().numpy()[0], "err vs oracle", err, "oracle vs closed form", ref)
    assert np.all(err <= 10 * np.maximum(ref, 1e-12)), (err, ref)


def test_blind_sd_workflow():
    """Section 3.1.2 on a reduced low-statistical-dimension workload: the sketch
    size is chosen without sd (s0 = min(m, n)); sd_hat and s_i come from the
    sketch's singular values only; a second sketch of size alpha ceil(sd_hat at
    the smallest lambda) gives the same solutions."""
    p = W.lowsd(m=20000, n=2000, N=8, decay=40.0, lam_lo=1e-4, lam_hi=1e-1)
    alpha = 2.0
    pr = tik.Problems.from_numpy([p.A], [p.b])
    s0 = min(p.m, p.n, 4096)
    sk = tik.sketch(pr, tik.GAUSS, [s0], 11, sketch_dtype=tik.BF16)
    pc = tik.precond(sk, p.lams, tik.ROUTE_LOWRANK, alpha)
    sig = pc.sigma(0)
    sdh = pc.sd_hat[0]
    sd_true = np.array([oracle.statistical_dimension(p.sigma, lam) for lam in p.lams])
    print("sd_hat", np.round(sdh, 1), "sd", np.round(sd_true, 1))
    assert np.all(np.abs(sdh - sd_true) <= 0.05 * sd_true)
    for i, lam in enumerate(p.lams):
        assert abs(sdh[i] - oracle.sd_hat(sig, lam)) <= 1e-10 * sdh[i]
        # the rank: an integer decided in FP64 from the same singular values on
        # both sides; summation order may differ only where sd_hat sits on an integer
        want = oracle.lowrank_truncation(sig, lam, alpha, s0)
        got = pc.rank(0, i)
        sd_o = oracle.sd_hat(sig, lam)
        assert got == want or (abs(sd_o - round(sd_o)) < 1e-9 and abs(got - want) <= math.ceil(alpha)), \
            (i, got, want)
        assert got < s0
    Xo = oracle.solve(p.A, p.b, p.lams)
    r0 = tik.lsqr_batch(pr, pc, tik.MIXED_BATCHED, 1e-10, 300)
    e0 = oracle.rel_err(r0.x_numpy(0), Xo)
    # second sketch, sized from the estimate (Algorithm 3 step 1)
    s1 = int(math.ceil(alpha * math.ceil(sdh.max())))
    assert abs(s1 - alpha * math.ceil(sd_true.max())) <= 0.05 * s1
    sk1 = tik.sketch(pr, tik.GAUSS, [s1], 12, sketch_dtype=tik.BF16)
    pc1 = tik.precond(sk1, p.lams, tik.ROUTE_LOWRANK, alpha)
    r1 = tik.lsqr_batch(pr, pc1, tik.MIXED_BATCHED, 1e-10, 300)
    e1 = oracle.rel_err(r1.x_numpy(0), Xo)
    print("s0", s0, "s1", s1, "errors", e0.max(), e1.max(), "iterations", r0.iters.cpu().numpy().max(),
          r1.iters.cpu().numpy().max())
    assert np.all(e0 <= 1e-8) and np.all(e1 <= 1e-8)
    assert np.all(r0.status.cpu().numpy() == tik.ST_CONVERGED)
    assert np.all(r1.status.cpu().numpy() == tik.ST_CONVERGED)
