"""GPU parity of the low-statistical-dimension route (Algorithms 3 and 4).

The preconditioner R_i^{-1} = lam_i^{-1/2} (I - V_i S_i V_i^T) is built from the
SVD of one Gaussian sketch (QR of the sketch's transpose + one-sided Jacobi on
the GPU) and truncated per lambda to s_i = alpha ceil(sd_hat(lam_i)).  The SVD,
the estimates and the dense preconditioners are compared with the oracle's
(numpy SVD of the same downloaded sketch); the solutions with the oracle's
direct QR solve.  Every call goes through the C ABI.
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


def _lowrank(plist, s=None, alpha=2.0, seed=0, sketch_dtype=tik.F64):
    pr = tik.Problems.from_numpy([p.A for p in plist], [p.b for p in plist])
    s = s or [p.s for p in plist]
    sk = tik.sketch(pr, tik.GAUSS, s, seed, sketch_dtype=sketch_dtype)
    lams = np.stack([p.lams for p in plist])
    pc = tik.precond(sk, lams, tik.ROUTE_LOWRANK, alpha)
    return pr, sk, pc


@pytest.fixture(scope="module")
def small():
    # sigma_i = exp(-i/50), n = 1500: sd_{1e-3} ~ 173, s = 2 * 173 = 346
    return W.lowsd(m=6000, n=1500, N=8, decay=50.0, lam_lo=1e-3, lam_hi=1e-1)


def _check_ranks(pc, sig_o, lams, alpha, s, k=0):
    for i, lam in enumerate(lams):
        want = oracle.lowrank_truncation(sig_o, lam, alpha, s)
        got = pc.rank(k, i)
        if got != want:
            # the rank is an integer decided in FP64 from slightly different
            # singular values: it may only differ where sd_hat sits on a boundary
            sd = oracle.sd_hat(sig_o, lam)
            assert abs(sd - round(sd)) < 1e-9 and abs(got - want) <= math.ceil(alpha), (i, got, want)


@contextlib.contextmanager
def cholqr(value):
    old = tik.get_option("cholqr_panels")
    tik.set_option("cholqr_panels", value)
    try:
        yield
    finally:
        tik.set_option("cholqr_panels", old)


@pytest.mark.parametrize("panels", [1, 0])
def test_svd_and_preconditioner_match_oracle(small, panels):
    """panels = 1: QR panels by Cholesky QR and reflector reconstruction; 0: one launch per column."""
    p = small
    with cholqr(panels):
        pr, sk, pc = _lowrank([p])
    Y = sk.Y(0)
    s, n = Y.shape
    assert (s, n) == (p.s, p.n)
    sig_o, V_o = oracle.lowrank_factors(Y)
    sig = pc.sigma(0)
    print("sigma[0] %.6e sigma[-1] %.3e  max |dsigma| / sigma_0 = %.2e"
          % (sig[0], sig[-1], np.max(np.abs(sig - sig_o)) / sig_o[0]))
    assert np.all(np.diff(sig) <= 0)
    assert np.max(np.abs(sig - sig_o)) <= 1e-12 * sig_o[0]
    # estimates and ranks (Section 3.1.2, Algorithm 3 steps 5-7)
    sd_o = np.array([oracle.sd_hat(sig_o, l) for l in p.lams])
    assert np.allclose(pc.sd_hat[0], sd_o, rtol=1e-11, atol=0)
    _check_ranks(pc, sig_o, p.lams, 2.0, s)
    # V: orthonormal right singular vectors, Y v_j has norm sigma_j
    imax = int(np.argmax([pc.rank(0, i) for i in range(p.lams.size)]))
    V = pc.data(0, imax)
    r = V.shape[1]
    assert np.max(np.abs(V.T @ V - np.eye(r))) <= 1e-12
    assert np.max(np.abs(np.linalg.norm(Y @ V, axis=0) - sig[:r])) <= 1e-12 * sig[0]
    # the dense preconditioner of eq. RinvOver for every lambda
    for i, lam in enumerate(p.lams):
        si = pc.rank(0, i)
        Vi = pc.data(0, i)
        assert Vi.shape == (n, si)
        Rg = (np.eye(n) - (Vi * oracle.lowrank_S(sig[:si], lam)[None, :]) @ Vi.T) / math.sqrt(lam)
        Ro = oracle.lowrank_rinv(V_o, sig_o, lam, si)
        err = np.max(np.abs(Rg - Ro)) * math.sqrt(lam)
        assert err <= 1e-9, (i, err)


@pytest.mark.parametrize("mode", [tik.F64_BATCHED, tik.PLAIN_F64_PER_LAMBDA, tik.MIXED_BATCHED])
def test_lowrank_solve_tall(small, mode):
    p = small
    pr, sk, pc = _lowrank([p])
    tol = 1e-12 if mode != tik.MIXED_BATCHED else 1e-10
    res = tik.lsqr_batch(pr, pc, mode, tol, 300)
    torch.cuda.synchronize()
    err = oracle.rel_err(res.x_numpy(0), oracle.solve(p.A, p.b, p.lams))
    st = res.status.cpu().numpy()[0]
    its = res.iters.cpu().numpy()[0]
    print("lowrank tall mode", mode, "max rel err %.2e" % err.max(), "iters", its,
          "ranks", [pc.rank(0, i) for i in range(p.lams.size)])
    assert np.all(st == tik.ST_CONVERGED), st
    assert np.all(err <= (1e-10 if mode != tik.MIXED_BATCHED else 1e-8)), err
    if mode != tik.MIXED_BATCHED:
        assert its.max() <= 200, its


@pytest.mark.parametrize("mode", [tik.F64_BATCHED, tik.MIXED_BATCHED])
def test_lowrank_solve_wide(small, mode):
    """Algorithm 4: the same spectrum transposed, U_i of the sketch Y = A X."""
    rng = np.random.default_rng(21)
    A = np.asfortranarray(small.A.T)              # 1500 x 6000, FP32
    b = A.astype(np.float64) @ rng.standard_normal(A.shape[1]) + 1e-3 * rng.standard_normal(A.shape[0])
    p = W.Problem("lowsd_wide", A, b, small.lams, small.s, "gauss", "lowrank", 1e-10, 0)
    pr, sk, pc = _lowrank([p])
    assert sk.Y(0).shape == (p.s, p.m)
    tol = 1e-12 if mode != tik.MIXED_BATCHED else 1e-10
    res = tik.lsqr_batch(pr, pc, mode, tol, 300)
    torch.cuda.synchronize()
    err = oracle.rel_err(res.x_numpy(0), oracle.solve(p.A, p.b, p.lams))
    st = res.status.cpu().numpy()[0]
    print("lowrank wide mode", mode, "max rel err %.2e" % err.max(), "iters", res.iters.cpu().numpy()[0])
    assert np.all(st == tik.ST_CONVERGED), st
    assert np.all(err <= (1e-10 if mode != tik.MIXED_BATCHED else 1e-8)), err


def test_lowrank_ragged_batch_and_bf16_sketch():
    """Two problems of different sizes and sketch sizes in one batch; BF16 sketch."""
    plist = [W.lowsd(m=3000, n=700, N=6, decay=30.0, lam_lo=1e-3, lam_hi=3e-1, seed=1),
             W.lowsd(m=5000, n=1200, N=6, decay=60.0, lam_lo=2e-3, lam_hi=1e-1, seed=2)]
    assert plist[0].s != plist[1].s
    for sdt in (tik.F64, tik.BF16):
        pr, sk, pc = _lowrank(plist, sketch_dtype=sdt)
        for k, p in enumerate(plist):
            sig_o, _ = oracle.lowrank_factors(sk.Y(k))
            assert np.max(np.abs(pc.sigma(k) - sig_o)) <= 1e-12 * sig_o[0]
            _check_ranks(pc, sig_o, p.lams, 2.0, p.s, k)
        res = tik.lsqr_batch(pr, pc, tik.F64_BATCHED, 1e-12, 300)
        torch.cuda.synchronize()
        st = res.status.cpu().numpy()
        for k, p in enumerate(plist):
            err = oracle.rel_err(res.x_numpy(k), oracle.solve(p.A, p.b, p.lams))
            print("ragged lowrank", sdt, k, "max rel err %.2e" % err.max(), res.iters.cpu().numpy()[k])
            assert np.all(err <= 1e-10), err
        assert np.all(st == tik.ST_CONVERGED), st


def test_lowrank_degenerate_inputs():
    rng = np.random.default_rng(3)
    good = W.lowsd(m=2000, n=400, N=3, decay=20.0, lam_lo=1e-2, lam_hi=1e-1, seed=4)
    zero = W.Problem("zero", np.zeros((1500, 300), order="F"), rng.standard_normal(1500),
                     np.array([1e-2, 1e-1, 1.0]), 40, "gauss", "lowrank", 1e-10, 0)
    bad_A = np.asfortranarray(rng.standard_normal((1200, 200)))
    bad_A[5, 7] = np.nan
    bad = W.Problem("nan", bad_A, rng.standard_normal(1200), np.array([1e-2, 1e-1, 1.0]), 30,
                    "gauss", "lowrank", 1e-10, 0)
    plist = [good, zero, bad]
    # FP32 and FP64 storage cannot share a batch: solve the FP64 pair, then the FP32 one
    pr, sk, pc = _lowrank([zero, bad])
    st = pc.status
    assert np.all(st[0] == tik.ST_CONVERGED)          # A = 0: R^{-1} = lam^{-1/2} I
    assert [pc.rank(0, i) for i in range(3)] == [0, 0, 0]
    assert np.all(st[1] == tik.ST_NOTPD)              # non-finite sketch: no preconditioner
    assert np.all(np.isnan(pc.sd_hat[1]))
    res = tik.lsqr_batch(pr, pc, tik.F64_BATCHED, 1e-12, 50)
    torch.cuda.synchronize()
    rs = res.status.cpu().numpy()
    assert np.all(rs[0] == tik.ST_CONVERGED)
    assert np.all(res.x_numpy(0) == 0.0)              # A^T b = 0
    assert np.all(rs[1] == tik.ST_NOTPD)
    pr, sk, pc = _lowrank([good])
    res = tik.lsqr_batch(pr, pc, tik.F64_BATCHED, 1e-12, 300)
    torch.cuda.synchronize()
    err = oracle.rel_err(res.x_numpy(0), oracle.solve(good.A, good.b, good.lams))
    assert np.all(err <= 1e-10), err
    del plist


def test_lowrank_argument_errors(small):
    p = small
    pr = tik.Problems.from_numpy([p.A], [p.b])
    sk = tik.sketch(pr, tik.GAUSS, [p.s], 0)
    with pytest.raises(tik.TikError) as e:
        tik.precond(sk, p.lams, tik.ROUTE_LOWRANK, 0.5)      # alpha < 1
    assert e.value.rc == tik.EINVAL
    sk2 = tik.sketch(pr, tik.GAUSS, [p.n + 8], 0)          # s > n: nothing to truncate
    with pytest.raises(tik.TikError) as e:
        tik.precond(sk2, p.lams, tik.ROUTE_LOWRANK, 2.0)
    assert e.value.rc == tik.EINVAL
    pc = tik.precond(sk, p.lams, tik.ROUTE_CHOL)
    with pytest.raises(tik.TikError):
        pc.sigma(0)                                          # Cholesky route keeps no SVD


def test_svd_rank_deficient_sketch_mixes_panel_paths():
    """A of exact rank 10 and a sketch of 64 rows: the first QR panel (32 columns
    of rank 10) has a singular scaled Gram matrix and is factored column by
    column; the later panels hold rounding-level residuals and take the
    Cholesky QR path.  The singular values still match numpy's SVD of the same
    downloaded sketch, V stays orthonormal, and the solutions match the oracle."""
    rng = np.random.default_rng(7)
    m, n, r, N = 3000, 400, 10, 4
    Ua = np.linalg.qr(rng.standard_normal((m, r)))[0]
    Va = np.linalg.qr(rng.standard_normal((n, r)))[0]
    A = np.asfortranarray((Ua * np.logspace(0, -3, r)[None, :]) @ Va.T)
    b = A @ rng.standard_normal(n) + 1e-3 * rng.standard_normal(m)
    lams = np.logspace(-4, -1, N)
    p = W.Problem("rank10", A, b, lams, 64, "gauss", "lowrank", 1e-10, 0)
    tik.prof_reset()
    tik.prof_enable(True)
    try:
        pr, sk, pc = _lowrank([p])
        col_panels = tik.prof_query("lr_colqr")[1]
        cqr_panels = tik.prof_query("lr_cqr_recon")[1]
    finally:
        tik.prof_enable(False)
    print("panels: column by column", col_panels, "Cholesky QR", cqr_panels)
    assert col_panels >= 1 and cqr_panels >= 1
    Y = sk.Y(0)
    sig_o = np.linalg.svd(Y, compute_uv=False)
    sig = pc.sigma(0)
    print("sigma", sig[:12], "max |dsigma| / sigma_0 = %.2e" % (np.max(np.abs(sig - sig_o)) / sig_o[0]))
    assert np.max(np.abs(sig - sig_o)) <= 1e-12 * sig_o[0]
    assert np.all(sig[r:] <= 1e-12 * sig[0])
    V = pc.data(0, int(np.argmax([pc.rank(0, i) for i in range(N)])))
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) <= 1e-12
    res = tik.lsqr_batch(pr, pc, tik.F64_BATCHED, 1e-13, 300)
    err = oracle.rel_err(res.x_numpy(0), oracle.solve(A, b, lams))
    assert np.all(res.status.cpu().numpy() == tik.ST_CONVERGED)
    assert np.all(err <= 1e-10), err
