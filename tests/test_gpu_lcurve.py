"""The L-curve of Section 4.3 on the GPU (tik_lcurve, tik_lcurve_corner) against
the oracle: both norms elementwise and the corner index, through the C ABI."""

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2203_07329_amd import tik

pytestmark = pytest.mark.gpu


def _solve(plist, embed, s=None, tol=1e-13, mode=tik.F64_BATCHED):
    pr = tik.Problems.from_numpy([p.A for p in plist], [p.b for p in plist])
    sk = tik.sketch(pr, embed, s or [p.s for p in plist], 1)
    pc = tik.precond(sk, np.stack([p.lams for p in plist]))
    res = tik.lsqr_batch(pr, pc, mode, tol, 400)
    torch.cuda.synchronize()
    return pr, res


CASES = {
    # the 2000 x 100 workload (N = 10, lambda 1e-6..1: the corner is interior)
    "over_svd": lambda: ([W.over_svd()], tik.SRHT, None),
    # FP32 problems of uneven size, several column chunks for the wider ones
    "ragged": lambda: (W.ragged(nprob=5, m_lo=600, m_hi=4000, n_lo=20, n_hi=300, N=8), tik.GAUSS, None),
    # a wide FP32 problem (Algorithm 2), its 6000 columns split over chunks
    "wide": lambda: ([W.under_scaled(m=50, n=6000, N=12)], tik.GAUSS, [200]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_lcurve_norms_and_corner(case):
    plist, embed, s = CASES[case]()
    pr, res = _solve(plist, embed, s)
    xn, rn = tik.lcurve(pr, res.X)
    xn, rn = xn.cpu().numpy(), rn.cpu().numpy()
    for k, p in enumerate(plist):
        X = res.x_numpy(k)
        # the norm computation itself: the same x on the host
        hx, hr = oracle.lcurve_norms(p.A, p.b, X)
        assert np.allclose(xn[k], hx, rtol=1e-13, atol=0), (k, xn[k], hx)
        # b - A x cancels where the residual is small: both sides' rounding is
        # then of the order u (||b|| + ||A||_F ||x||), far above u ||A x - b||
        floor = 1e-13 * (np.linalg.norm(p.b) + np.linalg.norm(p.A.astype(np.float64)) * hx)
        assert np.all(np.abs(rn[k] - hr) <= 1e-12 * hr + floor), (k, rn[k], hr)
        # against the oracle's own solutions
        ox, orr = oracle.lcurve_norms(p.A, p.b, oracle.solve(p.A, p.b, p.lams))
        ex, er = np.abs(xn[k] - ox) / ox, np.abs(rn[k] - orr) / orr
        print(case, k, "max rel err ||x|| %.2e ||Ax-b|| %.2e" % (ex.max(), er.max()))
        assert np.all(ex <= 1e-10) and np.all(er <= 1e-10)
        if p.lams.size >= 3:
            c, _ = tik.lcurve_corner(p.lams, xn[k], rn[k])
            assert c == oracle.lcurve_corner(p.lams, ox, orr), (k, c)


def test_lcurve_rejects_mixed_storage():
    a = W.over_svd(m=300, n=20, N=3)
    bq = W.ragged(nprob=1, m_lo=300, m_hi=301, n_lo=20, n_hi=21, N=3)[0]
    pr = tik.Problems.from_numpy([a.A, bq.A], [a.b, bq.b])
    X = [torch.zeros((3, 20), dtype=torch.float64, device="cuda") for _ in range(2)]
    with pytest.raises(tik.TikError):
        tik.lcurve(pr, X)
