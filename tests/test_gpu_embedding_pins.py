"""Quality pins on the GPU's own embedding X, through the C ABI.

* The SRHT is compared with an explicit Sylvester Hadamard matrix applied with
  the signs and sampled rows regenerated on the host from the seed (Philox4x32-10
  written from its published definition, tests/philox_ref.py, and the same
  Feistel permutation restated from its definition): bit for bit on integer
  inputs, whose transforms are exact.
* Lemma 2.1 (tall Cholesky route), its underdetermined counterpart of Section
  2.2, Theorem 3.2 (low-rank route, Algorithm 3) and the theorem of Section
  3.3.2 (Algorithm 4) are checked with the X the GPU used, extracted by
  sketching the identity with the same seed, and the preconditioners the GPU
  built from it.
"""

import math

import numpy as np
import pytest
from scipy.linalg import hadamard

import oracle
import workloads as W
from paper_2203_07329_amd import tik
from philox_ref import philox4x32_10

pytestmark = pytest.mark.gpu

TAG_PERM, TAG_SIGN = 0x5052504D, 0x5349474E


def _key(seed):
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)


def _feistel(x, k, key):
    """Bijection of [0, 2^k): a balanced Feistel network on 2h bits (h = ceil(k/2))
    with six Philox round functions, restricted to [0, 2^k) by cycle walking."""
    h = (k + 1) >> 1
    mask = (1 << h) - 1
    for _ in range((1 << k) + 1):
        L, R = x >> h, x & mask
        for r in range(6):
            f = int(philox4x32_10(np.array([[R, r, TAG_PERM, k]], dtype=np.uint32), key)[0, 0]) & mask
            L, R = R, L ^ f
        x = (L << h) | R
        if x < (1 << k):
            return x
    raise AssertionError("cycle walk did not end")


def srht_host(A, s, seed):
    """(1/sqrt(s)) S H D [A; 0] with H the +-1 Sylvester Hadamard matrix of order m'."""
    m = A.shape[0]
    k = max(0, int(math.ceil(math.log2(m))))
    mp = 1 << k
    key = _key(seed)
    rows = np.sort([0 if k == 0 else _feistel(i, k, key) for i in range(s)])
    words = (mp + 31) >> 5
    w = np.arange(words)
    ctr = np.stack([w >> 2, np.zeros(words), np.full(words, TAG_SIGN), np.zeros(words)], axis=1).astype(np.uint32)
    out = philox4x32_10(ctr, key)
    bits = out[np.arange(words), w & 3].astype(np.uint64)
    neg = ((bits[np.arange(mp) >> 5] >> (np.arange(mp) & 31).astype(np.uint64)) & np.uint64(1)).astype(bool)
    Ap = np.zeros((mp, A.shape[1]))
    Ap[:m] = A
    Ap[neg] *= -1.0
    return rows, (1.0 / math.sqrt(s)) * (hadamard(mp).astype(np.float64) @ Ap)[rows]


def test_host_philox_known_answers():
    """The published known-answer vectors of Philox4x32-10 (Random123)."""
    kat = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
           ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for c, k, want in kat:
        got = philox4x32_10(np.array([c], dtype=np.uint32), np.array(k, dtype=np.uint32))[0]
        assert [int(v) for v in got] == list(want)


@pytest.mark.parametrize("m,n,s,seed", [(1000, 6, 64, 5), (4096, 3, 200, 17), (3000, 4, 123, 2**40 + 9)])
def test_srht_equals_explicit_sylvester(m, n, s, seed):
    rng = np.random.default_rng(m)
    A = rng.integers(-8, 9, size=(m, n)).astype(np.float64)      # integer data: exact transforms
    pr = tik.Problems.from_numpy([A], [np.ones(m)])
    Y = tik.sketch(pr, tik.SRHT, [s], seed).Y(0)
    rows, Yh = srht_host(A, s, seed)
    assert len(set(rows.tolist())) == s
    assert np.array_equal(Y, Yh)


def _signs_rows(m, s, seed):
    k = max(0, int(math.ceil(math.log2(m))))
    mp = 1 << k
    key = _key(seed)
    rows = np.sort([0 if k == 0 else _feistel(i, k, key) for i in range(s)])
    words = (mp + 31) >> 5
    w = np.arange(words)
    ctr = np.stack([w >> 2, np.zeros(words), np.full(words, TAG_SIGN), np.zeros(words)], axis=1).astype(np.uint32)
    bits = philox4x32_10(ctr, key)[np.arange(words), w & 3].astype(np.uint64)
    neg = ((bits[np.arange(mp) >> 5] >> (np.arange(mp) & 31).astype(np.uint64)) & np.uint64(1)).astype(bool)
    return mp, rows, neg


def srht_host_sylvester(A, s, seed):
    """The same sketch through Sylvester's recursion H_2h = [[H_h, H_h], [H_h, -H_h]]
    applied level by level to the padded, sign-flipped columns (exact on integers);
    for orders whose explicit matrix does not fit in memory."""
    m = A.shape[0]
    mp, rows, neg = _signs_rows(m, s, seed)
    Z = np.zeros((mp, A.shape[1]))
    Z[:m] = A
    Z[neg] *= -1.0
    h = 1
    while h < mp:
        V = Z.reshape(mp // (2 * h), 2, h, -1)
        top, bot = V[:, 0].copy(), V[:, 1].copy()
        V[:, 0] = top + bot
        V[:, 1] = top - bot
        h *= 2
    return rows, (1.0 / math.sqrt(s)) * Z[rows]


@pytest.mark.parametrize("m,n,s,seed,f32", [(20000, 256, 300, 3, False), (40000, 260, 5000, 11, True),
                                            (16384, 300, 8192, 2**33 + 1, False)])
def test_srht_column_resident_equals_sylvester(m, n, s, seed, f32):
    """The column-resident transform (m' >= 2^14, n >= 256, s <= 8192: one
    workgroup per column, buckets of 2^14 rows) on integer data: identical to the
    host's Sylvester recursion and to the two-pass transform, for a partial last
    bucket, a bucket wholly past m, FP32 storage and both register layouts of the
    sampled rows (s <= 4096 and s up to 8192)."""
    rng = np.random.default_rng(m + n)
    A = rng.integers(-8, 9, size=(m, n)).astype(np.float32 if f32 else np.float64)
    pr = tik.Problems.from_numpy([A], [np.ones(m)])
    old = tik.get_option("srht_cols")
    try:
        tik.set_option("srht_cols", 1)
        Y1 = tik.sketch(pr, tik.SRHT, [s], seed).Y(0)
        tik.set_option("srht_cols", 0)
        Y0 = tik.sketch(pr, tik.SRHT, [s], seed).Y(0)
    finally:
        tik.set_option("srht_cols", old)
    rows, Yh = srht_host_sylvester(A.astype(np.float64), s, seed)
    assert len(set(rows.tolist())) == s
    assert np.array_equal(Y1, Yh)
    assert np.array_equal(Y0, Yh)


def test_srht_column_resident_rounding_matches_two_pass():
    """On real-valued data the two transforms sum in different orders: the
    sketches agree to a few ulps of the column norms."""
    m, n, s = 30000, 256, 2000
    rng = np.random.default_rng(5)
    A = rng.standard_normal((m, n)) * np.logspace(0, -8, n)[None, :]
    pr = tik.Problems.from_numpy([A], [np.ones(m)])
    old = tik.get_option("srht_cols")
    try:
        tik.set_option("srht_cols", 1)
        Y1 = tik.sketch(pr, tik.SRHT, [s], 9).Y(0)
        tik.set_option("srht_cols", 0)
        Y0 = tik.sketch(pr, tik.SRHT, [s], 9).Y(0)
    finally:
        tik.set_option("srht_cols", old)
    scale = np.linalg.norm(A, axis=0) * math.sqrt(1 << 15) / math.sqrt(s)
    err = np.max(np.abs(Y1 - Y0) / scale[None, :])
    print("max |Y_cols - Y_twopass| / (column scale) = %.2e" % err)
    assert err <= 1e-14


def _extract_X(m, s, embed, seed, sdt=tik.F64):
    I = np.eye(m)
    pr = tik.Problems.from_numpy([I], [np.ones(m)])
    return tik.sketch(pr, embed, [s], seed, sketch_dtype=sdt).Y(0)


@pytest.mark.parametrize("embed", [tik.SRHT, tik.GAUSS])
def test_lemma21_with_gpu_embedding(embed):
    p = W.over_svd(m=1024, n=60, N=4, sig_lo=1e-8, lam_lo=1e-12, lam_hi=1e-2)
    s, seed = 240, 21
    X = _extract_X(p.m, s, embed, seed)
    pr = tik.Problems.from_numpy([p.A], [p.b])
    sk = tik.sketch(pr, embed, [s], seed)
    assert np.allclose(sk.Y(0), X @ p.A, rtol=1e-12, atol=1e-12 * np.abs(sk.Y(0)).max())
    pc = tik.precond(sk, p.lams)
    bound = oracle.lemma21_bound(X @ p.U)
    for i, lam in enumerate(p.lams):
        B = np.vstack([p.A, math.sqrt(lam) * np.eye(p.n)])
        k = np.linalg.cond(B @ pc.data(0, i))
        print("lambda %.0e kappa(B R^-1) %.4f Lemma 2.1 bound %.4f" % (lam, k, bound))
        assert k <= bound * (1 + 1e-6)


def test_thm32_with_gpu_embedding():
    """Theorem 3.2 with the GPU's Gaussian X and its untruncated low-rank R (alpha large)."""
    # sd_lam from 5.5 to 10.5 against s = 190: eps of Theorem 3.2 about 0.25 to 0.4
    p = W.over_svd(m=2000, n=200, N=3, sig_lo=1e-40, lam_lo=1e-4, lam_hi=1e-2)
    s, seed = 190, 8
    X = _extract_X(p.m, s, tik.GAUSS, seed)
    pr = tik.Problems.from_numpy([p.A], [p.b])
    sk = tik.sketch(pr, tik.GAUSS, [s], seed)
    pc = tik.precond(sk, p.lams, tik.ROUTE_LOWRANK, 1e6)
    sig = pc.sigma(0)
    for i, lam in enumerate(p.lams):
        assert pc.rank(0, i) == s
        V = pc.data(0, i)
        Rinv = oracle.lowrank_rinv(V, sig, lam)
        U1 = p.U * (p.sigma / np.sqrt(p.sigma ** 2 + lam))[None, :]
        eps = oracle.thm32_eps(U1, X)
        assert eps < 1
        B = np.vstack([p.A, math.sqrt(lam) * np.eye(p.n)])
        k = np.linalg.cond(B @ Rinv)
        print("lambda %.0e kappa %.4f Theorem 3.2 bound %.4f (eps %.3f)" % (lam, k, oracle.thm32_bound(eps), eps))
        assert k <= oracle.thm32_bound(eps) * (1 + 1e-6)


def _wide_X(m, n, s, seed):
    """X (n x s) of a wide sketch Y = A X, from sketches of [0 .. I_m .. 0]: rows jm..(j+1)m."""
    X = np.zeros((n, s))
    for j0 in range(0, n, m):
        w = min(m, n - j0)
        E = np.zeros((m, n))
        E[np.arange(w), j0 + np.arange(w)] = 1.0
        pr = tik.Problems.from_numpy([E], [np.ones(m)])
        Yt = tik.sketch(pr, tik.GAUSS, [s], seed).Y(0)       # s x m = (E X)^T
        X[j0:j0 + w] = Yt[:, :w].T
    return X


def test_wide_lemma_and_thm34_with_gpu_embedding():
    """Algorithm 2 (Cholesky, the underdetermined lemma of Section 2.2) and Algorithm 4
    (low rank, the theorem of Section 3.3.2) with the GPU's X of a wide sketch."""
    rng = np.random.default_rng(3)
    m, n = 50, 400
    U = W.haar(rng, m, m)
    VA = W.haar(rng, n, m)
    sigma = np.exp(-np.arange(m) / 5.0)
    A = np.asfortranarray((U * sigma) @ VA.T)
    b = A @ rng.standard_normal(n)
    s, seed = 48, 31
    X = _wide_X(m, n, s, seed)
    pr = tik.Problems.from_numpy([A], [b])
    sk = tik.sketch(pr, tik.GAUSS, [s], seed)
    assert np.allclose(sk.Y(0), (A @ X).T, rtol=1e-12, atol=1e-12 * np.abs(sk.Y(0)).max())
    lams = np.array([1e-6, 1e-3, 1e-1])
    s_chol = 160
    Xc = _wide_X(m, n, s_chol, seed)
    skc = tik.sketch(pr, tik.GAUSS, [s_chol], seed)
    pcc = tik.precond(skc, lams)
    bound = oracle.lemma21_bound(Xc.T @ VA)
    pcl = tik.precond(sk, lams, tik.ROUTE_LOWRANK, 1e6)
    sig = pcl.sigma(0)
    for i, lam in enumerate(lams):
        D = np.hstack([A, math.sqrt(lam) * np.eye(m)])
        kc = np.linalg.cond(pcc.data(0, i).T @ D)                    # R^{-T} D
        assert kc <= bound * (1 + 1e-6), (lam, kc, bound)
        Uy = pcl.data(0, i)                                          # left singular vectors of Y
        RiT = oracle.lowrank_rinv(Uy, sig, lam)
        VD = np.linalg.svd(D, full_matrices=False)[2].T
        V1 = VD[:n]
        eps = float(np.linalg.norm(V1.T @ X @ X.T @ V1 - V1.T @ V1, 2))
        kl = np.linalg.cond(RiT @ D)
        print("lambda %.0e chol kappa %.4f (bound %.4f); low rank kappa %.4f (bound %.4f, eps %.3f)"
              % (lam, kc, bound, kl, oracle.thm32_bound(eps) if eps < 1 else float("inf"), eps))
        if eps < 1:
            assert kl <= oracle.thm32_bound(eps) * (1 + 1e-6)
