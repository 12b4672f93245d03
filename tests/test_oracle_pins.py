"""Pins for the CPU oracle: each check ties it to something other than itself.

* closed forms on A = U diag(sigma) V^T with known factors (SVD identity);
* exact rational arithmetic on tiny inputs (brute force);
* a LAPACK least-squares cross-check (SVD-based gelsd, a different route);
* the paper's identities (Definition 1 vs Lemma 3.1, eq. RinvOver, the BP2
  equivalence of Section 4.1, Lemma 2.1, Theorem 3.2);
* planted mistakes: a plausible slip in the oracle must break one pin.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import tikhonov as T
import workloads as W


# ----------------------------------------------------------------------------
# helpers

def closed_form(U, sigma, V, b, lams):
    """x_lam = V diag(sigma / (sigma^2 + lam)) U^T b for A = U diag(sigma) V^T."""
    c = U.T @ b
    return np.stack([V @ (sigma / (sigma ** 2 + lam) * c) for lam in lams], axis=1)


def exact_tikhonov(A, b, lam):
    """Exact rational solution of (A^T A + lam I) x = A^T b (Gauss-Jordan on Fractions)."""
    m, n = A.shape
    Af = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(m)]
    bf = [Fraction(float(v)) for v in b]
    lf = Fraction(float(lam))
    M = [[sum(Af[k][i] * Af[k][j] for k in range(m)) + (lf if i == j else 0) for j in range(n)]
         for i in range(n)]
    r = [sum(Af[k][i] * bf[k] for k in range(m)) for i in range(n)]
    for col in range(n):
        piv = next(i for i in range(col, n) if M[i][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        r[col], r[piv] = r[piv], r[col]
        for i in range(n):
            if i != col and M[i][col] != 0:
                f = M[i][col] / M[col][col]
                M[i] = [a - f * c for a, c in zip(M[i], M[col])]
                r[i] -= f * r[col]
    return np.array([float(r[i] / M[i][i]) for i in range(n)])


def small_under(m=30, n=120, seed=3, sig_lo=1e-3):
    rng = np.random.default_rng(seed)
    U = W.haar(rng, m, m)
    V = W.haar(rng, n, m)
    sigma = np.logspace(0, math.log10(sig_lo), m)
    A = (U * sigma) @ V.T
    b = A @ rng.standard_normal(n) + 1e-3 * rng.standard_normal(m)
    return A, b, U, sigma, V


# ----------------------------------------------------------------------------
# x_lam pins

@pytest.mark.parametrize("m,n", [(300, 40), (2000, 100)])
def test_closed_form_over(m, n):
    p = W.over_svd(m=m, n=n, N=10)
    X = oracle.solve(p.A, p.b, p.lams)
    Xc = closed_form(p.U, p.sigma, p.V, p.b, p.lams)
    err = T.rel_err(X, Xc)
    # A is formed from its factors with rounding; kappa(B) <= 1e3 here
    assert np.all(err < 1e-11), err


def test_closed_form_under():
    A, b, U, sigma, V = small_under()
    lams = np.logspace(-6, 0, 7)
    X = oracle.solve(A, b, lams)
    Xc = closed_form(U, sigma, V, b, lams)
    assert np.all(T.rel_err(X, Xc) < 1e-10)


@pytest.mark.parametrize("shape", [(6, 3), (3, 6), (5, 5), (7, 2)])
@pytest.mark.parametrize("lam", [0.5, 1e-3, 3.0])
def test_brute_force_rational(shape, lam):
    rng = np.random.default_rng(abs(hash(shape)) % 1000)
    A = rng.standard_normal(shape)
    b = rng.standard_normal(shape[0])
    x = oracle.solve(A, b, [lam])[:, 0]
    xe = exact_tikhonov(A, b, lam)
    assert T.rel_err(x, xe) < 1e-13


def test_lapack_crosscheck():
    p = W.over_svd(m=500, n=60, N=5, sig_lo=1e-3)
    X = oracle.solve(p.A, p.b, p.lams)
    for i, lam in enumerate(p.lams):
        B = np.vstack([p.A, math.sqrt(lam) * np.eye(p.n)])
        bh = np.concatenate([p.b, np.zeros(p.n)])
        xl = np.linalg.lstsq(B, bh, rcond=None)[0]
        assert T.rel_err(X[:, i], xl) < 1e-11
    A, b, *_ = small_under(m=20, n=70)
    Xu = oracle.solve(A, b, [1e-2, 1.0])
    for i, lam in enumerate([1e-2, 1.0]):
        D = np.hstack([A, math.sqrt(lam) * np.eye(20)])
        z = np.linalg.lstsq(D, b, rcond=None)[0]
        assert T.rel_err(Xu[:, i], z[:70]) < 1e-11


def test_fp32_storage_is_exact_upcast():
    p = W.under_scaled(m=40, n=300, N=3)
    assert p.A.dtype == np.float32
    X1 = oracle.solve(p.A, p.b, p.lams)
    X2 = oracle.solve(p.A.astype(np.float64), p.b, p.lams)
    assert np.array_equal(X1, X2)


# ----------------------------------------------------------------------------
# statistical dimension

def test_sd_definition_matches_lemma31():
    # ||U_1||_F^2 = sd_lam(A), U_1 the top m rows of B's left singular vectors
    rng = np.random.default_rng(5)
    m, n = 120, 25
    A = rng.standard_normal((m, n)) * np.logspace(0, -4, n)
    sig = np.linalg.svd(A, compute_uv=False)
    for lam in [1e-6, 1e-3, 1.0]:
        B = np.vstack([A, math.sqrt(lam) * np.eye(n)])
        UB = np.linalg.svd(B, full_matrices=False)[0]
        assert abs(np.sum(UB[:m] ** 2) - oracle.statistical_dimension(sig, lam)) < 1e-10


def test_sd_special_cases_and_integral():
    sig = np.ones(8)
    assert oracle.statistical_dimension(sig, 0.0) == 8.0          # lam = 0: the rank
    assert abs(oracle.statistical_dimension(sig, 1.0) - 4.0) < 1e-15  # sigma^2 = lam: half
    sigma = np.exp(-np.arange(1, 10001) / 200.0)
    for lam in [1e-4, 1e-1]:
        integral = 100.0 * math.log((1.0 + lam) / lam)
        sd = oracle.statistical_dimension(sigma, lam)
        assert abs(sd - integral) <= 1.0, (lam, sd, integral)
    # the low-sd workload's sketch size: 2 * ceil(sd at lam=1e-4)
    assert 2 * math.ceil(oracle.statistical_dimension(sigma, 1e-4)) == 1842


# ----------------------------------------------------------------------------
# preconditioners and their quality bounds

def _kappa(M):
    s = np.linalg.svd(M, compute_uv=False)
    return s[0] / s[-1]


def test_bp2_equivalence():
    # R from QR of [XA; sqrt(lam) I] (BP2, Section 4.1) equals chol(C + lam I)
    rng = np.random.default_rng(7)
    Y = rng.standard_normal((80, 30)) * np.logspace(0, -5, 30)
    for lam in [1e-8, 1e-2]:
        R = oracle.chol_precond(Y, lam)
        Rq = np.linalg.qr(np.vstack([Y, math.sqrt(lam) * np.eye(30)]), mode="r")
        Rq = Rq * np.sign(np.diag(Rq))[:, None]
        assert np.allclose(R, Rq, rtol=1e-9, atol=1e-12 * np.abs(R).max())
        C = Y.T @ Y + lam * np.eye(30)
        assert np.linalg.norm(R.T @ R - C) <= 1e-13 * np.linalg.norm(C)


def test_lowrank_rinv_identity():
    # with untruncated V (s < n), R^{-T}(Y^T Y + lam I)R^{-1} = I (eq. RinvOver)
    rng = np.random.default_rng(11)
    Y = rng.standard_normal((15, 60))
    sig, V = oracle.lowrank_factors(Y)
    for lam in [1e-4, 1e-1, 10.0]:
        Ri = oracle.lowrank_rinv(V, sig, lam)
        assert np.allclose(Ri, Ri.T)
        G = Ri.T @ (Y.T @ Y + lam * np.eye(60)) @ Ri
        # rounding grows with the spread (sigma_1^2 + lam) / lam of the factors
        assert np.linalg.norm(G - np.eye(60)) < 1e-13 * (1 + sig[0] ** 2 / lam)
        # eigenvalues (sigma^2 + lam)^(-1/2) on span V, lam^(-1/2) elsewhere
        ev = np.sort(np.linalg.eigvalsh(Ri))
        want = np.sort(np.concatenate([1 / np.sqrt(sig ** 2 + lam),
                                       np.full(60 - 15, 1 / math.sqrt(lam))]))
        assert np.allclose(ev, want, rtol=1e-10)


def _lowsd_problem(m=600, n=80, decay=8.0, seed=2):
    rng = np.random.default_rng(seed)
    U = W.haar(rng, m, n)
    V = W.haar(rng, n, n)
    sig = np.exp(-np.arange(1, n + 1) / decay)
    return (U * sig) @ V.T, U, sig, V


def test_lemma21_bound():
    A, UA, sig, V = _lowsd_problem(m=500, n=20, decay=4.0)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((80, 500)) / math.sqrt(80)
    for lam in [1e-10, 1e-4, 1e-1]:
        R = oracle.chol_precond(X @ A, lam)
        B = np.vstack([A, math.sqrt(lam) * np.eye(20)])
        k = _kappa(B @ np.linalg.inv(R))
        assert k <= oracle.lemma21_bound(X @ UA) * (1 + 1e-8)


def test_thm32_bound_chol_and_lowrank():
    A, UA, sig, V = _lowsd_problem()
    m, n = A.shape
    rng = np.random.default_rng(9)
    for lam in [1e-3, 1e-2]:
        sd = oracle.statistical_dimension(sig, lam)
        s = min(m, int(16 * math.ceil(sd)))
        X = rng.standard_normal((s, m)) / math.sqrt(s)
        U1 = UA * (sig / np.sqrt(sig ** 2 + lam))[None, :]
        eps = oracle.thm32_eps(U1, X)
        assert eps < 1
        bound = oracle.thm32_bound(eps)
        B = np.vstack([A, math.sqrt(lam) * np.eye(n)])
        Y = X @ A
        kc = _kappa(B @ np.linalg.inv(oracle.chol_precond(Y, lam)))
        sY, VY = oracle.lowrank_factors(Y)
        kl = _kappa(B @ oracle.lowrank_rinv(VY, sY, lam))
        assert kc <= bound * (1 + 1e-8) and kl <= bound * (1 + 1e-8), (kc, kl, bound)
        assert abs(kc - kl) < 1e-6 * kc      # any R with R^T R = Y^T Y + lam I


def _lsqr_energy_error(M, c, ys, iters):
    """||M (y_l - y*)|| / ||M y*|| after exactly `iters` steps of scipy's LSQR from y0 = 0."""
    from scipy.sparse.linalg import lsqr
    y = lsqr(M, c, atol=0.0, btol=0.0, conlim=0.0, iter_lim=iters)[0]
    return float(np.linalg.norm(M @ (y - ys)) / np.linalg.norm(c))


@pytest.mark.parametrize("kappa", [2.0, 10.0, 100.0])
def test_iteration_bound_against_lsqr(kappa):
    """Section 3.3: LSQR's error contracts like CG on M^T M.

    Independent check: scipy's LSQR (Paige & Saunders) on consistent systems
    M y = c whose operator has a prescribed condition number.  After the
    bound's count the error in the M^T M energy norm is below eps, for a
    geometric and a Chebyshev-node spectrum.  The bound is also not loose:
    for kappa = 2 and 10 half its count is not enough, and for kappa = 100
    the count of the printed form (sqrt(kappa) in place of kappa) is far too
    small.  A slip in the bound's formula fails one of these.
    """
    rng = np.random.default_rng(int(kappa))
    m, n = 900, 400
    U = W.haar(rng, m, n)
    V = W.haar(rng, n, n)
    t = np.cos(np.arange(n) * np.pi / (n - 1))          # Chebyshev extreme points, ends included
    lo = 1.0 / kappa ** 2
    spectra = {"geometric": np.logspace(0, -math.log10(kappa), n),
               "chebyshev": np.sqrt((1 + lo) / 2 + (1 - lo) / 2 * t)}
    for name, sig in spectra.items():
        M = (U * sig) @ V.T
        assert abs(np.linalg.cond(M) / kappa - 1) < 1e-6
        ys = rng.standard_normal(n)
        c = M @ ys
        for eps in (1e-6, 1e-10):
            L = oracle.lsqr_iteration_bound(kappa, eps)
            assert _lsqr_energy_error(M, c, ys, L) <= eps, (name, eps, L)
            if kappa <= 10:
                assert _lsqr_energy_error(M, c, ys, L // 2) > eps, (name, eps, L)
            else:
                Ls = oracle.lsqr_iteration_bound(math.sqrt(kappa), eps)
                assert _lsqr_energy_error(M, c, ys, Ls) > 1e3 * eps, (name, eps, Ls)


def test_iteration_bound_special_cases():
    assert oracle.lsqr_iteration_bound(1.0, 1e-10) == 1          # M orthonormal: one step
    ks = [1.5, 2, 4, 8, 16]
    its = [oracle.lsqr_iteration_bound(k, 1e-8) for k in ks]
    assert its == sorted(its)
    # O(log 1/eps): squaring eps roughly doubles the count
    a, b = oracle.lsqr_iteration_bound(10.0, 1e-5), oracle.lsqr_iteration_bound(10.0, 1e-10)
    assert 1.8 * a <= b <= 2.2 * a


# ---------------------------------------------------------------------------
# Algorithm 2 / Algorithm 4 (wide problems): preconditioners from Y = A X

def _wide_problem(m=40, n=300, s=160, seed=8, decay=6.0):
    rng = np.random.default_rng(seed)
    U = W.haar(rng, m, m)
    V = W.haar(rng, n, m)
    sig = np.exp(-np.arange(m) / decay)
    A = (U * sig) @ V.T
    X = rng.standard_normal((n, s)) / math.sqrt(s)
    return A, U, sig, V, X


def test_chol_precond_under_bp2_mirror_and_lemma():
    """Algorithm 2 steps 3-4: R^T R = Y Y^T + lam I_m.

    Pins: R equals the R factor (diagonal made positive) of the Householder QR
    of [Y^T; sqrt(lam) I_m] (the wide mirror of BP2, Section 4.1), a route that
    never forms Y Y^T; and the preconditioned D = [A sqrt(lam) I] obeys the
    condition bound of the underdetermined lemma of Section 2.2, in its
    general form max(1, s_max(X^T V_A)) / min(1, s_min(X^T V_A)).
    """
    A, UA, sig, VA, X = _wide_problem()
    m = A.shape[0]
    Y = A @ X
    for lam in [1e-10, 1e-4, 1e-1]:
        R = oracle.chol_precond_under(Y, lam)
        assert R.shape == (m, m) and np.array_equal(R, np.triu(R))
        Rq = np.linalg.qr(np.vstack([Y.T, math.sqrt(lam) * np.eye(m)]), mode="r")
        Rq = Rq * np.sign(np.diag(Rq))[:, None]
        assert np.linalg.norm(R - Rq) <= 1e-10 * np.linalg.norm(R), lam
        D = np.hstack([A, math.sqrt(lam) * np.eye(m)])
        k = _kappa(np.linalg.solve(R.T, D))
        assert k <= oracle.lemma21_bound(X.T @ VA) * (1 + 1e-8), (lam, k)


def test_lowrank_left_factors_rinv_and_thm34():
    """Algorithm 4 step 4: U and sigma of Y = A X (m x s, s < m).

    Pins: with R^{-T} = lam^{-1/2} (I_m - U S U^T) (the wide form of eq.
    RinvOver), R^{-T} (Y Y^T + lam I_m) R^{-1} = I; Y = U diag(sigma) W^T
    with W orthonormal; and the theorem of Section 3.3.2: kappa(R^{-T} D) <=
    sqrt((1 + eps) / (1 - eps)) with eps = ||V_1^T X X^T V_1 - V_1^T V_1||,
    V_1 the first n rows of D's right singular vectors, whose squared
    Frobenius norm is sd_lam(A) (the underdetermined lemma of Section 3.3.2).
    """
    A, UA, sig, VA, _ = _wide_problem(m=60, n=500, s=0, decay=3.0)
    m, n = A.shape
    rng = np.random.default_rng(21)
    for lam in [1e-3, 1e-2]:
        sd = oracle.statistical_dimension(sig, lam)
        s = min(m - 1, int(6 * math.ceil(sd)))
        X = rng.standard_normal((n, s)) / math.sqrt(s)
        Y = A @ X
        sY, U = oracle.lowrank_factors(Y, side="left")
        assert U.shape == (m, s) and sY.shape == (s,)
        # U orthonormal and spans Y's columns; sigma are Y's singular values
        # (the square roots of the eigenvalues of the s x s Gram matrix)
        assert np.allclose(U.T @ U, np.eye(s), atol=1e-12)
        assert np.linalg.norm(Y - U @ (U.T @ Y)) <= 1e-13 * np.linalg.norm(Y)
        ev = np.sqrt(np.clip(np.linalg.eigvalsh(Y.T @ Y)[::-1], 0, None))
        assert np.allclose(sY, ev, rtol=0, atol=1e-7 * sY[0])
        RiT = oracle.lowrank_rinv(U, sY, lam)
        G = RiT @ (Y @ Y.T + lam * np.eye(m)) @ RiT.T
        assert np.linalg.norm(G - np.eye(m)) < 1e-13 * (1 + sY[0] ** 2 / lam)
        D = np.hstack([A, math.sqrt(lam) * np.eye(m)])
        VD = np.linalg.svd(D, full_matrices=False)[2].T          # (n + m) x m
        V1 = VD[:n]
        assert abs(np.sum(V1 ** 2) - sd) < 1e-10
        eps = float(np.linalg.norm(V1.T @ X @ X.T @ V1 - V1.T @ V1, 2))
        assert eps < 1
        k = _kappa(RiT @ D)
        assert k <= oracle.thm32_bound(eps) * (1 + 1e-8), (lam, k, eps)
    # a plausible slip: the right factor in place of the left one fails the identity
    sR, Vr = oracle.lowrank_factors(Y, side="right")
    assert Vr.shape != U.shape or not np.allclose(Vr, U)


def test_certify_bounds_error():
    p = W.over_svd(m=400, n=30, N=4, sig_lo=1e-4)
    X = oracle.solve(p.A, p.b, p.lams)
    rng = np.random.default_rng(1)
    for scale in [1e-6, 1e-9]:
        Xp = X + scale * rng.standard_normal(X.shape) * np.linalg.norm(X, axis=0)
        true = T.rel_err(Xp, X)
        bound = oracle.certify(p.A, p.b, p.lams, Xp)
        assert np.all(bound >= true * (1 - 1e-6)), (bound, true)
    assert np.all(oracle.certify(p.A, p.b, p.lams, X) < 1e-9)


# ----------------------------------------------------------------------------
# planted mistakes: each slip must break a pin above

def test_planted_dropped_sqrt(monkeypatch):
    monkeypatch.setattr(T.math, "sqrt", lambda v: v)       # uses lam for sqrt(lam)
    p = W.over_svd(m=300, n=40, N=4)
    err = T.rel_err(T.solve_over(p.A, p.b, p.lams), closed_form(p.U, p.sigma, p.V, p.b, p.lams))
    assert np.max(err) > 1e-3


def test_planted_transposed_solve(monkeypatch):
    real = T.solve_triangular
    monkeypatch.setattr(T, "solve_triangular",
                        lambda R, y, trans=0, lower=False: real(R, y, trans="N" if trans == "T" else "T",
                                                                lower=lower))
    A, b, U, sigma, V = small_under()
    lams = [1e-3, 1e-1]
    assert np.max(T.rel_err(T.solve_under(A, b, lams), closed_form(U, sigma, V, b, lams))) > 1e-3


def test_planted_S_without_square():
    rng = np.random.default_rng(11)
    Y = rng.standard_normal((15, 60))
    sig, V = oracle.lowrank_factors(Y)
    lam = 1e-1
    S_wrong = 1.0 - 1.0 / np.sqrt(1.0 + sig / lam)                    # sigma in place of sigma^2
    Ri = (np.eye(60) - (V * S_wrong) @ V.T) / math.sqrt(lam)
    G = Ri.T @ (Y.T @ Y + lam * np.eye(60)) @ Ri
    assert np.linalg.norm(G - np.eye(60)) > 1e-2


# ----------------------------------------------------------------------------
# generators

def test_generators_deterministic():
    a = W.over_svd(m=200, n=20, N=3)
    b = W.over_svd(m=200, n=20, N=3)
    assert np.array_equal(a.A, b.A) and np.array_equal(a.b, b.b)
    assert a.A.flags.f_contiguous
    c = W.over_svd(m=200, n=20, N=3, seed=1)
    assert not np.array_equal(a.A, c.A)
    full = W.ragged(nprob=6, m_lo=50, m_hi=90, n_lo=5, n_hi=20)
    part = W.ragged(nprob=6, m_lo=50, m_hi=90, n_lo=5, n_hi=20, first=3, count=2)
    assert np.array_equal(full[3].A, part[0].A) and np.array_equal(full[4].b, part[1].b)
    assert [(q.m, q.n) for q in full] == W.ragged_shapes(6, 50, 90, 5, 20)


def test_lowrank_truncation_rule():
    """Algorithm 3 steps 1 and 5: s_i = alpha ceil(sd_hat), capped at s.

    sigma_j^2 = lam makes every term of the estimate exactly 1/2, so
    sd_hat = s/2 in closed form; the rank then follows by hand.
    """
    lam = 0.25
    sig = np.full(10, 0.5)                       # sigma^2 = lam
    assert oracle.sd_hat(sig, lam) == 5.0
    assert oracle.lowrank_truncation(sig, lam, 2.0, 10) == 10
    assert oracle.lowrank_truncation(sig, lam, 1.0, 10) == 5
    assert oracle.lowrank_truncation(sig, lam, 1.5, 10) == 8   # ceil(1.5 * 5)
    assert oracle.lowrank_truncation(sig, lam, 3.0, 10) == 10  # capped at s
    # zero singular values contribute nothing (A = 0 keeps no direction)
    assert oracle.lowrank_truncation(np.zeros(6), lam, 2.0, 6) == 0
    # the rank never grows with lambda (sd is decreasing in lambda)
    rng = np.random.default_rng(4)
    sig = np.sort(rng.uniform(0, 1, 40))[::-1]
    ranks = [oracle.lowrank_truncation(sig, l, 2.0, 40) for l in np.logspace(-4, 1, 30)]
    assert all(a >= b for a, b in zip(ranks, ranks[1:]))


def _numpy_gradient(A, b, lams, X):
    ld = np.longdouble
    Al = np.asarray(A).astype(ld)
    R = np.asarray(b, dtype=ld)[:, None] - Al @ X.astype(ld)
    return (Al.T @ R - X.astype(ld) * np.asarray(lams, dtype=ld)[None, :]).astype(np.float64)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_native_gradient_matches_long_double_numpy(dtype):
    """The C helper computes the same extended-precision gradient as numpy long double."""
    from oracle import native
    if native.lib() is None:
        native.build_native()
    rng = np.random.default_rng(12)
    m, n, N = 700, 90, 5
    A = np.asfortranarray(rng.standard_normal((m, n)).astype(dtype))
    b = rng.standard_normal(m)
    lams = np.logspace(-3, 0, N)
    X = rng.standard_normal((n, N))
    Gc = native.gradient_ld(A, b, lams, X)
    Gn = _numpy_gradient(A, b, lams, X)
    assert np.max(np.abs(Gc - Gn)) <= 1e-13 * np.max(np.abs(Gn))
    # at the exact solution the gradient vanishes to extended-precision rounding
    Xo = oracle.solve(A, b, lams)
    G0 = native.gradient_ld(A, b, lams, Xo)
    assert np.max(np.abs(G0)) <= 1e-11 * np.max(np.abs(Gn))


def test_certify_planted_bounds_the_true_error():
    """The planted-factor bound is valid and tight; a wrong sigma keeps it valid."""
    p = W.lowsd(m=900, n=220, N=4, decay=20.0, lam_lo=1e-4, lam_hi=1e-1, seed=3)
    Xo = oracle.solve(p.A, p.b, p.lams)
    rng = np.random.default_rng(5)
    for eps in (1e-6, 1e-9):
        Xp = Xo + eps * rng.standard_normal(Xo.shape) * np.linalg.norm(Xo, axis=0)[None, :] / math.sqrt(p.n)
        true = oracle.rel_err(Xp, Xo)
        bnd = oracle.certify_planted(p.A, p.b, p.lams, Xp, p.sigma, p.V)
        plain = oracle.certify(p.A, p.b, p.lams, Xp)
        assert np.all(bnd >= true * (1 - 1e-6)), (bnd, true)
        assert np.all(bnd <= 1.5 * true + 1e-12), (bnd, true)
        assert np.all(plain >= bnd * (1 - 1e-6))          # the planted bound is the sharper one
    bad = oracle.certify_planted(p.A, p.b, p.lams, Xp, 1.7 * p.sigma, p.V)
    assert np.all(bad >= true * (1 - 1e-6))


# ---------------------------------------------------------------------------
# L-curve (Section 4.3)

def _ellipse(a=3.0, b=1.0, n=41, seed=0):
    """Samples of (a cos t, b sin t) on an uneven grid of t in [-1.2, 1.2]."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(-1.2, 1.2, n))
    return t, a * np.cos(t), b * np.sin(t)


def test_lcurve_curvature_ellipse():
    """Curvature of an ellipse traversed counter-clockwise: ab / (a^2 sin^2 t + b^2 cos^2 t)^(3/2),
    largest at t = 0 when a > b; the three-point differences are second order."""
    a, b = 3.0, 1.0
    for n in (41, 161):
        t, x, y = _ellipse(a, b, n)
        k = oracle.lcurve_curvature(t, x, y)
        exact = a * b / (a * a * np.sin(t) ** 2 + b * b * np.cos(t) ** 2) ** 1.5
        assert np.isnan(k[0]) and np.isnan(k[-1])
        h = np.max(np.diff(t))
        assert np.max(np.abs(k[1:-1] - exact[1:-1]) / exact[1:-1]) < 40 * h * h, n
        assert int(np.nanargmax(k)) == int(np.argmin(np.abs(t[1:-1]))) + 1
    # clockwise traversal flips the sign
    t, x, y = _ellipse(a, b, 41)
    assert np.all(oracle.lcurve_curvature(t, x, -y)[1:-1] < 0)


def test_lcurve_corner_through_logs():
    """lcurve_corner takes logs of lambda and of both norms: an ellipse in log space
    has its corner where t = log lambda is closest to 0, whatever the input order."""
    t, x, y = _ellipse(2.0, 0.5, 31, seed=4)
    lams, rn, xn = np.exp(t), np.exp(x), np.exp(y)
    want = int(np.argmin(np.abs(t[1:-1]))) + 1
    assert oracle.lcurve_corner(lams, xn, rn) == want
    perm = np.random.default_rng(1).permutation(t.size)
    assert perm[oracle.lcurve_corner(lams[perm], xn[perm], rn[perm])] == want


def test_lcurve_norms_closed_form():
    """||x_lam||^2 = sum (sigma c / (sigma^2 + lam))^2 and ||A x_lam - b||^2 =
    sum (lam c / (sigma^2 + lam))^2 + ||b - U U^T b||^2 with c = U^T b (SVD identity)."""
    p = W.over_svd(m=600, n=50, N=9, lam_lo=1e-10, lam_hi=1e2)
    X = oracle.solve(p.A, p.b, p.lams)
    xn, rn = oracle.lcurve_norms(p.A, p.b, X)
    c = p.U.T @ p.b
    perp = np.linalg.norm(p.b - p.U @ c)
    for i, lam in enumerate(p.lams):
        d = p.sigma ** 2 + lam
        xw = np.linalg.norm(p.sigma * c / d)
        rw = math.sqrt(np.sum((lam * c / d) ** 2) + perp ** 2)
        assert abs(xn[i] - xw) <= 1e-11 * xw and abs(rn[i] - rw) <= 1e-10 * rw, (lam, xn[i], xw, rn[i], rw)


def test_bp2_precond_matches_cholesky_and_survives_breakdown():
    """BP2 (Section 4.1): R from the QR of [Y; sqrt(lam) I] equals chol(Y^T Y + lam I)
    where that exists; where the Cholesky factorization of the Gram matrix breaks down
    (kappa(C + lam I) beyond 1/u), the QR factor still exists and still preconditions
    B = [A; sqrt(lam) I] to the Lemma 2.1 bound."""
    from numpy.linalg import LinAlgError
    rng = np.random.default_rng(7)
    Y = rng.standard_normal((80, 30)) * np.logspace(0, -5, 30)
    for lam in [1e-8, 1e-2]:
        assert np.allclose(oracle.bp2_precond(Y, lam), oracle.chol_precond(Y, lam), rtol=1e-9,
                           atol=1e-12 * np.abs(Y).max() ** 2)
    A, UA, sig, V = _lowsd_problem(m=600, n=40, decay=40 / (10 * math.log(10)))   # sigma 1 .. ~1e-10
    X = rng.standard_normal((160, 600)) / math.sqrt(160)
    Y = X @ A
    lam = 1e-24
    with pytest.raises(LinAlgError):
        oracle.chol_precond(Y, lam)
    R = oracle.bp2_precond(Y, lam)
    assert np.all(np.diag(R) > 0) and np.array_equal(R, np.triu(R))
    B = np.vstack([A, math.sqrt(lam) * np.eye(40)])
    k = _kappa(np.linalg.solve(R.T, B.T).T)
    assert k <= oracle.lemma21_bound(X @ UA) * 1.01, k


def test_host_philox_known_answers_cpu():
    """The tests' host Philox4x32-10 reproduces the published known-answer vectors."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from philox_ref import philox4x32_10
    got = philox4x32_10(np.array([[0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344]], dtype=np.uint32),
                        np.array([0xA4093822, 0x299F31D0], dtype=np.uint32))[0]
    assert [int(v) for v in got] == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]
