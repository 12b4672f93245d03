"""Plain FP64 reference computations (test infrastructure only; see package doc).

Every routine is the textbook definition written out with numpy/LAPACK
primitives (Householder QR, triangular solve, SVD, Cholesky) as steps; there
is no blocking, fusion or reordering beyond what the definition states.
"""

from __future__ import annotations

import math
from typing import Iterable, Optional, Tuple

import numpy as np
from scipy.linalg import solve_triangular


def _as_f64(A: np.ndarray) -> np.ndarray:
    # FP32-stored problems are solved exactly as stored: the upcast is exact.
    return np.asarray(A, dtype=np.float64)


def solve_over(A: np.ndarray, b: np.ndarray, lams: Iterable[float]) -> np.ndarray:
    """x_lam for m >= n via Householder QR of B = [A; sqrt(lam) I_n] (eq. regLLSover).

    QR is taken in two stages that are exactly the QR of [A; sqrt(lam) I] with
    right-hand side [b; 0]: first A = Q R_A together with c = Q^T b (the QR of
    the bordered matrix [A b] delivers both), then for each lam the QR of the
    2n x n matrix [R_A; sqrt(lam) I] bordered by [c; 0].  Since
    diag(Q, I) has orthonormal columns, both stages minimise the same norm up
    to the constant ||(I - Q Q^T) b||.  Back substitution gives x_lam.
    Returns an (n, N) array, column i for lams[i].
    """
    A = _as_f64(A)
    m, n = A.shape
    if m < n:
        raise ValueError("solve_over needs m >= n")
    b = np.asarray(b, dtype=np.float64).reshape(m)
    Rb = np.linalg.qr(np.column_stack([A, b]), mode="r")       # (n+1) x (n+1)
    RA = Rb[:n, :n]
    c = Rb[:n, n]
    lams = np.asarray(list(lams), dtype=np.float64)
    X = np.empty((n, lams.size))
    for i, lam in enumerate(lams):
        K = np.zeros((2 * n, n + 1))
        K[:n, :n] = RA
        K[:n, n] = c
        K[n:, :n] = math.sqrt(lam) * np.eye(n)
        R2 = np.linalg.qr(K, mode="r")
        X[:, i] = solve_triangular(R2[:n, :n], R2[:n, n], lower=False)
    return X


def solve_under(A: np.ndarray, b: np.ndarray, lams: Iterable[float]) -> np.ndarray:
    """x_lam for m < n as the top n entries of the minimum-norm solution of
    [A sqrt(lam) I_m] z = b (eq. regLLSunder).

    With the Householder QR A^T = Q_A R_L (so A = R_L^T Q_A^T), the QR of the
    2m x m matrix [R_L; sqrt(lam) I] = Q_2 R_2 gives R_2^T R_2 = A A^T + lam I
    and the minimum-norm solution of [R_L^T sqrt(lam) I] z = b is
    z = Q_2 R_2^{-T} b; the first m entries of z mapped back by Q_A are x_lam.
    Returns an (n, N) array.
    """
    A = _as_f64(A)
    m, n = A.shape
    if m >= n:
        raise ValueError("solve_under needs m < n")
    b = np.asarray(b, dtype=np.float64).reshape(m)
    QA, RL = np.linalg.qr(A.T, mode="reduced")                  # n x m, m x m
    lams = np.asarray(list(lams), dtype=np.float64)
    X = np.empty((n, lams.size))
    for i, lam in enumerate(lams):
        K = np.vstack([RL, math.sqrt(lam) * np.eye(m)])
        Q2, R2 = np.linalg.qr(K, mode="reduced")
        w = solve_triangular(R2, b, trans="T", lower=False)      # R_2^{-T} b
        z = Q2 @ w
        X[:, i] = QA @ z[:m]
    return X


def solve(A: np.ndarray, b: np.ndarray, lams: Iterable[float]) -> np.ndarray:
    """x_lam = argmin ||A x - b||^2 + lam ||x||^2 (eq. regLLS) for each lam."""
    m, n = np.shape(A)
    return solve_over(A, b, lams) if m >= n else solve_under(A, b, lams)


def rel_err(x: np.ndarray, xref: np.ndarray) -> np.ndarray:
    """Per-column ||x - xref||_2 / ||xref||_2."""
    x = np.asarray(x, dtype=np.float64)
    xref = np.asarray(xref, dtype=np.float64)
    if x.ndim == 1:
        return float(np.linalg.norm(x - xref) / np.linalg.norm(xref))
    return np.linalg.norm(x - xref, axis=0) / np.linalg.norm(xref, axis=0)


# ----------------------------------------------------------------------------
# Statistical dimension (Definition 1) and its sketch estimate (Section 3.1.2)

def statistical_dimension(sigma: np.ndarray, lam: float) -> float:
    """sd_lam(A) = sum_i 1 / (1 + lam / sigma_i^2) over the nonzero sigma_i."""
    s = np.asarray(sigma, dtype=np.float64)
    s = s[s > 0]
    return float(np.sum(1.0 / (1.0 + lam / (s * s))))


def sd_hat(sigma_Y: np.ndarray, lam: float) -> float:
    """Estimate of sd_lam(A) from the singular values of the sketch Y."""
    return statistical_dimension(sigma_Y, lam)


# ----------------------------------------------------------------------------
# Preconditioners written out densely (Algorithms 1-3)

def chol_precond(Y: np.ndarray, lam: float) -> np.ndarray:
    """Upper-triangular R with R^T R = Y^T Y + lam I_n (Algorithm 1, steps 3-4)."""
    Y = _as_f64(Y)
    C = Y.T @ Y + lam * np.eye(Y.shape[1])
    return np.linalg.cholesky(C).T


def bp2_precond(Y: np.ndarray, lam: float) -> np.ndarray:
    """R of the Householder QR of [Y; sqrt(lam) I] with a positive diagonal (the BP2
    preconditioner of Section 4.1): R^T R = Y^T Y + lam I without forming Y^T Y.
    For Algorithm 2 pass Y^T (the wide mirror)."""
    Y = _as_f64(Y)
    k = Y.shape[1]
    R = np.linalg.qr(np.vstack([Y, math.sqrt(lam) * np.eye(k)]), mode="r")
    return R * np.sign(np.diag(R))[:, None]


def chol_precond_under(Y: np.ndarray, lam: float) -> np.ndarray:
    """Upper-triangular R with R^T R = Y Y^T + lam I_m (Algorithm 2, steps 3-4)."""
    Y = _as_f64(Y)
    C = Y @ Y.T + lam * np.eye(Y.shape[0])
    return np.linalg.cholesky(C).T


def lowrank_factors(Y: np.ndarray, side: str = "right") -> Tuple[np.ndarray, np.ndarray]:
    """Economy SVD of the sketch (Algorithm 3 step 4 / Algorithm 4 step 4).

    side="right": Y = XA (s x n), returns (sigma, V) with V n x s.
    side="left":  Y = AX (m x s), returns (sigma, U) with U m x s.
    """
    Y = _as_f64(Y)
    U, sig, Vt = np.linalg.svd(Y, full_matrices=False)
    return (sig, Vt.T.copy()) if side == "right" else (sig, U)


def lowrank_S(sigma: np.ndarray, lam: float) -> np.ndarray:
    """Diagonal of S: S_jj = 1 - (1 + sigma_j^2 / lam)^(-1/2) (Section 3.1, Algorithm 3 step 7)."""
    s = np.asarray(sigma, dtype=np.float64)
    return 1.0 - 1.0 / np.sqrt(1.0 + s * s / lam)


def lowrank_rinv(V: np.ndarray, sigma: np.ndarray, lam: float,
                 k: Optional[int] = None) -> np.ndarray:
    """Dense R^{-1} = lam^{-1/2} (I - V_k S_k V_k^T) (eq. RinvOver), first k columns kept."""
    V = np.asarray(V, dtype=np.float64)
    k = V.shape[1] if k is None else k
    Vk = V[:, :k]
    S = lowrank_S(np.asarray(sigma)[:k], lam)
    return (np.eye(V.shape[0]) - (Vk * S[None, :]) @ Vk.T) / math.sqrt(lam)


def lowrank_truncation(sigma_Y: np.ndarray, lam: float, alpha: float, s: int) -> int:
    """Rank s_i kept for lam (Algorithm 3 steps 1 and 5, Algorithm 4 likewise).

    The algorithm sets s_i = alpha * ceil(sd_lam_i(A)) with the estimate of
    Section 3.1.2 in place of sd; it is capped at the sketch size s (the
    algorithm's own requirement alpha sd_lam_N <= n makes the cap inactive
    for exact estimates), and rounded up when alpha is not an integer.
    """
    sd = sd_hat(sigma_Y, lam)
    return int(min(s, math.ceil(alpha * math.ceil(sd))))


# ----------------------------------------------------------------------------
# Convergence statements

def lsqr_iteration_bound(kappa: float, eps: float) -> int:
    """Iterations after which LSQR's error has contracted by eps.

    LSQR is CG on the normal equations of the preconditioned operator, whose
    error in the energy norm contracts by at least (k-1)/(k+1) per step with
    k its condition number (Golub & Van Loan, Section 11.3, applied to the
    matrix M^T M whose condition number is k^2; Section 3.3 of the paper
    states this bound).  With the factor 2 of the CG bound, l >= log(2/eps) /
    log((k+1)/(k-1)) steps suffice.
    """
    if kappa <= 1.0:
        return 1
    return int(math.ceil(math.log(2.0 / eps) / math.log((kappa + 1.0) / (kappa - 1.0))))


def lemma21_bound(XU: np.ndarray) -> float:
    """Lemma 2.1: kappa(B R^{-1}) <= max(1, s_max(XU_A)) / min(1, s_min(XU_A))."""
    s = np.linalg.svd(np.asarray(XU, dtype=np.float64), compute_uv=False)
    return max(1.0, s[0]) / min(1.0, s[-1])


def thm32_eps(U1: np.ndarray, X: np.ndarray) -> float:
    """epsilon of condition (eq. cond1over): || U1^T X^T X U1 - U1^T U1 ||_2."""
    XU = X @ U1
    return float(np.linalg.norm(XU.T @ XU - U1.T @ U1, 2))


def thm32_bound(eps: float) -> float:
    """Theorem 3.2: kappa(B R^{-1}) <= sqrt((1 + eps) / (1 - eps))."""
    return math.sqrt((1.0 + eps) / (1.0 - eps))


# ----------------------------------------------------------------------------
# L-curve (Section 4.3, Fig. 4)

def lcurve_norms(A: np.ndarray, b: np.ndarray, X: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """(||x_i||_2, ||A x_i - b||_2) for every column x_i of X: the two axes of the L-curve."""
    A = _as_f64(A)
    X = np.asarray(X, dtype=np.float64).reshape(A.shape[1], -1)
    R = A @ X - np.asarray(b, dtype=np.float64).reshape(-1, 1)
    return np.linalg.norm(X, axis=0), np.linalg.norm(R, axis=0)


def lcurve_curvature(t: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Signed curvature (x'y'' - x''y') / (x'^2 + y'^2)^(3/2) of the plane curve
    (x(t), y(t)) at the interior sample points, t increasing, derivatives by the
    second-order three-point differences of an uneven grid; NaN at both ends."""
    t, x, y = (np.asarray(v, dtype=np.float64) for v in (t, x, y))
    k = np.full(t.size, np.nan)
    for j in range(1, t.size - 1):
        h1, h2 = t[j] - t[j - 1], t[j + 1] - t[j]
        d1 = np.array([-h2 / (h1 * (h1 + h2)), (h2 - h1) / (h1 * h2), h1 / (h2 * (h1 + h2))])
        d2 = np.array([2.0 / (h1 * (h1 + h2)), -2.0 / (h1 * h2), 2.0 / (h2 * (h1 + h2))])
        xs, ys = x[j - 1:j + 2], y[j - 1:j + 2]
        x1, y1, x2, y2 = d1 @ xs, d1 @ ys, d2 @ xs, d2 @ ys
        k[j] = (x1 * y2 - x2 * y1) / (x1 * x1 + y1 * y1) ** 1.5
    return k


def lcurve_corner(lams: np.ndarray, xnorm: np.ndarray, rnorm: np.ndarray) -> int:
    """Index of the L-curve's corner (Section 4.3): the largest curvature of
    (log ||A x - b||, log ||x||) as a function of log lambda (Hansen's
    criterion), over the interior points, lambda taken in increasing order."""
    lams = np.asarray(lams, dtype=np.float64)
    order = np.argsort(lams, kind="stable")
    k = lcurve_curvature(np.log(lams[order]), np.log(np.asarray(rnorm)[order]),
                         np.log(np.asarray(xnorm)[order]))
    return int(order[int(np.nanargmax(k))])


# ----------------------------------------------------------------------------
# A-posteriori certificate

def _gradient(A: np.ndarray, b: np.ndarray, lams: np.ndarray, X: np.ndarray,
              col_chunk: int = 256) -> np.ndarray:
    """G = A^T (b - A X) - X diag(lams), accumulated in 80-bit extended precision.

    Uses the C helper when it is built (same arithmetic, parallel), else numpy
    long double column block by column block.
    """
    from .native import gradient_ld
    G = gradient_ld(A, b, lams, X)
    if G is not None:
        return G
    A = np.asarray(A)
    m, n = A.shape
    X = np.asarray(X, dtype=np.float64).reshape(n, -1)
    ld = np.longdouble
    R = np.tile(np.asarray(b, dtype=ld).reshape(m, 1), (1, X.shape[1]))
    Xl = X.astype(ld)
    for c0 in range(0, n, col_chunk):
        Ac = A[:, c0:c0 + col_chunk].astype(ld)
        R -= Ac @ Xl[c0:c0 + col_chunk]
    G = np.empty((n, X.shape[1]), dtype=ld)
    for c0 in range(0, n, col_chunk):
        Ac = A[:, c0:c0 + col_chunk].astype(ld)
        G[c0:c0 + col_chunk] = Ac.T @ R
    G -= Xl * np.asarray(lams, dtype=ld)[None, :]
    return G.astype(np.float64)


def certify(A: np.ndarray, b: np.ndarray, lams: Iterable[float], X: np.ndarray) -> np.ndarray:
    """Upper bound on ||x - x_lam|| / ||x_lam|| for candidate solutions X (n, N).

    x_lam solves the normal equations (A^T A + lam I) x = A^T b of eq. regLLS,
    whose matrix has smallest eigenvalue at least lam.  With the gradient
    g = A^T (b - A x) - lam x, ||x - x_lam|| <= ||g|| / lam, and the triangle
    inequality turns that into the relative bound
    (||g|| / lam) / (||x|| - ||g|| / lam).  g is accumulated in 80-bit extended
    precision, so its own rounding error stays far below the FP64 errors being
    certified.  Returns one bound per column (inf where the bound is vacuous).
    """
    A = np.asarray(A)
    n = A.shape[1]
    lams = np.asarray(list(lams), dtype=np.float64)
    X = np.asarray(X, dtype=np.float64).reshape(n, -1)
    gn = np.linalg.norm(_gradient(A, b, lams, X), axis=0)
    dx = gn / lams
    xn = np.linalg.norm(X, axis=0)
    out = np.full(X.shape[1], np.inf)
    ok = xn > dx
    out[ok] = dx[ok] / (xn[ok] - dx[ok])
    return out


def certify_planted(A: np.ndarray, b: np.ndarray, lams: Iterable[float], X: np.ndarray,
                    sigma: np.ndarray, V: np.ndarray, steps: int = 2) -> np.ndarray:
    """Sharper bound on ||x - x_lam|| / ||x_lam|| when A was generated as U diag(sigma) V^T.

    The plain bound ||g|| / lam of ``certify`` overestimates by up to
    ||A||^2 / lam.  Here the generator's factors give an approximate inverse
    M^{-1} = V diag(1 / (sigma^2 + lam)) V^T of A^T A + lam I (exact for the
    planted matrix, close for its stored rounding).  Refinement with it:
    D <- D + M^{-1} g(X + D), repeated `steps` times with g in extended
    precision; then x_lam - X = D + (x_lam - (X + D)) and the last term is
    bounded by ||g(X + D)|| / lam as in ``certify``.  The bound holds whatever
    the quality of M^{-1}; a poor M^{-1} only makes it loose.
    """
    A = np.asarray(A)
    n = A.shape[1]
    lams = np.asarray(list(lams), dtype=np.float64)
    X = np.asarray(X, dtype=np.float64).reshape(n, -1)
    sig2 = np.asarray(sigma, dtype=np.float64) ** 2
    V = np.asarray(V, dtype=np.float64)
    Xc = X.copy()
    for _ in range(steps):
        G = _gradient(A, b, lams, Xc)
        Xc = Xc + V @ ((V.T @ G) / (sig2[:, None] + lams[None, :]))
    gn = np.linalg.norm(_gradient(A, b, lams, Xc), axis=0)
    bound = np.linalg.norm(Xc - X, axis=0) + gn / lams
    xn = np.linalg.norm(X, axis=0)
    out = np.full(X.shape[1], np.inf)
    ok = xn > bound
    out[ok] = bound[ok] / (xn[ok] - bound[ok])
    return out
