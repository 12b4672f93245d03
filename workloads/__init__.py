"""Seeded synthetic workloads for regularized least squares min ||Ax-b||^2 + lam ||x||^2.

This module only draws inputs.  It holds none of the method's arithmetic: no
sketch, no preconditioner, no solver.  Both the CPU oracle (through the tests)
and the GPU library (through the binding, bench and tests) consume what it
returns, so the two sides always see the very same numbers.

Recipe (Section 4 of the paper describes its test matrices as the product of
two orthogonal factors, taken from QR of Gaussian matrices, and a diagonal of
prescribed singular values; b = A x + noise with x ~ N(0, 1)).  Five families
mirror the five workloads of the benchmark plan:

  over_svd     A = U diag(sigma) V^T, U, V Haar, sigma logspaced 1 -> 1e-6
               (m=2000, n=100, N=10 lambdas in [1e-6, 1], FP64 storage)
  over_gauss   A = G diag(sigma), G ~ N(0,1), sigma logspaced 1 -> 1e-8
               (m=200000, n=2000, N=32 lambdas in [1e-8, 1e-1], FP64 storage)
  under_scaled A_ij = G_ij / j (1-based j), FP32 storage
               (m=2000, n=200000, N=32 lambdas in [1e-6, 1])
  lowsd        A = U diag(exp(-i/decay)) V^T, FP32 storage
               (m=100000, n=10000, decay=200, N=16 lambdas in [1e-4, 1e-1])
  ragged       many independent G_p diag(logspace(0,-6,n_p)) problems, FP32
               (256 problems, m_p ~ U[5000,50000], n_p ~ U[100,1000], 8 lambdas)
  decay50      the embedding-study matrices of Section 4.2: A = U diag(sigma) V^T,
               sigma logspaced 1 -> 1e-50, ||noise|| = 1e-3, lambdas 10 -> 1e-15,
               FP64 (m=50000, n=1000)

Every generator takes its sizes as arguments so tests can draw the same
family at reduced size.  Seeds derive from numpy.random.SeedSequence(seed)
spawned per family and per object, so each object is reproducible alone.

Haar factors follow Mezzadri (2007): Q from QR of a Gaussian matrix with its
columns multiplied by sign(diag(R)).

Layout: every matrix is returned as a numpy array of shape (m, n) in Fortran
(column-major) order, which is the layout the GPU library consumes (lda = m).
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

FAMILY_IDS = {"over_svd": 0, "over_gauss": 1, "under_scaled": 2, "lowsd": 3, "ragged": 4,
              "decay50": 5}


@dataclasses.dataclass
class Problem:
    """One regularized least squares problem and its solver settings."""

    name: str
    A: np.ndarray                 # (m, n), Fortran order, float64 or float32 storage
    b: np.ndarray                 # (m,), float64
    lams: np.ndarray              # (N,), float64
    s: int                        # sketch size
    embed: str                    # "srht" or "gauss"
    route: str                    # "chol" or "lowrank"
    tol: float                    # target relative forward error vs the oracle
    seed: int                     # sketch seed
    sigma: Optional[np.ndarray] = None   # prescribed singular values, when known
    U: Optional[np.ndarray] = None       # prescribed left factor (closed-form checks)
    V: Optional[np.ndarray] = None       # prescribed right factor
    x0: Optional[np.ndarray] = None      # planted coefficients
    alpha: float = 2.0            # low-sd oversampling factor

    @property
    def m(self) -> int:
        return int(self.A.shape[0])

    @property
    def n(self) -> int:
        return int(self.A.shape[1])

    @property
    def a_dtype(self) -> str:
        return "f64" if self.A.dtype == np.float64 else "f32"


def _rngs(family: str, seed: int, k: int) -> List[np.random.Generator]:
    root = np.random.SeedSequence([seed, FAMILY_IDS[family]])
    return [np.random.Generator(np.random.PCG64(c)) for c in root.spawn(k)]


def haar(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Orthonormal rows x cols frame with Haar distribution (Mezzadri 2007)."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return np.asfortranarray(q * d[None, :])


def _gaussian_colmajor(rng: np.random.Generator, m: int, n: int, dtype) -> np.ndarray:
    # draw column by column so the result is Fortran ordered without a copy
    return rng.standard_normal((n, m), dtype=dtype).T


def over_svd(m: int = 2000, n: int = 100, N: int = 10, seed: int = 0,
             sig_lo: float = 1e-6, lam_lo: float = 1e-6, lam_hi: float = 1.0,
             noise: float = 1e-3, s: Optional[int] = None, embed: str = "srht",
             tol: float = 1e-10) -> Problem:
    """A = U diag(logspace(0, log10 sig_lo, n)) V^T with Haar U, V (FP64)."""
    ru, rv, rx, re = _rngs("over_svd", seed, 4)
    U = haar(ru, m, n)
    V = haar(rv, n, n)
    sigma = np.logspace(0.0, math.log10(sig_lo), n)
    A = np.asfortranarray((U * sigma[None, :]) @ V.T)
    x0 = rx.standard_normal(n)
    b = A @ x0 + noise * re.standard_normal(m)
    lams = np.logspace(math.log10(lam_lo), math.log10(lam_hi), N)
    return Problem("over_svd", A, b, lams, s if s is not None else 4 * n, embed, "chol",
                   tol, seed, sigma=sigma, U=U, V=V, x0=x0)


def over_gauss(m: int = 200000, n: int = 2000, N: int = 32, seed: int = 0,
               sig_lo: float = 1e-8, lam_lo: float = 1e-8, lam_hi: float = 1e-1,
               noise: float = 1e-2, s: Optional[int] = None, embed: str = "srht",
               tol: float = 1e-8) -> Problem:
    """A = G diag(logspace(0, log10 sig_lo, n)), G ~ N(0, 1) (FP64)."""
    rg, rx, re = _rngs("over_gauss", seed, 3)
    sigma = np.logspace(0.0, math.log10(sig_lo), n)
    A = _gaussian_colmajor(rg, m, n, np.float64)
    A *= sigma[None, :]
    x0 = rx.standard_normal(n)
    b = A @ x0 + noise * re.standard_normal(m)
    lams = np.logspace(math.log10(lam_lo), math.log10(lam_hi), N)
    return Problem("over_gauss", A, b, lams, s if s is not None else 4 * n, embed, "chol",
                   tol, seed, sigma=None, x0=x0)


def under_scaled(m: int = 2000, n: int = 200000, N: int = 32, seed: int = 0,
                 lam_lo: float = 1e-6, lam_hi: float = 1.0, noise: float = 1e-3,
                 s: Optional[int] = None, embed: str = "gauss", tol: float = 1e-8) -> Problem:
    """A_ij = G_ij / j with 1-based column index j, stored in FP32; b in FP64."""
    rg, rx, re = _rngs("under_scaled", seed, 3)
    A = _gaussian_colmajor(rg, m, n, np.float32)
    A *= (1.0 / np.arange(1, n + 1, dtype=np.float64)).astype(np.float32)[None, :]
    x0 = rx.standard_normal(n)
    b = A.astype(np.float64) @ x0 + noise * re.standard_normal(m)
    lams = np.logspace(math.log10(lam_lo), math.log10(lam_hi), N)
    return Problem("under_scaled", A, b, lams, s if s is not None else 4 * m, embed, "chol",
                   tol, seed, x0=x0)


def lowsd(m: int = 100000, n: int = 10000, N: int = 16, seed: int = 0, decay: float = 200.0,
          lam_lo: float = 1e-4, lam_hi: float = 1e-1, noise: float = 1e-3,
          s: Optional[int] = None, sd_hint: Optional[float] = None, alpha: float = 2.0,
          tol: float = 1e-8, device=None) -> Problem:
    """A = U diag(exp(-i/decay)) V^T (i = 1..n), formed in FP64, stored in FP32.

    The sketch size is s = alpha * ceil(sd_hint) where sd_hint is the
    statistical dimension at the smallest lambda; the workload supplies it (it
    is the estimate Algorithm 3 takes as input).  For sigma_i = exp(-i/decay)
    the sum defining it is close to the integral (decay / 2) ln((1 + lam) / lam)
    (920.5 summed vs 921.0 integrated at decay=200, lam=1e-4); callers pass a
    hint or let s default to that integral, rounded up.

    With device (a torch device string) the orthogonal factors and the
    product are formed with torch on that device, which the full-size
    instance needs (QR of a 1e5 x 1e4 Gaussian); the Gaussians themselves are
    still drawn on the host from the same seeds.
    """
    ru, rv, rx, re = _rngs("lowsd", seed, 4)
    sigma = np.exp(-np.arange(1, n + 1, dtype=np.float64) / decay)
    gu = ru.standard_normal((m, n))
    gv = rv.standard_normal((n, n))
    if device is None:
        U = haar_from(gu)
        V = haar_from(gv)
        A64 = (U * sigma[None, :]) @ V.T
    else:
        import torch
        def _haar_t(g):
            q, r = torch.linalg.qr(torch.from_numpy(g).to(device))
            d = torch.sign(torch.diagonal(r))
            d[d == 0] = 1.0
            return q * d[None, :]
        Ut = _haar_t(gu)
        del gu
        Vt = _haar_t(gv)
        A64 = ((Ut * torch.from_numpy(sigma).to(device)[None, :]) @ Vt.T).cpu().numpy()
        U = None                      # m x n: not kept at full size
        V = np.asfortranarray(Vt.cpu().numpy())
        del Ut, Vt
    A = np.asfortranarray(A64.astype(np.float32))
    del A64
    x0 = rx.standard_normal(n)
    b = A.astype(np.float64) @ x0 + noise * re.standard_normal(m)
    lams = np.logspace(math.log10(lam_lo), math.log10(lam_hi), N)
    if s is None:
        hint = sd_hint if sd_hint is not None else 0.5 * decay * math.log((1.0 + lam_lo) / lam_lo)
        s = int(alpha * math.ceil(hint))
    return Problem("lowsd", A, b, lams, int(s), "gauss", "lowrank", tol, seed,
                   sigma=sigma, U=U, V=V, x0=x0, alpha=alpha)


def decay50(m: int = 50000, n: int = 1000, N: int = 16, seed: int = 0, sig_lo: float = 1e-50,
            lam_lo: float = 1e-15, lam_hi: float = 10.0, noise_norm: float = 1e-3) -> Problem:
    """A = U diag(logspace(0, log10 sig_lo, n)) V^T with Haar U (m x n), V (n x n), FP64;
    b = A x0 + eta with ||eta|| about noise_norm (the matrices of the paper's
    experiments: orthogonal factors of Gaussians, singular values decaying from 1
    to 1e-50, lambdas from 10 down to 1e-15)."""
    ru, rv, rx, re = _rngs("decay50", seed, 4)
    U = haar(ru, m, n)
    V = haar(rv, n, n)
    sigma = np.logspace(0, math.log10(sig_lo), n)
    A = np.asfortranarray((U * sigma[None, :]) @ V.T)
    x0 = rx.standard_normal(n)
    b = A @ x0 + (noise_norm / math.sqrt(m)) * re.standard_normal(m)
    lams = np.logspace(math.log10(lam_hi), math.log10(lam_lo), N)
    return Problem("decay50", A, b, lams, 2 * n, "gauss", "chol", 1e-10, seed,
                   sigma=sigma, U=U, V=V, x0=x0)


def haar_from(g: np.ndarray) -> np.ndarray:
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return np.asfortranarray(q * d[None, :])


def ragged(nprob: int = 256, m_lo: int = 5000, m_hi: int = 50000, n_lo: int = 100,
           n_hi: int = 1000, N: int = 8, seed: int = 0, lam_lo: float = 1e-6,
           lam_hi: float = 1e-1, noise: float = 1e-3, oversample: int = 4,
           tol: float = 1e-8, first: int = 0, count: Optional[int] = None) -> List[Problem]:
    """Independent problems A_p = G_p diag(logspace(0, -6, n_p)) in FP32.

    Sizes m_p ~ U{m_lo..m_hi}, n_p ~ U{n_lo..n_hi} are drawn from one stream,
    so problem p has the same shape and values whether the whole batch or a
    slice [first, first + count) is requested.
    """
    root = np.random.SeedSequence([seed, FAMILY_IDS["ragged"]])
    shape_rng, *per = [np.random.Generator(np.random.PCG64(c)) for c in root.spawn(1 + nprob)]
    ms = shape_rng.integers(m_lo, m_hi + 1, size=nprob)
    ns = shape_rng.integers(n_lo, n_hi + 1, size=nprob)
    ns = np.minimum(ns, ms)
    count = nprob - first if count is None else count
    lams = np.logspace(math.log10(lam_lo), math.log10(lam_hi), N)
    out = []
    for p in range(first, first + count):
        m, n = int(ms[p]), int(ns[p])
        rg = per[p]
        sigma = np.logspace(0.0, -6.0, n)
        A = _gaussian_colmajor(rg, m, n, np.float32)
        A *= sigma.astype(np.float32)[None, :]
        x0 = rg.standard_normal(n)
        b = A.astype(np.float64) @ x0 + noise * rg.standard_normal(m)
        out.append(Problem("ragged", A, b, lams.copy(), min(oversample * n, m), "gauss", "chol",
                           tol, seed * 100003 + p, x0=x0))
    return out


def ragged_shapes(nprob: int = 256, m_lo: int = 5000, m_hi: int = 50000, n_lo: int = 100,
                  n_hi: int = 1000, seed: int = 0):
    """The (m_p, n_p) list of the ragged family without drawing the matrices."""
    root = np.random.SeedSequence([seed, FAMILY_IDS["ragged"]])
    shape_rng = np.random.Generator(np.random.PCG64(root.spawn(1 + nprob)[0]))
    ms = shape_rng.integers(m_lo, m_hi + 1, size=nprob)
    ns = shape_rng.integers(n_lo, n_hi + 1, size=nprob)
    return [(int(a), int(min(b, a))) for a, b in zip(ms, ns)]


# Full-size instances of the five benchmark workloads.
def full(name: str, **kw):
    if name == "over_svd":
        return over_svd(**kw)
    if name == "over_gauss":
        return over_gauss(**kw)
    if name == "under_scaled":
        return under_scaled(**kw)
    if name == "lowsd":
        return lowsd(**kw)
    if name == "ragged":
        return ragged(**kw)
    raise KeyError(name)
