"""Seeded synthetic inputs for the QRCP tests and benchmark.

This module only *builds input matrices*; it holds none of the factorization's
arithmetic (no sketch, no pivoting, no QR of the input).  Both the CPU oracle
and the HIP library consume the same bytes produced here.

Recipes (the paper measures on synthetic matrices only: i.i.d. Gaussian inputs
for performance and a Kahan matrix for pivot quality, Sec. 1.4 and Sec. 6):

* ``usv``      A = U diag(sigma) V^T with U, V the orthonormal factors of
               seeded Gaussian matrices (the spectrum is prescribed).
* ``lowrank``  A = G1 G2 + eps * N, G1, G2, N seeded Gaussians (exact rank r
               plus a noise floor).
* ``gaussian`` i.i.d. N(0,1) entries (the paper's performance matrices).
* ``kahan``    the Kahan matrix in the parameterisation of Sec. 6 (equation
               for M with alpha = sin(theta), beta = -cos(theta)).

Every builder returns a Fortran-ordered (column-major) float64 array so that
``A.ctypes.data`` / a torch view of it is directly the LAPACK layout.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream)])


def _orth(g: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the columns of a Gaussian matrix (input building only)."""
    q, r = np.linalg.qr(g)
    # fix the column signs so the result does not depend on the LAPACK build
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


def spectrum(kind: str, n: int, **kw) -> np.ndarray:
    """Singular-value profiles used by the workloads.

    geometric: sigma_i = lo ** (i/(n-1)), i = 0..n-1 (1 down to ``lo``)
    power:     sigma_i = (i+1) ** (-p)
    rank:      sigma_i = (i+1) ** -1 for i < r, else 0
    """
    i = np.arange(n, dtype=np.float64)
    if kind == "geometric":
        lo = kw.get("lo", 1e-10)
        return lo ** (i / max(n - 1, 1))
    if kind == "power":
        return (i + 1.0) ** (-kw.get("p", 2.0))
    if kind == "rank":
        r = kw["r"]
        s = 1.0 / (i + 1.0)
        s[r:] = 0.0
        return s
    raise ValueError(kind)


def usv(m: int, n: int, sigma: np.ndarray, seed: int) -> np.ndarray:
    """A = U diag(sigma) V^T, U = orth(G_U, m x n), V = orth(G_V, n x n)."""
    assert len(sigma) == n and m >= n
    u = _orth(_rng(seed, 1).standard_normal((m, n)))
    v = _orth(_rng(seed, 2).standard_normal((n, n)))
    return np.asfortranarray((u * sigma) @ v.T)


def lowrank(m: int, n: int, r: int, noise: float, seed: int) -> np.ndarray:
    g1 = _rng(seed, 3).standard_normal((m, r))
    g2 = _rng(seed, 4).standard_normal((r, n))
    a = g1 @ g2
    if noise:
        a += noise * _rng(seed, 5).standard_normal((m, n))
    return np.asfortranarray(a)


def gaussian(m: int, n: int, seed: int) -> np.ndarray:
    return np.asfortranarray(_rng(seed, 7).standard_normal((m, n)))


def orthogonal_columns(m: int, n: int, sigma: np.ndarray, seed: int):
    """A = Q diag(sigma) Pi^T with orthonormal Q and a random column permutation.

    Returns (A, perm) where column j of A is sigma[perm_inv[j]] * q_{perm_inv[j]};
    i.e. ``perm[t]`` is the column of A holding the t-th largest norm when
    ``sigma`` is sorted in decreasing order.
    """
    q = _orth(_rng(seed, 8).standard_normal((m, n)))
    perm = _rng(seed, 9).permutation(n)
    a = np.empty((m, n), order="F")
    a[:, perm] = q * sigma
    return a, perm


def kahan(n: int, p: float = 1000.0, theta: float = 1.2) -> np.ndarray:
    """Kahan matrix as parameterised in Sec. 6: diag(alpha^i) * T + eps*p*diag(n..1),
    T upper triangular with beta on the diagonal and 1 above it."""
    alpha, beta = math.sin(theta), -math.cos(theta)
    t = np.triu(np.ones((n, n)), 1) + beta * np.eye(n)
    d = alpha ** np.arange(n, dtype=np.float64)
    a = d[:, None] * t + np.finfo(np.float64).eps * p * np.diag(np.arange(n, 0, -1, dtype=np.float64))
    return np.asfortranarray(a)


def config_matrix(name: str, seed: int | None = None) -> tuple[np.ndarray, dict]:
    """Host-side builders for the small named workloads (the 16384^2 and larger
    ones are built on the device by ``workloads.device``)."""
    if name == "c1":
        m, n = 1024, 512
        seed = 20250701 if seed is None else seed
        a = usv(m, n, spectrum("geometric", n, lo=1e-10), seed)
        return a, dict(m=m, n=n, b=64, gamma=1.25, tol=0.0, sketch_seed=42)
    raise ValueError(name)
