"""Device-side builders of the large seeded workloads (16384^2 and up).

Input building only (no part of the factorization): Gaussian matrices from a
seeded torch generator, orthonormal factors from torch's QR, products with
torch matmul, all in FP64 on the GPU.  The result is returned column-major
(stride(0) == 1).
"""
from __future__ import annotations

import torch


def _gen(seed: int, stream: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1000003 + int(stream)) & 0x7FFFFFFFFFFFFFFF)
    return g


def _colmajor(a: torch.Tensor) -> torch.Tensor:
    return a.t().contiguous().t()


def gaussian(m: int, n: int, seed: int, stream: int = 7, device="cuda") -> torch.Tensor:
    g = _gen(seed, stream, device)
    # generated as the (n, m) row-major transpose: that is (m, n) column-major
    return torch.randn(n, m, generator=g, dtype=torch.float64, device=device).t()


def orth(m: int, n: int, seed: int, stream: int, device="cuda") -> torch.Tensor:
    q, r = torch.linalg.qr(torch.randn(m, n, generator=_gen(seed, stream, device),
                                       dtype=torch.float64, device=device))
    s = torch.sign(torch.diagonal(r))
    s[s == 0] = 1.0
    return q * s


def usv(m: int, n: int, sigma: torch.Tensor, seed: int, device="cuda") -> torch.Tensor:
    """A = U diag(sigma) V^T with U = orth(m x n), V = orth(n x n)."""
    u = orth(m, n, seed, 1, device)
    v = orth(n, n, seed, 2, device)
    u.mul_(sigma.to(device=device, dtype=torch.float64)[None, :])
    a = u @ v.t()
    del u, v
    return _colmajor(a)


def power_spectrum(n: int, p: float = 2.0) -> torch.Tensor:
    return (torch.arange(n, dtype=torch.float64) + 1.0) ** (-p)


def geometric_spectrum(n: int, lo: float) -> torch.Tensor:
    i = torch.arange(n, dtype=torch.float64)
    return lo ** (i / max(n - 1, 1))


def lowrank(m: int, n: int, r: int, noise: float, seed: int, device="cuda") -> torch.Tensor:
    g1 = torch.randn(m, r, generator=_gen(seed, 3, device), dtype=torch.float64, device=device)
    g2 = torch.randn(r, n, generator=_gen(seed, 4, device), dtype=torch.float64, device=device)
    a = g1 @ g2
    del g1, g2
    if noise:
        a.add_(torch.randn(m, n, generator=_gen(seed, 5, device), dtype=torch.float64,
                           device=device), alpha=noise)
    return _colmajor(a)
