"""Test-side checks of a factorization on the GPU with plain torch FP64 ops
(no part of the method: these only read the GEQP3-format output).

``residual_orth`` forms A P - Q R and Q^T Q - I by applying the stored
reflectors block by block (compact WY with T from the UT identity
T^{-1} = diag(1/tau) + striu(Y^T Y)), so it runs at sizes where the oracle's
explicit, reflector-by-reflector Q would take too long.
"""
import torch


def _apply_q(A, tau, rank, X, nb=256):
    """X <- Q X with Q = H_0 ... H_{rank-1} from A's stored reflectors."""
    for s in reversed(range(0, rank, nb)):
        k = min(nb, rank - s)
        y = torch.tril(A[s:, s:s + k], -1)
        y[:k, :k] += torch.eye(k, dtype=A.dtype, device=A.device)
        t_inv = torch.diag(1.0 / tau[s:s + k]) + torch.triu(y.t() @ y, 1)
        t = torch.linalg.solve_triangular(t_inv, torch.eye(k, dtype=A.dtype, device=A.device),
                                          upper=True)
        X[s:] -= y @ (t @ (y.t() @ X[s:]))
    return X


def residual_orth(A0, A, jpiv, tau, rank):
    """(||A0 P - Q R||_F / ||A0||_F, ||Q^T Q - I||_F) with Q's first n columns;
    the residual block A(rank:, rank:) is part of R's place in the output."""
    m, n = A.shape
    x = torch.zeros(m, n, dtype=A.dtype, device=A.device)
    x[:rank] = torch.triu(A[:rank])
    if rank < n:
        x[rank:, rank:] = A[rank:, rank:]
    _apply_q(A, tau, rank, x)
    res = float(torch.linalg.norm(A0[:, jpiv] - x) / torch.linalg.norm(A0))
    del x
    kq = min(rank, n)
    q = torch.zeros(m, kq, dtype=A.dtype, device=A.device)
    q[:kq, :kq] = torch.eye(kq, dtype=A.dtype, device=A.device)
    _apply_q(A, tau, rank, q)
    orth = float(torch.linalg.norm(q.t() @ q - torch.eye(kq, dtype=A.dtype, device=A.device)))
    return res, orth


def r_rows_by_column(a_out, jpiv, rows):
    """R(0:rows, :) keyed by original column index: out[:, j] is the column of
    R that belongs to input column j (entries below the diagonal zeroed)."""
    import numpy as np
    r = np.triu(np.asarray(a_out)[:rows])
    out = np.empty_like(r)
    out[:, np.asarray(jpiv)] = r
    return out
