"""Pins of the oracle's further options, each against something other than
the oracle itself:

* any aspect ratio (Sec. 1.3): for m < n, A P = Q R with R m x n upper
  trapezoidal; R equals NumPy's R of A[:, J] up to row signs (uniqueness of
  the QR of a matrix whose leading m x m block is nonsingular);
* truncated output (a GEQP3RK-style stop at max_rank): the blocks before the
  stop are those of the full factorization (pivots identical, R rows equal);
  ||A||_F^2 = ||R(0:l, :)||_F^2 + ||A(l:, l:)||_F^2 (Q is orthogonal), and the
  residual block is at least the best rank-l error (Eckart-Young);
* Householder panel (qr_tall = GEQRF, Sec. 2.3): its panel step is LAPACK's
  dgeqrf; both panels factor the same pivoted matrix, so the pivots agree
  and R agrees up to row signs (QR uniqueness), and the sketch update is
  invariant to those row signs (Rsk11 R11^{-1} R12).
"""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W
from oracle import bqrrp as O


def _resid_orth_full(a0, res):
    """||A P - Q [R; residual]||_F / ||A||_F with the full Q of the stored
    reflectors, and ||Q_l^T Q_l - I||_F."""
    m, n = a0.shape
    l = res.rank
    q = O.form_q(res.a, res.tau[:l], ncols=m)
    rr = np.zeros((m, n))
    rr[:l] = np.triu(res.a[:l])
    rr[l:, l:] = res.a[l:, l:]
    nrm = np.linalg.norm(a0)
    return (np.linalg.norm(a0[:, res.jpiv] - q @ rr) / nrm,
            np.linalg.norm(q[:, :l].T @ q[:, :l] - np.eye(l)))


def _rows_by_column(a_out, jpiv, rows):
    """R(0:rows, :) with its columns put back in input-column order."""
    out = np.empty((rows, a_out.shape[1]))
    out[:, jpiv] = np.triu(a_out[:rows])
    return out


@pytest.mark.parametrize("m,n,b", [(96, 160, 32), (100, 300, 64), (64, 64 + 37, 16), (40, 200, 64)])
def test_wide_matrix_is_qr_of_pivoted_matrix(m, n, b):
    a = W.gaussian(m, n, seed=m + n)
    res = O.bqrrp(a, b, 1.25, 5, 0.0)
    assert res.rank == m
    assert sorted(res.jpiv.tolist()) == list(range(n))
    assert np.all((res.tau >= 1.0 - 1e-12) & (res.tau <= 2.0 + 1e-12))
    resid, orth = O.residual_and_orth(a, res)
    assert resid <= 1e-12 and orth <= 1e-12
    r_np = np.linalg.qr(a[:, res.jpiv], mode="r")
    r_or = np.triu(res.a[:m])
    sign = np.sign(np.diag(r_or)) * np.sign(np.diag(r_np))
    assert np.max(np.abs(r_or - sign[:, None] * r_np)) <= 1e-12 * np.linalg.norm(a)


def test_wide_exact_rank():
    a = W.lowrank(80, 200, 30, 0.0, seed=3)
    res = O.bqrrp(a, 16, 1.25, 2, 1e-12)
    assert res.rank == 30
    resid, _ = _resid_orth_full(a, res)
    assert resid <= 1e-12


@pytest.mark.parametrize("lim,b", [(64, 32), (96, 32), (50, 32), (17, 16), (1, 8)])
def test_truncated_output_prefix_of_full_run(lim, b):
    m, n = 300, 160
    a = W.usv(m, n, W.spectrum("geometric", n, lo=1e-8), seed=21)
    full = O.bqrrp(a, b, 1.25, 9, 0.0)
    tr = O.bqrrp(a, b, 1.25, 9, 0.0, max_rank=lim)
    assert tr.rank == lim
    assert full.min_margin() >= 1e-8
    assert np.array_equal(tr.jpiv[:lim], full.jpiv[:lim])
    assert np.all(tr.tau[lim:] == 0.0)
    nrm = np.linalg.norm(a)
    err = np.max(np.abs(_rows_by_column(tr.a, tr.jpiv, lim) - _rows_by_column(full.a, full.jpiv, lim)))
    if lim % b == 0:
        assert err == 0.0            # the same blocks, the same arithmetic
    else:
        assert err <= 1e-13 * nrm    # the last panel is narrower
    resid, orth = _resid_orth_full(a, tr)
    assert resid <= 1e-12 and orth <= 1e-12
    # Q orthogonal: the Frobenius norm splits over R's rows and the residual
    rn = np.linalg.norm(np.triu(tr.a[:lim]))
    en = np.linalg.norm(tr.a[lim:, lim:])
    assert abs(rn ** 2 + en ** 2 - nrm ** 2) <= 1e-13 * nrm ** 2
    # Eckart-Young: no rank-l approximation beats the tail singular values
    sig = np.linalg.svd(a, compute_uv=False)
    assert en >= np.sqrt(np.sum(sig[lim:] ** 2)) * (1 - 1e-12)


def test_truncated_output_zero_and_beyond():
    a = W.gaussian(60, 40, seed=4)
    r0 = O.bqrrp(a, 16, 1.25, 1, 0.0, max_rank=0)
    assert r0.rank == 0 and np.array_equal(r0.a, a) and np.array_equal(r0.jpiv, np.arange(40))
    rb = O.bqrrp(a, 16, 1.25, 1, 0.0, max_rank=1000)
    rf = O.bqrrp(a, 16, 1.25, 1, 0.0)
    assert rb.rank == 40 and np.array_equal(rb.a, rf.a) and np.array_equal(rb.jpiv, rf.jpiv)


def test_householder_panel_is_dgeqrf():
    # single block: the HQR panel is GEQRF of A[:, J], i.e. LAPACK dgeqrf
    a = W.usv(200, 48, W.spectrum("geometric", 48, lo=1e-6), seed=8)
    res = O.bqrrp(a, 64, 1.25, 4, 0.0, qr_tall="geqrf")
    qr, tau_l = sl.qr(a[:, res.jpiv], mode="raw")[0]
    nrm = np.linalg.norm(a)
    assert np.max(np.abs(np.triu(res.a[:48]) - np.triu(qr[:48]))) <= 1e-13 * nrm
    # tau of reflector j is fixed only to about eps * kappa (1e6 here)
    np.testing.assert_allclose(res.tau, tau_l, rtol=1e-9, atol=0)
    assert np.max(np.abs(np.tril(res.a, -1) - np.tril(qr, -1))) <= 1e-10


@pytest.mark.parametrize("m,n,b", [(1024, 512, 64), (300, 171, 32), (97, 61, 16), (80, 200, 32)])
def test_householder_panel_agrees_with_cholqr_panel(m, n, b):
    if m >= n:
        a = W.usv(m, n, W.spectrum("geometric", n, lo=1e-10), seed=m + 3)
    else:
        a = W.gaussian(m, n, seed=m + 3)
    rc = O.bqrrp(a, b, 1.25, 42, 0.0)
    rh = O.bqrrp(a, b, 1.25, 42, 0.0, qr_tall="geqrf")
    assert rh.rank == rc.rank == min(m, n)
    assert rc.min_margin() >= 1e-8 and rh.min_margin() >= 1e-8
    assert np.array_equal(rh.jpiv, rc.jpiv)
    l = rh.rank
    sign = np.sign(np.diag(rh.a)[:l]) * np.sign(np.diag(rc.a)[:l])
    nrm = np.linalg.norm(a)
    assert np.max(np.abs(np.triu(rh.a[:l]) - sign[:, None] * np.triu(rc.a[:l]))) <= 1e-12 * nrm
    resid, orth = O.residual_and_orth(a, rh)
    assert resid <= 1e-12 and orth <= 1e-12


def test_householder_panel_exact_rank():
    a = W.lowrank(400, 200, 70, 0.0, seed=13)
    res = O.bqrrp(a, 32, 1.25, 6, 1e-12, qr_tall="geqrf")
    assert res.rank == 70
    resid, orth = _resid_orth_full(a, res)
    assert resid <= 1e-12 and orth <= 1e-12
