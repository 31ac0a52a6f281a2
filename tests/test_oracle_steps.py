"""Pins of the oracle's sub-steps against LAPACK (via SciPy), closed forms and
brute force.  Each test names the step of the paper it pins."""
import numpy as np
import pytest
import scipy.linalg as sl
from scipy.linalg import lapack

from oracle import bqrrp as O


def _rng(s):
    return np.random.default_rng(s)


# ---- Alg. 2: GETRF pivots and the pivot-format conversion -------------------
@pytest.mark.parametrize("shape", [(200, 40), (40, 40), (513, 80), (37, 80)])
def test_getrf_pivots_equal_lapack(shape):
    x = _rng(shape[0]).standard_normal(shape)
    ipiv, _ = O.getrf_pivots(x)
    _, piv = sl.lu_factor(x)
    assert np.array_equal(ipiv, piv[: len(ipiv)])


def test_getrf_zero_column_keeps_position():
    x = _rng(1).standard_normal((30, 6))
    x[:, 2] = 0.0
    x[5:, 3] = 0.0  # after elimination the 4th column is still nonzero above
    ipiv, _ = O.getrf_pivots(x)
    _, piv = sl.lu_factor(x)
    assert np.array_equal(ipiv, piv[:6])
    assert ipiv[2] == 2


def test_getrf_tie_takes_smallest_position():
    x = np.zeros((6, 2))
    x[[1, 4], 0] = [-3.0, 3.0]
    x[:, 1] = np.arange(6)
    ipiv, m = O.getrf_pivots(x)
    assert ipiv[0] == 1 and m[0] == 0.0


def test_piv_transform_matches_lu_permutation():
    x = _rng(2).standard_normal((120, 30))
    ipiv, _ = O.getrf_pivots(x)
    jq = O.piv_transform(ipiv, 120)
    p, l, u = sl.lu(x)                 # x = P L U  ->  (P^T x) = L U
    assert np.array_equal(x[jq], p.T @ x)
    assert sorted(jq) == list(range(120))


# ---- GEQRF (Householder, DLARFG convention) ---------------------------------
@pytest.mark.parametrize("shape", [(80, 300), (80, 80), (100, 37), (5, 9)])
def test_householder_qr_equals_dgeqrf(shape):
    a = _rng(sum(shape)).standard_normal(shape)
    r, v, tau = O.householder_qr(a)
    qr, tau_l, _, info = lapack.dgeqrf(a)
    assert info == 0
    kk = min(shape)
    scale = np.abs(a).max()
    assert np.max(np.abs(r[:kk] - np.triu(qr)[:kk])) < 1e-13 * scale * max(shape)
    assert np.allclose(tau, tau_l, rtol=1e-12, atol=1e-14)
    assert np.allclose(np.tril(v, -1)[:, :kk], np.tril(qr, -1)[:, :kk], rtol=1e-10, atol=1e-12)


def test_larfg_special_cases():
    beta, v, tau = O.larfg(2.0, np.zeros(3))
    assert beta == 2.0 and tau == 0.0 and not v.any()
    beta, v, tau = O.larfg(0.0, np.array([3.0, 4.0]))
    assert beta == -5.0 and tau == 1.0
    assert np.allclose(v, [0.6, 0.8])
    beta, v, tau = O.larfg(-3.0, np.array([4.0]))
    assert beta == 5.0 and np.isclose(tau, 1.6)


def test_geqrf_oracle_equals_dgeqrf():
    a = _rng(9).standard_normal((150, 60))
    out, tau = O.geqrf(a)
    qr, tau_l, _, _ = lapack.dgeqrf(a)
    assert np.allclose(out, qr, rtol=1e-11, atol=1e-12)
    assert np.allclose(tau, tau_l, rtol=1e-12)
    q = O.form_q(out, tau, ncols=60)
    assert np.linalg.norm(q @ np.triu(out[:60]) - a) < 1e-12 * np.linalg.norm(a)


def test_qrcp_wide_lu_is_permuted_qr():
    msk = _rng(4).standard_normal((40, 200))
    jsk, rsk, ipiv, _ = O.qrcp_wide_lu(msk)
    # Rsk is an R factor of the permuted sketch: Rsk^T Rsk = (M P)^T (M P)
    mp = msk[:, jsk]
    assert np.allclose(rsk.T @ rsk, mp.T @ mp, rtol=1e-10, atol=1e-10)
    # first b pivots do not depend on how many extra sketch rows were used
    # beyond b when the sketch grows (the LU pivot column order only
    # depends on the leading rows): pin with the transposed-LU definition
    _, piv = sl.lu_factor(msk.T)
    assert np.array_equal(jsk, O.piv_transform(piv[:40], 200))


# ---- tri_rank (Sec. 2.2) ----------------------------------------------------
def test_tri_rank_cases():
    r = np.diag([3.0, 2.0, 1e-12, 1.0])
    assert O.tri_rank(r, 4, tol=1e-10, ref=3.0) == 2
    assert O.tri_rank(r, 4, tol=0.0, ref=3.0) == 4
    assert O.tri_rank(np.diag([1.0, np.nan, 1.0]), 3, 0.0, 1.0) == 1
    assert O.tri_rank(np.zeros((3, 3)), 3, 0.0, 0.0) == 0
    assert O.tri_rank(r, 2, tol=0.5, ref=3.0) == 2


# ---- Cholesky QR (Alg. 3, App. B) ---------------------------------------------
def test_cholesky_upper_equals_numpy():
    a = _rng(5).standard_normal((60, 20))
    g = a.T @ a
    r, t = O.cholesky_upper(g)
    assert t == 20
    assert np.allclose(r, np.linalg.cholesky(g).T, rtol=1e-12, atol=1e-12)


def test_cholesky_breakdown_index():
    a = _rng(6).standard_normal((60, 8))
    a[:, 5] = a[:, 1] - 2 * a[:, 3]          # exactly dependent column 5
    g = a.T @ a
    g[5, :] = g[:, 5] = 0.0
    _, t = O.cholesky_upper(g)
    assert t == 5


def test_cholqr_orthonormal_and_product():
    m = _rng(7).standard_normal((500, 30)) @ np.diag(np.logspace(0, -4, 30))
    for passes in (1, 2):
        q, rc, k = O.cholqr(m, passes)
        assert k == 30
        assert np.linalg.norm(q.T @ q - np.eye(30)) < (1e-8 if passes == 1 else 1e-14)
        assert np.linalg.norm(q @ rc - m) < 1e-13 * np.linalg.norm(m)
        assert np.allclose(rc, np.triu(rc))


# ---- Householder reconstruction (Alg. 3, ORHR_COL) ----------------------------
@pytest.mark.parametrize("m,k", [(300, 40), (64, 64), (100, 1)])
def test_reconstruction_reproduces_q(m, k):
    q, _ = np.linalg.qr(_rng(m + k).standard_normal((m, k)))
    y, tau, dsig, u = O.householder_reconstruct(q)
    assert np.allclose(np.triu(y, 1), 0) and np.allclose(np.diag(y), 1)
    assert np.all(tau >= 1.0 - 1e-14) and np.all(tau <= 2.0 + 1e-14)
    # H = H_0 ... H_{k-1} applied to [I; 0] by LAPACK's DORMQR
    h, _, info = lapack.dormqr("L", "N", y, tau, np.eye(m, k), lwork=max(1, 64 * k))
    assert info == 0
    assert np.max(np.abs(h - q * dsig)) < 1e-14 * np.sqrt(m)
    assert np.allclose(tau, -dsig * np.diag(u))


def test_larft_equals_dormqr_transpose():
    m, k, n = 200, 24, 31
    q, _ = np.linalg.qr(_rng(11).standard_normal((m, k)))
    y, tau, _, _ = O.householder_reconstruct(q)
    c = _rng(12).standard_normal((m, n))
    t = O.larft(y, tau)
    ours = O.apply_qt(y, t, c)
    ref, _, info = lapack.dormqr("L", "T", y, tau, c, lwork=64 * n)
    assert info == 0
    assert np.max(np.abs(ours - ref)) < 1e-13 * np.abs(c).max()
    # the UT-transform identity: T^{-1} = diag(1/tau) + strictly-upper(Y^T Y)
    tinv = np.diag(1 / tau) + np.triu(y.T @ y, 1)
    assert np.allclose(np.linalg.inv(tinv), t, rtol=1e-10, atol=1e-12)


# ---- sketch update (Alg. 1 last step; Duersch-Gu Sec. 4) -----------------------
def test_sketch_update_is_sketch_of_trailing_block():
    """Brute force on a small problem: after block 0 the updated sketch equals
    W(:, b:) R22 with W = Qsk^T S Q, where S A P = Qsk Rsk and Q is the full
    orthogonal factor of block 0's reflectors."""
    m, n, b, gamma, seed = 60, 24, 6, 1.5, 3
    a = _rng(13).standard_normal((m, n)) @ np.diag(np.logspace(0, -3, n))
    d = int(np.ceil(gamma * b))
    s_op = O.sketch_operator(d, m, seed)
    msk = s_op @ a
    jsk, rsk, _, _ = O.qrcp_wide_lu(msk)
    qsk = msk[:, jsk][:, :d] @ np.linalg.inv(rsk[:, :d])
    res = O.bqrrp(a, b, gamma, seed, 0.0, msk=msk)
    # recover block 0's reflectors from the output (first b columns)
    q_full = O.form_q(res.a[:, :b], res.tau[:b], ncols=m)
    assert np.linalg.norm(q_full.T @ q_full - np.eye(m)) < 1e-12
    # trailing block after block 0: Q^T A P restricted to rows b:, cols b:
    ap0 = a[:, jsk]
    r_full = q_full.T @ ap0
    w = qsk.T @ s_op @ q_full
    expected = w[:, b:] @ r_full[b:, b:]
    # the oracle's own updated sketch is the input of its block 1
    res = O.bqrrp(a, b, gamma, seed, 0.0, msk=msk, trace_sketch=True)
    got = res.trace[1].msk_in
    assert np.linalg.norm(got - expected) < 1e-12 * np.linalg.norm(msk)
    # and the identity W(:, :b) = [Rsk11 R11^{-1}; 0]
    r11 = np.triu(r_full[:b, :b])
    assert np.linalg.norm(w[:, :b] @ r11 - rsk[:, :b]) < 1e-12 * np.linalg.norm(msk)
