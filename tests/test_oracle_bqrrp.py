"""End-to-end pins of the BQRRP oracle (Alg. 1 with Alg. 2 and Alg. 3).

What fixes the result independently of the oracle's own code:
* the GEQP3 output format (Sec. 1.3): A P = Q R with Q from the stored
  reflectors, R upper trapezoidal, J a permutation -> residual and
  orthogonality bounds;
* a single block (b >= n) is an unpivoted QR of the LU-pivoted matrix, so R
  equals NumPy's R of A[:, J] up to row signs;
* orthogonal columns with well separated norms: Businger-Golub (LAPACK
  DGEQP3) pivots are known in closed form (sorted norms) and R = diag(+-sigma);
* exact-rank inputs give that rank (Sec. 2.2: with exact rank detection the
  method returns l = rank(M));
* exact power-of-two scaling commutes with every step (bitwise), and a column
  permutation of the input only relabels the pivots.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads as W
from oracle import bqrrp as O


def _check_format(a0, res, resid_tol=1e-12, orth_tol=1e-12):
    m, n = a0.shape
    assert sorted(res.jpiv.tolist()) == list(range(n))
    l = res.rank
    assert np.all(res.tau[l:] == 0.0)
    assert np.all((res.tau[:l] >= 1.0 - 1e-12) & (res.tau[:l] <= 2.0 + 1e-12))
    resid, orth = O.residual_and_orth(a0, res)
    assert resid <= resid_tol, resid
    assert orth <= orth_tol, orth
    return resid, orth


def test_c1_config_parity_bars():
    a, cfg = W.config_matrix("c1")
    res = O.bqrrp(a, cfg["b"], cfg["gamma"], cfg["sketch_seed"], cfg["tol"])
    assert res.status == O.OK and res.rank == 512
    _check_format(a, res)
    # rank-revealing: |R_kk| tracks sigma_k within a modest factor
    sig = W.spectrum("geometric", 512, lo=1e-10)
    ratio = np.abs(np.diag(res.a)[:512]) / sig
    assert ratio.min() > 1e-3 and ratio.max() < 1e3


def test_cholqr2_option_same_pivots():
    a, cfg = W.config_matrix("c1")
    r1 = O.bqrrp(a, 64, 1.25, 42, 0.0, cholqr_passes=1)
    r2 = O.bqrrp(a, 64, 1.25, 42, 0.0, cholqr_passes=2)
    assert np.array_equal(r1.jpiv, r2.jpiv)
    _check_format(a, r2)


@pytest.mark.parametrize("m,n,b", [(300, 300, 64), (400, 171, 32), (128, 128, 128), (97, 61, 16)])
def test_shapes_ragged_and_square(m, n, b):
    a = W.usv(m, n, W.spectrum("power", n, p=1.0), seed=m * n)
    res = O.bqrrp(a, b, 1.25, 11, 0.0)
    assert res.rank == n
    _check_format(a, res)


def test_single_block_is_qr_of_pivoted_matrix():
    a = W.gaussian(90, 40, seed=3)
    res = O.bqrrp(a, 64, 1.25, 5, 0.0)
    r_np = np.linalg.qr(a[:, res.jpiv], mode="r")
    r = np.triu(res.a[:40])
    sgn = np.sign(np.diag(r)) * np.sign(np.diag(r_np))
    assert np.max(np.abs(r - sgn[:, None] * r_np)) < 1e-12 * np.linalg.norm(a)


def test_single_block_pivots_are_lu_pivots_of_sketch():
    a = W.gaussian(90, 40, seed=4)
    d = 80
    msk = O.sketch_operator(d, 90, 9) @ a
    res = O.bqrrp(a, 64, 1.25, 9, 0.0)
    _, piv = sl.lu_factor(msk.T)
    assert np.array_equal(res.jpiv, O.piv_transform(piv[: min(d, 40)], 40))


def test_businger_golub_closed_form_orthogonal_columns():
    """A = Q diag(sigma) Pi^T, sigma_j = r^-j: column-norm pivoting (DGEQP3)
    picks the columns in sigma order and R = diag(+-sigma).  The LU pivots on
    the sketch agree unless a Gaussian draw reverses a pair, which has
    probability about (2/pi)/r per adjacent pair."""
    m, n, b, r = 64, 12, 4, 1e4
    sigma = r ** -np.arange(n, dtype=np.float64)
    agree = 0
    trials = 300
    for seed in range(trials):
        a, perm = W.orthogonal_columns(m, n, sigma, seed)
        _, _, p_bg = sl.qr(a, pivoting=True, mode="economic")
        assert np.array_equal(p_bg, perm)                 # brute-force BG = closed form
        res = O.bqrrp(a, b, 1.25, seed + 1000, 0.0)
        if np.array_equal(res.jpiv, perm):
            agree += 1
            assert np.allclose(np.abs(np.diag(res.a)[:n]), sigma, rtol=1e-10)
    assert agree >= trials - 2, agree


def test_geqp3_on_sketch_variant_matches_bg():
    m, n, b, r = 64, 12, 4, 100.0
    sigma = r ** -np.arange(n, dtype=np.float64)
    agree = 0
    for seed in range(100):
        a, perm = W.orthogonal_columns(m, n, sigma, seed)
        res = O.bqrrp(a, b, 2.0, seed + 7, 0.0, qrcp_wide="geqp3")
        agree += np.array_equal(res.jpiv, perm)
        _check_format(a, res)
    assert agree >= 99, agree


@pytest.mark.parametrize("r,b", [(40, 16), (48, 16), (1, 8)])
def test_exact_rank_detected(r, b):
    a = W.lowrank(200, 120, r, 0.0, seed=r)
    res = O.bqrrp(a, b, 1.25, 3, 1e-10)
    assert res.rank == r
    resid, orth = _check_format(a, res)
    # trailing block ~ 0
    trail = res.a[r:, r:]
    assert np.linalg.norm(trail) <= 1e-12 * np.linalg.norm(a)


def test_zero_matrix_rank_zero():
    a = np.zeros((50, 20), order="F")
    res = O.bqrrp(a, 8, 1.25, 1, 0.0)
    assert res.rank == 0 and not res.tau.any()
    assert np.array_equal(res.jpiv, np.arange(20))
    assert not res.a.any()


def test_nonfinite_input_reports_status():
    a = W.gaussian(40, 20, seed=1)
    a[3, 4] = np.nan
    res = O.bqrrp(a, 8, 1.25, 1, 0.0)
    assert res.status == O.ERR_NONFINITE


def test_power_of_two_scaling_is_bitwise():
    a = W.usv(256, 128, W.spectrum("geometric", 128, lo=1e-6), seed=8)
    r1 = O.bqrrp(a, 32, 1.25, 4, 0.0)
    r2 = O.bqrrp(a * 2.0 ** 7, 32, 1.25, 4, 0.0)
    assert np.array_equal(r1.jpiv, r2.jpiv)
    assert np.array_equal(r1.tau, r2.tau)
    upper = np.triu(np.ones_like(a, dtype=bool))
    assert np.array_equal(r1.a[upper] * 2.0 ** 7, r2.a[upper])
    assert np.array_equal(r1.a[~upper], r2.a[~upper])


def test_column_permutation_only_relabels_pivots():
    a = W.usv(256, 128, W.spectrum("geometric", 128, lo=1e-6), seed=9)
    pi = np.random.default_rng(0).permutation(128)
    r1 = O.bqrrp(a, 32, 1.25, 4, 0.0)
    r2 = O.bqrrp(np.asfortranarray(a[:, pi]), 32, 1.25, 4, 0.0)
    assert np.array_equal(pi[r2.jpiv], r1.jpiv)
    assert np.max(np.abs(np.triu(r1.a) - np.triu(r2.a))) < 1e-13 * np.linalg.norm(a)


def test_tall_matrix_and_canonical_flops():
    a = W.usv(600, 150, W.spectrum("geometric", 150, lo=1e-12), seed=12)
    res = O.bqrrp(a, 32, 1.25, 2, 0.0)
    _check_format(a, res)
    assert O.canonical_flops(16384, 16384) == pytest.approx(5.864062014e12, rel=1e-9)
    assert O.truncated_flops(100, 100, 100) == pytest.approx(O.canonical_flops(100, 100))


def test_fp32_trailing_and_bf16_sketch_variants_run():
    a = W.usv(512, 256, W.spectrum("geometric", 256, lo=1e-14), seed=13)
    res = O.bqrrp(a, 32, 1.25, 2, 0.0, sketch_precision="bf16", cholqr_passes=2)
    _check_format(a, res)
    res = O.bqrrp(a, 32, 1.25, 2, 0.0, sketch_precision="bf16", cholqr_passes=2,
                  trailing_precision="f32")
    resid, orth = O.residual_and_orth(a, res)
    assert resid < 1e-5 and orth < 1e-10
