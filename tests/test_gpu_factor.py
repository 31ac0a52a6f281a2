"""End-to-end parity of qrcp_factor / qrcp_geqrf (HIP, through the C ABI) with
the CPU oracle: identical pivots where the oracle's pivot margins are clear,
R within 1e-12 ||A||_F, residual and orthogonality within 1e-12."""
import numpy as np
import pytest

from oracle import bqrrp as O
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

R_TOL = 1e-12
MARGIN = 1e-8


@pytest.fixture(scope="module")
def Q():
    from paper_2507_00976_amd import qrcp
    return qrcp


def run_gpu(Q, a, b, gamma=1.25, seed=42, tol=0.0, **kw):
    A = Q.colmajor(torch.from_numpy(np.asarray(a, dtype=np.float64)).cuda())
    A, jpiv, tau, rank = Q.factor(A, b, gamma, seed, tol, **kw)
    torch.cuda.synchronize()
    return O.Result(a=A.cpu().numpy(), jpiv=jpiv.cpu().numpy(), tau=tau.cpu().numpy(), rank=rank)


def compare(a, got, ref, strict_pivots=True, tau_rtol=None):
    """Pivots identical when the oracle's pivot margins are clear; R to
    1e-12 ||A||_F (R is row-graded, so errors are absolute).  Y and tau belong
    to directions of singular value sigma_k and are determined only to about
    eps ||A|| / sigma_k, so they are compared elementwise only when the caller
    states a tolerance (well-conditioned inputs); otherwise they are checked
    through the residual and orthogonality bars."""
    assert got.rank == ref.rank
    if strict_pivots and ref.min_margin() >= MARGIN:
        assert np.array_equal(got.jpiv, ref.jpiv)
        nrm = np.linalg.norm(a)
        l = ref.rank
        assert np.max(np.abs(np.triu(got.a[:l]) - np.triu(ref.a[:l]))) <= R_TOL * nrm
        if tau_rtol is not None:
            np.testing.assert_allclose(got.tau, ref.tau, rtol=tau_rtol, atol=1e-12)
    assert sorted(got.jpiv.tolist()) == list(range(a.shape[1]))
    resid, orth = O.residual_and_orth(a, got)
    assert resid <= R_TOL and orth <= R_TOL, (resid, orth)


def test_c1_config(Q):
    a, cfg = W.config_matrix("c1")
    ref = O.bqrrp(a, cfg["b"], cfg["gamma"], cfg["sketch_seed"], cfg["tol"])
    got = run_gpu(Q, a, cfg["b"], cfg["gamma"], cfg["sketch_seed"], cfg["tol"])
    assert ref.min_margin() >= MARGIN
    compare(a, got, ref)


@pytest.mark.parametrize("m,n,b,gamma", [(300, 300, 64, 1.25), (400, 171, 32, 1.25), (128, 128, 128, 1.25),
                                         (97, 61, 16, 2.0), (600, 150, 32, 1.0), (1000, 999, 100, 1.5)])
def test_shapes(Q, m, n, b, gamma):
    a = W.usv(m, n, W.spectrum("power", n, p=1.0), seed=m * n)
    ref = O.bqrrp(a, b, gamma, 11, 0.0)
    got = run_gpu(Q, a, b, gamma, 11, 0.0)
    compare(a, got, ref, tau_rtol=1e-9)


@pytest.mark.parametrize("m,n,b", [(1, 1, 1), (5, 1, 1), (1, 5, 2), (2, 2, 1), (33, 3, 2), (3, 33, 8),
                                   (64, 64, 1), (17, 40, 40), (40, 17, 64)])
def test_degenerate_shapes(Q, m, n, b):
    # single rows or columns, one-column blocks (d = 2), blocks wider than the
    # matrix, sketches with more rows than the matrix
    a = W.gaussian(m, n, 100 + m + 7 * n + 11 * b)
    ref = O.bqrrp(a, b, 1.25, 42, 0.0)
    got = run_gpu(Q, a, b)
    compare(a, got, ref)


def test_cholqr2_option(Q):
    a, cfg = W.config_matrix("c1")
    ref = O.bqrrp(a, 64, 1.25, 42, 0.0, cholqr_passes=2)
    got = run_gpu(Q, a, 64, 1.25, 42, 0.0, cholqr_passes=2)
    compare(a, got, ref)


@pytest.mark.parametrize("r,b", [(40, 16), (48, 16), (1, 8)])
def test_exact_rank(Q, r, b):
    """G1 G2 of exact rank r: the rank and the r selected columns match the
    oracle.  The order of the other columns is decided by LU steps on the
    rounding noise of a rank-r sketch, so it is not unique (any order is a
    valid result); the exit-block tests below pin the whole order on inputs
    where it is determined."""
    a = W.lowrank(200, 120, r, 0.0, seed=r)
    ref = O.bqrrp(a, b, 1.25, 3, 1e-10)
    got = run_gpu(Q, a, b, 1.25, 3, 1e-10)
    assert got.rank == ref.rank == r
    resid, orth = O.residual_and_orth(a, got)
    assert resid <= 1e-12 and orth <= 1e-12
    assert np.linalg.norm(got.a[r:, r:]) <= 1e-12 * np.linalg.norm(a)
    if ref.min_margin() >= MARGIN:
        assert np.array_equal(got.jpiv[:r], ref.jpiv[:r])
    assert sorted(got.jpiv.tolist()) == list(range(a.shape[1]))


def _zero_column_matrix(m, n, r, seed):
    """r nonzero columns (spectrum (i+1)^-1) scattered among n - r zero columns:
    the sketch of a zero column is exactly zero, so every LU step among them is
    an exact tie decided by the smallest position (IDAMAX), identically on
    both sides."""
    b = W.usv(m, r, 1.0 / (np.arange(r) + 1.0), seed)
    a = np.zeros((m, n), order="F")
    a[:, np.random.default_rng(seed).permutation(n)[:r]] = b
    return a


def _gap_matrix(m, n, r, gap, seed):
    sig = 1.0 / (np.arange(n) + 1.0)
    sig[r:] *= gap
    return W.usv(m, n, sig, seed)


@pytest.mark.parametrize("kind,m,n,r,b,tol", [("zero", 300, 160, 70, 32, 0.0),
                                              ("zero", 500, 300, 100, 64, 0.0),
                                              ("gap", 300, 160, 70, 32, 1e-3),
                                              ("gap", 500, 300, 100, 64, 1e-3)])
def test_exit_block_whole_permutation(Q, kind, m, n, r, b, tol):
    """An early exit (tri_rank stops at r inside a block): every block runs the
    full GETRF of its sketch (Alg. 2), so the columns no block selects come out
    in the order the oracle gives, and the residual block A(r:, r:) holds them
    in that order.  The inputs make that order unique: exact zero columns
    (exact ties), or a spectrum gap of 1e-4 whose tail keeps clear LU margins."""
    a = _zero_column_matrix(m, n, r, 5) if kind == "zero" else _gap_matrix(m, n, r, 1e-4, 6)
    ref = O.bqrrp(a, b, 1.25, 3, tol)
    got = run_gpu(Q, a, b, 1.25, 3, tol)
    assert ref.rank == got.rank == r
    if kind == "gap":
        assert ref.min_margin() >= 1e-5
    assert np.array_equal(got.jpiv, ref.jpiv)
    nrm = np.linalg.norm(a)
    assert np.max(np.abs(np.triu(got.a[:r]) - np.triu(ref.a[:r]))) <= R_TOL * nrm
    assert np.max(np.abs(got.a[r:, r:] - ref.a[r:, r:])) <= R_TOL * nrm
    assert np.array_equal(got.tau[r:], np.zeros(min(m, n) - r))
    if kind == "zero":
        assert not got.a[r:, r:].any()
    # A P = Q [R11 R12; 0 A(r:, r:)] with the full Q of the r reflectors (the
    # residual block is not negligible for the gap input)
    q = O.form_q(got.a, got.tau[:r], ncols=m)
    rr = np.zeros((m, n))
    rr[:r] = np.triu(got.a[:r])
    rr[r:, r:] = got.a[r:, r:]
    assert np.linalg.norm(a[:, got.jpiv] - q @ rr) <= R_TOL * nrm
    assert np.linalg.norm(q[:, :r].T @ q[:, :r] - np.eye(r)) <= R_TOL


def test_zero_matrix(Q):
    a = np.zeros((64, 24))
    got = run_gpu(Q, a, 8)
    assert got.rank == 0 and not got.tau.any() and not got.a.any()
    assert np.array_equal(got.jpiv, np.arange(24))


def test_nonfinite_input(Q):
    a = W.gaussian(64, 24, seed=1)
    a[3, 4] = np.nan
    with pytest.raises(Q.QrcpError) as e:
        run_gpu(Q, a, 8)
    assert e.value.code == Q.QRCP_ERR_NONFINITE


def test_one_based_pivots(Q):
    a = W.gaussian(100, 40, seed=2)
    g0 = run_gpu(Q, a, 16)
    g1 = run_gpu(Q, a, 16, pivot_base=1)
    assert np.array_equal(g1.jpiv, g0.jpiv + 1)


def test_precision_variants(Q):
    """BF16 sketch (+ FP32 trailing update): parity unpinned by construction;
    checked by the stated accuracy bars."""
    a = W.usv(1024, 512, W.spectrum("geometric", 512, lo=1e-14), seed=13)
    g = run_gpu(Q, a, 64, 1.25, 42, 0.0, sketch_precision=1, cholqr_passes=2)
    resid, orth = O.residual_and_orth(a, g)
    assert resid < 1e-12 and orth < 1e-12
    g = run_gpu(Q, a, 64, 1.25, 42, 0.0, sketch_precision=1, cholqr_passes=2, trailing_precision=1)
    resid, orth = O.residual_and_orth(a, g)
    assert resid < 1e-5 and orth < 1e-10


@pytest.mark.parametrize("m,n,nb", [(1024, 512, 64), (300, 300, 32), (777, 333, 100)])
def test_geqrf_matches_oracle(Q, m, n, nb):
    a = W.gaussian(m, n, seed=m)
    A = Q.colmajor(torch.from_numpy(a).cuda())
    A, tau = Q.geqrf(A, nb)
    got = A.cpu().numpy()
    ref, tau_ref = O.geqrf(a)
    assert np.max(np.abs(np.triu(got) - np.triu(ref))) <= 1e-12 * np.linalg.norm(a)
    np.testing.assert_allclose(tau.cpu().numpy(), tau_ref, rtol=1e-10)
    assert np.max(np.abs(np.tril(got, -1) - np.tril(ref, -1))) <= 1e-10



@pytest.mark.parametrize("b", [128, 512])
def test_lowrank_rank_detection_repeatable(Q, b):
    """A = G1 G2 + 1e-12 N (exact rank 512 plus noise far below tol): the
    detected rank is 512, as the oracle's; the 512 selected columns are the
    oracle's and R(0:512, :) agrees column by column (keyed by input column:
    the order of the unselected columns is decided by LU steps on the noise,
    not unique); repeated runs are bitwise identical (b = 512 uses the
    640-row sketch and its own head kernel)."""
    from gpu_check import r_rows_by_column
    m, r = 2048, 512
    a = W.lowrank(m, m, r, 1e-12, 20250702)
    ref = O.bqrrp(a, b, 1.25, 42, 1e-10)
    runs = [run_gpu(Q, a, b, 1.25, 42, 1e-10) for _ in range(3)]
    for got in runs:
        assert got.rank == ref.rank == r
        assert np.array_equal(got.jpiv, runs[0].jpiv)
        assert np.array_equal(got.tau, runs[0].tau)
        assert np.array_equal(got.a, runs[0].a)
    got = runs[0]
    if ref.min_margin() >= MARGIN:
        assert np.array_equal(got.jpiv[:r], ref.jpiv[:r])
    assert sorted(got.jpiv[:r].tolist()) == sorted(ref.jpiv[:r].tolist())
    diff = r_rows_by_column(got.a, got.jpiv, r) - r_rows_by_column(ref.a, ref.jpiv, r)
    assert np.max(np.abs(diff)) <= R_TOL * np.linalg.norm(a)
    resid, orth = O.residual_and_orth(a, got)
    assert resid <= R_TOL and orth <= R_TOL


@pytest.mark.parametrize("m,n,b,gamma,tol", [(1500, 1200, 128, 1.25, 0.0), (700, 650, 64, 2.0, 0.0),
                                             (400, 171, 32, 1.25, 0.0), (2048, 2048, 256, 1.25, 0.0),
                                             (900, 900, 64, 1.25, 1e-9)])
def test_pivot_steps_limited_to_block(Q, m, n, b, gamma, tol):
    """pivot_steps = 1 stops the pivot selection after the block's k elimination
    steps instead of the full GETRF of the sketch: partial pivoting at step j
    depends only on the steps before j, and the columns left behind are
    selected among again by the next block, so the selected columns are those
    of the full GETRF and the factors agree to rounding (the trailing columns
    are processed in another order)."""
    sig = 1.0 / (np.arange(n) + 1.0) ** 2
    if tol > 0:
        sig[n // 2:] = 0.0
    a = W.usv(m, n, sig, seed=m + 3 * n)
    full = run_gpu(Q, a, b, gamma, 5, tol)
    part = run_gpu(Q, a, b, gamma, 5, tol, pivot_steps=1)
    assert part.rank == full.rank
    r = full.rank
    assert np.array_equal(part.jpiv[:r], full.jpiv[:r])
    if r == min(m, n):
        assert np.array_equal(part.jpiv, full.jpiv)
        nrm = np.linalg.norm(a)
        assert np.max(np.abs(np.triu(part.a) - np.triu(full.a))) <= R_TOL * nrm
        np.testing.assert_allclose(part.tau, full.tau, rtol=1e-9, atol=1e-12)
    resid, orth = O.residual_and_orth(a, part)
    assert resid <= R_TOL and orth <= R_TOL


# ---- the headline block parameters: b = 256, d = 320 -------------------------
def test_headline_block_square(Q):
    """2048^2, sigma_i = (i+1)^-2, b = 256, d = 320 against the whole oracle:
    the 20-wide register sketch-QR head, the 256-order blocked Cholesky and
    sign-modified LU, the split-K W = Y^T C and the lookahead all run."""
    m = n = 2048
    a = W.usv(m, n, W.spectrum("power", n, p=2.0), seed=1)
    ref = O.bqrrp(a, 256, 1.25, 42, 0.0)
    assert ref.min_margin() >= MARGIN
    got = run_gpu(Q, a, 256, 1.25, 42, 0.0)
    compare(a, got, ref, tau_rtol=1e-9)


def test_headline_block_first_block_wide_sketch(Q):
    """8192 x 4608 (n_i > 4096: the pivot selection with two rows per lane over
    36 workgroups), b = 256, d = 320: the first block against the oracle's
    first block (identical 256 pivots, R(0:256, :) column by column to
    1e-12 ||A||_F), and the whole factorization's residual and orthogonality."""
    from gpu_check import r_rows_by_column, residual_orth
    import workloads.device as WD
    m, n, b = 8192, 4608, 256
    A0 = WD.usv(m, n, WD.power_spectrum(n, 2.0), 17, "cuda")
    a = A0.cpu().numpy()
    ref = O.bqrrp(a, b, 1.25, 42, 0.0, max_blocks=1)
    assert ref.min_margin() >= MARGIN
    A = Q.colmajor(A0.clone())
    A, jpiv, tau, rank = Q.factor(A, b, 1.25, 42, 0.0)
    torch.cuda.synchronize()
    assert rank == n
    jp = jpiv.cpu().numpy()
    assert np.array_equal(jp[:b], ref.jpiv[:b])
    got = A[:b].cpu().numpy()
    diff = r_rows_by_column(got, jp, b) - r_rows_by_column(ref.a[:b], ref.jpiv, b)
    nrm = np.linalg.norm(a)
    assert np.max(np.abs(diff)) <= R_TOL * nrm
    res, orth = residual_orth(A0, A, jpiv, tau, rank)
    assert res <= R_TOL and orth <= R_TOL, (res, orth)

