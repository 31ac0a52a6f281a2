"""Parity of each step of the per-block loop: HIP kernels (through the C ABI)
against the CPU oracle on the same seeded inputs."""
import numpy as np
import pytest

from oracle import bqrrp as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def Q():
    from paper_2507_00976_amd import qrcp
    return qrcp


def dev(a):
    from paper_2507_00976_amd import qrcp
    return qrcp.colmajor(torch.from_numpy(np.asarray(a, dtype=np.float64)).cuda())


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ---- a1: Philox words and the Gaussian operator ----------------------------
def test_philox_words_bitwise(Q):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    out = Q.philox(torch.from_numpy(ctr.view(np.int32)).cuda(), 123456789, 987654321)
    got = host(out).view(np.uint32)
    ref = np.stack(O.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], (123456789, 987654321)), 1)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("m,d,seed", [(1024, 80, 42), (777, 33, 2 ** 40 + 5)])
def test_sketch_operator_matches_oracle(Q, m, d, seed):
    st = host(Q.sketch_operator(m, d, seed))          # m x d = S^T
    ref = O.sketch_operator(d, m, seed).T
    np.testing.assert_allclose(st, ref, rtol=1e-13, atol=1e-14)


# ---- a2: sketch GEMM --------------------------------------------------------
@pytest.mark.parametrize("m,n,d", [(1024, 512, 80), (700, 333, 40), (300, 300, 320)])
def test_sketch_gemm_f64(Q, m, n, d):
    a = W.gaussian(m, n, seed=m + n)
    got = host(Q.sketch(dev(a), d, 7, 0))
    ref = O.sketch(a, d, 7, "f64")
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)) * np.sqrt(m)


@pytest.mark.parametrize("m,n,d", [(1024, 512, 80), (3001, 700, 320), (777, 65, 33), (40000, 130, 160),
                                   (100, 3, 321)])
def test_sketch_gemm_bf16(Q, m, n, d):
    # d <= 320: the product holding all d rows per tile, with ragged K (m), ragged
    # column strips and several K splits; d = 321: the general BF16 product
    a = W.gaussian(m, n, seed=3 + m)
    got = host(Q.sketch(dev(a), d, 7, 1))
    ref = O.sketch(a, d, 7, "bf16")
    s = O.to_bf16(O.sketch_operator(d, m, 7)).astype(np.float64)
    bound = np.abs(s) @ np.abs(O.to_bf16(a).astype(np.float64))
    assert np.all(np.abs(got - ref) <= 1e-5 * bound)


# ---- a3: LU pivots -------------------------------------------------------------
@pytest.mark.parametrize("d,ni", [(80, 512), (80, 37), (320, 1000), (33, 5000), (64, 64), (97, 3000),
                                  (700, 4096), (320, 16384)])
def test_lu_pivots_match_oracle(Q, d, ni):
    msk = W.gaussian(d, ni, seed=d * ni)
    ipiv_ref, margins = O.getrf_pivots(msk.T)
    assert margins.min() > 1e-10
    ipiv, jsk = Q.lu_pivots(dev(msk))
    assert np.array_equal(host(ipiv), ipiv_ref)
    assert np.array_equal(host(jsk), O.piv_transform(ipiv_ref, ni))


def test_lu_zero_columns_and_ties(Q):
    msk = W.gaussian(16, 200, seed=1)
    msk[3, :] = 0.0                    # an all-zero LU column: pivot stays in place
    msk[:, 50] = msk[:, 7]             # equal |pivot| candidates
    ipiv_ref, _ = O.getrf_pivots(msk.T)
    ipiv, jsk = Q.lu_pivots(dev(msk))
    assert np.array_equal(host(ipiv), ipiv_ref)
    z = np.zeros((8, 100))
    ipiv, jsk = Q.lu_pivots(dev(z))
    assert np.array_equal(host(ipiv), np.arange(8))
    assert np.array_equal(host(jsk), np.arange(100))


def test_lu_nonfinite_reports_status(Q):
    msk = W.gaussian(16, 300, seed=2)
    msk[5, 250] = np.inf
    with pytest.raises(Q.QrcpError) as e:
        Q.lu_pivots(dev(msk))
    assert e.value.code == Q.QRCP_ERR_NONFINITE


# ---- a4: sketch QR ---------------------------------------------------------------
@pytest.mark.parametrize("d,ni", [(80, 512), (80, 40), (320, 2000), (100, 100), (640, 900)])
def test_sketch_qr_matches_oracle(Q, d, ni):
    b = W.gaussian(d, ni, seed=d + ni) @ np.diag(np.logspace(0, -3, ni))
    got = host(Q.sketch_qr(dev(b)))
    ref, _, _ = O.householder_qr(b)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.linalg.norm(b)
    assert np.all(np.tril(got, -1) == 0.0)


@pytest.mark.parametrize("d,ni", [(640, 3000), (960, 1200), (400, 2000)])
def test_sketch_qr_repeatable_wide_sketch(Q, d, ni):
    # sketches of more than 320 rows use the panel kernel with 16- and 8-wide
    # panels; repeated runs must be bitwise identical and match the oracle
    b = W.gaussian(d, ni, seed=3 * d + ni)
    runs = [host(Q.sketch_qr(dev(b))) for _ in range(3)]
    for got in runs[1:]:
        assert np.array_equal(got, runs[0])
    ref, _, _ = O.householder_qr(b)
    assert np.max(np.abs(runs[0] - ref)) <= 1e-12 * np.linalg.norm(b)


def test_sketch_qr_zero_column(Q):
    # a zero column gives tau = 0 (H_j = I) inside the head and in the tail's T
    b = W.gaussian(40, 90, seed=9)
    b[:, 5] = 0.0
    got = host(Q.sketch_qr(dev(b)))
    ref, _, _ = O.householder_qr(b)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.linalg.norm(b)


# ---- a7-a8: preconditioned Cholesky QR -----------------------------------------
@pytest.mark.parametrize("mi,k,passes", [(3000, 64, 1), (3000, 64, 2), (4000, 256, 1), (4000, 256, 2),
                                         (1000, 200, 1)])
def test_cholqr_matches_oracle(Q, mi, k, passes):
    # the preconditioner is the R factor of a sketch of the panel (as in the
    # method), so M^pre is well conditioned and Q is determined to rounding;
    # k = 256 runs the blocked Cholesky over resident workgroups
    p = W.usv(mi, k, W.spectrum("geometric", k, lo=1e-6), seed=4)
    rs = np.linalg.qr(O.sketch_operator(int(1.25 * k), mi, 5) @ p, mode="r")
    mpre = O.solve_triangular(rs, p.T, trans="T", lower=False).T
    qr_, rc_, keff_ = O.cholqr(mpre, passes)
    P, rc, keff = Q.cholqr(dev(p), dev(rs), passes)
    assert keff == keff_ == k
    # Cholesky QR's Q moves by about eps kappa(M^pre)^2 per unit of rounding in
    # the Gram matrix, whose m_i-term sums differ in order between the two
    # sides: bound by m_i eps kappa^2 (kappa ~ 15-19 here)
    kap = np.linalg.cond(mpre)
    assert np.max(np.abs(host(P) - qr_)) < mi * np.finfo(float).eps * kap ** 2
    assert np.max(np.abs(host(rc) - rc_)) < 1e-10 * np.abs(rc_).max()


def test_cholqr_breakdown_truncates(Q):
    mi, k = 500, 16
    p = W.gaussian(mi, k, seed=6)
    p[:, 9] = 0.0                       # exactly singular Gram: breakdown at column 9
    rs = np.eye(k)
    _, _, keff_ = O.cholqr(p, 1)
    _, _, keff = Q.cholqr(dev(p), dev(rs), 1)
    assert keff == keff_ == 9


# ---- a9: Householder reconstruction ---------------------------------------------
@pytest.mark.parametrize("mi,k", [(3000, 64), (1000, 256), (100, 100), (257, 33)])
def test_reconstruct_matches_oracle(Q, mi, k):
    q, _ = np.linalg.qr(W.gaussian(mi, k, seed=mi + k))
    y_, tau_, d_, u_ = O.householder_reconstruct(q)
    out, tau, dsig = Q.reconstruct(dev(q))
    out = host(out)
    assert np.array_equal(host(dsig), d_)
    np.testing.assert_allclose(host(tau), tau_, rtol=1e-12)
    assert np.max(np.abs(np.tril(out, -1) - np.tril(y_, -1))) < 1e-11
    assert np.max(np.abs(np.triu(out[:k]) - u_)) < 1e-12


# ---- a10-a11: T and the trailing update -------------------------------------------
@pytest.mark.parametrize("mi,k,nc", [(2000, 64, 700), (1000, 256, 1500), (300, 17, 5)])
def test_apply_qt_matches_oracle(Q, mi, k, nc):
    q, _ = np.linalg.qr(W.gaussian(mi, k, seed=1))
    y, tau, _, _ = O.householder_reconstruct(q)
    c = W.gaussian(mi, nc, seed=2)
    ref = O.apply_qt(y, O.larft(y, tau), c)
    ystore = np.array(y)
    ystore[np.triu_indices(k)] = 7.0          # above-diagonal garbage must be ignored
    got = host(Q.apply_qt(dev(ystore), torch.from_numpy(tau).cuda(), dev(c), 0))
    assert np.max(np.abs(got - ref)) < 1e-12 * np.abs(c).max() * np.sqrt(k)


def test_apply_qt_fp32_variant(Q):
    mi, k, nc = 1000, 64, 300
    q, _ = np.linalg.qr(W.gaussian(mi, k, seed=3))
    y, tau, _, _ = O.householder_reconstruct(q)
    c = W.gaussian(mi, nc, seed=4)
    ref = O.apply_qt(y, O.larft(y, tau), c)
    got = host(Q.apply_qt(dev(y), torch.from_numpy(tau).cuda(), dev(c), 1))
    assert np.max(np.abs(got - ref)) < 1e-4 * np.abs(c).max()


# ---- a12: sketch update ---------------------------------------------------------------
def test_sketch_update_matches_formula(Q):
    d, b, nt = 80, 64, 300
    rsk = np.triu(W.gaussian(d, b + nt, seed=8))
    r11 = np.triu(W.gaussian(b, b, seed=9)) + 8 * np.eye(b)
    r12 = W.gaussian(b, nt, seed=10)
    x = O.solve_triangular(r11, rsk[:b, :b].T, trans="T", lower=False).T
    ref = np.array(rsk)
    ref[:b, b:] = rsk[:b, b:] - x @ r12
    got = host(Q.sketch_update(dev(rsk), b, dev(r11), dev(r12)))
    assert np.max(np.abs(got - ref)) < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("d,b,nt", [(80, 64, 300), (320, 256, 2000)])
def test_sketch_update_one_pass_form(Q, d, b, nt):
    """The form qrcp_factor uses after one Cholesky QR pass, Rc^{-1} diag(D) R12,
    against the paper's Rsk12 - Rsk11 R11^{-1} R12 with R11 = diag(D) Rc Rsk11
    (Alg. 3's R11 with the signs of the reconstruction)."""
    rng = np.random.default_rng(d + b)
    rsk = np.triu(W.gaussian(d, b + nt, seed=11))
    rsk[np.arange(b), np.arange(b)] = np.abs(rsk[np.arange(b), np.arange(b)]) + 4.0
    rc = np.triu(W.gaussian(b, b, seed=12)) * 0.05
    rc[np.arange(b), np.arange(b)] = 1.0 + 0.1 * np.abs(rc[np.arange(b), np.arange(b)])
    dsig = rng.choice([-1.0, 1.0], size=b)
    r12 = W.gaussian(b, nt, seed=13)
    r11 = dsig[:, None] * (rc @ rsk[:b, :b])
    x = O.solve_triangular(r11, rsk[:b, :b].T, trans="T", lower=False).T   # Rsk11 R11^{-1}
    ref = np.array(rsk)
    ref[:b, b:] = rsk[:b, b:] - x @ r12
    got = host(Q.sketch_update_chol(dev(rsk), b, dev(rc), torch.from_numpy(dsig).cuda(), dev(r12)))
    assert np.max(np.abs(got - ref)) < 1e-12 * np.abs(ref).max() * np.sqrt(b)
    assert np.array_equal(got[:, :b], rsk[:, :b])
