"""The Cholesky and sign-modified LU factorizations spread over resident
workgroups (orders up to 256) give bitwise the factors of the single-workgroup
kernels they replace: same products in the same order.  Covers ragged orders,
a Cholesky breakdown, CholQR2 and whole factorizations."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def Q():
    from paper_2507_00976_amd import qrcp
    return qrcp


def dev(Q, a):
    return Q.colmajor(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda())


def host(t):
    return t.cpu().numpy()


def single_and_multi(monkeypatch, fn):
    monkeypatch.setenv("QRCP_SMALLFACT", "single")
    a = fn()
    torch.cuda.synchronize()
    monkeypatch.delenv("QRCP_SMALLFACT")
    b = fn()
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("mi,k,passes", [(3000, 256, 1), (1000, 200, 1), (500, 33, 2), (300, 32, 1),
                                         (200, 7, 1), (2000, 256, 2)])
def test_cholqr_bitwise(Q, monkeypatch, mi, k, passes):
    p = W.usv(mi, k, W.spectrum("geometric", k, lo=1e-5), seed=mi + k)
    rs = np.eye(k)
    (p1, r1, k1), (p2, r2, k2) = single_and_multi(
        monkeypatch, lambda: Q.cholqr(dev(Q, p), dev(Q, rs), passes))
    assert k1 == k2 == k
    assert np.array_equal(host(r1), host(r2))
    assert np.array_equal(host(p1), host(p2))


@pytest.mark.parametrize("col", [0, 31, 70, 255])
def test_cholqr_breakdown_bitwise(Q, monkeypatch, col):
    mi, k = 800, 256
    p = W.gaussian(mi, k, seed=col + 1)
    p[:, col] = 0.0                      # singular Gram: breakdown at `col`
    rs = np.eye(k)
    (_, r1, k1), (_, r2, k2) = single_and_multi(
        monkeypatch, lambda: Q.cholqr(dev(Q, p), dev(Q, rs), 1))
    assert k1 == k2 == col
    assert np.array_equal(host(r1)[:col, :col], host(r2)[:col, :col])


@pytest.mark.parametrize("mi,k", [(3000, 256), (1000, 256), (257, 33), (100, 100), (64, 64), (40, 5)])
def test_reconstruct_bitwise(Q, monkeypatch, mi, k):
    q, _ = np.linalg.qr(W.gaussian(mi, k, seed=3 * mi + k))
    (o1, t1, d1), (o2, t2, d2) = single_and_multi(monkeypatch, lambda: Q.reconstruct(dev(Q, q)))
    assert np.array_equal(host(d1), host(d2))
    assert np.array_equal(host(t1), host(t2))
    assert np.array_equal(host(o1), host(o2))


@pytest.mark.parametrize("m,n,b,tol", [(2048, 1536, 256, 0.0), (1500, 1000, 128, 1e-12)])
def test_factor_bitwise(Q, monkeypatch, m, n, b, tol):
    sig = 1.0 / (np.arange(n) + 1.0) ** 2
    if tol > 0:
        sig[n // 2:] = 0.0
    a = W.usv(m, n, sig, seed=m + n)

    def run():
        A = dev(Q, a)
        out = Q.factor(A, b, 1.25, 42, tol)
        return tuple(host(x) if hasattr(x, "cpu") else x for x in out)

    r1, r2 = single_and_multi(monkeypatch, run)
    assert r1[3] == r2[3]
    for x, y in zip(r1[:3], r2[:3]):
        assert np.array_equal(x, y)
