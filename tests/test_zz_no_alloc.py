"""qrcp_factor_noalloc (the library's fixed device workspace, no caller
buffer) against qrcp_factor on the same inputs, through the C ABI: identical
pivots and rank, and A and tau bitwise equal (the same kernels in the same
order).  Two calls in a row, the second on a smaller input, so the second
runs over what the first left in the shared array."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def Q():
    from paper_2507_00976_amd import qrcp
    return qrcp


def _both(Q, a, b, gamma, seed, tol, **kw):
    m, n = a.shape
    A0 = Q.colmajor(torch.from_numpy(a).cuda())
    A1 = A0.clone()
    A2 = Q.colmajor(A0.clone())
    _, jp1, tau1, r1 = Q.factor(A1, b, gamma, seed, tol, **kw)
    jp2 = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    tau2 = torch.full((min(m, n),), np.nan, dtype=torch.float64, device="cuda")
    _, jp2, tau2, r2 = Q.factor_noalloc(A2, b, gamma, seed, tol, jpiv=jp2, tau=tau2, **kw)
    torch.cuda.synchronize()
    return (A1.cpu().numpy(), jp1.cpu().numpy(), tau1.cpu().numpy(), r1,
            A2.cpu().numpy(), jp2.cpu().numpy(), tau2.cpu().numpy(), r2)


def _check_equal(res):
    a1, j1, t1, r1, a2, j2, t2, r2 = res
    assert r1 == r2
    assert np.array_equal(j1, j2)
    assert np.array_equal(a1, a2)
    assert np.array_equal(t1, t2)


def test_noalloc_matches_factor_twice():
    from paper_2507_00976_amd import qrcp as Q
    # first call: 1024 x 512, b = 64 (several blocks, full rank)
    a = W.usv(1024, 512, W.spectrum("geometric", 512, lo=1e-10), seed=11)
    print("noalloc call 1: 1024x512 b=64", flush=True)
    r = _both(Q, a, 64, 1.25, 42, 0.0)
    _check_equal(r)
    assert r[3] == 512
    # second call, smaller, rank deficient with a ragged last block
    a = W.lowrank(300, 170, 90, 0.0, seed=12)
    print("noalloc call 2: 300x170 rank 90 b=32", flush=True)
    r = _both(Q, a, 32, 1.25, 7, 1e-13)
    _check_equal(r)
    assert r[3] == 90


def test_noalloc_rejects_oversize():
    from paper_2507_00976_amd import qrcp as Q
    need = Q.workspace_size(4096, 4096, 256, 1.25)
    assert need > Q.noalloc_max_bytes()
    A = Q.colmajor(torch.zeros(4096, 4096, dtype=torch.float64, device="cuda"))
    jp = torch.empty(4096, dtype=torch.int64, device="cuda")
    tau = torch.empty(4096, dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QrcpError) as e:
        Q.factor_noalloc(A, 256, 1.25, 1, 0.0, jpiv=jp, tau=tau)
    assert e.value.code == Q.QRCP_ERR_WORKSPACE
