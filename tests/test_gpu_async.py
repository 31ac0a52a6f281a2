"""qrcp_factor_async (C ABI): the whole factorization enqueued without
read-backs, rank and status in device memory.  Against qrcp_factor on the
same inputs: pivots, rank and status identical, A and tau bitwise equal
(qrcp_factor is the same enqueued work followed by one read-back), over full
rank, exit blocks of reduced rank, the zero matrix, a non-finite input, wide
and truncated shapes and the panel and pivot options."""
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


def _pair(Q, a, b, gamma=1.25, seed=42, tol=0.0, **kw):
    A0 = Q.colmajor(torch.from_numpy(np.asarray(a, dtype=np.float64)).cuda())
    A1 = Q.colmajor(A0.clone())
    A2 = Q.colmajor(A0.clone())
    print(f"async vs blocking {a.shape} b={b} tol={tol} {kw}", flush=True)
    _, j1, t1, r1 = Q.factor(A1, b, gamma, seed, tol, **kw)
    _, j2, t2, rdev, sdev = Q.factor_async(A2, b, gamma, seed, tol, **kw)
    torch.cuda.synchronize()
    return (A1, j1, t1, r1), (A2, j2, t2, int(rdev.item()), int(sdev.item()))


def _same(x, y):
    A1, j1, t1, r1 = x
    A2, j2, t2, r2, s2 = y
    assert s2 == 0
    assert r1 == r2
    assert torch.equal(j1, j2)
    assert torch.equal(A1, A2)
    assert torch.equal(t1, t2)


@pytest.mark.parametrize("case", ["full", "ragged", "exact_rank", "gap_exit", "wide", "trunc",
                                  "hqr", "hqr_rank", "geqp3", "cholqr2", "cholqr2_rank", "single",
                                  "one_row", "one_col", "b1", "bf16_sketch"])
def test_async_matches_blocking(Q, case):
    kw, tol, b = {}, 0.0, 32
    if case == "full":
        a, b = W.usv(1024, 512, W.spectrum("geometric", 512, lo=1e-10), seed=1), 64
    elif case == "ragged":
        a = W.usv(400, 171, W.spectrum("power", 171, p=1.0), seed=2)
    elif case == "exact_rank":
        a, tol = W.lowrank(400, 200, 70, 0.0, seed=3), 1e-12
    elif case == "gap_exit":
        sig = 1.0 / (np.arange(160) + 1.0)
        sig[70:] *= 1e-4
        a, tol = W.usv(300, 160, sig, 6), 1e-3
    elif case == "wide":
        a = W.gaussian(96, 200, seed=4)
    elif case == "trunc":
        a, kw = W.usv(300, 160, W.spectrum("geometric", 160, lo=1e-8), seed=5), {"max_rank": 50}
    elif case == "hqr":
        a, kw = W.usv(500, 300, W.spectrum("geometric", 300, lo=1e-9), seed=6), {"qr_tall": 1}
    elif case == "hqr_rank":
        a, tol, kw = W.lowrank(400, 200, 70, 0.0, seed=7), 1e-12, {"qr_tall": 1}
    elif case == "geqp3":
        a, kw = W.usv(300, 171, W.spectrum("geometric", 171, lo=1e-8), seed=8), {"qrcp_wide": 1}
    elif case == "cholqr2":
        a, kw = W.usv(600, 300, W.spectrum("geometric", 300, lo=1e-12), seed=9), {"cholqr_passes": 2}
    elif case == "cholqr2_rank":
        a, tol, kw = W.lowrank(400, 200, 50, 0.0, seed=10), 1e-12, {"cholqr_passes": 2}
    elif case == "single":
        a, b = W.usv(256, 100, W.spectrum("geometric", 100, lo=1e-6), seed=11), 128
    elif case == "one_row":
        a, b = W.gaussian(1, 5, seed=12), 2
    elif case == "one_col":
        a, b = W.gaussian(5, 1, seed=13), 1
    elif case == "b1":
        a, b = W.gaussian(64, 40, seed=14), 1
    elif case == "bf16_sketch":
        a, kw = (W.usv(700, 400, W.spectrum("geometric", 400, lo=1e-9), seed=15),
                 {"sketch_precision": 1, "cholqr_passes": 2})
    x, y = _pair(Q, a, b, 1.25, 42, tol, **kw)
    _same(x, y)


def test_async_rank_status_on_device(Q):
    """The rank of an exact-rank input and the status of a non-finite input
    arrive in the device words; the zero matrix gives rank 0."""
    a = W.lowrank(300, 120, 40, 0.0, seed=12)
    A = Q.colmajor(torch.from_numpy(a).cuda())
    _, jpiv, tau, rdev, sdev = Q.factor_async(A, 16, 1.25, 3, 1e-12)
    torch.cuda.synchronize()
    assert int(rdev.item()) == 40 and int(sdev.item()) == 0
    ref = O.bqrrp(a, 16, 1.25, 3, 1e-12)
    assert ref.rank == 40
    assert np.array_equal(jpiv.cpu().numpy()[:40], ref.jpiv[:40])
    z = Q.colmajor(torch.zeros(64, 24, dtype=torch.float64, device="cuda"))
    _, jz, tz, rz, sz = Q.factor_async(z, 8)
    torch.cuda.synchronize()
    assert int(rz.item()) == 0 and int(sz.item()) == 0 and not tz.any() and not z.any()
    assert torch.equal(jz.cpu(), torch.arange(24))
    g = W.gaussian(64, 24, seed=1)
    g[3, 4] = np.nan
    B = Q.colmajor(torch.from_numpy(g).cuda())
    _, _, _, rb, sb = Q.factor_async(B, 8)
    torch.cuda.synchronize()
    assert int(sb.item()) == Q.QRCP_ERR_NONFINITE
    e = Q.colmajor(torch.zeros(0, 5, dtype=torch.float64, device="cuda"))
    _, je, te, re_, se = Q.factor_async(e, 4)
    torch.cuda.synchronize()
    assert int(re_.item()) == 0 and int(se.item()) == 0 and torch.equal(je.cpu(), torch.arange(5))


def test_async_returns_before_the_work(Q):
    """The call only enqueues: several factorizations are issued back to back
    on one stream with no synchronization between them, then checked."""
    mats = [W.usv(512, 256, W.spectrum("geometric", 256, lo=1e-8), seed=20 + i) for i in range(3)]
    outs = []
    for a in mats:
        A = Q.colmajor(torch.from_numpy(a).cuda())
        outs.append(Q.factor_async(A, 64, 1.25, 5, 0.0))
    torch.cuda.synchronize()
    for a, (A, jpiv, tau, rdev, sdev) in zip(mats, outs):
        assert int(sdev.item()) == 0 and int(rdev.item()) == 256
        ref = O.bqrrp(a, 64, 1.25, 5, 0.0)
        assert np.array_equal(jpiv.cpu().numpy(), ref.jpiv)
        assert np.max(np.abs(np.triu(A.cpu().numpy()) - np.triu(ref.a))) <= 1e-12 * np.linalg.norm(a)
