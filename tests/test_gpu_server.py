"""Request server (qrcp_server_*): requests of mixed shapes in flight together
give bitwise the same results as the same requests factored one at a time."""
import numpy as np
import pytest
import torch

from workloads import spectrum, usv

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(20250706)
    reqs = []
    for i in range(12):
        m = int(np.exp(rng.uniform(np.log(256), np.log(2048))))
        n = int(np.exp(rng.uniform(np.log(64), np.log(min(m, 512)))))
        kind = ["geometric", "harmonic", "exact"][i % 3]
        if kind == "geometric":
            sig = spectrum("geometric", n, lo=1e-10)
        elif kind == "harmonic":
            sig = 1.0 / (np.arange(n) + 1.0)
        else:
            sig = 1.0 / (np.arange(n) + 1.0)
            sig[n // 2:] = 0.0
        a = usv(m, n, sig, 7000 + i)
        b = min(64, n)
        tol = 1e-13 if kind == "exact" else 0.0
        reqs.append((a, b, tol))
    return reqs


def test_server_matches_alone():
    from paper_2507_00976_amd import qrcp
    reqs = _requests()
    alone = []
    for a, b, tol in reqs:
        A = qrcp.colmajor(torch.from_numpy(a).cuda())
        out = qrcp.factor(A, b, 1.25, 42, tol)
        torch.cuda.synchronize()
        alone.append(out)
    with qrcp.Server(slots=4) as srv:
        tickets = []
        for a, b, tol in reqs:
            A = qrcp.colmajor(torch.from_numpy(a).cuda())
            tickets.append(srv.submit(A, b, 1.25, 42, tol))
        mixed = [srv.wait(t) for t in tickets]
        assert srv.pending() == 0
    for (A1, j1, t1, r1), (A2, j2, t2, r2, timing) in zip(alone, mixed):
        assert r1 == r2
        assert torch.equal(j1, j2)
        assert torch.equal(t1, t2)
        assert torch.equal(A1, A2)
        assert timing["submit_ms"] <= timing["start_ms"] <= timing["end_ms"]
    # exact-rank requests report rank n/2
    for (a, b, tol), (_, _, _, r, _) in zip(reqs, mixed):
        if tol > 0:
            assert r == a.shape[1] // 2


def test_server_small_budget_serializes():
    """A budget that holds one workspace at a time still completes every request."""
    from paper_2507_00976_amd import qrcp
    reqs = _requests()[:4]
    need = max(qrcp.workspace_size(a.shape[0], a.shape[1], b) for a, b, _ in reqs)
    with qrcp.Server(slots=3, hbm_budget=need + need // 2) as srv:
        tickets = [srv.submit(qrcp.colmajor(torch.from_numpy(a).cuda()), b, 1.25, 42, tol)
                   for a, b, tol in reqs]
        for t in tickets:
            assert srv.wait(t)[3] > 0


def test_server_rejects_unsupported():
    from paper_2507_00976_amd import qrcp
    with qrcp.Server(slots=1) as srv:
        # a sketch of more than 1024 rows can never be admitted
        A = qrcp.colmajor(torch.zeros(2048, 1000, dtype=torch.float64, device="cuda"))
        with pytest.raises(qrcp.QrcpError) as e:
            srv.submit(A, 900, 1.25)
        assert e.value.code == qrcp.QRCP_ERR_UNSUPPORTED


def test_server_wide_request_matches_alone():
    """Wide requests (m < n) are admitted and give what a lone call gives."""
    import numpy as np
    import workloads as W
    from paper_2507_00976_amd import qrcp
    a = W.gaussian(96, 200, seed=41)
    A1 = qrcp.colmajor(torch.from_numpy(a).cuda())
    A1, j1, t1, r1 = qrcp.factor(A1, 32, 1.25, 3, 0.0)
    with qrcp.Server(slots=2) as srv:
        A2 = qrcp.colmajor(torch.from_numpy(a).cuda())
        t = srv.submit(A2, 32, 1.25, 3, 0.0)
        A2, j2, t2, r2, _ = srv.wait(t)
    torch.cuda.synchronize()
    assert r1 == r2 == 96
    assert torch.equal(j1, j2) and torch.equal(A1, A2) and torch.equal(t1, t2)
