"""Regression fixtures of the oracle (written by tests/golden/make_golden.py,
which calls only the oracle): they catch accidental changes of its arithmetic."""
import os

import numpy as np

import workloads as W
from oracle import bqrrp as O

G = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_philox_fixture():
    for line in open(os.path.join(G, "philox_words.txt")):
        if line.startswith("#"):
            continue
        lhs, rhs = line.split("->")
        c = [int(t) for t in lhs.split()]
        want = [int(t) for t in rhs.split()]
        got = O.philox4x32_10(np.uint32(c[0]), np.uint32(c[1]), np.uint32(c[2]), np.uint32(c[3]), (c[4], c[5]))
        assert [int(v) for v in got] == want


def test_bqrrp_fixture():
    rows = {}
    for line in open(os.path.join(G, "bqrrp_96x48.txt")):
        if line.startswith("#"):
            continue
        key, *vals = line.split()
        rows[key] = vals
    a = W.usv(96, 48, W.spectrum("geometric", 48, lo=1e-8), seed=77)
    res = O.bqrrp(a, 16, 1.25, 42, 0.0)
    assert res.rank == int(rows["rank"][0])
    assert res.jpiv.tolist() == [int(v) for v in rows["jpiv"]]
    np.testing.assert_allclose(np.abs(np.diag(res.a)), [float(v) for v in rows["absdiag"]], rtol=1e-9)
    np.testing.assert_allclose(res.tau, [float(v) for v in rows["tau"]], rtol=1e-9)
