"""Pins of the oracle's sketching operator (Philox4x32-10 + Box-Muller).

The paper only asks for i.i.d. mean-zero Gaussian entries drawn once (Alg. 1
sampling step, Sec. 2 remark, Sec. 3 footnote on the variance).  The pins:
* Philox words equal rocRAND's Philox4x32-10 block function (a library routine);
* the Gaussians have N(0,1) moments and pass a Kolmogorov-Smirnov test;
* rows are uncorrelated; S for a smaller d is the prefix of S for a larger d.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import bqrrp as O

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_rr")
    src = os.path.join(HERE, "helpers", "philox_rocrand.cpp")
    r = subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", "-o", exe, src],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build rocRAND reference: " + r.stderr[-400:])

    def run(rows):
        inp = "\n".join(" ".join(str(int(v)) for v in row) for row in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)
    return run


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(1)
    rows = rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64)
    rows[0] = 0
    rows[1] = 2 ** 32 - 1
    ref = rocrand_philox(rows)
    for i, (c0, c1, c2, c3, k0, k1) in enumerate(rows):
        got = O.philox4x32_10(np.uint32(c0), np.uint32(c1), np.uint32(c2), np.uint32(c3),
                              (int(k0), int(k1)))
        assert [int(g) for g in got] == [int(v) for v in ref[i]], i


def test_philox_vectorised_equals_scalar():
    rows = np.arange(50, dtype=np.uint32)
    vec = O.philox4x32_10(rows, np.uint32(7), np.uint32(0), np.uint32(0), O.seed_key(99))
    for j in (0, 13, 49):
        sc = O.philox4x32_10(np.uint32(j), np.uint32(7), np.uint32(0), np.uint32(0), O.seed_key(99))
        assert [int(v[j]) for v in vec] == [int(s) for s in sc]


def test_gaussian_moments_and_ks():
    s = O.sketch_operator(64, 20000, seed=42)
    x = s.ravel()
    n = x.size
    assert abs(x.mean()) < 5 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(stats.skew(x)) < 5 * np.sqrt(6.0 / n)
    assert abs(stats.kurtosis(x)) < 5 * np.sqrt(24.0 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # both halves of the Box-Muller pair are N(0,1) on their own
    assert stats.kstest(s[0::2].ravel(), "norm").pvalue > 1e-4
    assert stats.kstest(s[1::2].ravel(), "norm").pvalue > 1e-4


def test_rows_uncorrelated():
    s = O.sketch_operator(40, 50000, seed=7)
    c = np.corrcoef(s)
    off = c[~np.eye(40, dtype=bool)]
    assert np.max(np.abs(off)) < 6 / np.sqrt(50000)


def test_seed_changes_stream_and_prefix_property():
    a = O.sketch_operator(100, 333, seed=5)
    b = O.sketch_operator(80, 333, seed=5)
    c = O.sketch_operator(81, 333, seed=5)
    assert np.array_equal(a[:80], b)
    assert np.array_equal(a[:81], c)
    d = O.sketch_operator(80, 333, seed=6)
    assert not np.any(d == b)


def test_uniform_words():
    rows = np.arange(200000, dtype=np.uint32)
    words = np.concatenate(O.philox4x32_10(rows, np.uint32(0), np.uint32(0), np.uint32(0), (1, 2)))
    top = (words >> np.uint32(24)).astype(np.int64)
    hist = np.bincount(top, minlength=256)
    chi2 = ((hist - hist.mean()) ** 2 / hist.mean()).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(3).standard_normal(10000) * 1e3
    x[:4] = [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9]
    ours = O.to_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))
