"""Writes the regression fixtures in this folder.  Calls only ``oracle`` and the
seeded input builders in ``workloads``; never the HIP library.

The paper prints no worked numerical example, so these fixtures are not paper
values: they freeze the oracle's output on small seeded inputs so that an
accidental change of its arithmetic shows up as a test failure.  Regenerate
(``python tests/golden/make_golden.py``) only with a commit message that names
the passage of the paper justifying the change.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bqrrp as O  # noqa: E402
import workloads as W  # noqa: E402


def philox_fixture():
    lines = ["# c0 c1 c2 c3 k0 k1 -> x0 x1 x2 x3 (Philox4x32-10)"]
    rng = np.random.default_rng(2025)
    for _ in range(16):
        c = [int(v) for v in rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)]
        x = O.philox4x32_10(np.uint32(c[0]), np.uint32(c[1]), np.uint32(c[2]), np.uint32(c[3]), (c[4], c[5]))
        lines.append(" ".join(map(str, c)) + " -> " + " ".join(str(int(v)) for v in x))
    return "\n".join(lines) + "\n"


def bqrrp_fixture():
    a = W.usv(96, 48, W.spectrum("geometric", 48, lo=1e-8), seed=77)
    res = O.bqrrp(a, 16, 1.25, 42, 0.0)
    out = [f"# usv(96, 48, geometric 1e-8, seed=77); b=16 gamma=1.25 sketch seed=42 tol=0",
           f"rank {res.rank}",
           f"min_margin {res.min_margin():.6e}",
           "jpiv " + " ".join(map(str, res.jpiv.tolist())),
           "absdiag " + " ".join(f"{v:.17e}" for v in np.abs(np.diag(res.a))),
           "tau " + " ".join(f"{v:.17e}" for v in res.tau)]
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    with open(os.path.join(HERE, "philox_words.txt"), "w") as f:
        f.write(philox_fixture())
    with open(os.path.join(HERE, "bqrrp_96x48.txt"), "w") as f:
        f.write(bqrrp_fixture())
    print("wrote fixtures")
