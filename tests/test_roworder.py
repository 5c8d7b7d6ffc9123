"""Host logic of the streaming check kernel's row order (csrc/roworder.hip),
checked on the CPU: a small C++ driver compiled with the source builds the
order for a graph and reports, under a model of one XCD's L2 as an LRU cache
of the last 8,192 bits (256-byte tiles of posteriors) touched, how often a
row finds its bits cached in index order and in the built order."""
import os
import subprocess

import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_10424_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("roworder") / "roworder_check")
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(ROOT, "tests", "native", "roworder_check.cpp"), os.path.join(CSRC, "roworder.hip"),
           "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        pytest.fail(res.stderr[-2000:])
    return out


def run(checker, m, n, rows, cols, cap=8192):
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.searchsorted(rows, np.arange(m + 1))
    lines = [f"{m} {n}"] + [" ".join([str(rp[i + 1] - rp[i])] + [str(x) for x in cols[rp[i]:rp[i + 1]]])
                            for i in range(m)]
    res = subprocess.run([checker, str(cap)], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0 and res.stdout.startswith("ok"), res.stdout + res.stderr
    return [float(x) for x in res.stdout.split()[1:3]]



def test_n64800_order_raises_modelled_hits(checker):
    m, n, rows, cols = wl.large_qc_code(seed=5, dense=False)
    nat, built = run(checker, m, n, np.asarray(rows), np.asarray(cols))
    # index order about 0.12, the built order about 0.38 (of the 0.71 that
    # repeated bits allow)
    assert nat < 0.2 and built > 0.3


def test_order_on_small_and_irregular_graphs(checker):
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    r, c = np.nonzero(H)
    run(checker, 512, 1024, r, c, cap=256)
    H = wl.random_irregular_code(300, 150, seed=3)
    r, c = np.nonzero(H)
    run(checker, H.shape[0], H.shape[1], r, c, cap=64)
