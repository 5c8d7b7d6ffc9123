"""Host logic of the on-chip decoder's bank-conflict-free LDS layout
(csrc/layout.hip), checked on the CPU: a small C++ driver compiled with the
layout source checks, per graph, that the tables hold every row and bit
once, give every message its own position, list each bit's messages in
ascending check order (the column sum order of eq. lambda_j), and that no
message read or write of a wavefront conflicts on the LDS banks."""
import os
import subprocess

import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_10424_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("layout") / "layout_check")
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(ROOT, "tests", "native", "layout_check.cpp"), os.path.join(CSRC, "layout.hip"),
           "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        pytest.fail(res.stderr[-2000:])
    return out


def run(checker, H, geometry=()):
    m, n = H.shape
    lines = [f"{m} {n}"]
    for i in range(m):
        c = np.nonzero(H[i])[0]
        lines.append(" ".join([str(len(c))] + [str(x) for x in c]))
    res = subprocess.run([checker] + [str(x) for x in geometry], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.startswith("ok"), res.stdout + res.stderr
    return float(res.stdout.split()[1])


@pytest.mark.parametrize("n,m,seed", [(96, 48, 1), (1024, 512, 2), (200, 100, 7), (2048, 1024, 3)])
def test_layout_36_regular(checker, n, m, seed):
    load = run(checker, wl.regular_ldpc(n, m, 3, 6, seed=seed))
    # posterior gathers: near one bank access per half-wave (random: about 3.5)
    assert load <= 1.5


def test_layout_other_degrees(checker):
    run(checker, wl.regular_ldpc(240, 60, 2, 8, seed=4))
    run(checker, wl.regular_ldpc(300, 200, 4, 6, seed=5))


def test_layout_paper_example(checker):
    run(checker, wl.paper_tanner_example())


# (rows per thread, bits per thread, bit-side stride) of the layout variants
# for the eight QC codes (one row degree, columns of degree 2, 3 and 6 or 4)
QC_GEOMETRY = {6: [(2, 4, 6), (1, 2, 6)], 9: [(2, 6, 6)], 12: [(1, 4, 6)], 16: [(1, 6, 4)]}


@pytest.mark.parametrize("k", range(8))
def test_layout_qc_family_padded_columns(checker, k):
    c = wl.qc_multi_code_family(seed=7)[k]
    H = c["H"]
    dc = int(H.sum(axis=1).max())
    assert int(H.sum(axis=1).min()) == dc
    done = 0
    for rpt, cpt, dvs in QC_GEOMETRY[dc]:
        m, n = H.shape
        nt = max(-(-m // rpt), -(-n // cpt))
        if -(-nt // 64) * 64 > 512:
            continue
        load = run(checker, H, (rpt, cpt, dvs))
        assert load <= 1.25
        done += 1
    assert done >= 1


# the same with bits in ascending degree and the profile of messages read per
# bit slot index (hex, 4 bits per index)
QC_PROFILE = {6: [(2, 4, 6, "6332"), (1, 2, 6, "63")], 9: [(2, 6, 6, "633222")], 12: [(1, 4, 6, "6332")],
              16: [(1, 6, 4, "433222")]}


@pytest.mark.parametrize("k", [0, 2, 4, 5, 6, 7])
def test_layout_qc_family_degree_profile(checker, k):
    c = wl.qc_multi_code_family(seed=7)[k]
    H = c["H"]
    m, n = H.shape
    dc = int(H.sum(axis=1).max())
    done = 0
    for rpt, cpt, dvs, prof in QC_PROFILE[dc]:
        nt = -(-max(-(-m // rpt), -(-n // cpt)) // 64) * 64
        caps = [int(x, 16) for x in reversed(prof)]
        deg = np.sort(H.sum(axis=0))
        if nt > 512 or any(caps[p // nt] < deg[p] for p in range(n)):
            continue
        # posterior gathers as even as without the profile (a histogram that
        # started from the unsorted placement once left them near 2)
        assert run(checker, H, (rpt, cpt, dvs, prof)) <= 1.25
        done += 1
    assert done >= 1


def test_layout_profile_that_does_not_hold(checker):
    # a profile of two messages for every slot cannot hold degree-3 bits
    H = wl.regular_ldpc(512, 256, 3, 6, seed=9)
    m, n = H.shape
    lines = [f"{m} {n}"] + [" ".join([str(int(r.sum()))] + [str(x) for x in np.nonzero(r)[0]]) for r in H]
    res = subprocess.run([checker, "2", "4", "3", "2222"], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, timeout=60)
    assert res.stdout.startswith("FAIL no layout")


def test_layout_stride_above_degree(checker):
    # a (3,6) code laid out with room for six messages per bit: three zero entries each
    run(checker, wl.regular_ldpc(512, 256, 3, 6, seed=9), (2, 4, 6))
    run(checker, wl.regular_ldpc(512, 256, 3, 6, seed=9), (1, 2, 3))
