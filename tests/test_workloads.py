"""Seeded input generators (no GPU)."""
import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl


def test_regular_code_is_regular_and_simple():
    for n, m, seed in [(96, 48, 1), (1024, 512, 2)]:
        H = wl.regular_ldpc(n, m, 3, 6, seed=seed)
        assert H.shape == (m, n) and H.max() == 1
        assert np.all(H.sum(0) == 3) and np.all(H.sum(1) == 6)  # 0/1 entries: no double edges
        assert np.array_equal(H, wl.regular_ldpc(n, m, 3, 6, seed=seed))


def test_encoder_codewords_satisfy_checks(orc):
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    enc = wl.gf2_encoder(H)
    assert enc.k == 96 - enc.rank
    c = enc.random_codewords(200, seed=9)
    assert not orc.syndrome(H, c).any()
    assert c.any(axis=1).sum() > 190  # not all-zero


def test_tree_codes_are_trees():
    for seed in range(40):
        H = wl.tree_code(1 + seed % 6, seed=seed, max_check_degree=2 + seed % 4)
        m, n = H.shape
        assert np.all(H.sum(1) >= 2)
        assert int(H.sum()) == n + m - 1  # a connected bipartite graph with E = V - 1 is a tree
        assert n <= 16


def test_large_qc_code_profile():
    m, n, rows, cols = wl.large_qc_code(seed=5, dense=False)
    assert (m, n) == (32400, 64800) and rows.size == 226800
    rdeg = np.bincount(rows, minlength=m)
    cdeg = np.bincount(cols, minlength=n)
    assert np.all(rdeg == 7)
    assert np.bincount(cdeg).tolist()[2:] == [32400, 19440, 0, 0, 0, 0, 12960]
    assert np.unique(rows.astype(np.int64) * n + cols).size == rows.size


def test_multi_code_family():
    fam = wl.qc_multi_code_family(seed=7)
    assert len(fam) == 8
    for c in fam:
        H = c["H"]
        assert H.shape == (c["m"], c["n"]) and H.max() == 1
        assert c["n"] in (576, 1152, 1728, 2304)
        assert set(np.unique(H.sum(0))) <= {2, 3, 4, 6}
        assert H.sum(1).min() >= 2


def test_awgn_llr_statistics():
    r = wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=100, n=96, batch=1000)
    s = wl.sigma_for_ebn0(2.0, 0.5)
    assert r.dtype == np.float32 and r.shape == (1000, 96)
    # LLR = 2y/s^2 with y ~ N(1, s^2): mean 2/s^2, std 2/s
    assert abs(r.mean() - 2 / s**2) < 0.05 * 2 / s**2
    assert abs(r.std() - 2 / s) < 0.05 * 2 / s
    assert np.array_equal(r, wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=100, n=96, batch=1000))
