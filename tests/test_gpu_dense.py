"""The dense map-reduce decoder (Algorithm 2) through the C-ABI against the
CPU oracle: same decisions, iterations and flags, posteriors within the
parity tolerance (a zero posterior may differ in sign)."""
import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl
from parity import assert_parity, note, oracle_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def dense(tdev, H, llr, L, flags=0):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    g = ldpc.build_graph(torch.from_numpy(np.ascontiguousarray(H)).to(dev))
    out = ldpc.minsum_decode_dense(g, torch.from_numpy(np.ascontiguousarray(llr, dtype=np.float32)).to(dev), L,
                                   flags=flags)
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in out)


@pytest.mark.parametrize("L,flags", [(20, 0), (0, 0), (3, 1), (23, 6 << 8)])
def test_dense_small_regular(tdev, L, flags):
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    llr = wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=100, n=96, batch=300)
    note(f"[dense] C0 L={L} flags={flags}")
    assert_parity(dense(tdev, H, llr, L, flags), oracle_decode(H, llr, L, flags), f"dense C0 L={L}")


@pytest.mark.parametrize("seed", range(3))
def test_dense_irregular(tdev, seed):
    H = wl.random_irregular_code(150, 60, seed=seed, dv_choices=(0, 1, 2, 3, 5))
    llr = np.random.default_rng(seed).normal(1.0, 1.5, size=(130, 150)).astype(np.float32)
    note(f"[dense] irregular seed {seed}")
    assert_parity(dense(tdev, H, llr, 25), oracle_decode(H, llr, 25), f"dense irregular {seed}")


def test_dense_equals_oracle_dense_form(tdev):
    """Frame by frame against the oracle's literal Algorithm 2 as well."""
    import oracle
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    llr = wl.bpsk_awgn_llr(None, 1.5, 0.5, seed=9, n=96, batch=24)
    got = dense(tdev, H, llr, 15)
    for f in range(llr.shape[0]):
        b, p, it, ok = oracle.minsum_dense(H, llr[f], 15)
        assert np.array_equal(got[0][f], b) and got[2][f] == it and got[3][f] == ok
        assert np.array_equal(got[1][f], p)  # == treats +0 and -0 as equal


def test_dense_matches_sparse_on_medium_code(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    llr = wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=302, n=1024, batch=200)
    got = dense(tdev, H, llr, 50)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    sp = tuple(t.cpu().numpy() for t in ldpc.minsum_decode(g, torch.from_numpy(llr).to(dev), 50))
    note(f"[dense] n=1024 mean iters {got[2].mean():.2f}")
    assert np.array_equal(got[0], sp[0]) and np.array_equal(got[2], sp[2]) and np.array_equal(got[3], sp[3])
    assert np.array_equal(got[1], sp[1])
