"""Full-size workloads in the launch configuration bench.py times, checked on
frames the oracle decodes one by one (GPU, HIP path through the C-ABI)."""
import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl
from parity import assert_parity, note, oracle_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _decode_full(H, llr_t, L, tune_ebn0, flags=0):
    """Autotune on the full batch as bench.py does, then decode with the
    chosen launch configuration."""
    import torch
    from paper_2507_10424_amd import ldpc
    g = ldpc.build_graph(torch.from_numpy(H).to(llr_t.device))
    tuning = ldpc.autotune(g, min(llr_t.shape[0], 65536), L, tune_ebn0)
    note(f"[large] tuned launch: {tuning}")
    out = ldpc.minsum_decode(g, llr_t, L, flags=flags)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def _check_all_frames(H, out, L):
    """Properties every frame must have at any size: iterations within
    [0, L]; a frame that stopped early is a codeword; the flag is the
    codeword test of the returned decision; bits are the slicer of post."""
    import scipy.sparse as sp
    gb, gp, gi, go = out
    assert gi.min() >= 0 and gi.max() <= L
    assert np.all(go[gi < L] == 1)
    syn = (sp.csr_matrix(H.astype(np.int32)) @ gb.T.astype(np.int32)) % 2  # m x B, by a sparse product
    assert np.array_equal(go == 1, ~np.asarray(syn).any(axis=0))
    assert np.array_equal(gb, (gp < 0).astype(np.uint8))


def _sample(iters, k, rng):
    """k frames: the slowest, the fastest and random ones."""
    idx = {int(np.argmax(iters)), int(np.argmin(iters))}
    while len(idx) < k:
        idx.add(int(rng.integers(iters.size)))
    return np.array(sorted(idx))


def test_regular1024_full_batch(dev):
    """(3,6) n=1024, 65536 random codewords at 2.0 dB, L=50, auto path."""
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    enc = wl.gf2_encoder(H)
    cw = enc.random_codewords_torch(65536, 202, dev)
    llr = wl.bpsk_awgn_llr_torch(cw, 2.0, 0.5, 302, dev)
    gb, gp, gi, go = _decode_full(H, llr, 50, 2.0)
    _check_all_frames(H, (gb, gp, gi, go), 50)
    idx = _sample(gi, 192, np.random.default_rng(0))
    note(f"[large] n=1024 full batch, checking {idx.size} frames, mean iters {gi.mean():.2f}")
    ref = oracle_decode(H, llr.cpu().numpy()[idx], 50)
    assert_parity((gb[idx], gp[idx], gi[idx], go[idx]), ref, "n=1024 sampled")


@pytest.mark.parametrize("ebn0", [1.0, 1.6])
def test_qc64800_full_batch(dev, ebn0):
    """Irregular QC n=64800, 4096 all-zero frames, L=50 (streaming path)."""
    H = wl.large_qc_code(seed=5)
    llr = wl.bpsk_awgn_llr_torch(None, ebn0, 0.5, 500, dev, n=H.shape[1], batch=4096)
    gb, gp, gi, go = _decode_full(H, llr, 50, 1.2)
    _check_all_frames(H, (gb, gp, gi, go), 50)
    idx = _sample(gi, 4, np.random.default_rng(1))
    note(f"[large] n=64800 at {ebn0} dB, checking frames {idx.tolist()}, mean iters {gi.mean():.2f}")
    ref = oracle_decode(H, llr.cpu().numpy()[idx], 50)
    assert_parity((gb[idx], gp[idx], gi[idx], go[idx]), ref, f"n=64800 {ebn0} dB sampled")
