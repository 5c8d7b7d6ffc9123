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
    idx = _sample(gi, 48, np.random.default_rng(1))
    note(f"[large] n=64800 at {ebn0} dB, checking {idx.size} frames, mean iters {gi.mean():.2f}")
    ref = oracle_decode(H, llr.cpu().numpy()[idx], 50)
    assert_parity((gb[idx], gp[idx], gi[idx], go[idx]), ref, f"n=64800 {ebn0} dB sampled")


def test_qc64800_learned_full_batch(dev):
    """The shipped learned weights on the n = 64800 code, 4096 frames at
    1.4 dB, T = 25, in the default (chunked streaming) launch; sampled frames
    against the oracle's learned decoder."""
    import json
    import os
    import torch
    from paper_2507_10424_amd import ldpc
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "paper_2507_10424_amd", "weights", "nms_qc64800.json")) as f:
        rec = json.load(f)
    alpha = np.asarray(rec["alpha"], np.float32)
    beta = np.asarray(rec["beta"], np.float32)
    T = alpha.shape[0]
    H = wl.large_qc_code(seed=5)
    llr = wl.bpsk_awgn_llr_torch(None, 1.4, 0.5, 510, dev, n=H.shape[1], batch=4096)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    out = ldpc.nms_decode(g, llr, T, torch.from_numpy(alpha).to(dev), torch.from_numpy(beta).to(dev))
    torch.cuda.synchronize()
    gb, gp, gi, go = (t.cpu().numpy() for t in out)
    _check_all_frames(H, (gb, gp, gi, go), T)
    idx = _sample(gi, 24, np.random.default_rng(2))
    note(f"[large] learned n=64800, checking {idx.size} frames, mean iters {gi.mean():.2f}")
    ref = oracle_decode(H, llr.cpu().numpy()[idx], T, 0, alpha, beta)
    assert_parity((gb[idx], gp[idx], gi[idx], go[idx]), ref, "learned n=64800 sampled")


def test_regular1024_concurrent_streams(dev):
    """Three full 65,536-frame decodes issued on three streams at once, as
    bench.py does, give the outputs of the same decodes run one after
    another."""
    import torch
    from paper_2507_10424_amd import ldpc
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    enc = wl.gf2_encoder(H)
    llrs = []
    for k, eb in enumerate((1.0, 2.5, 4.0)):
        cw = enc.random_codewords_torch(65536, 220 + k, dev)
        llrs.append(wl.bpsk_awgn_llr_torch(cw, eb, 0.5, 320 + k, dev))
    ref = [[t.clone() for t in ldpc.minsum_decode(g, x, 50) if t is not None] for x in llrs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(device=dev) for _ in llrs]
    cur = torch.cuda.current_stream()
    outs = []
    for s, x in zip(streams, llrs):
        s.wait_stream(cur)
        with torch.cuda.stream(s):
            ws = torch.empty(max(1, ldpc.workspace_bytes(g, x.shape[0])), dtype=torch.uint8, device=dev)
            outs.append((ldpc.minsum_decode(g, x, 50, workspace=ws), ws))
    for s in streams:
        cur.wait_stream(s)
    torch.cuda.synchronize()
    for k, ((o, _), r) in enumerate(zip(outs, ref)):
        for a, b in zip([t for t in o if t is not None], r):
            assert torch.equal(a, b), f"stream {k}"
