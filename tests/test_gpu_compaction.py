"""Frame compaction of the streaming decoder (GPU): batches of at least 16
tiles of 64 frames with early exit, where frames stop at many different
iterations, so that compaction plans go ahead; every output is compared with
the oracle."""
import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl
from parity import assert_parity, note, oracle_decode

pytestmark = pytest.mark.gpu

STREAM = 2  # LDPC_FORCE_STREAM


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_10424_amd import ldpc
    ldpc.load_library()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def code():
    return wl.regular_ldpc(1024, 512, 3, 6, seed=2)


def run(tdev, H, llr_np, L, flags=0, chunk=-1, alpha=None, beta=None):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    ldpc.set_tuning(g, 2, stream_waves=4, stream_nt=-1, stream_chunk=chunk)
    x = torch.from_numpy(llr_np).to(dev)
    if alpha is None:
        out = ldpc.minsum_decode(g, x, L, flags=flags | STREAM)
    else:
        out = ldpc.nms_decode(g, x, L, torch.from_numpy(alpha).to(dev), torch.from_numpy(beta).to(dev),
                              flags=flags | STREAM)
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in out)


@pytest.mark.parametrize("ebn0,B", [(2.5, 2048), (2.0, 1500), (3.0, 1089)])
def test_compacted_batch_matches_oracle(tdev, code, ebn0, B):
    note(f"[compaction] whole batch Eb/N0={ebn0} B={B}")
    llr = wl.bpsk_awgn_llr(None, ebn0, 0.5, seed=int(ebn0 * 10) + B, n=1024, batch=B)
    got = run(tdev, code, llr, 50)
    ref = oracle_decode(code, llr, 50)
    assert_parity(got, ref, f"compaction {ebn0} dB B={B}")
    # frames stop at many iterations (the plans have something to pack)
    assert len(np.unique(ref[2])) > 8


def test_compaction_with_check_period_and_chunks(tdev, code):
    B = 64 * 40  # chunks of 16, 16 and 8 tiles
    llr = wl.bpsk_awgn_llr(None, 2.3, 0.5, seed=77, n=1024, batch=B)
    flags = 3 << 8  # codeword test after every 3rd iteration
    note(f"[compaction] chunks of 16 tiles, period 3, B={B}")
    got = run(tdev, code, llr, 40, flags=flags, chunk=16)
    ref = oracle_decode(code, llr, 40, flags=flags)
    assert_parity(got, ref, "compaction, chunks of 16 tiles, period 3")


def test_compaction_learned_decoder(tdev, code):
    B = 1300
    T = 30
    rng = np.random.default_rng(9)
    alpha = rng.uniform(0.6, 1.1, size=(T, 1)).astype(np.float32)
    beta = rng.uniform(0.0, 0.3, size=(T, 1)).astype(np.float32)
    llr = wl.bpsk_awgn_llr(None, 2.4, 0.5, seed=78, n=1024, batch=B)
    note(f"[compaction] learned decoder B={B}")
    got = run(tdev, code, llr, T, alpha=alpha, beta=beta)
    ref = oracle_decode(code, llr, T, alpha=alpha, beta=beta)
    assert_parity(got, ref, "compaction, learned decoder")


def test_no_early_exit_keeps_every_frame(tdev, code):
    B = 1100
    llr = wl.bpsk_awgn_llr(None, 2.5, 0.5, seed=79, n=1024, batch=B)
    got = run(tdev, code, llr, 12, flags=1)  # LDPC_NO_EARLY_EXIT: nothing stops, nothing compacts
    ref = oracle_decode(code, llr, 12, flags=1)
    assert_parity(got, ref, "no early exit")
