"""Decode calls captured into HIP graphs and replayed (GPU): every replay,
with eager work and synchronisations between replays, matches an eager
decode of the same inputs."""
import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.mark.parametrize("flags", [0, 2])  # auto (on-chip) and forced streaming
@pytest.mark.parametrize("n", [96, 1024])
@pytest.mark.parametrize("B", [700, 1500])  # streaming: 1,500 frames (24 tiles) are compacted
def test_replays_match_eager(tdev, flags, n, B):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    H = wl.regular_ldpc(n, n // 2, 3, 6, seed=1 if n == 96 else 2)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    cap = ldpc.CapturedDecode(g, B, 30, flags=flags)
    for rep in range(4):
        x = wl.bpsk_awgn_llr_torch(None, 1.0 + 0.5 * rep, 0.5, 900 + rep, dev, n=n, batch=B)
        cap.llr.copy_(x)
        got = [t.clone() for t in cap.replay()]
        torch.cuda.synchronize()
        want = ldpc.minsum_decode(g, x.clone(), 30, flags=flags)
        torch.cuda.synchronize()
        for a, b in zip(got, want):
            assert torch.equal(a, b), (rep, flags, n, B)


def test_multi_code_replays(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    fam = wl.qc_multi_code_family(seed=7)[:4]
    graphs = [ldpc.build_graph(torch.from_numpy(c["H"]).to(dev)) for c in fam]
    Bs = [300, 64, 200, 129]
    cap = ldpc.CapturedDecode(graphs, Bs, 40)
    for rep in range(3):
        xs = [wl.bpsk_awgn_llr_torch(None, 1.8 + 0.3 * rep, c["rate"], 70 + 10 * rep + k, dev, n=c["n"], batch=B)
              for k, (c, B) in enumerate(zip(fam, Bs))]
        for dst, x in zip(cap.llrs, xs):
            dst.copy_(x)
        got = [[t.clone() for t in o] for o in cap.replay()]
        torch.cuda.synchronize()
        for g, x, o in zip(graphs, xs, got):
            want = ldpc.minsum_decode(g, x, 40)
            torch.cuda.synchronize()
            for a, b in zip(o, want):
                assert torch.equal(a, b)
