"""Launch choices (GPU): every on-chip variant, occupancy cap and streaming
workgroup size gives the same outputs; the autotuner keeps a valid choice."""
import itertools

import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl
from parity import assert_parity, oracle_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def test_all_launch_choices_agree(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    llr_np = wl.bpsk_awgn_llr(None, 1.75, 0.5, seed=31, n=1024, batch=900)
    llr = torch.from_numpy(llr_np).to(dev)
    ref = oracle_decode(H, llr_np, 40)
    tried = 0
    for v, wpc, wps in itertools.product(range(42), (0, 1, 3), (0, 4)):
        try:
            ldpc.set_tuning(g, 1, variant=v, wg_per_cu=wpc, waves_per_simd=wps)
        except ldpc.LdpcError as e:
            assert e.status == -6
            continue
        out = ldpc.minsum_decode(g, llr, 40)
        torch.cuda.synchronize()
        assert_parity(tuple(t.cpu().numpy() for t in out), ref, f"variant {v} wpc {wpc} wps {wps}")
        tried += 1
    for waves, nt in itertools.product((1, 2, 4, 8), (0, 1)):
        ldpc.set_tuning(g, 2, stream_waves=waves, stream_nt=nt)
        out = ldpc.minsum_decode(g, llr, 40)
        torch.cuda.synchronize()
        assert_parity(tuple(t.cpu().numpy() for t in out), ref, f"stream waves {waves} non-temporal {nt}")
    assert tried >= 6 * 3 * 2
    # the learned update in both forms of the bank-conflict-free layout
    rng = np.random.default_rng(5)
    T = 40
    alpha = rng.uniform(0.6, 1.1, size=(T, 1)).astype(np.float32)
    beta = rng.uniform(0.0, 0.3, size=(T, 1)).astype(np.float32)
    ref_nms = oracle_decode(H, llr_np, T, alpha=alpha, beta=beta)
    for v in (14, 15):
        ldpc.set_tuning(g, 1, variant=v, waves_per_simd=4)
        out = ldpc.nms_decode(g, llr, T, torch.from_numpy(alpha).to(dev), torch.from_numpy(beta).to(dev))
        torch.cuda.synchronize()
        assert_parity(tuple(t.cpu().numpy() for t in out), ref_nms, f"learned, variant {v}")
    ldpc.set_tuning(g, None)
    assert ldpc.get_tuning(g)["path"] == 0


def test_autotune_keeps_valid_choice(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    best = ldpc.autotune(g, 4000, 20, 2.0)
    assert best["path"] in (1, 2) and best["ms"] > 0
    assert ldpc.get_tuning(g)["path"] == best["path"]
    llr_np = wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=100, n=96, batch=1000)
    out = ldpc.minsum_decode(g, torch.from_numpy(llr_np).to(dev), 20)
    torch.cuda.synchronize()
    assert_parity(tuple(t.cpu().numpy() for t in out), oracle_decode(H, llr_np, 20), "autotuned")


@pytest.mark.parametrize("B", [1, 3, 4, 5, 130, 777])
def test_four_slot_variants_ragged(tdev, B):
    """The four-slot variants (float4 LDS state) refill each slot on its own;
    batches that leave slots empty or uneven must decode like the oracle."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    llr_np = wl.bpsk_awgn_llr(None, 1.5, 0.5, seed=500 + B, n=96, batch=B)
    ref = oracle_decode(H, llr_np, 25)
    for v in (8, 9):
        for wpc in (0, 1):
            ldpc.set_tuning(g, 1, variant=v, wg_per_cu=wpc)
            out = ldpc.minsum_decode(g, torch.from_numpy(llr_np).to(dev), 25)
            torch.cuda.synchronize()
            assert_parity(tuple(t.cpu().numpy() for t in out), ref, f"variant {v} wpc {wpc} B {B}")


def test_stream_chunks_agree(tdev):
    """Chunked streaming (all iterations of a group of 64-frame tiles before
    the next group) decodes every frame like the oracle, for chunk sizes that
    divide the tiles, leave a ragged last chunk, exceed them, and by size;
    with the unrolled check kernel, the general one, learned weights and a
    codeword-test period."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    import oracle
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    llr_np = wl.bpsk_awgn_llr(None, 1.75, 0.5, seed=33, n=1024, batch=900)  # 15 tiles, the last ragged
    llr = torch.from_numpy(llr_np).to(dev)
    ref = oracle_decode(H, llr_np, 40)
    ref_p3 = oracle_decode(H, llr_np, 40, ldpc.check_period(3))
    for chunk, nt in itertools.product((1, 2, 4, 7, 15, 100, 0, -1), (0, 1)):
        ldpc.set_tuning(g, 2, stream_waves=4, stream_nt=nt, stream_chunk=chunk)
        assert ldpc.get_tuning(g)["stream_chunk"] == chunk
        out = ldpc.minsum_decode(g, llr, 40)
        torch.cuda.synchronize()
        assert_parity(tuple(t.cpu().numpy() for t in out), ref, f"chunk {chunk} non-temporal {nt}")
        if chunk in (4, -1):
            out = ldpc.minsum_decode(g, llr, 40, flags=ldpc.check_period(3))
            torch.cuda.synchronize()
            assert_parity(tuple(t.cpu().numpy() for t in out), ref_p3, f"chunk {chunk} period 3")

    Hi = wl.random_irregular_code(300, 150, seed=8, dv_choices=(0, 2, 3, 4, 6))
    gi = ldpc.build_graph(torch.from_numpy(Hi).to(dev))
    rng = np.random.default_rng(9)
    x_np = rng.normal(0.8, 1.3, size=(333, 300)).astype(np.float32)
    C = oracle.check_degrees(Hi).size
    T = 15
    alpha = rng.uniform(0.5, 1.2, size=(T, C)).astype(np.float32)
    beta = rng.uniform(0.0, 0.4, size=(T, C)).astype(np.float32)
    ref_i = oracle_decode(Hi, x_np, 30)
    ref_n = oracle_decode(Hi, x_np, T, 0, alpha, beta)
    x = torch.from_numpy(x_np).to(dev)
    for chunk in (1, 3, -1):
        ldpc.set_tuning(gi, 2, stream_waves=2, stream_chunk=chunk)
        out = ldpc.minsum_decode(gi, x, 30)
        torch.cuda.synchronize()
        assert_parity(tuple(t.cpu().numpy() for t in out), ref_i, f"irregular chunk {chunk}")
        out = ldpc.nms_decode(gi, x, T, torch.from_numpy(alpha).to(dev), torch.from_numpy(beta).to(dev))
        torch.cuda.synchronize()
        assert_parity(tuple(t.cpu().numpy() for t in out), ref_n, f"irregular nms chunk {chunk}")
    with pytest.raises(ldpc.LdpcError) as e:
        ldpc.set_tuning(gi, 2, stream_chunk=-2)
    assert e.value.status == -1


def test_kernel_timing_changes_no_output(tdev):
    """With per-kernel timing on, every timed kernel goes through
    hipExtLaunchKernel with its arguments marshalled by the library; the
    outputs must equal those of ordinary launches, and the launch counts must
    be what the decode issued."""
    import ctypes
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    lib = ldpc.load_library()
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    llr = torch.from_numpy(wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=77, n=1024, batch=700)).to(dev)
    Hd = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    gd = ldpc.build_graph(torch.from_numpy(Hd).to(dev))
    llrd = torch.from_numpy(wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=78, n=96, batch=300)).to(dev)
    runs = [("onchip", lambda: ldpc.minsum_decode(g, llr, 30, flags=ldpc.LDPC_FORCE_ONCHIP), {2: 1}),
            ("stream", lambda: ldpc.minsum_decode(g, llr, 30, flags=ldpc.LDPC_FORCE_STREAM), {0: 30, 1: 30}),
            ("dense", lambda: ldpc.minsum_decode_dense(gd, llrd, 30), {3: 30, 4: 30})]
    for name, fn, counts in runs:
        ref = fn()
        torch.cuda.synchronize()
        assert lib.ldpc_timing_enable(1) == 0
        got = fn()
        torch.cuda.synchronize()
        for kid, want in counts.items():
            ms, n = ctypes.c_double(), ctypes.c_int64()
            assert lib.ldpc_timing_read(kid, ctypes.byref(ms), ctypes.byref(n)) == 0
            assert n.value == want and ms.value > 0, (name, kid, n.value)
        assert lib.ldpc_timing_enable(0) == 0
        for a, b in zip(ref, got):
            if a is not None:
                assert torch.equal(a, b), name


def test_every_variant_on_qc_family(tdev):
    """Every on-chip variant that fits each of the eight QC codes (row degrees
    6, 9, 12, 16; bit degrees 2/3/6 or 2/3/4), at both register budgets,
    decodes like the oracle, plain and learned: among them the one-slot
    variants, the bit degree masked at 4 and the bank-conflict-free layout
    with columns padded to its stride."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    fam = wl.qc_multi_code_family(seed=7)
    for k, c in enumerate(fam):
        B = 90 + 13 * k
        llr_np = wl.bpsk_awgn_llr(None, 2.0, c["rate"], seed=400 + k, n=c["n"], batch=B)
        ref = oracle_decode(c["H"], llr_np, 30)
        g = ldpc.build_graph(torch.from_numpy(c["H"]).to(dev))
        llr = torch.from_numpy(llr_np).to(dev)
        # the learned update on the first 40 frames
        T = 30
        rng = np.random.default_rng(60 + k)
        alpha = rng.uniform(0.6, 1.1, size=(T, 1)).astype(np.float32)
        beta = rng.uniform(0.0, 0.3, size=(T, 1)).astype(np.float32)
        ref_nms = oracle_decode(c["H"], llr_np[:40], T, alpha=alpha, beta=beta)
        al, be = torch.from_numpy(alpha).to(dev), torch.from_numpy(beta).to(dev)
        tried = 0
        for v, wps in itertools.product(range(42), (0, 4, 3)):
            try:
                ldpc.set_tuning(g, 1, variant=v, waves_per_simd=wps)
            except ldpc.LdpcError as e:
                assert e.status == -6
                continue
            out = ldpc.minsum_decode(g, llr, 30)
            torch.cuda.synchronize()
            assert_parity(tuple(t.cpu().numpy() for t in out), ref, f"code {k} variant {v} wps {wps}")
            out = ldpc.nms_decode(g, llr[:40].contiguous(), T, al, be)
            torch.cuda.synchronize()
            assert_parity(tuple(t.cpu().numpy() for t in out), ref_nms, f"learned, code {k} variant {v} wps {wps}")
            tried += 1
        assert tried >= 2, f"code {k}: no variant fits"
