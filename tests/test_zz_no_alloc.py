"""The decode entry point that allocates nothing (ldpc_minsum_decode_noalloc)
against ldpc_minsum_decode, called through the C-ABI: identical outputs on
both kernel paths, on two calls in a row with the second smaller, and the
size limit refused before any launch."""
import ctypes

import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl
from parity import note

pytestmark = pytest.mark.gpu

SCRATCH = 16 << 20  # LDPC_NOALLOC_SCRATCH_BYTES


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_10424_amd import ldpc
    lib = ldpc.load_library()
    return torch, torch.device("cuda:0"), ldpc, lib


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _run(torch, dev, ldpc, lib, g, llr, L, flags, noalloc):
    B, n = llr.shape
    bits = torch.full((B, n), 7, dtype=torch.uint8, device=dev)
    post = torch.full((B, n), float("nan"), dtype=torch.float32, device=dev)
    iters = torch.full((B,), -9, dtype=torch.int32, device=dev)
    ok = torch.full((B,), 9, dtype=torch.uint8, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    if noalloc:
        st = lib.ldpc_minsum_decode_noalloc(g.handle, _p(llr), B, L, flags, _p(bits), _p(post), _p(iters), _p(ok),
                                            stream)
    else:
        need = int(lib.ldpc_decode_workspace_bytes(g.handle, B, flags))
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        st = lib.ldpc_minsum_decode(g.handle, _p(llr), B, L, flags, _p(bits), _p(post), _p(iters), _p(ok), _p(ws),
                                    ws.numel(), stream)
    assert st == 0, ldpc.LdpcError(st, "decode")
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (bits, post, iters, ok)]


@pytest.mark.parametrize("path", ["onchip", "stream"])
def test_noalloc_equals_workspace_decode(env, path):
    torch, dev, ldpc, lib = env
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    flags = ldpc.LDPC_FORCE_ONCHIP if path == "onchip" else ldpc.LDPC_FORCE_STREAM
    # first call larger than the second, so stale scratch contents would show
    for B, eb, seed in ((340 if path == "stream" else 20000, 1.8, 31), (130, 2.2, 32)):
        note(f"[noalloc] path={path} B={B} Eb/N0={eb}")
        need = int(lib.ldpc_decode_workspace_bytes(g.handle, B, flags))
        assert need <= SCRATCH
        llr = torch.from_numpy(wl.bpsk_awgn_llr(None, eb, 0.5, seed=seed, n=1024, batch=B)).to(dev)
        want = _run(torch, dev, ldpc, lib, g, llr, 50, flags, noalloc=False)
        got = _run(torch, dev, ldpc, lib, g, llr, 50, flags, noalloc=True)
        for a, b, name in zip(got, want, ("bits", "post", "iters", "ok")):
            assert np.array_equal(a, b), (path, B, name)
        assert want[2].min() >= 0 and want[2].max() <= 50


def test_noalloc_stream_with_frame_compaction(env):
    """The streaming path with frame compaction (chunks of at least 16 tiles):
    the n = 96 code, 2,000 then 1,100 frames, both within the scratch array,
    so the plans, copies and both state sets live in it."""
    torch, dev, ldpc, lib = env
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    flags = ldpc.LDPC_FORCE_STREAM
    for B, eb, seed in ((2000, 2.0, 41), (1100, 2.5, 42)):
        note(f"[noalloc] path=stream n=96 B={B} Eb/N0={eb}")
        assert (B + 63) // 64 >= 16  # chunks of 16 tiles or more are compacted
        need = int(lib.ldpc_decode_workspace_bytes(g.handle, B, flags))
        assert need <= SCRATCH
        llr = torch.from_numpy(wl.bpsk_awgn_llr(None, eb, 0.5, seed=seed, n=96, batch=B)).to(dev)
        want = _run(torch, dev, ldpc, lib, g, llr, 50, flags, noalloc=False)
        got = _run(torch, dev, ldpc, lib, g, llr, 50, flags, noalloc=True)
        for a, b, name in zip(got, want, ("bits", "post", "iters", "ok")):
            assert np.array_equal(a, b), (B, name)
        # frames stop at different iterations, so the plans have frames to pack
        assert want[2].min() < 10 and want[2].max() > 20


def test_noalloc_refuses_oversized_workspace(env):
    torch, dev, ldpc, lib = env
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    B = 4096  # streaming path: 4096 frames need about 168 MB of workspace
    flags = ldpc.LDPC_FORCE_STREAM
    assert int(lib.ldpc_decode_workspace_bytes(g.handle, B, flags)) > SCRATCH
    llr = torch.zeros((B, 1024), dtype=torch.float32, device=dev)
    bits = torch.full((B, 1024), 7, dtype=torch.uint8, device=dev)
    iters = torch.full((B,), -9, dtype=torch.int32, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    st = lib.ldpc_minsum_decode_noalloc(g.handle, _p(llr), B, 10, flags, _p(bits), None, _p(iters), None, stream)
    assert st == -5  # LDPC_EWORKSPACE
    torch.cuda.synchronize()
    assert int(bits.max()) == 7 and int(iters.min()) == -9  # nothing launched
