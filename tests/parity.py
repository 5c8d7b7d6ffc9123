"""Helpers of the GPU parity tests: run the HIP path through the C-ABI and
the CPU oracle on the same seeded inputs, and compare them."""
from __future__ import annotations

import sys

import numpy as np

import oracle

POST_RTOL = 1e-5  # |gpu - oracle| <= 1e-5 (1 + |oracle|) on posterior LLRs


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_decode(H, llr, L, flags=0, alpha=None, beta=None, graph=None, want_post=True):
    import torch
    from paper_2507_10424_amd import ldpc
    dev = torch.device("cuda:0")
    g = graph if graph is not None else ldpc.build_graph(torch.from_numpy(np.ascontiguousarray(H)).to(dev))
    x = torch.from_numpy(np.ascontiguousarray(llr, dtype=np.float32)).to(dev)
    if alpha is None:
        out = ldpc.minsum_decode(g, x, L, flags=flags, want_post=want_post)
    else:
        out = ldpc.nms_decode(g, x, L, torch.from_numpy(alpha).to(dev), torch.from_numpy(beta).to(dev),
                              flags=flags, want_post=want_post)
    torch.cuda.synchronize()
    bits, post, iters, ok = (None if t is None else t.cpu().numpy() for t in out)
    return bits, post, iters, ok


def oracle_decode(H, llr, L, flags=0, alpha=None, beta=None):
    early = not (flags & 1)
    period = max(1, (flags >> 8) & 0xFF)  # codeword-test period in bits 8..15 of the flags
    if alpha is None:
        return oracle.minsum_decode(H, llr, L, early_exit=early, check_period=period)
    return oracle.nms_decode(H, llr, L, alpha, beta, early_exit=early, check_period=period)


def assert_parity(gpu, ref, what=""):
    gb, gp, gi, go = gpu
    ob, op, oi, oo = ref
    bad = np.nonzero(np.any(gb != ob, axis=1))[0]
    assert bad.size == 0, f"{what}: hard decisions differ in {bad.size} frames, first {bad[:5]}"
    assert np.array_equal(gi, oi), f"{what}: iterations differ at frames {np.nonzero(gi != oi)[0][:5]}"
    assert np.array_equal(go, oo), f"{what}: convergence flags differ"
    if gp is not None:
        err = np.abs(gp.astype(np.float64) - op) - POST_RTOL * (1.0 + np.abs(op))
        assert np.all(err <= 0), f"{what}: posterior differs, worst excess {err.max():.3g}"


def check(H, llr, L, flags=0, alpha=None, beta=None, what=""):
    note(f"[parity] {what} m={H.shape[0]} n={H.shape[1]} B={llr.shape[0]} L={L} flags={flags}")
    from paper_2507_10424_amd import ldpc
    try:
        gpu = gpu_decode(H, llr, L, flags, alpha, beta)
    except ldpc.LdpcError as e:
        if e.status == -6 and flags & ldpc.LDPC_FORCE_ONCHIP:
            import pytest
            pytest.skip("graph does not fit the on-chip path")
        raise
    ref = oracle_decode(H, llr, L, flags, alpha, beta)
    assert_parity(gpu, ref, what)
    return gpu, ref
