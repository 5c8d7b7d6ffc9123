"""Seeded random sweep (GPU): code shapes, batch sizes (up to the sizes the
streaming decoder compacts), iteration limits, flags (no early exit,
codeword-test period), kernel paths, launch choices (on-chip variant,
register budget and workgroups per CU; streaming wavefronts, non-temporal
messages and chunks) and learned weights, every case against the CPU oracle.
LDPC_RANDOM_CASES sets the number of cases (48 by default)."""
import os

import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl
from parity import assert_parity, note, oracle_decode

pytestmark = pytest.mark.gpu

N_CASES = int(os.environ.get("LDPC_RANDOM_CASES", "48"))


def _case(k):
    rng = np.random.default_rng(10_000 + k)
    kind = rng.choice(["regular", "irregular", "qc"])
    if kind == "regular":
        dv, dc = [(3, 6), (2, 4), (4, 8), (3, 9)][rng.integers(4)]
        m = int(rng.integers(4, 60)) * dv
        n = m * dc // dv
        H = wl.regular_ldpc(n, m, dv, dc, seed=int(rng.integers(1 << 30)))
    elif kind == "irregular":
        n = int(rng.integers(20, 700))
        m = int(rng.integers(n // 6 + 2, n // 2 + 3))
        H = None
        for cap in (int(rng.choice([8, 16, 40])), 40, 64):  # a shape may need rows above the first cap
            try:
                H = wl.random_irregular_code(n, m, seed=int(rng.integers(1 << 30)), dv_choices=(0, 1, 2, 3, 4, 6),
                                             max_row_degree=cap)
                break
            except RuntimeError:
                continue
        assert H is not None
    else:
        Z = int(rng.choice([8, 16, 24]))
        H = wl.qc_irregular_ldpc(12, 6, Z, [2] * 6 + [3] * 4 + [6] * 2, seed=int(rng.integers(1 << 30)))
    B = int(rng.choice([1, 7, 64, 65, 130, 333]))
    L = int(rng.integers(0, 31))
    flags = int(rng.choice([0, 1, 2 << 8, 5 << 8]))  # early exit, none, period 2, period 5
    path = int(rng.choice([0, 2, 4]))                 # auto, streaming, on-chip
    learned = bool(rng.random() < 0.3) and L >= 1
    llr = (rng.normal(1.0, rng.uniform(0.6, 2.0), size=(B, H.shape[1])) * rng.uniform(0.5, 4.0)).astype(np.float32)
    return kind, H, B, L, flags, path, learned, llr, rng


@pytest.mark.parametrize("k", range(N_CASES))
def test_random_case(k):
    import torch
    from paper_2507_10424_amd import ldpc
    import oracle
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kind, H, B, L, flags, path, learned, llr, rng = _case(k)
    dev = torch.device("cuda:0")
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    rs = np.random.default_rng(777 + k)
    if rs.random() < 0.35:  # large enough for frame compaction on the streaming path
        B = int(rs.choice([1024, 1100, 1500, 2049]))
        llr = (rs.normal(1.0, rs.uniform(0.6, 2.0), size=(B, H.shape[1])) * rs.uniform(0.5, 4.0)).astype(np.float32)
    tun = None
    if path == 2 or (path == 0 and rs.random() < 0.5):
        tun = dict(path=2, stream_waves=int(rs.choice([1, 2, 4, 8])), stream_nt=int(rs.choice([-1, 0, 1])),
                   stream_chunk=int(rs.choice([-1, 0, 1, 2, 16])))
        ldpc.set_tuning(g, **tun)
    elif path in (0, 4):
        for _ in range(20):  # a variant that fits the graph, if one of 20 draws does
            cand = dict(path=1, variant=int(rs.integers(0, 42)), wg_per_cu=int(rs.integers(0, 5)),
                        waves_per_simd=int(rs.choice([0, 4, 3])))
            try:
                ldpc.set_tuning(g, **cand)
                tun = cand
                break
            except ldpc.LdpcError:
                continue
    note(f"[random {k}] {kind} m={H.shape[0]} n={H.shape[1]} B={B} L={L} flags={flags} path={path} "
         f"learned={learned} tuning={tun}")
    x = torch.from_numpy(llr).to(dev)
    try:
        if learned:
            C = len(oracle.check_degrees(H))
            alpha = rng.uniform(0.6, 1.1, size=(L, C)).astype(np.float32)
            beta = rng.uniform(0.0, 0.4, size=(L, C)).astype(np.float32)
            out = ldpc.nms_decode(g, x, L, torch.from_numpy(alpha).to(dev), torch.from_numpy(beta).to(dev),
                                  flags=flags | path)
            ref = oracle_decode(H, llr, L, flags, alpha, beta)
        else:
            out = ldpc.minsum_decode(g, x, L, flags=flags | path)
            ref = oracle_decode(H, llr, L, flags)
    except ldpc.LdpcError as e:
        if e.status == -6 and path == 4:
            pytest.skip("graph does not fit the on-chip path")
        raise
    torch.cuda.synchronize()
    assert_parity(tuple(t.cpu().numpy() for t in out), ref, f"random case {k}")
