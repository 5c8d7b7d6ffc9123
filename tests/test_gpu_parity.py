"""HIP path vs the CPU oracle, element by element, through the C-ABI."""
import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl
from parity import assert_parity, check, gpu_decode, note, oracle_decode

pytestmark = pytest.mark.gpu

PATHS = {"stream": 2, "onchip": 4}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_10424_amd import ldpc
    ldpc.load_library()


@pytest.mark.parametrize("path", sorted(PATHS))
def test_small_regular_code_full(path):
    """(3,6) Gallager code n=96, 1000 all-zero frames at Eb/N0 = 2 dB, L = 20."""
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    llr = wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=100, n=96, batch=1000)
    check(H, llr, 20, PATHS[path], what=f"C0 {path}")


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("B", [1, 63, 64, 65, 130])
def test_ragged_batches(path, B):
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    enc = wl.gf2_encoder(H)
    cw = enc.random_codewords(B, seed=B)
    llr = wl.bpsk_awgn_llr(cw, 1.5, 0.5, seed=B + 1)
    check(H, llr, 15, PATHS[path], what=f"ragged {path}")


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("L", [0, 1, 2])
@pytest.mark.parametrize("flags", [0, 1])
def test_iteration_limits(path, L, flags):
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    llr = wl.bpsk_awgn_llr(None, 1.0, 0.5, seed=7, n=96, batch=200)
    check(H, llr, L, PATHS[path] | flags, what=f"L={L} {path}")


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("period", [2, 6])
@pytest.mark.parametrize("L", [20, 23])
def test_check_period(path, period, L):
    """The paper's termination variant: codeword test before the first
    iteration and after every k-th one (k = 6 in its GPU experiments)."""
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    llr = wl.bpsk_awgn_llr(None, 1.5, 0.5, seed=31 + period, n=96, batch=700)
    gpu, ref = check(H, llr, L, PATHS[path] | (period << 8), what=f"period {period} {path}")
    assert np.all((ref[2] % period == 0) | (ref[2] == L))
    Hi = wl.random_irregular_code(500, 230, seed=4, dv_choices=(2, 3, 4, 6), max_row_degree=16)
    llr = np.random.default_rng(period).normal(1.2, 1.4, size=(300, 500)).astype(np.float32)
    check(Hi, llr, L, PATHS[path] | (period << 8), what=f"period {period} irregular {path}")


@pytest.mark.parametrize("path", sorted(PATHS))
def test_paper_example_codewords(path):
    from oracle_pins import codebook
    H = wl.paper_tanner_example()
    book = codebook(H)
    r = (1.5 * (1.0 - 2.0 * book.astype(np.float32))).astype(np.float32)
    gpu, _ = check(H, r, 10, PATHS[path], what="paper 5x10 codewords")
    assert np.all(gpu[2] == 0) and np.array_equal(gpu[0], book) and np.array_equal(gpu[1], r)


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("seed", range(6))
def test_irregular_codes(path, seed):
    """Irregular degrees, bits of degree 0, rows longer than 32."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(40, 300))
    m = int(rng.integers(n // 6, n // 2))
    H = wl.random_irregular_code(n, m, seed=seed, dv_choices=(0, 1, 2, 3, 4, 6, 9), max_row_degree=64)
    if seed % 2 == 0:
        H = np.vstack([H, np.zeros((1, n), np.uint8)])  # a row of degree 0
    llr = rng.normal(1.0, 1.3, size=(int(rng.integers(50, 260)), n)).astype(np.float32)
    check(H, llr, 25, PATHS[path], what=f"irregular {seed} {path}")
    check(H, llr, 25, PATHS[path] | 1, what=f"irregular {seed} {path} no-exit")


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("shape", [(60, 24), (500, 230), (900, 420), (2000, 900), (1800, 420)])
def test_irregular_moderate_degrees(path, shape):
    """Irregular codes with row and column degrees <= 16 (the on-chip limits),
    from a few rows to about a thousand."""
    n, m = shape
    H = wl.random_irregular_code(n, m, seed=n + m, dv_choices=(0, 1, 2, 3, 4, 5), max_row_degree=16)
    rng = np.random.default_rng(n)
    llr = rng.normal(1.2, 1.2, size=(333, n)).astype(np.float32)
    check(H, llr, 30, PATHS[path], what=f"irregular moderate {shape} {path}")


@pytest.mark.parametrize("path", sorted(PATHS))
def test_long_rows(path):
    """Check rows of degree 30..60 (beyond a 32-bit sign mask)."""
    H = wl.random_irregular_code(300, 8, seed=9, dv_choices=(1, 2), max_row_degree=64)
    assert H.sum(1).max() > 32
    llr = np.random.default_rng(9).normal(1.5, 1.0, size=(150, 300)).astype(np.float32)
    check(H, llr, 20, PATHS[path], what="long rows")
    check(H, llr, 20, PATHS[path] | 1, what="long rows no-exit")


@pytest.mark.parametrize("path", sorted(PATHS))
def test_tree_codes_no_early_exit(path):
    for seed in range(12):
        H = wl.tree_code(2 + seed % 6, seed=1000 + seed, max_check_degree=2 + seed % 4)
        m, n = H.shape
        llr = np.random.default_rng(seed).normal(0.5, 1.5, size=(70, n)).astype(np.float32)
        check(H, llr, n + m, PATHS[path] | 1, what=f"tree {seed}")


@pytest.mark.parametrize("path", sorted(PATHS))
def test_adversarial_llrs(path):
    """Exact ties between magnitudes, signed zeros, extreme scales."""
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    rng = np.random.default_rng(3)
    vals = np.array([1.0, -1.0, 2.0, -2.0, 0.5, -0.5, 0.0, -0.0], np.float32)
    a = vals[rng.integers(0, vals.size, size=(300, 96))]
    a[:100] += np.float32(1.0)  # mostly positive, still many ties
    b = a * np.float32(2.0 ** 60)
    c = a * np.float32(2.0 ** -60)
    d = np.zeros((10, 96), np.float32)
    e = -np.zeros((10, 96), np.float32)
    for name, llr in [("ties", a), ("huge", b), ("tiny", c), ("zeros", d), ("negzeros", e)]:
        check(H, llr, 20, PATHS[path], what=f"adversarial {name}")


@pytest.mark.parametrize("path", sorted(PATHS))
def test_non_finite_llrs_stay_in_their_frame(path):
    """Infinite and NaN LLRs (outside the contract: their frames' outputs are
    unspecified) leave every other frame equal to the oracle, and the outputs
    of their own frames within their ranges."""
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    L = 20
    llr = wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=51, n=96, batch=256).astype(np.float32)
    bad = np.arange(40, 72)
    rng = np.random.default_rng(52)
    for k, f in enumerate(bad):
        if k % 4 == 0:
            llr[f, :] = np.nan
        else:
            cols = rng.choice(96, size=1 + k % 5, replace=False)
            llr[f, cols] = [np.inf, -np.inf, np.nan][k % 3]
    note(f"[parity] non-finite LLRs path={path} frames={bad.size} of {llr.shape[0]}")
    gb, gp, gi, go = gpu_decode(H, llr, L, PATHS[path])
    good = np.setdiff1d(np.arange(llr.shape[0]), bad)
    ref = oracle_decode(H, llr[good], L, PATHS[path])
    assert_parity((gb[good], gp[good], gi[good], go[good]), ref, "finite frames beside non-finite ones")
    assert np.isin(gb[bad], (0, 1)).all() and np.isin(go[bad], (0, 1)).all()
    assert (gi[bad] >= 0).all() and (gi[bad] <= L).all()


@pytest.mark.parametrize("path", sorted(PATHS))
def test_nms_weights(path):
    H = wl.random_irregular_code(120, 60, seed=4, dv_choices=(2, 3, 4))
    import oracle
    C = oracle.check_degrees(H).size
    rng = np.random.default_rng(5)
    T = 12
    alpha = rng.uniform(0.5, 1.2, size=(T, C)).astype(np.float32)
    beta = rng.uniform(0.0, 0.4, size=(T, C)).astype(np.float32)
    llr = rng.normal(1.0, 1.2, size=(300, 120)).astype(np.float32)
    check(H, llr, T, PATHS[path], alpha, beta, what="nms")
    check(H, llr, 7, PATHS[path] | 1, alpha, beta, what="nms no-exit")
    ones, zeros = np.ones((T, C), np.float32), np.zeros((T, C), np.float32)
    g1 = gpu_decode(H, llr, T, PATHS[path], ones, zeros)
    g0 = gpu_decode(H, llr, T, PATHS[path])
    for x, y in zip(g1, g0):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("path", sorted(PATHS))
def test_nms_disjoint_single_checks(path):
    """Learned update on disjoint single checks of degrees 5, 3, 7, 3 (a row's
    degree class differs from its row index), its own weights per iteration
    and class, offsets that zero some messages, dyadic inputs: every step is
    exact in binary32, so the posteriors must equal the oracle's bit for bit."""
    degs = (5, 3, 7, 3)
    H = np.zeros((len(degs), sum(degs)), np.uint8)
    col = 0
    for i, d in enumerate(degs):
        H[i, col:col + d] = 1
        col += d
    rng = np.random.default_rng(23)
    T, C = 4, 3
    alpha = (rng.integers(1, 8, size=(T, C)) / 4.0).astype(np.float32)
    beta = (rng.integers(0, 24, size=(T, C)) / 4.0).astype(np.float32)
    mag = rng.integers(1, 256, size=(150, H.shape[1])) / 32.0
    llr = (np.where(rng.random(mag.shape) < 0.4, -1.0, 1.0) * mag).astype(np.float32)
    for t in range(1, T + 1):
        gpu, ref = check(H, llr, t, PATHS[path] | 1, alpha, beta, what=f"nms single checks t={t} {path}")
        assert np.array_equal(gpu[1], ref[1])
    check(H, llr, T, PATHS[path], alpha, beta, what=f"nms single checks early exit {path}")


@pytest.mark.parametrize("path", sorted(PATHS))
def test_nms_shipped_weights_many_refills(path):
    """The shipped learned weights of the (3,6) n = 1024 code (one weight
    class: the exact-degree kernels, weights read once per workgroup),
    20,011 frames at 2.0 and 2.5 dB, so every slot refills many times and
    each refill takes its LLRs from the look-ahead; early exit, an iteration
    limit below T and a codeword-test period of 6."""
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(root, "paper_2507_10424_amd", "weights", "nms_regular1024.json")) as f:
        rec = json.load(f)
    alpha = np.asarray(rec["alpha"], np.float32)
    beta = np.asarray(rec["beta"], np.float32)
    T = alpha.shape[0]
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    enc = wl.gf2_encoder(H)
    for eb, seed in ((2.0, 91), (2.5, 92)):
        cw = enc.random_codewords(20011, seed=seed)
        llr = wl.bpsk_awgn_llr(cw, eb, 0.5, seed=seed + 10)
        check(H, llr, T, PATHS[path], alpha, beta, what=f"shipped weights {eb} dB {path}")
    check(H, llr, T - 7, PATHS[path], alpha, beta, what=f"shipped weights L=T-7 {path}")
    check(H, llr, T, PATHS[path] | (6 << 8), alpha, beta, what=f"shipped weights period 6 {path}")


@pytest.mark.parametrize("path", sorted(PATHS))
def test_medium_code_subset(path):
    """(3,6) n=1024 code, random codewords, 4096 frames at 1.5 dB, L = 50."""
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    enc = wl.gf2_encoder(H)
    cw = enc.random_codewords(4096, seed=201)
    llr = wl.bpsk_awgn_llr(cw, 1.5, 0.5, seed=301)
    check(H, llr, 50, PATHS[path], what="C1 subset")


@pytest.mark.parametrize("path", sorted(PATHS))
def test_determinism(path):
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    llr = wl.bpsk_awgn_llr(None, 1.25, 0.5, seed=5, n=1024, batch=700)
    a = gpu_decode(H, llr, 30, PATHS[path])
    b = gpu_decode(H, llr, 30, PATHS[path])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_paths_agree_and_auto_choice():
    """Both kernel paths give identical outputs; without a flag the on-chip
    path is taken when the graph fits."""
    from paper_2507_10424_amd import ldpc
    import torch
    H = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    llr = wl.bpsk_awgn_llr(None, 1.5, 0.5, seed=8, n=1024, batch=500)
    a = gpu_decode(H, llr, 40, ldpc.LDPC_FORCE_STREAM)
    b = gpu_decode(H, llr, 40, ldpc.LDPC_FORCE_ONCHIP)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    g = ldpc.build_graph(torch.from_numpy(H).cuda())
    assert ldpc.workspace_bytes(g, 500) == ldpc.workspace_bytes(g, 500, ldpc.LDPC_FORCE_ONCHIP)
    assert ldpc.workspace_bytes(g, 500) < ldpc.workspace_bytes(g, 500, ldpc.LDPC_FORCE_STREAM)


@pytest.mark.parametrize("path", sorted(PATHS))
def test_largest_onchip_regular_code(path):
    """(3,6) code n = 2048: 512 threads of two rows and four bits each and
    65 KB of LDS state, the largest (3,6) code the on-chip path takes; the
    streaming path decodes the same frames."""
    H = wl.regular_ldpc(2048, 1024, 3, 6, seed=8)
    llr = wl.bpsk_awgn_llr(None, 1.75, 0.5, seed=88, n=2048, batch=300)
    check(H, llr, 40, PATHS[path], what=f"n=2048 {path}")


def test_onchip_refuses_too_many_threads():
    """n = 4096 needs 1024 threads of two rows: the on-chip path reports
    LDPC_EUNSUPPORTED when forced, and the automatic choice streams."""
    import torch
    from paper_2507_10424_amd import ldpc
    H = wl.regular_ldpc(4096, 2048, 3, 6, seed=9)
    g = ldpc.build_graph(torch.from_numpy(H).to("cuda:0"))
    x = torch.from_numpy(wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=9, n=4096, batch=70)).to("cuda:0")
    with pytest.raises(ldpc.LdpcError) as e:
        ldpc.minsum_decode(g, x, 10, flags=PATHS["onchip"])
    assert e.value.status == -6
    out = ldpc.minsum_decode(g, x, 10)
    torch.cuda.synchronize()
    assert_parity(tuple(t.cpu().numpy() for t in out), oracle_decode(H, x.cpu().numpy(), 10), "n=4096 auto")


@pytest.mark.parametrize("B", [1023, 1025, 5003, 20011])
def test_every_frame_decoded_once(B):
    """Frame numbers come from up to 16 counters (one per 1,024 frames) that
    hand out interleaved frames and run dry at different times; every frame
    must be decoded exactly once.  The outputs are prefilled with values no
    decode produces, so a skipped frame shows; a frame decoded twice would
    still match, but then another would be skipped."""
    import torch
    from paper_2507_10424_amd import ldpc
    dev = torch.device("cuda:0")
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    llr = wl.bpsk_awgn_llr(None, 2.5, 0.5, seed=1300 + B, n=96, batch=B)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    out = ldpc._outputs(B, 96, dev, True)
    out[0].fill_(7)
    out[1].fill_(float("nan"))
    out[2].fill_(-7)
    out[3].fill_(9)
    ldpc.minsum_decode(g, torch.from_numpy(llr).to(dev), 30, flags=ldpc.LDPC_FORCE_ONCHIP, out=out)
    torch.cuda.synchronize()
    got = tuple(t.cpu().numpy() for t in out)
    assert (got[2] >= 0).all() and (got[3] <= 1).all() and (got[0] <= 1).all() and not np.isnan(got[1]).any()
    assert_parity(got, oracle_decode(H, llr, 30), f"B={B}")
