"""Learned decoder on the GPU: training forward/backward against the FP64
oracle, checkpoint recompute, frame generator, Adam, and the gain of a short
training run over plain Min-Sum."""
import numpy as np
import pytest

import oracle
from paper_2507_10424_amd import workloads as wl
from parity import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def _graph(torch, dev, H):
    from paper_2507_10424_amd import ldpc
    return ldpc.build_graph(torch.from_numpy(H).to(dev))


def _weights(T, C, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.6, 1.05, size=(T, C)).astype(np.float32),
            rng.uniform(0.0, 0.3, size=(T, C)).astype(np.float32))


CODES = {
    "regular96": lambda: wl.regular_ldpc(96, 48, 3, 6, seed=1),
    "irregular": lambda: wl.random_irregular_code(120, 50, seed=11, dv_choices=(1, 2, 3, 4), max_row_degree=12),
    "regular1024": lambda: wl.regular_ldpc(1024, 512, 3, 6, seed=2),
}


@pytest.mark.parametrize("code", ["regular96", "irregular"])
def test_forward_equals_decoder_and_oracle_loss(tdev, code):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    H = CODES[code]()
    C = oracle.check_degrees(H).size
    T, K = 7, 3
    a, b = _weights(T, C, 1)
    llr = wl.bpsk_awgn_llr(None, 1.5, 1 - H.shape[0] / H.shape[1], seed=3, n=H.shape[1], batch=64)
    g = _graph(torch, dev, H)
    at, bt, lt = (torch.from_numpy(x).to(dev) for x in (a, b, llr))
    ws = torch.empty(ldpc.train_workspace_bytes(g, 64, T, K), dtype=torch.uint8, device=dev)
    loss, post = ldpc.nms_train_forward(g, lt, at, bt, K, ws, want_post=True)
    _, dpost, _, _ = ldpc.nms_decode(g, lt, T, at, bt, flags=ldpc.LDPC_NO_EARLY_EXIT)
    torch.cuda.synchronize()
    assert np.array_equal(post.cpu().numpy(), dpost.cpu().numpy())
    _, opost, _, _ = oracle.nms_decode(H, llr, T, a, b, early_exit=False)
    assert np.array_equal(post.cpu().numpy(), opost)
    ref, _, _, _ = oracle.nms_train_loss_grad(H, llr.astype(np.float64), a.astype(np.float64),
                                              b.astype(np.float64), grad=False)
    assert abs(float(loss) - ref) <= 2e-5 * abs(ref)


U32 = 2.0 ** -24  # unit roundoff of binary32


def rounding_depth(H, T, B):
    """Roundings along the longest dependency chain of the binary32 backward
    (per iteration: the column sum of dv messages and the loss derivative,
    one subtraction, the weighted sums over a row's dc edges; after the
    sweep: a thread's rows, the block reduction and the sum over B frames),
    with a few for the sigmoid's exponential and division."""
    dv = int(H.sum(axis=0).max())
    dc = int(H.sum(axis=1).max())
    rows_per_thread = -(-H.shape[0] // 256)
    return T * (dv + 2 * dc + 8) + 2 * dc * rows_per_thread + B + 16


def assert_grad_parity(H, T, B, got, ref, what):
    """Every gradient entry within k u of the oracle's magnitude bound: the
    forward error bound of a binary32 evaluation of the reverse sweep whose
    decisions (argmin positions, signs, clip masks) are those of the binary32
    forward, which the oracle follows.  No entry is exempt."""
    k = rounding_depth(H, T, B)
    for name, bname in (("galpha", "aalpha"), ("gbeta", "abeta"), ("gllr", "allr")):
        if got.get(name) is None:
            continue
        g = got[name].astype(np.float64)
        err = np.abs(g - ref[name])
        tol = k * U32 * ref[bname] + 1e-30
        worst = float((err / tol).max())
        note(f"[nms-grad] {what} {name}: max |err| {err.max():.3e}, worst err / (k u bound) {worst:.3f} (k = {k})")
        assert np.all(err <= tol), (what, name, int((err > tol).sum()), worst)


@pytest.mark.parametrize("code", ["regular96", "irregular", "regular1024"])
def test_gradient_matches_fp64_oracle(tdev, code):
    """The GPU's binary32 forward and backward against the oracle's reverse
    sweep in double precision along the binary32 forward's decisions, entry by
    entry for alpha, beta and the LLRs."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    H = CODES[code]()
    C = oracle.check_degrees(H).size
    T, K, B = 10, 2, 16
    a, b = _weights(T, C, 2)
    llr = wl.bpsk_awgn_llr(None, 2.0, 1 - H.shape[0] / H.shape[1], seed=4, n=H.shape[1], batch=B)
    g = _graph(torch, dev, H)
    at, bt, lt = (torch.from_numpy(x).to(dev) for x in (a, b, llr))
    ws = torch.empty(ldpc.train_workspace_bytes(g, B, T, K), dtype=torch.uint8, device=dev)
    loss, post = ldpc.nms_train_forward(g, lt, at, bt, K, ws, want_post=True)
    ga, gb, gl = ldpc.nms_train_backward(g, lt, at, bt, K, ws, want_llr_grad=True)
    torch.cuda.synchronize()
    ref = oracle.nms_train_grad_f32_forward(H, llr, a, b, llr_grad=True)
    assert np.array_equal(post.cpu().numpy().astype(np.float64), ref["post"])  # same forward decisions
    assert abs(float(loss) - ref["loss"]) <= 2e-5 * abs(ref["loss"])
    assert_grad_parity(H, T, B, {"galpha": ga.cpu().numpy(), "gbeta": gb.cpu().numpy(), "gllr": gl.cpu().numpy()},
                       ref, code)


def test_checkpoint_interval_and_determinism(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    H = CODES["regular96"]()
    T, B = 9, 48
    a, b = _weights(T, 1, 5)
    llr = wl.bpsk_awgn_llr(None, 1.8, 0.5, seed=6, n=96, batch=B)
    g = _graph(torch, dev, H)
    at, bt, lt = (torch.from_numpy(x).to(dev) for x in (a, b, llr))
    outs = []
    for K in (1, 2, 3, 4, 9, 9):
        ws = torch.empty(ldpc.train_workspace_bytes(g, B, T, K), dtype=torch.uint8, device=dev)
        loss, _ = ldpc.nms_train_forward(g, lt, at, bt, K, ws)
        ga, gb, gl = ldpc.nms_train_backward(g, lt, at, bt, K, ws, want_llr_grad=True)
        outs.append([loss.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy(), gl.cpu().numpy()])
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            assert np.array_equal(x, y)


def test_autograd_function(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    from paper_2507_10424_amd.nms import NMSLoss
    H = CODES["regular96"]()
    T, K, B = 5, 2, 32
    a, b = _weights(T, 1, 7)
    llr = wl.bpsk_awgn_llr(None, 1.8, 0.5, seed=8, n=96, batch=B)
    g = _graph(torch, dev, H)
    at = torch.from_numpy(a).to(dev).requires_grad_(True)
    bt = torch.from_numpy(b).to(dev).requires_grad_(True)
    lt = torch.from_numpy(llr).to(dev).requires_grad_(True)
    ws = torch.empty(ldpc.train_workspace_bytes(g, B, T, K), dtype=torch.uint8, device=dev)
    loss = NMSLoss.apply(at, bt, lt, g, K, ws)
    (3.0 * loss).backward()
    ga, gb, gl = ldpc.nms_train_backward(g, lt.detach(), at.detach(), bt.detach(), K, ws, want_llr_grad=True)
    torch.cuda.synchronize()
    for x, y in [(at.grad, ga), (bt.grad, gb), (lt.grad, gl)]:
        assert torch.allclose(x, 3.0 * y, rtol=1e-6, atol=0)


def test_awgn_generator(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    llr = ldpc.awgn_llr(2000, 1000, 0.5, 2.0, seed=99, device=dev)
    again = ldpc.awgn_llr(2000, 1000, 0.5, 2.0, seed=99, device=dev)
    other = ldpc.awgn_llr(2000, 1000, 0.5, 2.0, seed=100, device=dev)
    assert torch.equal(llr, again) and not torch.equal(llr, other)
    s = wl.sigma_for_ebn0(2.0, 0.5)
    x = llr.double().cpu().numpy()
    assert abs(x.mean() - 2 / s**2) < 0.01 * 2 / s**2
    assert abs(x.std() - 2 / s) < 0.01 * 2 / s
    z = (x * s * s / 2 - 1) / s  # standard normal
    assert abs(np.mean(z**4) - 3.0) < 0.05  # Gaussian kurtosis
    cw = (torch.rand((300, 64), device=dev) < 0.5).to(torch.uint8)
    l2, eb = ldpc.awgn_llr(300, 64, 0.5, (1.0, 3.0), seed=5, device=dev, codewords=cw, want_ebn0=True)
    e = eb.cpu().numpy()
    assert e.min() >= 1.0 and e.max() < 3.0 and e.std() > 0.4
    flips = (l2 < 0).to(torch.uint8) != cw
    assert flips.float().mean() < 0.2


def test_adam_step(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    rng = np.random.default_rng(3)
    p = rng.normal(size=37).astype(np.float32)
    m1 = np.zeros(37, np.float32)
    m2 = np.zeros(37, np.float32)
    pt, m1t, m2t = (torch.from_numpy(x.copy()).to(dev) for x in (p, m1, m2))
    for step in range(1, 6):
        gr = rng.normal(size=37).astype(np.float32)
        ldpc.adam_step(pt, torch.from_numpy(gr).to(dev), m1t, m2t, 0.01, step)
        m1 = 0.9 * m1 + 0.1 * gr
        m2 = 0.999 * m2 + 0.001 * gr * gr
        p = p - 0.01 * (m1 / (1 - 0.9**step)) / (np.sqrt(m2 / (1 - 0.999**step)) + 1e-8)
    torch.cuda.synchronize()
    assert np.allclose(pt.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_training_gains_over_plain(tdev):
    """A short training run on the n=1024 code lowers the loss and, at the
    same 10 iterations, decodes fresh 2 dB frames with fewer bit errors than
    plain Min-Sum."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    from paper_2507_10424_amd.nms import NMSTrainer, frame_errors
    H = CODES["regular1024"]()
    g = _graph(torch, dev, H)
    tr = NMSTrainer(g, T=10, batch=512, ckpt_every=2, ebn0_range=(1.0, 3.0), lr=2e-2, seed=77)
    tr.train(120)
    hist = torch.stack(tr.history).cpu().numpy()
    note(f"[nms-train] loss first {hist[:10].mean():.4f} last {hist[-10:].mean():.4f}")
    assert hist[-20:].mean() < hist[:10].mean()
    llr = ldpc.awgn_llr(8192, 1024, 0.5, 2.0, seed=2024, device=dev)
    fe_p, be_p, it_p, _, _ = frame_errors(g, llr, 10)
    fe_n, be_n, it_n, _, _ = frame_errors(g, llr, 10, tr.alpha, tr.beta)
    note(f"[nms-train] 2 dB, 10 iterations: plain FER {fe_p / 8192:.4f} BER {be_p / 8192 / 1024:.2e}; "
         f"learned FER {fe_n / 8192:.4f} BER {be_n / 8192 / 1024:.2e}")
    assert be_n < be_p and fe_n <= fe_p


def test_gradient_with_state_in_device_memory(tdev):
    """A code whose per-frame training state exceeds one workgroup's LDS
    (QC, 180 x 90 base graph of the n = 64800 profile lifted by Z = 36)."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    cd = np.concatenate([np.full(36, 8), np.full(54, 3), np.full(90, 2)])
    cd = cd[np.random.default_rng(5).permutation(cd.size)]
    H = wl.qc_irregular_ldpc(180, 90, 36, cd, seed=9)
    C = oracle.check_degrees(H).size
    T, K, B = 4, 2, 3
    a, b = _weights(T, C, 12)
    llr = wl.bpsk_awgn_llr(None, 1.4, 0.5, seed=13, n=H.shape[1], batch=B)
    g = _graph(torch, dev, H)
    at, bt, lt = (torch.from_numpy(x).to(dev) for x in (a, b, llr))
    ws = torch.empty(ldpc.train_workspace_bytes(g, B, T, K), dtype=torch.uint8, device=dev)
    loss, post = ldpc.nms_train_forward(g, lt, at, bt, K, ws, want_post=True)
    ga, gb, _ = ldpc.nms_train_backward(g, lt, at, bt, K, ws)
    torch.cuda.synchronize()
    _, opost, _, _ = oracle.nms_decode(H, llr, T, a, b, early_exit=False)
    assert np.array_equal(post.cpu().numpy(), opost)
    ref = oracle.nms_train_grad_f32_forward(H, llr, a, b, llr_grad=False)
    assert abs(float(loss) - ref["loss"]) <= 2e-5 * abs(ref["loss"])
    assert_grad_parity(H, T, B, {"galpha": ga.cpu().numpy(), "gbeta": gb.cpu().numpy()}, ref, "qc6480")


N_RANDOM_GRAD = int(__import__("os").environ.get("LDPC_RANDOM_GRAD", "8"))


@pytest.mark.parametrize("k", range(N_RANDOM_GRAD))
def test_random_gradient_cases(tdev, k):
    """Seeded random codes (regular, irregular, QC), T = 1..12, checkpoint
    intervals 1, 2, 3 or T, 1..40 frames, random weights and Eb/N0: forward
    posteriors, loss and every gradient entry against the oracle's reverse
    sweep along the binary32 decisions.  LDPC_RANDOM_GRAD sets the number of
    cases (8 by default)."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    rs = np.random.default_rng(9000 + k)
    kind = rs.choice(["regular", "irregular", "qc"])
    if kind == "regular":
        dv, dc = [(3, 6), (2, 4), (4, 8)][rs.integers(3)]
        m = int(rs.integers(4, 40)) * dv
        H = wl.regular_ldpc(m * dc // dv, m, dv, dc, seed=int(rs.integers(1 << 30)))
    elif kind == "irregular":
        n = int(rs.integers(20, 400))
        m = int(rs.integers(n // 6 + 2, n // 2 + 3))
        H = None
        for cap in (12, 16, 40):
            try:
                H = wl.random_irregular_code(n, m, seed=int(rs.integers(1 << 30)), dv_choices=(1, 2, 3, 4, 6),
                                             max_row_degree=cap)
                break
            except RuntimeError:
                continue
        if H is None:
            pytest.skip("no code of this shape")
    else:
        Z = int(rs.choice([8, 16, 24]))
        H = wl.qc_irregular_ldpc(12, 6, Z, [2] * 6 + [3] * 4 + [6] * 2, seed=int(rs.integers(1 << 30)))
    C = oracle.check_degrees(H).size
    if C > 8:
        pytest.skip("more than 8 degree classes (the training kernels' limit)")
    T = int(rs.integers(1, 13))
    K = int(rs.choice([1, 2, 3, T]))
    B = int(rs.integers(1, 41))
    a = rs.uniform(0.5, 1.1, size=(T, C)).astype(np.float32)
    b = rs.uniform(0.0, 0.4, size=(T, C)).astype(np.float32)
    llr = wl.bpsk_awgn_llr(None, float(rs.uniform(0.5, 3.5)), max(0.1, 1 - H.shape[0] / H.shape[1]),
                           seed=int(rs.integers(1 << 30)), n=H.shape[1], batch=B)
    note(f"[nms-grad random {k}] {kind} m={H.shape[0]} n={H.shape[1]} T={T} K={K} B={B}")
    g = _graph(torch, dev, H)
    at, bt, lt = (torch.from_numpy(x).to(dev) for x in (a, b, llr))
    ws = torch.empty(ldpc.train_workspace_bytes(g, B, T, K), dtype=torch.uint8, device=dev)
    loss, post = ldpc.nms_train_forward(g, lt, at, bt, K, ws, want_post=True)
    ga, gb, gl = ldpc.nms_train_backward(g, lt, at, bt, K, ws, want_llr_grad=True)
    torch.cuda.synchronize()
    ref = oracle.nms_train_grad_f32_forward(H, llr, a, b, llr_grad=True)
    assert np.array_equal(post.cpu().numpy().astype(np.float64), ref["post"])
    assert abs(float(loss) - ref["loss"]) <= 2e-5 * abs(ref["loss"])
    assert_grad_parity(H, T, B, {"galpha": ga.cpu().numpy(), "gbeta": gb.cpu().numpy(), "gllr": gl.cpu().numpy()},
                       ref, f"random {k}")
