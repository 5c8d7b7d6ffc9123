"""FP64 oracle of the learned decoder's training loss and gradient (no GPU):
pinned by finite differences and by the FP32 decoding oracle."""
import numpy as np
import pytest

import oracle
from paper_2507_10424_amd import workloads as wl


def _softplus(z):
    return np.logaddexp(0.0, z)


@pytest.mark.parametrize("case", range(4))
def test_gradient_matches_finite_differences(case):
    rng = np.random.default_rng(40 + case)
    if case == 0:
        H = wl.paper_tanner_example()
    elif case == 1:
        H = wl.regular_ldpc(24, 12, 3, 6, seed=3)
    elif case == 2:
        H = wl.random_irregular_code(30, 12, seed=4, dv_choices=(1, 2, 3), max_row_degree=8)
    else:
        H = wl.tree_code(5, seed=7)
    C = oracle.check_degrees(H).size
    n = H.shape[1]
    T = 4
    llr = rng.normal(0.6, 1.3, size=(3, n))
    tg = (rng.random((3, n)) < 0.2).astype(np.uint8) if case == 1 else None
    alpha = rng.uniform(0.6, 1.1, size=(T, C))
    beta = rng.uniform(0.0, 0.3, size=(T, C))
    loss, ga, gb, gl = oracle.nms_train_loss_grad(H, llr, alpha, beta, targets=tg, llr_grad=True)
    h = 1e-6

    def L(a=alpha, b=beta, r=llr):
        return oracle.nms_train_loss_grad(H, r, a, b, targets=tg, grad=False)[0]

    for name, arr, g in [("alpha", alpha, ga), ("beta", beta, gb), ("llr", llr, gl)]:
        for idx in np.ndindex(arr.shape):
            p, q = arr.copy(), arr.copy()
            p[idx] += h
            q[idx] -= h
            kw = {"alpha": dict(a=p), "beta": dict(b=p), "llr": dict(r=p)}[name]
            kq = {"alpha": dict(a=q), "beta": dict(b=q), "llr": dict(r=q)}[name]
            fd = (L(**kw) - L(**kq)) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 + 1e-5 * abs(fd), (name, idx, fd, g[idx])


def test_forward_matches_decoding_oracle():
    """With alpha = 1, beta = 0 the FP64 loss equals the loss computed from
    the FP32 decoding oracle's posteriors after 1..T iterations (up to FP32
    rounding)."""
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    llr = wl.bpsk_awgn_llr(None, 1.5, 0.5, seed=9, n=96, batch=16)
    T = 6
    loss64, _, _, _ = oracle.nms_train_loss_grad(H, llr.astype(np.float64), np.ones((T, 1)), np.zeros((T, 1)),
                                                 grad=False)
    total = 0.0
    for t in range(1, T + 1):
        _, post, _, _ = oracle.minsum_decode(H, llr, t, early_exit=False)
        total += _softplus(-post.astype(np.float64)).sum()
    loss32 = total / llr.size
    assert abs(loss64 - loss32) <= 1e-5 * abs(loss64)


def test_zero_offset_large_scale_is_plain_shape():
    """Gradients vanish for beta where every message is clipped to zero, and
    the loss is then that of r alone in every iteration."""
    H = wl.paper_tanner_example()
    llr = np.random.default_rng(3).normal(1.0, 1.0, size=(2, 10))
    T = 3
    alpha = np.ones((T, 1))
    beta = np.full((T, 1), 1e6)  # max(alpha mu - beta, 0) = 0 everywhere
    loss, ga, gb, _ = oracle.nms_train_loss_grad(H, llr, alpha, beta)
    assert np.all(ga == 0) and np.all(gb == 0)
    assert abs(loss - T * _softplus(-llr).sum() / llr.size) < 1e-12


def _codes():
    return [wl.regular_ldpc(96, 48, 3, 6, seed=1),
            wl.random_irregular_code(120, 50, seed=11, dv_choices=(1, 2, 3, 4), max_row_degree=12),
            wl.paper_tanner_example()]


@pytest.mark.parametrize("ci", range(3))
def test_f32_forward_equals_decoding_oracle(ci):
    """The binary32 forward of the gradient oracle is the decoding oracle's
    learned decoder without early exit: posteriors after T iterations agree
    bit for bit, and its loss is the loss of the FP64 forward up to binary32
    rounding."""
    H = _codes()[ci]
    C = oracle.check_degrees(H).size
    n = H.shape[1]
    rng = np.random.default_rng(60 + ci)
    T = 7
    a = rng.uniform(0.6, 1.05, size=(T, C)).astype(np.float32)
    b = rng.uniform(0.0, 0.3, size=(T, C)).astype(np.float32)
    llr = wl.bpsk_awgn_llr(None, 1.5, 1 - H.shape[0] / n, seed=70 + ci, n=n, batch=24)
    got = oracle.nms_train_grad_f32_forward(H, llr, a, b)
    _, post, _, _ = oracle.nms_decode(H, llr, T, a, b, early_exit=False)
    assert np.array_equal(got["post"].astype(np.float32), post)
    assert np.array_equal(got["post"], post.astype(np.float64))  # exactly representable
    ref, _, _, _ = oracle.nms_train_loss_grad(H, llr.astype(np.float64), a.astype(np.float64), b.astype(np.float64),
                                              grad=False)
    assert abs(got["loss"] - ref) <= 1e-5 * abs(ref)


def test_f32_forward_gradient_equals_fp64_on_exact_inputs():
    """Dyadic LLRs and weights (few significant bits, small exponents) make
    every binary32 operation of the forward exact, so the binary32 forward
    and the FP64 forward take identical values and decisions, and the two
    gradients must agree to the last bit."""
    rng = np.random.default_rng(81)
    for H in _codes():
        C = oracle.check_degrees(H).size
        n = H.shape[1]
        T = 5
        llr = rng.integers(-24, 25, size=(6, n)).astype(np.float64) / 8.0
        a = rng.choice([0.5, 0.75, 0.875, 1.0], size=(T, C))
        b = rng.choice([0.0, 0.125, 0.25], size=(T, C))
        got = oracle.nms_train_grad_f32_forward(H, llr, a, b)
        _, ga, gb, gl = oracle.nms_train_loss_grad(H, llr, a, b, llr_grad=True)
        assert np.array_equal(got["galpha"], ga) and np.array_equal(got["gbeta"], gb)
        assert np.array_equal(got["gllr"], gl)


def test_f32_forward_gradient_close_to_fp64_and_bounded():
    """On Gaussian inputs the gradient along the binary32 forward is the
    gradient of the same objective: it matches the FP64 one closely on almost
    every entry (only entries behind a binary32 / FP64 tie difference can
    differ), and the magnitude bound dominates every entry."""
    H = _codes()[0]
    T = 10
    a, b = (np.random.default_rng(5).uniform(lo, hi, size=(T, 1)).astype(np.float32)
            for lo, hi in ((0.6, 1.05), (0.0, 0.3)))
    llr = wl.bpsk_awgn_llr(None, 2.0, 0.5, seed=4, n=96, batch=16)
    got = oracle.nms_train_grad_f32_forward(H, llr, a, b)
    _, ga, gb, gl = oracle.nms_train_loss_grad(H, llr.astype(np.float64), a.astype(np.float64),
                                               b.astype(np.float64), llr_grad=True)
    for g32, g64, bound in ((got["galpha"], ga, got["aalpha"]), (got["gbeta"], gb, got["abeta"]),
                            (got["gllr"], gl, got["allr"])):
        assert np.all(np.abs(g32) <= bound * (1 + 1e-12))
        rel = np.abs(g32 - g64) / (np.abs(g64) + 1e-300)
        assert np.median(rel) < 1e-5
        assert np.mean(np.abs(g32 - g64) <= 1e-4 * bound) >= 0.95
