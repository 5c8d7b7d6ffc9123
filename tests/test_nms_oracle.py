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
