"""Pins of the CPU oracle: checks against facts that the paper and the
mathematics fix, independent of the oracle's own code.

Each ``pin_*`` takes an oracle object and raises AssertionError when the
oracle disagrees with the fact it pins.  The pins are also run against copies
of the oracle with planted mistakes (see test_oracle_pins.py) to show that
each plausible mistake fails at least one of them.
"""
from __future__ import annotations

import itertools
import os

import numpy as np

from paper_2507_10424_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------------------
# helpers: brute force over GF(2), independent of the oracle
# ---------------------------------------------------------------------------

def codebook(H: np.ndarray) -> np.ndarray:
    """All codewords of H by enumeration of {0,1}^n (n <= 20)."""
    m, n = H.shape
    assert n <= 20
    idx = np.arange(1 << n, dtype=np.int64)
    words = ((idx[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    syn = (words @ H.T.astype(np.int64)) & 1
    return words[np.all(syn == 0, axis=1)].astype(np.uint8)


def max_marginals(H: np.ndarray, r: np.ndarray, book: np.ndarray | None = None):
    """Exhaustive max-log decoding: the best codeword and, per bit, the
    difference between the best correlation with the bit at 0 and at 1.
    With LLR r_j = log p(y|0)/p(y|1), the log-likelihood of c is
    sum_j (1 - 2 c_j) r_j / 2 up to a constant."""
    book = codebook(H) if book is None else book
    score = (1.0 - 2.0 * book.astype(np.float64)) @ r.astype(np.float64) / 2.0
    best = book[int(np.argmax(score))]
    n = H.shape[1]
    mm = np.empty(n)
    for j in range(n):
        z = score[book[:, j] == 0]
        o = score[book[:, j] == 1]
        mm[j] = (z.max() if z.size else -np.inf) - (o.max() if o.size else -np.inf)
    return best, mm


def read_tanner_golden():
    sets, vecs = [], []
    with open(os.path.join(GOLDEN, "paper_tanner_5x10.txt")) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            lhs, rhs = line.split(":", 1)[1].split("|")
            sets.append([int(v) for v in lhs.split()])
            vecs.append([int(v) for v in rhs.split()])
    return sets, vecs


def read_spc_golden():
    d = {}
    with open(os.path.join(GOLDEN, "paper_spc_k6.txt")) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            k, v = line.split(":")
            d[k.strip()] = [int(x) for x in v.split()]
    return d


def wagner(r: np.ndarray) -> np.ndarray:
    """Textbook ML decoder of a single parity check: hard decisions, and if
    their parity is odd, flip the least reliable bit."""
    b = (r < 0).astype(np.uint8)
    if b.sum() % 2:
        j = int(np.argmin(np.abs(r)))
        b[j] ^= 1
    return b


# ---------------------------------------------------------------------------
# pins
# ---------------------------------------------------------------------------

def pin_codewords_stop_at_iteration0(orc):
    """A noiseless codeword at any positive scale is already a codeword:
    0 iterations, the codeword back, the LLRs untouched (paper example)."""
    H = wl.paper_tanner_example()
    book = codebook(H)
    assert book.shape[0] == 32
    for kappa in (0.5, 1.0, 3.75):
        r = (kappa * (1.0 - 2.0 * book.astype(np.float32))).astype(np.float32)
        bits, post, iters, ok = orc.minsum_decode(H, r, 20)
        assert np.array_equal(bits, book)
        assert np.array_equal(post, r)
        assert np.all(iters == 0) and np.all(ok == 1)


def pin_max_iter_zero(orc):
    """L = 0: the channel decision, the channel LLRs, 0 iterations and ok
    equal to codebook membership of the channel decision."""
    H = wl.paper_tanner_example()
    book = {tuple(c) for c in codebook(H)}
    rng = np.random.default_rng(11)
    r = rng.normal(1.0, 1.2, size=(64, 10)).astype(np.float32)
    r[:8] = (1.0 - 2.0 * np.array(sorted(book)[:8], dtype=np.float32)) * 2.0
    bits, post, iters, ok = orc.minsum_decode(H, r, 0)
    assert np.array_equal(bits, (r < 0).astype(np.uint8))
    assert np.array_equal(post, r)
    assert np.all(iters == 0)
    want = np.array([tuple(b) in book for b in (r < 0).astype(np.uint8)], dtype=np.uint8)
    assert np.array_equal(ok, want)
    assert ok[:8].all()


def pin_single_check_wagner(orc):
    """A single parity check of degree d: Min-Sum decides as the Wagner rule
    and stops after 0 iterations (even parity) or 1 (odd parity)."""
    rng = np.random.default_rng(12)
    for d in range(2, 13):
        H = np.ones((1, d), dtype=np.uint8)
        r = rng.normal(0.3, 1.5, size=(40, d)).astype(np.float32)
        bits, post, iters, ok = orc.minsum_decode(H, r, 5)
        for f in range(r.shape[0]):
            assert np.array_equal(bits[f], wagner(r[f])), (d, f)
            even = int((r[f] < 0).sum()) % 2 == 0
            assert iters[f] == (0 if even else 1), (d, f, iters[f])
            assert ok[f] == 1


def pin_paper_spc_example(orc):
    """The paper's SPC (k = 6, I = {1,2,4,5}): bits outside I carry no check
    and keep s = r; bits in I follow the Wagner rule."""
    g = read_spc_golden()
    H = np.array([g["indicator"]], dtype=np.uint8)
    idx = np.array(g["index_set"]) - 1
    free = np.setdiff1d(np.arange(g["k"][0]), idx)
    rng = np.random.default_rng(13)
    r = rng.normal(0.5, 1.5, size=(50, 6)).astype(np.float32)
    bits, post, iters, ok = orc.minsum_decode(H, r, 3, early_exit=False)
    assert np.array_equal(post[:, free], r[:, free])
    for f in range(r.shape[0]):
        assert np.array_equal(bits[f, idx], wagner(r[f, idx]))
    assert np.all(ok == 1) and np.all(iters == 3)


def pin_single_check_closed_form(orc):
    """One iteration on a single check of degree d: the message to bit j is
    the product of the other signs times the smallest other magnitude, and
    the posterior is r_j plus that message."""
    rng = np.random.default_rng(14)
    for d in (2, 3, 5, 8, 17, 32):
        H = np.ones((1, d), dtype=np.uint8)
        r = rng.normal(0.0, 2.0, size=(20, d)).astype(np.float32)
        _, post, iters, _ = orc.minsum_decode(H, r, 1, early_exit=False)
        assert np.all(iters == 1)
        for f in range(r.shape[0]):
            for j in range(d):
                others = np.delete(r[f], j)
                msg = np.float32(np.prod(np.where(others < 0, -1.0, 1.0)) * np.abs(others).min())
                assert post[f, j] == np.float32(r[f, j] + msg), (d, f, j)


def pin_trees_equal_max_marginals(orc):
    """Cycle-free codes: after enough iterations Min-Sum is exact max-log
    decoding, so the posterior is the exhaustive max-marginal LLR and the
    decision is the best codeword."""
    checked = 0
    for seed in range(60):
        H = wl.tree_code(n_checks=int(2 + seed % 6), seed=1000 + seed, max_check_degree=2 + seed % 4,
                         max_bits=16)
        m, n = H.shape
        rng = np.random.default_rng(2000 + seed)
        r = rng.normal(0.5, 1.5, size=(6, n)).astype(np.float32)
        bits, post, iters, ok = orc.minsum_decode(H, r, n + m, early_exit=False)
        book = codebook(H)
        for f in range(r.shape[0]):
            best, mm = max_marginals(H, r[f], book)
            tol = 1e-5 * float(np.abs(r[f]).sum())
            assert np.max(np.abs(post[f].astype(np.float64) - mm)) <= tol, (seed, f)
            if np.min(np.abs(mm)) > tol:
                assert np.array_equal(bits[f], best), (seed, f)
                assert ok[f] == 1
            checked += 1
    assert checked >= 300


def pin_repetition_chain(orc):
    """Repetition code as a chain of 2-bit checks: every converged posterior
    is the sum of all channel LLRs."""
    rng = np.random.default_rng(15)
    for n in (2, 3, 7, 12):
        H = wl.chain_code(n)
        r = rng.normal(0.2, 1.0, size=(10, n)).astype(np.float32)
        _, post, _, _ = orc.minsum_decode(H, r, 2 * n, early_exit=False)
        total = r.astype(np.float64).sum(axis=1, keepdims=True)
        tol = 1e-5 * np.abs(r).sum(axis=1, keepdims=True)
        assert np.all(np.abs(post - total) <= tol), n


def pin_codeword_symmetry(orc):
    """Min-Sum commutes with flipping the signs of a codeword's bits:
    decode(r * (1-2c)) = (bits xor c, same iterations, post * (1-2c))."""
    H96 = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    enc = wl.gf2_encoder(H96)
    cases = [(wl.paper_tanner_example(), codebook(wl.paper_tanner_example())),
             (H96, enc.random_codewords(12, seed=3))]
    rng = np.random.default_rng(16)
    for H, cws in cases:
        n = H.shape[1]
        r = rng.normal(1.0, 1.0, size=(cws.shape[0], n)).astype(np.float32)
        flip = (1.0 - 2.0 * cws.astype(np.float32))
        b0, p0, i0, o0 = orc.minsum_decode(H, r, 25)
        b1, p1, i1, o1 = orc.minsum_decode(H, r * flip, 25)
        assert np.array_equal(b1, b0 ^ cws)
        assert np.array_equal(i1, i0) and np.array_equal(o1, o0)
        nz = p0 != 0
        assert np.array_equal((p1 * flip)[nz], p0[nz])


def pin_power_of_two_scaling(orc):
    """Plain Min-Sum is homogeneous: scaling the LLRs by 2^k scales every
    message by 2^k exactly, so decisions and iterations are unchanged."""
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    r = wl.bpsk_awgn_llr(None, 1.5, 0.5, seed=17, n=96, batch=40)
    b0, p0, i0, o0 = orc.minsum_decode(H, r, 20)
    for k in (-3, 5):
        s = np.float32(2.0 ** k)
        b1, p1, i1, o1 = orc.minsum_decode(H, r * s, 20)
        assert np.array_equal(b1, b0) and np.array_equal(i1, i0) and np.array_equal(o1, o0)
        assert np.array_equal(p1, p0 * s)


def pin_dense_map_reduce_form(orc):
    """Algorithm 2 on dense masked matrices, with the min0/min1/argmin and
    total-sign reductions, reaches the same decisions, iterations and (up to
    the sign of zero) posteriors as the graph form."""
    rng = np.random.default_rng(18)
    codes = [wl.paper_tanner_example(), wl.regular_ldpc(24, 12, 3, 6, seed=4),
             wl.random_irregular_code(30, 14, seed=5, dv_choices=(0, 1, 2, 3, 4)),
             wl.tree_code(5, seed=6)]
    for H in codes:
        m, n = H.shape
        r = rng.normal(0.8, 1.3, size=(8, n)).astype(np.float32)
        r[0, :3] = 0.0
        r[1, :2] = -0.0
        bits, post, iters, ok = orc.minsum_decode(H, r, 12)
        for f in range(r.shape[0]):
            b, p, it, o = orc.minsum_dense(H, r[f], 12)
            assert np.array_equal(b, bits[f]) and it == iters[f] and o == ok[f]
            assert np.array_equal(p, post[f])  # == treats +0 and -0 as equal


def pin_no_early_exit_runs_L(orc):
    """Without early exit every frame runs L iterations; a noiseless codeword
    is a fixed point and ends as a codeword."""
    H = wl.paper_tanner_example()
    book = codebook(H)
    r = (2.0 * (1.0 - 2.0 * book.astype(np.float32))).astype(np.float32)
    bits, post, iters, ok = orc.minsum_decode(H, r, 7, early_exit=False)
    assert np.all(iters == 7) and np.all(ok == 1)
    assert np.array_equal(bits, book)


def pin_nms_unit_weights(orc):
    """Scale 1 and offset 0 in every iteration and degree class give plain
    Min-Sum back bit for bit."""
    H = wl.random_irregular_code(40, 20, seed=8, dv_choices=(1, 2, 3, 4))
    C = orc.check_degrees(H).size
    r = np.random.default_rng(19).normal(0.9, 1.2, size=(16, 40)).astype(np.float32)
    alpha = np.ones((10, C), np.float32)
    beta = np.zeros((10, C), np.float32)
    a = orc.minsum_decode(H, r, 10)
    b = orc.nms_decode(H, r, 10, alpha, beta)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def pin_nms_single_checks_closed_form(orc):
    """The learned check update on disjoint single checks of degrees 5, 3, 7
    and 3 (rows in that order, so a row's degree class -- the rank of its
    degree among the distinct row degrees, 3 < 5 < 7 -- differs from its row
    index).  On a single check the extrinsic input of every iteration is the
    channel LLR, so after t iterations (no early exit) the posterior is
    r_j + sign product of the other r times max(alpha[t-1][c] mu - beta[t-1][c], 0),
    mu the smallest other |r|.  Inputs and weights are multiples of 1/32 and
    1/4 of small size, so every step is exact in binary32 and the closed form
    is compared bit for bit.  Each (iteration, class) has its own weights,
    and some offsets exceed alpha mu, where the message is zero."""
    degs = (5, 3, 7, 3)
    n = sum(degs)
    H = np.zeros((len(degs), n), np.uint8)
    col = 0
    for i, d in enumerate(degs):
        H[i, col:col + d] = 1
        col += d
    classes = {3: 0, 5: 1, 7: 2}
    assert orc.check_degrees(H).tolist() == [3, 5, 7]
    rng = np.random.default_rng(23)
    T, C = 4, 3
    alpha = (rng.integers(1, 8, size=(T, C)) / 4.0).astype(np.float32)  # 0.25 .. 1.75
    beta = (rng.integers(0, 24, size=(T, C)) / 4.0).astype(np.float32)  # 0 .. 5.75
    assert len({(a, b) for a, b in zip(alpha.ravel(), beta.ravel())}) == T * C
    mag = rng.integers(1, 256, size=(24, n)) / 32.0  # 1/32 .. 8
    r = (np.where(rng.random((24, n)) < 0.4, -1.0, 1.0) * mag).astype(np.float32)
    zero_messages = 0
    for t in range(1, T + 1):
        bits, post, iters, _ = orc.nms_decode(H, r, t, alpha, beta, early_exit=False)
        assert np.all(iters == t)
        col = 0
        for i, d in enumerate(degs):
            c = classes[d]
            for j in range(col, col + d):
                others = np.delete(r[:, col:col + d], j - col, axis=1).astype(np.float64)
                sigma = np.prod(np.where(others < 0, -1.0, 1.0), axis=1)
                mu = np.abs(others).min(axis=1)
                v = np.maximum(float(alpha[t - 1, c]) * mu - float(beta[t - 1, c]), 0.0)
                zero_messages += int((v == 0).sum())
                want = (r[:, j].astype(np.float64) + sigma * v).astype(np.float32)
                assert np.array_equal(post[:, j], want), (t, i, j)
                assert np.array_equal(bits[:, j], (want < 0).astype(np.uint8)), (t, i, j)
            col += d
    assert zero_messages > 0


ALL_PINS = [
    pin_codewords_stop_at_iteration0,
    pin_max_iter_zero,
    pin_single_check_wagner,
    pin_paper_spc_example,
    pin_single_check_closed_form,
    pin_trees_equal_max_marginals,
    pin_repetition_chain,
    pin_codeword_symmetry,
    pin_power_of_two_scaling,
    pin_dense_map_reduce_form,
    pin_no_early_exit_runs_L,
    pin_nms_unit_weights,
    pin_nms_single_checks_closed_form,
]
