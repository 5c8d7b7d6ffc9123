"""Seeded synthetic inputs for Min-Sum decoding: parity matrices, codewords and
channel LLRs.

This module is shared by the tests, the benchmark and the smoke check.  It
holds none of the decoder's arithmetic: it builds Tanner graphs, draws
codewords and adds BPSK/AWGN noise.  Both the CPU oracle and the HIP path take
what it returns as plain inputs.

Conventions
-----------
* H is a dense ``uint8`` array of shape (m, n) holding 0/1 (the paper keeps H
  as an m x n binary matrix whose rows are single parity checks, Sec. II-A).
* LLR polarity: a positive LLR favours bit 0.  BPSK maps bit c to x = 1 - 2c,
  y = x + sigma * N(0, 1), and the channel LLR is 2 y / sigma^2.
* Eb/N0 is in dB and sigma^2 = 1 / (2 R 10^(EbN0/10)) with the design rate
  R = 1 - m / n.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "regular_ldpc", "qc_irregular_ldpc", "qc_multi_code_family", "gf2_encoder",
    "sigma_for_ebn0", "bpsk_awgn_llr", "tree_code", "chain_code",
    "paper_tanner_example", "paper_spc_example", "dense_from_edges",
    "random_irregular_code",
]


# --------------------------------------------------------------------------
# Tanner graphs
# --------------------------------------------------------------------------

def dense_from_edges(m: int, n: int, rows, cols) -> np.ndarray:
    H = np.zeros((m, n), dtype=np.uint8)
    H[np.asarray(rows, dtype=np.int64), np.asarray(cols, dtype=np.int64)] = 1
    return H


def _socket_graph(bit_deg: np.ndarray, chk_deg: np.ndarray, rng) -> tuple:
    """Random bipartite multigraph by one shuffle of bit sockets against check
    sockets, then seeded swaps until no (check, bit) pair repeats."""
    E = int(bit_deg.sum())
    assert E == int(chk_deg.sum()), "edge counts of the two sides differ"
    bit_of = np.repeat(np.arange(bit_deg.size), bit_deg)
    chk_of = np.repeat(np.arange(chk_deg.size), chk_deg)
    perm = rng.permutation(E)
    bits = bit_of[perm]
    nb = bit_deg.size

    def key(k):
        return int(chk_of[k]) * nb + int(bits[k])

    for _sweep in range(1000):
        keys = chk_of.astype(np.int64) * nb + bits
        order = np.argsort(keys, kind="stable")
        ks = keys[order]
        dup = order[1:][ks[1:] == ks[:-1]]
        if dup.size == 0:
            return chk_of.copy(), bits.copy()
        present = set(keys.tolist())
        for k in dup.tolist():
            for _try in range(1000):
                k2 = int(rng.integers(E))
                a_new = int(chk_of[k]) * nb + int(bits[k2])
                b_new = int(chk_of[k2]) * nb + int(bits[k])
                if k2 == k or a_new in present or b_new in present or a_new == b_new:
                    continue
                present.discard(key(k))
                present.discard(key(k2))
                bits[k], bits[k2] = bits[k2], bits[k]
                present.add(key(k))
                present.add(key(k2))
                break
    raise RuntimeError("could not remove double edges")


def regular_ldpc(n: int, m: int, dv: int = 3, dc: int = 6, seed: int = 1) -> np.ndarray:
    """Gallager-style (dv, dc)-regular H by edge-socket permutation, with no
    double edges.  Returns a dense (m, n) uint8 matrix."""
    if n * dv != m * dc:
        raise ValueError("n*dv must equal m*dc")
    rng = np.random.default_rng(seed)
    chk, bit = _socket_graph(np.full(n, dv), np.full(m, dc), rng)
    return dense_from_edges(m, n, chk, bit)


def random_irregular_code(n: int, m: int, seed: int, dv_choices=(1, 2, 3, 4, 5),
                          min_row_degree: int = 2, max_row_degree: int = 40) -> np.ndarray:
    """Irregular random H for stress tests: column degrees drawn from
    ``dv_choices`` (0 allowed), row degrees as equal as the total permits but
    randomly perturbed, every row of degree >= ``min_row_degree``."""
    rng = np.random.default_rng(seed)
    for _attempt in range(100):
        dv = rng.choice(np.asarray(dv_choices), size=n)
        dv = np.minimum(dv, m)
        E = int(dv.sum())
        if E < min_row_degree * m:
            continue
        # as equal as possible, then random unit moves between rows
        cap = min(max_row_degree, n)
        if E > cap * m:
            continue
        dc = np.full(m, E // m)
        dc[: E - dc.sum()] += 1
        for _ in range(2 * m):
            a, b = rng.integers(m, size=2)
            if dc[a] > min_row_degree and dc[b] < cap:
                dc[a] -= 1
                dc[b] += 1
        try:
            chk, bit = _socket_graph(dv, dc, rng)
        except RuntimeError:
            continue
        return dense_from_edges(m, n, chk, bit)
    raise RuntimeError("could not draw an irregular code")


def _qc_base(n_base_cols: int, m_base: int, col_degrees: np.ndarray, rng) -> tuple:
    """Base graph for a quasi-cyclic code: column degrees as given, row
    degrees as equal as possible, no double edges."""
    E = int(col_degrees.sum())
    row_deg = np.full(m_base, E // m_base)
    row_deg[: E - row_deg.sum()] += 1
    rng_rows = rng.permutation(m_base)
    row_deg = row_deg[rng_rows]
    return _socket_graph(col_degrees, row_deg, rng)


def qc_irregular_ldpc(n_base_cols: int, m_base: int, Z: int, col_degrees, seed: int,
                      dense: bool = True):
    """Quasi-cyclic H lifted from a random base graph: each base edge (R, C)
    with a random shift p in [0, Z) becomes the Z x Z circulant that joins row
    R*Z + r to column C*Z + (r + p) mod Z.

    Returns the dense (m_base*Z, n_base_cols*Z) matrix, or (m, n, rows, cols)
    when ``dense`` is False."""
    col_degrees = np.asarray(col_degrees, dtype=np.int64)
    assert col_degrees.size == n_base_cols
    rng = np.random.default_rng(seed)
    chk, bit = _qc_base(n_base_cols, m_base, col_degrees, rng)
    shifts = rng.integers(0, Z, size=chk.size)
    r = np.arange(Z)
    rows = (chk[:, None] * Z + r[None, :]).reshape(-1)
    cols = (bit[:, None] * Z + (r[None, :] + shifts[:, None]) % Z).reshape(-1)
    m, n = m_base * Z, n_base_cols * Z
    if not dense:
        return m, n, rows, cols
    return dense_from_edges(m, n, rows, cols)


def large_qc_code(seed: int = 5, dense: bool = True):
    """Rate-1/2 irregular QC code with n = 64800, m = 32400, Z = 360: 180 base
    columns with bit degrees 8/3/2 on 20/30/50 % of them and 90 base rows of
    degree 7 (630 base edges)."""
    cd = np.concatenate([np.full(36, 8), np.full(54, 3), np.full(90, 2)])
    rng = np.random.default_rng(seed)
    cd = cd[rng.permutation(cd.size)]
    return qc_irregular_ldpc(180, 90, 360, cd, seed=seed + 1000, dense=dense)


def qc_multi_code_family(seed: int = 7):
    """Eight irregular QC codes of 24 base columns, Z in {24, 48, 72, 96},
    rates {1/2, 2/3, 3/4, 5/6}, bit degrees 2/3/6 on 12/8/4 base columns
    (degree 6 is capped at the number of base rows).  Returns a list of dicts
    with keys H, n, m, Z, rate, batch."""
    specs = [(24, 0.5, 16384), (24, 5 / 6, 512), (48, 2 / 3, 8192), (48, 0.75, 1024),
             (72, 0.5, 4096), (72, 0.75, 2048), (96, 2 / 3, 6144), (96, 5 / 6, 3072)]
    out = []
    for k, (Z, R, batch) in enumerate(specs):
        mb = int(round(24 * (1 - R)))
        cd = np.concatenate([np.full(12, 2), np.full(8, 3), np.full(4, min(6, mb))])
        rng = np.random.default_rng(seed * 100 + k)
        cd = cd[rng.permutation(cd.size)]
        H = qc_irregular_ldpc(24, mb, Z, cd, seed=seed * 100 + k + 50)
        out.append(dict(H=H, n=24 * Z, m=mb * Z, Z=Z, rate=R, batch=batch))
    return out


def tree_code(n_checks: int, seed: int, max_check_degree: int = 4, max_bits: int = 16):
    """Random cycle-free Tanner graph: every new check joins one existing bit
    and 1..max_check_degree-1 new bits, so every check has degree >= 2 and the
    graph is a tree.  Returns a dense H (m, n)."""
    rng = np.random.default_rng(seed)
    n = 1
    rows, cols = [], []
    for i in range(n_checks):
        room = max_bits - n
        if room < 1:
            break
        new = int(rng.integers(1, min(max_check_degree - 1, room) + 1))
        parent = int(rng.integers(n))
        members = [parent] + list(range(n, n + new))
        n += new
        for j in members:
            rows.append(i)
            cols.append(j)
    m = max(rows) + 1
    # shuffle column order so bit indices are not sorted by depth
    perm = rng.permutation(n)
    cols = [int(perm[c]) for c in cols]
    return dense_from_edges(m, n, rows, cols)


def chain_code(n: int) -> np.ndarray:
    """Repetition code of length n as the chain of checks b_j + b_{j+1} = 0."""
    H = np.zeros((n - 1, n), dtype=np.uint8)
    for j in range(n - 1):
        H[j, j] = H[j, j + 1] = 1
    return H


def paper_tanner_example() -> np.ndarray:
    """The 5 x 10 Tanner graph of Sec. II-A, read from its index sets
    I_1..I_5 (1-based bit indices)."""
    sets = [(1, 2, 3, 6, 7, 10), (1, 3, 5, 6, 8, 9), (3, 4, 5, 7, 9, 10),
            (2, 4, 5, 6, 8, 10), (1, 2, 4, 7, 8, 9)]
    H = np.zeros((5, 10), dtype=np.uint8)
    for i, s in enumerate(sets):
        for j in s:
            H[i, j - 1] = 1
    return H


def paper_spc_example() -> np.ndarray:
    """The single parity check of Sec. II-A: k = 6, I = {1, 2, 4, 5}."""
    return np.array([[1, 1, 0, 1, 1, 0]], dtype=np.uint8)


# --------------------------------------------------------------------------
# Encoding over GF(2)
# --------------------------------------------------------------------------

class gf2_encoder:
    """Systematic encoder from the reduced row echelon form of H over GF(2):
    information bits sit on the free (non-pivot) columns and each pivot
    column's bit is the XOR of the free bits its RREF row selects."""

    def __init__(self, H: np.ndarray):
        R = (np.asarray(H, dtype=np.uint8) & 1).copy()
        m, n = R.shape
        pivots = []
        row = 0
        for col in range(n):
            if row >= m:
                break
            nz = np.nonzero(R[row:, col])[0]
            if nz.size == 0:
                continue
            p = row + int(nz[0])
            if p != row:
                R[[row, p]] = R[[p, row]]
            hit = np.nonzero(R[:, col])[0]
            hit = hit[hit != row]
            if hit.size:
                R[hit] ^= R[row]
            pivots.append(col)
            row += 1
        self.rank = row
        self.n = n
        self.pivots = np.asarray(pivots, dtype=np.int64)
        mask = np.ones(n, dtype=bool)
        mask[self.pivots] = False
        self.free = np.nonzero(mask)[0]
        self.k = self.free.size
        # parity rows restricted to the free columns: (rank, k)
        self._P = R[: self.rank][:, self.free].astype(np.float32)

    def encode(self, info: np.ndarray) -> np.ndarray:
        """info: (B, k) 0/1 -> codewords (B, n) uint8."""
        info = np.asarray(info, dtype=np.uint8)
        B = info.shape[0]
        c = np.zeros((B, self.n), dtype=np.uint8)
        c[:, self.free] = info
        # float32 matmul is exact here: sums of at most k ones < 2^24
        step = 8192
        for b0 in range(0, B, step):
            par = info[b0:b0 + step].astype(np.float32) @ self._P.T
            c[b0:b0 + step][:, self.pivots] = (par.astype(np.int64) & 1).astype(np.uint8)
        return c

    def random_codewords_torch(self, B: int, seed: int, device):
        """Random codewords generated on ``device`` with torch (seeded
        Philox on a GPU): (B, n) uint8 tensor."""
        import torch
        gen = torch.Generator(device=device)
        gen.manual_seed(int(seed))
        info = torch.randint(0, 2, (B, self.k), generator=gen, device=device, dtype=torch.uint8)
        P = torch.from_numpy(self._P.astype(np.float64)).to(device)
        free = torch.from_numpy(self.free).to(device)
        piv = torch.from_numpy(self.pivots).to(device)
        c = torch.zeros((B, self.n), dtype=torch.uint8, device=device)
        c[:, free] = info
        step = 16384
        for b0 in range(0, B, step):
            par = info[b0:b0 + step].to(torch.float64) @ P.T  # exact: integer sums < 2^53
            c[b0:b0 + step, piv] = torch.remainder(par, 2.0).to(torch.uint8)
        return c

    def random_codewords(self, B: int, seed: int) -> np.ndarray:
        rng = np.random.default_rng(seed)
        info = rng.integers(0, 2, size=(B, self.k), dtype=np.uint8)
        return self.encode(info)


# --------------------------------------------------------------------------
# Channel
# --------------------------------------------------------------------------

def bpsk_awgn_llr_torch(codewords, ebn0_db: float, rate: float, seed: int, device, n: int | None = None,
                        batch: int | None = None):
    """Channel LLRs generated on ``device`` with torch (seeded Philox
    normals): float32 (B, n) tensor.  ``codewords=None`` with ``batch``, ``n``
    gives the all-zero codeword."""
    import torch
    sigma = sigma_for_ebn0(ebn0_db, rate)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    shape = (batch, n) if codewords is None else tuple(codewords.shape)
    noise = torch.randn(shape, generator=gen, device=device, dtype=torch.float32)
    x = 1.0 if codewords is None else 1.0 - 2.0 * codewords.to(torch.float32)
    return ((x + sigma * noise) * (2.0 / (sigma * sigma))).to(torch.float32).contiguous()


def sigma_for_ebn0(ebn0_db: float, rate: float) -> float:
    return float(np.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))))


def bpsk_awgn_llr(codewords: np.ndarray, ebn0_db: float, rate: float, seed: int,
                  n: int | None = None, batch: int | None = None) -> np.ndarray:
    """Channel LLRs (float32, shape (B, n)) for BPSK over AWGN.  Pass
    ``codewords=None`` with ``batch`` and ``n`` for the all-zero codeword."""
    sigma = sigma_for_ebn0(ebn0_db, rate)
    rng = np.random.default_rng(seed)
    if codewords is None:
        shape = (batch, n)
        x = 1.0
    else:
        shape = codewords.shape
        x = 1.0 - 2.0 * codewords.astype(np.float64)
    out = np.empty(shape, dtype=np.float32)
    rows = max(1, (1 << 22) // max(1, shape[1]))
    for b0 in range(0, shape[0], rows):
        b1 = min(shape[0], b0 + rows)
        noise = rng.standard_normal((b1 - b0, shape[1]))
        xv = x if np.isscalar(x) else x[b0:b1]
        out[b0:b1] = (2.0 * (xv + sigma * noise) / (sigma * sigma)).astype(np.float32)
    return out
