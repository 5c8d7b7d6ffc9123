"""Several codes decoded in one persistent launch (GPU): per-code parity with
the oracle and equality with one launch per code."""
import numpy as np
import pytest

from paper_2507_10424_amd import workloads as wl
from parity import assert_parity, note, oracle_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def test_eight_qc_codes_one_launch(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    fam = wl.qc_multi_code_family(seed=7)
    jobs, inputs = [], []
    for k, c in enumerate(fam):
        B = 96 + 37 * k  # uneven batches
        llr = wl.bpsk_awgn_llr(None, 2.0, c["rate"], seed=600 + k, n=c["n"], batch=B)
        g = ldpc.build_graph(torch.from_numpy(c["H"]).to(dev))
        jobs.append((g, torch.from_numpy(llr).to(dev)))
        inputs.append((c["H"], llr))
    outs = ldpc.minsum_decode_multi(jobs, 50)
    torch.cuda.synchronize()
    for k, ((H, llr), o, (g, lt)) in enumerate(zip(inputs, outs, jobs)):
        got = tuple(t.cpu().numpy() for t in o)
        note(f"[multi] code {k}: n={H.shape[1]} m={H.shape[0]} B={llr.shape[0]} mean iters {got[2].mean():.2f}")
        assert_parity(got, oracle_decode(H, llr, 50), f"multi code {k}")
        single = ldpc.minsum_decode(g, lt, 50)
        torch.cuda.synchronize()
        for x, y in zip(o, single):
            assert torch.equal(x, y)


def test_multi_mixed_sizes_and_empty_job(tdev):
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    codes = [wl.regular_ldpc(96, 48, 3, 6, seed=1), wl.regular_ldpc(1024, 512, 3, 6, seed=2),
             wl.random_irregular_code(300, 120, seed=3, dv_choices=(1, 2, 3, 4), max_row_degree=8)]
    Bs = [500, 0, 130]
    jobs, inputs = [], []
    for k, (H, B) in enumerate(zip(codes, Bs)):
        llr = np.random.default_rng(k).normal(1.1, 1.2, size=(B, H.shape[1])).astype(np.float32)
        g = ldpc.build_graph(torch.from_numpy(H).to(dev))
        jobs.append((g, torch.from_numpy(llr).to(dev)))
        inputs.append((H, llr))
    outs = ldpc.minsum_decode_multi(jobs, 30)
    torch.cuda.synchronize()
    for k, ((H, llr), o) in enumerate(zip(inputs, outs)):
        if llr.shape[0] == 0:
            continue
        assert_parity(tuple(t.cpu().numpy() for t in o), oracle_decode(H, llr, 30), f"mixed {k}")


def test_multi_with_wide_variant_job(tdev):
    """A code with bit degree above 8 needs the widest masked kernel variant,
    which runs in a launch of its own next to the shared multi-code launch."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    wide = wl.random_irregular_code(400, 160, seed=11, dv_choices=(2, 3, 12), max_row_degree=16)
    assert wide.sum(axis=0).max() > 8
    codes = [wl.regular_ldpc(96, 48, 3, 6, seed=1), wide, wl.regular_ldpc(1024, 512, 3, 6, seed=2)]
    Bs = [300, 257, 129]
    jobs, inputs = [], []
    for k, (H, B) in enumerate(zip(codes, Bs)):
        llr = np.random.default_rng(40 + k).normal(1.0, 1.3, size=(B, H.shape[1])).astype(np.float32)
        g = ldpc.build_graph(torch.from_numpy(H).to(dev))
        jobs.append((g, torch.from_numpy(llr).to(dev)))
        inputs.append((H, llr))
    outs = ldpc.minsum_decode_multi(jobs, 40)
    torch.cuda.synchronize()
    for k, ((H, llr), o, (g, lt)) in enumerate(zip(inputs, outs, jobs)):
        got = tuple(t.cpu().numpy() for t in o)
        note(f"[multi-wide] code {k}: n={H.shape[1]} B={llr.shape[0]} mean iters {got[2].mean():.2f}")
        assert_parity(got, oracle_decode(H, llr, 40), f"multi wide {k}")
        single = ldpc.minsum_decode(g, lt, 40)
        torch.cuda.synchronize()
        for x, y in zip(o, single):
            assert torch.equal(x, y)


def test_multi_big_job_runs_alone(tdev):
    """A batch large enough to fill the GPU on its own goes to a launch of its
    own kernel inside the same call; outputs are unchanged."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    codes = [wl.regular_ldpc(96, 48, 3, 6, seed=1), wl.regular_ldpc(1024, 512, 3, 6, seed=2),
             wl.random_irregular_code(300, 120, seed=3, dv_choices=(1, 2, 3, 4), max_row_degree=8)]
    Bs = [300, 10000, 130]  # the n = 1024 job fills the GPU alone
    jobs, inputs = [], []
    for k, (H, B) in enumerate(zip(codes, Bs)):
        llr = wl.bpsk_awgn_llr(None, 1.5, 0.5, seed=70 + k, n=H.shape[1], batch=B)
        g = ldpc.build_graph(torch.from_numpy(H).to(dev))
        jobs.append((g, torch.from_numpy(llr).to(dev)))
        inputs.append((H, llr))
    outs = ldpc.minsum_decode_multi(jobs, 30)
    torch.cuda.synchronize()
    for k, ((H, llr), o, (g, lt)) in enumerate(zip(inputs, outs, jobs)):
        single = ldpc.minsum_decode(g, lt, 30)
        torch.cuda.synchronize()
        for x, y in zip(o, single):
            assert torch.equal(x, y), f"job {k}"
        sel = slice(0, min(llr.shape[0], 3000))
        got = tuple(t[sel].cpu().numpy() for t in o)
        assert_parity(got, oracle_decode(H, llr[sel], 30), f"big/small {k}")


def test_multi_check_period_and_no_early_exit(tdev):
    """The multi-code call honours the codeword-test period and
    LDPC_NO_EARLY_EXIT like the single-code decode."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    fam = wl.qc_multi_code_family(seed=7)[:3]
    jobs, inputs = [], []
    for k, c in enumerate(fam):
        B = 150 + 50 * k
        llr = wl.bpsk_awgn_llr(None, 2.0, c["rate"], seed=800 + k, n=c["n"], batch=B)
        g = ldpc.build_graph(torch.from_numpy(c["H"]).to(dev))
        jobs.append((g, torch.from_numpy(llr).to(dev)))
        inputs.append((c["H"], llr))
    for flags in (ldpc.check_period(6), ldpc.LDPC_NO_EARLY_EXIT):
        outs = ldpc.minsum_decode_multi(jobs, 30, flags=flags)
        torch.cuda.synchronize()
        for k, ((H, llr), o) in enumerate(zip(inputs, outs)):
            assert_parity(tuple(t.cpu().numpy() for t in o), oracle_decode(H, llr, 30, flags), f"multi flags {flags} {k}")


def test_big_jobs_of_one_kernel_share_a_launch(tdev):
    """Jobs that each fill the GPU and use the same kernel run in one launch,
    one after another with no barrier between them (a workgroup starts the
    next job while others finish the last frames of the previous one): two
    (3,6) codes of different sizes, several batches each, plus a small job of
    a third code in the shared launch, all against the oracle, twice."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    Ha = wl.regular_ldpc(1024, 512, 3, 6, seed=2)
    Hb = wl.regular_ldpc(2048, 1024, 3, 6, seed=6)
    Hc = wl.random_irregular_code(120, 60, seed=5, dv_choices=(2, 3, 4))
    ga, gb, gc = (ldpc.build_graph(torch.from_numpy(H).to(dev)) for H in (Ha, Hb, Hc))
    spec = [(Ha, ga, 3000, 1.5), (Hb, gb, 1500, 2.0), (Ha, ga, 2600, 2.5), (Hc, gc, 77, 1.5), (Hb, gb, 1300, 1.0)]
    jobs, inputs, refs = [], [], []
    for k, (H, g, B, eb) in enumerate(spec):
        llr = wl.bpsk_awgn_llr(None, eb, 0.5, seed=900 + k, n=H.shape[1], batch=B)
        jobs.append((g, torch.from_numpy(llr).to(dev)))
        inputs.append((H, llr))
        refs.append(oracle_decode(H, llr, 40))
    import ctypes
    lib = ldpc.load_library()
    for rep in range(2):
        lib.ldpc_timing_enable(1)
        outs = ldpc.minsum_decode_multi(jobs, 40)
        torch.cuda.synchronize()
        ms, launches = ctypes.c_double(), ctypes.c_int64()
        assert lib.ldpc_timing_read(2, ctypes.byref(ms), ctypes.byref(launches)) == 0
        lib.ldpc_timing_enable(0)
        # one launch per graph for the big jobs, one shared launch for the small one
        assert launches.value == 3
        for k, o in enumerate(outs):
            assert_parity(tuple(t.cpu().numpy() for t in o), refs[k], f"shared launch job {k} rep {rep}")


def test_qc_family_configured_batches_one_call(tdev):
    """The eight QC codes at their configured batches (512 to 16,384 frames,
    41,472 in all) in one ldpc_minsum_decode_multi call, as the benchmark runs
    them: every output of a sample of each code's frames (its first and last
    frames and a seeded random draw) equals the oracle's."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    fam = wl.qc_multi_code_family(seed=7)
    jobs, inputs = [], []
    for k, c in enumerate(fam):
        llr = wl.bpsk_awgn_llr(None, 2.0, c["rate"], seed=300 + k, n=c["n"], batch=c["batch"])
        g = ldpc.build_graph(torch.from_numpy(c["H"]).to(dev))
        jobs.append((g, torch.from_numpy(llr).to(dev)))
        inputs.append((c["H"], llr))
    note(f"[multi] configured batches {[c['batch'] for c in fam]}")
    outs = ldpc.minsum_decode_multi(jobs, 50)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    for k, ((H, llr), o) in enumerate(zip(inputs, outs)):
        B = llr.shape[0]
        pick = np.unique(np.concatenate([np.arange(24), np.arange(B - 24, B), rng.choice(B, 48, replace=False)]))
        got = tuple(t.cpu().numpy()[pick] for t in o)
        note(f"[multi] code {k}: n={H.shape[1]} B={B}, {pick.size} frames checked, mean iters {got[2].mean():.2f}")
        assert_parity(got, oracle_decode(H, llr[pick], 50), f"configured batch, code {k}")


def test_sixteen_jobs_and_one_more(tdev):
    """The most jobs one call takes (16): the eight QC codes at small batches,
    then eight (3,6) codes (four graphs, each twice, some large enough for a
    launch of their own), every frame against the oracle; a 17th job is
    refused before anything runs."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    specs = [(c["H"], c["rate"], 40 + 25 * k) for k, c in enumerate(wl.qc_multi_code_family(seed=7))]
    regs = [wl.regular_ldpc(96, 48, 3, 6, seed=1), wl.regular_ldpc(1024, 512, 3, 6, seed=2),
            wl.regular_ldpc(192, 96, 3, 6, seed=3), wl.regular_ldpc(480, 240, 3, 6, seed=4)]
    specs += [(regs[k % 4], 0.5, B) for k, B in enumerate((300, 4000, 120, 257, 64, 3000, 1, 500))]
    graphs = {}
    jobs, inputs = [], []
    for k, (H, rate, B) in enumerate(specs):
        key = id(H)
        if key not in graphs:
            graphs[key] = ldpc.build_graph(torch.from_numpy(H).to(dev))
        llr = wl.bpsk_awgn_llr(None, 2.0, rate, seed=600 + k, n=H.shape[1], batch=B)
        jobs.append((graphs[key], torch.from_numpy(llr).to(dev)))
        inputs.append((H, llr))
    assert len(jobs) == 16
    note(f"[multi] 16 jobs, batches {[s[2] for s in specs]}")
    outs = ldpc.minsum_decode_multi(jobs, 30)
    torch.cuda.synchronize()
    for k, ((H, llr), o) in enumerate(zip(inputs, outs)):
        assert_parity(tuple(t.cpu().numpy() for t in o), oracle_decode(H, llr, 30), f"16 jobs, job {k}")
    with pytest.raises(ldpc.LdpcError) as e:
        ldpc.minsum_decode_multi(jobs + [jobs[0]], 30)
    assert e.value.name == "LDPC_EUNSUPPORTED"


N_RANDOM_CALLS = int(__import__("os").environ.get("LDPC_RANDOM_MULTI", "6"))


@pytest.mark.parametrize("k", range(N_RANDOM_CALLS))
def test_random_job_lists(tdev, k):
    """Seeded random calls: 1 to 16 jobs drawn from thirteen codes (a code may
    appear in several jobs), batches of 0 to 700 frames, launch choices set on
    some graphs, random L and flags; every job against the oracle.
    LDPC_RANDOM_MULTI sets the number of calls (6 by default)."""
    torch, dev = tdev
    from paper_2507_10424_amd import ldpc
    pool = [c["H"] for c in wl.qc_multi_code_family(seed=7)] + [
        wl.regular_ldpc(96, 48, 3, 6, seed=1), wl.regular_ldpc(1024, 512, 3, 6, seed=2),
        wl.regular_ldpc(240, 120, 3, 6, seed=5),
        wl.random_irregular_code(300, 120, seed=3, dv_choices=(1, 2, 3, 4), max_row_degree=8),
        wl.random_irregular_code(200, 90, seed=9, dv_choices=(2, 3, 6), max_row_degree=16)]
    rs = np.random.default_rng(5000 + k)
    idx = rs.integers(0, len(pool), size=int(rs.integers(1, 17)))
    L = int(rs.integers(0, 40))
    flags = int(rs.choice([0, 1, 2 << 8, 3 << 8]))
    graphs, jobs, inputs = {}, [], []
    for h in idx:
        H = pool[h]
        if h not in graphs:
            graphs[h] = ldpc.build_graph(torch.from_numpy(H).to(dev))
            if rs.random() < 0.3:
                for _ in range(10):  # a variant that fits, if one of 10 draws does
                    try:
                        ldpc.set_tuning(graphs[h], 1, variant=int(rs.integers(0, 42)),
                                        wg_per_cu=int(rs.integers(0, 5)), waves_per_simd=int(rs.choice([0, 4, 3])))
                        break
                    except ldpc.LdpcError:
                        continue
        B = int(rs.choice([0, 1, 7, 64, 200, 700]))
        llr = (rs.normal(1.0, rs.uniform(0.6, 1.6), size=(B, H.shape[1])) * rs.uniform(0.5, 3.0)).astype(np.float32)
        jobs.append((graphs[h], torch.from_numpy(llr).to(dev)))
        inputs.append((H, llr))
    note(f"[multi random {k}] codes {idx.tolist()} batches {[x.shape[0] for _, x in inputs]} L={L} flags={flags}")
    outs = ldpc.minsum_decode_multi(jobs, L, flags=flags)
    torch.cuda.synchronize()
    for j, ((H, llr), o) in enumerate(zip(inputs, outs)):
        if llr.shape[0]:
            assert_parity(tuple(t.cpu().numpy() for t in o), oracle_decode(H, llr, L, flags), f"random {k} job {j}")
