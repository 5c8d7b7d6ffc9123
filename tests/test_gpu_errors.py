"""Error paths of the C-ABI on a GPU: bad H, bad arguments, small workspace."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def test_bad_parity_matrices(torch_dev):
    torch, dev = torch_dev
    from paper_2507_10424_amd import ldpc
    H = np.ones((3, 6), np.uint8)
    H[1, 2] = 2
    with pytest.raises(ldpc.LdpcError) as e:
        ldpc.build_graph(torch.from_numpy(H).to(dev))
    assert e.value.status == -2
    H = np.zeros((3, 6), np.uint8)
    H[0, :3] = 1
    H[1, 4] = 1  # degree-1 row
    with pytest.raises(ldpc.LdpcError) as e:
        ldpc.build_graph(torch.from_numpy(H).to(dev))
    assert e.value.status == -2


def test_graph_info(torch_dev):
    torch, dev = torch_dev
    from paper_2507_10424_amd import ldpc
    from paper_2507_10424_amd import workloads as wl
    import oracle
    H = wl.random_irregular_code(80, 30, seed=3, dv_choices=(0, 1, 2, 3))
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    assert (g.m, g.n, g.E) == (30, 80, int(H.sum()))
    assert g.dc_max == int(H.sum(1).max()) and g.dv_max == int(H.sum(0).max())
    assert g.check_degrees == oracle.check_degrees(H).tolist()


def test_decode_argument_errors(torch_dev):
    torch, dev = torch_dev
    import ctypes
    from paper_2507_10424_amd import ldpc
    from paper_2507_10424_amd import workloads as wl
    lib = ldpc.load_library()
    H = wl.regular_ldpc(96, 48, 3, 6, seed=1)
    g = ldpc.build_graph(torch.from_numpy(H).to(dev))
    llr = torch.ones((10, 96), device=dev)
    bits = torch.empty((10, 96), dtype=torch.uint8, device=dev)
    iters = torch.empty((10,), dtype=torch.int32, device=dev)
    need = ldpc.workspace_bytes(g, 10)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    P = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = ldpc._stream(dev)
    assert lib.ldpc_minsum_decode(g.handle, P(llr), 10, -1, 0, P(bits), None, P(iters), None, P(ws), need, st) == -1
    assert lib.ldpc_minsum_decode(g.handle, P(llr), -1, 5, 0, P(bits), None, P(iters), None, P(ws), need, st) == -1
    assert lib.ldpc_minsum_decode(g.handle, None, 10, 5, 0, P(bits), None, P(iters), None, P(ws), need, st) == -1
    assert lib.ldpc_minsum_decode(g.handle, P(llr), 10, 5, 0, P(bits), None, P(iters), None, P(ws), need - 1,
                                  st) == -5
    assert lib.ldpc_minsum_decode(g.handle, P(llr), 10, 5, 0, P(bits), None, P(iters), None, None, 0, st) == -5
    assert lib.ldpc_minsum_decode(g.handle, None, 0, 5, 0, None, None, None, None, None, 0, st) == 0
    for bad_flags in (1 << 3, 1 << 16, 6):  # unknown bits; both paths forced
        assert lib.ldpc_minsum_decode(g.handle, P(llr), 10, 5, bad_flags, P(bits), None, P(iters), None, P(ws),
                                      need, st) == -1
    a = torch.ones((4, len(g.check_degrees)), device=dev)
    assert lib.ldpc_nms_decode(g.handle, P(llr), 10, 5, 0, P(a), P(a), 4, P(bits), None, P(iters), None, P(ws),
                               need, st) == -1  # max_iter > T
    torch.cuda.synchronize()
    ok = ldpc.minsum_decode(g, llr, 5, want_post=False)
    torch.cuda.synchronize()
    assert ok[1] is None and int(ok[2].max()) == 0
