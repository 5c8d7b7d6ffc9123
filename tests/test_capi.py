"""The C-ABI library without a GPU: it loads, exports every declared entry
point, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldpc.h")
LIB = os.path.join(ROOT, "paper_2507_10424_amd", "libldpc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ldpc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (bind to torch's HIP runtime, as the package does)
    if not os.path.exists(LIB):
        pytest.fail("libldpc.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["ldpc_build_graph", "ldpc_graph_info", "ldpc_graph_destroy", "ldpc_decode_workspace_bytes",
                 "ldpc_minsum_decode", "ldpc_nms_decode", "ldpc_status_string"]:
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    lib.ldpc_status_string.restype = ctypes.c_char_p
    seen = set()
    for st in range(0, -7, -1):
        s = lib.ldpc_status_string(st).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 7
    assert lib.ldpc_status_string(-99).decode() == "unknown status"


def test_null_arguments_rejected_without_device(lib):
    vp = ctypes.c_void_p
    lib.ldpc_build_graph.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, ctypes.POINTER(vp)]
    out = vp(1234)
    assert lib.ldpc_build_graph(None, 4, 8, None, ctypes.byref(out)) == -1
    assert out.value is None
    assert lib.ldpc_build_graph(vp(256), 0, 8, None, ctypes.byref(out)) == -1
    assert lib.ldpc_build_graph(vp(256), 4, 8, None, None) == -1
    lib.ldpc_decode_workspace_bytes.restype = ctypes.c_size_t
    lib.ldpc_decode_workspace_bytes.argtypes = [vp, ctypes.c_int32, ctypes.c_uint32]
    assert lib.ldpc_decode_workspace_bytes(None, 100, 0) == 0
    lib.ldpc_minsum_decode.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, vp, vp, vp, vp, vp,
                                       ctypes.c_size_t, vp]
    assert lib.ldpc_minsum_decode(None, None, 10, 5, 0, None, None, None, None, None, 0, None) == -1
    lib.ldpc_nms_decode.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, vp, vp, ctypes.c_int32,
                                    vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    assert lib.ldpc_nms_decode(None, None, 10, 5, 0, None, None, 5, None, None, None, None, None, 0, None) == -1
    lib.ldpc_graph_destroy.argtypes = [vp]
    lib.ldpc_graph_destroy(None)
    lib.ldpc_graph_info.argtypes = [vp] + [vp] * 7 + [ctypes.c_int32]
    assert lib.ldpc_graph_info(None, None, None, None, None, None, None, None, 0) == -1
