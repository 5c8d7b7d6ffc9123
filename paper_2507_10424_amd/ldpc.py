"""Python binding of libldpc (argument marshalling only).

Every step of decoding runs in the HIP kernels of ``libldpc.so``; this module
passes torch tensors' device pointers and torch's current HIP stream through
ctypes.  If the library is missing it raises: there is no fallback.

The entry points mirror ``include/ldpc.h``:

    g = build_graph(H)                                  # H: (m, n) uint8 on the GPU
    bits, post, iters, ok = minsum_decode(g, llr, max_iter)
"""
from __future__ import annotations

import ctypes
import os

import torch  # imported first so that libldpc binds to torch's HIP runtime

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libldpc.so")

LDPC_NO_EARLY_EXIT = 1 << 0
LDPC_FORCE_STREAM = 1 << 1
LDPC_FORCE_ONCHIP = 1 << 2

_STATUS = {0: "LDPC_OK", -1: "LDPC_EINVAL", -2: "LDPC_EBADH", -3: "LDPC_ENOMEM", -4: "LDPC_EHIP",
           -5: "LDPC_EWORKSPACE", -6: "LDPC_EUNSUPPORTED"}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)

_lib = None


class LdpcError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        self.name = _STATUS.get(status, str(status))
        msg = load_library().ldpc_status_string(status).decode()
        super().__init__(f"{what}: {self.name} ({msg})")


def load_library():
    """Load libldpc.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc, gfx950); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    lib.ldpc_build_graph.argtypes = [_vp, _i32, _i32, _vp, ctypes.POINTER(_vp)]
    lib.ldpc_build_graph.restype = ctypes.c_int
    lib.ldpc_graph_info.argtypes = [_vp, _i32p, _i32p, _i64p, _i32p, _i32p, _i32p, _i32p, _i32]
    lib.ldpc_graph_info.restype = ctypes.c_int
    lib.ldpc_graph_destroy.argtypes = [_vp]
    lib.ldpc_graph_destroy.restype = None
    lib.ldpc_decode_workspace_bytes.argtypes = [_vp, _i32, _u32]
    lib.ldpc_decode_workspace_bytes.restype = ctypes.c_size_t
    lib.ldpc_minsum_decode.argtypes = [_vp, _vp, _i32, _i32, _u32, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.ldpc_minsum_decode.restype = ctypes.c_int
    lib.ldpc_status_string.argtypes = [ctypes.c_int]
    lib.ldpc_status_string.restype = ctypes.c_char_p
    if hasattr(lib, "ldpc_nms_decode"):
        lib.ldpc_nms_decode.argtypes = [_vp, _vp, _i32, _i32, _u32, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.c_size_t, _vp]
        lib.ldpc_nms_decode.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Graph:
    """A built Tanner graph (owns the library's device arrays)."""

    def __init__(self, handle: ctypes.c_void_p, device: torch.device):
        self._h = handle
        self.device = device
        lib = load_library()
        m, n, dc, dv, nc = (ctypes.c_int32() for _ in range(5))
        E = ctypes.c_int64()
        st = lib.ldpc_graph_info(handle, ctypes.byref(m), ctypes.byref(n), ctypes.byref(E), ctypes.byref(dc),
                                 ctypes.byref(dv), ctypes.byref(nc), None, 0)
        if st:
            raise LdpcError(st, "ldpc_graph_info")
        degs = (ctypes.c_int32 * max(1, nc.value))()
        lib.ldpc_graph_info(handle, None, None, None, None, None, None, degs, nc.value)
        self.m, self.n, self.E = m.value, n.value, E.value
        self.dc_max, self.dv_max = dc.value, dv.value
        self.check_degrees = [degs[k] for k in range(nc.value)]

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            load_library().ldpc_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_graph(H: torch.Tensor) -> Graph:
    """ldpc_build_graph: H is an (m, n) uint8 0/1 tensor on a GPU."""
    if H.dtype != torch.uint8 or H.dim() != 2 or not H.is_cuda:
        raise ValueError("H must be a 2-D uint8 CUDA tensor")
    H = H.contiguous()
    lib = load_library()
    out = ctypes.c_void_p()
    with torch.cuda.device(H.device):
        st = lib.ldpc_build_graph(_ptr(H), H.shape[0], H.shape[1], _stream(H.device), ctypes.byref(out))
    if st:
        raise LdpcError(st, "ldpc_build_graph")
    return Graph(out, H.device)


def workspace_bytes(g: Graph, B: int, flags: int = 0) -> int:
    return int(load_library().ldpc_decode_workspace_bytes(g.handle, int(B), int(flags)))


def _outputs(B, n, device, want_post):
    bits = torch.empty((B, n), dtype=torch.uint8, device=device)
    post = torch.empty((B, n), dtype=torch.float32, device=device) if want_post else None
    iters = torch.empty((B,), dtype=torch.int32, device=device)
    ok = torch.empty((B,), dtype=torch.uint8, device=device)
    return bits, post, iters, ok


def _check_llr(g: Graph, llr: torch.Tensor):
    if llr.dtype != torch.float32 or llr.dim() != 2 or llr.shape[1] != g.n or not llr.is_cuda:
        raise ValueError(f"llr must be a (B, {g.n}) float32 CUDA tensor")
    return llr.contiguous()


def minsum_decode(g: Graph, llr: torch.Tensor, max_iter: int, flags: int = 0, want_post: bool = True,
                  workspace: torch.Tensor | None = None, out=None):
    """ldpc_minsum_decode.  Returns (bits uint8 (B,n), post float32 (B,n) or
    None, iters int32 (B,), ok uint8 (B,)), all on llr's device, enqueued on
    torch's current stream."""
    llr = _check_llr(g, llr)
    B = llr.shape[0]
    bits, post, iters, ok = out if out is not None else _outputs(B, g.n, llr.device, want_post)
    need = workspace_bytes(g, B, flags)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=llr.device)
    lib = load_library()
    with torch.cuda.device(llr.device):
        st = lib.ldpc_minsum_decode(g.handle, _ptr(llr), B, int(max_iter), int(flags), _ptr(bits), _ptr(post),
                                    _ptr(iters), _ptr(ok), _ptr(workspace), workspace.numel(),
                                    _stream(llr.device))
    if st:
        raise LdpcError(st, "ldpc_minsum_decode")
    return bits, post, iters, ok


def nms_decode(g: Graph, llr: torch.Tensor, max_iter: int, alpha: torch.Tensor, beta: torch.Tensor,
               flags: int = 0, want_post: bool = True, workspace: torch.Tensor | None = None, out=None):
    """ldpc_nms_decode: normalised/offset Min-Sum with per-iteration,
    per-check-degree weights alpha, beta of shape (T, n_classes), float32,
    on the GPU."""
    lib = load_library()
    if not hasattr(lib, "ldpc_nms_decode"):
        raise RuntimeError("libldpc.so has no ldpc_nms_decode")
    llr = _check_llr(g, llr)
    B = llr.shape[0]
    T = alpha.shape[0]
    if alpha.shape != (T, len(g.check_degrees)) or beta.shape != alpha.shape:
        raise ValueError("alpha and beta must be (T, n_classes)")
    alpha = alpha.contiguous().float()
    beta = beta.contiguous().float()
    bits, post, iters, ok = out if out is not None else _outputs(B, g.n, llr.device, want_post)
    need = workspace_bytes(g, B, flags)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=llr.device)
    with torch.cuda.device(llr.device):
        st = lib.ldpc_nms_decode(g.handle, _ptr(llr), B, int(max_iter), int(flags), _ptr(alpha), _ptr(beta), T,
                                 _ptr(bits), _ptr(post), _ptr(iters), _ptr(ok), _ptr(workspace),
                                 workspace.numel(), _stream(llr.device))
    if st:
        raise LdpcError(st, "ldpc_nms_decode")
    return bits, post, iters, ok
