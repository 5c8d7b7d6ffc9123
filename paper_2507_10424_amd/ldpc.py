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
LDPC_CHECK_PERIOD_SHIFT = 8


def check_period(k: int) -> int:
    """Flag bits for the codeword-test period k (1..255): with early exit a
    frame is tested before the first iteration and after every k-th one."""
    k = int(k)
    if not 1 <= k <= 255:
        raise ValueError("check period must be in 1..255")
    return k << LDPC_CHECK_PERIOD_SHIFT

_STATUS = {0: "LDPC_OK", -1: "LDPC_EINVAL", -2: "LDPC_EBADH", -3: "LDPC_ENOMEM", -4: "LDPC_EHIP",
           -5: "LDPC_EWORKSPACE", -6: "LDPC_EUNSUPPORTED"}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)

_lib = None


class LdpcTuning(ctypes.Structure):
    """struct ldpc_tuning of include/ldpc.h"""
    _fields_ = [("path", ctypes.c_int32), ("variant", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("stream_waves", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("ms", ctypes.c_float),
                ("stream_nt", ctypes.c_int32), ("stream_chunk", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LdpcJob(ctypes.Structure):
    """struct ldpc_job of include/ldpc.h"""
    _fields_ = [("g", ctypes.c_void_p), ("llr_dev", ctypes.c_void_p), ("B", ctypes.c_int32),
                ("bits_dev", ctypes.c_void_p), ("post_dev", ctypes.c_void_p), ("iters_dev", ctypes.c_void_p),
                ("ok_dev", ctypes.c_void_p)]


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
    lib.ldpc_minsum_decode_noalloc.argtypes = [_vp, _vp, _i32, _i32, _u32, _vp, _vp, _vp, _vp, _vp]
    lib.ldpc_minsum_decode_noalloc.restype = ctypes.c_int
    lib.ldpc_dense_workspace_bytes.argtypes = [_vp, _i32]
    lib.ldpc_dense_workspace_bytes.restype = ctypes.c_size_t
    lib.ldpc_minsum_decode_dense.argtypes = [_vp, _vp, _i32, _i32, _u32, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                             _vp]
    lib.ldpc_minsum_decode_dense.restype = ctypes.c_int
    lib.ldpc_status_string.argtypes = [ctypes.c_int]
    lib.ldpc_status_string.restype = ctypes.c_char_p
    lib.ldpc_nms_decode.argtypes = [_vp, _vp, _i32, _i32, _u32, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp]
    lib.ldpc_nms_decode.restype = ctypes.c_int
    lib.ldpc_nms_train_workspace_bytes.argtypes = [_vp, _i32, _i32, _i32]
    lib.ldpc_nms_train_workspace_bytes.restype = ctypes.c_size_t
    lib.ldpc_nms_train_forward.argtypes = [_vp, _vp, _vp, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _vp,
                                           ctypes.c_size_t, _vp]
    lib.ldpc_nms_train_forward.restype = ctypes.c_int
    lib.ldpc_nms_train_backward.argtypes = [_vp, _vp, _vp, _i32, _i32, _vp, _vp, _i32, ctypes.c_float, _vp, _vp,
                                            _vp, _vp, ctypes.c_size_t, _vp]
    lib.ldpc_nms_train_backward.restype = ctypes.c_int
    lib.ldpc_awgn_llr.argtypes = [_vp, _i32, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_uint64, _vp, _vp, _vp]
    lib.ldpc_awgn_llr.restype = ctypes.c_int
    lib.ldpc_adam_step.argtypes = [_vp, _vp, _vp, _vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, _i32, _vp]
    lib.ldpc_adam_step.restype = ctypes.c_int
    lib.ldpc_multi_workspace_bytes.argtypes = [_i32]
    lib.ldpc_multi_workspace_bytes.restype = ctypes.c_size_t
    lib.ldpc_minsum_decode_multi.argtypes = [ctypes.POINTER(LdpcJob), _i32, _i32, _u32, _vp, ctypes.c_size_t, _vp]
    lib.ldpc_minsum_decode_multi.restype = ctypes.c_int
    lib.ldpc_graph_set_tuning.argtypes = [_vp, ctypes.POINTER(LdpcTuning)]
    lib.ldpc_graph_set_tuning.restype = ctypes.c_int
    lib.ldpc_graph_get_tuning.argtypes = [_vp, ctypes.POINTER(LdpcTuning)]
    lib.ldpc_graph_get_tuning.restype = ctypes.c_int
    lib.ldpc_autotune_workspace_bytes.argtypes = [_vp, _i32]
    lib.ldpc_autotune_workspace_bytes.restype = ctypes.c_size_t
    lib.ldpc_autotune.argtypes = [_vp, _i32, _i32, ctypes.c_float, _vp, ctypes.c_size_t, _vp,
                                  ctypes.POINTER(LdpcTuning)]
    lib.ldpc_autotune.restype = ctypes.c_int
    lib.ldpc_timing_enable.argtypes = [ctypes.c_int]
    lib.ldpc_timing_enable.restype = ctypes.c_int
    lib.ldpc_timing_read.argtypes = [_i32, ctypes.POINTER(ctypes.c_double), _i64p]
    lib.ldpc_timing_read.restype = ctypes.c_int
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


NOALLOC_SCRATCH_BYTES = 16 << 20  # LDPC_NOALLOC_SCRATCH_BYTES


def minsum_decode_noalloc(g: Graph, llr: torch.Tensor, max_iter: int, flags: int = 0, out=None):
    """ldpc_minsum_decode_noalloc: the decode with the library's own scratch
    memory instead of a workspace (decodes needing more than 16 MiB of
    workspace are refused).  ``out`` = (bits, post or None, iters, ok)
    preallocated; without it the outputs are allocated here."""
    llr = _check_llr(g, llr)
    B = llr.shape[0]
    bits, post, iters, ok = out if out is not None else _outputs(B, g.n, llr.device, True)
    lib = load_library()
    with torch.cuda.device(llr.device):
        st = lib.ldpc_minsum_decode_noalloc(g.handle, _ptr(llr), B, int(max_iter), int(flags), _ptr(bits),
                                            _ptr(post), _ptr(iters), _ptr(ok), _stream(llr.device))
    if st:
        raise LdpcError(st, "ldpc_minsum_decode_noalloc")
    return bits, post, iters, ok


def dense_workspace_bytes(g: Graph, B: int) -> int:
    return int(load_library().ldpc_dense_workspace_bytes(g.handle, int(B)))


def minsum_decode_dense(g: Graph, llr: torch.Tensor, max_iter: int, flags: int = 0, want_post: bool = True,
                        workspace: torch.Tensor | None = None, out=None):
    """ldpc_minsum_decode_dense: the dense map-reduce form (Algorithm 2), an
    ablation of the sparse decoders.  Same outputs as minsum_decode."""
    llr = _check_llr(g, llr)
    B = llr.shape[0]
    bits, post, iters, ok = out if out is not None else _outputs(B, g.n, llr.device, want_post)
    if workspace is None:
        workspace = torch.empty(max(dense_workspace_bytes(g, B), 1), dtype=torch.uint8, device=llr.device)
    lib = load_library()
    with torch.cuda.device(llr.device):
        st = lib.ldpc_minsum_decode_dense(g.handle, _ptr(llr), B, int(max_iter), int(flags), _ptr(bits),
                                          _ptr(post), _ptr(iters), _ptr(ok), _ptr(workspace), workspace.numel(),
                                          _stream(llr.device))
    if st:
        raise LdpcError(st, "ldpc_minsum_decode_dense")
    return bits, post, iters, ok


def nms_decode(g: Graph, llr: torch.Tensor, max_iter: int, alpha: torch.Tensor, beta: torch.Tensor,
               flags: int = 0, want_post: bool = True, workspace: torch.Tensor | None = None, out=None):
    """ldpc_nms_decode: normalised/offset Min-Sum with per-iteration,
    per-check-degree weights alpha, beta of shape (T, n_classes), float32,
    on the GPU."""
    lib = load_library()
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


# ---------------------------------------------------------------------------
# training of the learned decoder, synthetic frames, Adam
# ---------------------------------------------------------------------------

def train_workspace_bytes(g: Graph, B: int, T: int, ckpt_every: int) -> int:
    return int(load_library().ldpc_nms_train_workspace_bytes(g.handle, int(B), int(T), int(ckpt_every)))


def _check_weights(g: Graph, alpha: torch.Tensor, beta: torch.Tensor):
    T = alpha.shape[0]
    if alpha.shape != (T, len(g.check_degrees)) or beta.shape != alpha.shape:
        raise ValueError("alpha and beta must be (T, n_classes)")
    if alpha.dtype != torch.float32 or beta.dtype != torch.float32 or not alpha.is_cuda or not beta.is_cuda:
        raise ValueError("alpha and beta must be float32 CUDA tensors")
    return alpha.contiguous(), beta.contiguous(), T


def nms_train_forward(g: Graph, llr: torch.Tensor, alpha: torch.Tensor, beta: torch.Tensor, ckpt_every: int,
                      workspace: torch.Tensor, target: torch.Tensor | None = None, want_post: bool = False):
    """ldpc_nms_train_forward: returns (loss (1,) float32 tensor, post or None)."""
    llr = _check_llr(g, llr)
    alpha, beta, T = _check_weights(g, alpha, beta)
    B = llr.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=llr.device)
    post = torch.empty((B, g.n), dtype=torch.float32, device=llr.device) if want_post else None
    tg = None if target is None else target.to(torch.uint8).contiguous()
    with torch.cuda.device(llr.device):
        st = load_library().ldpc_nms_train_forward(g.handle, _ptr(llr), _ptr(tg), B, T, _ptr(alpha), _ptr(beta),
                                                   int(ckpt_every), _ptr(loss), _ptr(post), _ptr(workspace),
                                                   workspace.numel(), _stream(llr.device))
    if st:
        raise LdpcError(st, "ldpc_nms_train_forward")
    return loss, post


def nms_train_backward(g: Graph, llr: torch.Tensor, alpha: torch.Tensor, beta: torch.Tensor, ckpt_every: int,
                       workspace: torch.Tensor, grad_loss: float = 1.0, target: torch.Tensor | None = None,
                       want_llr_grad: bool = False):
    """ldpc_nms_train_backward: returns (galpha, gbeta, gllr or None)."""
    llr = _check_llr(g, llr)
    alpha, beta, T = _check_weights(g, alpha, beta)
    B = llr.shape[0]
    ga = torch.empty_like(alpha)
    gb = torch.empty_like(beta)
    gl = torch.empty_like(llr) if want_llr_grad else None
    tg = None if target is None else target.to(torch.uint8).contiguous()
    with torch.cuda.device(llr.device):
        st = load_library().ldpc_nms_train_backward(g.handle, _ptr(llr), _ptr(tg), B, T, _ptr(alpha), _ptr(beta),
                                                    int(ckpt_every), float(grad_loss), _ptr(ga), _ptr(gb), _ptr(gl),
                                                    _ptr(workspace), workspace.numel(), _stream(llr.device))
    if st:
        raise LdpcError(st, "ldpc_nms_train_backward")
    return ga, gb, gl


def awgn_llr(B: int, n: int, rate: float, ebn0_db, seed: int, device, codewords: torch.Tensor | None = None,
             want_ebn0: bool = False):
    """ldpc_awgn_llr: (B, n) float32 LLRs of BPSK over AWGN generated on the
    GPU; ebn0_db is a value or a (lo, hi) range drawn per frame."""
    lo, hi = (float(ebn0_db), float(ebn0_db)) if not isinstance(ebn0_db, (tuple, list)) else map(float, ebn0_db)
    llr = torch.empty((B, n), dtype=torch.float32, device=device)
    eb = torch.empty((B,), dtype=torch.float32, device=device) if want_ebn0 else None
    cw = None if codewords is None else codewords.to(torch.uint8).contiguous()
    with torch.cuda.device(llr.device):
        st = load_library().ldpc_awgn_llr(_ptr(cw), int(B), int(n), float(rate), lo, hi,
                                          ctypes.c_uint64(int(seed) & ((1 << 64) - 1)), _ptr(llr), _ptr(eb),
                                          _stream(llr.device))
    if st:
        raise LdpcError(st, "ldpc_awgn_llr")
    return (llr, eb) if want_ebn0 else llr


def adam_step(param: torch.Tensor, grad: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor, lr: float, step: int,
              betas=(0.9, 0.999), eps: float = 1e-8):
    """ldpc_adam_step on contiguous float32 CUDA tensors, in place."""
    for t in (param, grad, m1, m2):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("adam_step needs contiguous float32 CUDA tensors")
    with torch.cuda.device(param.device):
        st = load_library().ldpc_adam_step(_ptr(param), _ptr(grad), _ptr(m1), _ptr(m2), param.numel(), float(lr),
                                           float(betas[0]), float(betas[1]), float(eps), int(step),
                                           _stream(param.device))
    if st:
        raise LdpcError(st, "ldpc_adam_step")


def minsum_decode_multi(jobs, max_iter: int, flags: int = 0, want_post: bool = True, workspace=None, outs=None):
    """ldpc_minsum_decode_multi: jobs is a list of (Graph, llr) pairs decoded
    in one launch.  Returns a list of (bits, post, iters, ok), one per job."""
    if not jobs:
        raise ValueError("no jobs")
    lib = load_library()
    arr = (LdpcJob * len(jobs))()
    results = []
    for k, (g, llr) in enumerate(jobs):
        llr = _check_llr(g, llr)
        o = outs[k] if outs is not None else _outputs(llr.shape[0], g.n, llr.device, want_post)
        results.append((llr, o))
        bits, post, iters, ok = o
        arr[k] = LdpcJob(g.handle.value, llr.data_ptr(), llr.shape[0], bits.data_ptr(),
                         post.data_ptr() if post is not None else None, iters.data_ptr(), ok.data_ptr())
    dev = jobs[0][1].device
    need = int(lib.ldpc_multi_workspace_bytes(len(jobs)))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        st = lib.ldpc_minsum_decode_multi(arr, len(jobs), int(max_iter), int(flags), _ptr(workspace),
                                          workspace.numel(), _stream(dev))
    if st:
        raise LdpcError(st, "ldpc_minsum_decode_multi")
    return [o for _, o in results]


class CapturedDecode:
    """A decode call captured once into a HIP graph (torch.cuda.CUDAGraph)
    and replayed.  Inputs and outputs are static buffers: copy new LLRs into
    ``.llr`` (or the per-job LLR tensors of a multi-code capture) and call
    ``replay()``.

    jobs: a Graph (single code) or a list of Graphs (one multi-code launch);
    batches: B, or one B per graph."""

    def __init__(self, jobs, batches, max_iter: int, flags: int = 0, want_post: bool = True,
                 alpha: torch.Tensor | None = None, beta: torch.Tensor | None = None):
        self.multi = isinstance(jobs, (list, tuple))
        graphs = list(jobs) if self.multi else [jobs]
        Bs = list(batches) if self.multi else [batches]
        dev = graphs[0].device
        self.graphs, self.max_iter, self.flags = graphs, max_iter, flags
        self.alpha, self.beta = alpha, beta
        self.llrs = [torch.zeros((B, g.n), dtype=torch.float32, device=dev) for g, B in zip(graphs, Bs)]
        self.outs = [_outputs(B, g.n, dev, want_post) for g, B in zip(graphs, Bs)]
        if self.multi:
            need = int(load_library().ldpc_multi_workspace_bytes(len(graphs)))
        else:
            need = workspace_bytes(graphs[0], Bs[0], flags)
        self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        side = torch.cuda.Stream(device=dev)  # default priority
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            self._run()  # warm-up outside the capture (kernel attributes, lazy loading)
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._run()

    @property
    def llr(self):
        return self.llrs[0]

    def _run(self):
        if self.multi:
            minsum_decode_multi(list(zip(self.graphs, self.llrs)), self.max_iter, self.flags, workspace=self.ws,
                                outs=self.outs)
        elif self.alpha is not None:
            nms_decode(self.graphs[0], self.llrs[0], self.max_iter, self.alpha, self.beta, flags=self.flags,
                       workspace=self.ws, out=self.outs[0])
        else:
            minsum_decode(self.graphs[0], self.llrs[0], self.max_iter, flags=self.flags, workspace=self.ws,
                          out=self.outs[0])

    def replay(self):
        self.graph.replay()
        return self.outs if self.multi else self.outs[0]


def set_tuning(g: Graph, path: int | None = None, variant: int = -1, wg_per_cu: int = 0, stream_waves: int = 4,
               waves_per_simd: int = 0, stream_nt: int = -1, stream_chunk: int = -1):
    """ldpc_graph_set_tuning; path None clears the record."""
    lib = load_library()
    t = None if path is None else ctypes.byref(LdpcTuning(path, variant, wg_per_cu, stream_waves, waves_per_simd,
                                                          0.0, stream_nt, stream_chunk))
    st = lib.ldpc_graph_set_tuning(g.handle, t)
    if st:
        raise LdpcError(st, "ldpc_graph_set_tuning")


def get_tuning(g: Graph) -> dict:
    t = LdpcTuning()
    st = load_library().ldpc_graph_get_tuning(g.handle, ctypes.byref(t))
    if st:
        raise LdpcError(st, "ldpc_graph_get_tuning")
    return t.as_dict()


def autotune(g: Graph, B: int, max_iter: int, ebn0_db: float) -> dict:
    """ldpc_autotune: time the launch choices on B synthetic frames and keep
    the fastest in the graph's tuning record.  Returns it as a dict."""
    lib = load_library()
    need = int(lib.ldpc_autotune_workspace_bytes(g.handle, int(B)))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=g.device)
    best = LdpcTuning()
    with torch.cuda.device(g.device):
        st = lib.ldpc_autotune(g.handle, int(B), int(max_iter), float(ebn0_db), _ptr(ws), ws.numel(),
                               _stream(g.device), ctypes.byref(best))
    if st:
        raise LdpcError(st, "ldpc_autotune")
    return best.as_dict()
