"""ctypes binding of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "minsum_oracle.c")
SRC_GRAD = os.path.join(HERE, "nms_grad_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_f32p = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i32 = ctypes.c_int32


LIB_SANITIZED = os.path.join(HERE, "liboracle_san.so")
# Sanitizer build: AddressSanitizer (out-of-bounds and use-after-free on the
# heap and stack) and UndefinedBehaviorSanitizer (signed overflow, bad shifts,
# misaligned or null accesses), every finding fatal.  A process that loads it
# must preload the two runtimes (sanitizer_env).
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def build_oracle(mutant: int = 0, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the oracle (or a variant with a planted mistake, or the
    sanitizer build) and return the path of the shared library."""
    if sanitize:
        out = out or LIB_SANITIZED
    out = out or (LIB if mutant == 0 else os.path.join(HERE, f"liboracle_mutant{mutant}.so"))
    opt = SANITIZE_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc", *opt, "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           f"-DORACLE_MUTANT={mutant}", SRC, SRC_GRAD, "-o", out + ".tmp", "-lpthread", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _period(early_exit, check_period):
    k = int(check_period)
    if k < 1:
        raise ValueError("check_period must be >= 1")
    return k if early_exit else 0


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


class Oracle:
    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        lib.oracle_minsum_decode.argtypes = [_u8p, _i32, _i32, _f32p, _i32, _i32, _i32, _u8p, _f32p,
                                             _i32p, _u8p, _i32]
        lib.oracle_minsum_decode.restype = ctypes.c_int
        lib.oracle_nms_decode.argtypes = [_u8p, _i32, _i32, _f32p, _i32, _i32, _i32, _f32p, _f32p, _i32,
                                          _i32, _u8p, _f32p, _i32p, _u8p, _i32]
        lib.oracle_nms_decode.restype = ctypes.c_int
        lib.oracle_minsum_dense.argtypes = [_u8p, _i32, _i32, _f32p, _i32, _i32, _u8p, _f32p, _i32p, _u8p]
        lib.oracle_minsum_dense.restype = ctypes.c_int
        lib.oracle_syndrome.argtypes = [_u8p, _i32, _i32, _u8p, _i32, _u8p]
        lib.oracle_syndrome.restype = ctypes.c_int
        lib.oracle_check_degrees.argtypes = [_u8p, _i32, _i32, _i32p, _i32]
        lib.oracle_check_degrees.restype = _i32
        _f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_nms_train_loss_grad.argtypes = [_u8p, _i32, _i32, _f64p, _u8p, _i32, _f64p, _f64p, _i32, _i32,
                                                   _f64p, _f64p, _f64p, _f64p]
        lib.oracle_nms_train_loss_grad.restype = ctypes.c_int
        lib.oracle_nms_train_loss_grad_ex.argtypes = [_u8p, _i32, _i32, _f64p, _u8p, _i32, _f64p, _f64p, _i32, _i32,
                                                      _i32, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        lib.oracle_nms_train_loss_grad_ex.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def minsum_decode(self, H, llr, max_iter, early_exit=True, nthreads=0, check_period=1):
        """Algorithm 1 on every frame of ``llr`` (B, n).  Returns
        (bits uint8 (B,n), post float32 (B,n), iters int32 (B,), ok uint8 (B,)).
        With early exit the codeword test runs before the first iteration and
        after every ``check_period``-th one."""
        H = np.ascontiguousarray(H, dtype=np.uint8)
        llr = np.ascontiguousarray(llr, dtype=np.float32)
        m, n = H.shape
        B = llr.shape[0]
        assert llr.shape == (B, n)
        bits = np.empty((B, n), np.uint8)
        post = np.empty((B, n), np.float32)
        iters = np.empty(B, np.int32)
        ok = np.empty(B, np.uint8)
        st = self.lib.oracle_minsum_decode(_p(H, _u8p), m, n, _p(llr, _f32p), B, int(max_iter),
                                           _period(early_exit, check_period), _p(bits, _u8p), _p(post, _f32p),
                                           _p(iters, _i32p), _p(ok, _u8p), int(nthreads))
        if st:
            raise ValueError(f"oracle_minsum_decode status {st}")
        return bits, post, iters, ok

    def nms_decode(self, H, llr, max_iter, alpha, beta, early_exit=True, nthreads=0, check_period=1):
        H = np.ascontiguousarray(H, dtype=np.uint8)
        llr = np.ascontiguousarray(llr, dtype=np.float32)
        alpha = np.ascontiguousarray(alpha, dtype=np.float32)
        beta = np.ascontiguousarray(beta, dtype=np.float32)
        T, C = alpha.shape
        assert beta.shape == (T, C)
        m, n = H.shape
        B = llr.shape[0]
        bits = np.empty((B, n), np.uint8)
        post = np.empty((B, n), np.float32)
        iters = np.empty(B, np.int32)
        ok = np.empty(B, np.uint8)
        st = self.lib.oracle_nms_decode(_p(H, _u8p), m, n, _p(llr, _f32p), B, int(max_iter),
                                        _period(early_exit, check_period), _p(alpha, _f32p), _p(beta, _f32p), T, C,
                                        _p(bits, _u8p), _p(post, _f32p), _p(iters, _i32p), _p(ok, _u8p),
                                        int(nthreads))
        if st:
            raise ValueError(f"oracle_nms_decode status {st}")
        return bits, post, iters, ok

    def minsum_dense(self, H, r, max_iter, early_exit=True):
        """Algorithm 2 on one frame r (n,)."""
        H = np.ascontiguousarray(H, dtype=np.uint8)
        r = np.ascontiguousarray(r, dtype=np.float32)
        m, n = H.shape
        bits = np.empty(n, np.uint8)
        post = np.empty(n, np.float32)
        it = np.empty(1, np.int32)
        ok = np.empty(1, np.uint8)
        st = self.lib.oracle_minsum_dense(_p(H, _u8p), m, n, _p(r, _f32p), int(max_iter), int(bool(early_exit)),
                                          _p(bits, _u8p), _p(post, _f32p), _p(it, _i32p), _p(ok, _u8p))
        if st:
            raise ValueError(f"oracle_minsum_dense status {st}")
        return bits, post, int(it[0]), int(ok[0])

    def syndrome(self, H, bits):
        H = np.ascontiguousarray(H, dtype=np.uint8)
        bits = np.ascontiguousarray(np.atleast_2d(bits), dtype=np.uint8)
        m, n = H.shape
        out = np.empty((bits.shape[0], m), np.uint8)
        st = self.lib.oracle_syndrome(_p(H, _u8p), m, n, _p(bits, _u8p), bits.shape[0], _p(out, _u8p))
        if st:
            raise ValueError("oracle_syndrome failed")
        return out

    def nms_train_loss_grad(self, H, llr, alpha, beta, targets=None, grad=True, llr_grad=False):
        """FP64 training loss of the learned decoder (T = alpha.shape[0]
        unrolled iterations, no early exit) and its gradient.  Returns
        (loss, galpha, gbeta, gllr) with None for what was not asked."""
        _f64p = ctypes.POINTER(ctypes.c_double)
        H = np.ascontiguousarray(H, dtype=np.uint8)
        llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float64)
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        T, C = alpha.shape
        m, n = H.shape
        B = llr.shape[0]
        tg = None if targets is None else np.ascontiguousarray(np.atleast_2d(targets), dtype=np.uint8)
        loss = np.zeros(1)
        ga = np.zeros((T, C)) if grad else None
        gb = np.zeros((T, C)) if grad else None
        gl = np.zeros((B, n)) if (grad and llr_grad) else None
        st = self.lib.oracle_nms_train_loss_grad(_p(H, _u8p), m, n, _p(llr, _f64p), _p(tg, _u8p), B,
                                                 _p(alpha, _f64p), _p(beta, _f64p), T, C, _p(loss, _f64p),
                                                 _p(ga, _f64p), _p(gb, _f64p), _p(gl, _f64p))
        if st:
            raise ValueError(f"oracle_nms_train_loss_grad status {st}")
        return float(loss[0]), ga, gb, gl

    def nms_train_grad_f32_forward(self, H, llr, alpha, beta, targets=None, llr_grad=True):
        """The training gradient along the binary32 decoder's forward: the
        forward of T = alpha.shape[0] iterations in binary32 arithmetic (the
        decoding oracle's), the reverse sweep in double along its argmin
        positions, signs and clip masks.  ``llr``, ``alpha`` and ``beta`` are
        taken as float32.  Returns a dict with loss, galpha, gbeta, gllr (None
        unless llr_grad), the magnitude bounds aalpha, abeta, allr of those
        entries (the sweep with absolute values of every term) and post, the
        posteriors after iteration T."""
        _f64p = ctypes.POINTER(ctypes.c_double)
        H = np.ascontiguousarray(H, dtype=np.uint8)
        llr = np.ascontiguousarray(np.atleast_2d(np.asarray(llr, dtype=np.float32)), dtype=np.float64)
        alpha = np.ascontiguousarray(np.asarray(alpha, dtype=np.float32), dtype=np.float64)
        beta = np.ascontiguousarray(np.asarray(beta, dtype=np.float32), dtype=np.float64)
        T, C = alpha.shape
        m, n = H.shape
        B = llr.shape[0]
        tg = None if targets is None else np.ascontiguousarray(np.atleast_2d(targets), dtype=np.uint8)
        loss = np.zeros(1)
        out = {k: np.zeros((T, C)) for k in ("galpha", "gbeta", "aalpha", "abeta")}
        out["gllr"] = np.zeros((B, n)) if llr_grad else None
        out["allr"] = np.zeros((B, n)) if llr_grad else None
        out["post"] = np.zeros((B, n))
        st = self.lib.oracle_nms_train_loss_grad_ex(
            _p(H, _u8p), m, n, _p(llr, _f64p), _p(tg, _u8p), B, _p(alpha, _f64p), _p(beta, _f64p), T, C, 1,
            _p(loss, _f64p), _p(out["galpha"], _f64p), _p(out["gbeta"], _f64p), _p(out["gllr"], _f64p),
            _p(out["aalpha"], _f64p), _p(out["abeta"], _f64p), _p(out["allr"], _f64p), _p(out["post"], _f64p))
        if st:
            raise ValueError(f"oracle_nms_train_loss_grad_ex status {st}")
        out["loss"] = float(loss[0])
        return out

    def check_degrees(self, H):
        H = np.ascontiguousarray(H, dtype=np.uint8)
        m, n = H.shape
        deg = np.zeros(n + 1, np.int32)
        c = self.lib.oracle_check_degrees(_p(H, _u8p), m, n, _p(deg, _i32p), n + 1)
        if c < 0:
            raise ValueError(f"oracle_check_degrees status {c}")
        return deg[:c].copy()


_default: Oracle | None = None


def sanitizer_env() -> dict:
    """Environment of a process that loads the sanitizer build: the ASan and
    UBSan runtimes preloaded (the interpreter itself is not instrumented, so
    leak reports, which would be Python's, are off) and the oracle path in
    LDPC_ORACLE_LIB."""
    rt = [subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True, check=True).stdout.strip()
          for n in ("libasan.so", "libubsan.so")]
    env = dict(os.environ)
    env["LD_PRELOAD"] = ":".join(rt)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["LDPC_ORACLE_LIB"] = LIB_SANITIZED
    return env


def load_oracle() -> Oracle:
    """The oracle library: LDPC_ORACLE_LIB if set (the sanitizer build),
    else liboracle.so, rebuilt when a source is newer."""
    global _default
    if _default is None and os.environ.get("LDPC_ORACLE_LIB"):
        _default = Oracle(os.environ["LDPC_ORACLE_LIB"])
    if _default is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(SRC_GRAD)):
            build_oracle()
        _default = Oracle(LIB)
    return _default


def minsum_decode(*a, **k):
    return load_oracle().minsum_decode(*a, **k)


def nms_decode(*a, **k):
    return load_oracle().nms_decode(*a, **k)


def minsum_dense(*a, **k):
    return load_oracle().minsum_dense(*a, **k)


def syndrome(*a, **k):
    return load_oracle().syndrome(*a, **k)


def check_degrees(*a, **k):
    return load_oracle().check_degrees(*a, **k)


def nms_train_grad_f32_forward(*a, **k):
    return load_oracle().nms_train_grad_f32_forward(*a, **k)


def nms_train_loss_grad(*a, **k):
    return load_oracle().nms_train_loss_grad(*a, **k)
