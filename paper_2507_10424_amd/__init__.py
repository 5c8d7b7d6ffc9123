"""Batched Min-Sum LDPC decoding on MI355X (gfx950).

The decoder runs as hand-written HIP kernels behind the C-ABI library
``libldpc.so`` (declared in ``include/ldpc.h``); ``paper_2507_10424_amd.ldpc``
is the thin ctypes binding.  ``workloads`` builds seeded synthetic inputs.
"""
__all__ = ["ldpc", "workloads"]
