"""CPU oracle for batched Min-Sum LDPC decoding (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``minsum_oracle.c`` (plain C,
compiled with ``-ffp-contract=off`` and no fast-math) through ctypes and shares
nothing with the HIP library.
"""
from .binding import (Oracle, build_oracle, load_oracle, minsum_decode, nms_decode,  # noqa: F401
                      minsum_dense, syndrome, check_degrees, nms_train_loss_grad,
                      nms_train_grad_f32_forward)
