"""MI355X (gfx950) evaluator for GOFMM compressions of dense SPD matrices.

The compression is built on the host and K~W runs in hand-written HIP kernels
inside libgofmm.so; this package is the thin Python binding of its C ABI
(include/gofmm.h).
"""
from .gofmm import (ANGLE, BF16, BF16X3, FP32, GRAM_L2, Compression, GofmmError,  # noqa: F401
                    KernelSampler, PySampler, Server, batched_spin_limit, batched_status,
                    evaluate_batched, lib, params)
