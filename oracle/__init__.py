"""FP64 CPU oracle for SFSeg's power iteration -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP path.
"""
from .sfseg_oracle import (OracleConfig, ZeroNormError, build_adjacency,  # noqa: F401
                           build_adjacency_exact, build_adjacency_multi, gaussian_taps,
                           power_iteration, spacetime_kernel, unary_weights)
