"""MI355X-native 13CO(2-1) PPV radiative-transfer path (IRIS-SO hot path).

Submodules:
  workloads -- seeded synthetic inputs (no radiative-transfer arithmetic)
  rt        -- PyTorch-facing binding of the HIP library (forward, adjoint,
               autograd Function, batched plans)
  metrics   -- error metrics used in reports (normwise errors, TSRE, TAM)
  build     -- hipcc build of the HIP library for gfx950

The HIP library is loaded lazily by ``rt``; importing this package does not
touch the GPU.
"""

__all__ = ["workloads", "rt", "metrics", "build"]
