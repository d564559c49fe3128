"""MI355X-native HVOX: chunked 3D type-3 NUFFT synthesis and analysis
(Kashani et al., arXiv 2306.06007) as HIP kernels for gfx950 behind a C ABI.

``Plan(uvw, xyz, eps, dtype)`` plans the transforms; ``Plan.synthesis`` and
``Plan.analysis`` run them on torch GPU tensors.  ``autograd`` wraps them as
differentiable functions, ``serve`` runs a continuous-batching request
loop, and ``radio`` offers dirty2vis / vis2dirty on direction-cosine images.
``workloads`` generates seeded synthetic inputs."""
from .hvox import (EXPORTS, HvoxError, KERNELS, Plan, alg1, kernel_params, load_library,
                   partition, rel_l2)

__all__ = ["EXPORTS", "HvoxError", "KERNELS", "Plan", "alg1", "kernel_params",
           "load_library", "partition", "rel_l2"]
