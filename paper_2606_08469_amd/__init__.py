"""OctaOctree neural-radiosity hot path on AMD Instinct MI355X (gfx950).

The query (octree descent, octahedral bilinear fetch per level, decoder MLP)
and the residual step's forward and backward run in hand-written HIP kernels
behind the C-ABI of ``liboctaoctree.so`` (include/octaoctree.h); this package
holds that library's sources (``csrc/``), its build script and the thin
Python binding.
"""
from .binding import (  # noqa: F401
    MLP, OctaOctree, RadiosityResidual, Tree, build_octree, cast_params, device_batch, encode_query, mlp_fwd,
    query_fwd, residual_bwd, residual_fwd, residual_workspace_bytes,
)
