"""OctaOctree neural-radiosity hot path on AMD Instinct MI355X (gfx950).

The query (octree descent, octahedral bilinear fetch per level, decoder MLP)
and the residual step's forward and backward run in hand-written HIP kernels
behind the C-ABI of ``liboctaoctree.so`` (include/octaoctree.h); this package
holds that library's sources (``csrc/``), its build script and the thin
Python binding. The binding (and torch) load on first use of one of its
names.
"""
_BINDING_NAMES = ("MLP", "OctaOctree", "RadiosityResidual", "Tree", "build_octree", "cast_params", "device_batch",
                  "encode_query", "mlp_fwd", "query_fwd", "residual_bwd", "residual_fwd", "residual_workspace_bytes")


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
