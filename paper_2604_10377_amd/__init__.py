"""MI355X (gfx950) regularised functional-map solver.

The compute path is libfmap.so (HIP kernels behind the C ABI of
include/fmap.h); `fmap` is its thin Python binding, `synth` draws seeded
synthetic inputs.  Importing the package does not load the library; the
first call does, and fails loudly if it is not built.
"""
__all__ = ["fmap", "synth"]
