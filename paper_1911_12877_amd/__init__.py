"""MI355X-native exact subgraph counting with symmetry-breaking restrictions
and degree orientation (GraphZero's compiled mining loops as HIP kernels).

Submodules are imported on demand: ``gz`` is the binding of the C-ABI library
``libgz.so``; ``synth`` draws the seeded synthetic input graphs.
"""
__version__ = "0.1.0"
